"""GPU parity of delay and phase tracking (the per-antenna model applied to
the spectra before accumulation) against the CPU oracle's rotation of its own
spectra, through the C ABI.  Tolerances as in test_gpu_parity."""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_1102_0148_amd as corr
import synth
from test_gpu_parity import TOL, coef_error, raw_to_complex

pytestmark = pytest.mark.gpu


def _model(N, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    return dict(delay=rng.uniform(-50, 50, N) * scale, delay_rate=rng.uniform(-0.3, 0.3, N) * scale,
                phase=rng.uniform(-1, 1, N), phase_rate=rng.uniform(-0.02, 0.02, N))


def _round_up(x, m):
    return (x + m - 1) // m * m


@pytest.mark.parametrize("K", [128, 256, 512, 1024])
def test_tracked_fp32_spectra_match_oracle(K):
    N, S = 5, 11
    print(f"\n[track spectra] N={N} K={K} S={S}", flush=True)
    packed = synth.packed(synth.recipe_plain(N=N, two_k=2 * K, seed=41), 0, S).contiguous()
    m = _model(N, seed=K)
    c = corr.Correlator(N, K, S)
    c.set_tracking(**m)
    c.process(packed.cuda())
    buf, n = c.debug_read_spectra()
    assert n == S
    got = corr.records_to_spectra(buf, corr.CORR_FP32, N, K, S)
    ref = oracle.track(oracle.spectra(packed.numpy(), S, N, K), **m)
    scale = np.sqrt(np.mean(np.abs(ref) ** 2))
    assert np.max(np.abs(got - ref)) <= 4e-6 * scale * math.log2(2 * K)


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
@pytest.mark.parametrize("N,K,S,chunk", [(20, 256, 300, 64), (44, 256, 1024, 0), (7, 512, 130, 128)])
def test_tracked_float_end_to_end(prec, N, K, S, chunk):
    """Chunks of 64 and 128 spectra check that each chunk counts its spectra
    from the start of the integration."""
    print(f"\n[track {prec}] N={N} K={K} S={S} chunk={chunk}", flush=True)
    packed = synth.packed(synth.recipe_plain(N=N, two_k=2 * K, seed=N + K), 0, S).contiguous()
    m = _model(N, seed=N * K)
    c = corr.Correlator(N, K, S, precision=prec, tiles=dict(chunk_spectra=chunk) if chunk else None)
    c.set_tracking(**m)
    c.process(packed.cuda())
    raw = raw_to_complex(c.read_cps_raw())
    ref = oracle.cmac_f64(oracle.track(oracle.spectra(packed.numpy(), S, N, K), **m))
    assert coef_error(raw, ref, N) <= TOL[corr.PRECISIONS[prec]]


def test_tracked_long_integration_large_phases():
    """8192 spectra with delay rates that take the phase to thousands of
    turns: the argument is reduced in double before the sine and cosine."""
    N, K, S = 6, 256, 8192
    packed = synth.packed(synth.recipe_plain(N=N, two_k=2 * K, seed=3), 0, S).contiguous()
    m = _model(N, seed=9, scale=2.0)
    c = corr.Correlator(N, K, S)
    c.set_tracking(**m)
    c.process(packed.cuda())
    raw = raw_to_complex(c.read_cps_raw())
    ref = oracle.cmac_f64(oracle.track(oracle.spectra(packed.numpy(), S, N, K), **m))
    assert coef_error(raw, ref, N) <= TOL[corr.CORR_FP32]


@pytest.mark.parametrize("prec", ["int8", "int16"])
def test_tracked_integer_forms(prec):
    """Scales as without tracking (a rotation keeps |X|); codes within one of
    the oracle's rule on the oracle's rotated spectra; the X-stage exact on
    the GPU's own codes."""
    N, K, S = 44, 256, 200
    code = corr.PRECISIONS[prec]
    quantise = oracle.quantise if prec == "int8" else oracle.quantise16
    cmac = oracle.cmac_i64 if prec == "int8" else oracle.cmac_i64_16
    packed = synth.packed(synth.recipe_plain(N=N, two_k=2 * K, seed=12), 0, S).contiguous()
    m = _model(N, seed=5)
    c = corr.Correlator(N, K, S, precision=prec, tiles=dict(chunk_spectra=_round_up(S, 64)))
    c.set_tracking(**m)
    c.process(packed.cuda())
    buf, n = c.debug_read_spectra()
    scales = c.read_scales()
    raw = c.read_cps_raw()
    q_gpu = corr.records_to_spectra(buf, code, N, K, S)
    np.testing.assert_array_equal(raw, cmac(q_gpu).astype(np.float64))
    spec = oracle.spectra(packed.numpy(), S, N, K)
    W = min(S, corr.CORR_CALIB_SPECTRA)
    np.testing.assert_allclose(scales, oracle.scales_n(spec, W, W, prec), rtol=1e-5)
    q_ref = quantise(oracle.track(spec, **m), scales)
    diff = q_gpu.astype(np.int32) - q_ref.astype(np.int32)
    assert np.max(np.abs(diff)) <= 1
    # int16 steps are 256 times finer, so the same float difference between
    # the GPU's and the oracle's spectra reaches a rounding tie more often
    assert np.mean(diff != 0) <= (1e-3 if prec == "int8" else 5e-3)


def test_tracking_undoes_circular_delays():
    """Antenna a's blocks circularly delayed by d_a + r_a s samples, tracked
    with delay d_a and delay rate r_a, correlate as the undelayed blocks do
    without tracking (DFT shift theorem)."""
    N, K, S = 8, 256, 64
    x = synth.samples(synth.recipe_plain(N=N, two_k=2 * K, rho=0.3, seed=8), 0, S).numpy()
    d = np.array([0, 5, -9, 17, 40, -3, 100, 1], dtype=np.float64)
    r = np.array([0, 1, 0, -2, 3, 0, 1, 0], dtype=np.float64)
    y = np.empty_like(x)
    for s in range(S):
        for a in range(N):
            y[s, a] = np.roll(x[s, a], int(d[a] + r[a] * s))
    plain = corr.Correlator(N, K, S)
    plain.process(synth.pack(torch.from_numpy(x)).cuda())
    ref = raw_to_complex(plain.read_cps_raw())
    c = corr.Correlator(N, K, S)
    c.set_tracking(delay=d, delay_rate=r)
    c.process(synth.pack(torch.from_numpy(y)).cuda())
    got = raw_to_complex(c.read_cps_raw())
    assert coef_error(got, ref, N) <= TOL[corr.CORR_FP32]


def test_tracking_off_restores_plain_path():
    N, K, S = 12, 256, 96
    packed = synth.packed(synth.recipe_plain(N=N, two_k=2 * K, seed=2), 0, S).contiguous().cuda()
    fresh = corr.Correlator(N, K, S)
    fresh.process(packed)
    ref = fresh.read_cps_raw()
    c = corr.Correlator(N, K, S)
    c.set_tracking(**_model(N, seed=1))
    c.process(packed)
    tracked = c.read_cps_raw()
    assert not np.array_equal(tracked, ref)
    c.set_tracking()
    c.process(packed)
    np.testing.assert_array_equal(c.read_cps_raw(), ref)


def test_tracking_rejects_bad_values():
    c = corr.Correlator(4, 128, 8)
    with pytest.raises(corr.CorrError) as e:
        c.set_tracking(delay=np.array([0.0, np.nan, 0.0, 0.0]))
    assert e.value.code == corr.CORR_EINVAL
    with pytest.raises(ValueError):
        c.set_tracking(phase=np.zeros(3))
