"""GPU parity of the 16-bit form (the paper's short complex type, here
requantised codes within +-32512 multiplied exactly on the int8 MFMA in
base-255 digits) against the CPU oracle, through the C ABI."""
import numpy as np
import pytest
import torch

import oracle
import paper_1102_0148_amd as corr
import synth
from test_gpu_parity import coef_error

pytestmark = pytest.mark.gpu
QMAX = 32512


@pytest.mark.parametrize("N,K,S,splits", [(44, 256, 200, 0), (5, 128, 33, 0), (64, 128, 40, 0),
                                          (96, 128, 72, 3), (160, 128, 24, 0), (44, 128, 300, 7)])
def test_int16_x_stage_on_oracle_codes(N, K, S, splits):
    """Random codes (extremes included) through corr_process_spectra: exact.
    N = 44 is one 3-block diagonal region; N = 64, 96 and 160 (padded to 192)
    use 2-block diagonal and 2 x 2 off-diagonal regions."""
    print(f"\n[int16 X] N={N} K={K} S={S} splits={splits}", flush=True)
    rng = np.random.default_rng(N * K + S)
    q = rng.integers(-QMAX, QMAX + 1, (S, N, K, 2)).astype(np.int16)
    q[rng.random((S, N, K, 2)) < 0.02] = QMAX
    q[rng.random((S, N, K, 2)) < 0.02] = -QMAX
    buf = torch.from_numpy(corr.spectra_to_records(q, corr.CORR_INT16)).cuda()
    c = corr.Correlator(N, K, S, precision="int16", tiles=dict(x_splits=splits) if splits else None)
    c.process_spectra(buf, S)
    raw = c.read_cps_raw()
    np.testing.assert_array_equal(raw, oracle.cmac_i64_16(q).astype(np.float64))


@pytest.mark.parametrize("N,K,S", [(44, 256, 300), (20, 512, 130), (96, 256, 64)])
def test_int16_end_to_end(N, K, S):
    """Scales by the int16 rule, codes within one of the oracle's rule on the
    oracle's spectra, the X-stage exact on the GPU's own codes, and the
    de-scaled result close to float64."""
    print(f"\n[int16] N={N} K={K} S={S}", flush=True)
    packed = synth.packed(synth.recipe_plain(N=N, two_k=2 * K, seed=N + 2 * K), 0, S).contiguous()
    c = corr.Correlator(N, K, S, precision="int16", tiles=dict(chunk_spectra=(S + 63) // 64 * 64))
    c.process(packed.cuda())
    buf, n = c.debug_read_spectra()
    assert n == S
    scales = c.read_scales()
    raw = c.read_cps_raw()
    q_gpu = corr.records_to_spectra(buf, corr.CORR_INT16, N, K, S)
    np.testing.assert_array_equal(raw, oracle.cmac_i64_16(q_gpu).astype(np.float64))
    spec = oracle.spectra(packed.numpy(), S, N, K)
    W = min(S, corr.CORR_CALIB_SPECTRA)
    np.testing.assert_allclose(scales, oracle.scales_n(spec, W, W, "int16"), rtol=1e-5)
    q_ref = oracle.quantise16(spec, scales)
    diff = q_gpu.astype(np.int32) - q_ref.astype(np.int32)
    assert np.max(np.abs(diff)) <= 1
    # steps 256 times finer than int8's: the float difference between the
    # GPU's and the oracle's spectra meets a rounding tie more often
    assert np.mean(diff != 0) <= 5e-3
    # physical units: the de-scaled result equals the oracle's own int16
    # result under the same rule (the codes differ by at most one in a few of
    # a thousand values), and with full scale at 8 rms nothing clips, so it is
    # within 1e-4 of float64: the 16-bit word's rounding, largest in channels
    # 0 and K/2, whose values are Gaussian integers that a scale just off an
    # integer maps to codes with one coherent rounding error
    c.process(packed.cuda())
    vis = c.read_cps()
    sc_ref = oracle.scales_n(spec, W, W, "int16")
    q_own = oracle.quantise16(spec, sc_ref)
    v16 = oracle.cmac_i64_16(q_own).astype(np.float64)
    den = np.empty((oracle.n_baselines(N), K))
    bl = 0
    for ia in range(N):
        for ib in range(ia, N):
            den[bl] = sc_ref[ia].astype(np.float64) * sc_ref[ib]
            bl += 1
    ref16 = (v16[..., 0] + 1j * v16[..., 1]) / den
    ref64 = oracle.cmac_f64(spec)
    err = coef_error(vis, ref16, N)
    err64 = coef_error(vis, ref64, N)
    print(f"  de-scaled vs the oracle's int16: {err:.3g}; vs float64: {err64:.3g}", flush=True)
    assert err <= 1e-4
    assert err64 <= 1e-4


def test_int16_process_spectra_longer_than_its_splits():
    """corr_process_spectra on more spectra than the handle's splits were
    sized for (chunk 64, one split): 40000 spectra of extreme codes would
    carry a digit cross sum of 4 * 40000 * 127^2 > 2^31 in one partial; the
    library runs them as ranges of at most 16384 spectra per split, so the
    sums stay exact."""
    N, K, S = 8, 128, 40000
    rng = np.random.default_rng(77)
    q = rng.integers(-QMAX, QMAX + 1, (S, N, K, 2)).astype(np.int16)
    q[:, :3] = QMAX          # antennas 0-2 at the largest code throughout
    q[:, 3] = -QMAX
    buf = torch.from_numpy(corr.spectra_to_records(q, corr.CORR_INT16)).cuda()
    c = corr.Correlator(N, K, S, precision="int16", tiles=dict(chunk_spectra=64, x_splits=1))
    c.process_spectra(buf, S)
    raw = c.read_cps_raw()
    np.testing.assert_array_equal(raw, oracle.cmac_i64_16(q).astype(np.float64))
    # no calibration has run: there are no scales to read or de-scale with
    with pytest.raises(corr.CorrError) as e:
        c.read_scales()
    assert e.value.code == corr.CORR_ESTATE
    c.close()


def test_int16_limits():
    """x_splits below chunk / 16384 is refused (digit sums must stay exact in
    int32); batches do not take int16 jobs."""
    N, K, S = 8, 128, 20000
    c = corr.Correlator(N, K, S, precision="int16", tiles=dict(chunk_spectra=20032, x_splits=1))
    with pytest.raises(corr.CorrError) as e:
        c.process(torch.zeros(S * N * K, dtype=torch.uint8, device="cuda"))
    assert e.value.code == corr.CORR_EINVAL
    ok = corr.Correlator(N, K, S, precision="int16", tiles=dict(chunk_spectra=20032))
    assert ok.tiles()["x_splits"] >= 2
    with pytest.raises(corr.CorrError):
        corr.Batch([(8, 128, 16, "int16")])
