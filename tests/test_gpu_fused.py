"""GPU parity of the fused F -> X pipeline (one persistent kernel per
integration: F workgroups fill a ring of record slots chunk by chunk, X
workgroups keep their accumulators across chunks) against the CPU oracle and
against the staged pipeline, through the C ABI."""
import numpy as np
import pytest
import torch

import oracle
import paper_1102_0148_amd as corr
import synth
from test_gpu_parity import TOL, coef_error, raw_to_complex

pytestmark = pytest.mark.gpu


def _packed(N, K, S, seed, tone=False):
    r = synth.recipe_tone(N=N, two_k=2 * K, seed=seed, tone_bin=K // 3, tone_amp=0.5) if tone else \
        synth.recipe_plain(N=N, two_k=2 * K, rho=0.05, seed=seed)
    return synth.packed(r, 0, S).contiguous()


def _fused(N, K, S, prec, packed, **params):
    c = corr.Correlator(N, K, S, precision=prec, pipeline=params or "fused")
    c.process(packed)
    return c


# (N, K, S, chunk, ring, F workgroups per CU, F CUs per XCD): several chunks
# with a ragged last one, ring depths 1-3, one and two antenna blocks (N = 8,
# 20) and three (N = 44); the mixed role layout and the split one
CASES = [(44, 256, 3000, 512, 3, 0, 0), (44, 256, 1000, 256, 1, 0, 0), (20, 512, 700, 128, 2, 0, 0),
         (8, 128, 2500, 1024, 2, 0, 0), (44, 1024, 300, 64, 3, 0, 0), (33, 256, 1200, 384, 2, 1, 0),
         (44, 256, 3000, 512, 3, 0, 12), (20, 512, 1100, 256, 2, 0, 4), (8, 128, 700, 64, 1, 0, 20)]


@pytest.mark.parametrize("N,K,S,chunk,ring,fpc,fcus", CASES)
@pytest.mark.parametrize("prec", ["fp32", "fp16", "int8"])
def test_fused_matches_oracle_and_staged(prec, N, K, S, chunk, ring, fpc, fcus):
    print(f"\n[fused] {prec} N={N} K={K} S={S} chunk={chunk} ring={ring} fpc={fpc} fcus={fcus}", flush=True)
    packed = _packed(N, K, S, seed=N + K + S, tone=prec != "fp32")
    x = packed.cuda()
    c = _fused(N, K, S, prec, x, chunk_spectra=chunk, ring_slots=ring, f_workgroups_per_cu=fpc,
               f_cus_per_xcd=fcus)
    print(f"  tiles {c.tiles()}", flush=True)
    raw = c.read_cps_raw()
    if prec == "int8":
        # same calibration and codes as the staged pipeline: identical sums
        s = corr.Correlator(N, K, S, precision=prec)
        s.process(x)
        np.testing.assert_array_equal(c.read_scales(), s.read_scales())
        np.testing.assert_array_equal(raw, s.read_cps_raw())
        # the codes of the last chunk's ring slot against the oracle's rule
        buf, n = c.debug_read_spectra()
        assert n == S - (S - 1) // chunk * chunk
        q = corr.records_to_spectra(buf, corr.CORR_INT8, N, K, n)
        spec = oracle.spectra(packed[S - n:].numpy(), n, N, K)
        diff = q.astype(np.int32) - oracle.quantise(spec, c.read_scales()).astype(np.int32)
        assert np.max(np.abs(diff)) <= 1 and np.mean(diff != 0) <= 1e-3
        return
    ref = oracle.correlate(packed.numpy(), S, N, K)
    err = coef_error(raw_to_complex(raw), ref, N)
    print(f"  coefficient error {err:.3g}", flush=True)
    assert err <= TOL[corr.PRECISIONS[prec]]


def test_fused_full_integration_sampled_baselines():
    """One whole N = 44, 512-point, 65536-spectrum integration, default fused
    parameters: fp32 against float64 on the baselines among five antennas,
    int8 identical to the staged pipeline."""
    N, K, S = 44, 256, 65536
    ants = [0, 7, 21, 38, 43]
    rows = [oracle.baseline_index(N, a, b) for i, a in enumerate(ants) for b in ants[i:]]
    packed = synth.packed(synth.recipe_plain(N=N, two_k=2 * K, rho=0.05, seed=1), 0, S, device="cuda").contiguous()
    c = corr.Correlator(N, K, S, precision="fp32", pipeline="fused")
    c.process(packed)
    print(f"\n[fused full size] fp32 tiles {c.tiles()}", flush=True)
    spec = oracle.spectra(packed[:, ants, :].cpu().numpy(), S, len(ants), K)
    ref = oracle.cmac_f64(spec)
    err = coef_error(raw_to_complex(c.read_cps_raw())[rows], ref, len(ants))
    print(f"  coefficient error {err:.3g}", flush=True)
    assert err <= TOL[corr.CORR_FP32]
    f8 = corr.Correlator(N, K, S, precision="int8", pipeline="fused")
    f8.process(packed)
    s8 = corr.Correlator(N, K, S, precision="int8", tiles="auto")
    s8.process(packed)
    np.testing.assert_array_equal(f8.read_cps_raw(), s8.read_cps_raw())


def test_fused_integrations_accumulate_and_replay():
    """Two integrations add up in the float64 buffer, and a handle runs the
    kernel again with the counters cleared each time (same result twice)."""
    N, K, S = 12, 256, 900
    x = _packed(N, K, S, seed=3).cuda()
    c = _fused(N, K, S, "fp32", x, chunk_spectra=128, ring_slots=2)
    one = c.read_cps_raw()
    c.process(x)
    c.process(x)
    two = c.read_cps_raw()
    np.testing.assert_array_equal(two, 2 * one)
    c.process(x)
    np.testing.assert_array_equal(c.read_cps_raw(), one)


def test_fused_refuses_what_it_does_not_cover():
    x = torch.zeros(64 * 64 * 256, dtype=torch.uint8, device="cuda")
    for N, prec in ((64, "fp32"), (8, "int16")):
        c = corr.Correlator(N, 256, 64, precision=prec, pipeline="fused")
        with pytest.raises(corr.CorrError) as e:
            c.process(x[: 64 * N * 256])
        assert e.value.code == corr.CORR_EINVAL
    c = corr.Correlator(8, 256, 64, pipeline="fused")
    c.set_tracking(delay=np.ones(8))
    with pytest.raises(corr.CorrError) as e:
        c.process(x[: 64 * 8 * 256])
    assert e.value.code == corr.CORR_EINVAL
    c = corr.Correlator(8, 256, 64)
    c.process(x[: 64 * 8 * 256])
    with pytest.raises(corr.CorrError) as e:
        corr.corr_set_pipeline(c.h, corr.CORR_PIPELINE_FUSED)
    assert e.value.code == corr.CORR_ESTATE
    with pytest.raises(corr.CorrError) as e:
        corr.corr_set_pipeline(c.h, 5)
    assert e.value.code == corr.CORR_EINVAL
    # both role layouts at once, and a split that leaves no X CUs
    c = corr.Correlator(8, 256, 64)
    with pytest.raises(corr.CorrError) as e:
        corr.corr_set_pipeline(c.h, corr.CORR_PIPELINE_FUSED, 0, 0, 1, 4)
    assert e.value.code == corr.CORR_EINVAL
    c = corr.Correlator(8, 256, 64, pipeline={"f_cus_per_xcd": 32})
    with pytest.raises(corr.CorrError) as e:
        c.process(x[: 64 * 8 * 256])
    assert e.value.code == corr.CORR_EINVAL


def test_autotuned_fused_gives_way_to_tracking():
    """Where the autotuner table picked the fused pipeline (fp16, N = 44,
    512-point, 65536 spectra), switching tracking on before the first
    process() moves the handle to the staged pipeline with the table's staged
    tiles; an explicit fused request keeps refusing tracking."""
    from paper_1102_0148_amd import tune
    N, K, S = 44, 256, 65536
    found = tune.lookup(N, K, S, "fp16")
    if not found or found.get("pipeline") != "fused":
        pytest.skip("the autotuner table does not pick the fused pipeline for this shape")
    c = corr.Correlator(N, K, S, precision="fp16", tiles="auto")
    assert c.pipeline == "fused"
    c.set_tracking(delay=np.full(N, 3.0))
    assert c.pipeline == "staged"
    assert {k: c.tiles()[k] for k in ("chunk_spectra", "x_splits", "f_group")} == \
        {k: found[k] for k in ("chunk_spectra", "x_splits", "f_group")}
    x = torch.zeros(S * N * K, dtype=torch.uint8, device="cuda")
    c.process(x)
    assert np.all(c.read_cps_raw() == 0)
    e = corr.Correlator(N, K, S, precision="fp16", pipeline="fused")
    e.set_tracking(delay=np.full(N, 3.0))
    with pytest.raises(corr.CorrError) as err:
        e.process(x)
    assert err.value.code == corr.CORR_EINVAL
