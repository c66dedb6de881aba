"""Full-size parity: one whole integration of the N = 44, 512-point, 65536-
spectrum workload in the launch configuration the benchmark times (tiles
from the autotuner's table), checked on sampled outputs the oracle computes
on its own: every baseline among five antennas, every channel.  The reduced
precision forms use the workload with a common tone at bin 77 (0.5 sigma)."""
import numpy as np
import pytest

import oracle
import paper_1102_0148_amd as corr
import synth
from test_gpu_parity import TOL, coef_error, raw_to_complex

pytestmark = pytest.mark.gpu
N, K, S = 44, 256, 65536
ANTS = [0, 7, 21, 38, 43]


def _sel_codes(buf, precision):
    """The integer codes of antennas ANTS from the exported records (without
    converting all 44): [S][len(ANTS)][K][2]."""
    tg = corr.record_times(precision)
    a_pad = corr.a_pad_of(N)
    ntq = ((S + tg - 1) // tg + corr.TQB - 1) // corr.TQB * corr.TQB
    rec = np.asarray(buf)[: ntq * K * a_pad * 16].reshape(ntq // corr.TQB, K, corr.TQB, a_pad, 16)
    sel = np.ascontiguousarray(rec[:, :, :, ANTS, :]).view(np.int8)
    if precision == corr.CORR_INT8:
        v = sel.reshape(ntq // corr.TQB, K, corr.TQB, len(ANTS), 2, tg).astype(np.int16)
    else:
        d = sel.reshape(ntq // corr.TQB, K, corr.TQB, len(ANTS), 2, 2, tg).astype(np.int32)
        v = 255 * d[:, :, :, :, 0] + d[:, :, :, :, 1]          # [tb][K][tr][ant][comp][t]
    # -> [tb][tr][t][ant][K][comp] -> [S][ant][K][2]
    v = np.transpose(v, (0, 2, 5, 3, 1, 4)).reshape(ntq * tg, len(ANTS), K, 2)[:S]
    return v.astype(np.int16 if precision == corr.CORR_INT16 else np.int8)


def _sub(raw, vis_sel):
    """Rows of the full [nb][K] result for the baselines among ANTS, in the
    order of a len(ANTS)-antenna baseline list."""
    rows = [oracle.baseline_index(N, a, b) for i, a in enumerate(ANTS) for b in ANTS[i:]]
    return raw[rows]


@pytest.mark.parametrize("prec", ["fp32", "fp16", "int8", "int16"])
def test_full_integration_sampled_baselines(prec):
    code = corr.PRECISIONS[prec]
    recipe = synth.recipe_plain(N=N, two_k=2 * K, rho=0.05, seed=1) if prec == "fp32" else \
        synth.recipe_tone(N=N, two_k=2 * K, seed=2, tone_bin=77, tone_amp=0.5)
    print(f"\n[full size] {prec} N={N} K={K} S={S}", flush=True)
    packed = synth.packed(recipe, 0, S, device="cuda").contiguous()
    c = corr.Correlator(N, K, S, precision=prec, tiles="auto")
    print(f"  tiles {c.tiles()}", flush=True)
    c.process(packed)
    spec = oracle.spectra(packed[:, ANTS, :].cpu().numpy(), S, len(ANTS), K)
    if prec in ("fp32", "fp16"):
        raw = raw_to_complex(c.read_cps_raw())
        ref = oracle.cmac_f64(spec)
        err = coef_error(_sub(raw, ref), ref, len(ANTS))
        print(f"  coefficient error on {len(ref)} baselines x {K} channels: {err:.3g}", flush=True)
        assert err <= TOL[code]
        return
    buf, n = c.debug_read_spectra()
    assert n == S
    scales = c.read_scales()
    raw = c.read_cps_raw()
    q = _sel_codes(buf, code)
    exact = oracle.cmac_i64(q) if prec == "int8" else oracle.cmac_i64_16(q)
    np.testing.assert_array_equal(_sub(raw, exact), exact.astype(np.float64))
    qref = oracle.quantise(spec, scales[ANTS]) if prec == "int8" else oracle.quantise16(spec, scales[ANTS])
    diff = q.astype(np.int32) - qref.astype(np.int32)
    assert np.max(np.abs(diff)) <= 1
    assert np.mean(diff != 0) <= 1e-3
    qmax = 127.0 if prec == "int8" else 32512.0
    W = corr.CORR_CALIB_SPECTRA
    np.testing.assert_allclose(scales[ANTS], oracle.scales_n(spec, W, W, qmax), rtol=1e-5)
