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
    assert np.mean(diff != 0) <= (1e-3 if prec == "int8" else 5e-3)
    W = corr.CORR_CALIB_SPECTRA
    np.testing.assert_allclose(scales[ANTS], oracle.scales_n(spec, W, W, prec), rtol=1e-5)


def _sel_codes_n(buf, precision, N_, K_, S_, ants):
    """As _sel_codes for another shape."""
    tg = corr.record_times(precision)
    a_pad = corr.a_pad_of(N_)
    ntq = ((S_ + tg - 1) // tg + corr.TQB - 1) // corr.TQB * corr.TQB
    rec = np.asarray(buf)[: ntq * K_ * a_pad * 16].reshape(ntq // corr.TQB, K_, corr.TQB, a_pad, 16)
    sel = np.ascontiguousarray(rec[:, :, :, ants, :]).view(np.int8)
    v = sel.reshape(ntq // corr.TQB, K_, corr.TQB, len(ants), 2, tg)
    v = np.transpose(v, (0, 2, 5, 3, 1, 4)).reshape(ntq * tg, len(ants), K_, 2)[:S_]
    return np.ascontiguousarray(v)


@pytest.mark.parametrize("prec", ["fp32", "int8"])
def test_large_n_full_size_sampled_baselines(prec):
    """N = 256, 1024-point, 16384 spectra with three delayed sources, in the
    benchmark's launch configuration: antennas from different 64-antenna
    region rows, so the sampled baselines fall in diagonal and off-diagonal
    regions (LDS-staged groups for int8)."""
    N_, K_, S_ = 256, 512, 16384
    ants = [0, 37, 70, 130, 200, 255]
    packed = synth.packed(synth.recipe_sources(N=N_, two_k=2 * K_, seed=4), 0, S_, device="cuda").contiguous()
    c = corr.Correlator(N_, K_, S_, precision=prec, tiles="auto")
    print(f"\n[large N] {prec} tiles {c.tiles()}", flush=True)
    c.process(packed)
    spec = oracle.spectra(packed[:, ants, :].cpu().numpy(), S_, len(ants), K_)
    rows = [oracle.baseline_index(N_, a, b) for i, a in enumerate(ants) for b in ants[i:]]
    if prec == "fp32":
        raw = raw_to_complex(c.read_cps_raw())
        ref = oracle.cmac_f64(spec)
        err = coef_error(raw[rows], ref, len(ants))
        print(f"  coefficient error {err:.3g}", flush=True)
        assert err <= TOL[corr.CORR_FP32]
        return
    buf, n = c.debug_read_spectra()
    raw = c.read_cps_raw()
    q = _sel_codes_n(buf, corr.CORR_INT8, N_, K_, S_, ants)
    np.testing.assert_array_equal(raw[rows], oracle.cmac_i64(q).astype(np.float64))


@pytest.mark.parametrize("mode", ["branches", "persistent"])
def test_batch_full_size_sampled_baselines(mode):
    """The 12-job batch of the benchmark (16384 spectra per job, int8 and
    fp32 alternating) with the autotuner's tiles, in both modes: the
    persistent kernel then runs its tuned x_splits and F items of 16-64
    tiles.  Every job's baselines among its first, a middle and its last
    antenna are checked: fp32 jobs against the float64 oracle; int8 jobs
    first bit for bit against a single-job correlator of the same shape
    (same calibration, so the same scales and codes), then bit for bit
    against the integer oracle on that correlator's exported codes."""
    recipes = synth.batch_jobs(12, seed=3)
    S_ = 16384
    jobs = [(r.N, r.K, S_, "fp32" if j % 2 == 0 else "int8") for j, r in enumerate(recipes)]
    xs = [synth.packed(r, 0, S_, device="cuda").contiguous() for r in recipes]
    print(f"\n[batch full size] {mode}", flush=True)
    b = corr.Batch(jobs, tiles="auto", mode=mode)
    b.process(xs)
    for j, (r, (N_, K_, _, prec)) in enumerate(zip(recipes, jobs)):
        ants = sorted({0, N_ // 2, N_ - 1})
        raw = b.read_cps_raw(j)
        rows = [oracle.baseline_index(N_, a, c) for i, a in enumerate(ants) for c in ants[i:]]
        if prec == "fp32":
            spec = oracle.spectra(xs[j][:, ants, :].cpu().numpy(), S_, len(ants), K_)
            err = coef_error(raw_to_complex(raw)[rows], oracle.cmac_f64(spec), len(ants))
            print(f"  job {j} N={N_} K={K_} fp32: {err:.3g}", flush=True)
            assert err <= TOL[corr.CORR_FP32]
            continue
        single = corr.Correlator(N_, K_, S_, precision="int8", tiles=dict(chunk_spectra=S_))
        single.process(xs[j])
        buf, n = single.debug_read_spectra()
        assert n == S_
        np.testing.assert_array_equal(b.read_scales(j), single.read_scales())
        np.testing.assert_array_equal(raw, single.read_cps_raw(), err_msg=f"job {j}: batch != single job")
        q = _sel_codes_n(buf, corr.CORR_INT8, N_, K_, S_, ants)
        np.testing.assert_array_equal(raw[rows], oracle.cmac_i64(q).astype(np.float64))
        print(f"  job {j} N={N_} K={K_} int8: bit-exact", flush=True)
        single.close()
        del buf
    b.close()


@pytest.mark.parametrize("prec", ["fp32", "fp16", "int8", "int16"])
def test_maximum_shape_sampled_baselines(prec):
    """The largest shape the library accepts: 512 antennas (eight 64-antenna
    region rows), 1024 channels (a 2048-point FFT), and a ragged 45 spectra
    (not a whole record in any form). Checked on baselines among antennas at
    the region edges."""
    N_, K_, S_ = corr.CORR_MAX_ANTENNAS, corr.CORR_MAX_CHANNELS, 45
    ants = [0, 1, 63, 64, 255, 256, 447, 510, 511]
    code = corr.PRECISIONS[prec]
    recipe = synth.recipe_plain(N=N_, two_k=2 * K_, rho=0.05, seed=9) if prec in ("fp32", "fp16") else \
        synth.recipe_tone(N=N_, two_k=2 * K_, seed=10, tone_bin=300, tone_amp=0.5)
    print(f"\n[max shape] {prec} N={N_} K={K_} S={S_}", flush=True)
    packed = synth.packed(recipe, 0, S_, device="cuda").contiguous()
    c = corr.Correlator(N_, K_, S_, precision=prec)
    c.process(packed)
    rows = [oracle.baseline_index(N_, a, b) for i, a in enumerate(ants) for b in ants[i:]]
    spec = oracle.spectra(packed[:, ants, :].cpu().numpy(), S_, len(ants), K_)
    raw = c.read_cps_raw()[rows]
    if prec in ("fp32", "fp16"):
        err = coef_error(raw_to_complex(raw), oracle.cmac_f64(spec), len(ants))
        print(f"  coefficient error {err:.3g}", flush=True)
        assert err <= TOL[code]
        return
    buf, n = c.debug_read_spectra()
    assert n == S_
    if prec == "int8":
        q = _sel_codes_n(buf, code, N_, K_, S_, ants)
        exact = oracle.cmac_i64(q)
    else:
        tg = corr.record_times(code)
        a_pad = corr.a_pad_of(N_)
        ntq = ((S_ + tg - 1) // tg + corr.TQB - 1) // corr.TQB * corr.TQB
        rec = np.asarray(buf)[: ntq * K_ * a_pad * 16].reshape(ntq // corr.TQB, K_, corr.TQB, a_pad, 16)
        d = np.ascontiguousarray(rec[:, :, :, ants, :]).view(np.int8)
        d = d.reshape(ntq // corr.TQB, K_, corr.TQB, len(ants), 2, 2, tg).astype(np.int32)
        v = 255 * d[:, :, :, :, 0] + d[:, :, :, :, 1]
        q = np.transpose(v, (0, 2, 5, 3, 1, 4)).reshape(ntq * tg, len(ants), K_, 2)[:S_].astype(np.int16)
        exact = oracle.cmac_i64_16(q)
    np.testing.assert_array_equal(raw, exact.astype(np.float64))
    c.close()


@pytest.mark.parametrize("prec,chunk,splits", [("int8", 8192, 2), ("fp32", 2048, 1)])
def test_cache_sized_chunks_full_integration(prec, chunk, splits):
    """A whole 65536-spectrum integration processed in chunks whose records
    fit the 256 MB Infinity Cache (int8: 8192 spectra, 201 MB; fp32: 2048
    spectra, 201 MB), so the X-stage reads each chunk soon after the F-stage
    wrote it: the same results as the whole-integration tiling."""
    code = corr.PRECISIONS[prec]
    recipe = synth.recipe_plain(N=N, two_k=2 * K, rho=0.05, seed=1) if prec == "fp32" else \
        synth.recipe_tone(N=N, two_k=2 * K, seed=2, tone_bin=77, tone_amp=0.5)
    print(f"\n[cache-sized chunks] {prec} chunk={chunk}", flush=True)
    packed = synth.packed(recipe, 0, S, device="cuda").contiguous()
    c = corr.Correlator(N, K, S, precision=prec, tiles=dict(chunk_spectra=chunk, x_splits=splits))
    c.process(packed)
    spec = oracle.spectra(packed[:, ANTS, :].cpu().numpy(), S, len(ANTS), K)
    raw = c.read_cps_raw()
    if prec == "fp32":
        ref = oracle.cmac_f64(spec)
        err = coef_error(_sub(raw_to_complex(raw), ref), ref, len(ANTS))
        print(f"  coefficient error {err:.3g}", flush=True)
        assert err <= TOL[code]
        return
    # the integer sums of the whole integration over the records of every
    # chunk equal the whole-integration tiling's, bit for bit
    w = corr.Correlator(N, K, S, precision=prec, tiles="auto")
    w.process(packed)
    np.testing.assert_array_equal(_sub(raw, None), _sub(w.read_cps_raw(), None))
    np.testing.assert_array_equal(c.read_scales(), w.read_scales())
