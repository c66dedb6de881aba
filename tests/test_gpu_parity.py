"""GPU parity: the HIP path through the C ABI against the CPU oracle, on the
same seeded inputs.  Needs an MI355X and the built libcorr.so.

Tolerances (coefficient units, |V - V64| / sqrt(V64_aa V64_bb), the error a
visibility carries relative to the noise power of its two antennas):
  fp32: 1e-5    float spectra and float MFMA sums over <= 2048 spectra per
                partial; the float FFT alone is good to ~1e-7 per bin
  fp16: 2e-3    half-precision spectra (2^-11 relative) dominate
  int8: exact   against the integer oracle on the same quantised spectra
"""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_1102_0148_amd as corr
import synth

pytestmark = pytest.mark.gpu

TOL = {corr.CORR_FP32: 1e-5, corr.CORR_FP16: 2e-3}


def _packed(recipe, S, device="cuda"):
    return synth.packed(recipe, 0, S, device="cpu").contiguous().to(device)


def coef_error(v, ref, N):
    """max over baselines and channels of |v - ref| / sqrt(ref_aa ref_bb)."""
    nb, K = ref.shape
    auto = np.empty((N, K))
    for a in range(N):
        auto[a] = ref[oracle.baseline_index(N, a, a)].real
    err = 0.0
    bl = 0
    for a in range(N):
        for b in range(a, N):
            den = np.sqrt(np.maximum(auto[a] * auto[b], 1e-300))
            err = max(err, float(np.max(np.abs(v[bl] - ref[bl]) / den)))
            bl += 1
    return err


def raw_to_complex(raw):
    return raw[..., 0] + 1j * raw[..., 1]


def run(N, K, S, packed, precision=corr.CORR_FP32, tiles=None):
    c = corr.Correlator(N, K, S, precision=precision, tiles=tiles)
    c.process(packed)
    raw = c.read_cps_raw()
    return c, raw


# ------------------------------------------------------------------ F-stage

@pytest.mark.parametrize("K", [128, 256, 512, 1024])
def test_fstage_fp32_spectra_match_oracle(K):
    N, S = 5, 11
    print(f"\n[fstage] N={N} K={K} S={S}", flush=True)
    r = synth.recipe_plain(N=N, two_k=2 * K, seed=31)
    packed = _packed(r, S)
    c, _ = run(N, K, S, packed)
    buf, n = c.debug_read_spectra()
    assert n == S
    got = corr.records_to_spectra(buf, corr.CORR_FP32, N, K, S)
    ref = oracle.spectra(packed.cpu().numpy(), S, N, K)
    scale = np.sqrt(np.mean(np.abs(ref) ** 2))
    assert np.max(np.abs(got - ref)) <= 2e-6 * scale * math.log2(2 * K)
    # bins 0 and K/2 are Gaussian integers, exact in float
    np.testing.assert_array_equal(got[:, :, 0], ref[:, :, 0].round())
    np.testing.assert_array_equal(got[:, :, K // 2], ref[:, :, K // 2].round())


@pytest.mark.parametrize("K", [256, 512])
def test_matrix_core_transform_spectra(K):
    """The transform of the reduced-precision records (on the matrix cores at
    K = 256 and 512) through fp16 records: every value within half an f16
    step (the record's rounding) plus the fp32 transform's error budget of
    the float64 oracle's spectrum, and bins 0 and K/2 (integers, here below
    2048) bit for bit."""
    N, S = 5, 12
    print(f"\n[matrix-core transform] N={N} K={K} S={S}", flush=True)
    r = synth.recipe_plain(N=N, two_k=2 * K, seed=41)
    packed = _packed(r, S)
    c = corr.Correlator(N, K, S, precision="fp16")
    c.process(packed)
    buf, n = c.debug_read_spectra()
    assert n == S
    got = corr.records_to_spectra(buf, corr.CORR_FP16, N, K, S)
    ref = oracle.spectra(packed.cpu().numpy(), S, N, K)
    budget = 2e-6 * np.sqrt(np.mean(np.abs(ref) ** 2)) * math.log2(2 * K)
    for g, x in ((got.real, ref.real), (got.imag, ref.imag)):
        step = 2.0 ** (np.floor(np.log2(np.maximum(np.abs(x), 2.0 ** -14))) - 10)
        excess = np.abs(g - x) - 0.5 * step
        assert np.all(excess <= budget), np.max(excess) / budget
    for b in (0, K // 2):
        assert np.max(np.abs(ref[:, :, b])) < 2048
        np.testing.assert_array_equal(got[:, :, b], ref[:, :, b].round())


@pytest.mark.parametrize("K", [256, 512])
def test_matrix_core_transform_extreme_samples(K):
    """The matrix-core transform (fp16 records) on the largest sample
    magnitudes: all -8, all 7, and 7 / -8 alternating.  Bin 0 is the sum of
    the samples (-16K, 14K and -K, exact in f16) bit for bit, bin K/2 is
    exactly zero, and every other bin is zero within the transform's error
    budget (the split halves of the twiddles leave residues of order 2^-21 of
    the complex transform's bin 0, K |x[2m] + i x[2m+1]| <= 8 sqrt(2) K)."""
    N, S = 3, 4
    print(f"\n[matrix-core transform, extreme samples] K={K}", flush=True)
    x = torch.full((S, N, 2 * K), -8, dtype=torch.int8)
    x[:, 1] = 7
    x[:, 2, 0::2] = 7
    x[:, 2, 1::2] = -8
    packed = synth.pack(x).cuda()
    c = corr.Correlator(N, K, S, precision="fp16")
    c.process(packed)
    buf, n = c.debug_read_spectra()
    assert n == S
    got = corr.records_to_spectra(buf, corr.CORR_FP16, N, K, S)
    ref = oracle.spectra(packed.cpu().numpy(), S, N, K)
    for a, dc in enumerate((-8 * 2 * K, 7 * 2 * K, -K)):
        np.testing.assert_array_equal(ref[:, a, 0], dc)
        np.testing.assert_array_equal(got[:, a, 0], dc)
        np.testing.assert_array_equal(got[:, a, K // 2], 0)
        rest = np.delete(got[:, a], [0, K // 2], axis=1)
        assert np.max(np.abs(rest)) <= 2e-6 * 8 * math.sqrt(2) * K * math.log2(2 * K), np.max(np.abs(rest))
    c.close()


def test_fstage_extreme_samples():
    """All -8 and all 7 samples (largest magnitudes): DC = 2K x, other bins 0."""
    N, K, S = 3, 256, 4
    x = torch.full((S, N, 2 * K), -8, dtype=torch.int8)
    x[:, 1] = 7
    x[:, 2, 0::2] = 7
    x[:, 2, 1::2] = -8
    packed = synth.pack(x).cuda()
    c, _ = run(N, K, S, packed)
    buf, _ = c.debug_read_spectra()
    got = corr.records_to_spectra(buf, corr.CORR_FP32, N, K, S)
    ref = oracle.spectra(packed.cpu().numpy(), S, N, K)
    np.testing.assert_array_equal(got[:, 0, 0], -8 * 2 * K)
    np.testing.assert_array_equal(got[:, 1, 0], 7 * 2 * K)
    assert np.max(np.abs(got - ref)) <= 1e-3


@pytest.mark.parametrize("N,prec,tiles", [(5, "fp32", None), (20, "fp16", None), (2, "int8", None),
                                           (33, "int16", None), (44, "fp32", dict(f_group=16)),
                                           (5, "fp32", dict(f_group=16))])
def test_padding_records_stay_zero(N, prec, tiles):
    """Records of the padding antennas (N up to the 16-antenna block) hold
    zeros after two integrations in the same buffer, whether the F-stage
    stores them as zeros (padding sharing a 128-byte line with real antennas;
    a float record may then hold -0.0) or never stores them (padding in lines
    of its own)."""
    K, S = 128, 40
    print(f"\n[padding] N={N} {prec} tiles={tiles}", flush=True)
    c = corr.Correlator(N, K, S, precision=prec, tiles=tiles)
    for seed in (61, 62):
        c.process(_packed(synth.recipe_plain(N=N, two_k=2 * K, seed=seed), S))
        buf, n = c.debug_read_spectra()
        c.read_cps()  # the integer forms need each integration read before the next
    a_pad = corr.a_pad_of(N)
    dt = {"fp32": np.float32, "fp16": np.float16, "int8": np.int8, "int16": np.int8}[prec]
    rec = buf.view(dt).reshape(-1, K, corr.TQB, a_pad, 16 // np.dtype(dt).itemsize)
    assert np.all(rec[:, :, :, N:] == 0)
    assert np.any(rec[:, :, :, :N] != 0)
    c.close()


# ------------------------------------------------------------------ FP32 end to end

@pytest.mark.parametrize("N,K,S", [(44, 256, 1024), (5, 128, 37), (20, 512, 100), (16, 1024, 24),
                                   (2, 256, 1), (96, 256, 64)])
def test_fp32_end_to_end(N, K, S):
    print(f"\n[fp32] N={N} K={K} S={S}", flush=True)
    r = synth.recipe_plain(N=N, two_k=2 * K, seed=N * 7 + K)
    packed = _packed(r, S)
    c, raw = run(N, K, S, packed)
    ref = oracle.correlate(packed.cpu().numpy(), S, N, K)
    v = raw_to_complex(raw)
    assert coef_error(v, ref, N) <= TOL[corr.CORR_FP32]
    for a in range(N):
        bl = oracle.baseline_index(N, a, a)
        assert np.all(raw[bl, :, 1] == 0.0) and np.all(raw[bl, :, 0] >= 0.0)


@pytest.mark.parametrize("N,K,S,splits", [(256, 512, 24, 0), (160, 128, 40, 0), (200, 128, 104, 1),
                                          (256, 128, 104, 3), (193, 256, 40, 2)])
def test_fp32_large_n_regions(N, K, S, splits):
    """N above 96 uses the multi-region X-stage: N = 160 (padded to 192)
    the diagonal and off-diagonal launches, N from 193 to 256 (16 blocks)
    the whole-channel groups, over k-block ranges that are whole rounds of
    the ring and ragged ones."""
    print(f"\n[fp32 large N] N={N} K={K} S={S} splits={splits}", flush=True)
    r = synth.recipe_sources(N=N, two_k=2 * K, seed=4)
    packed = _packed(r, S)
    c, raw = run(N, K, S, packed, tiles=dict(x_splits=splits) if splits else None)
    ref = oracle.correlate(packed.cpu().numpy(), S, N, K)
    assert coef_error(raw_to_complex(raw), ref, N) <= TOL[corr.CORR_FP32]


@pytest.mark.parametrize("N,K,S,splits", [(256, 128, 72, 0), (200, 128, 104, 3)])
def test_fp16_whole_channel_groups(N, K, S, splits):
    """fp16 at N from 193 to 256 runs the whole-channel X-stage groups: end
    to end against the float64 oracle within the fp16 bound, over whole and
    ragged split ranges."""
    print(f"\n[fp16 whole-channel] N={N} K={K} S={S} splits={splits}", flush=True)
    packed = _packed(synth.recipe_sources(N=N, two_k=2 * K, seed=5), S)
    c, raw = run(N, K, S, packed, precision=corr.CORR_FP16, tiles=dict(x_splits=splits) if splits else None)
    ref = oracle.correlate(packed.cpu().numpy(), S, N, K)
    assert coef_error(raw_to_complex(raw), ref, N) <= TOL[corr.CORR_FP16]


@pytest.mark.parametrize("tiles", [dict(chunk_spectra=64, x_splits=1, f_group=2),
                                   dict(chunk_spectra=128, x_splits=3, f_group=4),
                                   dict(chunk_spectra=256, x_splits=64, f_group=8)])
def test_fp32_tile_invariance(tiles):
    N, K, S = 44, 256, 300
    r = synth.recipe_plain(N=N, two_k=2 * K, seed=5)
    packed = _packed(r, S)
    _, raw = run(N, K, S, packed, tiles=tiles)
    ref = oracle.correlate(packed.cpu().numpy(), S, N, K)
    assert coef_error(raw_to_complex(raw), ref, N) <= TOL[corr.CORR_FP32]


def test_fp32_deterministic_and_read_clears():
    N, K, S = 44, 256, 512
    r = synth.recipe_plain(N=N, two_k=2 * K, seed=6)
    packed = _packed(r, S)
    c = corr.Correlator(N, K, S)
    c.process(packed)
    a = c.read_cps_raw()
    c.process(packed)
    b = c.read_cps_raw()
    np.testing.assert_array_equal(a, b)
    # two integrations accumulate: equals twice one (exactly, in float64 of
    # identical float partials)
    c.process(packed)
    c.process(packed)
    two = c.read_cps_raw()
    np.testing.assert_array_equal(two, 2 * a)


def test_async_read_matches_sync_read():
    N, K, S = 12, 256, 64
    packed = _packed(synth.recipe_plain(N=N, two_k=2 * K, seed=8), S)
    c = corr.Correlator(N, K, S)
    c.process(packed)
    dst = torch.empty(c.nb * K * 2, dtype=torch.float64, device="cuda")
    c.read_cps_async(dst)
    c.process(packed)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(dst.cpu().numpy().reshape(c.nb, K, 2), c.read_cps_raw())


def test_zero_input_gives_zero():
    N, K, S = 20, 256, 40
    packed = torch.zeros(S * N * K, dtype=torch.uint8, device="cuda")
    for prec in (corr.CORR_FP32, corr.CORR_FP16, corr.CORR_INT8):
        _, raw = run(N, K, S, packed, precision=prec)
        assert np.all(raw == 0.0)


# ------------------------------------------------------------------ INT8

def _int8_run(N, K, S, seed, tiles=None):
    r = synth.recipe_tone(N=N, two_k=2 * K, seed=seed)
    packed = _packed(r, S)
    c = corr.Correlator(N, K, S, precision="int8", tiles=tiles)
    c.process(packed)
    scales = c.read_scales()
    buf, n = c.debug_read_spectra()
    raw = c.read_cps_raw()
    return c, packed, scales, buf, n, raw


@pytest.mark.parametrize("N,K,S", [(44, 256, 1024), (7, 128, 45), (33, 512, 130)])
def test_int8_bit_exact_on_gpu_spectra(N, K, S):
    """The int64 oracle X-stage on the GPU's own int8 spectra equals the GPU
    result exactly; the GPU scales and quantised spectra follow the oracle's
    rule on the oracle's spectra."""
    print(f"\n[int8] N={N} K={K} S={S}", flush=True)
    tiles = dict(chunk_spectra=round_up(S, 64))  # one chunk, so it is exported whole
    c, packed, scales, buf, n, raw = _int8_run(N, K, S, seed=N + K, tiles=tiles)
    assert n == S
    q_gpu = corr.records_to_spectra(buf, corr.CORR_INT8, N, K, S)
    vi = oracle.cmac_i64(q_gpu)
    np.testing.assert_array_equal(raw, vi.astype(np.float64))
    spec = oracle.spectra(packed.cpu().numpy(), S, N, K)
    sc_ref = oracle.scales(spec, min(S, corr.CORR_CALIB_SPECTRA))
    np.testing.assert_allclose(scales, sc_ref, rtol=1e-5)
    q_ref = oracle.quantise(spec, scales)
    diff = q_gpu.astype(np.int32) - q_ref.astype(np.int32)
    assert np.max(np.abs(diff)) <= 1
    assert np.mean(diff != 0) <= 1e-3


@pytest.mark.parametrize("N,K,S,splits", [(44, 256, 200, 0), (64, 128, 33, 0), (256, 256, 16, 0),
                                          (160, 128, 24, 0), (256, 128, 200, 1), (256, 128, 200, 3),
                                          (200, 128, 136, 2)])
def test_int8_x_stage_on_oracle_spectra(N, K, S, splits):
    """Oracle-quantised spectra through corr_process_spectra: bit-exact.
    N = 160 (padded to 192) runs both region kinds in one launch; N = 256 and
    N = 200 (padded to 256) run the LDS-staged region groups, over k-block
    ranges that are whole rounds of the ring and ragged ones."""
    rng = np.random.default_rng(N * K + S)
    q = rng.integers(-127, 128, (S, N, K, 2)).astype(np.int8)
    q[:, :, :, :][rng.random((S, N, K, 2)) < 0.01] = 127
    buf = torch.from_numpy(corr.spectra_to_records(q, corr.CORR_INT8)).cuda()
    c = corr.Correlator(N, K, S, precision="int8", tiles=dict(x_splits=splits) if splits else None)
    c.process_spectra(buf, S)
    raw = c.read_cps_raw()
    np.testing.assert_array_equal(raw, oracle.cmac_i64(q).astype(np.float64))


def test_int8_tile_invariance_exact():
    N, K, S = 44, 256, 700
    outs = []
    for tiles in (dict(chunk_spectra=64, x_splits=1, f_group=2), dict(chunk_spectra=704, x_splits=7, f_group=8),
                  dict(chunk_spectra=128, x_splits=3, f_group=1)):
        _, _, _, _, _, raw = _int8_run(N, K, S, seed=3, tiles=tiles)
        outs.append(raw)
    np.testing.assert_array_equal(outs[0], outs[1])
    np.testing.assert_array_equal(outs[0], outs[2])


@pytest.mark.parametrize("prec,groups", [("fp32", (1, 2, 4, 8, 16)), ("fp16", (1, 2, 4, 8)),
                                         ("int8", (1, 2, 4, 8))])
def test_fstage_bit_identical_across_groups(prec, groups):
    """The F-stage's arithmetic is fully specified (explicit fused
    multiply-adds), so every tile shape gives the same bits."""
    N, K, S = 44, 256, 300
    packed = _packed(synth.recipe_tone(N=N, two_k=2 * K, seed=3), S)
    ref = None
    for g in groups:
        c = corr.Correlator(N, K, S, precision=prec, tiles=dict(chunk_spectra=320, f_group=g))
        c.process(packed)
        buf, n = c.debug_read_spectra()
        c.read_cps_raw()
        sp = corr.records_to_spectra(buf, corr.PRECISIONS[prec], N, K, n)
        if ref is None:
            ref = sp
        else:
            np.testing.assert_array_equal(sp, ref)


@pytest.mark.parametrize("prec,lim", [("int8", 127), ("int16", 32512)])
def test_saturation_count_matches_oracle_spectra(prec, lim):
    """The saturation counter counts the components whose rounded code lies
    beyond the clamp (Section 4's conversion to short integers).  The
    calibration window is three times quieter than the rest, so the later
    spectra clip often (int8 at 4 rms of the window: about one component in
    six; int16 at 8: about one in two hundred).  Expected: the components of
    the oracle's spectra, times the GPU's scales, that round beyond the
    clamp; only components within rounding of the bound may differ."""
    N, K, S, W = 12, 256, 1536, corr.CORR_CALIB_SPECTRA
    x = synth.samples(synth.recipe_plain(N=N, two_k=2 * K, seed=21), 0, S)
    x[:W] = torch.round(x[:W].float() / 3).to(torch.int8)
    packed = synth.pack(x).contiguous()
    print(f"\n[saturation] {prec} N={N} K={K} S={S}", flush=True)
    c = corr.Correlator(N, K, S, precision=prec, tiles=dict(chunk_spectra=S))
    c.process(packed.cuda())
    got = c.stats()["int8_saturated"]
    scales = c.read_scales()
    buf, n = c.debug_read_spectra()
    assert n == S
    spec = oracle.spectra(packed.numpy(), S, N, K)
    v = np.stack([spec.real, spec.imag], -1) * scales[None, :, :, None].astype(np.float64)
    want = int(np.count_nonzero(np.abs(np.rint(v)) > lim))
    assert want > (S - W) * N * K * 2 // (10 if prec == "int8" else 1000)
    assert abs(got - want) <= 2 + want // 10000, (got, want)
    # the codes themselves, clamped ones included, follow the oracle's rule
    mode = corr.CORR_INT8 if prec == "int8" else corr.CORR_INT16
    q_gpu = corr.records_to_spectra(buf, mode, N, K, S).astype(np.int32)
    q_ref = (oracle.quantise if prec == "int8" else oracle.quantise16)(spec, scales).astype(np.int32)
    assert np.max(np.abs(q_gpu)) == lim
    diff = q_gpu - q_ref
    assert np.max(np.abs(diff)) <= 1
    assert np.mean(diff != 0) <= 1e-3
    c.close()


def test_int8_physical_units_match_fp64():
    """De-scaled int8 visibilities estimate the float64 ones: the coefficient
    error is set by the quantisation step (1/127 of 4 rms per component)."""
    N, K, S = 12, 256, 1024
    r = synth.recipe_tone(N=N, two_k=2 * K, seed=12)
    packed = _packed(r, S)
    c = corr.Correlator(N, K, S, precision="int8")
    c.process(packed)
    v = c.read_cps()
    ref = oracle.correlate(packed.cpu().numpy(), S, N, K)
    assert coef_error(v, ref, N) <= 0.02


# ------------------------------------------------------------------ FP16

@pytest.mark.parametrize("N,K,S", [(44, 256, 1024), (9, 1024, 50)])
def test_fp16_matches_oracle(N, K, S):
    print(f"\n[fp16] N={N} K={K} S={S}", flush=True)
    r = synth.recipe_tone(N=N, two_k=2 * K, seed=N)
    packed = _packed(r, S)
    tiles = dict(chunk_spectra=round_up(S, 64))
    c = corr.Correlator(N, K, S, precision="fp16", tiles=tiles)
    c.process(packed)
    buf, n = c.debug_read_spectra()
    raw = raw_to_complex(c.read_cps_raw())
    half = corr.records_to_spectra(buf, corr.CORR_FP16, N, K, S)
    # same half-precision inputs: only the float accumulation differs
    ref_same = oracle.cmac_f64(half.astype(np.complex128))
    assert coef_error(raw, ref_same, N) <= 1e-5
    # the half values are the float64 spectra rounded to half
    spec = oracle.spectra(packed.cpu().numpy(), S, N, K)
    rounded = spec.real.astype(np.float32).astype(np.float16) + 1j * spec.imag.astype(np.float32).astype(np.float16)
    # the GPU rounds its float FFT to half, the oracle its float64 one: a value
    # can differ only where the two sit on either side of a half rounding tie
    mism = half != rounded
    assert np.mean(mism) < 1e-2
    scale = np.sqrt(np.mean(np.abs(spec) ** 2))
    for part in (np.real, np.imag):
        h, r_ = part(half)[mism].astype(np.float64), part(rounded)[mism].astype(np.float64)
        big = np.maximum(np.abs(h), np.abs(r_)).astype(np.float16)
        # one half ulp step, plus the float FFT's absolute error near zero
        tol = np.spacing(big).astype(np.float64) + 1e-5 * scale
        assert np.all(np.abs(h - r_) <= tol)
    # end to end against float64
    ref = oracle.cmac_f64(spec)
    assert coef_error(raw, ref, N) <= TOL[corr.CORR_FP16]


@pytest.mark.parametrize("N,K,S", [(44, 256, 96), (160, 128, 24), (256, 128, 100), (220, 128, 52)])
def test_fp16_x_stage_on_oracle_spectra(N, K, S):
    """Half spectra through corr_process_spectra against float64 on the same
    values; N = 160 runs both region kinds in one launch, N = 256 and N = 220
    (padded to 256) the LDS-staged region groups."""
    rng = np.random.default_rng(2)
    spec = (rng.standard_normal((S, N, K)) * 50 + 1j * rng.standard_normal((S, N, K)) * 50)
    half = spec.real.astype(np.float16).astype(np.float64) + 1j * spec.imag.astype(np.float16).astype(np.float64)
    buf = torch.from_numpy(corr.spectra_to_records(half, corr.CORR_FP16)).cuda()
    c = corr.Correlator(N, K, S, precision="fp16")
    c.process_spectra(buf, S)
    raw = raw_to_complex(c.read_cps_raw())
    assert coef_error(raw, oracle.cmac_f64(half), N) <= 1e-5


def test_fp32_process_spectra_longer_than_its_splits():
    """corr_process_spectra on 5000 spectra with tiles sized for chunks of 64
    (one split): run as ranges of at most 2048 spectra per partial, so the
    float error stays within the fp32 tolerance."""
    N, K, S = 12, 128, 5000
    rng = np.random.default_rng(5)
    common = rng.standard_normal((S, 1, K)) + 1j * rng.standard_normal((S, 1, K))
    spec = 40 * (rng.standard_normal((S, N, K)) + 1j * rng.standard_normal((S, N, K)) + 0.6 * common)
    spec = spec.real.astype(np.float32).astype(np.float64) + 1j * spec.imag.astype(np.float32).astype(np.float64)
    buf = torch.from_numpy(corr.spectra_to_records(spec, corr.CORR_FP32)).cuda()
    c = corr.Correlator(N, K, S, tiles=dict(chunk_spectra=64, x_splits=1))
    c.process_spectra(buf, S)
    raw = raw_to_complex(c.read_cps_raw())
    err = coef_error(raw, oracle.cmac_f64(spec), N)
    print(f"\n[fp32 long process_spectra] coefficient error {err:.3g}", flush=True)
    assert err <= TOL[corr.CORR_FP32]


# ------------------------------------------------------------------ state errors

def test_state_errors():
    N, K, S = 8, 128, 16
    packed = torch.zeros(S * N * K, dtype=torch.uint8, device="cuda")
    c = corr.Correlator(N, K, S)
    with pytest.raises(corr.CorrError) as e:
        c.read_cps_raw()
    assert e.value.code == corr.CORR_ESTATE
    c.process(packed)
    with pytest.raises(corr.CorrError) as e:
        corr.corr_set_precision(c.h, corr.CORR_INT8)
    assert e.value.code == corr.CORR_ESTATE
    with pytest.raises(corr.CorrError) as e:
        corr.corr_set_tiles(c.h, chunk_spectra=64)
    assert e.value.code == corr.CORR_ESTATE
    c.read_cps_raw()
    ci = corr.Correlator(N, K, S, precision="int8")
    ci.tiles()          # plans (allocates the scales) but calibrates nothing
    with pytest.raises(corr.CorrError) as e:
        ci.read_scales()
    assert e.value.code == corr.CORR_ESTATE
    ci.process(packed)
    with pytest.raises(corr.CorrError) as e:
        ci.process(packed)
    assert e.value.code == corr.CORR_ESTATE
    with pytest.raises(corr.CorrError) as e:
        corr.Correlator(N, K, 70000, precision="int8")
    assert e.value.code == corr.CORR_EINVAL
    with pytest.raises(corr.CorrError):
        corr.corr_process(c.h, packed.data_ptr() + 1, 0)


def round_up(x, m):
    return (x + m - 1) // m * m


@pytest.mark.parametrize("prec", ["fp32", "fp16", "int8", "int16"])
def test_every_autotuner_candidate_passes_parity(prec):
    """Each tile choice the autotuner may pick: float forms within tolerance
    of the oracle, int8 and int16 identical to every other candidate."""
    from paper_1102_0148_amd import tune
    N, K, S = 44, 256, 300
    packed = _packed(synth.recipe_plain(N=N, two_k=2 * K, seed=21), S)
    ref = oracle.correlate(packed.cpu().numpy(), S, N, K)
    cands = tune.candidates(N, K, S, prec)
    assert len(cands) >= 20
    first = None
    for t in cands:
        _, raw = run(N, K, S, packed, precision=corr.PRECISIONS[prec], tiles=t)
        if prec in ("int8", "int16"):
            if first is None:
                first = raw
            else:
                np.testing.assert_array_equal(raw, first)
        else:
            assert coef_error(raw_to_complex(raw), ref, N) <= TOL[corr.PRECISIONS[prec]], t


# ------------------------------------------------------------------ degenerate cases

@pytest.mark.parametrize("prec", ["fp32", "fp16", "int8", "int16"])
def test_single_spectrum_two_antennas(prec):
    """The smallest job: two antennas, 128 channels, one spectrum (one
    partial record, padded by zero spectra), in every form."""
    N, K, S = 2, 128, 1
    print(f"\n[degenerate] {prec} N={N} K={K} S={S}", flush=True)
    packed = _packed(synth.recipe_plain(N=N, two_k=2 * K, seed=71), S)
    c = corr.Correlator(N, K, S, precision=prec)
    c.process(packed)
    buf, n = c.debug_read_spectra()
    assert n == S
    raw = c.read_cps_raw()
    assert raw.shape == (3, K, 2)
    spec = oracle.spectra(packed.cpu().numpy(), S, N, K)
    code = corr.PRECISIONS[prec]
    if prec in ("fp32", "fp16"):
        assert coef_error(raw_to_complex(raw), oracle.cmac_f64(spec), N) <= TOL[code]
    else:
        q = corr.records_to_spectra(buf, code, N, K, S)
        exact = oracle.cmac_i64(q) if prec == "int8" else oracle.cmac_i64_16(q)
        np.testing.assert_array_equal(raw, exact.astype(np.float64))
    c.close()


@pytest.mark.parametrize("prec", ["fp32", "fp16", "int8", "int16"])
def test_all_zero_input(prec):
    """Silent antennas: every visibility is zero, and the integer forms give
    every zero-power channel the scale 1 (no division by zero)."""
    N, K, S = 5, 128, 40
    packed = torch.zeros(S * N * K, dtype=torch.uint8, device="cuda")
    c = corr.Correlator(N, K, S, precision=prec)
    c.process(packed)
    if prec in ("int8", "int16"):
        np.testing.assert_array_equal(c.read_scales(), np.ones((N, K), dtype=np.float32))
    raw = c.read_cps_raw()
    assert np.all(raw == 0)
    c.close()
