"""GPU parity of frame ingest (self-contained frames that may be lost,
repeated, reordered or corrupt) against the CPU oracle, through the C ABI:
the assembled integration and the counts bit-exact, and the correlation and
int8 calibration of an integration with lost spectra."""
import numpy as np
import pytest
import torch

import oracle
import paper_1102_0148_amd as corr
import synth
from test_gpu_parity import TOL, coef_error, raw_to_complex

pytestmark = pytest.mark.gpu


def _scenario(S, N, K, first, seed, lose=0.05, dup=0.03, n_bad=10):
    """Frames for S blocks: shuffled, a fraction lost, a fraction sent twice
    (the second copy with other payload), and n_bad corrupt headers."""
    rng = np.random.default_rng(seed)
    packed = synth.packed(synth.recipe_plain(N=N, two_k=2 * K, seed=seed), 0, S)
    other = synth.packed(synth.recipe_plain(N=N, two_k=2 * K, seed=seed + 1), 0, S)
    keep = [b for b in range(S) if rng.random() >= lose]
    order = list(rng.permutation(keep))
    fr = [synth.frames(packed, [first + int(b) for b in order], blocks=[int(b) for b in order])]
    dups = [int(b) for b in keep if rng.random() < dup]
    if dups:
        fr.append(synth.frames(other, [first + b for b in dups], blocks=dups))
    for i in range(n_bad):
        b = int(rng.integers(0, S))
        kind = i % 5
        kw = [dict(magic=0), dict(version=7), dict(n_elements=N + 2), dict(two_k=K), {}][kind]
        seq = first + S + i if kind == 4 else first + b
        fr.append(synth.frames(packed, [seq], blocks=[b], **kw))
    frames = torch.cat(fr)
    # interleave so the duplicates and corrupt frames are not all at the end
    perm = torch.from_numpy(rng.permutation(frames.shape[0]))
    return packed, frames[perm].contiguous()


@pytest.mark.parametrize("N,K,S", [(20, 256, 300), (44, 256, 1100), (5, 128, 37)])
def test_ingest_matches_oracle(N, K, S):
    first = (1 << 40) + 17
    print(f"\n[ingest] N={N} K={K} S={S}", flush=True)
    _, frames = _scenario(S, N, K, first, seed=N + S)
    n, stride = frames.shape
    c = corr.Correlator(N, K, S)
    out = c.ingest(frames.cuda(), n, stride, first)
    ref, st_ref, _ = oracle.ingest(frames.numpy(), n, stride, first, S, N, K)
    np.testing.assert_array_equal(out.cpu().numpy().reshape(S, N, K), ref)
    assert c.ingest_stats() == st_ref
    assert st_ref["spectra_lost"] > 0 and st_ref["frames_duplicate"] > 0 and st_ref["frames_rejected"] > 0


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_ingest_end_to_end_float(prec):
    N, K, S, first = 24, 256, 400, 5
    _, frames = _scenario(S, N, K, first, seed=3)
    n, stride = frames.shape
    c = corr.Correlator(N, K, S, precision=prec)
    out = c.ingest(frames.cuda(), n, stride, first)
    c.process(out)
    raw = raw_to_complex(c.read_cps_raw())
    ref_packed, _, _ = oracle.ingest(frames.numpy(), n, stride, first, S, N, K)
    ref = oracle.correlate(ref_packed, S, N, K)
    assert coef_error(raw, ref, N) <= TOL[corr.PRECISIONS[prec]]


@pytest.mark.parametrize("prec", ["int8", "int16"])
def test_ingest_calibration_counts_received_spectra(prec):
    """Lost spectra inside the calibration window: the scales divide by the
    spectra received; the next integration without ingest divides by W again."""
    N, K, S, first = 16, 256, 1500, 0
    code = corr.PRECISIONS[prec]
    cmac = oracle.cmac_i64 if prec == "int8" else oracle.cmac_i64_16
    _, frames = _scenario(S, N, K, first, seed=9, lose=0.2)
    n, stride = frames.shape
    c = corr.Correlator(N, K, S, precision=prec, tiles=dict(chunk_spectra=(S + 63) // 64 * 64))
    out = c.ingest(frames.cuda(), n, stride, first)
    c.process(out)
    scales = c.read_scales()
    raw = c.read_cps_raw()
    ref_packed, st, wv = oracle.ingest(frames.numpy(), n, stride, first, S, N, K)
    W = min(S, corr.CORR_CALIB_SPECTRA)
    assert 0 < wv < W
    spec = oracle.spectra(ref_packed, S, N, K)
    np.testing.assert_allclose(scales, oracle.scales_n(spec, W, wv, prec), rtol=1e-5)
    buf, m = c.debug_read_spectra()
    q = corr.records_to_spectra(buf, code, N, K, m)
    np.testing.assert_array_equal(raw, cmac(q).astype(np.float64))
    # the next integration is not an ingested one: the plain rule again
    c.process(out)
    np.testing.assert_allclose(c.read_scales(), oracle.scales_n(spec, W, W, prec), rtol=1e-5)
    c.read_cps_raw()


def test_ingest_nothing_arrives():
    N, K, S = 8, 128, 50
    c = corr.Correlator(N, K, S, precision="int8")
    frames = torch.zeros(1, 32 + N * K, dtype=torch.uint8, device="cuda")
    out = c.ingest(frames, 0, frames.shape[1], 0)
    assert c.ingest_stats() == dict(frames_accepted=0, frames_rejected=0, frames_duplicate=0, spectra_lost=S)
    assert int(out.count_nonzero()) == 0
    c.process(out)
    assert not np.any(c.read_cps_raw())
    np.testing.assert_array_equal(c.read_scales(), np.ones((N, K), dtype=np.float32))


def test_ingest_rejects_bad_arguments():
    N, K, S = 4, 128, 8
    c = corr.Correlator(N, K, S)
    with pytest.raises(corr.CorrError) as e:
        c.ingest_stats()
    assert e.value.code == corr.CORR_ESTATE
    frames = torch.zeros(4, 32 + N * K, dtype=torch.uint8, device="cuda")
    out = torch.empty(S * N * K, dtype=torch.uint8, device="cuda")
    for args in [(frames.data_ptr(), 4, 32 + N * K - 16, 0, out.data_ptr()),   # stride too small
                 (frames.data_ptr(), 4, 32 + N * K + 8, 0, out.data_ptr()),    # stride not a multiple of 16
                 (frames.data_ptr(), -1, 32 + N * K, 0, out.data_ptr()),       # negative count
                 (frames.data_ptr() + 8, 1, 32 + N * K, 0, out.data_ptr()),    # misaligned frames
                 (frames.data_ptr(), 1, 32 + N * K, 0, out.data_ptr() + 4),    # misaligned out
                 (0, 1, 32 + N * K, 0, out.data_ptr())]:
        with pytest.raises(corr.CorrError) as e:
            corr.corr_ingest(c.h, *args)
        assert e.value.code == corr.CORR_EINVAL
