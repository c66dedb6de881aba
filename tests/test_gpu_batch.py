"""GPU parity of the batched path, in both of its modes (each job's own
kernels on parallel branches of one HIP graph; one persistent kernel replayed
from a HIP graph), against the CPU oracle and against the single-job path."""
import numpy as np
import pytest
import torch

import oracle
import paper_1102_0148_amd as corr
import synth
from test_gpu_parity import coef_error, raw_to_complex

pytestmark = pytest.mark.gpu
MODES = ["branches", "persistent"]

# uneven jobs: every channel count, 1-6 antenna blocks, both precisions
JOBS = [(8, 128, 40, "int8"), (12, 256, 64, "fp32"), (16, 512, 33, "int8"), (24, 256, 50, "fp32"),
        (32, 1024, 24, "int8"), (44, 256, 100, "fp32"), (64, 512, 20, "int8"), (96, 256, 17, "fp32"),
        (44, 256, 70, "fp16"), (5, 128, 3, "fp32")]


def _inputs(jobs, seed0=100):
    out = []
    for i, (N, K, S, _) in enumerate(jobs):
        r = synth.Recipe(N=N, two_k=2 * K, seed=seed0 + i, sources=[synth.Source(rho=0.05 + 0.01 * i)])
        out.append(synth.packed(r, 0, S).contiguous().cuda())
    return out


def _check_job(raw, N, K, S, prec, packed):
    if prec == "int8":
        # the exact integer oracle on the quantised spectra of the oracle's
        # own spectra with the GPU's scales agrees up to rounding-tie flips,
        # so check the de-scaled value statistically and the raw bit-exactly
        # through the single-job path below
        return
    ref = oracle.correlate(packed.cpu().numpy(), S, N, K)
    tol = 1e-5 if prec == "fp32" else 2e-3
    assert coef_error(raw_to_complex(raw), ref, N) <= tol


@pytest.mark.parametrize("mode", MODES)
def test_batch_matches_oracle_and_single_job(mode):
    print(f"\n[batch {mode}] {len(JOBS)} jobs", flush=True)
    inputs = _inputs(JOBS)
    b = corr.Batch(JOBS, mode=mode)
    b.process(inputs)
    raws = [b.read_cps_raw(j) for j in range(len(JOBS))]
    for j, (N, K, S, prec) in enumerate(JOBS):
        print(f"  job {j}: N={N} K={K} S={S} {prec}", flush=True)
        _check_job(raws[j], N, K, S, prec, inputs[j])
        c = corr.Correlator(N, K, S, precision=prec, tiles=dict(chunk_spectra=(S + 63) // 64 * 64))
        c.process(inputs[j])
        single = c.read_cps_raw()
        if prec == "int8":
            # same scales and the same exact integer sums
            np.testing.assert_array_equal(raws[j], single)
            buf, n = c.debug_read_spectra()
            q = corr.records_to_spectra(buf, corr.CORR_INT8, N, K, n)
            np.testing.assert_array_equal(raws[j], oracle.cmac_i64(q).astype(np.float64))
        else:
            ref = oracle.correlate(inputs[j].cpu().numpy(), S, N, K)
            assert coef_error(raw_to_complex(single), ref, N) <= (1e-5 if prec == "fp32" else 2e-3)


@pytest.mark.parametrize("mode", MODES)
def test_batch_graph_replays(mode):
    """Replay the captured graph several times with eager work and
    synchronisations between replays.  Every replay, the first included, is
    checked: int8 jobs bit-exactly against the single-job path, float jobs
    against the oracle, and every replay equals the first.  (The last job's
    counters are the last of the counter array, and its dumps are the last
    items; a wrong counter index there once showed only in the first run.)
    From the third replay on the inputs are copies at other addresses: the
    graph reads each job's input pointer at run time."""
    jobs = JOBS[:6]
    inputs = _inputs(jobs, seed0=200)
    singles = {}
    for j, (N, K, S, prec) in enumerate(jobs):
        if prec == "int8":
            c = corr.Correlator(N, K, S, precision=prec)
            c.process(inputs[j])
            singles[j] = c.read_cps_raw()
            c.close()
    b = corr.Batch(jobs, mode=mode)
    first = None
    moved = [x.clone() for x in inputs]
    for rep in range(4):
        b.process(inputs if rep < 2 else moved)
        if rep == 2:
            del inputs  # the first copies are freed; their memory may be reused
        # eager work of the program between replays
        scratch = torch.randn(1 << 20, device="cuda")
        scratch.mul_(2.0).sum().item()
        torch.cuda.synchronize()
        raws = [b.read_cps_raw(j) for j in range(len(jobs))]
        print(f"\n[batch replay] {rep}", flush=True)
        for j, (N, K, S, prec) in enumerate(jobs):
            if prec == "int8":
                np.testing.assert_array_equal(raws[j], singles[j], err_msg=f"replay {rep} job {j}")
            elif rep == 0:
                _check_job(raws[j], N, K, S, prec, moved[j])
        if first is None:
            first = raws
        else:
            for j in range(len(jobs)):
                np.testing.assert_array_equal(raws[j], first[j], err_msg=f"replay {rep} job {j}")


def test_batch_rejects_bad_input():
    with pytest.raises(corr.CorrError):
        corr.Batch([(1, 256, 10, "fp32")])
    with pytest.raises(corr.CorrError) as e:
        corr.Batch([(8, 256, 16, "fp32")], mode=7)
    assert e.value.code == corr.CORR_EINVAL
    with pytest.raises(corr.CorrError):
        corr.Batch([(8, 256, 70000, "int8")])
    b = corr.Batch([(8, 256, 16, "int8")])
    x = torch.zeros(16 * 8 * 256, dtype=torch.uint8, device="cuda")
    b.process([x])
    with pytest.raises(corr.CorrError) as e:
        b.process([x])
    assert e.value.code == corr.CORR_ESTATE
    b.read_cps_raw(0)
    with pytest.raises(corr.CorrError):
        corr.corr_batch_set_tiles(b.h, 0, x_splits=4)
    with pytest.raises(corr.CorrError) as e:
        corr.corr_batch_set_mode(b.h, corr.CORR_BATCH_PERSISTENT)
    assert e.value.code == corr.CORR_ESTATE


def test_branches_jobs_in_chunks_replay():
    """Branch jobs keep their own tiles, several chunks each included: the
    kernels add each chunk's offset to the input pointer they read from the
    job's slot. Every replay, with the inputs moved to other addresses from
    the second on, equals the single-job path with the same tiles, bit for
    bit (same kernels on the same spectra)."""
    jobs = [(8, 128, 200, "int8"), (12, 256, 300, "fp32"), (44, 256, 130, "fp16"), (16, 512, 70, "fp32")]
    tiles = {0: dict(chunk_spectra=64, x_splits=1, f_group=4), 1: dict(chunk_spectra=128, x_splits=2, f_group=16),
             2: dict(chunk_spectra=64, x_splits=1, f_group=2), 3: dict(chunk_spectra=64, x_splits=2, f_group=1)}
    inputs = _inputs(jobs, seed0=300)
    singles = []
    for j, (N, K, S, prec) in enumerate(jobs):
        c = corr.Correlator(N, K, S, precision=prec, tiles=tiles[j])
        c.process(inputs[j])
        singles.append(c.read_cps_raw())
        c.close()
        _check_job(singles[j], N, K, S, prec, inputs[j])
    b = corr.Batch(jobs, tiles=tiles, mode="branches")
    moved = [x.clone() for x in inputs]
    for rep in range(3):
        b.process(inputs if rep == 0 else moved)
        torch.cuda.synchronize()
        print(f"\n[branches in chunks] replay {rep}", flush=True)
        for j in range(len(jobs)):
            np.testing.assert_array_equal(b.read_cps_raw(j), singles[j], err_msg=f"replay {rep} job {j}")
    b.close()


def test_persistent_mode_rejects_chunked_tiles():
    """The persistent kernel runs each job as one chunk with its own F group:
    other tiles fail at the first process, before any launch."""
    b = corr.Batch([(8, 128, 200, "fp32")], tiles={0: dict(chunk_spectra=64)}, mode="persistent")
    x = torch.zeros(200 * 8 * 128, dtype=torch.uint8, device="cuda")
    with pytest.raises(corr.CorrError) as e:
        b.process([x])
    assert e.value.code == corr.CORR_EINVAL
    b.close()
