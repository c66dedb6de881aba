"""Autotuner for the correlator's tile choices.

For one job shape (N antennas, K channels, n_spectra, precision) it times
every candidate (chunk_spectra, x_splits, f_group) with the library's own
stage timers (HIP events on the launch stream) over a few integrations of
synthetic input, and keeps the fastest; where the fused pipeline covers the
shape it also times the fused choices (ring chunk, slots, F workgroups per
CU) end to end against the best staged tiles and records which pipeline
Correlator(tiles="auto") should run.  Jobs of the persistent batch kernel
(one chunk per job, the F-stage group fixed) are tuned over x_splits in a
batch of their own; a branch of a batch graph runs the single-job kernels and
takes the single-job entries.  Results go to a JSON table keyed by (arch, N,
K, n_spectra, precision[, batch mode]) that Correlator(tiles="auto") and
Batch(tiles="auto") read.

Run on the GPU:  python -m paper_1102_0148_amd.tune --out tuned.json [shapes]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from typing import Dict, Iterable, List, Optional, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "tuned_tiles.json")
ARCH = "gfx950"
LDS_LIMIT = 160 * 1024
SPLITS = (1, 2, 4, 8, 12, 16, 24, 32, 48, 64)
# spectra one partial may sum, per form: fp32 partials stay short for
# accuracy (its three-product form cancels), fp16's error is its spectra's up
# to 16384; int16 digit sums must stay exact in int32; int8 sums always are
PARTIAL_LIMIT = {"fp32": 2048, "fp16": 16384, "int16": 16384, "int8": None}


def record_times(prec: str) -> int:
    return {"fp32": 2, "fp16": 4, "int8": 8, "int16": 4}[prec]


def f_lds_bytes(K: int, prec: str, group: int) -> int:
    L = K // 16
    fpr = 256 // L
    slot = K + K // 16 + 1
    return record_times(prec) * group * slot * 8 + fpr * K


def key(N: int, K: int, S: int, prec: str, batch=False, mode: Optional[str] = None) -> str:
    """Table key; batch is False (a single job), True or "persistent" (a job
    of the persistent batch kernel) or "branches" (a job on a branch of a
    batch graph, whose chunk and F group are fixed); mode "fused" is a single
    job on the fused pipeline (chunk, ring slots, F workgroups per CU)."""
    suffix = "" if not batch else (":branches" if batch == "branches" else ":batch")
    if mode == "fused":
        suffix += ":fused"
    return f"{ARCH}:N={N}:K={K}:S={S}:{prec}" + suffix


def candidates(N: int, K: int, S: int, prec: str) -> List[dict]:
    """Every tile choice the tuner considers for a single job."""
    whole = (S + 63) // 64 * 64
    chunks = sorted({c for c in (whole, whole // 2, whole // 4, 16384, 8192) if 1024 <= c <= whole and c % 64 == 0}
                    | {whole})
    groups = [g for g in (1, 2, 4, 8, 16) if f_lds_bytes(K, prec, g) <= LDS_LIMIT]
    out = []
    for chunk in chunks:
        for s in SPLITS:
            if PARTIAL_LIMIT[prec] and chunk / s > PARTIAL_LIMIT[prec]:
                continue
            for g in groups:
                out.append({"chunk_spectra": chunk, "x_splits": s, "f_group": g})
    return out


def load_table(path: str = TABLE) -> Dict[str, dict]:
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def lookup(N: int, K: int, S: int, prec: str, batch=False, path: str = TABLE, mode: Optional[str] = None) -> Optional[dict]:
    return load_table(path).get(key(N, K, S, prec, batch, mode))


def _time_single(corr, torch, N, K, S, prec, tiles, x, reps=3, warm=1) -> Dict[str, float]:
    """Per-integration stage times (ms) of one tile choice: F-stage, X-stage
    plus dump, calibration and their total, and the end-to-end time of an
    integration (process and an asynchronous read between HIP events, so the
    gaps between launches count too)."""
    c = corr.Correlator(N, K, S, precision=prec, tiles=tiles)
    dst = torch.empty(c.nb * K * 2, dtype=torch.float64, device="cuda")
    try:
        for _ in range(warm):
            c.process(x)
            c.read_cps_async(dst)
        c.enable_timing(True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            c.process(x)
            c.read_cps_async(dst)
        e1.record()
        torch.cuda.synchronize()
        st = c.stats()
        t = {"f": st["ms_f"] / reps, "x": (st["ms_x"] + st["ms_dump"]) / reps, "calib": st["ms_calib"] / reps}
        t["total"] = t["f"] + t["x"] + t["calib"]
        t["e2e"] = e0.elapsed_time(e1) / reps
        return t
    finally:
        c.close()
        del dst
        torch.cuda.empty_cache()


def _median(v: List[float]) -> float:
    v = sorted(v)
    return v[len(v) // 2] if len(v) % 2 else 0.5 * (v[len(v) // 2 - 1] + v[len(v) // 2])


def _rounds(corr, torch, N, K, S, prec, x, cands, stage, rounds=3, reps=4, log=print) -> List[Tuple[dict, float]]:
    """Median of `stage` time over `rounds` passes that time every candidate in
    turn, so a drift of the clock during the run falls on all of them alike."""
    seen: Dict[str, List[float]] = {}
    for r in range(rounds):
        for t in cands:
            ms = _time_single(corr, torch, N, K, S, prec, t, x, reps=reps, warm=1)[stage]
            seen.setdefault(json.dumps(t, sort_keys=True), []).append(ms)
            log(f"  {prec} N={N} K={K} {t} {stage} {ms:.4f} ms (round {r})")
    return [(json.loads(k), _median(v)) for k, v in seen.items()]


def final_candidates(top: List[dict], group: int, incumbent: Optional[dict] = None) -> List[dict]:
    """The choices of tune_single's last stage: the best (chunk, splits) pairs
    with the chosen F group, and the table's present entry (its three tiles)
    where there is one, so that a re-tune keeps it unless another choice
    beats it side by side on the same GPU."""
    out = [dict(t, f_group=group) for t in top]
    if incumbent and all(k in incumbent for k in ("chunk_spectra", "x_splits", "f_group")):
        inc = {k: incumbent[k] for k in ("chunk_spectra", "x_splits", "f_group")}
        if inc not in out:
            out.append(inc)
    return out


def tune_single(N: int, K: int, S: int, prec: str, log=print,
                incumbent: Optional[dict] = None) -> Tuple[dict, float, List[Tuple[dict, float]]]:
    """Stage 1 times every (chunk, splits) at the default F group; stage 2
    picks the group by the F-stage time alone (the only stage it changes),
    timing the groups in turn at the best chunk; stage 3 times the four best
    (chunk, splits) pairs of stage 1 with that group, and the incumbent
    table entry, in turn and keeps the lowest median end-to-end time (ties
    as in `pick`): the stage timers leave out the gaps between launches,
    which a choice with more chunks pays for."""
    import torch
    import paper_1102_0148_amd as corr
    import synth
    x = synth.packed(synth.recipe_plain(N=N, two_k=2 * K, seed=11), 0, S, device="cuda").contiguous()
    cands = candidates(N, K, S, prec)
    groups = sorted({c["f_group"] for c in cands})
    fpr = 256 // (K // 16)
    dg = max(1, fpr // record_times(prec))
    base_group = dg if dg in groups else min(groups)
    results = []
    for t in [c for c in cands if c["f_group"] == base_group]:
        ms = _time_single(corr, torch, N, K, S, prec, t, x)["total"]
        results.append((t, ms))
        log(f"  {prec} N={N} K={K} {t} {ms:.4f} ms")
    top = [t for t, _ in sorted(results, key=lambda r: r[1])[:4]]
    chunk, splits = top[0]["chunk_spectra"], top[0]["x_splits"]
    by_f = _rounds(corr, torch, N, K, S, prec, x,
                   [{"chunk_spectra": chunk, "x_splits": splits, "f_group": g} for g in groups], "f", log=log)
    group = min(by_f, key=lambda r: r[1])[0]["f_group"]
    # integrations are cheap next to building a correlator: ten per timing,
    # five rounds, against the drift of the clock between rounds
    final = _rounds(corr, torch, N, K, S, prec, x, final_candidates(top, group, incumbent), "e2e",
                    rounds=5, reps=10, log=log)
    best, best_ms = pick(final)
    return best, best_ms, results + final


def fused_candidates(N: int, K: int, S: int, prec: str) -> List[dict]:
    """Fused-pipeline choices: ring slots of about 24 to 96 MB of records,
    two or three slots, and the role layout: mixed with the default or one F
    workgroup per CU, or split with 12 to 24 of each XCD's 32 CUs on F.  The
    fused kernel covers fp32, fp16 and int8 at N <= 48."""
    if prec not in ("fp32", "fp16", "int8") or N > 48:
        return []
    a_pad = 16 * ((N + 15) // 16)
    per_spectrum = a_pad * K * 16 // record_times(prec)
    whole = (S + 63) // 64 * 64
    chunks = sorted({min(whole, max(64, (mb << 20) // per_spectrum // 64 * 64)) for mb in (24, 48, 72, 96)})
    layouts = [{"f_workgroups_per_cu": f, "f_cus_per_xcd": 0} for f in (0, 1)] + \
              [{"f_workgroups_per_cu": 0, "f_cus_per_xcd": n} for n in (12, 16, 20, 24)]
    return [dict(chunk_spectra=c, ring_slots=r, **l) for c in chunks for r in (2, 3) for l in layouts]


def _time_e2e(corr, torch, N, K, S, prec, x, tiles=None, pipeline=None, reps=4, warm=1) -> float:
    """End-to-end time of one integration (process and an asynchronous read,
    HIP events around them), for comparing pipelines."""
    c = corr.Correlator(N, K, S, precision=prec, tiles=tiles, pipeline=pipeline)
    dst = torch.empty(c.nb * K * 2, dtype=torch.float64, device="cuda")
    try:
        for _ in range(warm):
            c.process(x)
            c.read_cps_async(dst)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            c.process(x)
            c.read_cps_async(dst)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps
    finally:
        c.close()
        del dst
        torch.cuda.empty_cache()


def tune_pipeline(N: int, K: int, S: int, prec: str, staged: dict, log=print) -> Tuple[Optional[dict], float, float]:
    """Every fused choice timed once end to end, then the three fastest and
    the staged pipeline's best tiles in turn over five rounds of ten
    integrations each (medians).
    Returns the best fused choice (None where the kernel does not cover the
    shape), its median time and the staged median."""
    import torch
    import paper_1102_0148_amd as corr
    import synth
    cands = fused_candidates(N, K, S, prec)
    if not cands:
        return None, float("inf"), float("inf")
    x = synth.packed(synth.recipe_plain(N=N, two_k=2 * K, seed=11), 0, S, device="cuda").contiguous()
    first = []
    for p in cands:
        ms = _time_e2e(corr, torch, N, K, S, prec, x, pipeline=p)
        first.append((p, ms))
        log(f"  fused {prec} N={N} K={K} {p} {ms:.4f} ms")
    top = [p for p, _ in sorted(first, key=lambda r: r[1])[:3]]
    seen: Dict[str, List[float]] = {}
    for r in range(5):
        for p in top:
            seen.setdefault(json.dumps(p, sort_keys=True), []).append(
                _time_e2e(corr, torch, N, K, S, prec, x, pipeline=p, reps=10))
        seen.setdefault("staged", []).append(_time_e2e(corr, torch, N, K, S, prec, x, tiles=staged, reps=10))
    staged_ms = _median(seen.pop("staged"))
    best = min(((json.loads(k), _median(v)) for k, v in seen.items()), key=lambda r: r[1])
    log(f"  fused {prec} N={N} K={K} best {best[0]} {best[1]:.4f} ms; staged {staged_ms:.4f} ms")
    return best[0], best[1], staged_ms


TIE = 0.01


def pick(timed: List[Tuple[dict, float]]) -> Tuple[dict, float]:
    """The fastest tile choice, except that choices within TIE (relative) of
    it count as ties, which go to the fewest chunks, then the fewest splits
    (fewer launches and a smaller dump for the same time)."""
    fastest = min(ms for _, ms in timed)
    close = [(t, ms) for t, ms in timed if ms <= fastest * (1 + TIE)]
    return min(close, key=lambda r: (-r[0]["chunk_spectra"], r[0]["x_splits"], r[1]))


def tune_batch_job(N: int, K: int, S: int, prec: str, mode: str = "persistent", log=print) -> Tuple[dict, float]:
    """x_splits of one batch job (its chunk and F group are fixed in a
    batch), timed in a batch of its own in the given mode."""
    import torch
    import paper_1102_0148_amd as corr
    import synth
    x = synth.packed(synth.recipe_plain(N=N, two_k=2 * K, seed=12), 0, S, device="cuda").contiguous()
    best = None
    for s in SPLITS:
        if PARTIAL_LIMIT[prec] and S / s > PARTIAL_LIMIT[prec]:
            continue
        b = corr.Batch([(N, K, S, prec)], tiles={0: {"x_splits": s}}, mode=mode)
        try:
            b.process([x])
            b.read_cps_raw(0)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(3):
                b.process([x])
                b.read_cps_raw(0)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / 3
        finally:
            b.close()
        log(f"  batch {mode} {prec} N={N} K={K} x_splits={s} {ms:.4f} ms")
        if best is None or ms < best[1]:
            best = ({"x_splits": s}, ms)
    return best


def main(argv: Optional[Iterable[str]] = None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=TABLE)
    ap.add_argument("--single", default="44:256:65536:fp32,44:256:65536:fp16,44:256:65536:int8,44:256:65536:int16,"
                                        "256:512:16384:fp32,256:512:16384:int8")
    ap.add_argument("--batch", default="8:128:16384,12:256:16384,16:512:16384,24:256:16384,"
                                       "32:1024:16384,44:256:16384,64:512:16384,96:256:16384")
    ap.add_argument("--batch-precisions", default="int8,fp32")
    ap.add_argument("--batch-modes", default="persistent")
    ap.add_argument("--pipeline-only", action="store_true",
                    help="keep the table's staged tiles of each single shape and only choose the pipeline")
    args = ap.parse_args(argv)
    sys.path.insert(0, os.path.dirname(HERE))
    import torch
    torch.cuda.set_device(0)
    table = load_table(args.out)
    for item in filter(None, args.single.split(",")):
        N, K, S, prec = item.split(":")
        N, K, S = int(N), int(K), int(S)
        old = table.get(key(N, K, S, prec))
        if args.pipeline_only and old and "chunk_spectra" in old:
            best = {k: old[k] for k in ("chunk_spectra", "x_splits", "f_group")}
            ms = old.get("ms", 0.0)
        else:
            best, ms, _ = tune_single(N, K, S, prec, incumbent=old)
        entry = dict(best, ms=round(ms, 4), pipeline="staged")
        fbest, fms, sms = tune_pipeline(N, K, S, prec, best)
        if fbest is not None:
            table[key(N, K, S, prec, mode="fused")] = dict(fbest, ms=round(fms, 4))
            # the fused pipeline where it is faster end to end by more than a tie
            if fms < sms * (1 - TIE):
                entry["pipeline"] = "fused"
            entry["e2e_ms"] = {"staged": round(sms, 4), "fused": round(fms, 4)}
        table[key(N, K, S, prec)] = entry
        print(f"best {key(N, K, S, prec)}: {table[key(N, K, S, prec)]}", flush=True)
        with open(args.out, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
    for item in filter(None, args.batch.split(",")):
        N, K, S = (int(v) for v in item.split(":"))
        for prec in args.batch_precisions.split(","):
            for mode in args.batch_modes.split(","):
                best, ms = tune_batch_job(N, K, S, prec, mode)
                k = key(N, K, S, prec, batch=mode)
                table[k] = dict(best, ms=round(ms, 4))
                print(f"best {k}: {table[k]}", flush=True)
            with open(args.out, "w") as f:
                json.dump(table, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
