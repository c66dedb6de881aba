"""Throughput of the FX correlator hot path on one MI355X.

Workload: N = 44 antennas, 512-point real FFT -> K = 256 channels, 4-bit
samples (sigma = 2.5 Gaussian noise per antenna plus a common component at
rho = 0.05), 65536 spectra per integration (~33.5 M samples per antenna, about
1 s at the paper's ~35 MS/s), 4 consecutive integrations per step.  Inputs are
generated on the GPU and resident in HBM before timing starts.  One step = the
whole path (unpack, F-stage, corner turn, X-stage, float64 dump and the
asynchronous read of each integration's result) over the 4 integrations.

`value` is the float32 path's sustained rate in antenna-MS/s (antenna-samples
per second / 1e6); the fp16 and int8 forms run the same step on the same input
and are reported beside it with their X-stage TOPS, speedup over float32 and
measured error against the float64 oracle (on a 1024-spectrum sample).

`roofline` is for the dominant kernel of the float32 step, from HIP events the
library records around each stage on the stream it launches on.
`cpu_baseline` times the CPU oracle (float64 FFT + pairwise CMAC) on a bounded
sample of the same workload on this host's cores.
"""
import argparse
import json
import math
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N_ANT, TWO_K, S_INT, N_INT = 44, 512, 65536, 4
K = TWO_K // 2
PAPER_ANTENNA_MSPS = 1470.0     # 735 MB/s of 4-bit samples (abstract), 4-node Xeon system
PEAK = {"hbm_gbs": 8000.0, "fp32_tflops": 157.3, "fp16_tflops": 2500.0, "int8_tops": 5000.0}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


KERNEL_SOURCES = {"fstage_kernel": ("fstage_dev.h", "fstage.hip", "corr_internal.h"),
                  "xstage_kernel": ("xstage_dev.h", "xstage.hip", "corr_internal.h")}


def measured_traffic(kernel, spectra_per_launch):
    """HBM bytes per launch from the committed rocprofv3 counter runs
    (profiles/traffic.json), or None when the kernel's source has changed since
    the counters were taken or the launch covers a different number of spectra."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    entry = json.load(open(path)).get(kernel)
    if entry is None or f"{spectra_per_launch} spectra" not in entry.get("workload", ""):
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel.split("<")[0]]:
        h.update(open(os.path.join(ROOT, "paper_1102_0148_amd", "csrc", f), "rb").read())
    if h.hexdigest() != entry["source_sha256"]:
        return None
    return entry["fetch_bytes"] + entry["write_bytes"]


def counted_valu(kernel):
    """VALU lane-operations per antenna-sample of an F-stage kernel from the
    committed rocprofv3 counter run (profiles/valu.json), or None when the
    kernel's source has changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "valu.json")
    if not os.path.exists(path):
        return None
    entry = json.load(open(path)).get(kernel)
    if entry is None:
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel.split("<")[0]]:
        h.update(open(os.path.join(ROOT, "paper_1102_0148_amd", "csrc", f), "rb").read())
    if h.hexdigest() != entry["source_sha256"]:
        return None
    return entry["valu_lane_ops_per_antenna_sample"]


# VALU issue peak without packed-fp32 forms: 256 CUs x 64 lanes x 2.4 GHz
VALU_LANE_OPS_PEAK = 256 * 64 * 2.4e9


def f_stage_bounds(metrics, name, f_ms, group):
    """The F-stage of one form against its two candidate bounds: HBM (0.5 B
    read + the record bytes written per antenna-sample) and VALU issue (lane
    operations per antenna-sample counted by rocprofv3, over the event-timed
    duration)."""
    rec = {"fp32": 4.0, "fp16": 2.0, "int8": 1.0, "int16": 2.0}[name]
    a_s = metrics.antenna_samples(N_ANT, TWO_K, S_INT)
    gbs = a_s * (0.5 + rec) / (f_ms * 1e-3) / 1e9
    out = {"hbm": {"achieved_gbs": round(gbs, 1), "frac": round(gbs / PEAK["hbm_gbs"], 4),
                   "bytes_per_antenna_sample": 0.5 + rec}}
    prec_code = {"fp32": 0, "fp16": 1, "int8": 2, "int16": 3}[name]
    per_as = counted_valu(f"fstage_kernel<256, {prec_code}, {group}, false>")
    if per_as is not None:
        rate = per_as * a_s / (f_ms * 1e-3)
        out["alu"] = {"valu_lane_ops_per_antenna_sample": per_as, "achieved_lane_ops_per_s": float("%.4g" % rate),
                      "peak_lane_ops_per_s": VALU_LANE_OPS_PEAK, "frac": round(rate / VALU_LANE_OPS_PEAK, 4)}
    return out


def make_inputs(device):
    import synth
    recipe = synth.recipe_plain(N=N_ANT, two_k=TWO_K, rho=0.05, seed=1)
    bufs = []
    for i in range(N_INT):
        bufs.append(synth.packed(recipe, i * S_INT, (i + 1) * S_INT, device=device).contiguous())
        log(f"[bench] generated integration {i + 1}/{N_INT}")
    return bufs


def run_form(corr, torch, precision, inputs, steps, warmup, timing=False, tracking=None, pipeline=None):
    c = corr.Correlator(N_ANT, K, S_INT, precision=precision, tiles="auto", pipeline=pipeline)
    if tracking:
        c.set_tracking(**tracking)
    dst = torch.empty(c.nb * K * 2, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()

    def step():
        for x in inputs:
            c.process(x, stream)
            c.read_cps_async(dst, stream)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    if timing:
        c.enable_timing(True)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t0.record(stream)
    for _ in range(steps):
        step()
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = t0.elapsed_time(t1)
    stats = c.stats()
    tiles = c.tiles()
    tiles["pipeline"] = c.pipeline
    c.close()
    return ms / steps, wall / steps * 1e3, stats, tiles


def tracking_leg(corr, torch, metrics, inputs, steps, warmup, forms, pipelines=None):
    """The headline step with per-antenna delay and phase tracking switched on
    (delays up to 50 samples, with rates), in each form, against the same
    step without it.  Tracking runs in the staged pipeline; a form whose
    tuned pipeline is the fused one compares with its staged F time from the
    pipelines leg."""
    import numpy as np
    rng = np.random.default_rng(1)
    model = dict(delay=rng.uniform(-50, 50, N_ANT), delay_rate=rng.uniform(-1e-3, 1e-3, N_ANT),
                 phase=rng.uniform(-1, 1, N_ANT), phase_rate=rng.uniform(-1e-4, 1e-4, N_ANT))
    a_s = N_INT * metrics.antenna_samples(N_ANT, TWO_K, S_INT)
    out = {"model": "per-antenna delay U(-50, 50) samples, rate U(-1e-3, 1e-3) samples/spectrum, "
                    "phase U(-1, 1) turns, rate U(-1e-4, 1e-4) turns/spectrum"}
    for name in forms:
        ms, _, stats, tiles = run_form(corr, torch, name, inputs, steps, warmup, timing=True, tracking=model)
        n_int = steps * N_INT
        untracked = forms[name]["ms_per_integration"].get("f")
        if untracked is None and pipelines and name in pipelines:
            untracked = pipelines[name]["staged"].get("f_ms_per_integration")
        out[name] = {"antenna_msps": round(a_s / (ms * 1e-3) / 1e6, 1), "ms_per_step": round(ms, 4),
                     "pipeline": tiles["pipeline"], "f_ms_per_integration": round(stats["ms_f"] / n_int, 4),
                     "untracked_f_ms_per_integration": untracked}
        log(f"[bench] tracking {name}: {out[name]}")
    return out


def fused_leg(corr, torch, metrics, inputs, steps, warmup, forms):
    """Both pipelines of the fp32, fp16 and int8 steps: the staged one (F
    launch, X launch and dump per chunk) and the fused one (one persistent
    F + X kernel per integration, records handed over through a cache-sized
    ring, the autotuner's parameters).  The form above ran the pipeline the
    autotuner picked; this leg runs the other one."""
    a_s = N_INT * metrics.antenna_samples(N_ANT, TWO_K, S_INT)
    out = {}
    for name in ("fp32", "fp16", "int8"):
        if name not in forms:
            continue
        ran = forms[name]["tiles"]["pipeline"]
        other = "staged" if ran == "fused" else "fused"
        ms, _, stats, tiles = run_form(corr, torch, name, inputs, steps, warmup, timing=True, pipeline=other)
        n_int = steps * N_INT
        times = {ran: forms[name]["ms_per_step"], other: round(ms, 4)}
        out[name] = {"staged": {"ms_per_step": times["staged"],
                                "antenna_msps": round(a_s / (times["staged"] * 1e-3) / 1e6, 1)},
                     "fused": {"ms_per_step": times["fused"],
                               "antenna_msps": round(a_s / (times["fused"] * 1e-3) / 1e6, 1)},
                     "fused_speedup_vs_staged": round(times["staged"] / times["fused"], 3),
                     "autotuner_pipeline": ran}
        if other == "fused":
            out[name]["fused"]["ms_kernel_per_integration"] = round(stats["ms_fused"] / n_int, 4)
            out[name]["fused"]["tiles"] = tiles
        else:
            out[name]["staged"]["f_ms_per_integration"] = round(stats["ms_f"] / n_int, 4)
            out[name]["staged"]["tiles"] = tiles
        log(f"[bench] pipelines {name}: {out[name]}")
    return out


def ingest_leg(corr, torch, packed):
    """One N = 44 integration assembled from its 65536 frames, shuffled, by
    corr_ingest (frames built on the GPU from one header template)."""
    import synth
    S = S_INT
    stride = (synth.FRAME_HEADER_BYTES + N_ANT * K + 15) // 16 * 16
    hdr = synth.frames(packed[:1].cpu().view(1, N_ANT, K), [0])[0, :synth.FRAME_HEADER_BYTES].cuda()
    frames = torch.empty(S, stride, dtype=torch.uint8, device="cuda")
    frames[:, :synth.FRAME_HEADER_BYTES] = hdr
    frames[:, 8:16] = torch.arange(S, dtype=torch.int64, device="cuda").view(torch.uint8).view(S, 8)
    frames[:, synth.FRAME_HEADER_BYTES:synth.FRAME_HEADER_BYTES + N_ANT * K] = packed.view(S, N_ANT * K)
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    frames = frames[torch.randperm(S, device="cuda", generator=g)].contiguous()
    c = corr.Correlator(N_ANT, K, S)
    out = torch.empty(S * N_ANT * K, dtype=torch.uint8, device="cuda")
    c.ingest(frames, S, stride, 0, out)
    torch.cuda.synchronize()
    exact = bool(torch.equal(out, packed.view(-1)))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    e0.record()
    for _ in range(reps):
        c.ingest(frames, S, stride, 0, out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    st = c.ingest_stats()
    c.close()
    nbytes = S * stride + S * N_ANT * K
    res = {"workload": f"{S} frames of {stride} bytes (N={N_ANT}, {TWO_K}-pt), shuffled",
           "ms_per_integration": round(ms, 4), "gb_per_s": round(nbytes / (ms * 1e-3) / 1e9, 1),
           "bytes_moved": nbytes, "assembled_exactly": exact, "stats": st}
    log(f"[bench] ingest: {res}")
    return res


def accuracy(corr, torch, precision):
    """Coefficient error vs the float64 oracle on the first 1024 spectra."""
    import numpy as np
    import oracle
    import synth
    S = 1024
    recipe = synth.recipe_plain(N=N_ANT, two_k=TWO_K, rho=0.05, seed=1)
    packed = synth.packed(recipe, 0, S, device="cpu").contiguous()
    c = corr.Correlator(N_ANT, K, S, precision=precision)
    c.process(packed.cuda())
    v = c.read_cps()
    c.close()
    ref = oracle.correlate(packed.numpy(), S, N_ANT, K)
    auto = np.array([ref[oracle.baseline_index(N_ANT, a, a)].real for a in range(N_ANT)])
    err, bl = 0.0, 0
    for a in range(N_ANT):
        for b in range(a, N_ANT):
            err = max(err, float(np.max(np.abs(v[bl] - ref[bl]) / np.sqrt(auto[a] * auto[b]))))
            bl += 1
    return err


def large_n(corr, torch, metrics, steps, warmup):
    """N = 256 antennas, 1024-point FFT -> 512 channels, 16384 spectra with
    three delayed point sources: the X-stage-dominated case, int8 vs fp32."""
    import synth
    N, two_k, S = 256, 1024, 16384
    Kc = two_k // 2
    x = synth.packed(synth.recipe_sources(N=N, two_k=two_k, seed=4), 0, S, device="cuda").contiguous()
    out = {"workload": f"N={N}, {two_k}-pt FFT -> {Kc} channels, {S} spectra, 3 delayed sources"}
    for prec in ("fp32", "int8"):
        c = corr.Correlator(N, Kc, S, precision=prec, tiles="auto")
        dst = torch.empty(c.nb * Kc * 2, dtype=torch.float64, device="cuda")
        for _ in range(warmup):
            c.process(x); c.read_cps_async(dst)
        c.enable_timing(True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(steps):
            c.process(x); c.read_cps_async(dst)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        st = c.stats()
        x_ms = st["ms_x"] / steps
        out[prec] = {"antenna_msps": round(metrics.antenna_samples(N, two_k, S) / (ms * 1e-3) / 1e6, 1),
                     "ms_per_integration": round(ms, 4),
                     "x_tops": round(metrics.x_ops(N, Kc, S) / (x_ms * 1e-3) / 1e12, 2),
                     "x_mfma": x_mfma(metrics, N, Kc, S, prec, x_ms),
                     "ms_f": round(st["ms_f"] / steps, 4), "ms_x": round(x_ms, 4), "tiles": c.tiles()}
        c.close()
        log(f"[bench] large N {prec}: {out[prec]}")
    del x
    torch.cuda.empty_cache()
    out["int8_speedup_vs_fp32"] = round(out["int8"]["antenna_msps"] / out["fp32"]["antenna_msps"], 3)
    return out


def batch(corr, torch, metrics, steps, warmup):
    """12 uneven jobs, (N, FFT size) drawn from the paper-scale set, 16384
    spectra each, rho ~ U[0, 0.1], all-int8 and all-fp32, replayed from one HIP
    graph in both batch modes (each job's kernels on parallel branches; one
    persistent kernel), against the same jobs as separate correlators."""
    import synth
    recipes = synth.batch_jobs(12, seed=3)
    S = 16384
    xs = [synth.packed(r, 0, S, device="cuda").contiguous() for r in recipes]
    a_s = sum(metrics.antenna_samples(r.N, r.two_k, S) for r in recipes)
    out = {"workload": "12 jobs, (N, 2K) drawn from " + ", ".join(f"({n},{k})" for n, k in synth.BATCH_SHAPES)
           + f", {S} spectra each", "jobs": [[r.N, r.two_k] for r in recipes]}
    def time_batch(prec, mode):
        b = corr.Batch([(r.N, r.K, S, prec) for r in recipes], tiles="auto", mode=mode)
        for _ in range(warmup):
            b.process(xs)
            for j in range(len(recipes)):
                b.read_cps_raw(j)
        times = []
        for _ in range(steps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            b.process(xs)
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
            for j in range(len(recipes)):
                b.read_cps_raw(j)
        b.close()
        return sorted(times)[len(times) // 2]

    for prec in ("fp32", "int8"):
        ms = time_batch(prec, "branches")
        ms_pers = time_batch(prec, "persistent")
        # the same jobs as separate single-job correlators, one after another on
        # one stream (reads outside the timed region, as for the batch)
        cs = [corr.Correlator(r.N, r.K, S, precision=prec, tiles="auto") for r in recipes]
        sep = []
        for it in range(warmup + steps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            for c, x in zip(cs, xs):
                c.process(x)
            e1.record()
            torch.cuda.synchronize()
            if it >= warmup:
                sep.append(e0.elapsed_time(e1))
            for c in cs:
                c.read_cps_raw()
        for c in cs:
            c.close()
        ms_sep = sorted(sep)[len(sep) // 2]
        out[prec] = {"antenna_msps": round(a_s / (ms * 1e-3) / 1e6, 1), "mode": "branches",
                     "ms_per_batch": round(ms, 4), "separate_launches_ms": round(ms_sep, 4),
                     "batch_speedup_vs_separate": round(ms_sep / ms, 3),
                     "persistent_ms_per_batch": round(ms_pers, 4),
                     "persistent_speedup_vs_separate": round(ms_sep / ms_pers, 3)}
        log(f"[bench] batch {prec}: {out[prec]}")
    del xs
    torch.cuda.empty_cache()
    return out


def batch_fresh_process(steps, warmup):
    """The batch leg in a child process of its own (the caller falls back to
    timing it in its own process if the child fails).  A cooperative launch (the
    fused pipeline's kernel, which the headline step runs for fp16) slows every
    later multi-branch graph replay in the same process by about a tenth
    (int8 batch 2.07 -> 2.28 ms, the separate launches unchanged), so the
    batch and the separate launches it is compared with are both timed in a
    process that has made none.  The child's progress lines go to stderr."""
    cmd = [sys.executable, os.path.abspath(__file__), "--only-batch", "--steps", str(steps), "--warmup", str(warmup)]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, text=True, timeout=900)
    if r.returncode != 0:
        raise RuntimeError(f"batch leg failed with exit status {r.returncode}")
    out = json.loads(r.stdout.strip().splitlines()[-1])
    out["process"] = "fresh: no cooperative launch before it"
    return out


def x_mfma(metrics, N, K, S, prec, x_ms):
    """The X-stage's issued MFMA rate against the dense peak of its form
    (issued operations from the block-pair count; rocprofv3's
    SQ_INSTS_VALU_MFMA_MOPS counters give the same totals)."""
    if x_ms <= 0:
        return None
    rate = metrics.x_mfma_ops(N, K, S, prec) / (x_ms * 1e-3) / 1e12
    useful = metrics.x_ops(N, K, S) / (x_ms * 1e-3) / 1e12
    peak = metrics.MFMA_PEAK[prec]
    return {"issued": round(rate, 2), "peak": peak, "unit": "TFLOP/s" if prec.startswith("fp") else "TOPS",
            "frac": round(rate / peak, 4), "useful": round(useful, 2), "useful_frac": round(useful / peak, 4)}


def cpu_identity():
    """The host's CPU model and the logical CPUs this process may run on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    if not model:
        import platform
        model = platform.processor() or platform.machine()
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return model, avail


def cpu_baseline(inputs_cpu_sample, S_sample, S_one_thread, S_large=0):
    """The oracle timed on the host's cores; then on the large-N workload over
    a small sample; then on one thread over a smaller sample (the analogue of
    the paper's multicore-against-one-thread figure)."""
    import oracle
    threads = oracle.get_threads()
    t0 = time.perf_counter()
    oracle.correlate(inputs_cpu_sample, S_sample, N_ANT, K)
    dt = time.perf_counter() - t0
    rate = N_ANT * S_sample * TWO_K / dt / 1e6
    model, avail = cpu_identity()
    out = {"value": round(rate, 3), "unit": "antenna-MS/s", "cores": threads, "kind": "oracle",
           "cpu_model": model, "cpus_available": avail, "threads_used": threads,
           "sample": f"first {S_sample} spectra of integration 1 (N={N_ANT}, 2K={TWO_K}), "
                     f"float64 FFT + pairwise CMAC, {dt:.1f} s"}
    if S_large > 0:
        # the X-dominated case: the N = 256, 1024-point workload's first
        # S_large spectra (linear in spectra, so the rate stands for the whole)
        import synth
        NL, two_kl = 256, 1024
        xl = synth.packed(synth.recipe_sources(N=NL, two_k=two_kl, seed=4), 0, S_large).numpy()
        t0 = time.perf_counter()
        oracle.correlate(xl, S_large, NL, two_kl // 2)
        dtl = time.perf_counter() - t0
        out["large_n"] = {"value": round(NL * S_large * two_kl / dtl / 1e6, 3),
                          "x_gops": round(8.0 * NL * (NL + 1) / 2 * (two_kl // 2) * S_large / dtl / 1e9, 2),
                          "sample": f"first {S_large} spectra of the N={NL}, 2K={two_kl} workload, {dtl:.1f} s"}
    if S_one_thread > 0:
        oracle.set_threads(1)
        try:
            t0 = time.perf_counter()
            oracle.correlate(inputs_cpu_sample[:S_one_thread], S_one_thread, N_ANT, K)
            dt1 = time.perf_counter() - t0
        finally:
            oracle.set_threads(threads)
        rate1 = N_ANT * S_one_thread * TWO_K / dt1 / 1e6
        out["one_thread"] = {"value": round(rate1, 3), "sample": f"first {S_one_thread} spectra, {dt1:.1f} s",
                             "multicore_speedup": round(rate / rate1, 1)}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-spectra", type=int, default=65536)
    ap.add_argument("--cpu-spectra-one-thread", type=int, default=4096)
    ap.add_argument("--cpu-spectra-large-n", type=int, default=1024)
    ap.add_argument("--forms", default="fp32,fp16,int8,int16")
    ap.add_argument("--pipeline", default="tuned", choices=("tuned", "staged", "fused"),
                    help="the pipeline of every form: the autotuner's choice, or one for all (counter runs)")
    ap.add_argument("--no-extra", action="store_true", help="skip every workload beyond the headline step")
    ap.add_argument("--legs", default="fused,tracking,ingest,large_n,batch",
                    help="extra workloads to run after the headline step (comma list)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (scale reference for HBM counters)")
    ap.add_argument("--only-batch", action="store_true",
                    help="run the batch leg alone (--steps / --warmup as given) and print its JSON "
                         "(the full run starts it this way, in a process of its own)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(time-domain sharding across GPUs is a design note, not code)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1102_0148_amd as corr
    from paper_1102_0148_amd import metrics

    torch.cuda.set_device(0)
    if args.only_batch:
        print(json.dumps(batch(corr, torch, metrics, args.steps, args.warmup)))
        return
    if args.copy_probe:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)          # reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        del src, dst
    inputs = make_inputs("cuda")
    torch.cuda.synchronize()

    a_s_per_step = N_INT * metrics.antenna_samples(N_ANT, TWO_K, S_INT)
    xops_per_int = metrics.x_ops(N_ANT, K, S_INT)
    forms = {}
    for name in args.forms.split(","):
        ms, wall_ms, stats, tiles = run_form(corr, torch, name, inputs, args.steps, args.warmup, timing=True,
                                             pipeline=None if args.pipeline == "tuned" else args.pipeline)
        n_int = args.steps * N_INT
        x_ms = stats["ms_x"] / n_int
        f_ms = stats["ms_f"] / n_int
        if tiles["pipeline"] == "fused":
            # the autotuner picked the fused pipeline: one F + X kernel
            forms[name] = {
                "antenna_msps": round(a_s_per_step / (ms * 1e-3) / 1e6, 1),
                "ms_per_step": round(ms, 4),
                "x_tops": None,
                "ms_per_integration": {"fused": round(stats["ms_fused"] / n_int, 4),
                                       "dump": round(stats["ms_dump"] / n_int, 4),
                                       "calib": round(stats["ms_calib"] / n_int, 4)},
                "launches_per_integration": {"fused": stats["launches_fused"] // n_int},
                "tiles": tiles,
            }
            if name in ("int8", "int16"):
                forms[name]["saturated_fraction"] = stats["int8_saturated"] / max(
                    1, (args.steps + args.warmup) * N_INT * S_INT * N_ANT * K * 2)
            log(f"[bench] {name}: {forms[name]}")
            continue
        forms[name] = {
            "antenna_msps": round(a_s_per_step / (ms * 1e-3) / 1e6, 1),
            "ms_per_step": round(ms, 4),
            "x_tops": round(xops_per_int / (x_ms * 1e-3) / 1e12, 2) if x_ms > 0 else None,
            "ms_per_integration": {"f": round(f_ms, 4), "x": round(x_ms, 4),
                                   "dump": round(stats["ms_dump"] / n_int, 4),
                                   "calib": round(stats["ms_calib"] / n_int, 4)},
            "launches_per_integration": {"f": stats["launches_f"] // n_int, "x": stats["launches_x"] // n_int},
            "tiles": tiles,
            "x_mfma": x_mfma(metrics, N_ANT, K, S_INT, name, x_ms),
        }
        forms[name]["f_stage"] = f_stage_bounds(metrics, name, f_ms, tiles["f_group"])
        if name in ("int8", "int16"):
            forms[name]["saturated_fraction"] = stats["int8_saturated"] / max(
                1, (args.steps + args.warmup) * N_INT * S_INT * N_ANT * K * 2)
        log(f"[bench] {name}: {forms[name]}")
    for name in forms:
        forms[name]["coef_error_vs_fp64"] = float("%.3g" % accuracy(corr, torch, name))
        if "fp32" in forms:
            forms[name]["speedup_vs_fp32"] = round(forms[name]["antenna_msps"] / forms["fp32"]["antenna_msps"], 3)

    head = forms.get("fp32") or next(iter(forms.values()))
    ms_step = head["ms_per_step"]
    value = head["antenna_msps"]

    # roofline of the dominant kernel of the headline step
    st = head["ms_per_integration"]
    launches = head["launches_per_integration"]
    chunk = head["tiles"]["chunk_spectra"]
    if "fused" in st:
        # the fused kernel does F and X together; priced by its useful X flops
        flops = metrics.x_ops(N_ANT, K, S_INT)
        achieved = flops / (st["fused"] * 1e-3) / 1e12
        roof = {"kernel": "fx_kernel (fused F + X, fp32)", "bound": "mfma", "achieved": round(achieved, 2),
                "peak": PEAK["fp32_tflops"], "unit": "TFLOP/s", "frac": round(achieved / PEAK["fp32_tflops"], 4),
                "traffic": None, "per_launch": {"useful_flops": flops, "avg_ms": st["fused"]}}
    elif st["x"] >= st["f"]:
        per_launch_ms = st["x"] / max(1, launches["x"])
        flops = metrics.x_ops(N_ANT, K, chunk)
        achieved = flops / (per_launch_ms * 1e-3) / 1e12
        t = measured_traffic("xstage_kernel<0, 3, 1>", chunk)
        roof = {"kernel": "xstage_kernel (fp32 MFMA, Hermitian rank-T update)", "bound": "mfma",
                "achieved": round(achieved, 2), "peak": PEAK["fp32_tflops"], "unit": "TFLOP/s",
                "frac": round(achieved / PEAK["fp32_tflops"], 4), "traffic": t,
                "per_launch": {"useful_flops": flops, "avg_ms": round(per_launch_ms, 4)}}
    else:
        per_launch_ms = st["f"] / max(1, launches["f"])
        nbytes = metrics.antenna_samples(N_ANT, TWO_K, chunk) * (0.5 + 4.0)
        achieved = nbytes / (per_launch_ms * 1e-3) / 1e9
        t = measured_traffic(f"fstage_kernel<256, 0, {head['tiles']['f_group']}, false>", chunk)
        roof = {"kernel": "fstage_kernel (unpack + FFT + corner turn, fp32 records)", "bound": "hbm",
                "achieved": round(achieved, 1), "peak": PEAK["hbm_gbs"], "unit": "GB/s",
                "frac": round(achieved / PEAK["hbm_gbs"], 4), "traffic": t,
                "per_launch": {"algorithmic_bytes": nbytes, "avg_ms": round(per_launch_ms, 4)}}

    out = {
        "metric": "antenna-MS/s sustained (F+X) and X-stage TOPS: int8/FP16 vs FP32 path",
        "value": value,
        "unit": "antenna-MS/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": round(value / PAPER_ANTENNA_MSPS, 1),
        "baseline_note": "paper: ~735 MB/s of 4-bit input = 1470 antenna-MS/s on 4 dual Xeon E5430 nodes",
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"FX correlator N={N_ANT} antennas, {TWO_K}-pt real FFT -> {K} channels, "
                               f"{S_INT} spectra/integration x {N_INT} integrations, float32 path",
                   "N": N_ANT, "fft_points": TWO_K, "channels": K, "spectra_per_integration": S_INT,
                   "integrations_per_step": N_INT, "parallelism": "single GPU"},
        "x_tops": head["x_tops"],
        "forms": forms,
        "roofline": roof,
    }
    legs = set() if args.no_extra else set(x for x in args.legs.split(",") if x)
    if "fused" in legs:
        out["fused"] = fused_leg(corr, torch, metrics, inputs, max(2, args.steps // 2), 1, forms)
    if "tracking" in legs:
        out["tracking"] = tracking_leg(corr, torch, metrics, inputs, max(2, args.steps // 3), 1, forms,
                                       out.get("fused"))
    if "ingest" in legs:
        out["ingest"] = ingest_leg(corr, torch, inputs[0])
    del inputs
    torch.cuda.empty_cache()
    if "large_n" in legs:
        out["large_n"] = large_n(corr, torch, metrics, max(2, args.steps // 3), 1)
    if "batch" in legs:
        try:
            out["batch"] = batch_fresh_process(max(3, args.steps // 3), 1)
        except (RuntimeError, OSError, ValueError, subprocess.SubprocessError) as e:
            log(f"[bench] batch leg in a child process failed ({e}); timing it in this process")
            out["batch"] = batch(corr, torch, metrics, max(3, args.steps // 3), 1)
            out["batch"]["process"] = "this one, after a cooperative launch (the child process failed)"
    if not args.no_cpu_baseline:
        import numpy as np
        import synth
        recipe = synth.recipe_plain(N=N_ANT, two_k=TWO_K, rho=0.05, seed=1)
        sample = synth.packed(recipe, 0, args.cpu_spectra, device="cuda").cpu().numpy()
        out["cpu_baseline"] = cpu_baseline(sample, args.cpu_spectra, min(args.cpu_spectra_one_thread, args.cpu_spectra),
                                           args.cpu_spectra_large_n)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
