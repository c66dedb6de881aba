"""MI355X FX spectral correlator: Python binding of libcorr.so.

Module-level functions carry the C ABI's names (include/corr.h) and only
marshal arguments; every step of the correlator runs in the library's HIP
kernels.  PyTorch supplies device memory and streams.  If libcorr.so is not
built, the first call raises -- there is no CPU fallback.

    import paper_1102_0148_amd as corr
    c = corr.Correlator(N=44, K=256, n_spectra=1024)     # FP32 path
    c.process(packed_uint8_cuda_tensor)                  # [S][N][K] bytes
    vis = c.read_cps()                                   # complex64 [nb][K]
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcorr.so")

CORR_OK, CORR_EINVAL, CORR_ENOMEM, CORR_EHIP, CORR_ESTATE = 0, -1, -2, -3, -4
CORR_FP32, CORR_FP16, CORR_INT8, CORR_INT16 = 0, 1, 2, 3
CORR_CALIB_SPECTRA = 1024
CORR_MAX_ANTENNAS, CORR_MAX_CHANNELS = 512, 1024
PRECISIONS = {"fp32": CORR_FP32, "fp16": CORR_FP16, "int8": CORR_INT8, "int16": CORR_INT16}
CORR_BATCH_BRANCHES, CORR_BATCH_PERSISTENT = 0, 1
CORR_PIPELINE_STAGED, CORR_PIPELINE_FUSED = 0, 1
PIPELINES = {"staged": CORR_PIPELINE_STAGED, "fused": CORR_PIPELINE_FUSED}
BATCH_MODES = {"branches": CORR_BATCH_BRANCHES, "persistent": CORR_BATCH_PERSISTENT}

# Every symbol include/corr.h declares.
EXPORTS = (
    "corr_create", "corr_set_precision", "corr_set_tiles", "corr_get_tiles", "corr_process",
    "corr_set_tracking", "corr_ingest", "corr_get_ingest_stats",
    "corr_read_cps", "corr_read_cps_raw", "corr_read_cps_async", "corr_read_scales",
    "corr_spectra_bytes", "corr_process_spectra", "corr_debug_read_spectra", "corr_get_stats",
    "corr_enable_timing", "corr_destroy", "corr_last_error", "corr_batch_create",
    "corr_batch_set_tiles", "corr_batch_set_mode", "corr_batch_process", "corr_batch_read_cps",
    "corr_batch_read_cps_raw", "corr_batch_read_scales", "corr_process_noalloc", "corr_set_pipeline",
)


class CorrError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"[{code}] {message}")
        self.code = code


class corr_tiles(ctypes.Structure):
    _fields_ = [("chunk_spectra", ctypes.c_int), ("x_splits", ctypes.c_int), ("f_group", ctypes.c_int)]


class corr_stats(ctypes.Structure):
    _fields_ = [("spectra_accumulated", ctypes.c_int64), ("int8_saturated", ctypes.c_int64),
                ("precision", ctypes.c_int), ("chunk_spectra", ctypes.c_int),
                ("x_splits", ctypes.c_int), ("f_group", ctypes.c_int),
                ("ms_calib", ctypes.c_double), ("ms_f", ctypes.c_double),
                ("ms_x", ctypes.c_double), ("ms_dump", ctypes.c_double),
                ("launches_f", ctypes.c_int64), ("launches_x", ctypes.c_int64),
                ("ms_fused", ctypes.c_double), ("launches_fused", ctypes.c_int64)]


class corr_ingest_stats(ctypes.Structure):
    _fields_ = [("frames_accepted", ctypes.c_int64), ("frames_rejected", ctypes.c_int64),
                ("frames_duplicate", ctypes.c_int64), ("spectra_lost", ctypes.c_int64)]


class corr_job(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int), ("K", ctypes.c_int), ("n_spectra", ctypes.c_int),
                ("precision", ctypes.c_int)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libcorr.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1102_0148_amd.build` "
                           "(there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    P, I, I64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
    sigs = {
        "corr_create": (P, [I, I, I]),
        "corr_set_precision": (I, [P, I]),
        "corr_set_tiles": (I, [P, ctypes.POINTER(corr_tiles)]),
        "corr_get_tiles": (I, [P, ctypes.POINTER(corr_tiles)]),
        "corr_process": (I, [P, P, P]),
        "corr_set_tracking": (I, [P, P, P, P, P]),
        "corr_ingest": (I, [P, P, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64, P, P]),
        "corr_get_ingest_stats": (I, [P, ctypes.POINTER(corr_ingest_stats)]),
        "corr_read_cps": (I, [P, P]),
        "corr_read_cps_raw": (I, [P, P]),
        "corr_read_cps_async": (I, [P, P, P]),
        "corr_read_scales": (I, [P, P]),
        "corr_spectra_bytes": (ctypes.c_size_t, [P, I]),
        "corr_process_spectra": (I, [P, P, I, P]),
        "corr_debug_read_spectra": (I, [P, P, ctypes.POINTER(I)]),
        "corr_get_stats": (I, [P, ctypes.POINTER(corr_stats)]),
        "corr_enable_timing": (I, [P, I]),
        "corr_destroy": (None, [P]),
        "corr_last_error": (ctypes.c_char_p, []),
        "corr_batch_create": (P, [ctypes.POINTER(corr_job), I]),
        "corr_batch_set_tiles": (I, [P, I, ctypes.POINTER(corr_tiles)]),
        "corr_batch_set_mode": (I, [P, I]),
        "corr_batch_process": (I, [P, ctypes.POINTER(P), P]),
        "corr_batch_read_cps": (I, [P, I, P]),
        "corr_batch_read_cps_raw": (I, [P, I, P]),
        "corr_batch_read_scales": (I, [P, I, P]),
        "corr_process_noalloc": (I, [I, I, I, I, P, P, P, P]),
        "corr_set_pipeline": (I, [P, I, I, I, I, I]),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def corr_last_error() -> str:
    return load().corr_last_error().decode()


def _check(rc: int) -> int:
    if rc != CORR_OK:
        raise CorrError(rc, corr_last_error())
    return rc


def _handle(h):
    if not h:
        raise CorrError(CORR_EINVAL, corr_last_error() or "creation failed")
    return h


# ------------------------------------------------ C ABI, one wrapper per call

def corr_create(N: int, K: int, n_spectra: int):
    return _handle(load().corr_create(N, K, n_spectra))


def corr_set_precision(h, mode: int):
    return _check(load().corr_set_precision(h, mode))


def corr_ingest(h, frames_ptr: int, n_frames: int, frame_stride: int, first_seq: int, out_ptr: int,
                stream: int = 0):
    return _check(load().corr_ingest(h, frames_ptr, n_frames, frame_stride, first_seq, out_ptr, stream))


def corr_get_ingest_stats(h) -> dict:
    st = corr_ingest_stats()
    _check(load().corr_get_ingest_stats(h, ctypes.byref(st)))
    return {name: getattr(st, name) for name, _ in corr_ingest_stats._fields_}


def corr_set_tracking(h, delay=None, delay_rate=None, phase=None, phase_rate=None, N=None):
    """Arrays of N float64 (or None for zeros); all None switches tracking off."""
    arrs = []
    for v in (delay, delay_rate, phase, phase_rate):
        if v is None:
            arrs.append(None)
        else:
            a = np.ascontiguousarray(v, dtype=np.float64).ravel()
            if N is not None and a.size != N:
                raise ValueError(f"tracking arrays hold N={N} values, got {a.size}")
            arrs.append(a)
    ptrs = [None if a is None else _np_ptr(a) for a in arrs]
    return _check(load().corr_set_tracking(h, *ptrs))


def corr_set_tiles(h, chunk_spectra=0, x_splits=0, f_group=0):
    t = corr_tiles(chunk_spectra, x_splits, f_group)
    return _check(load().corr_set_tiles(h, ctypes.byref(t)))


def corr_get_tiles(h) -> dict:
    t = corr_tiles()
    _check(load().corr_get_tiles(h, ctypes.byref(t)))
    return {"chunk_spectra": t.chunk_spectra, "x_splits": t.x_splits, "f_group": t.f_group}


def corr_set_pipeline(h, pipeline: int, chunk_spectra: int = 0, ring_slots: int = 0, f_workgroups_per_cu: int = 0,
                      f_cus_per_xcd: int = 0):
    return _check(load().corr_set_pipeline(h, pipeline, chunk_spectra, ring_slots, f_workgroups_per_cu,
                                           f_cus_per_xcd))


def corr_process(h, packed_ptr: int, stream: int = 0):
    return _check(load().corr_process(h, packed_ptr, stream))


def corr_read_cps(h, out_ptr: int):
    return _check(load().corr_read_cps(h, out_ptr))


def corr_read_cps_raw(h, out_ptr: int):
    return _check(load().corr_read_cps_raw(h, out_ptr))


def corr_read_cps_async(h, dst_ptr: int, stream: int = 0):
    return _check(load().corr_read_cps_async(h, dst_ptr, stream))


def corr_read_scales(h, out_ptr: int):
    return _check(load().corr_read_scales(h, out_ptr))


def corr_spectra_bytes(h, n_spectra: int) -> int:
    return int(load().corr_spectra_bytes(h, n_spectra))


def corr_process_spectra(h, spectra_ptr: int, n_spectra: int, stream: int = 0):
    return _check(load().corr_process_spectra(h, spectra_ptr, n_spectra, stream))


def corr_debug_read_spectra(h, out_ptr: Optional[int]) -> int:
    n = ctypes.c_int(0)
    _check(load().corr_debug_read_spectra(h, out_ptr, ctypes.byref(n)))
    return n.value


def corr_get_stats(h) -> dict:
    s = corr_stats()
    _check(load().corr_get_stats(h, ctypes.byref(s)))
    return {name: getattr(s, name) for name, _ in corr_stats._fields_}


def corr_enable_timing(h, on: bool):
    return _check(load().corr_enable_timing(h, int(bool(on))))


def corr_destroy(h):
    if h:
        load().corr_destroy(h)


def corr_process_noalloc(N: int, K: int, n_spectra: int, precision: int, packed_ptr: int, cps_ptr: int,
                         scales_ptr: Optional[int] = None, stream: int = 0):
    return _check(load().corr_process_noalloc(N, K, n_spectra, precision, packed_ptr, cps_ptr, scales_ptr,
                                              stream))


def corr_batch_create(jobs):
    arr = (corr_job * len(jobs))(*[corr_job(*j) for j in jobs])
    return _handle(load().corr_batch_create(arr, len(jobs)))


def corr_batch_set_tiles(b, job: int, chunk_spectra=0, x_splits=0, f_group=0):
    t = corr_tiles(chunk_spectra, x_splits, f_group)
    return _check(load().corr_batch_set_tiles(b, job, ctypes.byref(t)))


def corr_batch_set_mode(b, mode: int):
    return _check(load().corr_batch_set_mode(b, mode))


def corr_batch_process(b, packed_ptrs, stream: int = 0):
    arr = (ctypes.c_void_p * len(packed_ptrs))(*packed_ptrs)
    return _check(load().corr_batch_process(b, arr, stream))


def corr_batch_read_cps(b, job: int, out_ptr: int):
    return _check(load().corr_batch_read_cps(b, job, out_ptr))


def corr_batch_read_cps_raw(b, job: int, out_ptr: int):
    return _check(load().corr_batch_read_cps_raw(b, job, out_ptr))


def corr_batch_read_scales(b, job: int, out_ptr: int):
    return _check(load().corr_batch_read_scales(b, job, out_ptr))


# ------------------------------------------------ torch-facing convenience

def _stream(stream) -> int:
    import torch
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _np_ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def n_baselines(N: int) -> int:
    return N * (N + 1) // 2


class Correlator:
    """One correlation (N antennas, K channels, n_spectra per integration)."""

    def __init__(self, N: int, K: int, n_spectra: int, precision="fp32", tiles=None, pipeline=None):
        """tiles: None (library defaults), "auto" (the autotuner's table,
        defaults where it has no entry) or a dict of corr_tiles fields.
        pipeline: None (with tiles="auto": the pipeline the autotuner found
        faster for this shape, else staged), "staged", or "fused" optionally
        with its parameters as a dict {"chunk_spectra", "ring_slots",
        "f_workgroups_per_cu", "f_cus_per_xcd"} (with tiles="auto", the
        autotuner's fused entry when it has one). A fused pipeline that only the autotuner chose gives
        way to the staged one with its tuned tiles when tracking is switched
        on before the first process() (the fused kernel does not track)."""
        self.N, self.K, self.S = N, K, n_spectra
        self.nb = n_baselines(N)
        self._fused = False
        self._staged_fallback = None
        self.h = corr_create(N, K, n_spectra)
        try:
            mode = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
            corr_set_precision(self.h, mode)
            self.precision = mode
            name = {v: k for k, v in PRECISIONS.items()}[mode]
            auto = isinstance(tiles, str) and tiles == "auto"
            chosen = False
            if pipeline is None and auto:
                from . import tune
                staged = tune.lookup(N, K, n_spectra, name)
                if staged and staged.get("pipeline") == "fused":
                    pipeline, chosen = "fused", True
            fused = pipeline == "fused" or isinstance(pipeline, dict)
            if fused:
                params = dict(pipeline) if isinstance(pipeline, dict) else {}
                if not params and isinstance(tiles, str) and tiles == "auto":
                    from . import tune
                    found = tune.lookup(N, K, n_spectra, name, mode="fused")
                    params = {k: found[k] for k in ("chunk_spectra", "ring_slots", "f_workgroups_per_cu",
                                                    "f_cus_per_xcd") if k in found} if found else {}
                corr_set_pipeline(self.h, CORR_PIPELINE_FUSED, **params)
                if chosen:
                    self._staged_fallback = {k: staged[k] for k in ("chunk_spectra", "x_splits", "f_group")} \
                        if "x_splits" in staged else {}
                tiles = None
                self._fused = True
            elif pipeline not in (None, "staged"):
                raise ValueError(f"unknown pipeline {pipeline!r}")
            if isinstance(tiles, str) and tiles == "auto":
                from . import tune
                found = tune.lookup(N, K, n_spectra, name)
                tiles = {k: found[k] for k in ("chunk_spectra", "x_splits", "f_group")} \
                    if found and "chunk_spectra" in found else None
            if tiles:
                corr_set_tiles(self.h, **tiles)
        except Exception:
            self.close()
            raise

    def close(self):
        if getattr(self, "h", None):
            corr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def tiles(self) -> dict:
        return corr_get_tiles(self.h)

    @property
    def pipeline(self) -> str:
        return "fused" if self._fused else "staged"

    def process(self, packed, stream=None):
        """packed: uint8 CUDA tensor holding n_spectra*N*K bytes."""
        assert packed.is_cuda and packed.numel() == self.S * self.N * self.K
        corr_process(self.h, packed.data_ptr(), _stream(stream))

    def ingest(self, frames, n_frames: int, frame_stride: int, first_seq: int, out=None, stream=None):
        """Assemble this integration from frames (a uint8 CUDA tensor holding
        n_frames frames of frame_stride bytes) into `out` (a uint8 CUDA tensor
        of n_spectra*N*K bytes, allocated if None), which is returned."""
        assert frames.is_cuda and frames.numel() >= n_frames * frame_stride
        if out is None:
            import torch
            out = torch.empty(self.S * self.N * self.K, dtype=torch.uint8, device=frames.device)
        assert out.is_cuda and out.numel() == self.S * self.N * self.K
        corr_ingest(self.h, frames.data_ptr(), n_frames, frame_stride, first_seq, out.data_ptr(), _stream(stream))
        return out

    def ingest_stats(self) -> dict:
        return corr_get_ingest_stats(self.h)

    def set_tracking(self, delay=None, delay_rate=None, phase=None, phase_rate=None):
        """Per-antenna delay (samples), delay rate (samples per spectrum), phase
        (turns) and phase rate (turns per spectrum) applied to the spectra
        before accumulation, from the next process() on; no arguments switch
        tracking off."""
        on = any(v is not None for v in (delay, delay_rate, phase, phase_rate))
        if on and self._fused and self._staged_fallback is not None:
            corr_set_pipeline(self.h, CORR_PIPELINE_STAGED)
            if self._staged_fallback:
                corr_set_tiles(self.h, **self._staged_fallback)
            self._fused, self._staged_fallback = False, None
        corr_set_tracking(self.h, delay, delay_rate, phase, phase_rate, N=self.N)

    def spectra_bytes(self, n_spectra: int) -> int:
        return corr_spectra_bytes(self.h, n_spectra)

    def process_spectra(self, spectra, n_spectra: int, stream=None):
        """spectra: CUDA tensor in the library's record layout."""
        assert spectra.is_cuda and spectra.numel() * spectra.element_size() >= self.spectra_bytes(n_spectra)
        corr_process_spectra(self.h, spectra.data_ptr(), n_spectra, _stream(stream))

    def read_cps_raw(self) -> np.ndarray:
        out = np.empty((self.nb, self.K, 2), dtype=np.float64)
        corr_read_cps_raw(self.h, _np_ptr(out))
        return out

    def read_cps(self) -> np.ndarray:
        out = np.empty((self.nb, self.K, 2), dtype=np.float32)
        corr_read_cps(self.h, _np_ptr(out))
        return out[..., 0] + 1j * out[..., 1]

    def read_cps_async(self, dst, stream=None):
        """dst: float64 CUDA tensor with nb*K*2 elements."""
        assert dst.numel() == self.nb * self.K * 2
        corr_read_cps_async(self.h, dst.data_ptr(), _stream(stream))

    def read_scales(self) -> np.ndarray:
        out = np.empty((self.N, self.K), dtype=np.float32)
        corr_read_scales(self.h, _np_ptr(out))
        return out

    def debug_read_spectra(self):
        n = corr_debug_read_spectra(self.h, None)
        out = np.empty(self.spectra_bytes(n), dtype=np.uint8)
        corr_debug_read_spectra(self.h, _np_ptr(out))
        return out, n

    def stats(self) -> dict:
        return corr_get_stats(self.h)

    def enable_timing(self, on: bool = True):
        corr_enable_timing(self.h, on)


# ------------------------------------------------ record layout (host side)

def record_times(precision: int) -> int:
    return {CORR_FP32: 2, CORR_FP16: 4, CORR_INT8: 8, CORR_INT16: 4}[precision]


TQB = 16  # records per time block


def a_pad_of(N: int) -> int:
    nblk = (N + 15) // 16
    return 16 * nblk if nblk <= 6 else (N + 63) // 64 * 64


def int16_digits(q: np.ndarray):
    """Base-255 digits of int16 codes (|q| <= 32512): q = 255 h + l, h and l
    in [-127, 127]."""
    q = np.asarray(q, dtype=np.int64)
    h = (2 * q + 255) // 510          # floor((q + 127.5) / 255)
    return h.astype(np.int8), (q - 255 * h).astype(np.int8)


def spectra_to_records(spec: np.ndarray, precision: int) -> np.ndarray:
    """Lay out spectra [S][N][K] (complex for fp32/fp16; integer [S][N][K][2]
    for int8 and int16) as the library's records [tq/16][K][tq%16][a_pad][re x
    TG | im x TG]; int16 records hold [h of re | h of im | l of re | l of im]
    (base-255 digits)."""
    tg = record_times(precision)
    if precision == CORR_INT16:
        S, N, K, _ = spec.shape
        a_pad = a_pad_of(N)
        ntq = ((S + tg - 1) // tg + TQB - 1) // TQB * TQB
        out = np.zeros((ntq // TQB, K, TQB, a_pad, 2, 2, tg), dtype=np.int8)
        tq = np.arange(S) // tg
        tb, tr, tt = tq // TQB, tq % TQB, np.arange(S) % tg
        for comp in range(2):
            h, l = int16_digits(np.transpose(spec[..., comp], (0, 2, 1)))
            out[tb, :, tr, :N, 0, comp, tt] = h
            out[tb, :, tr, :N, 1, comp, tt] = l
        return out.view(np.uint8).reshape(-1)
    if precision == CORR_INT8:
        S, N, K, _ = spec.shape
        re, im = spec[..., 0], spec[..., 1]
        dt = np.int8
    else:
        S, N, K = spec.shape
        re, im = spec.real, spec.imag
        dt = np.float32 if precision == CORR_FP32 else np.float16
    a_pad = a_pad_of(N)
    ntq = ((S + tg - 1) // tg + TQB - 1) // TQB * TQB
    out = np.zeros((ntq // TQB, K, TQB, a_pad, 2, tg), dtype=dt)
    tq = np.arange(S) // tg
    tb, tr, tt = tq // TQB, tq % TQB, np.arange(S) % tg
    # advanced indices (tb, tr, 0, tt) around the channel slice: [S][K][N]
    out[tb, :, tr, :N, 0, tt] = np.transpose(re, (0, 2, 1)).astype(dt)
    out[tb, :, tr, :N, 1, tt] = np.transpose(im, (0, 2, 1)).astype(dt)
    return out.view(np.uint8).reshape(-1)


def records_to_spectra(buf: np.ndarray, precision: int, N: int, K: int, S: int) -> np.ndarray:
    """Inverse of spectra_to_records: complex64 [S][N][K] (fp32/fp16, as float),
    int8 [S][N][K][2] (int8) or int16 [S][N][K][2] (int16)."""
    tg = record_times(precision)
    if precision == CORR_INT16:
        a_pad = a_pad_of(N)
        ntq = ((S + tg - 1) // tg + TQB - 1) // TQB * TQB
        rec = np.asarray(buf).view(np.int8)[: ntq * K * a_pad * 4 * tg].reshape(ntq // TQB, K, TQB, a_pad, 2, 2, tg)
        tq = np.arange(S) // tg
        tb, tr, tt = tq // TQB, tq % TQB, np.arange(S) % tg
        out = []
        for comp in range(2):
            h = rec[tb, :, tr, :N, 0, comp, tt].astype(np.int32)
            l = rec[tb, :, tr, :N, 1, comp, tt].astype(np.int32)
            out.append(np.transpose(255 * h + l, (0, 2, 1)).astype(np.int16))
        return np.stack(out, axis=-1)
    dt = {CORR_FP32: np.float32, CORR_FP16: np.float16, CORR_INT8: np.int8}[precision]
    a_pad = a_pad_of(N)
    ntq = ((S + tg - 1) // tg + TQB - 1) // TQB * TQB
    rec = np.asarray(buf).view(dt)[: ntq * K * a_pad * 2 * tg].reshape(ntq // TQB, K, TQB, a_pad, 2, tg)
    tq = np.arange(S) // tg
    tb, tr, tt = tq // TQB, tq % TQB, np.arange(S) % tg
    re = rec[tb, :, tr, :N, 0, tt]      # [S][K][N]
    im = rec[tb, :, tr, :N, 1, tt]
    re = np.transpose(re, (0, 2, 1))
    im = np.transpose(im, (0, 2, 1))
    if precision == CORR_INT8:
        return np.stack([re, im], axis=-1)
    return re.astype(np.float32) + 1j * im.astype(np.float32)


class Batch:
    """Many correlations of different shapes replayed from one captured HIP
    graph: each job's own kernels on parallel branches ("branches", the
    default) or one persistent kernel over every job ("persistent").
    jobs: list of (N, K, n_spectra, precision); tiles: "auto" (the
    autotuner's table) or {job index: corr_tiles fields}."""

    def __init__(self, jobs, tiles=None, mode="branches"):
        self.jobs = [(int(N), int(K), int(S), PRECISIONS[p] if isinstance(p, str) else int(p))
                     for (N, K, S, p) in jobs]
        self.mode = BATCH_MODES[mode] if isinstance(mode, str) else int(mode)
        self.h = corr_batch_create(self.jobs)
        if isinstance(tiles, str) and tiles == "auto":
            from . import tune
            names = {v: k for k, v in PRECISIONS.items()}
            tiles = {}
            for j, (N, K, S, p) in enumerate(self.jobs):
                # a branch runs the single-job kernels with the single-job
                # entry; the persistent kernel has entries of its own (one
                # chunk and its F group per job, x_splits tuned)
                if self.mode == CORR_BATCH_PERSISTENT:
                    found = tune.lookup(N, K, S, names[p], batch="persistent")
                    if found:
                        tiles[j] = {"x_splits": found["x_splits"]}
                else:
                    found = tune.lookup(N, K, S, names[p])
                    if found:
                        tiles[j] = {k: found[k] for k in ("chunk_spectra", "x_splits", "f_group")}
        try:
            corr_batch_set_mode(self.h, self.mode)
            for j, t in (tiles or {}).items():
                corr_batch_set_tiles(self.h, j, **t)
        except Exception:
            self.close()
            raise

    def close(self):
        if getattr(self, "h", None):
            corr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def process(self, packed_list, stream=None):
        assert len(packed_list) == len(self.jobs)
        for (N, K, S, _), x in zip(self.jobs, packed_list):
            assert x.is_cuda and x.numel() == S * N * K
        corr_batch_process(self.h, [x.data_ptr() for x in packed_list], _stream(stream))

    def read_cps_raw(self, j: int) -> np.ndarray:
        N, K, _, _ = self.jobs[j]
        out = np.empty((n_baselines(N), K, 2), dtype=np.float64)
        corr_batch_read_cps_raw(self.h, j, _np_ptr(out))
        return out

    def read_cps(self, j: int) -> np.ndarray:
        N, K, _, _ = self.jobs[j]
        out = np.empty((n_baselines(N), K, 2), dtype=np.float32)
        corr_batch_read_cps(self.h, j, _np_ptr(out))
        return out[..., 0] + 1j * out[..., 1]

    def read_scales(self, j: int) -> np.ndarray:
        N, K, _, _ = self.jobs[j]
        out = np.empty((N, K), dtype=np.float32)
        corr_batch_read_scales(self.h, j, _np_ptr(out))
        return out
