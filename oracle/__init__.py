"""CPU oracle for the FX correlator -- test infrastructure only.

This package is the slow, obviously correct reference the GPU path is checked
against.  Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import it.  The correlator library and its Python binding never
import, link or fall back to it, and it shares no code with them.

The arithmetic lives in ``oracle.c`` (plain C, float64 and exact int64), built
into ``liboracle.so`` by :func:`build`.  This module only marshals numpy arrays
into it.  What each function computes, and the readings of the paper it takes,
are stated in the C file's header.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(verbose: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (OpenMP, -O2, no fast-math)."""
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
           "-fno-fast-math", "-ffp-contract=off", _SRC, "-o", _LIB_PATH + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    i32, i64 = ctypes.c_int, ctypes.c_int64
    sigs = {
        "orc_baseline_index": (i64, [i32, i32, i32]),
        "orc_unpack": (i32, [P, i64, P]),
        "orc_fft": (i32, [i32, P, P]),
        "orc_fft_real": (i32, [P, i32, P]),
        "orc_spectra": (i32, [P, i32, i32, i32, P]),
        "orc_cmac_f64": (i32, [P, i32, i32, i32, i32, P]),
        "orc_scales": (i32, [P, i32, i32, i32, i32, P]),
        "orc_quantise": (i32, [P, i32, i32, i32, P, P]),
        "orc_cmac_i64": (i32, [P, i32, i32, i32, i32, P]),
        "orc_vis_single": (i32, [P, i32, i32, i32, i32, i32, i32, P]),
        "orc_track": (i32, [P, i32, i32, i32, i32, P, P, P, P]),
        "orc_ingest": (i32, [P, i64, i64, ctypes.c_uint64, i32, i32, i32, i32, P, P, P]),
        "orc_scales_n": (i32, [P, i32, i32, i32, i32, i32, ctypes.c_double, ctypes.c_double, P]),
        "orc_quantise16": (i32, [P, i32, i32, i32, P, P]),
        "orc_cmac_i64_16": (i32, [P, i32, i32, i32, i32, P]),
        "orc_set_threads": (i32, [i32]),
        "orc_get_threads": (i32, []),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(rc: int, name: str):
    if rc != 0:
        raise ValueError(f"{name} failed with status {rc}")


def n_baselines(N: int) -> int:
    return N * (N + 1) // 2


def baseline_index(N: int, a: int, b: int) -> int:
    return int(_load().orc_baseline_index(N, a, b))


def unpack(packed: np.ndarray) -> np.ndarray:
    """Signed 4-bit samples, low nibble first: uint8[...] -> int8[2*size]."""
    packed = np.ascontiguousarray(packed, dtype=np.uint8).ravel()
    out = np.empty(packed.size * 2, dtype=np.int8)
    _check(_load().orc_unpack(_ptr(packed), out.size, _ptr(out)), "orc_unpack")
    return out


def fft(z: np.ndarray) -> np.ndarray:
    """Forward, unnormalised complex FFT (power-of-two length) in float64."""
    z = np.asarray(z, dtype=np.complex128).ravel()
    re = np.ascontiguousarray(z.real)
    im = np.ascontiguousarray(z.imag)
    _check(_load().orc_fft(z.size, _ptr(re), _ptr(im)), "orc_fft")
    return re + 1j * im


def fft_real(x: np.ndarray) -> np.ndarray:
    """All 2K bins of the DFT of one real block (float64)."""
    x = np.ascontiguousarray(x, dtype=np.float64).ravel()
    out = np.empty((x.size, 2), dtype=np.float64)
    _check(_load().orc_fft_real(_ptr(x), x.size, _ptr(out)), "orc_fft_real")
    return out[:, 0] + 1j * out[:, 1]


def spectra(packed: np.ndarray, S: int, N: int, K: int) -> np.ndarray:
    """packed uint8 [S][N][K] -> complex128 spectra [S][N][K] (bins 0..K-1)."""
    packed = np.ascontiguousarray(packed, dtype=np.uint8)
    assert packed.size == S * N * K
    out = np.empty((S, N, K, 2), dtype=np.float64)
    _check(_load().orc_spectra(_ptr(packed), S, N, K, _ptr(out)), "orc_spectra")
    return out[..., 0] + 1j * out[..., 1]


def _spec_pairs(spec: np.ndarray) -> np.ndarray:
    spec = np.asarray(spec)
    pairs = np.empty(spec.shape + (2,), dtype=np.float64)
    pairs[..., 0] = spec.real
    pairs[..., 1] = spec.imag
    return pairs


def cmac_f64(spec: np.ndarray, full: bool = False) -> np.ndarray:
    """complex spectra [S][N][K] -> visibilities complex128.

    full=False: [nb][K] over a <= b in baseline order; full=True: [N][N][K].
    """
    S, N, K = spec.shape
    pairs = _spec_pairs(spec)
    rows = N * N if full else n_baselines(N)
    vis = np.empty((rows, K, 2), dtype=np.float64)
    _check(_load().orc_cmac_f64(_ptr(pairs), S, N, K, int(full), _ptr(vis)), "orc_cmac_f64")
    out = vis[..., 0] + 1j * vis[..., 1]
    return out.reshape(N, N, K) if full else out


def scales(spec: np.ndarray, W: int) -> np.ndarray:
    """int8 calibration scales float32 [N][K] from the first W spectra."""
    S, N, K = spec.shape
    pairs = _spec_pairs(spec)
    out = np.empty((N, K), dtype=np.float32)
    _check(_load().orc_scales(_ptr(pairs), S, N, K, W, _ptr(out)), "orc_scales")
    return out


def quantise(spec: np.ndarray, sc: np.ndarray) -> np.ndarray:
    """complex spectra [S][N][K] + scales [N][K] -> int8 [S][N][K][2] (re, im)."""
    S, N, K = spec.shape
    pairs = _spec_pairs(spec)
    sc = np.ascontiguousarray(sc, dtype=np.float32)
    assert sc.shape == (N, K)
    q = np.empty((S, N, K, 2), dtype=np.int8)
    _check(_load().orc_quantise(_ptr(pairs), S, N, K, _ptr(sc), _ptr(q)), "orc_quantise")
    return q


def cmac_i64(q: np.ndarray, full: bool = False) -> np.ndarray:
    """int8 [S][N][K][2] -> exact int64 visibilities [rows][K][2] (re, im)."""
    q = np.ascontiguousarray(q, dtype=np.int8)
    S, N, K, two = q.shape
    assert two == 2
    rows = N * N if full else n_baselines(N)
    vis = np.empty((rows, K, 2), dtype=np.int64)
    _check(_load().orc_cmac_i64(_ptr(q), S, N, K, int(full), _ptr(vis)), "orc_cmac_i64")
    return vis.reshape(N, N, K, 2) if full else vis


def vis_single(packed: np.ndarray, S: int, N: int, K: int, a: int, b: int, k: int) -> complex:
    """One visibility V[a,b,k] from single-bin DFTs of the packed samples."""
    packed = np.ascontiguousarray(packed, dtype=np.uint8)
    assert packed.size == S * N * K
    out = np.empty(2, dtype=np.float64)
    _check(_load().orc_vis_single(_ptr(packed), S, N, K, a, b, k, _ptr(out)), "orc_vis_single")
    return complex(out[0], out[1])


def ingest(frames: np.ndarray, n_frames: int, stride: int, first_seq: int, S: int, N: int, K: int,
           W: int = 1024):
    """Frames (uint8, n_frames x stride) -> (packed uint8 [S][N][K], stats
    dict, blocks received in the first min(S, W))."""
    frames = np.ascontiguousarray(frames, dtype=np.uint8)
    out = np.empty((S, N, K), dtype=np.uint8)
    st = np.zeros(4, dtype=np.int64)
    wv = np.zeros(1, dtype=np.int64)
    _check(_load().orc_ingest(_ptr(frames), n_frames, stride, first_seq, S, N, K, min(S, W), _ptr(out),
                              _ptr(st), _ptr(wv)), "orc_ingest")
    stats = dict(frames_accepted=int(st[0]), frames_rejected=int(st[1]), frames_duplicate=int(st[2]),
                 spectra_lost=int(st[3]))
    return out, stats, int(wv[0])


# Largest code and the multiple of the rms it stands for, per requantised form
FULL_SCALE = {"int8": (127.0, 4.0), "int16": (32512.0, 8.0)}


def scales_n(spec: np.ndarray, W: int, n_div: int, form: str = "int8") -> np.ndarray:
    """Scales of `form` ("int8" or "int16") over the first W spectra with the
    mean power taken over n_div spectra."""
    S, N, K = spec.shape
    qmax, clip = FULL_SCALE[form]
    pairs = _spec_pairs(spec)
    out = np.empty((N, K), dtype=np.float32)
    _check(_load().orc_scales_n(_ptr(pairs), S, N, K, W, n_div, qmax, clip, _ptr(out)), "orc_scales_n")
    return out


def quantise16(spec: np.ndarray, sc: np.ndarray) -> np.ndarray:
    """complex spectra [S][N][K] + scales [N][K] -> int16 [S][N][K][2]."""
    S, N, K = spec.shape
    pairs = _spec_pairs(spec)
    sc = np.ascontiguousarray(sc, dtype=np.float32)
    assert sc.shape == (N, K)
    q = np.empty((S, N, K, 2), dtype=np.int16)
    _check(_load().orc_quantise16(_ptr(pairs), S, N, K, _ptr(sc), _ptr(q)), "orc_quantise16")
    return q


def cmac_i64_16(q: np.ndarray, full: bool = False) -> np.ndarray:
    """int16 [S][N][K][2] -> exact int64 visibilities [rows][K][2]."""
    q = np.ascontiguousarray(q, dtype=np.int16)
    S, N, K, two = q.shape
    assert two == 2
    rows = N * N if full else n_baselines(N)
    vis = np.empty((rows, K, 2), dtype=np.int64)
    _check(_load().orc_cmac_i64_16(_ptr(q), S, N, K, int(full), _ptr(vis)), "orc_cmac_i64_16")
    return vis.reshape(N, N, K, 2) if full else vis


def track(spec: np.ndarray, delay=None, delay_rate=None, phase=None, phase_rate=None, s0: int = 0) -> np.ndarray:
    """Spectra [S][N][K] rotated by the per-antenna delay / phase model (a new
    array); spectrum s is spectrum s0 + s of the integration."""
    S, N, K = spec.shape
    pairs = _spec_pairs(spec)
    arrs = [None if v is None else np.ascontiguousarray(v, dtype=np.float64).ravel()
            for v in (delay, delay_rate, phase, phase_rate)]
    for v in arrs:
        assert v is None or v.size == N
    ptrs = [None if v is None else _ptr(v) for v in arrs]
    _check(_load().orc_track(_ptr(pairs), S, N, K, s0, *ptrs), "orc_track")
    return pairs[..., 0] + 1j * pairs[..., 1]


def correlate(packed: np.ndarray, S: int, N: int, K: int) -> np.ndarray:
    """Whole float64 path: packed [S][N][K] -> visibilities complex128 [nb][K]."""
    return cmac_f64(spectra(packed, S, N, K))


def set_threads(n: int) -> None:
    """Number of OpenMP threads the oracle's loops use (timing only)."""
    _check(_load().orc_set_threads(int(n)), "orc_set_threads")


def get_threads() -> int:
    return int(_load().orc_get_threads())
