"""Seeded synthetic antenna streams for the FX correlator.

This module only draws and packs input samples: it holds none of the
correlator's arithmetic (no transform, no cross-multiplication, no
quantisation of spectra).  It is the one piece shared by the CPU oracle's
tests, the GPU parity tests and the benchmark, so that both sides see the same
bytes.

Recipe (stands in for the live digitiser data of the paper, which is not
public): every antenna carries its own white Gaussian noise, plus optional
common components shared by all antennas, scaled by ``sigma`` and rounded to
signed 4-bit integers -8..7 (Section 1: 4-bit quantisation of each element's
stream).  Two samples are packed per byte, the earlier (even) sample in the
low nibble, and a frame is laid out [spectrum][antenna][2K samples] (Section
2.2: one packet carries contiguous samples of all elements and is one FFT
block).

  x_a[n] = clamp(rint(sigma * (sqrt(1 - sum rho) * g_a[n]
                               + sum_s sqrt(rho_s) * c_s[n - d_{s,a}])
                      + A cos(2 pi k0 n / 2K + phi)), -8, 7)

The random numbers come from torch generators seeded per (seed, stream,
chunk), so any range of spectra can be regenerated on its own, on the CPU or
on a GPU (the two devices give different, individually reproducible draws).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import torch

# spectra per generator chunk; a stream is drawn chunk by chunk so any range
# can be regenerated without drawing what precedes it
CHUNK_SPECTRA = 1024


@dataclass
class Source:
    """A common white signal seen by every antenna with an integer delay
    d_a = rint(delay_per_antenna * a) samples and power fraction rho."""
    rho: float
    delay_per_antenna: float = 0.0


@dataclass
class Recipe:
    N: int
    two_k: int
    sigma: float = 2.5
    sources: List[Source] = field(default_factory=list)
    tone_bin: Optional[int] = None
    tone_amp: float = 0.0          # in units of sigma
    tone_phase: float = 0.3
    seed: int = 0

    @property
    def K(self) -> int:
        return self.two_k // 2


def _gen(seed: int, stream: int, chunk: int, device) -> torch.Generator:
    g = torch.Generator(device=device)
    # a fixed mixing of the three integers into one 63-bit seed
    h = (seed * 0x9E3779B97F4A7C15 + stream * 0xBF58476D1CE4E5B9 + chunk * 0x94D049BB133111EB)
    g.manual_seed(h & 0x7FFFFFFFFFFFFFFF)
    return g


def _noise(seed: int, stream: int, n0: int, n1: int, chunk_len: int, device) -> torch.Tensor:
    """Samples [n0, n1) of white N(0,1) stream `stream` (n0 may be negative)."""
    out = []
    c0 = math.floor(n0 / chunk_len)
    c1 = math.floor((n1 - 1) / chunk_len)
    for c in range(c0, c1 + 1):
        g = _gen(seed, stream, c, device)
        blk = torch.randn(chunk_len, generator=g, device=device, dtype=torch.float32)
        lo = max(n0, c * chunk_len) - c * chunk_len
        hi = min(n1, (c + 1) * chunk_len) - c * chunk_len
        out.append(blk[lo:hi])
    return torch.cat(out)


def samples(recipe: Recipe, s0: int, s1: int, device="cpu") -> torch.Tensor:
    """Signed 4-bit samples of spectra [s0, s1): int8 tensor [s1-s0][N][2K]."""
    N, two_k = recipe.N, recipe.two_k
    chunk_len = CHUNK_SPECTRA * two_k
    n0, n1 = s0 * two_k, s1 * two_k
    rho_tot = sum(src.rho for src in recipe.sources)
    assert 0.0 <= rho_tot < 1.0
    own = math.sqrt(1.0 - rho_tot)
    t = torch.arange(n0, n1, device=device, dtype=torch.float64)
    tone = None
    if recipe.tone_bin is not None and recipe.tone_amp != 0.0:
        ang = 2.0 * math.pi * recipe.tone_bin * torch.remainder(t, two_k) / two_k + recipe.tone_phase
        tone = (recipe.tone_amp * recipe.sigma * torch.cos(ang)).to(torch.float32)
    common = []
    for j, src in enumerate(recipe.sources):
        dmax = int(round(abs(src.delay_per_antenna) * (N - 1)))
        c = _noise(recipe.seed, 1_000_000 + j, n0 - dmax, n1 + dmax, chunk_len, device)
        common.append((src, dmax, c))
    out = torch.empty((s1 - s0, N, two_k), dtype=torch.int8, device=device)
    for a in range(N):
        v = own * _noise(recipe.seed, a, n0, n1, chunk_len, device)
        for src, dmax, c in common:
            d = int(round(src.delay_per_antenna * a))
            # c holds samples [n0 - dmax, n1 + dmax); we want c[n - d]
            lo = dmax - d
            v = v + math.sqrt(src.rho) * c[lo:lo + (n1 - n0)]
        v = recipe.sigma * v
        if tone is not None:
            v = v + tone
        x = torch.clamp(torch.round(v), -8, 7).to(torch.int8)
        out[:, a, :] = x.view(s1 - s0, two_k)
    return out


def pack(x: torch.Tensor) -> torch.Tensor:
    """int8 samples [..., 2K] in -8..7 -> uint8 [..., K], low nibble = even."""
    lo = x[..., 0::2].to(torch.int16) & 0xF
    hi = x[..., 1::2].to(torch.int16) & 0xF
    return (lo | (hi << 4)).to(torch.uint8)


def packed(recipe: Recipe, s0: int, s1: int, device="cpu") -> torch.Tensor:
    """Packed frames of spectra [s0, s1): uint8 [s1-s0][N][K]."""
    return pack(samples(recipe, s0, s1, device))


# The workloads, each with the shape and statistics of the paper's 44-element,
# 512-point, 4-bit case or of the larger cases built around it.

def recipe_plain(N: int = 44, two_k: int = 512, rho: float = 0.05, seed: int = 0) -> Recipe:
    """Per-antenna noise sigma=2.5 plus one common component of power rho."""
    return Recipe(N=N, two_k=two_k, sources=[Source(rho=rho)], seed=seed)


def recipe_tone(N: int = 44, two_k: int = 512, rho: float = 0.05, seed: int = 2,
                tone_bin: int = 77, tone_amp: float = 0.5) -> Recipe:
    """As recipe_plain plus a common tone at an integer bin (amplitude in sigma)."""
    return Recipe(N=N, two_k=two_k, sources=[Source(rho=rho)], tone_bin=tone_bin,
                  tone_amp=tone_amp, seed=seed)


def recipe_sources(N: int = 256, two_k: int = 1024, seed: int = 4,
                   rhos: Sequence[float] = (0.03, 0.02, 0.01),
                   delays: Sequence[float] = (0.0, 0.25, 0.75)) -> Recipe:
    """Three common white point sources with per-antenna integer delays."""
    return Recipe(N=N, two_k=two_k, seed=seed,
                  sources=[Source(rho=r, delay_per_antenna=d) for r, d in zip(rhos, delays)])


# The uneven batch: (N, FFT size) pairs a job is drawn from.
BATCH_SHAPES: Tuple[Tuple[int, int], ...] = (
    (8, 256), (12, 512), (16, 1024), (24, 512), (32, 2048), (44, 512), (64, 1024), (96, 512))


def batch_jobs(n_jobs: int = 12, seed: int = 3) -> List[Recipe]:
    """n_jobs recipes with (N, 2K) drawn with replacement and rho ~ U[0, 0.1]."""
    g = torch.Generator().manual_seed(seed)
    idx = torch.randint(len(BATCH_SHAPES), (n_jobs,), generator=g).tolist()
    rhos = (torch.rand(n_jobs, generator=g, dtype=torch.float64) * 0.1).tolist()
    jobs = []
    for j, (i, r) in enumerate(zip(idx, rhos)):
        N, two_k = BATCH_SHAPES[i]
        jobs.append(Recipe(N=N, two_k=two_k, sources=[Source(rho=r)], seed=seed * 1000 + j))
    return jobs


# Frames: the packet form of the input (Section 2.2: each packet is one FFT
# block of every element, with a header giving its sample timing, datatype and
# element count).  The header layout is the library's interface: 32 bytes,
# little-endian, magic "OFRM", version 1, datatype 1 (4-bit), block number,
# elements, samples per element, 8 reserved bytes.
FRAME_MAGIC = 0x4D52464F
FRAME_HEADER_BYTES = 32


def frames(packed, seqs, blocks=None, stride: Optional[int] = None, two_k: Optional[int] = None,
           magic: int = FRAME_MAGIC, version: int = 1, datatype: int = 1, n_elements: Optional[int] = None):
    """Frames carrying packed blocks: packed uint8 [S][N][K]; frame i holds
    block blocks[i] (default i) and says it is block seqs[i].  Header fields
    can be given per frame (sequences) or for all frames, so tests can build
    corrupt headers.  Returns uint8 [n_frames][stride] (CPU)."""
    import numpy as np
    p = packed.cpu().numpy() if hasattr(packed, "cpu") else np.asarray(packed)
    S, N, K = p.shape
    n = len(seqs)
    blocks = list(range(n)) if blocks is None else list(blocks)
    payload = N * K
    stride = stride or (FRAME_HEADER_BYTES + payload + 15) // 16 * 16
    out = np.zeros((n, stride), dtype=np.uint8)

    def per(v, i):
        return v[i] if isinstance(v, (list, tuple, np.ndarray)) else v

    for i in range(n):
        hdr = np.zeros(FRAME_HEADER_BYTES, dtype=np.uint8)
        hdr[0:4] = np.frombuffer(np.uint32(per(magic, i)).tobytes(), dtype=np.uint8)
        hdr[4:6] = np.frombuffer(np.uint16(per(version, i)).tobytes(), dtype=np.uint8)
        hdr[6:8] = np.frombuffer(np.uint16(per(datatype, i)).tobytes(), dtype=np.uint8)
        hdr[8:16] = np.frombuffer(np.uint64(seqs[i]).tobytes(), dtype=np.uint8)
        ne = N if n_elements is None else per(n_elements, i)
        hdr[16:20] = np.frombuffer(np.uint32(ne).tobytes(), dtype=np.uint8)
        hdr[20:24] = np.frombuffer(np.uint32(2 * K if two_k is None else per(two_k, i)).tobytes(), dtype=np.uint8)
        out[i, :FRAME_HEADER_BYTES] = hdr
        out[i, FRAME_HEADER_BYTES:FRAME_HEADER_BYTES + payload] = p[blocks[i]].reshape(-1)
    return torch.from_numpy(out)
