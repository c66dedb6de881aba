"""Op counts and rates the benchmark reports (no correlator arithmetic).

Conventions:
  * F-stage flops per 2K-point real transform: 2.5 * 2K * log2(2K), the usual
    radix-2 count; for N = 44 and 2K = 512 it gives the paper's 0.99R Gflops
    (Section 1) exactly.
  * X-stage ops: 8 real operations per complex multiply-accumulate, over the
    N(N+1)/2 baselines including autos, per channel per spectrum (the useful
    triangle only; padding and the lower triangle are not counted).
  * antenna-MS/s: antenna-samples processed per second / 1e6 = N * S * 2K / t.
The paper's own X count (1.94R Gflops for N = 44) is about N^2 R flops, half of
this convention's 4 * N(N+1)/2 * R; both are printed beside results.
"""
import math


def n_baselines(N: int) -> int:
    return N * (N + 1) // 2


def fft_flops(two_k: int) -> float:
    return 2.5 * two_k * math.log2(two_k)


def f_flops(N: int, two_k: int, S: int) -> float:
    return fft_flops(two_k) * N * S


def x_ops(N: int, K: int, S: int) -> float:
    return 8.0 * n_baselines(N) * K * S


def antenna_samples(N: int, two_k: int, S: int) -> float:
    return float(N) * two_k * S


def antenna_msps(N: int, two_k: int, S: int, seconds: float) -> float:
    return antenna_samples(N, two_k, S) / seconds / 1e6


def paper_fft_gflops_per_msps(N: int, two_k: int) -> float:
    """F-stage Gflops needed per MS/s of sampling rate (Section 1's 0.99R)."""
    return fft_flops(two_k) * N / two_k / 1e3


def x_gops_per_msps(N: int) -> float:
    """This convention's X-stage Gops per MS/s: 8 nb K ops per 2K samples."""
    return 4.0 * n_baselines(N) / 1e3


def paper_x_gflops_per_msps(N: int) -> float:
    """The paper's X-stage figure read as N^2 flops per sample period."""
    return N * N / 1e3


def input_mbytes_per_s(N: int, R_msps: float, bits: int = 4) -> float:
    return N * R_msps * bits / 8.0
