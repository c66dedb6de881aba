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


# MFMA operations the X-stage issues per entry of a 16 x 16 antenna block pair
# per spectrum: fp32 forms three real products (re.re, im.im and
# (re+im).(re+im)), two operations each; fp16 and int8 form two real products
# over [re | im] operands of twice the length; int16 forms the int8 form's
# products for four pairs of base-255 digits.
MFMA_OPS_PER_ENTRY = {"fp32": 6, "fp16": 8, "int8": 8, "int16": 32}
# Dense MFMA peaks of MI355X per form (int16 runs on the int8 MFMA), in
# TFLOP/s or TOPS.
MFMA_PEAK = {"fp32": 157.3, "fp16": 2500.0, "int8": 5000.0, "int16": 5000.0}


def padded_antennas(N: int) -> int:
    """Antennas the X-stage computes over: whole 16-antenna blocks up to 96
    antennas, whole 64-antenna region rows beyond."""
    return 16 * ((N + 15) // 16) if N <= 96 else (N + 63) // 64 * 64


def x_mfma_ops(N: int, K: int, S: int, prec: str) -> float:
    """Operations the X-stage's MFMA instructions issue for S spectra: the
    regions tile the triangle of block pairs of the padded antennas, so every
    block pair is computed once (diagonal blocks in full)."""
    nblk = padded_antennas(N) // 16
    return float(MFMA_OPS_PER_ENTRY[prec]) * 256 * (nblk * (nblk + 1) // 2) * K * S


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
