"""The benchmark's op-count and rate conventions against the figures the paper
prints (tests/golden/paper_load_figures.json, each entry cited there)."""
import json
import os

from paper_1102_0148_amd import metrics

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_load_figures.json")


def test_paper_load_figures():
    g = json.load(open(GOLDEN))
    s1 = g["section_1"]
    N, two_k, R = s1["N"], s1["fft_points"], s1["R_msps"]
    # F-stage: 2.5 * 2K log2 2K flops per transform reproduces 0.99R exactly
    assert round(metrics.paper_fft_gflops_per_msps(N, two_k), 2) == s1["fft_gflops_per_msps"]
    # the paper's X figure reads as N^2 flops per sample period
    assert round(metrics.paper_x_gflops_per_msps(N), 2) == s1["xmac_gflops_per_msps"]
    total = (s1["fft_gflops_per_msps"] + s1["xmac_gflops_per_msps"]) * R
    assert total > s1["total_gflops_over"]
    assert metrics.input_mbytes_per_s(N, R, s1["bits_per_sample"]) == s1["input_mbytes_per_s"]
    # our X convention (8 ops per CMAC over baselines with autos) is ~2x the paper's
    assert abs(metrics.x_gops_per_msps(N) / metrics.paper_x_gflops_per_msps(N) - 2.0) < 0.05
    # "about 1000 baselines" matches N(N+1)/2 with autos
    assert abs(metrics.n_baselines(N) - g["section_3_3"]["baselines_approx"]) < 20


def test_abstract_rate_in_antenna_samples():
    g = json.load(open(GOLDEN))
    mb = g["abstract"]["input_mbytes_per_s"]
    # 4-bit samples: 2 antenna-samples per byte
    assert mb * 2 == 1470
    assert metrics.antenna_msps(44, 512, 1, 1.0) == 44 * 512 / 1e6


def test_x_mfma_ops_block_pairs():
    """N = 44 pads to 3 blocks of 16: 6 block pairs of 256 entries. The
    totals match the per-dispatch MFMA counters of the committed profile
    (fp32 1.55e11, int8 2.06e11, int16 8.25e11 per 65536-spectrum
    integration)."""
    from paper_1102_0148_amd import metrics
    assert metrics.padded_antennas(44) == 48
    assert metrics.padded_antennas(256) == 256 and metrics.padded_antennas(100) == 128
    base = 256 * 6 * 256 * 65536
    assert metrics.x_mfma_ops(44, 256, 65536, "fp32") == 6 * base
    assert metrics.x_mfma_ops(44, 256, 65536, "int8") == 8 * base
    assert metrics.x_mfma_ops(44, 256, 65536, "int16") == 32 * base
    assert abs(metrics.x_mfma_ops(44, 256, 65536, "fp32") - 1.5466e11) / 1.5466e11 < 1e-3
    assert abs(metrics.x_mfma_ops(44, 256, 65536, "int16") - 8.246e11) / 8.246e11 < 1e-3
