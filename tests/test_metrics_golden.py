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
