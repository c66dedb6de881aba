"""The autotuner's candidate space and table lookup (CPU)."""
import json

from paper_1102_0148_amd import tune


def test_candidates_respect_limits():
    for (N, K, S, prec) in [(44, 256, 65536, "fp32"), (44, 256, 65536, "int8"), (32, 1024, 16384, "fp16"),
                            (256, 512, 16384, "fp32"), (8, 128, 3, "int8"), (44, 256, 65536, "int16")]:
        c = tune.candidates(N, K, S, prec)
        assert c, (N, K, S, prec)
        for t in c:
            assert t["chunk_spectra"] % 64 == 0 and t["chunk_spectra"] <= (S + 63) // 64 * 64
            assert tune.f_lds_bytes(K, prec, t["f_group"]) <= tune.LDS_LIMIT
            assert 1 <= t["x_splits"] <= 64
            if tune.PARTIAL_LIMIT[prec]:
                assert t["chunk_spectra"] / t["x_splits"] <= tune.PARTIAL_LIMIT[prec]


def test_table_lookup(tmp_path):
    p = tmp_path / "t.json"
    p.write_text(json.dumps({tune.key(44, 256, 100, "fp32"): {"chunk_spectra": 128, "x_splits": 4, "f_group": 8},
                             tune.key(8, 128, 100, "int8", True): {"x_splits": 2}}))
    assert tune.lookup(44, 256, 100, "fp32", path=str(p))["x_splits"] == 4
    assert tune.lookup(8, 128, 100, "int8", batch=True, path=str(p)) == {"x_splits": 2}
    assert tune.lookup(8, 128, 100, "int8", path=str(p)) is None
