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


def test_pick_prefers_simpler_tiling_within_tie():
    a = {"chunk_spectra": 65536, "x_splits": 32, "f_group": 2}
    b = {"chunk_spectra": 65536, "x_splits": 8, "f_group": 2}
    c = {"chunk_spectra": 32768, "x_splits": 4, "f_group": 2}
    # b is within 1% of the fastest (a) and has fewer splits; c is within 1%
    # but takes two chunks
    assert tune.pick([(a, 1.5770), (b, 1.5783), (c, 1.5790)])[0] is b
    # outside the tie margin the fastest wins
    assert tune.pick([(a, 1.50), (b, 1.60)])[0] is a
    # among equal chunk and splits, the faster one
    assert tune.pick([(b, 1.60), (dict(b, f_group=4), 1.59)])[1] == 1.59


def test_keys_per_batch_mode():
    assert tune.key(8, 128, 100, "int8") == "gfx950:N=8:K=128:S=100:int8"
    assert tune.key(8, 128, 100, "int8", batch=True) == "gfx950:N=8:K=128:S=100:int8:batch"
    assert tune.key(8, 128, 100, "int8", batch="persistent") == "gfx950:N=8:K=128:S=100:int8:batch"
    assert tune.key(8, 128, 100, "int8", batch="branches") == "gfx950:N=8:K=128:S=100:int8:branches"



def test_fused_candidates_one_layout_each():
    """Every fused candidate names one role layout (the library refuses both
    at once), chunks stay within the integration, and shapes the fused
    kernel does not cover get none."""
    c = tune.fused_candidates(44, 256, 65536, "fp32")
    assert c and all((x["f_workgroups_per_cu"] == 0) or (x["f_cus_per_xcd"] == 0) for x in c)
    assert {x["f_cus_per_xcd"] for x in c} == {0, 12, 16, 20, 24}
    assert all(64 <= x["chunk_spectra"] <= 65536 and x["chunk_spectra"] % 64 == 0 for x in c)
    assert tune.fused_candidates(44, 256, 1000, "int8")[0]["chunk_spectra"] <= 1024
    assert tune.fused_candidates(44, 256, 65536, "int16") == []
    assert tune.fused_candidates(64, 256, 65536, "fp32") == []


def test_final_candidates_keep_the_incumbent():
    """The last stage times the best pairs with the chosen F group and the
    table's present entry, once, whatever else the entry holds."""
    top = [{"chunk_spectra": 65536, "x_splits": 4, "f_group": 8}, {"chunk_spectra": 32768, "x_splits": 8, "f_group": 8}]
    inc = {"chunk_spectra": 65536, "x_splits": 4, "f_group": 2, "ms": 1.3, "pipeline": "staged"}
    out = tune.final_candidates(top, 2, inc)
    assert out == [{"chunk_spectra": 65536, "x_splits": 4, "f_group": 2},
                   {"chunk_spectra": 32768, "x_splits": 8, "f_group": 2}]
    inc2 = dict(inc, x_splits=16)
    assert tune.final_candidates(top, 2, inc2)[-1] == {"chunk_spectra": 65536, "x_splits": 16, "f_group": 2}
    assert len(tune.final_candidates(top, 2, None)) == 2
    # a batch or fused entry (no tile triple) is not a staged candidate
    assert len(tune.final_candidates(top, 2, {"x_splits": 4, "ms": 1.0})) == 2
