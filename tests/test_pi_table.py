"""The versioned parameter table written by the autotuner: the library's
reader and the oracle's own reader must give the same parameters, which
the oracle's range check accepts, and the recorded choice must be the
fastest recorded candidate (no GPU needed)."""
import json
import os

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TABLE = os.path.join(ROOT, "paper_2302_03317_amd", "pi_table.json")


def _table():
    with open(TABLE) as fh:
        return json.load(fh)


def test_table_is_versioned_and_complete():
    t = _table()
    assert t["format"] == "ipscshuf parameter table"
    assert isinstance(t["version"], int) and t["version"] >= 1
    assert t["entries"], "no entries"
    for e in t["entries"]:
        for k in ("workload", "form", "elem_bytes", "params", "median_ms", "candidates", "definition_version"):
            assert k in e, k


def test_library_and_oracle_read_the_same_parameters():
    from paper_2302_03317_amd import autotune

    t = autotune.load_table(TABLE)
    for e in t["entries"]:
        p_lib, v_lib = autotune.lookup(t, e["workload"], e["elem_bytes"])
        p_or, v_or = oracle.params_from_table(TABLE, e["workload"], e["elem_bytes"])
        assert v_lib == v_or == t["version"]
        assert (p_lib.tile, p_lib.kmax_log2, p_lib.n0, p_lib.lmax) == (p_or.tile, p_or.kmax_log2, p_or.n0, p_or.lmax)
        assert oracle.check_params(p_or)


def test_recorded_choice_is_the_fastest_candidate():
    for e in _table()["entries"]:
        ok = [c for c in e["candidates"] if c.get("error_word") == 0 and "median_ms" in c]
        best = min(ok, key=lambda c: c["median_ms"])
        assert best["params"] == e["params"]
        assert e["median_ms"] == best["median_ms"]
        # every candidate lies within the definition's ranges and admits the
        # workload's largest array in one tiled level
        for c in e["candidates"]:
            q = c["params"]
            assert oracle.check_params(oracle.Params(q["tile"], q["kmax_log2"], q["n0"], q["lmax"]))
            assert (q["tile"] // 2) << q["kmax_log2"] >= e["largest_array"]


def test_definition_version_matches_the_library():
    from paper_2302_03317_amd import definition_version

    for e in _table()["entries"]:
        assert e["definition_version"] == definition_version()


def test_oracle_refuses_out_of_range_parameters(tmp_path):
    t = _table()
    e = dict(t["entries"][0])
    e["params"] = dict(e["params"], kmax_log2=9)  # above the definition's k <= 256
    t["entries"] = [e]
    p = tmp_path / "bad.json"
    p.write_text(json.dumps(t))
    with pytest.raises(ValueError):
        oracle.params_from_table(str(p), e["workload"], e["elem_bytes"])
    with pytest.raises(KeyError):
        oracle.params_from_table(str(p), "no_such_workload", 4)
