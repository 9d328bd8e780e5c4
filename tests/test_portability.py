"""The portability analysis on synthetic timing tables (no GPU): fractions of
the optimum, histograms, the cross-scenario matrix with the default-config
fallback, and Pennycook's metric (harmonic mean, 0 when unsupported)."""
import math

import pytest

from paper_2303_12374_amd import portability as P


def table():
    # two scenarios of one kernel; "b" cannot run in s2 (None), "c" is best in s2
    return {
        "k-8x8x8-f32": {"kernel": "k", "shape": [8, 8, 8], "dtype": "f32",
                        "times": {"default": 2.0, "a": 1.0, "b": 1.25, "c": 4.0}},
        "k-16x16x16-f32": {"kernel": "k", "shape": [16, 16, 16], "dtype": "f32",
                           "times": {"default": 3.0, "a": 6.0, "b": None, "c": 1.5}},
    }


def test_fractions_and_optimum():
    fr = P.fractions({"default": 2.0, "a": 1.0, "b": None, "c": 4.0})
    assert fr == {"default": 0.5, "a": 1.0, "c": 0.25}
    assert P.optimum({"default": 2.0, "a": 1.0, "c": 1.0}) == "a"  # ties: by name


def test_histogram_counts_every_configuration():
    fr = {"a": 1.0, "b": 0.95, "c": 0.5, "d": 0.05, "e": 0.0999}
    h = P.histogram(fr)
    assert sum(h) == len(fr)
    assert h[9] == 2 and h[5] == 1 and h[0] == 2


def test_efficiency_falls_back_to_default():
    t = table()["k-16x16x16-f32"]["times"]
    assert P.efficiency(t, "c") == 1.0
    assert P.efficiency(t, "b") == pytest.approx(1.5 / 3.0)   # not runnable: the default runs
    assert P.efficiency({"x": None}, "x") == 0.0


@pytest.mark.parametrize("effs,expect", [([0.5, 0.5, 0.5], 0.5), ([1.0, 0.5], 2 / 3), ([1.0, 0.0], 0.0),
                                         ([0.9, 0.6, 0.3], 3 / (1 / 0.9 + 1 / 0.6 + 1 / 0.3))])
def test_ppm_is_the_harmonic_mean(effs, expect):
    assert P.ppm(effs) == pytest.approx(expect)
    if min(effs) > 0:  # a harmonic mean lies between the extremes, below the arithmetic mean
        assert min(effs) <= P.ppm(effs) <= sum(effs) / len(effs) + 1e-15


def test_analysis_matrix_and_ppm_rows():
    rep = P.analyze(table())
    m = rep["matrix"]["k"]
    s1, s2 = "k-8x8x8-f32", "k-16x16x16-f32"
    assert m[s1][s1] == 1.0 and m[s2][s2] == 1.0        # each optimum on its own scenario
    assert m[s1][s2] == pytest.approx(1.5 / 6.0)          # "a" (best in s1) in s2
    assert m[s2][s1] == pytest.approx(1.0 / 4.0)          # "c" (best in s2) in s1
    rows = rep["ppm"]["k"]
    assert rows["runtime selection"]["ppm"] == 1.0
    assert rows["(default configuration)"]["best"] == pytest.approx(0.5)
    assert rows[s1]["ppm"] == pytest.approx(P.ppm([1.0, 0.25]))
    sc = rep["scenarios"][s1]
    assert sc["optimum"] == "a" and sc["config_C"] == "a" and sc["within_10pct"] == pytest.approx(0.25)
    assert rep["scenarios"][s2]["config_C_fraction"] == pytest.approx(0.25)
    md = P.report_markdown(rep, {"device": "test", "command": "x"})
    assert "PPM: k" in md and "runtime selection" in md and not math.isnan(rows[s2]["ppm"])


def test_merged_collections_keep_every_scenario_and_command(tmp_path):
    t = table()
    k1, k2 = list(t)
    a = {"meta": {"device": "gpu", "command": "run f32"}, "data": {k1: t[k1]}}
    b = {"meta": {"device": "gpu", "command": "run f64"}, "data": {k2: t[k2]}}
    data, meta = P.merge_collections([a, b])
    assert set(data) == {k1, k2} and meta["command"] == "run f32 ; run f64"
    with pytest.raises(SystemExit):
        P.merge_collections([a, {"meta": {"device": "other"}, "data": {}}])
    import json
    pa, pb = tmp_path / "a.json", tmp_path / "b.json"
    pa.write_text(json.dumps(a)), pb.write_text(json.dumps(b))
    assert P.main(["--out", str(tmp_path / "m"), "--from-json", f"{pa},{pb}"]) == 0
    assert "run f32 ; run f64" in (tmp_path / "m.md").read_text()
