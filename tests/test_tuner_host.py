"""Host logic of the autotuner and the learned tuner (no GPU): seeded training specs,
dataset arrays, regret and fallback arithmetic, model files."""
import json

import numpy as np

from paper_1112_5588_amd import _lib as L
from paper_1112_5588_amd import autotune, tuner


def test_catalog_default_is_the_papers_format():
    c = autotune.CATALOG[autotune.DEFAULT]
    assert c.fmt == "pjds" and c.block_height == 64 and c.layout == "jd" and c.sort_window == 0
    assert len(set(autotune.CONFIG_NAMES)) == len(autotune.CATALOG)
    keys = {c.storage_key() for c in autotune.CATALOG}
    assert len(keys) <= 16          # conversions per matrix in a sweep


def test_training_specs_are_seeded_and_cover_the_range():
    a = [tuner.matrix_spec(s) for s in range(100000, 100300)]
    b = [tuner.matrix_spec(s) for s in range(100000, 100300)]
    assert a == b
    ns = [s["n"] for s in a]
    assert 10_000 <= min(ns) and max(ns) <= 8_000_000
    assert {s["family"] for s in a} == set(tuner.FAMILIES)
    assert tuner.matrix_spec(200000) != tuner.matrix_spec(100000)


def toy_records():
    names = autotune.CONFIG_NAMES
    recs = []
    for i in range(6):
        t = {n: 1.0 + 0.1 * k + 0.01 * i for k, n in enumerate(names)}
        t[names[3]] = 0.5                      # configuration 3 is always fastest
        if i == 2:
            t["ellr"] = None                   # not built for this matrix
        recs.append({"key": str(100000 + i), "nnz": 1000 * (i + 1), "features": list(np.arange(24) + i),
                     "times_ms": t, "times_rev": autotune.TIMES_REV})
    return recs


def test_arrays_mask_missing_timings():
    X, y, t = tuner.arrays(toy_records())
    assert X.shape == (6, 24) and y.shape == (6, len(autotune.CATALOG))
    e = autotune.CONFIG_NAMES.index("ellr")
    assert np.isnan(t[2, e]) and np.isnan(y[2, e]) and np.isfinite(y[0, e])
    assert np.isclose(y[0, 3], np.log(0.5 / 1001))


def test_regret_and_fallback_arithmetic():
    X, _, t = tuner.arrays(toy_records())
    m = tuner.Model(np.zeros(L.mlp_param_count(24, len(autotune.CATALOG)), np.float32), X.mean(0), X.std(0) + 1,
                    np.zeros(len(autotune.CATALOG)), np.ones(len(autotune.CATALOG)))
    perfect = np.full(6, 3)
    r = tuner.evaluate(perfect, np.ones(6), X, t, m)
    assert r["regret"]["max"] == 0.0 and r["exact_pick_rate"] == 1.0 and r["fallback_rate"] == 0.0
    assert np.isclose(r["geomean_gain_over_default"], np.exp(np.mean(np.log(t[:, 0] / 0.5))))
    # picking the default costs exactly the default/best ratio; a tiny margin triggers the fallback
    r = tuner.evaluate(np.zeros(6, int), np.array([1, 1, 1, 0.0, 0.0, 1]), X, t, m)
    assert np.isclose(r["regret"]["max"], (t[:, 0] / 0.5 - 1).max())
    assert r["fallback_rate"] == 2 / 6
    assert np.isclose(r["regret_with_fallback"]["max"], max(t[i, 0] / 0.5 - 1 for i in (0, 1, 2, 5)))


def test_model_roundtrip(tmp_path):
    n = L.mlp_param_count(24, len(autotune.CATALOG))
    p = tuner.init_params(3)
    assert p.size == n and np.all(p[24 * 64:24 * 64 + 64] == 0)     # b1 starts at zero
    m = tuner.Model(p, np.zeros(24), np.ones(24), np.zeros(len(autotune.CATALOG)), np.ones(len(autotune.CATALOG)), {"x": 1})
    path = tmp_path / "m.json"
    m.save(str(path))
    m2 = tuner.Model.load(str(path))
    assert np.array_equal(m2.params, m.params) and m2.meta == {"x": 1}
    d = json.load(open(path))
    d["configs"] = d["configs"][:-1]
    json.dump(d, open(path, "w"))
    try:
        tuner.Model.load(str(path))
        raise AssertionError("catalog mismatch not detected")
    except ValueError:
        pass


def test_ellr_fit_from_features():
    X = np.zeros((2, 24))
    X[0, 13] = 1.0          # ELLPACK-R stores 2 x nnz
    X[1, 13] = 12.0         # 4096 x nnz
    ok = tuner.ellr_fits(X, np.array([1e6, 1e6]))
    assert ok.tolist() == [True, False]


def test_store_update_merges_and_compacts(tmp_path):
    from paper_1112_5588_amd import tuner
    p = str(tmp_path / "s.jsonl")
    st = autotune.ResultStore(p)
    st.add({"key": "1", "device": "d", "nnz": 5, "features": [0.0] * 24, "times_ms": {"a": 1.0}})
    st.add({"key": "2", "device": "d", "nnz": 5, "features": [0.0] * 24, "times_ms": {"a": 2.0}})
    rec = dict(st.records[("1", "d")])
    rec["times_ms"] = {**rec["times_ms"], "b": 3.0}
    st.add(rec)
    recs = tuner.load_records(p)
    assert [r["key"] for r in recs] == ["1", "2"] and recs[0]["times_ms"] == {"a": 1.0, "b": 3.0}
    assert len(open(p).read().splitlines()) == 3
    st.rewrite()
    assert len(open(p).read().splitlines()) == 2
    assert tuner.load_records(p) == recs


def test_records_timed_before_the_current_timing_are_masked():
    recs = toy_records()
    recs[1]["times_rev"] = autotune.TIMES_REV - 1       # an older sweep: none of its times count
    del recs[4]["times_rev"]
    _, y, t = tuner.arrays(recs)
    assert np.all(np.isnan(t[[1, 4]])) and np.all(np.isnan(y[[1, 4]]))
    assert np.isfinite(t[0]).all() and np.isfinite(t[5]).all()


def test_decision_rule_arithmetic():
    """The learned tuner's rule: the network's pick when it leads clearly, the fastest timed of
    its top k on a near tie, the exhaustive search far outside the training range."""
    X, _, t = tuner.arrays(toy_records())
    C = len(autotune.CATALOG)
    m = tuner.Model(np.zeros(L.mlp_param_count(24, C), np.float32), X.mean(0), X.std(0) + 1, np.zeros(C), np.ones(C))
    runnable = np.isfinite(t)
    best = np.where(runnable, t, np.inf).min(axis=1)
    # scores that rank the default first with a clear lead, config 3 (the fastest) second
    scores = np.full(t.shape, 5.0)
    scores[:, 0], scores[:, 3] = 0.0, 1.0
    r = tuner.evaluate_rule(scores, X, t, m, k=2, margin_min=0.5)
    assert r["fallback_rate"] == 0.0 and r["top_k_rate"] == 0.0 and r["configs_timed_mean"] == 0.0
    assert np.isclose(r["regret"]["max"], (t[:, 0] / best - 1).max())
    # a near tie between the two: both are timed and the fastest measured is used
    scores[:, 3] = 0.01
    r = tuner.evaluate_rule(scores, X, t, m, k=2, margin_min=0.5)
    assert r["top_k_rate"] == 1.0 and r["regret"]["max"] == 0.0 and r["configs_timed_mean"] == 2.0
    assert np.isclose(r["regret_network"]["max"], (t[:, 0] / best - 1).max())
    # a configuration that cannot run is never picked, however good its score
    e = autotune.CONFIG_NAMES.index("ellr")
    scores[:, e] = -10.0
    mode, cand = tuner.decide(scores, runnable, X, m, k=2, margin_min=0.5)
    assert all(cand[i, 0] == e for i in range(len(t)) if runnable[i, e])
    assert all(cand[i, 0] != e for i in range(len(t)) if not runnable[i, e])
    # far outside the training range: the exhaustive autotuner
    Xo = X.copy()
    Xo[4, 0] = m.f_mu[0] + 100 * m.f_sd[0]
    r = tuner.evaluate_rule(scores, Xo, t, m, k=2, margin_min=0.5)
    assert np.isclose(r["fallback_rate"], 1 / 6)


def test_partial_retime_takes_only_records_one_revision_behind():
    """Re-timing a subset of the catalog upgrades only records whose other times are current;
    re-timing every entry takes every older record."""
    rev = autotune.TIMES_REV
    recs = {("1", "d"): {"times_rev": rev}, ("2", "d"): {"times_rev": rev - 1}, ("3", "d"): {},
            ("4", "d"): {"times_rev": rev - 2}, ("5", "e"): {"times_rev": rev - 1}}
    seeds = [1, 2, 3, 4, 5, 6]
    assert tuner.retime_todo(recs, seeds, "d", every_config=False) == [2]
    assert tuner.retime_todo(recs, seeds, "d", every_config=True) == [2, 3, 4]
