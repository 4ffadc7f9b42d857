"""Autotuner and learned tuner on the GPU.

The learned tuner is retrained here from the committed sweep (timings of the exhaustive
autotuner on 4000 training and 500 held-out seeded matrices) with the library's network
kernels, and evaluated on the held-out matrices: its regret against the exhaustive search and
what it gains over the untuned default configuration."""
import os

import numpy as np
import pytest
import torch

import synth
from paper_1112_5588_amd import PjdsMatrix, autotune, tuner

pytestmark = pytest.mark.gpu

STORE = os.path.join(tuner.DATA_DIR, "sweep.jsonl")


def test_autotune_picks_the_fastest_configuration():
    A = synth.banded_stratified(60000, 5, halo=512)
    r = autotune.autotune(A, reps=5)
    assert set(r.times_ms) == set(autotune.CONFIG_NAMES)
    assert r.times_ms[r.best.name] == min(r.times_ms.values())
    assert r.speedup_over_default >= 1.0


def test_spmmv_and_batch_tuning_return_catalog_values():
    A = synth.laplacian_2d(128)
    M = PjdsMatrix.from_csr(A)
    (t, vpl, remap), times = autotune.tune_spmmv(M, 8)
    assert t in (1, 2, 4, 8, 16) and vpl in (1, 2, 4) and times[(t, vpl, remap)] == min(times.values())
    mats = [PjdsMatrix.from_csr(synth.banded_stratified(n, 1000 + k), split_len=-1) for k, n in enumerate((1000, 5000, 20000))]
    xs = [torch.from_numpy(synth.dense_x(M_.n_cols, 7)).cuda() for M_ in mats]
    ys = [torch.empty(M_.n_rows, dtype=torch.float64, device="cuda") for M_ in mats]
    g, times = autotune.tune_batch(mats, xs, ys, groups=(1, 8))
    assert g in (1, 8)


@pytest.fixture(scope="module")
def trained():
    recs = [r for r in tuner.load_records(STORE) if r.get("times_rev", 1) >= autotune.TIMES_REV]
    train_r = [r for r in recs if tuner.TRAIN_SEED0 <= int(r["key"]) < tuner.TEST_SEED0]
    test_r = [r for r in recs if int(r["key"]) >= tuner.TEST_SEED0]
    assert len(train_r) >= 1000 and len(test_r) >= 200
    X, y, _ = tuner.arrays(train_r)
    model = tuner.train(X, y, epochs=3000)
    return model, train_r, test_r


def test_training_converges(trained):
    model, _, _ = trained
    hist = model.meta["loss_history"]
    assert hist[-1][1] < 0.5 * hist[0][1]


def test_learned_tuner_regret_and_gain_on_held_out_matrices(trained):
    model, _, test_r = trained
    Xt, _, tt = tuner.arrays(test_r)
    rep = tuner.evaluate_rule(tuner.predict_scores(model, Xt), Xt, tt, model)
    # against the exhaustive autotuner (regret 0 by definition): the network's pick alone, and
    # the rule that times its three best candidates on a near tie
    assert rep["regret_network"]["median"] < 0.05
    assert rep["regret_network"]["mean"] < 0.15
    assert rep["regret"]["mean"] <= rep["regret_network"]["mean"] + 1e-12
    assert rep["regret"]["mean"] < 0.03
    assert rep["fallback_rate"] <= 0.25
    assert rep["configs_timed_mean"] < 0.5 * rep["configs_timed_exhaustive"]
    # what the network gains over the untuned default (pJDS, b_r 64, global sort)
    assert rep["geomean_gain_over_default_network_only"] > 1.05
    assert rep["geomean_gain_over_default"] <= rep["geomean_best_over_default"] + 1e-9


def test_committed_model_loads_and_predicts(trained):
    path = os.path.join(tuner.DATA_DIR, "model.json")
    m = tuner.Model.load(path)
    _, _, test_r = trained
    Xt, _, tt = tuner.arrays(test_r)
    idx, mg = tuner.predict_matrices(m, Xt, np.array([r["nnz"] for r in test_r], float))
    assert idx.min() >= 0 and idx.max() < len(autotune.CATALOG)
    # the decision rule never picks a configuration that cannot run on the matrix
    runnable = np.isfinite(tt)
    mode, cand = tuner.decide(tuner.predict_scores(m, Xt), runnable, Xt, m)
    assert np.all(runnable[np.arange(len(cand)), cand[:, 0]])
