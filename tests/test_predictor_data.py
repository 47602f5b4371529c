"""The committed tuning sweep and trained predictor: format, consistency with
the generator and the grid, and the held-out result stored with the model
(host only)."""
import json
import os

import numpy as np
import pytest

import matgen
from paper_2204_06666_amd import features
from paper_2204_06666_amd.predictor import N_PARAMS, ROWS_PER_WAVE, SLICE_ROWS, WIDTH_QUANTILES
from paper_2204_06666_amd.train_predictor import load_sweeps

DATA = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2204_06666_amd", "data")
SWEEP = os.path.join(DATA, "tuning_sweep.jsonl")
MODEL = os.path.join(DATA, "predictor_fp32.json")

pytestmark = pytest.mark.skipif(not os.path.exists(SWEEP), reason="no committed sweep")


def test_sweep_records():
    recs = load_sweeps([SWEEP])
    assert [r["i"] for r in recs] == list(range(len(recs)))
    for r in recs:
        assert r["slice_rows"] == list(SLICE_ROWS) and r["rows_per_wave"] == list(ROWS_PER_WAVE)
        assert r["width_q"] == list(WIDTH_QUANTILES)
        t = np.array(r["times_us"])
        assert t.shape == (6, 4, 4) and np.all(t > 0) and r["eq1"]["time_us"] > 0
        assert len(r["features"]) == 32


@pytest.mark.parametrize("i", [0, 3, 6, 9])
def test_recorded_features_match_the_generator(i):
    recs = {r["i"]: r for r in load_sweeps([SWEEP])}
    desc, A = matgen.tuning_matrix(i, n_hi=250_000)
    assert desc == recs[i]["desc"] and A.n_rows == recs[i]["n"] and A.nnz == recs[i]["nnz"]
    np.testing.assert_allclose(features(A), recs[i]["features"], rtol=1e-6, atol=1e-9)


def test_model_file():
    if not os.path.exists(MODEL):
        pytest.skip("no committed model")
    d = json.load(open(MODEL))
    assert len(d["params"]) == N_PARAMS and len(d["mean"]) == 32 and len(d["std"]) == 32
    m = d["meta"]
    n = len(load_sweeps([SWEEP]))
    assert 0 < m["n_train"] < n and m["n_held_out"] == n - m["n_train"]
    assert m["result"]["held_out"]["n"] == n - m["n_train"]


def test_recorded_result_meets_the_targets():
    """The held-out result stored with the committed model meets the targets
    (within 10% of the exhaustive best, geomean; faster than the Eq. 1
    default), and recomputing it on the CPU (FP64 reference network on the
    stored weights, committed sweep times) gives the same figures."""
    if not os.path.exists(MODEL):
        pytest.skip("no committed model")
    from oracle import mlp
    from paper_2204_06666_amd.predictor import decode_output
    from paper_2204_06666_amd.train_predictor import Predictor, evaluate
    d = json.load(open(MODEL))
    res = d["meta"]["result"]["held_out"]
    assert res["geomean_pred_over_best"] <= 1.10
    assert res["share_pred_within_1.10"] >= 0.7
    assert res["geomean_eq1_over_pred"] > 1.0
    pred = Predictor.load(MODEL)
    te = [r for r in load_sweeps([SWEEP]) if r["i"] >= d["meta"]["n_train"]]
    Y, _ = mlp.forward(pred.params.astype(np.float64), pred.normalise([r["features"] for r in te]).astype(np.float64))
    again = evaluate(te, [decode_output(y) for y in Y])
    assert abs(again["geomean_pred_over_best"] - res["geomean_pred_over_best"]) <= 0.01
    assert abs(again["geomean_eq1_over_pred"] - res["geomean_eq1_over_pred"]) <= 0.02


PROBE = os.path.join(DATA, "tuning_sweep_large_probe.jsonl")


def test_large_matrix_probe_and_the_range_guard():
    """12 matrices of 2.7e5-9.7e5 rows swept over the full grid: all lie above
    the committed network's training range, where its points are far from the
    best (checked here with the FP64 reference network) and the Eq. 1 default
    is within 10% of the grid's best (geomean), so Predictor.choose falls back
    to the default for them."""
    from oracle import mlp
    from paper_2204_06666_amd.predictor import decode_output
    from paper_2204_06666_amd.train_predictor import Predictor, evaluate
    probe = load_sweeps([PROBE])
    assert len(probe) == 12
    pred = Predictor.load(MODEL)
    lo, hi = pred.n_range
    assert all(r["n"] > hi for r in probe)
    Y, _ = mlp.forward(pred.params.astype(np.float64), pred.normalise([r["features"] for r in probe]).astype(np.float64))
    res = evaluate(probe, [decode_output(y) for y in Y])
    assert res["geomean_pred_over_best"] > 1.10
    assert res["geomean_eq1_over_best"] <= 1.10
    # the guard: points outside the range become None (the Eq. 1 default)
    pred.predict = lambda F, device=None: [(256, None, 64)] * len(np.atleast_2d(F))
    out = pred.choose([r["features"] for r in probe[:2]] + [probe[0]["features"]], [r["n"] for r in probe[:2]] + [lo])
    assert out == [None, None, (256, None, 64)]
