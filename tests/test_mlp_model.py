"""The committed learned model and its held-out evaluation (paper Sec. II:
a model trained on part of the tuning data predicts the kernel parameters of
every other shape).

The tuner's timing table over 600 random shapes (each at several run
lengths), the weights trained on the GPU from 500 of them, and the report of
the evaluation on the other 100 are committed together.  These CPU tests recompute that evaluation from the table
and the weights with the numpy forward pass of the model, so the reported
figures follow from committed data and not from the GPU run alone.
"""
import json
import os

import numpy as np
import pytest

from oracle import mlp_ref

DB_DIR = os.path.join(os.path.dirname(__file__), "..", "paper_1910_04796_amd", "tune_db")
TABLE = os.path.join(DB_DIR, "gfx950_random_all.csv.gz")
WEIGHTS = os.path.join(DB_DIR, "gfx950_mlp.txt")
REPORT = os.path.join(DB_DIR, "mlp_report.json")
RANDOM_DB = os.path.join(DB_DIR, "gfx950_random.txt")


def read_weights(path):
    lines = open(path).read().split("\n")
    assert lines[0].startswith("bsmm-mlp features")
    F = int(lines[0].split()[2])
    mean = np.array(lines[1].split()[1:], np.float32)
    sd = np.array(lines[2].split()[1:], np.float32)
    n = int(lines[3].split()[1])
    P = np.array(lines[4].split(), np.float32)
    assert len(mean) == F and len(sd) == F and len(P) == n == mlp_ref.param_count(F)
    return mean, sd, P


@pytest.fixture(scope="module")
def heldout():
    if not all(os.path.exists(p) for p in (TABLE, WEIGHTS, REPORT, RANDOM_DB)):
        pytest.skip("learned model files not committed")
    from paper_1910_04796_amd import bsmm, learn
    rows = learn.read_table(TABLE)
    shapes = sorted({(int(r[0]), int(r[1]), int(r[2])) for r in rows})
    rep = json.load(open(REPORT))
    held = learn.holdout_split(shapes, rep["held_out"], rep["seed"])
    sel = np.array([(int(r[0]), int(r[1]), int(r[2])) in held for r in rows])
    hrows = rows[sel]
    X = np.stack([bsmm.bsmm_mlp_features(int(r[0]), int(r[1]), int(r[2]), r[4:8].astype(np.int32), int(r[3]))
                  for r in hrows])
    mean, sd, P = read_weights(WEIGHTS)
    Xn = ((X - mean) / sd).astype(np.float32)
    pred, _ = mlp_ref.forward(P, Xn)
    return learn, rows, hrows, held, pred, rep


def test_table_covers_the_shapes(heldout):
    learn, rows, hrows, held, pred, rep = heldout
    shapes = {(int(r[0]), int(r[1]), int(r[2])) for r in rows}
    assert len(shapes) == rep["shapes"] == 600
    assert len(held) == rep["held_out"] == 100
    assert len(rows) - len(hrows) == rep["train_rows"]
    assert all(4 <= v <= 64 for s in shapes for v in s)
    assert (rows[:, learn.T_US] > 0).all()
    assert sorted({int(r[3]) for r in rows}) == rep["run_lengths"]


def test_heldout_evaluation_reproduces_report(heldout):
    """Best / pick over the held-out shapes, recomputed on the CPU, agrees
    with the GPU run's report (FP32 forward passes may break near-ties
    differently, hence the small tolerance)."""
    learn, rows, hrows, held, pred, rep = heldout
    ratios, speedups = learn.evaluate(hrows, held, pred, learn.read_plain(RANDOM_DB))
    n_cases = 100 * len(rep["run_lengths"])
    assert len(ratios) == n_cases == rep["heldout_cases"] and len(speedups) == n_cases
    assert (ratios <= 1.0).all() and (ratios > 0).all()
    r = rep["heldout_best_over_pick"]
    assert abs(ratios.mean() - r["mean"]) < 0.01
    assert abs((ratios >= 0.9).mean() - r["share_ge_0.9"]) <= 0.03
    g = rep["heldout_plain_over_pick"]["geomean"]
    assert abs(np.exp(np.log(speedups).mean()) - g) < 0.02 * g
    # The model is useful: on shapes it never saw it picks sets within 10 %
    # of the exhaustive best on most shapes and beats the plain rule overall.
    assert ratios.mean() > 0.9
    assert np.exp(np.log(speedups).mean()) > 1.2


def test_model_beats_random_choice(heldout):
    """Against the expected best / pick of a uniformly random candidate, the
    model's pick is better on average (a model that learned nothing is not)."""
    learn, rows, hrows, held, pred, rep = heldout
    ratios, _ = learn.evaluate(hrows, held, pred, {})
    rand = []
    key = [(int(r[0]), int(r[1]), int(r[2]), int(r[3])) for r in hrows]
    for c in sorted(set(key)):
        t = hrows[[i for i, k in enumerate(key) if k == c], learn.T_US]
        rand.append(np.mean(t.min() / t))
    assert ratios.mean() > np.mean(rand) + 0.1


HELDOUT_TABLE = os.path.join(DB_DIR, "gfx950_heldout_sizes_all.csv.gz")


def test_model_on_block_sizes_absent_from_the_database():
    """Shapes {6,14,22,30}^3, none of them in the tuning database nor in the
    model's training shapes, timed exhaustively by the tuner at three run
    lengths: the set the model ranks first runs at 0.95 or more of the
    exhaustive best on average, and at 0.75 or more in every case."""
    if not all(os.path.exists(p) for p in (HELDOUT_TABLE, WEIGHTS, RANDOM_DB)):
        pytest.skip("learned model files not committed")
    from paper_1910_04796_amd import bsmm, learn
    rows = learn.read_table(HELDOUT_TABLE)
    shapes = {(int(r[0]), int(r[1]), int(r[2])) for r in rows}
    assert shapes == {(m, n, k) for m in (6, 14, 22, 30) for n in (6, 14, 22, 30) for k in (6, 14, 22, 30)}
    train = {tuple(int(x) for x in l.split()[:3]) for l in open(RANDOM_DB) if l.strip() and l[0] != "#"}
    assert not shapes & train
    X = np.stack([bsmm.bsmm_mlp_features(int(r[0]), int(r[1]), int(r[2]), r[4:8].astype(np.int32), int(r[3]))
                  for r in rows])
    mean, sd, P = read_weights(WEIGHTS)
    pred, _ = mlp_ref.forward(P, ((X - mean) / sd).astype(np.float32))
    groups = {}
    for i, r in enumerate(rows):
        groups.setdefault((int(r[0]), int(r[1]), int(r[2]), int(r[3])), []).append(i)
    ratios = []
    for idx in groups.values():
        idx = np.array(idx)
        t = rows[idx, 8].astype(float)
        ratios.append(t.min() / float(rows[idx[np.argmin(pred[idx])], 8]))
    ratios = np.array(ratios)
    assert len(ratios) == 192
    assert ratios.mean() >= 0.95 and ratios.min() >= 0.75, (ratios.mean(), ratios.min())
