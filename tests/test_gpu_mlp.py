"""MLP kernels against the numpy FP32 reference (tolerance 1e-5, relative to
the largest magnitude of the compared quantity)."""
import numpy as np
import pytest

from oracle import mlp_ref as ref

from tests.helpers import lib

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _close(a, b):
    scale = max(1.0, float(np.max(np.abs(b))))
    return float(np.max(np.abs(np.asarray(a, np.float64) - np.asarray(b, np.float64)))) / scale


@pytest.mark.parametrize("F,n", [(9, 1), (9, 333), (5, 70)])
def test_forward(F, n):
    b = lib()
    rng = np.random.default_rng(F * 100 + n)
    P = ref.init_params(F, seed=n)
    X = rng.normal(size=(n, F)).astype(np.float32)
    y = b.bsmm_mlp_forward(P, X)
    yr, _ = ref.forward(P, X)
    assert _close(y, yr) <= TOL


@pytest.mark.parametrize("n", [1, 64, 257])
def test_gradient_and_loss(n):
    b = lib()
    F = 9
    rng = np.random.default_rng(n)
    P = ref.init_params(F, seed=7)
    X = rng.normal(size=(n, F)).astype(np.float32)
    T = rng.normal(size=n).astype(np.float32)
    g, loss = b.bsmm_mlp_grad(P, X, T)
    gr, lr_ = ref.grad(P, X, T)
    assert _close(g, gr) <= TOL
    assert abs(loss - lr_) <= TOL * max(1.0, abs(lr_))


def test_adam_steps():
    b = lib()
    F = 9
    rng = np.random.default_rng(1)
    P = ref.init_params(F, seed=3)
    M = np.zeros_like(P); V = np.zeros_like(P)
    Pr, Mr, Vr = P.copy(), M.copy(), V.copy()
    for step in range(1, 4):
        G = rng.normal(size=P.shape).astype(np.float32)
        b.bsmm_mlp_adam_step(F, P, G, M, V, step, lr=1e-3)
        Pr, Mr, Vr = ref.adam_step(Pr, G, Mr, Vr, step, lr=1e-3)
    assert _close(P, Pr) <= TOL and _close(M, Mr) <= TOL and _close(V, Vr) <= TOL


def test_training_reduces_loss():
    b = lib()
    F = 9
    rng = np.random.default_rng(5)
    X = rng.normal(size=(2000, F)).astype(np.float32)
    T = (np.sin(X[:, 0]) + 0.5 * X[:, 1] * X[:, 2]).astype(np.float32)
    P0 = ref.init_params(F, seed=0)
    l0 = float(np.mean((ref.forward(P0, X)[0] - T) ** 2))
    P, loss = b.bsmm_mlp_train(P0, X, T, epochs=40, batch=128, lr=2e-3, seed=1)
    assert loss < 0.2 * l0
    assert abs(loss - float(np.mean((ref.forward(P, X)[0] - T) ** 2))) <= 1e-4 * max(1.0, l0)
    P2, loss2 = b.bsmm_mlp_train(P0, X, T, epochs=40, batch=128, lr=2e-3, seed=1)
    assert np.array_equal(P, P2)  # fixed-order reductions: reproducible training


def test_model_selection_uses_argmin(tmp_path):
    """A weight file drives parameter selection for a shape absent from the
    database: the chosen set is the candidate with the lowest prediction."""
    b = lib()
    F = len(b.bsmm_mlp_features(4, 4, 4, np.array([1, 1, 0, 0], np.int32)))
    P = ref.init_params(F, seed=11)
    mean = np.zeros(F, np.float32); sd = np.ones(F, np.float32)
    path = tmp_path / "mlp.txt"
    with open(path, "w") as f:
        f.write(f"bsmm-mlp features {F}\nmean " + " ".join(map(repr, mean.tolist())) + "\n")
        f.write("std " + " ".join(map(repr, sd.tolist())) + "\n")
        f.write(f"params {len(P)}\n" + " ".join(repr(float(x)) for x in P) + "\n")
    m, n, k = 17, 29, 11
    cands = b.bsmm_tune_candidates(m, n, k)
    b.bsmm_set_option("tune_db", "")
    b.bsmm_set_option("mlp_weights", str(path))
    try:
        for R in (1, 8, 27):
            X = np.stack([b.bsmm_mlp_features(m, n, k, c, R) for c in cands])
            y, _ = ref.forward(P, X)
            want = tuple(int(x) for x in cands[int(np.argmin(y))])
            assert b.bsmm_select_params(m, n, k, R) == want, R
    finally:
        b.bsmm_set_option("mlp_weights", "")


def test_model_with_other_feature_count_is_ignored(tmp_path):
    """Weights trained on a different feature vector are not used: selection
    falls back to the plain rule."""
    b = lib()
    F = len(b.bsmm_mlp_features(4, 4, 4, np.array([1, 1, 0, 0], np.int32))) - 1
    P = ref.init_params(F, seed=12)
    path = tmp_path / "mlp_old.txt"
    with open(path, "w") as f:
        f.write(f"bsmm-mlp features {F}\nmean " + " ".join(["0.0"] * F) + "\n")
        f.write("std " + " ".join(["1.0"] * F) + "\n")
        f.write(f"params {len(P)}\n" + " ".join(repr(float(x)) for x in P) + "\n")
    b.bsmm_set_option("tune_db", "")
    b.bsmm_set_option("mlp_weights", str(path))
    try:
        assert b.bsmm_select_params(17, 29, 11) == b.bsmm_select_params(17, 29, 11)
        b.bsmm_set_option("mlp_weights", "")
        plain = b.bsmm_select_params(17, 29, 11)
        b.bsmm_set_option("mlp_weights", str(path))
        assert b.bsmm_select_params(17, 29, 11) == plain
    finally:
        b.bsmm_set_option("mlp_weights", "")


def test_model_not_extrapolated_past_trained_run_lengths():
    """Runs far longer than the tuner's (a tall-and-skinny product gives
    C blocks tens of thousands of products) are presented to the committed
    model as runs of 32, the longest it was trained on; (22, 22, 22) is not
    in the database, so the model decides."""
    b = lib()
    b.use_default_tuning()
    assert b.bsmm_select_params(22, 22, 22, 90112) == b.bsmm_select_params(22, 22, 22, 32)
    assert b.bsmm_select_params(22, 22, 22, 33) == b.bsmm_select_params(22, 22, 22, 32)
