"""Pins of the numpy model reference: back-propagation against central finite
differences in FP64, Adam's first step against its closed form, and a
learnable target."""
import numpy as np

from oracle import mlp_ref as ref


def test_backprop_matches_finite_differences():
    rng = np.random.default_rng(0)
    F = 9
    P = ref.init_params(F, seed=1, dtype=np.float64)
    # push some biases so both ReLU branches are exercised away from the kink
    X = rng.normal(size=(37, F))
    T = rng.normal(size=37)
    G, _ = ref.grad(P, X, T)
    idx = rng.choice(len(P), size=200, replace=False)
    h = 1e-6
    for i in idx:
        Pp = P.copy(); Pp[i] += h
        Pm = P.copy(); Pm[i] -= h
        fd = (ref.loss(Pp, X, T) - ref.loss(Pm, X, T)) / (2 * h)
        assert abs(fd - G[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, G[i])


def test_adam_first_step_closed_form():
    """With zero moments, the first bias-corrected step is lr * g / (|g| + eps)."""
    g = np.array([3.0, -0.5, 1e-3, 0.0])
    P = np.zeros(4)
    P1, M, V = ref.adam_step(P, g, np.zeros(4), np.zeros(4), 1, lr=0.01)
    assert np.allclose(P1, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)


def test_training_learns_a_smooth_target():
    rng = np.random.default_rng(3)
    F = 3
    X = rng.uniform(-1, 1, size=(512, F))
    T = X[:, 0] * 0.7 - X[:, 1] ** 2 + 0.2 * np.abs(X[:, 2])
    P = ref.init_params(F, seed=2, dtype=np.float64)
    M = np.zeros_like(P); V = np.zeros_like(P)
    l0 = ref.loss(P, X, T)
    step = 0
    for ep in range(60):
        for b in range(0, 512, 64):
            step += 1
            G, _ = ref.grad(P, X[b:b + 64], T[b:b + 64])
            P, M, V = ref.adam_step(P, G, M, V, step, lr=3e-3)
    assert ref.loss(P, X, T) < 0.05 * l0


def _adam_constant_gradient_pin(step_fn, steps=12, lr=0.01):
    """A constant gradient g gives moments m_t = (1 - b1^t) g and
    v_t = (1 - b2^t) g^2, so the bias-corrected estimates are exactly g and
    g^2 at every step and t steps move the parameters by t lr g / (|g| + eps)."""
    g = np.array([3.0, -0.5, 1e-3, -40.0])
    P = np.zeros(4)
    M = np.zeros(4)
    V = np.zeros(4)
    for t in range(1, steps + 1):
        P, M, V = step_fn(P, g, M, V, t, lr=lr)
        want = -t * lr * g / (np.abs(g) + 1e-8)
        if not np.allclose(P, want, rtol=1e-12, atol=0):
            return False
    return True


def test_adam_later_steps_closed_form():
    assert _adam_constant_gradient_pin(ref.adam_step)


def test_adam_pin_catches_stale_bias_correction():
    """Planted mistake: bias correction with the first step's powers at every
    step (right at step 1, wrong from step 2 on)."""
    def stale(P, G, M, V, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        M = b1 * M + (1 - b1) * G
        V = b2 * V + (1 - b2) * G * G
        return P - lr * (M / (1 - b1)) / (np.sqrt(V / (1 - b2)) + eps), M, V

    assert not _adam_constant_gradient_pin(stale)
