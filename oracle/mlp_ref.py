"""Plain numpy reference of the learned performance model (TEST
INFRASTRUCTURE ONLY: imported by tests/ alone).

The model is the two-hidden-layer ReLU perceptron
    y = W3 relu(W2 relu(W1 x + b1) + b2) + b3      (hidden width 64)
trained on the mean squared error with Adam (Kingma and Ba, "Adam: a method
for stochastic optimization", ICLR 2015).  Parameters are one flat array:
W1 [64 x F] row-major, b1 [64], W2 [64 x 64] row-major, b2 [64], W3 [64], b3 [1].
Every function works in the dtype of its inputs (float32 for parity with
the GPU, float64 for the finite-difference pin).
"""
import numpy as np

H = 64


def param_count(F):
    return H * F + H + H * H + H + H + 1


def unpack(P, F):
    o = 0
    W1 = P[o:o + H * F].reshape(H, F); o += H * F
    b1 = P[o:o + H]; o += H
    W2 = P[o:o + H * H].reshape(H, H); o += H * H
    b2 = P[o:o + H]; o += H
    W3 = P[o:o + H]; o += H
    b3 = P[o:o + 1]
    return W1, b1, W2, b2, W3, b3


def init_params(F, seed=0, dtype=np.float32):
    """He-uniform weights, zero biases."""
    rng = np.random.default_rng(seed)
    P = np.zeros(param_count(F), dtype=np.float64)
    W1, b1, W2, b2, W3, b3 = unpack(P, F)
    W1[:] = rng.uniform(-1, 1, W1.shape) * np.sqrt(6.0 / F)
    W2[:] = rng.uniform(-1, 1, W2.shape) * np.sqrt(6.0 / H)
    W3[:] = rng.uniform(-1, 1, W3.shape) * np.sqrt(6.0 / H)
    return P.astype(dtype)


def forward(P, X):
    F = X.shape[1]
    W1, b1, W2, b2, W3, b3 = unpack(P, F)
    a1 = X @ W1.T + b1
    h1 = np.maximum(a1, 0)
    a2 = h1 @ W2.T + b2
    h2 = np.maximum(a2, 0)
    y = h2 @ W3 + b3[0]
    return y, (h1, h2)


def loss(P, X, T):
    y, _ = forward(P, X)
    return np.mean((y - T) ** 2)


def grad(P, X, T):
    """Gradient of mean((y - T)^2) by back-propagation, and the loss."""
    F = X.shape[1]
    n = X.shape[0]
    W1, b1, W2, b2, W3, b3 = unpack(P, F)
    y, (h1, h2) = forward(P, X)
    dy = 2.0 * (y - T) / n
    G = np.zeros_like(P)
    gW1, gb1, gW2, gb2, gW3, gb3 = unpack(G, F)
    gW3[:] = dy @ h2
    gb3[0] = dy.sum()
    d2 = np.outer(dy, W3) * (h2 > 0)
    gW2[:] = d2.T @ h1
    gb2[:] = d2.sum(axis=0)
    d1 = (d2 @ W2) * (h1 > 0)
    gW1[:] = d1.T @ X
    gb1[:] = d1.sum(axis=0)
    return G, float(np.mean((y - T) ** 2))


def adam_step(P, G, M, V, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One bias-corrected Adam update; returns new (P, M, V)."""
    M = b1 * M + (1 - b1) * G
    V = b2 * V + (1 - b2) * G * G
    mh = M / (1 - b1 ** step)
    vh = V / (1 - b2 ** step)
    return P - lr * mh / (np.sqrt(vh) + eps), M, V
