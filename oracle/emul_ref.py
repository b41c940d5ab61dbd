"""Exact numpy reference of the split-precision FP64 emulation (TEST
INFRASTRUCTURE ONLY: imported by tests/ and the benchmark's CPU leg alone).

Method (Ozaki, Ogita, Oishi, Rump, "Error-free transformations of matrix
multiplication by using fast routines of matrix multiplication and its
applications", Numer. Algorithms 59, 2012; integer variant: Ootomo, Ozaki,
Yokota, "DGEMM on integer matrix multiplication unit", IJHPCA 2024), in the
order the method states it:

1. Row scale of A and column scale of B: sigma_i = 2^e_i with e_i the smallest
   integer such that max_k |a_ik| < 2^e_i (frexp exponent; an all-zero row
   gets e_i = 0).  Same for the columns of B (tau_j).
2. Digits: r = a / sigma_i (exact), then for s = 1..S:
   d_s = trunc(r * 2^7) in [-127, 127] and r <- r * 2^7 - d_s (both exact).
3. Integer products of digit pairs with s + t <= S + 1, grouped by weight:
   G_d = sum over s + t = d of A_s B_t, each an exact integer sum over the
   whole K (int64: |G_d| <= S K 127^2, far below 2^63).  K is split only to
   bound memory, and the pieces are added in int64, so the split cannot
   change G_d.
4. Horner in FP64 from the smallest weight: h = G_{S+1}; for d = S .. 2:
   h = h * 2^-7 + G_d; the value is v_ij = h * 2^(e_i + e_j - 14) (one
   power-of-two scaling, rounded only on under- or overflow).
5. C = beta * C + alpha * v, with beta == 0 meaning overwrite; the two
   products and the sum are separately rounded (no fused multiply-add).

Rows of A or columns of B holding an infinity or a NaN cannot be sliced
into digits; every product element they touch is NaN.
"""
import numpy as np

DIGIT_BITS = 7
RADIX = float(1 << DIGIT_BITS)
# k per piece of the integer products (memory bound of the int64 temporaries).
MEMORY_PIECE = 1 << 16


def row_exponents(X):
    """e_i with max_k |x_ik| < 2^e_i (smallest such integer); 0 for zero rows.
    Rows with a non-finite entry are reported separately by ``finite_rows``."""
    X = np.asarray(X, np.float64)
    fin = np.where(np.isfinite(X), np.abs(X), 0.0)
    mx = np.max(fin, axis=1) if X.shape[1] else np.zeros(X.shape[0])
    _, e = np.frexp(mx)
    return np.where(mx > 0, e, 0).astype(np.int64)


def finite_rows(X):
    X = np.asarray(X, np.float64)
    return np.all(np.isfinite(X), axis=1) if X.shape[1] else np.ones(X.shape[0], bool)


def digits(X, e, S):
    """S int8 digit matrices of the rows of X scaled by 2^-e (step 2)."""
    r = np.ldexp(np.asarray(X, np.float64), -e[:, None])
    out = []
    for _ in range(S):
        t = r * RADIX
        d = np.trunc(t)
        r = t - d
        out.append(d.astype(np.int8))
    return out


def weight_sums(Ad, Bd, S):
    """G_d (d = 2 .. S + 1) of step 3: exact int64 sums over the whole K.
    Ad[s] is M x K, Bd[t] is N x K (columns of B as rows)."""
    M, K = Ad[0].shape
    N = Bd[0].shape[0]
    G = {d: np.zeros((M, N), np.int64) for d in range(2, S + 2)}
    for k0 in range(0, K, MEMORY_PIECE):
        k1 = min(K, k0 + MEMORY_PIECE)
        for s in range(1, S + 1):
            a = Ad[s - 1][:, k0:k1].astype(np.int64)
            for t in range(1, S + 2 - s):
                G[s + t] += a @ Bd[t - 1][:, k0:k1].astype(np.int64).T
    return G


def emulate(A, B, S, alpha=1.0, beta=0.0, C=None):
    """Emulated FP64 product of dense A (M x K) and B (K x N)."""
    A = np.asarray(A, np.float64)
    B = np.asarray(B, np.float64)
    M, K = A.shape
    N = B.shape[1]
    fa, fb = finite_rows(A), finite_rows(B.T)
    A = np.where(fa[:, None], A, 0.0)
    Bt = np.where(fb[:, None], B.T, 0.0)
    ea = row_exponents(A)
    eb = row_exponents(Bt)
    if K == 0:
        v = np.zeros((M, N))
    else:
        G = weight_sums(digits(A, ea, S), digits(Bt, eb, S), S)
        h = G[S + 1].astype(np.float64)
        for d in range(S, 1, -1):
            h = h * (1.0 / RADIX) + G[d].astype(np.float64)
        v = np.ldexp(h, ea[:, None] + eb[None, :] - 2 * DIGIT_BITS)
    v = np.where(fa[:, None] & fb[None, :], v, np.nan)
    # alpha == 0 skips the products (BLAS convention), NaN included.
    out = alpha * v if alpha != 0.0 else np.zeros((M, N))
    if beta != 0.0 and C is not None:
        out = beta * np.asarray(C, np.float64) + out
    return out
