"""Exact numpy reference of the split-precision FP64 emulation (TEST
INFRASTRUCTURE ONLY: imported by tests/ and the benchmark's CPU leg alone).

Method (Ozaki, Ogita, Oishi, Rump, "Error-free transformations of matrix
multiplication by using fast routines of matrix multiplication and its
applications", Numer. Algorithms 59, 2012; integer variant: Ootomo, Ozaki,
Yokota, "DGEMM on integer matrix multiplication unit", IJHPCA 2024):

1. Row scale of A and column scale of B: sigma_i = 2^e_i with e_i the smallest
   integer such that max_k |a_ik| < 2^e_i (frexp exponent; an all-zero row
   gets e_i = 0).  Same for the columns of B (tau_j).
2. Digits: r = a / sigma_i (exact), then for s = 1..S:
   d_s = trunc(r * 2^7) in [-127, 127] and r <- r * 2^7 - d_s (both exact).
3. Integer products of digit pairs with s + t <= S + 1, exact in int64,
   grouped by weight: G_d = sum over s + t = d of A_s B_t.
4. Horner in FP64 from the smallest weight: h = G_{S+1}; for d = S .. 2:
   h = h * 2^-7 + G_d; the value is v_ij = sigma_i * tau_j * h * 2^-14
   (power-of-two scalings, exact).
5. K is processed in chunks (int32 exactness on the device); chunk values
   are summed in FP64 in chunk order.
6. C = beta * C + alpha * v, with beta == 0 meaning overwrite; the two
   products and the sum are separately rounded (no fused multiply-add).
"""
import numpy as np

DIGIT_BITS = 7
RADIX = float(1 << DIGIT_BITS)


def int32_chunk(S):
    """Largest K (multiple of 64) whose digit-pair sums stay below 2^31 in
    int32 for S slices: K * 127^2 * S < 2^31."""
    k = (2 ** 31 - 1) // (127 * 127 * S)
    return max(64, (k // 64) * 64)


def row_exponents(X):
    """e_i with max_k |x_ik| < 2^e_i (smallest such integer); 0 for zero rows."""
    mx = np.max(np.abs(X), axis=1) if X.shape[1] else np.zeros(X.shape[0])
    _, e = np.frexp(mx)
    return np.where(mx > 0, e, 0).astype(np.int64)


def digits(X, e, S):
    """S int8 digit matrices of the rows of X scaled by 2^-e."""
    r = np.ldexp(X, -e[:, None])
    out = []
    for _ in range(S):
        t = r * RADIX
        d = np.trunc(t)
        r = t - d
        out.append(d.astype(np.int8))
    return out


def emulate(A, B, S, alpha=1.0, beta=0.0, C=None, kchunk=None):
    """Emulated FP64 product of dense A (M x K) and B (K x N)."""
    A = np.asarray(A, np.float64)
    B = np.asarray(B, np.float64)
    M, K = A.shape
    N = B.shape[1]
    kchunk = kchunk or int32_chunk(S)
    ea = row_exponents(A)
    eb = row_exponents(B.T)
    Ad = digits(A, ea, S)
    Bd = digits(B.T, eb, S)
    acc = np.zeros((M, N))
    for c0 in range(0, K, kchunk):
        c1 = min(K, c0 + kchunk)
        G = {d: np.zeros((M, N), np.int64) for d in range(2, S + 2)}
        for s in range(1, S + 1):
            for t in range(1, S + 2 - s):
                G[s + t] += Ad[s - 1][:, c0:c1].astype(np.int64) @ Bd[t - 1][:, c0:c1].astype(np.int64).T
        h = G[S + 1].astype(np.float64)
        for d in range(S, 1, -1):
            h = h * (1.0 / RADIX) + G[d].astype(np.float64)
        v = np.ldexp(np.ldexp(h, -2 * DIGIT_BITS) , ea[:, None]) * np.ldexp(1.0, eb)[None, :]
        acc = v if c0 == 0 else acc + v
    out = alpha * acc
    if beta != 0.0 and C is not None:
        out = beta * np.asarray(C, np.float64) + out
    return out
