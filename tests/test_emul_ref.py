"""Pins of the emulation reference against exact arithmetic."""
from fractions import Fraction

import numpy as np

from oracle import emul_ref as er
from oracle import oracle as orc
from synth import rng_of, values_wide_range

# K beyond which an INT32 accumulator of the 7-slice method can overflow:
# the heaviest weight sums S = 7 digit pairs, each up to 127^2 per k.
K_INT32_7 = (2 ** 31 - 1) // (127 * 127 * 7)


def _exact_product(A, B):
    M, K = A.shape
    N = B.shape[1]
    Af = [[Fraction(float(x)) for x in row] for row in A]
    Bf = [[Fraction(float(x)) for x in row] for row in B]
    return [[sum(Af[i][k] * Bf[k][j] for k in range(K)) for j in range(N)] for i in range(M)]


def _dropped_bound(S, K):
    """Largest value of the dropped digit pairs (s + t > S + 1) per unit of
    sigma_i tau_j: 2S + 1 - d pairs of weight d, each at most 127^2 2^-7d per k."""
    return sum(Fraction(2 * S + 1 - d) * K * 127 * 127 / Fraction(2) ** (7 * d)
               for d in range(S + 2, 2 * S + 1))


def test_integer_inputs_exact_with_one_slice():
    """|x| <= 127 integers: one 7-bit digit holds every entry exactly, so the
    emulated product is the exact integer product."""
    rng = rng_of(1)
    A = rng.integers(-127, 128, size=(19, 33)).astype(np.float64)
    B = rng.integers(-127, 128, size=(33, 21)).astype(np.float64)
    exact = (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float64)
    assert np.array_equal(er.emulate(A, B, 1), exact)


def test_digits_reconstruct_entries():
    """Entries with at most 7*S significant bits below their row's scale are
    recovered exactly from their digits."""
    rng = rng_of(2)
    S = 4
    e = rng.integers(-5, 6, size=12)
    ints = rng.integers(-(2 ** 27) + 1, 2 ** 27, size=(12, 9))
    X = np.ldexp(ints.astype(np.float64), (e - 28)[:, None])
    ex = er.row_exponents(X)
    D = er.digits(X, ex, S)
    rec = sum(np.ldexp(D[s].astype(np.float64), -7 * (s + 1)) for s in range(S))
    assert np.array_equal(np.ldexp(rec, ex[:, None]), X)


def test_within_closed_form_bound_of_exact_product():
    """Digit-exact inputs (at most 41 bits below the row scale, S = 7 slices
    hold 49): the only differences from the exact rational product are the
    dropped digit pairs (s + t > S + 1, each term at most 127^2 2^-7d per k)
    and FP64 rounding of the Horner sum."""
    rng = rng_of(3)
    S, K = 7, 11
    A = np.ldexp(rng.integers(-(2 ** 40), 2 ** 40, size=(6, K)).astype(np.float64), -40)
    B = np.ldexp(rng.integers(-(2 ** 40), 2 ** 40, size=(K, 5)).astype(np.float64), -38)
    X = er.emulate(A, B, S)
    E = _exact_product(A, B)
    ea = er.row_exponents(A)
    eb = er.row_exponents(B.T)
    dropped = _dropped_bound(S, K)
    absprod = np.abs(A) @ np.abs(B)
    for i in range(6):
        for j in range(5):
            bound = dropped * Fraction(2) ** int(ea[i] + eb[j]) + Fraction(float(absprod[i, j])) / 2 ** 49
            assert abs(Fraction(float(X[i, j])) - E[i][j]) <= bound


def test_full_k_weight_sums_closed_form_beyond_int32():
    """Every digit 127 (entries 1 - 2^-49, scale 2^0) makes the weight sums
    G_d = (d - 1) K 127^2 exactly.  At K = 20,000 the heaviest one,
    7 K 127^2 = 2,258,060,000, exceeds 2^31, so a reference that accumulated
    in INT32, or rounded per K piece, could not meet the closed form: the
    recombined value must be the exact sum of G_d 2^-7d within the FP64
    rounding of S Horner steps over positive terms."""
    S, K = 7, 20000
    assert K > K_INT32_7
    x = 1.0 - 2.0 ** -49
    A = np.full((2, K), x)
    B = np.full((K, 3), x)
    X = er.emulate(A, B, S)
    exact = sum(Fraction((d - 1) * K * 127 * 127) / Fraction(2) ** (7 * d) for d in range(2, S + 2))
    assert 7 * K * 127 * 127 > 2 ** 31
    for v in X.ravel():
        assert abs(Fraction(float(v)) - exact) <= exact * S / Fraction(2) ** 53
    # and the exact product K x^2 differs from it only by the dropped pairs
    assert abs(Fraction(x) ** 2 * K - exact) <= _dropped_bound(S, K)


def test_full_k_random_digit_exact_beyond_int32():
    """Random digit-exact inputs at K = 20,000 > the INT32 bound of one
    accumulator: within the closed-form bound of the exact rational product
    (exact integer arithmetic on the 2^-40 / 2^-38 grids)."""
    rng = rng_of(11)
    S, K, M, N = 7, 20000, 3, 2
    ia = rng.integers(-(2 ** 40), 2 ** 40, size=(M, K))
    ib = rng.integers(-(2 ** 40), 2 ** 40, size=(K, N))
    A = np.ldexp(ia.astype(np.float64), -40)
    B = np.ldexp(ib.astype(np.float64), -38)
    X = er.emulate(A, B, S)
    ea, eb = er.row_exponents(A), er.row_exponents(B.T)
    dropped = _dropped_bound(S, K)
    absprod = np.abs(A) @ np.abs(B)
    for i in range(M):
        for j in range(N):
            e = sum(int(ia[i, k]) * int(ib[k, j]) for k in range(K))
            exact = Fraction(e) / Fraction(2) ** 78
            bound = dropped * Fraction(2) ** int(ea[i] + eb[j]) + Fraction(float(absprod[i, j])) / 2 ** 49
            assert abs(Fraction(float(X[i, j])) - exact) <= bound


def test_memory_pieces_do_not_change_the_result(monkeypatch):
    """Splitting K into pieces for memory adds integers: bit-identical."""
    rng = rng_of(5)
    A = values_wide_range(rng, 7 * 700).reshape(7, 700)
    B = values_wide_range(rng, 700 * 6).reshape(700, 6)
    whole = er.emulate(A, B, 7)
    monkeypatch.setattr(er, "MEMORY_PIECE", 64)
    assert np.array_equal(er.emulate(A, B, 7), whole)


def test_error_falls_with_slices():
    """Each extra 7-bit slice cuts the error by about 2^-7 until FP64 rounding
    dominates; seven slices meet the 1e-12 target on wide-range inputs."""
    rng = rng_of(4)
    A = values_wide_range(rng, 64 * 96).reshape(64, 96)
    B = values_wide_range(rng, 96 * 48).reshape(96, 48)
    ref = A @ B
    errs = [orc.rel_err(er.emulate(A, B, S), ref) for S in range(1, 8)]
    for s in range(3):
        assert errs[s + 1] < errs[s] * 2 ** -4
    assert errs[6] <= 1e-12


def test_alpha_beta():
    rng = rng_of(5)
    A = values_wide_range(rng, 20 * 300).reshape(20, 300)
    B = values_wide_range(rng, 300 * 10).reshape(300, 10)
    C = rng.uniform(-1, 1, (20, 10))
    X = er.emulate(A, B, 7, alpha=-0.5, beta=2.0, C=C)
    assert orc.rel_err(X, 2.0 * C - 0.5 * (A @ B)) <= 1e-12


def test_subnormal_rows_scale_exactly():
    """A row whose largest entry is subnormal (scale 2^e with e < -1022, so
    2^-e alone overflows): integer multiples of 2^-1074 with |n| <= 127 are
    one digit each, so the emulated product is the exact product, whose
    value is n 2^-1074 times an integer row of B (no rounding below 2^-1074
    as the integers are exact)."""
    rng = rng_of(12)
    n = rng.integers(-127, 128, size=(3, 9))
    A = np.ldexp(n.astype(np.float64), -1074)
    B = np.eye(9)[:, :4] * 1.0
    X = er.emulate(A, B, 1)
    assert np.array_equal(X, A[:, :4])
    assert np.all(np.isfinite(X))


def test_non_finite_rows_and_columns_give_nan():
    """Digits cannot hold Inf or NaN: a row of A (column of B) holding one
    makes its row (column) of the product NaN; every other element is the
    emulated product of the finite rows and columns."""
    rng = rng_of(13)
    A = rng.uniform(-1, 1, (5, 8))
    B = rng.uniform(-1, 1, (8, 4))
    A[1, 3] = np.inf
    B[6, 2] = np.nan
    X = er.emulate(A, B, 7)
    assert np.all(np.isnan(X[1, :])) and np.all(np.isnan(X[:, 2]))
    keep_r = [0, 2, 3, 4]
    keep_c = [0, 1, 3]
    ref = er.emulate(A[keep_r], B[:, keep_c], 7)
    assert np.array_equal(X[np.ix_(keep_r, keep_c)], ref)
    assert np.array_equal(er.emulate(A, B, 7, alpha=0.0), np.zeros((5, 4)))
