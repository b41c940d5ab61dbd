"""Pins of the emulation reference against exact arithmetic."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import emul_ref as er
from oracle import oracle as orc
from synth import rng_of, values_wide_range


def _exact_product(A, B):
    M, K = A.shape
    N = B.shape[1]
    Af = [[Fraction(float(x)) for x in row] for row in A]
    Bf = [[Fraction(float(x)) for x in row] for row in B]
    return [[sum(Af[i][k] * Bf[k][j] for k in range(K)) for j in range(N)] for i in range(M)]


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
    dropped = sum(Fraction(2 * S + 1 - d) * K * 127 * 127 / Fraction(2) ** (7 * d)
                  for d in range(S + 2, 2 * S + 1))
    absprod = np.abs(A) @ np.abs(B)
    for i in range(6):
        for j in range(5):
            bound = dropped * Fraction(2) ** int(ea[i] + eb[j]) + Fraction(float(absprod[i, j])) / 2 ** 49
            assert abs(Fraction(float(X[i, j])) - E[i][j]) <= bound


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


def test_alpha_beta_and_chunking():
    rng = rng_of(5)
    A = values_wide_range(rng, 20 * 300).reshape(20, 300)
    B = values_wide_range(rng, 300 * 10).reshape(300, 10)
    C = rng.uniform(-1, 1, (20, 10))
    X = er.emulate(A, B, 7, alpha=-0.5, beta=2.0, C=C, kchunk=128)
    assert orc.rel_err(X, 2.0 * C - 0.5 * (A @ B)) <= 1e-12
    assert er.int32_chunk(7) * 127 * 127 * 7 < 2 ** 31
