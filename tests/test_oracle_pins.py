"""Pins of the CPU reference against facts that do not come from itself.

Each pin is a function of the reference build (``mutant``), so the mutation
test at the end can show that planted mistakes (a transposed operand, a
dropped term, a wrong sign, a skipped index, a wrong comparison, a dropped
pattern part) each fail at least one of them.
"""
import itertools
import json
import os

import numpy as np
import pytest

from oracle import oracle as orc
from synth import BlockCSR, make_matrix, pattern_from_mask, rng_of, sparse_uniform

HERE = os.path.dirname(os.path.abspath(__file__))


def _mat(rbs, cbs, mask, data):
    rp, ci = pattern_from_mask(mask)
    return BlockCSR(np.asarray(rbs, np.int32), np.asarray(cbs, np.int32), rp, ci,
                    np.asarray(data, np.float64))


# ---------------------------------------------------------------- pins ----

def pin_dense_library(mutant=0):
    """Special case -> library routine: the block-sparse product equals the
    product of the densified matrices (numpy DGEMM), 460 x 460 in 23-blocks."""
    A, B = sparse_uniform(seed=3)
    C = orc.multiply(1.0, A, B, 0.0, mutant=mutant)
    ref = orc.to_dense(A) @ orc.to_dense(B)
    return orc.rel_err(orc.to_dense(C), ref) < 1e-13


def pin_integer_exact(mutant=0):
    """Integer-valued inputs: every partial sum is an integer below 2^53, so the
    FP64 result equals the exact int64 product bit for bit, with beta*C."""
    rng = rng_of(11)
    rbs = np.array([3, 5, 2, 7], np.int32)
    kbs = np.array([4, 1, 6], np.int32)
    cbs = np.array([2, 5, 3, 3, 1], np.int32)
    A = make_matrix(rng, rbs, kbs, 0.6, values="int")
    B = make_matrix(rng, kbs, cbs, 0.6, values="int")
    Cin = make_matrix(rng, rbs, cbs, 0.4, values="int")
    alpha, beta = 3.0, -2.0
    C = orc.multiply(alpha, A, B, beta, Cin, mutant=mutant)
    Ai = orc.to_dense(A).astype(np.int64)
    Bi = orc.to_dense(B).astype(np.int64)
    Ci = orc.to_dense(Cin).astype(np.int64)
    exact = 3 * (Ai @ Bi) - 2 * Ci
    return np.array_equal(orc.to_dense(C), exact.astype(np.float64))


def _brute_force(rbs, kbs, cbs, amask, bmask, cmask, Ad, Bd, Cd, alpha, beta):
    """Python-integer triple loop over the dense matrices and explicit sets."""
    nbr, nbk, nbc = len(rbs), len(kbs), len(cbs)
    pat = set()
    for i in range(nbr):
        for j in range(nbc):
            if cmask[i][j] or any(amask[i][k] and bmask[k][j] for k in range(nbk)):
                pat.add((i, j))
    M, K, N = sum(rbs), sum(kbs), sum(cbs)
    out = [[0] * N for _ in range(M)]
    for r in range(M):
        for c in range(N):
            s = 0
            for q in range(K):
                s += int(Ad[r][q]) * int(Bd[q][c])
            out[r][c] = alpha * s + beta * int(Cd[r][c])
    return pat, out


def pin_brute_force(mutant=0):
    """Every A/B pattern of a 2x2 block grid (plus random old C patterns),
    block sizes from {1,2,3}, checked against Python-integer brute force."""
    rng = rng_of(5)
    rbs, kbs, cbs = [2, 3], [1, 3], [3, 2]
    for abits in range(16):
        for bbits in range(16):
            amask = [[(abits >> (2 * i + k)) & 1 for k in range(2)] for i in range(2)]
            bmask = [[(bbits >> (2 * k + j)) & 1 for j in range(2)] for k in range(2)]
            cmask = [[int(rng.integers(0, 2)) for _ in range(2)] for _ in range(2)]
            A = make_matrix(rng, rbs, kbs, values="int", mask=amask)
            B = make_matrix(rng, kbs, cbs, values="int", mask=bmask)
            Cin = make_matrix(rng, rbs, cbs, values="int", mask=cmask)
            alpha, beta = 2, -1
            C = orc.multiply(alpha, A, B, beta, Cin, mutant=mutant)
            pat, out = _brute_force(rbs, kbs, cbs, amask, bmask, cmask, orc.to_dense(A),
                                    orc.to_dense(B), orc.to_dense(Cin), alpha, beta)
            got = {(i, int(C.col_ind[p])) for i in range(2)
                   for p in range(int(C.row_ptr[i]), int(C.row_ptr[i + 1]))}
            if got != pat:
                return False
            D = orc.to_dense(C)
            # Entries outside the output pattern are zero in the exact result too
            # (no product and no old block there).
            if not np.array_equal(D, np.asarray(out, dtype=np.float64)):
                return False
    return True


def pin_identity_permutation(mutant=0):
    """Closed forms: identity blocks on A's diagonal give C = B exactly;
    a block permutation of identity blocks gives the permuted B exactly."""
    rng = rng_of(7)
    sizes = np.array([4, 4, 4, 4, 4], np.int32)
    B = make_matrix(rng, sizes, sizes, 0.5)
    eye = np.eye(4).T.ravel()
    A = _mat(sizes, sizes, np.eye(5, dtype=bool), np.tile(eye, 5))
    C = orc.multiply(1.0, A, B, 0.0, mutant=mutant)
    if not np.array_equal(orc.to_dense(C), orc.to_dense(B)):
        return False
    perm = np.array([3, 0, 4, 1, 2])
    mask = np.zeros((5, 5), bool)
    mask[np.arange(5), perm] = True
    P = _mat(sizes, sizes, mask, np.tile(eye, 5))
    C = orc.multiply(1.0, P, B, 0.0, mutant=mutant)
    Bd = orc.to_dense(B)
    expect = np.concatenate([Bd[4 * p:4 * p + 4] for p in perm])
    return np.array_equal(orc.to_dense(C), expect)


def pin_all_ones(mutant=0):
    """Closed form: all-ones blocks give C_ij = sum_K [A_IK][B_KJ] * k_K."""
    rng = rng_of(9)
    rbs = np.array([2, 3, 1], np.int32)
    kbs = np.array([5, 1, 3, 2], np.int32)
    cbs = np.array([4, 2], np.int32)
    amask = rng.random((3, 4)) < 0.6
    bmask = rng.random((4, 2)) < 0.6
    A = make_matrix(rng, rbs, kbs, mask=amask, values=lambda r, n: np.ones(n))
    B = make_matrix(rng, kbs, cbs, mask=bmask, values=lambda r, n: np.ones(n))
    C = orc.multiply(1.0, A, B, 0.0, mutant=mutant)
    D = orc.to_dense(C)
    ro = np.concatenate([[0], np.cumsum(rbs)])
    co = np.concatenate([[0], np.cumsum(cbs)])
    for i in range(3):
        for j in range(2):
            v = sum(int(kbs[k]) for k in range(4) if amask[i, k] and bmask[k, j])
            if not np.all(D[ro[i]:ro[i + 1], co[j]:co[j + 1]] == v):
                return False
    return True


def pin_rank_one(mutant=0):
    """Closed form: A = u v^T, B = v w^T (full patterns) give C = (v.v) u w^T."""
    rng = rng_of(13)
    rbs = np.array([3, 6, 2], np.int32)
    kbs = np.array([5, 4], np.int32)
    cbs = np.array([2, 7], np.int32)
    u, v, w = rng.uniform(-1, 1, 11), rng.uniform(-1, 1, 9), rng.uniform(-1, 1, 9)

    def from_dense(D, rb, cb):
        ro = np.concatenate([[0], np.cumsum(rb)])
        co = np.concatenate([[0], np.cumsum(cb)])
        parts = [D[ro[i]:ro[i + 1], co[j]:co[j + 1]].T.ravel() for i in range(len(rb)) for j in range(len(cb))]
        return _mat(rb, cb, np.ones((len(rb), len(cb)), bool), np.concatenate(parts))

    A = from_dense(np.outer(u, v), rbs, kbs)
    B = from_dense(np.outer(v, w), kbs, cbs)
    C = orc.multiply(1.0, A, B, 0.0, mutant=mutant)
    return orc.rel_err(orc.to_dense(C), float(v @ v) * np.outer(u, w)) < 1e-14


def pin_scalars(mutant=0):
    """BLAS conventions: beta = 0 ignores NaN in the old C; alpha = 0 ignores NaN
    in A and B and returns beta*C over the union pattern."""
    rng = rng_of(17)
    sizes = np.array([3, 2, 4], np.int32)
    A = make_matrix(rng, sizes, sizes, 0.5)
    B = make_matrix(rng, sizes, sizes, 0.5)
    Cin = make_matrix(rng, sizes, sizes, 0.5)
    Cnan = BlockCSR(Cin.rbs, Cin.cbs, Cin.row_ptr, Cin.col_ind, np.full_like(Cin.data, np.nan))
    C0 = orc.multiply(1.5, A, B, 0.0, Cnan, mutant=mutant)
    ref = 1.5 * (orc.to_dense(A) @ orc.to_dense(B))
    if not (np.all(np.isfinite(C0.data)) and orc.rel_err(orc.to_dense(C0), ref) < 1e-14):
        return False
    Anan = BlockCSR(A.rbs, A.cbs, A.row_ptr, A.col_ind, np.full_like(A.data, np.nan))
    C1 = orc.multiply(0.0, Anan, B, 0.5, Cin, mutant=mutant)
    return np.array_equal(orc.to_dense(C1), 0.5 * orc.to_dense(Cin))


def pin_beta_accumulate(mutant=0):
    """beta != 0 adds beta times the old block, including old blocks that get
    no product (they survive with beta*C)."""
    rng = rng_of(19)
    sizes = np.array([2, 3, 2, 3], np.int32)
    A = make_matrix(rng, sizes, sizes, 0.3, values="int")
    B = make_matrix(rng, sizes, sizes, 0.3, values="int")
    Cin = make_matrix(rng, sizes, sizes, 0.5, values="int")
    C = orc.multiply(1.0, A, B, 2.0, Cin, mutant=mutant)
    exact = orc.to_dense(A).astype(np.int64) @ orc.to_dense(B).astype(np.int64) \
        + 2 * orc.to_dense(Cin).astype(np.int64)
    return np.array_equal(orc.to_dense(C), exact.astype(np.float64))


def pin_filter_boundaries(mutant=0):
    """Filter edge cases: eps = 0 keeps everything, eps = inf drops every finite
    block, a block whose squared norm equals eps^2 exactly is kept, one at a
    quarter of it is dropped."""
    sizes = np.array([2, 2], np.int32)
    mask = np.array([[1, 1], [1, 0]], bool)
    # block norms^2: 4*(0.5^2)=1, 4*(0.25^2)=0.25, 4*(1)=4
    data = np.concatenate([np.full(4, 0.5), np.full(4, 0.25), np.full(4, 1.0)])
    M = _mat(sizes, sizes, mask, data)
    if orc.apply_filter(M, 0.0, mutant).row_ptr[-1] != 3:
        return False
    if orc.apply_filter(M, np.inf, mutant).row_ptr[-1] != 0:
        return False
    F = orc.apply_filter(M, 1.0, mutant)  # eps^2 = 1: first kept (tie), second dropped
    return list(F.col_ind) == [0, 0] and list(F.row_ptr) == [0, 1, 2] and np.array_equal(
        F.data, np.concatenate([np.full(4, 0.5), np.full(4, 1.0)]))


def pin_compensated_bound(mutant=0):
    """Plain FP64 accumulation stays within 1e-14 of the Dot2 (twice-working-
    precision) result on 23-blocks: far inside the 1e-12 tolerance."""
    A, B = sparse_uniform(seed=21)
    C = orc.multiply(1.0, A, B, 0.0, mutant=mutant)
    Cc = orc.multiply(1.0, A, B, 0.0, compensated=True, mutant=mutant)
    e = orc.rel_err(orc.to_dense(C), orc.to_dense(Cc))
    return 0.0 < e < 1e-14 or e == 0.0


PINS = [pin_dense_library, pin_integer_exact, pin_brute_force, pin_identity_permutation,
        pin_all_ones, pin_rank_one, pin_scalars, pin_beta_accumulate, pin_filter_boundaries,
        pin_compensated_bound]


@pytest.mark.parametrize("pin", PINS, ids=lambda f: f.__name__)
def test_pin(pin):
    assert pin(0)


def test_sampled_rows_match_full():
    A, B = sparse_uniform(seed=1)
    full = orc.multiply(1.0, A, B, 0.0)
    part = orc.multiply(1.0, A, B, 0.0, rows=(5, 12))
    s0, s1 = int(full.row_ptr[5]), int(full.row_ptr[12])
    assert np.array_equal(part.col_ind, full.col_ind[s0:s1])
    sizes = orc.block_sizes(full.rbs, full.cbs, full.row_ptr, full.col_ind)
    e0 = int(sizes[:s0].sum())
    assert np.array_equal(part.data, full.data[e0:e0 + len(part.data)])


def test_pattern_of_row_range_matches_full():
    """The pattern restricted to a row range (with an old C, beta != 0) is
    that range of the full pattern and empty elsewhere; the multiply of the
    range agrees with the full multiply, also for the first and last rows."""
    rng = rng_of(77)
    s = np.array([5, 13, 23, 32, 5, 13, 7, 23, 32, 5, 9], np.int32)
    A = make_matrix(rng, s, s, 0.3)
    B = make_matrix(rng, s, s, 0.3)
    Cin = make_matrix(rng, s, s, 0.2)
    rp, ci = orc.pattern(A, B, Cin)
    full = orc.multiply(0.5, A, B, -1.0, Cin)
    for r0, r1 in ((0, 1), (3, 8), (10, 11), (0, 11), (4, 4)):
        prp, pci = orc.pattern(A, B, Cin, rows=(r0, r1))
        assert len(prp) == len(rp)
        assert np.array_equal(np.diff(prp)[r0:r1], np.diff(rp)[r0:r1])
        assert not np.diff(prp)[:r0].any() and not np.diff(prp)[r1:].any()
        assert np.array_equal(pci, ci[rp[r0]:rp[r1]])
        part = orc.multiply(0.5, A, B, -1.0, Cin, rows=(r0, r1))
        sizes = orc.block_sizes(full.rbs, full.cbs, full.row_ptr, full.col_ind)
        e0 = int(sizes[:int(full.row_ptr[r0])].sum())
        e1 = int(sizes[:int(full.row_ptr[r1])].sum())
        assert np.array_equal(part.col_ind, full.col_ind[full.row_ptr[r0]:full.row_ptr[r1]])
        assert np.array_equal(part.data[:e1 - e0], full.data[e0:e1])


def test_dense_library_on_dense_panels():
    """32-blocks at full occupancy (a small version of the dense workload)."""
    from synth import dense_square
    A, B = dense_square(seed=2, n=256, bs=32)
    C = orc.multiply(1.0, A, B, 0.0)
    assert orc.rel_err(orc.to_dense(C), orc.to_dense(A) @ orc.to_dense(B)) < 1e-14


def test_densified_panel_shapes_golden():
    with open(os.path.join(HERE, "golden", "densified_panels.json")) as f:
        g = json.load(f)
    for c in g["cases"]:
        a, b = orc.densified_panel_shapes(c["M"], c["N"], c["K"], c["Pt"], c["t"])
        assert list(a) == c["A"] and list(b) == c["B"]


def test_shape_mismatch_rejected():
    rng = rng_of(0)
    A = make_matrix(rng, [2, 3], [4, 5], 1.0)
    B = make_matrix(rng, [4, 6], [2], 1.0)
    with pytest.raises(ValueError):
        orc.multiply(1.0, A, B, 0.0)


@pytest.mark.parametrize("mutant", [1, 2, 3, 4, 5, 6])
def test_pins_catch_planted_mistakes(mutant):
    failed = [p.__name__ for p in PINS if not p(mutant)]
    assert failed, f"mutant {mutant} passed every pin"
