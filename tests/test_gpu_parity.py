"""Parity of the HIP path (through the C-ABI) with the CPU reference.

Tolerance: relative Frobenius error <= 1e-12 for FP64 results; bit-exact for
integer-valued inputs (every partial sum is an integer below 2^53, so any
summation order gives the exact result), for index work (patterns, stacks)
and for pure copies.
"""
import itertools

import numpy as np
import pytest

from oracle import oracle as orc
from synth import (BlockCSR, banded_uneven, dense_square, make_matrix, pattern_from_mask, rng_of,
                   sparse_uniform)

from tests.helpers import check_against_oracle, gpu_multiply, lib, set_path

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _mat(rbs, cbs, mask, data):
    rp, ci = pattern_from_mask(mask)
    return BlockCSR(np.asarray(rbs, np.int32), np.asarray(cbs, np.int32), rp, ci,
                    np.asarray(data, np.float64))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_sparse_uniform_460(seed):
    """460 x 460 in 23-blocks, 10 % occupancy, beta = 0 (stack path)."""
    A, B = sparse_uniform(seed=seed)
    R = orc.multiply(1.0, A, B, 0.0)
    X, st = gpu_multiply(1.0, A, B, 0.0)
    assert st["path"] == 1
    check_against_oracle(X, R, TOL)
    # closed form of the product count: sum_K nnz(col K of A) * nnz(row K of B)
    col_cnt = np.bincount(A.col_ind, minlength=len(A.cbs))
    row_cnt = np.diff(B.row_ptr)
    assert st["n_products"] == int((col_cnt * row_cnt).sum())


@pytest.mark.parametrize("path", ["stack", "dense"])
def test_integer_exact(path):
    rng = rng_of(31)
    rbs = np.array([3, 5, 2, 7, 1, 4], np.int32)
    kbs = np.array([4, 1, 6, 2, 9], np.int32)
    cbs = np.array([2, 5, 3, 3, 1, 8, 6], np.int32)
    A = make_matrix(rng, rbs, kbs, 0.5, values="int")
    B = make_matrix(rng, kbs, cbs, 0.5, values="int")
    Cin = make_matrix(rng, rbs, cbs, 0.3, values="int")
    for alpha, beta in [(1.0, 0.0), (3.0, -2.0), (-1.0, 1.0), (0.0, 2.0)]:
        R = orc.multiply(alpha, A, B, beta, Cin)
        X, _ = gpu_multiply(alpha, A, B, beta, Cin, path=path)
        check_against_oracle(X, R, 0.0)


@pytest.mark.parametrize("path", ["stack", "dense"])
def test_identity_and_permutation(path):
    rng = rng_of(7)
    sizes = np.array([4, 4, 4, 4, 4], np.int32)
    B = make_matrix(rng, sizes, sizes, 0.5)
    eye = np.eye(4).T.ravel()
    A = _mat(sizes, sizes, np.eye(5, dtype=bool), np.tile(eye, 5))
    X, _ = gpu_multiply(1.0, A, B, 0.0, path=path)
    assert np.array_equal(orc.to_dense(X), orc.to_dense(B))
    perm = np.array([3, 0, 4, 1, 2])
    mask = np.zeros((5, 5), bool)
    mask[np.arange(5), perm] = True
    P = _mat(sizes, sizes, mask, np.tile(eye, 5))
    X, _ = gpu_multiply(1.0, P, B, 0.0, path=path)
    Bd = orc.to_dense(B)
    assert np.array_equal(orc.to_dense(X), np.concatenate([Bd[4 * p:4 * p + 4] for p in perm]))


def test_brute_force_all_2x2_patterns():
    """Every A/B pattern of a 2x2 block grid with sizes {1,2,3}, random old C
    patterns, integer values: bit-exact against the reference."""
    rng = rng_of(5)
    rbs, kbs, cbs = [2, 3], [1, 3], [3, 2]
    for abits, bbits in itertools.product(range(16), range(16)):
        amask = [[(abits >> (2 * i + k)) & 1 for k in range(2)] for i in range(2)]
        bmask = [[(bbits >> (2 * k + j)) & 1 for j in range(2)] for k in range(2)]
        cmask = [[int(rng.integers(0, 2)) for _ in range(2)] for _ in range(2)]
        A = make_matrix(rng, rbs, kbs, values="int", mask=amask)
        B = make_matrix(rng, kbs, cbs, values="int", mask=bmask)
        Cin = make_matrix(rng, rbs, cbs, values="int", mask=cmask)
        R = orc.multiply(2.0, A, B, -1.0, Cin)
        X, st = gpu_multiply(2.0, A, B, -1.0, Cin)
        try:
            check_against_oracle(X, R, 0.0)
        except AssertionError as e:
            raise AssertionError(f"A pattern {amask}, B pattern {bmask}, C pattern {cmask}, "
                                 f"stats {st}: {e}") from None


@pytest.mark.parametrize("n,bs", [(256, 32), (299, 23), (200, 40)])
def test_dense_path_small(n, bs):
    """Dense inputs go through merge + FP64 MFMA GEMM; sizes that are not
    multiples of the 128 x 128 x 16 tile exercise the zero padding."""
    rng = rng_of(n)
    sizes = np.full(n // bs, bs, np.int32)
    A = make_matrix(rng, sizes, sizes, 1.0)
    B = make_matrix(rng, sizes, sizes, 1.0)
    Cin = make_matrix(rng, sizes, sizes, 1.0)
    for beta in (0.0, 0.5):
        R = orc.multiply(1.25, A, B, beta, Cin)
        X, st = gpu_multiply(1.25, A, B, beta, Cin)
        assert st["path"] == 2
        check_against_oracle(X, R, TOL)


@pytest.mark.parametrize("occ", [1.0, 0.6])
def test_dense_path_small_blocks(occ):
    """Blocks of fewer than 64 elements are merged 64 blocks per wave:
    uneven sizes up to 7 x 7, a ragged last chunk of blocks, and a partly
    occupied pattern (zero-filled gaps in the panels); integer entries give
    the exact result."""
    rng = rng_of(88)
    s = np.array([1, 2, 3, 5, 7], np.int32)
    rbs, kbs, cbs = (rng.choice(s, size=x) for x in (37, 101, 23))
    A = make_matrix(rng, rbs, kbs, occ, values="int")
    B = make_matrix(rng, kbs, cbs, occ, values="int")
    Cin = make_matrix(rng, rbs, cbs, 1.0, values="int")
    assert len(B.col_ind) % 64 != 0
    R = orc.multiply(2.0, A, B, -1.0, Cin)
    X, st = gpu_multiply(2.0, A, B, -1.0, Cin, path="dense")
    assert st["path"] == 2
    check_against_oracle(X, R, 0.0)


@pytest.mark.parametrize("kb", ["16", "32"])
def test_dense_tall_skinny_split_k(kb):
    """Few output tiles and a long k (the paper's tall-and-skinny shape, in
    small): the GEMM splits k across workgroups and a second kernel sums the
    partial tiles in a fixed order.  Ragged M and N, beta != 0 into an
    existing C; integer entries give the exact result, random ones the
    reference within the tolerance; repeated runs are bitwise equal."""
    b = lib()
    rng = rng_of(314)
    rbs = np.array([23, 23, 23, 23, 23, 13, 5], np.int32)      # M = 133
    cbs = np.array([32, 32, 32, 23, 13, 5, 5, 7], np.int32)    # N = 149
    kbs = np.full(600, 23, np.int32)                          # K = 13,800
    b.bsmm_set_option("dense_kb", kb)
    try:
        for values in ("int", "uniform"):
            A = make_matrix(rng, rbs, kbs, 1.0, values=values)
            B = make_matrix(rng, kbs, cbs, 1.0, values=values)
            Cin = make_matrix(rng, rbs, cbs, 1.0, values=values)
            R = orc.multiply(2.0, A, B, -1.0, Cin)
            X, st = gpu_multiply(2.0, A, B, -1.0, Cin)
            assert st["path"] == 2
            check_against_oracle(X, R, 0.0 if values == "int" else TOL)
            X2, _ = gpu_multiply(2.0, A, B, -1.0, Cin)
            assert np.array_equal(X.data, X2.data)
        # A sparse C (the dense path forced on inputs with an empty block
        # row and column): the split epilogue skips absent blocks.
        mask_a = np.ones((len(rbs), len(kbs)), bool)
        mask_a[2, :] = False
        mask_b = np.ones((len(kbs), len(cbs)), bool)
        mask_b[:, 4] = False
        A = make_matrix(rng, rbs, kbs, mask=mask_a)
        B = make_matrix(rng, kbs, cbs, mask=mask_b)
        R = orc.multiply(1.0, A, B, 0.0)
        X, st = gpu_multiply(1.0, A, B, 0.0, path="dense")
        assert st["path"] == 2 and st["c_nnzb_after"] < len(rbs) * len(cbs)
        check_against_oracle(X, R, TOL)
    finally:
        b.bsmm_set_option("dense_kb", "16")


def test_dense_rect_ragged():
    """Rectangular dense product with uneven block sizes on every side."""
    rng = rng_of(77)
    rbs = rng.integers(1, 40, size=7).astype(np.int32)
    kbs = rng.integers(1, 40, size=29).astype(np.int32)
    cbs = rng.integers(1, 40, size=5).astype(np.int32)
    A = make_matrix(rng, rbs, kbs, 1.0)
    B = make_matrix(rng, kbs, cbs, 1.0)
    R = orc.multiply(1.0, A, B, 0.0)
    X, st = gpu_multiply(1.0, A, B, 0.0)
    assert st["path"] == 2
    check_against_oracle(X, R, TOL)


@pytest.mark.parametrize("path", ["stack", "dense"])
def test_forced_paths_agree(path):
    """The stack path on dense inputs and the dense path on sparse inputs
    both reach the reference result (same pattern, same values)."""
    for A, B in [dense_square(seed=4, n=192, bs=32), sparse_uniform(seed=4)]:
        R = orc.multiply(1.0, A, B, 0.0)
        X, st = gpu_multiply(1.0, A, B, 0.0, path=path)
        assert st["path"] == (1 if path == "stack" else 2)
        check_against_oracle(X, R, TOL)


@pytest.mark.parametrize("occ", [0.01, 0.10, 0.30])
def test_uneven_banded_with_filter(occ):
    """Block sizes drawn from {5,13,23,32}, banded magnitudes, filter 1e-10."""
    A, B = banded_uneven(seed=3, occupancy=occ, target=1500)
    for eps in (0.0, 1e-10, 1e-3):
        R = orc.multiply(1.0, A, B, 0.0, filter_eps=eps)
        X, st = gpu_multiply(1.0, A, B, 0.0, eps=eps)
        check_against_oracle(X, R, TOL)


def test_large_blocks_chunked_k():
    """Blocks with k far above what one LDS region holds and C blocks wider
    than one wavefront's tiles (chunking over k, passes over tiles)."""
    rng = rng_of(12)
    rbs = np.array([70, 129], np.int32)
    kbs = np.array([300, 17, 257], np.int32)
    cbs = np.array([90, 3], np.int32)
    A = make_matrix(rng, rbs, kbs, 1.0)
    B = make_matrix(rng, kbs, cbs, 0.7)
    R = orc.multiply(1.0, A, B, 0.0)
    X, st = gpu_multiply(1.0, A, B, 0.0, path="stack")
    check_against_oracle(X, R, TOL)


def test_beta_with_pattern_growth():
    """Old C blocks move to the grown pattern and are scaled by beta, also
    those that receive no product."""
    rng = rng_of(41)
    sizes = np.array([3, 6, 2, 5], np.int32)
    A = make_matrix(rng, sizes, sizes, 0.3)
    B = make_matrix(rng, sizes, sizes, 0.3)
    Cin = make_matrix(rng, sizes, sizes, 0.6)
    for beta in (0.0, 1.0, -0.75):
        R = orc.multiply(0.5, A, B, beta, Cin)
        X, _ = gpu_multiply(0.5, A, B, beta, Cin)
        check_against_oracle(X, R, TOL)


def test_nan_semantics():
    """beta = 0 ignores NaN in the old C; alpha = 0 ignores NaN in A and B."""
    rng = rng_of(17)
    sizes = np.array([3, 2, 4], np.int32)
    A = make_matrix(rng, sizes, sizes, 0.5)
    B = make_matrix(rng, sizes, sizes, 0.5)
    Cin = make_matrix(rng, sizes, sizes, 0.5)
    Cnan = BlockCSR(Cin.rbs, Cin.cbs, Cin.row_ptr, Cin.col_ind, np.full_like(Cin.data, np.nan))
    X, _ = gpu_multiply(1.5, A, B, 0.0, Cnan)
    check_against_oracle(X, orc.multiply(1.5, A, B, 0.0, Cnan), TOL)
    Anan = BlockCSR(A.rbs, A.cbs, A.row_ptr, A.col_ind, np.full_like(A.data, np.nan))
    X, _ = gpu_multiply(0.0, Anan, B, 0.5, Cin)
    check_against_oracle(X, orc.multiply(0.0, Anan, B, 0.5, Cin), 0.0)


def test_filter_boundaries():
    sizes = np.array([2, 2], np.int32)
    eye = np.eye(2).T.ravel()
    A = _mat(sizes, sizes, np.eye(2, dtype=bool), np.tile(eye, 2))
    mask = np.array([[1, 1], [1, 0]], bool)
    Bdata = np.concatenate([np.full(4, 0.5), np.full(4, 0.25), np.full(4, 1.0)])
    B = _mat(sizes, sizes, mask, Bdata)
    for eps in (0.0, 1.0, np.inf, 0.6):
        R = orc.multiply(1.0, A, B, 0.0, filter_eps=eps)
        X, st = gpu_multiply(1.0, A, B, 0.0, eps=eps)
        check_against_oracle(X, R, 0.0)


def test_empty_and_degenerate():
    rng = rng_of(3)
    sizes = np.array([4, 5], np.int32)
    Z = make_matrix(rng, sizes, sizes, nnzb=0)
    B = make_matrix(rng, sizes, sizes, 1.0)
    X, st = gpu_multiply(1.0, Z, B, 0.0)
    assert int(X.row_ptr[-1]) == 0
    Cin = make_matrix(rng, sizes, sizes, 0.5)
    X, _ = gpu_multiply(1.0, Z, B, 2.0, Cin)
    check_against_oracle(X, orc.multiply(1.0, Z, B, 2.0, Cin), 0.0)
    # no block rows at all
    E = BlockCSR(np.zeros(0, np.int32), sizes, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0))
    X, _ = gpu_multiply(1.0, E, B, 0.0)
    assert len(X.row_ptr) == 1


def _tall_skinny_sparse(seed):
    """3 block rows of A against 700 block columns (half occupied) and B with
    4 block columns: few C rows, long A rows, so the stack builder splits
    every A row over several workgroups."""
    rng = rng_of(seed)
    ms = np.array([5, 13, 5], np.int32)
    ks = rng.choice(np.array([5, 13, 23], np.int32), size=700)
    ns = np.array([13, 5, 23, 5], np.int32)
    return make_matrix(rng, ms, ks, 0.5), make_matrix(rng, ks, ns, 0.5)


def _wide_c(seed, nbr, nbk, occ_a, occ_b, nbc=9000):
    """C with more block columns (9000, sizes 1-3) than the stack builder's
    LDS column map holds (8192): the count and fill phases search C's rows
    in global memory instead."""
    rng = rng_of(seed)
    sizes = np.array([1, 2, 3], np.int32)
    ms, ks, ns = (rng.choice(sizes, size=x) for x in (nbr, nbk, nbc))
    return make_matrix(rng, ms, ks, occ_a), make_matrix(rng, ks, ns, occ_b)


@pytest.mark.parametrize("workload", ["banded", "tall_skinny", "wide", "wide_tall_skinny"])
def test_stack_contents_exact(workload):
    """The stacks hold exactly the (I,K,J) products of the block patterns,
    runs ordered by class then C block, K ascending inside a run (also when
    long A rows are counted and filled in parts by several workgroups, and
    when C has more block columns than the LDS column map holds)."""
    b = lib()
    if workload == "banded":
        A, B = banded_uneven(seed=9, occupancy=0.1, target=600)
    elif workload == "tall_skinny":
        A, B = _tall_skinny_sparse(seed=19)
    elif workload == "wide":
        A, B = _wide_c(seed=23, nbr=40, nbk=300, occ_a=0.1, occ_b=0.02)
    else:
        A, B = _wide_c(seed=29, nbr=3, nbk=700, occ_a=0.5, occ_b=0.01, nbc=8500)
    R = orc.multiply(1.0, A, B, 0.0)
    MA, MB = b.Matrix.from_blocks(A), b.Matrix.from_blocks(B)
    MC = b.Matrix.from_blocks(R)
    s = b.bsmm_inspect_stacks(MA.handle, MB.handle, MC.handle)
    # enumerate the expected products by brute force over the patterns
    a_rows = np.repeat(np.arange(len(A.rbs)), np.diff(A.row_ptr))
    b_rows = np.repeat(np.arange(len(B.rbs)), np.diff(B.row_ptr))
    c_index = {(int(i), int(j)): p for p, (i, j) in enumerate(
        zip(np.repeat(np.arange(len(R.rbs)), np.diff(R.row_ptr)), R.col_ind))}
    expect = set()
    for pa in range(len(A.col_ind)):
        k = int(A.col_ind[pa])
        for pb in range(int(B.row_ptr[k]), int(B.row_ptr[k + 1])):
            expect.add((c_index[(int(a_rows[pa]), int(B.col_ind[pb]))], pa, pb))
    got = set()
    rp = s["run_ptr"]
    for r in range(len(s["run_cblk"])):
        ks = []
        for q in range(int(rp[r]), int(rp[r + 1])):
            got.add((int(s["run_cblk"][r]), int(s["prod_ablk"][q]), int(s["prod_bblk"][q])))
            ks.append(int(A.col_ind[s["prod_ablk"][q]]))
        assert ks == sorted(ks) and len(set(ks)) == len(ks)
    assert got == expect
    assert len(got) == len(s["prod_ablk"])
    key = list(zip(s["run_class"].tolist(), s["run_cblk"].tolist()))
    assert key == sorted(key)
    for M in (MA, MB, MC):
        M.close()


def test_tall_skinny_parts_match_reference():
    """The split count and fill of long A rows: plain and tuned stacks reach
    the reference result; integer entries exactly."""
    for kernel in ("plain", "tuned"):
        rng = rng_of(23)
        ms = np.array([5, 13, 5], np.int32)
        ks = rng.choice(np.array([5, 13, 23], np.int32), size=700)
        ns = np.array([13, 5, 23, 5], np.int32)
        A = make_matrix(rng, ms, ks, 0.5, values="int")
        B = make_matrix(rng, ks, ns, 0.5, values="int")
        Cin = make_matrix(rng, ms, ns, 0.5, values="int")
        X, st = gpu_multiply(1.0, A, B, 3.0, Cin, path="stack", kernel=kernel)
        check_against_oracle(X, orc.multiply(1.0, A, B, 3.0, Cin), 0.0)


def test_stack_chunk_bitwise():
    """The batch cap (products per launch) never changes the result."""
    A, B = banded_uneven(seed=5, occupancy=0.1, target=800)
    ref, _ = gpu_multiply(1.0, A, B, 0.0)
    for chunk in (1, 7, 30000):
        X, _ = gpu_multiply(1.0, A, B, 0.0, chunk=chunk)
        assert np.array_equal(X.data, ref.data)


@pytest.mark.parametrize("kernel", ["plain", "tuned"])
@pytest.mark.parametrize("panel", [1, 397, 1500])
def test_stack_row_panels(kernel, panel):
    """Stacks built and run over panels of C block rows (a cap on the
    products held at once) give the same bits as whole stacks: every C
    block is updated by one run in one panel, in the same product order.
    A cap of 1 puts every block row in a panel of its own; beta != 0 into an
    existing C and the filter run after the last panel."""
    b = lib()
    A, B = banded_uneven(seed=41, occupancy=0.15, target=1100)
    assert int(np.diff(np.asarray(B.row_ptr))[np.asarray(A.col_ind)].sum()) > 2 * 1500
    rng = rng_of(42)
    Cin = make_matrix(rng, A.rbs, B.cbs, 0.2)
    ref, st0 = gpu_multiply(0.75, A, B, -0.5, Cin, eps=1e-3, kernel=kernel)
    assert st0["n_row_panels"] == 1
    b.bsmm_set_option("stack_panel", str(panel))
    try:
        X, st = gpu_multiply(0.75, A, B, -0.5, Cin, eps=1e-3, kernel=kernel)
    finally:
        b.bsmm_set_option("stack_panel", "1073741824")
    assert st["n_products"] == st0["n_products"] and st["n_runs"] == st0["n_runs"]
    assert st["n_classes"] == st0["n_classes"]
    brp, arp = np.asarray(B.row_ptr), np.asarray(A.row_ptr)
    busy = sum(any(brp[k + 1] > brp[k] for k in np.asarray(A.col_ind)[arp[i]:arp[i + 1]])
               for i in range(len(A.rbs)))
    if panel == 1:
        assert st["n_row_panels"] == busy
    else:
        assert st["n_row_panels"] >= -(-st0["n_products"] // panel) > 1
    check_against_oracle(X, ref, 0.0)
    R = orc.multiply(0.75, A, B, -0.5, Cin, filter_eps=1e-3)
    check_against_oracle(X, R, TOL)


def test_stack_row_panels_no_plan_reuse():
    """A multiply built in row panels keeps no plan: with the plan cache on,
    repeated multiplies into one C still give beta*C + alpha*A*B."""
    b = lib()
    A, B = banded_uneven(seed=43, occupancy=0.2, target=700)
    nprod = int(np.diff(np.asarray(B.row_ptr))[np.asarray(A.col_ind)].sum())
    assert nprod > 1000
    b.bsmm_set_option("stack_panel", str(nprod // 5))
    b.bsmm_set_option("plan_cache", "1")
    set_path("stack", "tuned")
    try:
        MA, MB = b.Matrix.from_blocks(A), b.Matrix.from_blocks(B)
        MC = b.Matrix.empty(A.rbs, B.cbs)
        for beta in (0.0, 0.5, 0.5):
            b.multiply(1.0, MA, MB, beta, MC)
            assert b.bsmm_last_stats()["n_row_panels"] > 1
        X = MC.to_host()
        for M in (MA, MB, MC):
            M.close()
    finally:
        b.bsmm_set_option("stack_panel", "1073741824")
        b.bsmm_set_option("plan_cache", "0")
        set_path()
    check_against_oracle(X, orc.multiply(1.75, A, B, 0.0), TOL)


def test_stack_row_panels_split_rows_bitwise():
    """Row panels of few block rows each split long A rows into parts (more
    workgroups per panel): 300 block rows of about 160 A blocks, panels of
    about 10 rows, so each row is counted and filled in 2 parts, where the
    whole stacks take 1.  Parts are contiguous K ranges placed in order, so
    the runs keep their K order and the bits equal those of whole stacks."""
    b = lib()
    rng = rng_of(44)
    s = np.array([1, 2, 3, 5], np.int32)
    ms, ks, ns = (rng.choice(s, size=x) for x in (300, 400, 200))
    A = make_matrix(rng, ms, ks, 0.4, values="int")
    B = make_matrix(rng, ks, ns, 0.05, values="int")
    assert len(A.col_ind) // 300 >= 128
    X1, st1 = gpu_multiply(1.0, A, B, 0.0, path="stack", kernel="plain")
    assert st1["n_row_panels"] == 1
    b.bsmm_set_option("stack_panel", str(st1["n_products"] // 30))
    try:
        X2, st2 = gpu_multiply(1.0, A, B, 0.0, path="stack", kernel="plain")
    finally:
        b.bsmm_set_option("stack_panel", "1073741824")
    assert st2["n_row_panels"] >= 30
    check_against_oracle(X2, X1, 0.0)
    check_against_oracle(X2, orc.multiply(1.0, A, B, 0.0), 0.0)


def test_run_to_run_deterministic():
    A, B = banded_uneven(seed=6, occupancy=0.3, target=800)
    X1, _ = gpu_multiply(1.0, A, B, 0.0)
    X2, _ = gpu_multiply(1.0, A, B, 0.0, repeat=2)
    assert np.array_equal(X1.data, X2.data)


def test_repeated_multiply_reuses_pattern():
    """Second multiply into the same C (pattern unchanged): beta*C + alpha*AB."""
    A, B = sparse_uniform(seed=8)
    b = lib()
    set_path()
    MA, MB = b.Matrix.from_blocks(A), b.Matrix.from_blocks(B)
    MC = b.Matrix.empty(A.rbs, B.cbs)
    b.multiply(1.0, MA, MB, 0.0, MC)
    b.multiply(1.0, MA, MB, 1.0, MC)
    X = MC.to_host()
    R = orc.multiply(2.0, A, B, 0.0)
    check_against_oracle(X, R, TOL)
    for M in (MA, MB, MC):
        M.close()


def test_torch_allocator_and_stream():
    torch = pytest.importorskip("torch")
    b = lib()
    b.use_torch_allocator()
    try:
        A, B = sparse_uniform(seed=2)
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            X, _ = gpu_multiply(1.0, A, B, 0.0)
        check_against_oracle(X, orc.multiply(1.0, A, B, 0.0), TOL)
    finally:
        b.bsmm_set_allocator()


def test_device_resident_input():
    torch = pytest.importorskip("torch")
    b = lib()
    A, B = sparse_uniform(seed=11)
    dA = torch.from_numpy(A.data).cuda()
    MA = b.Matrix.from_blocks(A, data=dA)
    MB = b.Matrix.from_blocks(B)
    MC = b.Matrix.empty(A.rbs, B.cbs)
    b.multiply(1.0, MA, MB, 0.0, MC)
    out = torch.empty(MC.info()[3], dtype=torch.float64, device="cuda")
    rp, ci, _ = b.bsmm_copy_out(MC.handle, device_out=out)
    R = orc.multiply(1.0, A, B, 0.0)
    assert np.array_equal(rp, R.row_ptr) and np.array_equal(ci, R.col_ind)
    assert orc.rel_err(out.cpu().numpy(), R.data) <= TOL
    for M in (MA, MB, MC):
        M.close()


def test_full_size_dense_square_sampled():
    """N = 8192 in 32-blocks, every block stored (the dense workload), in the
    benchmark's launch configuration; two sampled block rows checked against
    the reference computed row by row."""
    A, B = dense_square(seed=0, n=8192, bs=32)
    X, st = gpu_multiply(1.0, A, B, 0.0)
    assert st["path"] == 2 and st["flops"] == 2.0 * 8192 ** 3
    sizes = orc.block_sizes(X.rbs, X.cbs, X.row_ptr, X.col_ind)
    for r0 in (0, 201):
        R = orc.multiply(1.0, A, B, 0.0, rows=(r0, r0 + 1))
        s0, s1 = int(X.row_ptr[r0]), int(X.row_ptr[r0 + 1])
        e0 = int(sizes[:s0].sum())
        e1 = e0 + int(sizes[s0:s1].sum())
        assert np.array_equal(X.col_ind[s0:s1], R.col_ind)
        assert orc.rel_err(X.data[e0:e1], R.data) <= TOL


@pytest.mark.parametrize("n,bs", [(256, 32), (299, 23)])
def test_dense_k_step_32(n, bs):
    """The 32-deep k-step variant of the dense GEMM (zero-padded K)."""
    b = lib()
    rng = rng_of(n + 1)
    sizes = np.full(n // bs, bs, np.int32)
    A = make_matrix(rng, sizes, sizes, 1.0)
    B = make_matrix(rng, sizes, sizes, 1.0)
    Cin = make_matrix(rng, sizes, sizes, 1.0)
    b.bsmm_set_option("dense_kb", "32")
    try:
        X, st = gpu_multiply(0.75, A, B, -0.5, Cin)
    finally:
        b.bsmm_set_option("dense_kb", "16")
    assert st["path"] == 2
    check_against_oracle(X, orc.multiply(0.75, A, B, -0.5, Cin), TOL)
