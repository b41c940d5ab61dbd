"""Norm-bound screen of the symbolic phase (option "prescreen"): C blocks
whose bound |alpha| sum_K ||A_IK|| ||B_KJ|| + |beta| ||C_IJ|| lies below the
filter threshold are left out of the pattern and their products skipped.
Those blocks always fail the filter, so the result must be the same bits as
without the screen, and the reference's within tolerance; non-finite
inputs, thresholds the screen leaves alone, FP32 data and the plan cache
are covered."""
import numpy as np
import pytest

from oracle import oracle as orc
from synth import BlockCSR, banded_uneven, make_matrix, pattern_from_mask, rng_of

from tests.helpers import check_against_oracle, gpu_multiply, lib

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _both(alpha, A, B, beta=0.0, Cin=None, eps=1e-10, kernel="tuned"):
    """The multiply with the screen on and off: (result, stats) of each."""
    b = lib()
    try:
        b.bsmm_set_option("prescreen", "1")
        X1, st1 = gpu_multiply(alpha, A, B, beta, Cin, eps=eps, path="stack", kernel=kernel)
        b.bsmm_set_option("prescreen", "0")
        X0, st0 = gpu_multiply(alpha, A, B, beta, Cin, eps=eps, path="stack", kernel=kernel)
    finally:
        b.bsmm_set_option("prescreen", "1")
    return (X1, st1), (X0, st0)


def _steep(seed, occ=0.3, target=3000):
    # Decay of 3 block rows: products reach C blocks 160 rows off the
    # diagonal whose bound is far below 1e-10.
    return banded_uneven(seed=seed, occupancy=occ, target=target, decay=3.0)


@pytest.mark.parametrize("kernel", ["plain", "tuned"])
def test_screen_same_bits(kernel):
    A, B = _steep(71)
    (X1, st1), (X0, st0) = _both(-1.5, A, B, kernel=kernel)
    assert st0["n_screened"] == 0 and st0["n_products_run"] == st0["n_products"]
    assert st1["n_screened"] > 0 and st1["n_products_run"] < st1["n_products"] == st0["n_products"]
    assert st1["c_nnzb_before"] == st0["c_nnzb_before"] - st1["n_screened"]
    check_against_oracle(X1, X0, 0.0)
    check_against_oracle(X1, orc.multiply(-1.5, A, B, 0.0, filter_eps=1e-10), TOL)


def test_screen_with_old_blocks():
    """beta != 0: old C blocks far from the diagonal, most of them tiny
    (screened: the new pattern loses them) and some large (kept by their
    own norm although no product reaches them above the threshold)."""
    A, B = _steep(72)
    rng = rng_of(73)
    n = len(A.rbs)
    I, J = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    mask = (np.abs(I - J) > 120) & (rng.random((n, n)) < 0.3)
    rp, ci = pattern_from_mask(mask)
    sizes = np.asarray(A.rbs, np.int64)[np.repeat(np.arange(n), np.diff(rp))] * np.asarray(B.cbs, np.int64)[ci]
    scale = np.where(rng.random(len(ci)) < 0.1, 1.0, 1e-30)
    data = rng.uniform(-1, 1, int(sizes.sum())) * np.repeat(scale, sizes)
    Cin = BlockCSR(A.rbs, B.cbs, rp, ci.astype(np.int32), data)
    (X1, st1), (X0, st0) = _both(0.5, A, B, 0.25, Cin)
    assert st1["n_screened"] > 0
    check_against_oracle(X1, X0, 0.0)
    check_against_oracle(X1, orc.multiply(0.5, A, B, 0.25, Cin, filter_eps=1e-10), TOL)


def test_screen_keeps_non_finite():
    """NaN and infinity in far A blocks: every C block they reach has a
    non-finite bound and stays; the results agree bit for bit (NaN where
    NaN)."""
    A, B = _steep(74)
    ap = np.asarray(A.row_ptr)
    rows = np.repeat(np.arange(len(A.rbs)), np.diff(ap))
    far = np.nonzero(np.abs(rows - np.asarray(A.col_ind)) > 60)[0]
    sizes = orc.block_sizes(A.rbs, A.cbs, A.row_ptr, A.col_ind)
    start = np.concatenate([[0], np.cumsum(sizes)])
    data = np.array(A.data)
    data[start[far[0]]] = np.nan
    data[start[far[-1]] + 1] = np.inf
    A = BlockCSR(A.rbs, A.cbs, A.row_ptr, A.col_ind, data)
    (X1, st1), (X0, _) = _both(1.0, A, B)
    assert st1["n_screened"] > 0
    check_against_oracle(X1, X0, 0.0)


def test_screen_extreme_magnitudes():
    """A blocks scaled to 1e-200, 1e-280 and 1e200: block norms outside
    [2^-500, 2^500] take the scaled second pass or the sqrt(len) max bound,
    and bounds of 1e150 and above keep their blocks; same bits as without
    the screen."""
    A, B = _steep(78)
    sizes = orc.block_sizes(A.rbs, A.cbs, A.row_ptr, A.col_ind)
    rng = rng_of(79)
    scale = rng.choice([1.0, 1e-200, 1e-280, 1e200], len(sizes), p=[0.7, 0.1, 0.1, 0.1])
    A = BlockCSR(A.rbs, A.cbs, A.row_ptr, A.col_ind, np.asarray(A.data) * np.repeat(scale, sizes))
    (X1, st1), (X0, _) = _both(1.0, A, B)
    assert st1["n_screened"] > 0
    check_against_oracle(X1, X0, 0.0)


@pytest.mark.parametrize("eps,screens", [(np.inf, True), (1e-200, False), (0.0, False)])
def test_screen_thresholds(eps, screens):
    """eps = inf drops every finite block either way; thresholds below
    1e-150 (and 0, no filter) leave the screen off."""
    A, B = _steep(75, target=2000)
    (X1, st1), (X0, _) = _both(1.0, A, B, eps=eps)
    assert (st1["n_screened"] > 0) == screens
    check_against_oracle(X1, X0, 0.0)


def test_screen_fp32():
    """FP32 block data: the margin grows with the FP32 rounding of the sums;
    same bits as without the screen."""
    from tests.test_gpu_f32 import _as_f32, _f32_multiply
    A, B = _steep(76, target=2500)
    A, B = _as_f32(A), _as_f32(B)
    b = lib()
    try:
        b.bsmm_set_option("prescreen", "1")
        X1, st1 = _f32_multiply(1.0, A, B, 0.0, eps=1e-6, path="stack", kernel="tuned")
        b.bsmm_set_option("prescreen", "0")
        X0, st0 = _f32_multiply(1.0, A, B, 0.0, eps=1e-6, path="stack", kernel="tuned")
    finally:
        b.bsmm_set_option("prescreen", "1")
    assert st1["n_screened"] > 0 and st0["n_screened"] == 0
    check_against_oracle(X1, X0, 0.0)


def _two_clusters(seed, nb=40, bs=4):
    """A and B full inside two diagonal clusters of block rows, with tiny
    (1e-30) bridge blocks between the clusters: the C blocks across the
    clusters have bounds near 1e-30, every other C block a norm near 1."""
    rng = rng_of(seed)
    sizes = np.full(nb, bs, np.int32)
    h = nb // 2
    I, K = np.meshgrid(np.arange(nb), np.arange(nb), indexing="ij")
    same = (I < h) == (K < h)
    out = []
    for _ in range(2):
        mask = same | (rng.random((nb, nb)) < 0.1)
        rp, ci = pattern_from_mask(mask)
        rows = np.repeat(np.arange(nb), np.diff(rp))
        scale = np.where(same[rows, ci], 1.0, 1e-30)
        data = rng.uniform(-1, 1, len(ci) * bs * bs) * np.repeat(scale, bs * bs)
        out.append(BlockCSR(sizes, sizes, rp, ci.astype(np.int32), data))
    return out


def test_screen_plan_cache_threshold():
    """A plan whose pattern the screen chose is replayed only for the same
    threshold: after two multiplies at 1e-10 (the second a replay), one at
    1e-40 must form the cross-cluster blocks again."""
    A, B = _two_clusters(77)
    b = lib()
    b.bsmm_set_option("plan_cache", "1")
    b.bsmm_set_option("path", "stack")
    b.bsmm_set_option("stack_kernel", "tuned")
    try:
        MA, MB = b.Matrix.from_blocks(A), b.Matrix.from_blocks(B)
        MC = b.Matrix.empty(A.rbs, B.cbs)
        b.multiply(1.0, MA, MB, 0.0, MC, 1e-10)
        st1 = b.bsmm_last_stats()
        assert st1["n_screened"] > 0 and st1["c_nnzb_after"] == st1["c_nnzb_before"]
        b.multiply(1.0, MA, MB, 0.0, MC, 1e-10)
        st2 = b.bsmm_last_stats()
        assert st2["n_screened"] == st1["n_screened"]
        check_against_oracle(MC.to_host(), orc.multiply(1.0, A, B, 0.0, filter_eps=1e-10), TOL)
        b.multiply(1.0, MA, MB, 0.0, MC, 1e-40)
        st3 = b.bsmm_last_stats()
        assert st3["n_screened"] == 0
        X = MC.to_host()
        for M in (MA, MB, MC):
            M.close()
    finally:
        b.bsmm_set_option("plan_cache", "0")
        b.bsmm_set_option("path", "auto")
        b.bsmm_set_option("stack_kernel", "plain")
    R = orc.multiply(1.0, A, B, 0.0, filter_eps=1e-40)
    assert len(R.col_ind) > len(orc.multiply(1.0, A, B, 0.0, filter_eps=1e-10).col_ind)
    check_against_oracle(X, R, TOL)


def _with_options(opts, fn):
    b = lib()
    saved = {k: b.bsmm_get_option(k) for k in opts}
    try:
        for k, v in opts.items():
            b.bsmm_set_option(k, v)
        return fn()
    finally:
        for k, v in saved.items():
            b.bsmm_set_option(k, v)


@pytest.mark.parametrize("kernel", ["plain", "tuned"])
def test_screen_row_panels(kernel):
    """Stacks built in row panels over a screened pattern: the panel split
    counts only the products run; same bits as whole, unscreened stacks."""
    A, B = _steep(80, target=2500)
    (X0, st0), _ = _both(1.0, A, B, kernel=kernel)
    (X1, st1), (X2, _) = _with_options({"stack_panel": "2000"}, lambda: _both(1.0, A, B, kernel=kernel))
    assert st1["n_row_panels"] > 1 and st1["n_screened"] == st0["n_screened"] > 0
    assert st1["n_products_run"] == st0["n_products_run"]
    check_against_oracle(X1, X0, 0.0)
    check_against_oracle(X2, X0, 0.0)


def test_screen_split_long_rows():
    """Few C block rows with long A rows (count and fill split every A row
    into parts) and magnitudes 10^-i / 10^-j per block row / column, so that
    the blocks far from the corner are screened; integer-scaled values keep
    the comparison exact against the unscreened multiply."""
    rng = rng_of(81)
    ms = np.full(12, 4, np.int32)
    ks = rng.choice(np.array([4, 5, 7], np.int32), 1500)
    ns = np.full(12, 4, np.int32)
    A = make_matrix(rng, ms, ks, 0.6)
    B = make_matrix(rng, ks, ns, 0.6)
    ra = np.repeat(np.arange(len(ms)), np.diff(np.asarray(A.row_ptr)))
    A.data = np.asarray(A.data) * np.repeat(10.0 ** (-2.0 * ra), orc.block_sizes(A.rbs, A.cbs, A.row_ptr, A.col_ind))
    cb = np.asarray(B.col_ind)
    B.data = np.asarray(B.data) * np.repeat(10.0 ** (-2.0 * cb), orc.block_sizes(B.rbs, B.cbs, B.row_ptr, B.col_ind))
    for kernel in ("plain", "tuned"):
        (X1, st1), (X0, _) = _both(1.0, A, B, kernel=kernel)
        assert st1["n_screened"] > 0
        check_against_oracle(X1, X0, 0.0)
        check_against_oracle(X1, orc.multiply(1.0, A, B, 0.0, filter_eps=1e-10), TOL)


def test_screen_jit_classes():
    """One product depth (every A block column 13 wide): the classes run on
    kernels compiled at run time, over a screened pattern."""
    A, B = banded_uneven(seed=82, occupancy=0.3, target=2600, decay=3.0, choices=(13,))
    (X1, st1), (X0, _) = _with_options({"jit": "1", "stack_params": "16 16 0 4"},
                                       lambda: _both(1.0, A, B, kernel="tuned"))
    assert st1["n_screened"] > 0 and st1["n_jit_classes"] > 0
    check_against_oracle(X1, X0, 0.0)
    check_against_oracle(X1, orc.multiply(1.0, A, B, 0.0, filter_eps=1e-10), TOL)


def test_screen_plain_with_beta():
    A, B = _steep(83, target=2000)
    Cin = make_matrix(rng_of(84), A.rbs, B.cbs, 0.2)
    (X1, st1), (X0, _) = _both(2.0, A, B, -0.5, Cin, kernel="plain")
    assert st1["n_screened"] > 0
    check_against_oracle(X1, X0, 0.0)
    check_against_oracle(X1, orc.multiply(2.0, A, B, -0.5, Cin, filter_eps=1e-10), TOL)
