"""Matrices with more blocks than one launch has waves: N = 16384 in blocks
of 2 (67,108,864 blocks per operand, four times the 2^22 - 1 workgroups of
four waves a launch may have).  The merge, block-offset, scaling, norm and
compaction kernels stride over their blocks by the grid, so every block is
reached; checked on sampled block rows against the CPU reference."""
import numpy as np
import pytest

from oracle import oracle as orc
from synth import BlockCSR, pattern_full, rng_of, values_uniform

from tests.helpers import gpu_multiply, lib

pytestmark = pytest.mark.gpu
TOL = 1e-12
N, BS = 16384, 2


def _operands():
    rng = rng_of(61)
    sizes = np.full(N // BS, BS, np.int32)
    A = BlockCSR(sizes, sizes, *pattern_full(len(sizes), len(sizes)), values_uniform(rng, N * N))
    B = BlockCSR(sizes, sizes, *pattern_full(len(sizes), len(sizes)), values_uniform(rng, N * N))
    return A, B


def _eps_for_rows(A, B, rows):
    """A threshold inside a wide relative gap of the sampled rows' squared
    block norms (so that summation order cannot flip a decision there)."""
    s = np.sort(np.concatenate([orc.block_sumsq(orc.multiply(1.0, A, B, 0.0, rows=(r, r + 1)))
                                for r in rows]))
    lo, hi = len(s) * 2 // 5, len(s) * 3 // 5
    gaps = s[lo + 1:hi + 1] / np.maximum(s[lo:hi], 1e-300)
    i = lo + int(np.argmax(gaps))
    assert s[i + 1] > s[i] * (1 + 1e-9)
    return float(np.sqrt(np.sqrt(s[i] * s[i + 1])))


@pytest.mark.parametrize("path", ["dense", "emul"])
def test_more_blocks_than_grid_waves(path):
    A, B = _operands()
    rows = [0, 4095, N // BS - 1]
    eps = _eps_for_rows(A, B, rows)
    b = lib()
    if path == "emul":
        b.bsmm_set_option("emul_slices", "7")
    X, st = gpu_multiply(1.0, A, B, 0.0, eps=eps, path=path)
    assert st["c_nnzb_before"] == (N // BS) ** 2 > 4 * ((1 << 22) - 1)
    assert 0 < st["c_nnzb_after"] < st["c_nnzb_before"]
    sizes = orc.block_sizes(X.rbs, X.cbs, X.row_ptr, X.col_ind)
    start = np.concatenate([[0], np.cumsum(sizes)])
    for r0 in rows:
        R = orc.multiply(1.0, A, B, 0.0, filter_eps=eps, rows=(r0, r0 + 1))
        s0, s1 = int(X.row_ptr[r0]), int(X.row_ptr[r0 + 1])
        assert np.array_equal(X.col_ind[s0:s1], R.col_ind), f"row {r0} pattern"
        assert orc.rel_err(X.data[int(start[s0]):int(start[s1])], R.data) <= TOL, f"row {r0}"
