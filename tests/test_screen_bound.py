"""The premise of the symbolic screen, checked on the CPU reference: every
block of C = beta C_in + alpha A B satisfies
||C_IJ||_F <= |alpha| sum_K ||A_IK||_F ||B_KJ||_F + |beta| ||C_in,IJ||_F
(triangle inequality and submultiplicativity of the Frobenius norm), so a
block whose bound, grown by a rounding margin, lies below eps is one the
filter drops.  Norms here are numpy's, bounds summed with Python floats per
block: nothing is shared with the library's screen."""
import numpy as np
import pytest

from oracle import oracle as orc
from synth import banded_uneven, make_matrix, rng_of


def _norms(M):
    """{(I, J): Frobenius norm} of a block-CSR matrix."""
    sizes = orc.block_sizes(M.rbs, M.cbs, M.row_ptr, M.col_ind)
    start = np.concatenate([[0], np.cumsum(sizes)])
    rows = np.repeat(np.arange(len(M.rbs)), np.diff(np.asarray(M.row_ptr)))
    data = np.asarray(M.data)
    return {(int(i), int(j)): float(np.linalg.norm(data[start[p]:start[p + 1]]))
            for p, (i, j) in enumerate(zip(rows, np.asarray(M.col_ind)))}


def _bounds(alpha, A, B, beta, Cin):
    na, nb = _norms(A), _norms(B)
    brow = {}
    for (k, j), v in nb.items():
        brow.setdefault(k, []).append((j, v))
    out = {}
    for (i, k), va in na.items():
        for j, vb in brow.get(k, []):
            out[(i, j)] = out.get((i, j), 0.0) + abs(alpha) * va * vb
    if Cin is not None:
        for key, vc in _norms(Cin).items():
            out[key] = out.get(key, 0.0) + abs(beta) * vc
    return out


@pytest.mark.parametrize("seed,alpha,beta", [(81, 1.0, 0.0), (82, -2.5, 0.75)])
def test_every_block_within_its_bound(seed, alpha, beta):
    A, B = banded_uneven(seed=seed, occupancy=0.3, target=700, decay=2.0)
    Cin = make_matrix(rng_of(seed + 100), A.rbs, B.cbs, 0.3) if beta else None
    bounds = _bounds(alpha, A, B, beta, Cin)
    C = orc.multiply(alpha, A, B, beta, Cin)
    norms = _norms(C)
    assert set(norms) == set(bounds)
    ratio = max(norms[k] / bounds[k] for k in norms if bounds[k] > 0)
    assert ratio <= 1.0 + 1e-12
    # The bound is not vacuous: it spans many orders of magnitude here.
    vals = np.array([bounds[k] for k in norms])
    assert vals.max() / vals[vals > 0].min() > 1e10


def test_screened_blocks_are_filtered():
    """Blocks with bound * (1 + 1e-6) < eps are absent from the filtered
    reference result, and some blocks fall there."""
    A, B = banded_uneven(seed=83, occupancy=0.3, target=700, decay=2.0)
    eps = 1e-10
    bounds = _bounds(1.0, A, B, 0.0, None)
    screened = {k for k, v in bounds.items() if v * (1 + 1e-6) < eps}
    assert len(screened) > 10
    kept = set(_norms(orc.multiply(1.0, A, B, 0.0, filter_eps=eps)))
    assert not (screened & kept)
