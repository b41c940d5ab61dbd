"""Filtered matrices keep their kept blocks in place: the filter rewrites the
index only and the dropped blocks leave gaps in the storage (unless the
gaps would be most of it, when the data are packed).  Such a matrix must
behave like a packed one everywhere: copied out (host and device), used as
A or B on every path, as C with beta != 0 or beta == 0 on an unchanged
pattern, filtered again, screened, and in the allocation-free entry point."""
import numpy as np
import pytest

from oracle import oracle as orc
from synth import BlockCSR, banded_uneven, make_matrix, rng_of

from tests.helpers import check_against_oracle, device_rows, lib, set_path

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _holed(b, seed, eps=1e-10, target=1600):
    """A device matrix with gaps: C = A B filtered with the screen off (the
    filter then drops the far blocks), and its host copy."""
    A, B = banded_uneven(seed=seed, occupancy=0.3, target=target, decay=3.0)
    MA, MB = b.Matrix.from_blocks(A), b.Matrix.from_blocks(B)
    MH = b.Matrix.empty(A.rbs, B.cbs)
    b.bsmm_set_option("prescreen", "0")
    try:
        b.multiply(1.0, MA, MB, 0.0, MH, eps)
    finally:
        b.bsmm_set_option("prescreen", "1")
    st = b.bsmm_last_stats()
    assert 0 < st["c_nnzb_after"] < st["c_nnzb_before"]
    # Fewer than half of the elements dropped: the data stayed in place.
    R = orc.multiply(1.0, A, B, 0.0, filter_eps=eps)
    MA.close()
    MB.close()
    return MH, R


def test_copy_out_host_and_device():
    b = lib()
    MH, R = _holed(b, 90)
    check_against_oracle(MH.to_host(), R, TOL)
    n = len(R.rbs)
    for r0, r1 in ((0, 3), (n // 2, n // 2 + 5), (n - 2, n)):
        rows = orc.multiply(1.0, *banded_uneven(seed=90, occupancy=0.3, target=1600, decay=3.0), 0.0,
                            filter_eps=1e-10, rows=(r0, r1))
        check_against_oracle(device_rows(MH, r0, r1), rows, TOL)
    MH.close()


@pytest.mark.parametrize("path,kernel", [("stack", "plain"), ("stack", "tuned"), ("dense", "plain"),
                                         ("emul", "plain")])
def test_holed_operands(path, kernel):
    """The matrix with gaps as A and as B (the other operand random)."""
    b = lib()
    MH, H = _holed(b, 91)
    rng = rng_of(92)
    G = make_matrix(rng, H.cbs, H.rbs, 0.4)
    set_path(path, kernel)
    try:
        MG = b.Matrix.from_blocks(G)
        for left in (True, False):
            MX = b.Matrix.empty(H.rbs if left else G.rbs, G.cbs if left else H.cbs)
            b.multiply(1.0, MH if left else MG, MG if left else MH, 0.0, MX, 0.0)
            R = orc.multiply(1.0, H, G, 0.0) if left else orc.multiply(1.0, G, H, 0.0)
            check_against_oracle(MX.to_host(), R, 1e-11 if path == "emul" else TOL)
            MX.close()
        MG.close()
    finally:
        set_path()
        MH.close()


def test_holed_c_accumulate_and_refilter():
    """The matrix with gaps as C: beta != 0 over a grown pattern (old blocks
    moved in from the gapped storage), then beta = 0 and beta = 2 on the
    same pattern (every block of the product already stored), each
    filtered again."""
    b = lib()
    A, B = banded_uneven(seed=93, occupancy=0.3, target=1600, decay=3.0)
    MH, H = _holed(b, 93)
    MA, MB = b.Matrix.from_blocks(A), b.Matrix.from_blocks(B)
    ref = H
    for beta, eps in ((0.5, 1e-10), (0.0, 1e-12), (2.0, 1e-9)):
        set_path("stack", "tuned")
        try:
            b.multiply(1.0, MA, MB, beta, MH, eps)
        finally:
            set_path()
        ref = orc.multiply(1.0, A, B, beta, ref, filter_eps=eps)
        check_against_oracle(MH.to_host(), ref, TOL)
    for M in (MA, MB, MH):
        M.close()


def test_holed_operands_screened():
    """Block norms of operands with gaps feed the screen (sizes from the
    block rows, not from the offsets)."""
    b = lib()
    MH, H = _holed(b, 94, target=2400)
    MX = b.Matrix.empty(H.rbs, H.cbs)
    set_path("stack", "tuned")
    try:
        b.multiply(1.0, MH, MH, 0.0, MX, 1e-6)
        st = b.bsmm_last_stats()
    finally:
        set_path()
    assert st["n_screened"] > 0
    check_against_oracle(MX.to_host(), orc.multiply(1.0, H, H, 0.0, filter_eps=1e-6), TOL)
    MX.close()
    MH.close()


def test_filter_packs_when_mostly_dropped():
    """A filter that drops most of the elements packs the data; the result
    is the same either way."""
    b = lib()
    A, B = banded_uneven(seed=95, occupancy=0.3, target=1600, decay=3.0)
    MA, MB = b.Matrix.from_blocks(A), b.Matrix.from_blocks(B)
    MC = b.Matrix.empty(A.rbs, B.cbs)
    eps = 3.0
    b.bsmm_set_option("prescreen", "0")
    try:
        b.multiply(1.0, MA, MB, 0.0, MC, eps)
    finally:
        b.bsmm_set_option("prescreen", "1")
    st = b.bsmm_last_stats()
    R = orc.multiply(1.0, A, B, 0.0, filter_eps=eps)
    assert st["c_nnzb_after"] * 3 < st["c_nnzb_before"]
    check_against_oracle(MC.to_host(), R, TOL)
    for M in (MA, MB, MC):
        M.close()


def test_noalloc_into_holed_c():
    """The allocation-free entry point writes into C's gapped storage: C
    holds the product pattern plus old blocks outside it, half of them tiny,
    which a filtered multiply drops (leaving gaps); the next call computes
    every product block and scales the remaining old blocks by beta (their
    sizes from the block rows, not from the offsets)."""
    b = lib()
    rng = rng_of(96)
    n = 30
    sizes = rng.choice(np.array([5, 13, 23, 32], np.int32), n)
    I, J = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    band = np.abs(I - J)
    A = make_matrix(rng, sizes, sizes, mask=band <= 1)
    B = make_matrix(rng, sizes, sizes, mask=band <= 1)
    Cin = make_matrix(rng, sizes, sizes, mask=(band <= 2) | ((band >= 6) & (rng.random((n, n)) < 0.3)))
    far = np.repeat(band[np.repeat(np.arange(n), np.diff(np.asarray(Cin.row_ptr))), np.asarray(Cin.col_ind)] >= 6,
                    orc.block_sizes(Cin.rbs, Cin.cbs, Cin.row_ptr, Cin.col_ind))
    tiny = np.repeat(rng.random(len(Cin.col_ind)) < 0.5, orc.block_sizes(Cin.rbs, Cin.cbs, Cin.row_ptr,
                                                                          Cin.col_ind))
    Cin.data = np.where(far & tiny, np.asarray(Cin.data) * 1e-30, np.asarray(Cin.data))
    MA, MB, MC = b.Matrix.from_blocks(A), b.Matrix.from_blocks(B), b.Matrix.from_blocks(Cin)
    b.bsmm_set_option("prescreen", "0")  # the screen would leave the tiny blocks out before
    try:
        b.multiply(1.0, MA, MB, 1.0, MC, 1e-20)
    finally:
        b.bsmm_set_option("prescreen", "1")
    st = b.bsmm_last_stats()
    assert st["c_nnzb_after"] < st["c_nnzb_before"] == len(Cin.col_ind)
    C1 = MC.to_host()
    check_against_oracle(C1, orc.multiply(1.0, A, B, 1.0, Cin, filter_eps=1e-20), TOL)
    b.bsmm_multiply_noalloc(1.0, MA.handle, MB.handle, 3.0, MC.handle)
    check_against_oracle(MC.to_host(), orc.multiply(1.0, A, B, 3.0, C1), TOL)
    for M in (MA, MB, MC):
        M.close()
