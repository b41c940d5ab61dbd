"""The allocation-free multiply (bsmm_multiply_noalloc) against bsmm_multiply.

Both entry points run the same kernels in the same order, so their results
must agree bit for bit.  Each case calls the allocation-free entry point
twice in a row, the second time on a smaller input, so the second call runs
on a scratch region still holding the first call's contents.  A counting
device allocator checks that no allocation happens inside the call."""
import numpy as np
import pytest

from synth import banded_uneven, make_matrix, rng_of

from tests.helpers import check_against_oracle, lib, set_path

pytestmark = pytest.mark.gpu


class CountingAllocator:
    """Device memory from torch's caching allocator, with a call count."""

    def __init__(self):
        import torch
        self.dev = torch.cuda.current_device()
        self.calls = 0

    def alloc(self, nbytes, stream):
        import torch
        self.calls += 1
        return torch.cuda.caching_allocator_alloc(nbytes, self.dev, stream if stream else None)

    def dealloc(self, ptr, nbytes, stream):
        import torch
        torch.cuda.caching_allocator_delete(ptr)


@pytest.fixture
def counting():
    b = lib()
    ca = CountingAllocator()
    b.bsmm_set_allocator(ca.alloc, ca.dealloc)
    try:
        yield ca
    finally:
        b.bsmm_set_allocator()


def _with_pattern_of(b, MA, MB, rbs, cbs, rng):
    """A C holding the product pattern of A*B with random values."""
    from synth import BlockCSR, block_elems
    T = b.Matrix.empty(rbs, cbs)
    b.multiply(1.0, MA, MB, 0.0, T)
    X = T.to_host()
    T.close()
    n = int(np.sum(block_elems(rbs, cbs, X.row_ptr, X.col_ind)))
    return BlockCSR(np.asarray(rbs, np.int32), np.asarray(cbs, np.int32), X.row_ptr, X.col_ind,
                    rng.uniform(-1.0, 1.0, n))


def _compare(A, B, alpha, beta, counting, path, kernel):
    """C_ref by bsmm_multiply, C_na by bsmm_multiply_noalloc (same C_in);
    returns (host C_na, stats of the allocation-free call)."""
    b = lib()
    rng = rng_of(7)
    set_path(path, kernel)
    try:
        MA, MB = b.Matrix.from_blocks(A), b.Matrix.from_blocks(B)
        Cin = _with_pattern_of(b, MA, MB, A.rbs, B.cbs, rng)
        Mref, Mna = b.Matrix.from_blocks(Cin), b.Matrix.from_blocks(Cin)
        b.multiply(alpha, MA, MB, beta, Mref)
        ref = Mref.to_host()
        before = counting.calls
        b.bsmm_multiply_noalloc(alpha, MA.handle, MB.handle, beta, Mna.handle)
        st = b.bsmm_last_stats()
        got = Mna.to_host()
        assert counting.calls == before, "the allocation-free multiply allocated device memory"
        check_against_oracle(got, ref, 0.0)
        for M in (MA, MB, Mref, Mna):
            M.close()
    finally:
        set_path()
    return got, st


@pytest.mark.parametrize("path,kernel", [("stack", "plain"), ("stack", "tuned"), ("dense", "plain")])
def test_noalloc_matches_multiply_twice_shrinking(counting, path, kernel):
    rng = rng_of(3)
    sizes = [5, 13, 23, 32, 7, 16]
    rbs = rng.choice(sizes, 14).astype(np.int32)
    kbs = rng.choice(sizes, 12).astype(np.int32)
    cbs = rng.choice(sizes, 15).astype(np.int32)
    A = make_matrix(rng, rbs, kbs, 0.4)
    B = make_matrix(rng, kbs, cbs, 0.4)
    _, st1 = _compare(A, B, 1.5, 0.5, counting, path, kernel)
    assert st1["path"] == (2 if path == "dense" else 1)
    # second call, smaller input, on the scratch the first call left behind
    A2 = make_matrix(rng, rbs[:5], kbs[:4], 0.6)
    B2 = make_matrix(rng, kbs[:4], cbs[:6], 0.6)
    _, st2 = _compare(A2, B2, -1.0, 0.0, counting, path, kernel)
    assert st2["n_products"] < st1["n_products"]


def test_noalloc_banded_split_runs(counting):
    """Long runs on few C blocks (split over waves with partial blocks in the
    scratch region), then the 1 % banded workload shape at small size."""
    rng = rng_of(5)
    A = make_matrix(rng, [32, 32], [23] * 300, 1.0)
    B = make_matrix(rng, [23] * 300, [32, 32], 1.0)
    _compare(A, B, 1.0, 0.0, counting, "stack", "tuned")
    U, V = banded_uneven(seed=1, occupancy=0.3, target=3000)
    _compare(U, V, 1.0, 1.0, counting, "stack", "tuned")


def test_noalloc_rejects_missing_pattern_and_oversize(counting):
    b = lib()
    rng = rng_of(11)
    A = make_matrix(rng, [8, 8], [8, 8], 1.0)
    B = make_matrix(rng, [8, 8], [8, 8], 1.0)
    MA, MB = b.Matrix.from_blocks(A), b.Matrix.from_blocks(B)
    MC = b.Matrix.empty(A.rbs, B.cbs)
    try:
        with pytest.raises(b.BsmmError) as e:
            b.bsmm_multiply_noalloc(1.0, MA.handle, MB.handle, 0.0, MC.handle)
        assert e.value.status == b.BSMM_EINDEX
        assert MC.info()[2] == 0
    finally:
        for M in (MA, MB, MC):
            M.close()
    # Dense panels of 2 x 3072^2 doubles (144 MiB) exceed the 64 MiB region.
    set_path("dense")
    n, bs = 3072, 256
    A = make_matrix(rng, [bs] * (n // bs), [bs] * (n // bs), 1.0)
    MA = b.Matrix.from_blocks(A)
    try:
        Cin = _with_pattern_of(b, MA, MA, A.rbs, A.cbs, rng)
        MC = b.Matrix.from_blocks(Cin)
        before = MC.to_host().data.copy()
        with pytest.raises(b.BsmmError) as e:
            b.bsmm_multiply_noalloc(1.0, MA.handle, MA.handle, 1.0, MC.handle)
        assert e.value.status == b.BSMM_ERANGE
        assert np.array_equal(MC.to_host().data, before)
        MC.close()
    finally:
        MA.close()
        set_path()


def test_noalloc_wide_c(counting):
    """C wider than the stack builder's LDS map (9,000 block columns, counted
    and filled in windows): the allocation-free multiply matches
    bsmm_multiply twice in a row, and a C pattern missing one product block
    is rejected with EINDEX before C is written."""
    from synth import BlockCSR
    b = lib()
    rng = rng_of(13)
    s = np.array([1, 2, 3], np.int32)
    ms, ks, ns = (rng.choice(s, size=x) for x in (40, 60, 9000))
    A = make_matrix(rng, ms, ks, 0.2)
    B = make_matrix(rng, ks, ns, 0.01)
    _compare(A, B, 1.0, 0.5, counting, "stack", "plain")
    _compare(make_matrix(rng, ms[:10], ks, 0.2), B, 2.0, 0.0, counting, "stack", "plain")
    MA, MB = b.Matrix.from_blocks(A), b.Matrix.from_blocks(B)
    try:
        full = _with_pattern_of(b, MA, MB, A.rbs, B.cbs, rng)
        rp = np.asarray(full.row_ptr)
        # drop the first stored block (row_ptr entries past its row shift by one)
        row0 = int(np.searchsorted(rp, 0, side="right")) - 1
        size0 = int(ms[row0]) * int(ns[int(full.col_ind[0])])
        holed = BlockCSR(full.rbs, full.cbs, np.maximum(rp - 1, 0), np.asarray(full.col_ind)[1:],
                         np.asarray(full.data)[size0:])
        MC = b.Matrix.from_blocks(holed)
        before = MC.to_host().data.copy()
        with pytest.raises(b.BsmmError) as e:
            b.bsmm_multiply_noalloc(1.0, MA.handle, MB.handle, 1.0, MC.handle)
        assert e.value.status == b.BSMM_EINDEX
        assert np.array_equal(MC.to_host().data, before)
        MC.close()
    finally:
        MA.close()
        MB.close()
