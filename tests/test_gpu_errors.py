"""Error classes of the C-ABI that need matrix handles (hence a device):
shape mismatch, aliasing, bad filter threshold, results beyond the index
range, unsupported stack-path shapes, allocator failure, and matrices used
on two streams.  Validation failures leave every argument untouched."""
import numpy as np
import pytest

from oracle import oracle as orc
from synth import make_matrix, rng_of

from tests.helpers import check_against_oracle, lib, set_path

pytestmark = pytest.mark.gpu


def _status(fn, *a):
    b = lib()
    with pytest.raises(b.BsmmError) as e:
        fn(*a)
    return e.value.status


def _mats(rng, rbs, kbs, cbs, occ=1.0):
    A = make_matrix(rng, rbs, kbs, occ)
    B = make_matrix(rng, kbs, cbs, occ)
    return A, B


def test_shape_alias_and_threshold_leave_c_untouched():
    b = lib()
    rng = rng_of(0)
    A = make_matrix(rng, [4, 6], [2, 3], 1.0)
    B = make_matrix(rng, [3, 2], [5], 1.0)        # same total rows, other split
    Cin = make_matrix(rng, [4, 6], [5], 1.0)
    MA, MB, MC = b.Matrix.from_blocks(A), b.Matrix.from_blocks(B), b.Matrix.from_blocks(Cin)
    try:
        before = MC.to_host()
        assert _status(b.multiply, 1.0, MA, MB, 0.0, MC) == b.BSMM_ESHAPE
        B2 = make_matrix(rng, [2, 3], [5], 1.0)
        MB2 = b.Matrix.from_blocks(B2)
        MCbad = b.Matrix.empty([4, 6], [2, 3])
        assert _status(b.multiply, 1.0, MA, MB2, 0.0, MCbad) == b.BSMM_ESHAPE
        assert _status(b.multiply, 1.0, MA, MB2, 0.0, MA) == b.BSMM_EINVAL    # C aliases A
        assert _status(b.multiply, 1.0, MA, MB2, 0.0, MC, -1e-3) == b.BSMM_EINVAL
        assert _status(b.multiply, 1.0, MA, MB2, 0.0, MC, float("nan")) == b.BSMM_EINVAL
        after = MC.to_host()
        assert np.array_equal(before.row_ptr, after.row_ptr)
        assert np.array_equal(before.data, after.data)
        # A == B is allowed (square blocks)
        S = make_matrix(rng, [3, 4], [3, 4], 1.0)
        MS = b.Matrix.from_blocks(S)
        MS2 = b.Matrix.empty([3, 4], [3, 4])
        b.multiply(1.0, MS, MS, 0.0, MS2)
        check_against_oracle(MS2.to_host(), orc.multiply(1.0, S, S, 0.0), 1e-14)
        for M in (MB2, MCbad, MS, MS2):
            M.close()
    finally:
        for M in (MA, MB, MC):
            M.close()


def test_result_beyond_index_range():
    """C of 2^23 x 2^25 elements (2^48) exceeds the 2^47 elements a matrix
    may hold: ERANGE from the symbolic phase, before C is allocated."""
    b = lib()
    A = make_matrix(rng_of(1), [1 << 23], [1], 1.0, values="zeros")
    B = make_matrix(rng_of(1), [1], [1 << 25], 1.0, values="zeros")
    MA, MB = b.Matrix.from_blocks(A), b.Matrix.from_blocks(B)
    MC = b.Matrix.empty([1 << 23], [1 << 25])
    try:
        for path in ("auto", "stack"):
            set_path(path)
            assert _status(b.multiply, 1.0, MA, MB, 0.0, MC) == b.BSMM_ERANGE
            assert MC.info()[2] == 0
    finally:
        set_path()
        for M in (MA, MB, MC):
            M.close()


def test_stack_path_limits_are_rejected_before_work():
    """Block columns of A wider than 65,535 (the product entry holds k in 16
    bits) are refused on the stack path with ENOTSUP, and the dense path
    takes them; C with more block columns than the stack builder's LDS map
    (8,192) goes through the stack path."""
    b = lib()
    rng = rng_of(2)
    A = make_matrix(rng, [2], [70000], 1.0)
    B = make_matrix(rng, [70000], [3], 1.0)
    MA, MB = b.Matrix.from_blocks(A), b.Matrix.from_blocks(B)
    MC = b.Matrix.empty([2], [3])
    try:
        set_path("stack")
        assert _status(b.multiply, 1.0, MA, MB, 0.0, MC) == b.BSMM_ENOTSUP
        assert "65535" in b.bsmm_last_error()
        set_path("auto")
        b.multiply(1.0, MA, MB, 0.0, MC)
        check_against_oracle(MC.to_host(), orc.multiply(1.0, A, B, 0.0), 1e-13)
    finally:
        set_path()
        for M in (MA, MB, MC):
            M.close()
    A = make_matrix(rng, [1], [1], 1.0, values="int")
    B = make_matrix(rng, [1], np.ones(9000, np.int32), 0.5, values="int")
    MA, MB = b.Matrix.from_blocks(A), b.Matrix.from_blocks(B)
    MC = b.Matrix.empty([1], np.ones(9000, np.int32))
    try:
        set_path("stack")
        b.multiply(1.0, MA, MB, 0.0, MC)
        check_against_oracle(MC.to_host(), orc.multiply(1.0, A, B, 0.0), 0.0)
    finally:
        set_path()
        for M in (MA, MB, MC):
            M.close()


def test_allocator_failure_gives_enomem_and_recovers():
    """An allocator that returns NULL: create fails with ENOMEM; a multiply
    whose allocations start failing part-way returns ENOMEM; with a working
    allocator again the same multiply is correct."""
    import torch
    b = lib()
    rng = rng_of(3)
    A, B = _mats(rng, [13, 5, 23], [7, 32], [23, 5], occ=0.7)
    b.bsmm_set_allocator(lambda n, s: 0, lambda p, n, s: None)
    try:
        assert _status(b.Matrix.from_blocks, A) == b.BSMM_ENOMEM
    finally:
        b.bsmm_set_allocator()
    MA, MB = b.Matrix.from_blocks(A), b.Matrix.from_blocks(B)
    MC = b.Matrix.empty(A.rbs, B.cbs)
    live = {}
    try:
        for budget in (0, 1, 3):
            calls = [0]

            def alloc(n, s, budget=budget):
                calls[0] += 1
                if calls[0] > budget:
                    return 0
                t = torch.empty(n, dtype=torch.uint8, device="cuda")
                live[t.data_ptr()] = t
                return t.data_ptr()

            def dealloc(p, n, s):
                live.pop(p, None)

            b.bsmm_set_allocator(alloc, dealloc)
            set_path("stack", "tuned")
            assert _status(b.multiply, 1.0, MA, MB, 0.0, MC) == b.BSMM_ENOMEM
            b.bsmm_set_allocator()
        b.multiply(1.0, MA, MB, 0.0, MC)
        check_against_oracle(MC.to_host(), orc.multiply(1.0, A, B, 0.0), 1e-13)
    finally:
        b.bsmm_set_allocator()
        set_path()
        for M in (MA, MB, MC):
            M.close()


def test_matrix_created_on_one_stream_multiplied_on_another():
    """C is created on stream s1 and multiplied, with a filter that drops
    blocks (so its buffers are replaced), on stream s2 of the same priority;
    fresh matrices are then created on s1 from the pool.  Results equal the
    reference every time."""
    import torch
    b = lib()
    rng = rng_of(4)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    A, B = _mats(rng, [13, 5, 23, 32] * 3, [5, 32, 13] * 4, [23, 13, 5] * 3, occ=0.5)
    Cin = make_matrix(rng, A.rbs, B.cbs, 0.4)
    R = orc.multiply(1.0, A, B, 0.5, Cin, filter_eps=2.0)
    for rep in range(3):
        MA = b.Matrix.from_blocks(A, stream=s1)
        MB = b.Matrix.from_blocks(B, stream=s1)
        MC = b.Matrix.from_blocks(Cin, stream=s1)
        set_path("stack", "tuned")
        try:
            b.multiply(1.0, MA, MB, 0.5, MC, 2.0, stream=s2)
            others = [b.Matrix.from_blocks(Cin, stream=s1) for _ in range(3)]
            X = MC.to_host(stream=s1)
            check_against_oracle(X, R, 1e-13)
            for M in others:
                M.close()
        finally:
            set_path()
            for M in (MA, MB, MC):
                M.close()
