"""Split-precision FP64 emulation on INT8 matrix cores: bit-exact against the
exact numpy reference of the same method, and within 1e-12 of FP64."""
import numpy as np
import pytest

from oracle import emul_ref as er
from oracle import oracle as orc
from synth import make_matrix, rng_of, wide_range_sparse

from tests.helpers import check_against_oracle, gpu_multiply, lib

pytestmark = pytest.mark.gpu


def _emul(A, B, alpha, beta, Cin, S):
    b = lib()
    b.bsmm_set_option("emul_slices", str(S))
    try:
        return gpu_multiply(alpha, A, B, beta, Cin, path="emul")
    finally:
        b.bsmm_set_option("emul_slices", "7")


@pytest.mark.parametrize("S", [1, 3, 7, 8])
def test_bit_exact_against_reference(S):
    rng = rng_of(100 + S)
    rbs = rng.integers(5, 33, size=4).astype(np.int32)
    kbs = rng.integers(5, 33, size=6).astype(np.int32)
    cbs = rng.integers(5, 33, size=3).astype(np.int32)
    A = make_matrix(rng, rbs, kbs, 1.0, values="wide")
    B = make_matrix(rng, kbs, cbs, 1.0, values="wide")
    Cin = make_matrix(rng, rbs, cbs, 1.0)
    for alpha, beta in [(1.0, 0.0), (-0.75, 1.5)]:
        X, st = _emul(A, B, alpha, beta, Cin, S)
        assert st["path"] == 3
        R = er.emulate(orc.to_dense(A), orc.to_dense(B), S, alpha, beta, orc.to_dense(Cin))
        D = orc.to_dense(X)
        bad = np.argwhere(D != R)
        assert len(bad) == 0, f"{len(bad)} mismatches, first {bad[:3].tolist()}: {D[tuple(bad[0])]} vs {R[tuple(bad[0])]}"


def test_multi_chunk_k():
    """K above the INT32-exact chunk (8 slices: 16640) is summed in FP64 per
    chunk, in chunk order, exactly as the reference does."""
    rng = rng_of(7)
    S = 8
    rbs = np.array([20, 12], np.int32)
    kbs = np.full(170, 100, np.int32)
    cbs = np.array([16, 9], np.int32)
    A = make_matrix(rng, rbs, kbs, 1.0, values="wide")
    B = make_matrix(rng, kbs, cbs, 1.0, values="wide")
    X, _ = _emul(A, B, 1.0, 0.0, None, S)
    R = er.emulate(orc.to_dense(A), orc.to_dense(B), S, kchunk=er.int32_chunk(S))
    assert er.int32_chunk(S) < 17000
    assert np.array_equal(orc.to_dense(X), R)


def test_integer_inputs_exact_with_one_slice():
    rng = rng_of(9)
    s = np.full(5, 16, np.int32)
    A = make_matrix(rng, s, s, 1.0, values=lambda r, n: r.integers(-127, 128, n).astype(float))
    B = make_matrix(rng, s, s, 1.0, values=lambda r, n: r.integers(-127, 128, n).astype(float))
    X, _ = _emul(A, B, 1.0, 0.0, None, 1)
    exact = orc.to_dense(A).astype(np.int64) @ orc.to_dense(B).astype(np.int64)
    assert np.array_equal(orc.to_dense(X), exact.astype(np.float64))


def test_sparse_wide_range_within_fp64_tolerance():
    """23-blocks, 20 % occupancy, entries spanning 1e-6 .. 1e2: the emulated
    result (7 slices) is within 1e-12 of the FP64 reference, same pattern."""
    A, B = wide_range_sparse(seed=1, nb=40, bs=23, occupancy=0.2)
    X, _ = _emul(A, B, 1.0, 0.0, None, 7)
    check_against_oracle(X, orc.multiply(1.0, A, B, 0.0), 1e-12)


@pytest.mark.parametrize("tile", ["t64", "t128", "t128k32", "t128w8"])
@pytest.mark.parametrize("S", [2, 7])
def test_tile_variants_bit_exact_over_many_tiles(tile, S):
    """Several workgroup tiles in each direction with ragged edges, sparse
    A, B and C (missing blocks read as zero, C's missing blocks stay
    unstored): both tile variants equal the reference bit for bit."""
    b = lib()
    rng = rng_of(300 + S)
    rbs = rng.integers(5, 33, size=14).astype(np.int32)
    kbs = rng.integers(5, 33, size=40).astype(np.int32)
    cbs = rng.integers(5, 33, size=11).astype(np.int32)
    A = make_matrix(rng, rbs, kbs, 0.7, values="wide")
    B = make_matrix(rng, kbs, cbs, 0.7, values="wide")
    Cin = make_matrix(rng, rbs, cbs, 0.5)
    b.bsmm_set_option("emul_kernel", tile)
    try:
        for alpha, beta in [(1.0, 0.0), (0.5, -2.0)]:
            X, st = _emul(A, B, alpha, beta, Cin, S)
            assert st["path"] == 3
            rp, ci = orc.pattern(A, B, Cin)
            assert np.array_equal(X.row_ptr, rp) and np.array_equal(X.col_ind, ci)
            # Blocks outside the pattern get no product and no old value, so
            # the dense reference is zero there as well.
            R = er.emulate(orc.to_dense(A), orc.to_dense(B), S, alpha, beta, orc.to_dense(Cin))
            D = orc.to_dense(X)
            bad = np.argwhere(D != R)
            assert len(bad) == 0, f"{len(bad)} mismatches, first {bad[:3].tolist()}"
    finally:
        b.bsmm_set_option("emul_kernel", "t128w8")
