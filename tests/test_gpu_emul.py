"""Split-precision FP64 emulation on INT8 matrix cores: bit-exact against the
exact numpy reference of the same method, and within 1e-12 of FP64."""
import numpy as np
import pytest

from oracle import emul_ref as er
from oracle import oracle as orc
from synth import make_matrix, rng_of, wide_range_sparse

from tests.helpers import check_against_oracle, from_dense, gpu_multiply, lib

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
    """K above the INT32-exact chunk of the device (8 slices: 16,640): the
    chunks add their weight sums into exact int64 partials, so the result
    equals the reference, whose weight sums run over the whole K, bit for
    bit (for 7 and 8 slices, with beta * C)."""
    rng = rng_of(7)
    for S in (7, 8):
        rbs = np.array([20, 12], np.int32)
        kbs = np.full(200, 100, np.int32)
        cbs = np.array([16, 9], np.int32)
        A = make_matrix(rng, rbs, kbs, 1.0, values="wide")
        B = make_matrix(rng, kbs, cbs, 1.0, values="wide")
        Cin = make_matrix(rng, rbs, cbs, 1.0)
        assert 20000 > (2 ** 31 - 1) // (127 * 127 * S)
        X, _ = _emul(A, B, 0.5, -1.0, Cin, S)
        R = er.emulate(orc.to_dense(A), orc.to_dense(B), S, 0.5, -1.0, orc.to_dense(Cin))
        D = orc.to_dense(X)
        bad = np.argwhere(D != R)
        assert len(bad) == 0, f"S={S}: {len(bad)} mismatches, first {bad[:3].tolist()}"


def test_multi_chunk_k_beyond_int32_closed_form():
    """Every digit 127 (entries 1 - 2^-49) at K = 20,000: the heaviest weight
    sum, 7 K 127^2, exceeds 2^31, so the chunked INT32 sums must be carried
    exactly; the device result equals the reference bit for bit."""
    S = 7
    x = 1.0 - 2.0 ** -49
    rbs = np.array([16], np.int32)
    kbs = np.full(625, 32, np.int32)
    cbs = np.array([8], np.int32)
    A = make_matrix(rng_of(0), rbs, kbs, 1.0, values=lambda r, n: np.full(n, x))
    B = make_matrix(rng_of(0), kbs, cbs, 1.0, values=lambda r, n: np.full(n, x))
    X, _ = _emul(A, B, 1.0, 0.0, None, S)
    R = er.emulate(orc.to_dense(A), orc.to_dense(B), S)
    assert np.array_equal(orc.to_dense(X), R)


def test_subnormal_and_non_finite_rows():
    """A row of A whose largest entry is subnormal is scaled exactly; a row
    of A holding Inf and a column of B holding NaN give NaN in their row and
    column of the product; everything else equals the reference."""
    rng = rng_of(8)
    rbs = np.array([8, 8], np.int32)
    kbs = np.array([16, 16], np.int32)
    cbs = np.array([8, 8], np.int32)
    A = make_matrix(rng, rbs, kbs, 1.0, values="wide")
    B = make_matrix(rng, kbs, cbs, 1.0, values="wide")
    Ad = orc.to_dense(A)
    Bd = orc.to_dense(B)
    Ad[2, :] = np.ldexp(rng.integers(-127, 128, 32).astype(np.float64), -1074)
    Ad[11, 5] = np.inf
    Bd[20, 13] = np.nan
    A2 = from_dense(Ad, rbs, kbs)
    B2 = from_dense(Bd, kbs, cbs)
    X, _ = _emul(A2, B2, 1.0, 0.0, None, 7)
    R = er.emulate(Ad, Bd, 7)
    D = orc.to_dense(X)
    same = (D == R) | (np.isnan(D) & np.isnan(R))
    assert np.all(same), np.argwhere(~same)[:4].tolist()
    assert np.all(np.isnan(D[11, :])) and np.all(np.isnan(D[:, 13]))
    assert np.all(np.isfinite(D[2, :8])) and np.any(D[2, :] != 0)


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
