"""Single-precision matrices (paper, Sec. II: the library takes single- and
double-precision numbers).  FP32 block data run through the same stacks and
kernels computing in FP32: exact on integer inputs whose sums stay below
2^24, and within 1e-5 of the FP64 reference on FP32-representable inputs."""
import numpy as np
import pytest

from oracle import oracle as orc
from synth import BlockCSR, banded_uneven, make_matrix, rng_of

from tests.helpers import check_against_oracle, lib, set_path

pytestmark = pytest.mark.gpu
TOL32 = 1e-5


def _as_f32(M):
    """The same matrix with values rounded to FP32 (kept as float64, which
    represents them exactly): the reference's inputs."""
    return BlockCSR(M.rbs, M.cbs, M.row_ptr, M.col_ind, np.asarray(M.data, np.float32).astype(np.float64))


def _f32_multiply(alpha, A, B, beta, Cin=None, eps=0.0, path="auto", kernel="plain", params="", repeat=1):
    """C <- filter(beta C + alpha A B) on FP32 matrices; the host copy of C
    (float64 holding the FP32 values) and the stats."""
    b = lib()
    set_path(path, kernel)
    b.bsmm_set_option("stack_params", params)
    try:
        MA = b.Matrix.from_blocks(A, dtype="f32")
        MB = b.Matrix.from_blocks(B, dtype="f32")
        MC = (b.Matrix.from_blocks(Cin, dtype="f32") if Cin is not None
              else b.Matrix.empty(A.rbs, B.cbs, dtype="f32"))
        for _ in range(repeat):
            b.multiply(alpha, MA, MB, beta, MC, eps)
        st = b.bsmm_last_stats()
        X = MC.to_host()
        assert X.data.dtype == np.float32
        X.data = X.data.astype(np.float64)
        for M in (MA, MB, MC):
            M.close()
    finally:
        set_path()
        b.bsmm_set_option("stack_params", "")
    return X, st


def _int_case(seed, sizes, occ, nbr=9, nbk=8, nbc=10):
    rng = rng_of(seed)
    rbs = rng.choice(sizes, nbr).astype(np.int32)
    kbs = rng.choice(sizes, nbk).astype(np.int32)
    cbs = rng.choice(sizes, nbc).astype(np.int32)
    A = make_matrix(rng, rbs, kbs, occ, values="int")
    B = make_matrix(rng, kbs, cbs, occ, values="int")
    Cin = make_matrix(rng, rbs, cbs, 0.4, values="int")
    return A, B, Cin


@pytest.mark.parametrize("path,kernel,params", [
    ("stack", "plain", ""), ("stack", "tuned", "16 16 0 4"), ("stack", "tuned", "2 3 8 2"),
    ("stack", "tuned", ""), ("dense", "plain", "")])
def test_f32_exact_on_integers(path, kernel, params):
    """Integer entries in [-8, 8]: every partial sum is an integer below
    2^24, so FP32 arithmetic is exact and the result equals the FP64
    reference bit for bit (alpha, beta integers, old C present)."""
    A, B, Cin = _int_case(5, [5, 13, 23, 32, 7], 0.5)
    R = orc.multiply(2.0, A, B, -1.0, Cin)
    X, st = _f32_multiply(2.0, A, B, -1.0, Cin, path=path, kernel=kernel, params=params)
    assert st["path"] == (2 if path == "dense" else 1)
    check_against_oracle(X, R, 0.0)


def test_f32_scheduled_kernel_exact_on_integers():
    """The scheduled MFMA launch (classes up to 32 x 32) in FP32."""
    b = lib()
    A, B = banded_uneven(seed=51, occupancy=0.3, target=1500)
    rng = rng_of(52)
    A.data = rng.integers(-8, 9, A.data.size).astype(np.float64)
    B.data = rng.integers(-8, 9, B.data.size).astype(np.float64)
    R = orc.multiply(1.0, A, B, 0.0)
    saved = b.bsmm_get_option("stack_tile")
    b.bsmm_set_option("stack_tile", "8")
    try:
        X, st = _f32_multiply(1.0, A, B, 0.0, path="stack", kernel="tuned", params="16 16 0 4")
    finally:
        b.bsmm_set_option("stack_tile", saved)
    assert st["n_sched_runs"] == st["n_runs"] > 0
    check_against_oracle(X, R, 0.0)


@pytest.mark.parametrize("path,kernel", [("stack", "plain"), ("stack", "tuned"), ("dense", "plain")])
def test_f32_random_within_tolerance(path, kernel):
    """Uniform values rounded to FP32, uneven blocks, beta != 0, the filter:
    within 1e-5 of the FP64 reference of the same (FP32-representable)
    inputs."""
    A, B = banded_uneven(seed=53, occupancy=0.25, target=2000)
    A, B = _as_f32(A), _as_f32(B)
    rng = rng_of(54)
    Cin = _as_f32(make_matrix(rng, A.rbs, B.cbs, 0.1))
    R = orc.multiply(0.5, A, B, 0.25, Cin)
    X, st = _f32_multiply(0.5, A, B, 0.25, Cin, path=path, kernel=kernel)
    check_against_oracle(X, R, TOL32)
    eps = _eps_in_gap(orc.multiply(1.0, A, B, 0.0))
    R = orc.multiply(1.0, A, B, 0.0, filter_eps=eps)
    X, st = _f32_multiply(1.0, A, B, 0.0, eps=eps, path=path, kernel=kernel)
    assert st["c_nnzb_after"] < st["c_nnzb_before"]
    check_against_oracle(X, R, TOL32)


def _eps_in_gap(R):
    """A threshold that drops about half of the blocks of R and sits in the
    widest relative gap between neighbouring squared block norms there, so
    that FP32 rounding of the norms cannot change a keep decision."""
    s = np.sort(orc.block_sumsq(R))
    lo, hi = len(s) * 2 // 5, len(s) * 3 // 5
    gaps = s[lo + 1:hi + 1] / np.maximum(s[lo:hi], 1e-300)
    i = lo + int(np.argmax(gaps))
    assert s[i + 1] > s[i] * (1 + 1e-4)
    return float(np.sqrt(np.sqrt(s[i] * s[i + 1])))


def test_f32_dense_split_k_and_full_size_rows():
    """Few output tiles with a long k (split over workgroups, partial tiles
    summed in FP32 in a fixed order), and the dense 4096 product in
    32-blocks checked on sampled block rows."""
    rng = rng_of(55)
    A = _as_f32(make_matrix(rng, [128, 128], [64] * 512, 1.0))
    B = _as_f32(make_matrix(rng, [64] * 512, [128, 128], 1.0))
    X, st = _f32_multiply(1.0, A, B, 0.0)
    assert st["path"] == 2
    check_against_oracle(X, orc.multiply(1.0, A, B, 0.0), TOL32)
    from synth import dense_square
    A, B = dense_square(seed=3, n=4096, bs=32)
    A, B = _as_f32(A), _as_f32(B)
    X, st = _f32_multiply(1.0, A, B, 0.0)
    sizes = orc.block_sizes(X.rbs, X.cbs, X.row_ptr, X.col_ind)
    start = np.concatenate([[0], np.cumsum(sizes)])
    for r in (0, 77, 127):
        R = orc.multiply(1.0, A, B, 0.0, rows=(r, r + 1))
        s0, s1 = int(X.row_ptr[r]), int(X.row_ptr[r + 1])
        assert orc.rel_err(X.data[int(start[s0]):int(start[s1])], R.data) <= TOL32


def test_f32_type_errors_and_noalloc():
    b = lib()
    rng = rng_of(56)
    A = make_matrix(rng, [8, 8], [8, 8], 1.0, values="int")
    M64 = b.Matrix.from_blocks(A)
    M32 = b.Matrix.from_blocks(A, dtype="f32")
    C32 = b.Matrix.empty(A.rbs, A.cbs, dtype="f32")
    try:
        assert b.bsmm_matrix_dtype(M32.handle) == b.BSMM_F32
        assert b.bsmm_matrix_dtype(M64.handle) == b.BSMM_F64
        with pytest.raises(b.BsmmError) as e:
            b.multiply(1.0, M64, M32, 0.0, C32)
        assert e.value.status == b.BSMM_EINVAL
        b.bsmm_set_option("path", "emul")
        with pytest.raises(b.BsmmError) as e:
            b.multiply(1.0, M32, M32, 0.0, C32)
        assert e.value.status == b.BSMM_ENOTSUP
        b.bsmm_set_option("path", "auto")
        import ctypes
        d = np.zeros(256, np.float64)
        assert b._lib.bsmm_copy_out(M32.handle, None, None, ctypes.c_void_p(d.ctypes.data), 0, None) \
            == b.BSMM_EINVAL
        # allocation-free multiply on FP32 data, into the product pattern
        b.multiply(1.0, M32, M32, 0.0, C32)
        ref = C32.to_host().data.copy()
        b.bsmm_multiply_noalloc(1.0, M32.handle, M32.handle, 0.0, C32.handle)
        assert np.array_equal(C32.to_host().data, ref)
        R = orc.multiply(1.0, A, A, 0.0)
        assert np.array_equal(ref.astype(np.float64), R.data)
    finally:
        b.bsmm_set_option("path", "auto")
        for M in (M64, M32, C32):
            M.close()
