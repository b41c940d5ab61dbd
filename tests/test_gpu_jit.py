"""Run-time compiled small-block kernels (option "jit"): classes whose
products share one depth k run on a kernel compiled with hiprtc for their
(m, n, k); exact on integer inputs, within the FP64 tolerance on random
values, cached across multiplies, and replaced by the precompiled kernels
where no kernel is compiled."""
import numpy as np
import pytest

from oracle import oracle as orc
from synth import make_matrix, rng_of

from tests.helpers import check_against_oracle, gpu_multiply, lib

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _jit(A, B, beta=0.0, Cin=None, alpha=1.0, params="16 16 0 4", dtype="f64", repeat=1):
    b = lib()
    b.bsmm_set_option("jit", "1")
    b.bsmm_set_option("stack_params", params)
    try:
        if dtype == "f64":
            return gpu_multiply(alpha, A, B, beta, Cin, path="stack", kernel="tuned", repeat=repeat)
        from tests.test_gpu_f32 import _f32_multiply
        return _f32_multiply(alpha, A, B, beta, Cin, path="stack", kernel="tuned", params=params, repeat=repeat)
    finally:
        b.bsmm_set_option("jit", "0")
        b.bsmm_set_option("stack_params", "")


def _uniform_k_case(seed, k, values="int", occ=0.5):
    rng = rng_of(seed)
    rbs = rng.choice([5, 13, 23, 32, 48], 9).astype(np.int32)
    cbs = rng.choice([5, 13, 23, 32, 64], 8).astype(np.int32)
    kbs = np.full(7, k, np.int32)
    A = make_matrix(rng, rbs, kbs, occ, values=values)
    B = make_matrix(rng, kbs, cbs, occ, values=values)
    Cin = make_matrix(rng, rbs, cbs, 0.3, values=values)
    return A, B, Cin


@pytest.mark.parametrize("k", [22, 5, 32, 13, 1, 17])
def test_jit_exact_on_integers(k):
    b = lib()
    A, B, Cin = _uniform_k_case(100 + k, k)
    R = orc.multiply(2.0, A, B, -1.0, Cin)
    c0 = b.bsmm_jit_stats()[0]
    X, st = _jit(A, B, beta=-1.0, Cin=Cin, alpha=2.0)
    assert st["n_jit_classes"] == st["n_classes"] > 1
    assert b.bsmm_jit_stats()[0] > c0
    check_against_oracle(X, R, 0.0)


def test_jit_fp32_exact_on_integers():
    A, B, Cin = _uniform_k_case(201, 23)
    R = orc.multiply(1.0, A, B, 1.0, Cin)
    X, st = _jit(A, B, beta=1.0, Cin=Cin, dtype="f32")
    assert st["n_jit_classes"] == st["n_classes"]
    check_against_oracle(X, R, 0.0)


def test_jit_random_values_and_cache():
    """Random values within the tolerance; a second multiply of the same
    shapes compiles nothing new."""
    b = lib()
    A, B, Cin = _uniform_k_case(301, 22, values="uniform")
    R = orc.multiply(0.5, A, B, 0.25, Cin)
    X, st = _jit(A, B, beta=0.25, Cin=Cin, alpha=0.5)
    check_against_oracle(X, R, TOL)
    compiled, hits, _, _ = b.bsmm_jit_stats()
    X, st = _jit(A, B, alpha=0.5, repeat=2)  # beta = 0: the repeat overwrites C
    compiled2, hits2, _, _ = b.bsmm_jit_stats()
    assert compiled2 == compiled and hits2 >= hits + 2 * st["n_jit_classes"]
    check_against_oracle(X, orc.multiply(0.5, A, B, 0.0), TOL)


def test_jit_not_used_for_uneven_depths_or_deep_k():
    """Mixed block-column sizes (no single k) and k beyond the compiled
    range take the precompiled kernels, with the same result quality."""
    rng = rng_of(401)
    rbs = np.array([13, 23, 32], np.int32)
    kbs = np.array([5, 13, 23, 32], np.int32)
    A = make_matrix(rng, rbs, kbs, 1.0, values="int")
    B = make_matrix(rng, kbs, rbs, 1.0, values="int")
    X, st = _jit(A, B)
    assert st["n_jit_classes"] == 0
    check_against_oracle(X, orc.multiply(1.0, A, B, 0.0), 0.0)
    A = make_matrix(rng, rbs, np.array([300, 300], np.int32), 1.0, values="int")
    B = make_matrix(rng, np.array([300, 300], np.int32), rbs, 1.0, values="int")
    X, st = _jit(A, B)
    assert st["n_jit_classes"] == 0
    check_against_oracle(X, orc.multiply(1.0, A, B, 0.0), 0.0)
