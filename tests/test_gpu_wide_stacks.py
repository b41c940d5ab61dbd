"""Stack path with C wider than the stack builder's LDS column map (more
than 8,192 block columns): products counted and filled window by window,
4,096 block columns of C mapped in LDS at a time.  Exact on integer inputs
against the CPU reference, for plain and tuned kernels, with A rows split
into parts, and with the stacks built in row panels (same bits as whole
stacks)."""
import numpy as np
import pytest

from oracle import oracle as orc
from synth import make_matrix, rng_of

from tests.helpers import check_against_oracle, gpu_multiply, lib

pytestmark = pytest.mark.gpu


def _wide(seed, nbr, nbk, occ_a, occ_b, nbc, sizes=(1, 2, 3, 5)):
    rng = rng_of(seed)
    s = np.array(sizes, np.int32)
    ms, ks, ns = (rng.choice(s, size=x) for x in (nbr, nbk, nbc))
    return (make_matrix(rng, ms, ks, occ_a, values="int"), make_matrix(rng, ks, ns, occ_b, values="int"),
            make_matrix(rng, ms, ns, 0.01, values="int"))


@pytest.mark.parametrize("kernel", ["plain", "tuned"])
def test_wide_c_exact(kernel):
    A, B, Cin = _wide(71, nbr=120, nbk=400, occ_a=0.05, occ_b=0.01, nbc=12000)
    R = orc.multiply(1.0, A, B, -0.5, Cin)
    X, st = gpu_multiply(1.0, A, B, -0.5, Cin, path="stack", kernel=kernel)
    assert len(B.cbs) > 8192 and st["n_products"] > 0
    check_against_oracle(X, R, 0.0)


def test_wide_c_split_rows_exact():
    """Three C block rows, long A rows: the count and fill run in parts."""
    A, B, _ = _wide(73, nbr=3, nbk=900, occ_a=0.5, occ_b=0.01, nbc=9000)
    X, st = gpu_multiply(1.0, A, B, 0.0, path="stack", kernel="tuned")
    check_against_oracle(X, orc.multiply(1.0, A, B, 0.0), 0.0)


def test_wide_c_row_panels_bitwise():
    A, B, _ = _wide(79, nbr=200, nbk=300, occ_a=0.05, occ_b=0.01, nbc=10000, sizes=(4, 7))
    b = lib()
    X1, st1 = gpu_multiply(1.0, A, B, 0.0, path="stack", kernel="plain")
    b.bsmm_set_option("stack_panel", str(max(1, st1["n_products"] // 7)))
    try:
        X2, st2 = gpu_multiply(1.0, A, B, 0.0, path="stack", kernel="plain")
    finally:
        b.bsmm_set_option("stack_panel", str(1 << 30))
    assert st2["n_row_panels"] > 1
    check_against_oracle(X2, X1, 0.0)


def _banded_wide(seed, nbr=120, nbk=400, nbc=20000):
    """Banded A (each C block row reaches about 20 K) times banded B (each K
    reaches about 200 columns around 50 K): a C block row covers one or two
    of the five 4,096-column windows, and some B rows cross a window edge."""
    rng = rng_of(seed)
    s = np.array([1, 2, 3], np.int32)
    ms, ks, ns = (rng.choice(s, size=x) for x in (nbr, nbk, nbc))
    I, K = np.meshgrid(np.arange(nbr), np.arange(nbk), indexing="ij")
    mask_a = (np.abs(K - I * nbk / nbr) < 10) & (rng.random((nbr, nbk)) < 0.6)
    K2, J = np.meshgrid(np.arange(nbk), np.arange(nbc), indexing="ij")
    mask_b = (np.abs(J - K2 * nbc / nbk) < 100) & (rng.random((nbk, nbc)) < 0.3)
    return make_matrix(rng, ms, ks, mask=mask_a, values="int"), make_matrix(rng, ks, ns, mask=mask_b, values="int")


@pytest.mark.parametrize("kernel", ["plain", "tuned"])
def test_wide_c_banded_windows_exact(kernel):
    """C of 20,000 block columns counted and filled window by window: rows
    whose products fill only some windows, B rows split at window edges;
    exact against the CPU reference, and row panels give the same bits as
    whole stacks."""
    A, B = _banded_wide(83)
    R = orc.multiply(1.0, A, B, 0.0)
    X1, st1 = gpu_multiply(1.0, A, B, 0.0, path="stack", kernel=kernel)
    assert len(B.cbs) == 20000 and st1["n_products"] > 0
    check_against_oracle(X1, R, 0.0)
    b = lib()
    b.bsmm_set_option("stack_panel", str(max(1, st1["n_products"] // 20)))
    try:
        X2, st2 = gpu_multiply(1.0, A, B, 0.0, path="stack", kernel=kernel)
    finally:
        b.bsmm_set_option("stack_panel", str(1 << 30))
    assert st2["n_row_panels"] > 1
    check_against_oracle(X2, X1, 0.0)
