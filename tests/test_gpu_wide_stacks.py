"""Stack path with C wider than the stack builder's LDS column map (more
than 8,192 block columns): products counted and filled through a binary
search of C's rows in global memory.  Exact on integer inputs against the
CPU reference, for plain and tuned kernels, with A rows split into parts,
and with the stacks built in row panels (same bits as whole stacks)."""
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
