"""Scheduled small-block kernel: every MFMA class with blocks up to 32 x 32
in one launch, runs ordered by tiles of C blocks.  Each run is computed by
the same per-run code as the per-class kernels, so the two give the same
bits; against the reference: exact on integer inputs, within the FP64
tolerance otherwise."""
import numpy as np
import pytest

from oracle import oracle as orc
from synth import banded_uneven, make_matrix, rng_of

from tests.helpers import check_against_oracle, gpu_multiply, lib

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _run(A, B, beta=0.0, Cin=None, eps=0.0, tile=0, sched="static", params="", repeat=1):
    b = lib()
    saved = {k: b.bsmm_get_option(k) for k in ("stack_tile", "stack_sched", "stack_params")}
    b.bsmm_set_option("stack_tile", str(tile))
    b.bsmm_set_option("stack_sched", sched)
    b.bsmm_set_option("stack_params", params)
    try:
        return gpu_multiply(1.0, A, B, beta, Cin, eps=eps, path="stack", kernel="tuned", repeat=repeat)
    finally:
        for k, v in saved.items():
            b.bsmm_set_option(k, v)


def _int_banded(seed, occ, target):
    A, B = banded_uneven(seed=seed, occupancy=occ, target=target)
    rng = rng_of(seed + 1)
    A.data = rng.integers(-8, 9, A.data.size).astype(np.float64)
    B.data = rng.integers(-8, 9, B.data.size).astype(np.float64)
    return A, B


@pytest.mark.parametrize("tile,sched", [(1, "static"), (3, "static"), (16, "dynamic"), (65536, "static"),
                                        (7, "dynamic")])
def test_sched_exact_on_integers(tile, sched):
    A, B = _int_banded(31, 0.3, 1500)
    rng = rng_of(2)
    Cin = make_matrix(rng, A.rbs, B.cbs, 0.2, values="int")
    R = orc.multiply(1.0, A, B, -1.0, Cin)
    X, st = _run(A, B, beta=-1.0, Cin=Cin, tile=tile, sched=sched, params="16 16 0 4")
    assert st["n_classes"] == 16 and st["n_sched_runs"] == st["n_runs"]
    check_against_oracle(X, R, 0.0)


@pytest.mark.parametrize("sched", ["static", "dynamic"])
def test_sched_bitwise_equals_class_kernels(sched):
    """Random values: same bits as the per-class launches, and within the
    tolerance of the reference, with the filter."""
    A, B = banded_uneven(seed=37, occupancy=0.2, target=2500)
    Xc, _ = _run(A, B, eps=1e-10, tile=0, params="16 16 0 2")
    Xs, st = _run(A, B, eps=1e-10, tile=8, sched=sched, params="16 16 0 2")
    assert st["n_sched_runs"] == st["n_runs"]
    check_against_oracle(Xs, Xc, 0.0)
    check_against_oracle(Xs, orc.multiply(1.0, A, B, 0.0, filter_eps=1e-10), TOL)


def test_sched_mixed_with_class_kernels():
    """Scheduled classes (at least 4096 runs each), classes of blocks above
    32 (per-class MFMA kernels) and classes of few long runs (split over
    waves) in one graph."""
    rng = rng_of(41)
    rbs = np.array([5] * 70 + [13] * 70 + [40, 40], np.int32)
    kbs = np.array([7] * 30 + [3] * 400, np.int32)
    cbs = np.array([5] * 70 + [23] * 70 + [44, 44], np.int32)
    A = make_matrix(rng, rbs, kbs, 0.25)
    B = make_matrix(rng, kbs, cbs, 0.25)
    Cin = make_matrix(rng, rbs, cbs, 0.5)
    R = orc.multiply(1.0, A, B, 0.5, Cin)
    X, st = _run(A, B, beta=0.5, Cin=Cin, tile=2, sched="dynamic", params="16 16 0 4")
    assert st["n_classes"] == 9 and 0 < st["n_sched_runs"] < st["n_runs"]
    check_against_oracle(X, R, TOL)


def test_sched_plan_cache_replays():
    """Replays of the planned graph (dynamic schedule: the run counter is
    reset by a kernel node on every replay) give the same result."""
    b = lib()
    A, B = banded_uneven(seed=43, occupancy=0.3, target=1500)
    R = orc.multiply(1.0, A, B, 0.0)
    b.bsmm_set_option("plan_cache", "1")
    try:
        X, st = _run(A, B, tile=4, sched="dynamic", params="16 16 0 4", repeat=4)
    finally:
        b.bsmm_set_option("plan_cache", "0")
    check_against_oracle(X, R, TOL)


def test_sched_short_runs_chunked_and_small_fallback():
    """Runs of about one product (several schedule entries per counter
    update), and a product with too few runs for the schedule (classes
    launched on their own): both match the reference."""
    A, B = banded_uneven(seed=47, occupancy=0.02, target=12000)
    R = orc.multiply(1.0, A, B, 0.0, filter_eps=1e-10)
    X, st = _run(A, B, eps=1e-10, tile=32, sched="dynamic", params="16 16 0 4")
    assert st["n_sched_runs"] == st["n_runs"] >= 4096 and st["n_products"] < 4 * st["n_runs"]
    check_against_oracle(X, R, TOL)
    A, B = banded_uneven(seed=48, occupancy=0.3, target=600)
    R = orc.multiply(1.0, A, B, 0.0)
    X, st = _run(A, B, tile=32, sched="dynamic", params="16 16 0 4")
    assert st["n_runs"] < 4096 and st["n_sched_runs"] == 0
    check_against_oracle(X, R, TOL)


def _eps_in_gap(R):
    """A threshold that drops about half of the blocks of R, in the widest
    relative gap between neighbouring squared block norms there."""
    s = np.sort(orc.block_sumsq(R))
    lo, hi = len(s) * 2 // 5, len(s) * 3 // 5
    gaps = s[lo + 1:hi + 1] / np.maximum(s[lo:hi], 1e-300)
    i = lo + int(np.argmax(gaps))
    assert s[i + 1] > s[i] * (1 + 1e-9)
    return float(np.sqrt(np.sqrt(s[i] * s[i + 1])))


@pytest.mark.parametrize("beta", [0.0, 0.75])
def test_sched_norms_feed_the_filter(beta):
    """With a filter, the scheduled kernel hands the squared norms of the
    blocks it writes to the filter (blocks of other classes are measured by
    the filter itself): same kept blocks and bits as the per-class launches,
    whose blocks the filter measures; also through plan-cache replays with
    a filter that keeps every block."""
    b = lib()
    A, B = banded_uneven(seed=61, occupancy=0.3, target=2500)
    Cin = make_matrix(rng_of(62), A.rbs, B.cbs, 0.4) if beta else None
    eps = _eps_in_gap(orc.multiply(1.0, A, B, beta, Cin))
    R = orc.multiply(1.0, A, B, beta, Cin, filter_eps=eps)
    Xc, stc = _run(A, B, beta=beta, Cin=Cin, eps=eps, tile=0, params="16 16 0 2")
    Xs, sts = _run(A, B, beta=beta, Cin=Cin, eps=eps, tile=8, sched="dynamic", params="16 16 0 2")
    assert sts["n_sched_runs"] == sts["n_runs"] and 0 < sts["c_nnzb_after"] < sts["c_nnzb_before"]
    check_against_oracle(Xs, Xc, 0.0)
    check_against_oracle(Xs, R, TOL)
    if beta:
        return
    # A threshold below every norm keeps C's pattern, so the repeats replay
    # the plan, whose launches write the norms into the plan's buffer.
    b.bsmm_set_option("plan_cache", "1")
    try:
        Xr, st = _run(A, B, eps=1e-150, tile=8, sched="dynamic", params="16 16 0 2", repeat=3)
    finally:
        b.bsmm_set_option("plan_cache", "0")
    assert st["c_nnzb_after"] == st["c_nnzb_before"]
    check_against_oracle(Xr, orc.multiply(1.0, A, B, 0.0), TOL)
