"""The scheduled launch reading A's blocks from row-major copies (option
"stack_at"): the same products in the same MFMA order, so the same bits as
reading A in place, for FP64 and FP32; a replayed plan copies A again, so
new values of A are seen."""
import numpy as np
import pytest

from oracle import oracle as orc
from synth import banded_uneven

from tests.helpers import check_against_oracle, gpu_multiply, lib, set_path

pytestmark = pytest.mark.gpu


def _case(seed):
    # Enough runs (C blocks) for the scheduled launch.
    return banded_uneven(seed=seed, occupancy=0.3, target=2600, decay=6.0)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_transposed_a_same_bits(dtype):
    from tests.test_gpu_f32 import _as_f32, _f32_multiply
    A, B = _case(101)
    b = lib()
    out = {}
    try:
        for at in ("0", "1"):
            b.bsmm_set_option("stack_at", at)
            if dtype == "f64":
                out[at] = gpu_multiply(-0.5, A, B, 0.0, eps=1e-10, path="stack", kernel="tuned")
            else:
                out[at] = _f32_multiply(-0.5, _as_f32(A), _as_f32(B), 0.0, eps=1e-6, path="stack",
                                        kernel="tuned")
    finally:
        b.bsmm_set_option("stack_at", "auto")
    (X0, st0), (X1, st1) = out["0"], out["1"]
    assert st1["n_sched_runs"] > 4096 and st1["n_sched_runs"] == st0["n_sched_runs"]
    check_against_oracle(X1, X0, 0.0)


def test_transposed_a_replay_sees_new_values():
    """FP32 (copies by default) with the plan cache: the second multiply
    replays the plan after A was doubled in place (same pattern and
    buffers, so the plan still holds) and must use the doubled values."""
    from tests.test_gpu_f32 import TOL32, _as_f32
    A, B = _case(102)
    A, B = _as_f32(A), _as_f32(B)
    b = lib()
    b.bsmm_set_option("plan_cache", "1")
    set_path("stack", "tuned")
    try:
        MA, MB = b.Matrix.from_blocks(A, dtype="f32"), b.Matrix.from_blocks(B, dtype="f32")
        MC = b.Matrix.empty(A.rbs, B.cbs, dtype="f32")
        b.multiply(1.0, MA, MB, 0.0, MC, 0.0)
        R1 = orc.multiply(1.0, A, B, 0.0)
        X1 = MC.to_host()
        X1.data = X1.data.astype(np.float64)
        check_against_oracle(X1, R1, TOL32)
        # A <- 2 A in place: an empty product into A keeps its pattern.
        E1 = b.Matrix.empty(A.rbs, A.rbs, dtype="f32")
        E2 = b.Matrix.empty(A.rbs, A.cbs, dtype="f32")
        b.multiply(1.0, E1, E2, 2.0, MA, 0.0)
        b.multiply(1.0, MA, MB, 0.0, MC, 0.0)
        st = b.bsmm_last_stats()
        X2 = MC.to_host()
        X2.data = X2.data.astype(np.float64)
        for M in (MA, MB, MC, E1, E2):
            M.close()
    finally:
        b.bsmm_set_option("plan_cache", "0")
        set_path()
    assert st["n_sched_runs"] > 4096
    check_against_oracle(X2, orc.multiply(2.0, A, B, 0.0), TOL32)
