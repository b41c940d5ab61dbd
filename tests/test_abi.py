"""CPU-side checks of the C-ABI library: it loads without a GPU, exports
every function declared in include/bsmm.h, and rejects malformed input on
the host before touching a device."""
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "bsmm.h")).read()
    return sorted(set(re.findall(r"\b(bsmm_[a-z_]+)\s*\(", txt)))


def test_exports_every_declared_function():
    from paper_1910_04796_amd import bsmm
    so = bsmm.LIB_PATH
    out = subprocess.run(["nm", "-D", "--defined-only", so], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\sT\s(bsmm_\w+)", out))
    declared = _declared()
    assert declared, "no declarations found"
    missing = [f for f in declared if f not in exported]
    assert not missing, f"declared but not exported: {missing}"
    for f in declared:
        assert hasattr(bsmm._lib, f)
    assert set(bsmm.EXPORTED) == set(declared)


def _err(fn, *a):
    from paper_1910_04796_amd import bsmm
    with pytest.raises(bsmm.BsmmError) as e:
        fn(*a)
    return e.value.status


def test_create_rejects_malformed_input():
    from paper_1910_04796_amd import bsmm as b
    c = b.bsmm_create_matrix
    assert _err(c, 2, [1, 0], 2, [1, 1], 0, [0, 0, 0], [], None) == b.BSMM_EINVAL
    assert _err(c, 2, [1, 1], 2, [1, -3], 0, [0, 0, 0], [], None) == b.BSMM_EINVAL
    assert _err(c, 2, [1, 1], 2, [1, 1], 2, [0, 1, 2], [1, 5], None) == b.BSMM_EINDEX
    assert _err(c, 2, [1, 1], 2, [1, 1], 2, [0, 2, 2], [1, 0], None) == b.BSMM_EINDEX
    assert _err(c, 2, [1, 1], 2, [1, 1], 2, [0, 2, 2], [1, 1], None) == b.BSMM_EINDEX
    assert _err(c, 2, [1, 1], 2, [1, 1], 2, [1, 1, 2], [1, 1], None) == b.BSMM_EINDEX
    assert _err(c, 2, [1, 1], 2, [1, 1], 2, [0, 2, 1], [0, 1], None) == b.BSMM_EINDEX
    assert _err(c, 2, [1, 1], 2, [1, 1], 3, [0, 1, 2], [0, 1], None) == b.BSMM_EINDEX


def test_create_typed_rejects_unknown_type_and_malformed_input():
    """The element-type check and the index checks of the typed create run
    on the host, before any HIP call."""
    import ctypes
    from paper_1910_04796_amd import bsmm as b
    rbs = np.array([1, 1], np.int32)
    rp = np.array([0, 0, 0], np.int64)
    h = ctypes.c_void_p()
    st = b._lib.bsmm_create_matrix_typed(2, rbs.ctypes.data_as(b._i32p), 2, rbs.ctypes.data_as(b._i32p), 0,
                                         rp.ctypes.data_as(b._i64p), None, 7, None, 0, None, ctypes.byref(h))
    assert st == b.BSMM_EINVAL and "element type" in b.bsmm_last_error()
    c = b.bsmm_create_matrix
    assert _err(lambda: c(2, [1, 1], 2, [1, 1], 2, [0, 1, 2], [1, 5], None, dtype="f32")) == b.BSMM_EINDEX
    assert _err(lambda: c(2, [0, 1], 2, [1, 1], 0, [0, 0, 0], [], None, dtype="f32")) == b.BSMM_EINVAL


def test_multiply_rejects_null_handles():
    from paper_1910_04796_amd import bsmm as b
    assert _err(b.bsmm_multiply, 1.0, None, None, 0.0, None, 0.0, 0) == b.BSMM_EINVAL


def test_options_round_trip():
    from paper_1910_04796_amd import bsmm as b
    for k, v in [("path", "dense"), ("path", "stack"), ("path", "emul"), ("path", "auto"),
                 ("emul_slices", "5"), ("emul_slices", "7"), ("plan_cache", "1"), ("plan_cache", "0"),
                 ("stack_kernel", "tuned"),
                 ("stack_kernel", "plain"), ("stack_chunk", "30000"), ("stack_chunk", "0"),
                 ("stack_panel", "1000"), ("stack_panel", "0"), ("stack_panel", "1073741824"),
                 ("verbose", "1"), ("verbose", "0"),
                 ("emul_kernel", "t64"), ("emul_kernel", "t128"), ("emul_kernel", "t128w8"), ("emul_kernel", "t128k32"), ("dense_kb", "32"), ("dense_kb", "16")]:
        b.bsmm_set_option(k, v)
        assert b.bsmm_get_option(k) == v
    assert _err(b.bsmm_set_option, "path", "sideways") == b.BSMM_EINVAL
    assert _err(b.bsmm_set_option, "nope", "1") == b.BSMM_EINVAL
    assert _err(b.bsmm_set_option, "stack_chunk", "-4") == b.BSMM_EINVAL
    assert _err(b.bsmm_set_option, "stack_panel", "-1") == b.BSMM_EINVAL
    assert _err(b.bsmm_set_option, "stack_panel", "1e9") == b.BSMM_EINVAL
    assert _err(b.bsmm_set_option, "verbose", "yes") == b.BSMM_EINVAL
    assert _err(b.bsmm_set_option, "emul_kernel", "t96") == b.BSMM_EINVAL


def test_last_error_is_set():
    from paper_1910_04796_amd import bsmm as b
    _err(b.bsmm_set_option, "nope", "1")
    assert "nope" in b.bsmm_last_error()


def test_tuning_database_lookup_by_run_length(tmp_path):
    """Parameter selection from a database file is host work: the entry of a
    shape is the one whose run length is nearest on a log scale, a line
    without a run length counts as R = 8, and absent shapes take the plain
    rule."""
    from paper_1910_04796_amd import bsmm as b
    db = tmp_path / "db.txt"
    db.write_text("# m n k R tm tn kc waves best plain\n"
                  "23 23 23 1 4 4 8 1 1.0 2.0\n"
                  "23 23 23 16 16 16 0 4 1.0 2.0\n"
                  "5 5 5 1 2 4 1\n")
    saved = {o: b.bsmm_get_option(o) for o in ("tune_db", "mlp_weights")}
    b.bsmm_set_option("mlp_weights", "")
    b.bsmm_set_option("tune_db", "")
    plain = b.bsmm_select_params(23, 23, 23, 8)
    b.bsmm_set_option("tune_db", str(db))
    try:
        assert b.bsmm_select_params(23, 23, 23, 1) == (4, 4, 8, 1)
        assert b.bsmm_select_params(23, 23, 23, 3) == (4, 4, 8, 1)   # log2 3 < 2
        assert b.bsmm_select_params(23, 23, 23, 5) == (16, 16, 0, 4)  # log2 5 > 2
        assert b.bsmm_select_params(23, 23, 23, 1000) == (16, 16, 0, 4)
        assert b.bsmm_select_params(5, 5, 5, 64) == (1, 2, 4, 1)
        assert b.bsmm_select_params(13, 13, 13, 8) == b.bsmm_select_params(13, 13, 13, 1)
        assert _err(b.bsmm_select_params, 23, 23, 23, 0) == b.BSMM_EINVAL
        b.bsmm_set_option("tune_db", "")
        assert b.bsmm_select_params(23, 23, 23, 8) == plain
    finally:
        for o, v in saved.items():
            b.bsmm_set_option(o, v)


def test_model_features_of_run_length():
    """The learned model's feature vector is host work; only the last
    feature, log2 of the run length, depends on the run length."""
    from paper_1910_04796_amd import bsmm as b
    p = np.array([16, 16, 0, 4], np.int32)
    f1, f8, f64 = (b.bsmm_mlp_features(23, 13, 7, p, R) for R in (1, 8, 64))
    assert len(f1) == 11
    assert np.array_equal(f1[:-1], f8[:-1]) and np.array_equal(f1[:-1], f64[:-1])
    assert (f1[-1], f8[-1], f64[-1]) == (0.0, 3.0, 6.0)
    assert f1[9] == 1.0  # matrix-core set
    assert b.bsmm_mlp_features(23, 13, 7, np.array([2, 2, 0, 0], np.int32), 8)[9] == 0.0
    # lanes cover m x n; the matrix-core tile also pads k to a multiple of 4
    assert np.isclose(f1[8], (23 * 13) / (2 * 1 * 256) * 7 / 8)


def test_create_range_errors_before_any_device_call():
    """ERANGE is decided from the index alone, before any HIP call (so also
    on a machine without a GPU): 2^47 or more elements, more than 2^31 - 1
    blocks."""
    from paper_1910_04796_amd import bsmm as b
    c = b.bsmm_create_matrix
    assert _err(c, 1, [1 << 24], 1, [1 << 23], 1, [0, 1], [0], None) == b.BSMM_ERANGE
    big = (1 << 31)
    assert _err(c, 1, [1], 1, [1], big, [0, big], [0], None) == b.BSMM_ERANGE
    assert "2^47" in b.bsmm_last_error() or "too many" in b.bsmm_last_error()


def test_create_and_multiply_argument_errors():
    """EINVAL on null arguments and bad option values of the allocator:
    a deallocator is required with an allocator."""
    import ctypes
    from paper_1910_04796_amd import bsmm as b
    st = b._lib.bsmm_create_matrix(1, None, 1, None, 0, None, None, None, 0, None, None)
    assert st == b.BSMM_EINVAL
    st = b._lib.bsmm_set_allocator(b.ALLOC_FN(lambda n, s, c: None), b.DEALLOC_FN(), None)
    assert st == b.BSMM_EINVAL
    assert _err(b.bsmm_multiply, 1.0, None, None, 0.0, None, float("nan"), 0) == b.BSMM_EINVAL
