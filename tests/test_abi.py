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


def test_multiply_rejects_null_handles():
    from paper_1910_04796_amd import bsmm as b
    assert _err(b.bsmm_multiply, 1.0, None, None, 0.0, None, 0.0, 0) == b.BSMM_EINVAL


def test_options_round_trip():
    from paper_1910_04796_amd import bsmm as b
    for k, v in [("path", "dense"), ("path", "stack"), ("path", "emul"), ("path", "auto"),
                 ("emul_slices", "5"), ("emul_slices", "7"), ("plan_cache", "1"), ("plan_cache", "0"),
                 ("stack_kernel", "tuned"),
                 ("stack_kernel", "plain"), ("stack_chunk", "30000"), ("stack_chunk", "0"),
                 ("emul_kernel", "t64"), ("emul_kernel", "t128"), ("emul_kernel", "t128w8"), ("emul_kernel", "t128k32"), ("dense_kb", "32"), ("dense_kb", "16")]:
        b.bsmm_set_option(k, v)
        assert b.bsmm_get_option(k) == v
    assert _err(b.bsmm_set_option, "path", "sideways") == b.BSMM_EINVAL
    assert _err(b.bsmm_set_option, "nope", "1") == b.BSMM_EINVAL
    assert _err(b.bsmm_set_option, "stack_chunk", "-4") == b.BSMM_EINVAL
    assert _err(b.bsmm_set_option, "emul_kernel", "t96") == b.BSMM_EINVAL


def test_last_error_is_set():
    from paper_1910_04796_amd import bsmm as b
    _err(b.bsmm_set_option, "nope", "1")
    assert "nope" in b.bsmm_last_error()
