"""Python face of the CPU reference (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It shares no code with the GPU library.

What it computes (paper, Sec. II, the local multiplication): every output
block is a sum of pairwise products of small dense blocks,
``C(I,J) = beta*C(I,J) + alpha * sum_K A(I,K) B(K,J)``, over the union of
the old C pattern and the symbolic product pattern, followed by the
per-block filter.  The arithmetic lives in ``bsmm_oracle.c``; this file only
marshals arrays and compacts the filtered result.

Matrices are duck-typed: any object with ``rbs`` (int32 block-row sizes),
``cbs`` (int32 block-column sizes), ``row_ptr`` (int64), ``col_ind``
(int32) and ``data`` (float64, blocks packed in CSR order, column-major
inside a block).
"""
import ctypes
import os
from typing import NamedTuple, Optional

import numpy as np

from . import build as _build

_LIBS = {}

_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_f64p = ctypes.POINTER(ctypes.c_double)
_u8p = ctypes.POINTER(ctypes.c_uint8)


class OracleMatrix(NamedTuple):
    rbs: np.ndarray
    cbs: np.ndarray
    row_ptr: np.ndarray
    col_ind: np.ndarray
    data: np.ndarray


def load(mutant: int = 0):
    """Loads (building if absent) the reference library or one of its mutants."""
    if mutant in _LIBS:
        return _LIBS[mutant]
    path = _build.lib_path(mutant)
    if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
        _build.build(mutant)
    lib = ctypes.CDLL(path)
    lib.orc_pattern.argtypes = [ctypes.c_int32, ctypes.c_int32, _i64p, _i32p, _i64p, _i32p,
                                _i64p, _i32p, _i64p, _i32p]
    lib.orc_pattern.restype = ctypes.c_int
    lib.orc_multiply.argtypes = [ctypes.c_double, ctypes.c_double,
                                 ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                 _i32p, _i32p, _i32p,
                                 _i64p, _i32p, _f64p,
                                 _i64p, _i32p, _f64p,
                                 _i64p, _i32p, _f64p,
                                 _i64p, _i32p, _f64p,
                                 ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    lib.orc_multiply.restype = ctypes.c_int
    lib.orc_block_sumsq.argtypes = [ctypes.c_int32, _i32p, _i32p, _i64p, _i32p, _f64p, _f64p]
    lib.orc_block_sumsq.restype = ctypes.c_int
    lib.orc_filter_keep.argtypes = [ctypes.c_int64, _f64p, ctypes.c_double, _u8p]
    lib.orc_filter_keep.restype = ctypes.c_int
    _LIBS[mutant] = lib
    return lib


def _p(a, t):
    if a is None:
        return None
    return a.ctypes.data_as(t)


def _arrays(M):
    return (np.ascontiguousarray(M.rbs, dtype=np.int32), np.ascontiguousarray(M.cbs, dtype=np.int32),
            np.ascontiguousarray(M.row_ptr, dtype=np.int64), np.ascontiguousarray(M.col_ind, dtype=np.int32),
            np.ascontiguousarray(M.data, dtype=np.float64))


def check_compatible(A, B, C=None):
    """Shape rules of the local multiply: A's block columns are B's block rows
    (sizes compared elementwise), C is A-rows by B-columns."""
    if len(A.cbs) != len(B.rbs) or np.any(np.asarray(A.cbs) != np.asarray(B.rbs)):
        raise ValueError("A block columns do not match B block rows")
    if C is not None:
        if (len(C.rbs) != len(A.rbs) or np.any(np.asarray(C.rbs) != np.asarray(A.rbs))
                or len(C.cbs) != len(B.cbs) or np.any(np.asarray(C.cbs) != np.asarray(B.cbs))):
            raise ValueError("C block sizes do not match A rows x B columns")


def pattern(A, B, C=None, mutant: int = 0, rows: Optional[tuple] = None):
    """Output pattern: old C pattern united with {(I,J): some K has A(I,K), B(K,J)}.

    rows=(r0, r1) computes block rows [r0, r1) only (every other row is
    returned empty): each output row depends on its own A and C rows alone.
    """
    lib = load(mutant)
    check_compatible(A, B, C)
    a = _arrays(A)
    b = _arrays(B)
    nbr, nbc = len(a[0]), len(b[1])
    r0, r1 = (0, nbr) if rows is None else (int(rows[0]), int(rows[1]))
    if not (0 <= r0 <= r1 <= nbr):
        raise ValueError("row range out of bounds")
    a_rp = a[2][r0:r1 + 1] - a[2][r0]
    a_ci = a[3][a[2][r0]:a[2][r1]]
    c_rp = c_ci = None
    if C is not None:
        c = _arrays(C)
        c_rp = c[2][r0:r1 + 1] - c[2][r0]
        c_ci = c[3][c[2][r0]:c[2][r1]]
    n = r1 - r0
    rp = np.zeros(n + 1, dtype=np.int64)
    st = lib.orc_pattern(n, nbc, _p(a_rp, _i64p), _p(a_ci, _i32p), _p(b[2], _i64p), _p(b[3], _i32p),
                         _p(c_rp, _i64p), _p(c_ci, _i32p), _p(rp, _i64p), None)
    if st:
        raise MemoryError("reference pattern: out of memory")
    ci = np.zeros(max(int(rp[-1]), 1), dtype=np.int32)
    st = lib.orc_pattern(n, nbc, _p(a_rp, _i64p), _p(a_ci, _i32p), _p(b[2], _i64p), _p(b[3], _i32p),
                         _p(c_rp, _i64p), _p(c_ci, _i32p), _p(rp, _i64p), _p(ci, _i32p))
    if st:
        raise MemoryError("reference pattern: out of memory")
    full = np.concatenate([np.zeros(r0, np.int64), rp, np.full(nbr - r1, rp[-1], np.int64)])
    return full, ci[: int(rp[-1])]


def block_sizes(rbs, cbs, row_ptr, col_ind):
    """Element count of every block, in CSR order."""
    rows = np.repeat(np.arange(len(rbs)), np.diff(row_ptr))
    return np.asarray(rbs, dtype=np.int64)[rows] * np.asarray(cbs, dtype=np.int64)[col_ind]


def block_sumsq(M, mutant: int = 0):
    lib = load(mutant)
    rbs, cbs, rp, ci, data = _arrays(M)
    out = np.zeros(max(int(rp[-1]), 1), dtype=np.float64)
    st = lib.orc_block_sumsq(len(rbs), _p(rbs, _i32p), _p(cbs, _i32p), _p(rp, _i64p), _p(ci, _i32p),
                             _p(data, _f64p), _p(out, _f64p))
    if st:
        raise MemoryError("reference block norms: out of memory")
    return out[: int(rp[-1])]


def apply_filter(M, eps: float, mutant: int = 0) -> OracleMatrix:
    """Drops every block whose squared Frobenius norm is strictly below eps^2
    (only when eps > 0) and compacts index and data."""
    lib = load(mutant)
    rbs, cbs, rp, ci, data = _arrays(M)
    n = int(rp[-1])
    s = block_sumsq(M, mutant)
    keep = np.zeros(max(n, 1), dtype=np.uint8)
    lib.orc_filter_keep(n, _p(s, _f64p), float(eps), _p(keep, _u8p))
    keep = keep[:n].astype(bool)
    sizes = block_sizes(rbs, cbs, rp, ci)
    elem_keep = np.repeat(keep, sizes)
    rows = np.repeat(np.arange(len(rbs)), np.diff(rp))
    new_counts = np.bincount(rows[keep], minlength=len(rbs))
    new_rp = np.zeros(len(rbs) + 1, dtype=np.int64)
    np.cumsum(new_counts, out=new_rp[1:])
    return OracleMatrix(rbs, cbs, new_rp, ci[keep].astype(np.int32), data[elem_keep])


def multiply(alpha: float, A, B, beta: float, C=None, filter_eps: float = 0.0, *,
             rows: Optional[tuple] = None, compensated: bool = False, nthreads: int = 0,
             mutant: int = 0) -> OracleMatrix:
    """C_out = filter_eps(beta*C + alpha*A*B) in block-CSR.

    rows=(r0, r1) restricts the numeric phase to block rows [r0, r1); the
    result then holds only those rows (its ``rbs`` is the slice).
    """
    if not (filter_eps >= 0.0):
        raise ValueError("filter_eps must be >= 0")
    lib = load(mutant)
    check_compatible(A, B, C)
    a = _arrays(A)
    b = _arrays(B)
    nbr, nbk, nbc = len(a[0]), len(b[0]), len(b[1])
    c = _arrays(C) if C is not None else (None,) * 5
    r0, r1 = (0, nbr) if rows is None else (int(rows[0]), int(rows[1]))
    if not (0 <= r0 <= r1 <= nbr):
        raise ValueError("row range out of bounds")
    o_rp, o_ci = pattern(A, B, C, mutant, rows=(r0, r1))
    sizes = block_sizes(a[0], b[1], o_rp, o_ci)
    nelem = int(sizes[o_rp[r0]:o_rp[r1]].sum())
    o_data = np.zeros(max(nelem, 1), dtype=np.float64)
    if r1 > r0:
        st = lib.orc_multiply(float(alpha), float(beta), nbr, nbk, nbc,
                              _p(a[0], _i32p), _p(b[0], _i32p), _p(b[1], _i32p),
                              _p(a[2], _i64p), _p(a[3], _i32p), _p(a[4], _f64p),
                              _p(b[2], _i64p), _p(b[3], _i32p), _p(b[4], _f64p),
                              _p(c[2], _i64p), _p(c[3], _i32p), _p(c[4], _f64p),
                              _p(o_rp, _i64p), _p(o_ci, _i32p), _p(o_data, _f64p),
                              r0, r1, 1 if compensated else 0, int(nthreads))
        if st:
            raise MemoryError("reference multiply: out of memory")
    sub_rp = o_rp[r0:r1 + 1] - o_rp[r0]
    sub = OracleMatrix(a[0][r0:r1], b[1], sub_rp, o_ci[o_rp[r0]:o_rp[r1]], o_data[:nelem])
    if filter_eps > 0.0:
        sub = apply_filter(sub, filter_eps, mutant)
    return sub


def to_dense(M) -> np.ndarray:
    """Dense FP64 matrix of a block-CSR matrix (absent blocks are zero)."""
    rbs = np.asarray(M.rbs, dtype=np.int64)
    cbs = np.asarray(M.cbs, dtype=np.int64)
    ro = np.concatenate([[0], np.cumsum(rbs)])
    co = np.concatenate([[0], np.cumsum(cbs)])
    D = np.zeros((int(ro[-1]), int(co[-1])), dtype=np.float64)
    off = 0
    for i in range(len(rbs)):
        for p in range(int(M.row_ptr[i]), int(M.row_ptr[i + 1])):
            j = int(M.col_ind[p])
            m, n = int(rbs[i]), int(cbs[j])
            D[ro[i]:ro[i] + m, co[j]:co[j] + n] = np.asarray(M.data[off:off + m * n]).reshape(n, m).T
            off += m * n
    return D


def rel_err(X: np.ndarray, R: np.ndarray) -> float:
    """||X - R||_F / ||R||_F with the squares summed in extended precision;
    the absolute error when ||R||_F == 0."""
    d = (np.asarray(X, dtype=np.float64) - np.asarray(R, dtype=np.float64)).ravel().astype(np.longdouble)
    r = np.asarray(R, dtype=np.float64).ravel().astype(np.longdouble)
    num = np.sqrt(np.sum(d * d))
    den = np.sqrt(np.sum(r * r))
    return float(num / den) if den > 0 else float(num)


def densified_panel_shapes(M: int, N: int, K: int, p_tilde: int, t: int):
    """Densified block shapes of Sec. III, Eqs. (1)-(2): A is
    (M / (t * Pt)) x (K / Pt) and B is (K / Pt) x (N / Pt) on a Pt x Pt rank
    grid with t threads per rank.  Non-integral shapes raise ValueError."""
    if M % (t * p_tilde) or K % p_tilde or N % p_tilde:
        raise ValueError("sizes not divisible by the grid")
    return (M // (t * p_tilde), K // p_tilde), (K // p_tilde, N // p_tilde)
