"""ctypes binding of libbsmm (include/bsmm.h): argument marshalling only.

Every function keeps the C name and raises ``BsmmError`` on a non-zero
status.  All computation happens in the HIP library; PyTorch is used only
for device memory (the caching allocator, registered through
``use_torch_allocator``) and streams.  Importing this module fails loudly
when the library has not been built.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbsmm.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libbsmm.so not found at {LIB_PATH}; build it with "
                      "`python -c 'import __graft_entry__ as g; g.build()'`")

# One HIP runtime per process: PyTorch ships its own HIP runtime, and a
# second runtime initialised in the same process sees no device.  Loading
# torch first makes the dynamic loader bind libbsmm's libamdhip64.so.7
# dependency to the copy torch already holds (same SONAME), so device
# memory and streams from torch are valid in the library.
try:
    import torch as _torch  # noqa: F401
except ImportError:  # plain C-ABI use without PyTorch: the system runtime
    _torch = None

_lib = ctypes.CDLL(LIB_PATH)

# Tuning results shipped with the package for gfx950 (tuning database and
# learned-model weights); the tuned path reads them by default.
DEFAULT_TUNE_DB = os.path.join(_HERE, "tune_db", "gfx950.txt")
DEFAULT_MLP = os.path.join(_HERE, "tune_db", "gfx950_mlp.txt")

BSMM_OK, BSMM_EINVAL, BSMM_ESHAPE, BSMM_EINDEX = 0, -1, -2, -3
BSMM_ENOMEM, BSMM_EDEVICE, BSMM_ERANGE, BSMM_ENOTSUP = -4, -5, -6, -7
BSMM_F64, BSMM_F32 = 0, 1
DTYPES = {"f64": BSMM_F64, "f32": BSMM_F32}
NP_DTYPES = {BSMM_F64: np.float64, BSMM_F32: np.float32}
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ESHAPE", -3: "EINDEX", -4: "ENOMEM",
                -5: "EDEVICE", -6: "ERANGE", -7: "ENOTSUP"}

_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_f64p = ctypes.POINTER(ctypes.c_double)

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
DEALLOC_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)


class bsmm_multiply_stats(ctypes.Structure):
    _fields_ = [("path", ctypes.c_int32), ("n_classes", ctypes.c_int32),
                ("n_products", ctypes.c_int64), ("n_runs", ctypes.c_int64),
                ("c_nnzb_before", ctypes.c_int64), ("c_nnzb_after", ctypes.c_int64),
                ("flops", ctypes.c_double), ("n_row_panels", ctypes.c_int64),
                ("n_sched_runs", ctypes.c_int64), ("n_jit_classes", ctypes.c_int64),
                ("n_screened", ctypes.c_int64), ("n_products_run", ctypes.c_int64)]


_lib.bsmm_create_matrix.argtypes = [_i32, _i32p, _i32, _i32p, _i64, _i64p, _i32p, _vp, ctypes.c_int,
                                    _vp, ctypes.POINTER(_vp)]
_lib.bsmm_create_matrix_typed.argtypes = [_i32, _i32p, _i32, _i32p, _i64, _i64p, _i32p, _i32, _vp,
                                          ctypes.c_int, _vp, ctypes.POINTER(_vp)]
_lib.bsmm_matrix_dtype.argtypes = [_vp, _i32p]
_lib.bsmm_copy_out_typed.argtypes = [_vp, _i64p, _i32p, _vp, ctypes.c_int, _vp]
_lib.bsmm_multiply.argtypes = [ctypes.c_double, _vp, _vp, ctypes.c_double, _vp, ctypes.c_double, _vp]
_lib.bsmm_multiply_noalloc.argtypes = [ctypes.c_double, _vp, _vp, ctypes.c_double, _vp, _vp]
_lib.bsmm_destroy_matrix.argtypes = [_vp]
_lib.bsmm_matrix_info.argtypes = [_vp, _i32p, _i32p, _i64p, _i64p]
_lib.bsmm_copy_out.argtypes = [_vp, _i64p, _i32p, _vp, ctypes.c_int, _vp]
_lib.bsmm_set_allocator.argtypes = [ALLOC_FN, DEALLOC_FN, _vp]
_lib.bsmm_set_option.argtypes = [ctypes.c_char_p, ctypes.c_char_p]
_lib.bsmm_get_option.argtypes = [ctypes.c_char_p, ctypes.c_char_p, ctypes.c_size_t]
_lib.bsmm_last_error.restype = ctypes.c_char_p
_lib.bsmm_last_error.argtypes = []
_lib.bsmm_last_stats.argtypes = [ctypes.POINTER(bsmm_multiply_stats)]
_lib.bsmm_inspect_stacks.argtypes = [_vp, _vp, _vp, _i64p, _i64p, _i64p, _i32p, _i64p, _i64p, _i64p, _vp]
_lib.bsmm_kernel_times.argtypes = [_f64p, _i64p, _f64p, _i64p, ctypes.c_int]
_lib.bsmm_jit_stats.argtypes = [_i64p, _i64p, _i64p, _f64p]
_lib.bsmm_measure_peaks.argtypes = [_f64p, _f64p, _f64p, _f64p, _f64p, _f64p, _f64p, _i64, _vp]
_lib.bsmm_tune_candidates.argtypes = [_i32, _i32, _i32, _i32p, _i32p]
_lib.bsmm_tune_shape.argtypes = [_i32, _i32, _i32, _i64, _i32, _i32, _i32p, _i32, _f64p, _vp]
_lib.bsmm_select_params.argtypes = [_i32, _i32, _i32, _i32, _i32p]
_f32p = ctypes.POINTER(ctypes.c_float)
_lib.bsmm_mlp_param_count.argtypes = [_i32, _i64p]
_lib.bsmm_mlp_features.argtypes = [_i32, _i32, _i32, _i32, _i32p, _f32p, _i32p]
_lib.bsmm_mlp_forward.argtypes = [_i32, _f32p, _i64, _f32p, _f32p]
_lib.bsmm_mlp_grad.argtypes = [_i32, _f32p, _i64, _f32p, _f32p, _f32p, _f32p]
_lib.bsmm_mlp_adam_step.argtypes = [_i32, _f32p, _f32p, _f32p, _f32p, _i32, ctypes.c_float,
                                    ctypes.c_float, ctypes.c_float, ctypes.c_float]
_lib.bsmm_mlp_train.argtypes = [_i32, _f32p, _i64, _f32p, _f32p, _i32, _i32, ctypes.c_float,
                                ctypes.c_uint64, _f32p]
for _f in ("bsmm_mlp_param_count", "bsmm_mlp_features", "bsmm_mlp_forward", "bsmm_mlp_grad",
           "bsmm_mlp_adam_step", "bsmm_mlp_train","bsmm_tune_candidates", "bsmm_tune_shape", "bsmm_select_params", "bsmm_kernel_times", "bsmm_jit_stats", "bsmm_measure_peaks", "bsmm_create_matrix", "bsmm_multiply", "bsmm_multiply_noalloc", "bsmm_destroy_matrix",
           "bsmm_matrix_info", "bsmm_copy_out", "bsmm_create_matrix_typed", "bsmm_matrix_dtype",
           "bsmm_copy_out_typed", "bsmm_set_allocator", "bsmm_set_option", "bsmm_get_option",
           "bsmm_last_stats", "bsmm_inspect_stacks"):
    getattr(_lib, _f).restype = ctypes.c_int

EXPORTED = ("bsmm_create_matrix", "bsmm_create_matrix_typed", "bsmm_matrix_dtype", "bsmm_copy_out_typed",
            "bsmm_multiply", "bsmm_multiply_noalloc", "bsmm_destroy_matrix", "bsmm_matrix_info",
            "bsmm_copy_out", "bsmm_set_allocator", "bsmm_set_option", "bsmm_get_option",
            "bsmm_last_error", "bsmm_last_stats", "bsmm_inspect_stacks", "bsmm_kernel_times", "bsmm_jit_stats",
            "bsmm_measure_peaks",
            "bsmm_tune_candidates", "bsmm_tune_shape", "bsmm_select_params",
            "bsmm_mlp_param_count", "bsmm_mlp_features", "bsmm_mlp_forward", "bsmm_mlp_grad",
            "bsmm_mlp_adam_step", "bsmm_mlp_train")


class BsmmError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def _check(st):
    if st != BSMM_OK:
        raise BsmmError(st, bsmm_last_error())


def _stream(stream):
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        except ImportError:
            pass
        return ctypes.c_void_p(0)
    if hasattr(stream, "cuda_stream"):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def _arr(a, dtype):
    return np.ascontiguousarray(np.asarray(a), dtype=dtype)


def _ptr(a, t):
    return a.ctypes.data_as(t) if a is not None and a.size > 0 else ctypes.cast(None, t)


def bsmm_last_error():
    return _lib.bsmm_last_error().decode()


def bsmm_create_matrix(nbr, row_blk_sizes, nbc, col_blk_sizes, nnzb, blk_row_ptr, blk_col_ind,
                       data=None, data_on_device=None, stream=None, dtype="f64"):
    """Returns an opaque handle (int).  ``data`` is a numpy array (host), a
    torch CUDA tensor (device), or None for zeros; ``dtype`` "f64" or "f32"
    (host data are converted to it, device data must already be of it)."""
    code = DTYPES[dtype]
    npt = NP_DTYPES[code]
    rbs = _arr(row_blk_sizes, np.int32)
    cbs = _arr(col_blk_sizes, np.int32)
    rp = _arr(blk_row_ptr, np.int64)
    ci = _arr(blk_col_ind, np.int32)
    keep = None
    if data is None:
        dptr, on_dev = None, 0
    elif hasattr(data, "data_ptr"):
        keep = data.contiguous()
        dptr, on_dev = keep.data_ptr(), 1 if keep.is_cuda else 0
        if not on_dev:
            keep = keep.numpy().astype(npt, copy=False)
            dptr = keep.ctypes.data
    else:
        keep = _arr(data, npt)
        dptr, on_dev = (keep.ctypes.data if keep.size else None), 0
    if data_on_device is not None:
        on_dev = int(bool(data_on_device))
    h = ctypes.c_void_p()
    st = _lib.bsmm_create_matrix_typed(int(nbr), _ptr(rbs, _i32p), int(nbc), _ptr(cbs, _i32p), int(nnzb),
                                       rp.ctypes.data_as(_i64p), _ptr(ci, _i32p), code, dptr, on_dev,
                                       _stream(stream), ctypes.byref(h))
    _check(st)
    return h.value


def bsmm_multiply(alpha, A, B, beta, C, filter_eps=0.0, stream=None):
    _check(_lib.bsmm_multiply(float(alpha), A, B, float(beta), C, float(filter_eps), _stream(stream)))


def bsmm_multiply_noalloc(alpha, A, B, beta, C, stream=None):
    _check(_lib.bsmm_multiply_noalloc(float(alpha), A, B, float(beta), C, _stream(stream)))


def bsmm_destroy_matrix(m):
    _check(_lib.bsmm_destroy_matrix(m))


def bsmm_matrix_info(m):
    nbr, nbc, nnzb, ne = _i32(), _i32(), _i64(), _i64()
    _check(_lib.bsmm_matrix_info(m, ctypes.byref(nbr), ctypes.byref(nbc), ctypes.byref(nnzb),
                                 ctypes.byref(ne)))
    return nbr.value, nbc.value, nnzb.value, ne.value


def bsmm_matrix_dtype(m):
    d = _i32()
    _check(_lib.bsmm_matrix_dtype(m, ctypes.byref(d)))
    return d.value


def bsmm_copy_out(m, stream=None, device_out=None):
    """Returns (row_ptr, col_ind, data) as numpy arrays, data in the matrix's
    element type; with ``device_out`` (a CUDA tensor of nelems elements of
    that type) the data go there instead."""
    nbr, nbc, nnzb, ne = bsmm_matrix_info(m)
    rp = np.zeros(nbr + 1, dtype=np.int64)
    ci = np.zeros(max(nnzb, 1), dtype=np.int32)
    if device_out is not None:
        _check(_lib.bsmm_copy_out_typed(m, rp.ctypes.data_as(_i64p), ci.ctypes.data_as(_i32p),
                                        ctypes.c_void_p(device_out.data_ptr()), 1, _stream(stream)))
        return rp, ci[:nnzb], device_out
    data = np.zeros(max(ne, 1), dtype=NP_DTYPES[bsmm_matrix_dtype(m)])
    _check(_lib.bsmm_copy_out_typed(m, rp.ctypes.data_as(_i64p), ci.ctypes.data_as(_i32p),
                                    ctypes.c_void_p(data.ctypes.data), 0, _stream(stream)))
    return rp, ci[:nnzb], data[:ne]


_alloc_keepalive = []


def bsmm_set_allocator(alloc=None, dealloc=None, ctx=None):
    """Registers Python callables alloc(nbytes, stream) -> int pointer and
    dealloc(ptr, nbytes, stream); no arguments restores hipMalloc/hipFree."""
    if alloc is None:
        _check(_lib.bsmm_set_allocator(ALLOC_FN(), DEALLOC_FN(), None))
        _alloc_keepalive.clear()
        return

    def _a(nbytes, stream, _ctx):
        try:
            return int(alloc(int(nbytes), stream or 0)) or None
        except Exception:  # the C side turns NULL into ENOMEM
            return None

    def _d(ptr, nbytes, stream, _ctx):
        try:
            dealloc(ptr, int(nbytes), stream or 0)
        except Exception:
            pass

    fa, fd = ALLOC_FN(_a), DEALLOC_FN(_d)
    _check(_lib.bsmm_set_allocator(fa, fd, None))
    _alloc_keepalive[:] = [fa, fd]


def use_torch_allocator(device=None):
    """Device memory of the library comes from PyTorch's caching allocator."""
    import torch
    dev = torch.cuda.current_device() if device is None else device

    def alloc(nbytes, stream):
        return torch.cuda.caching_allocator_alloc(nbytes, dev, stream if stream else None)

    def dealloc(ptr, nbytes, stream):
        torch.cuda.caching_allocator_delete(ptr)

    bsmm_set_allocator(alloc, dealloc)


def bsmm_set_option(key, value):
    _check(_lib.bsmm_set_option(str(key).encode(), str(value).encode()))


def bsmm_get_option(key):
    buf = ctypes.create_string_buffer(4096)
    _check(_lib.bsmm_get_option(str(key).encode(), buf, 4096))
    return buf.value.decode()


def bsmm_last_stats():
    s = bsmm_multiply_stats()
    _check(_lib.bsmm_last_stats(ctypes.byref(s)))
    return {f: getattr(s, f) for f, _ in bsmm_multiply_stats._fields_}


def bsmm_inspect_stacks(A, B, C, stream=None):
    nr, npr = _i64(0), _i64(0)
    _check(_lib.bsmm_inspect_stacks(A, B, C, ctypes.byref(nr), ctypes.byref(npr), None, None, None,
                                    None, None, _stream(stream)))
    run_cblk = np.zeros(max(nr.value, 1), np.int64)
    run_class = np.zeros(max(nr.value, 1), np.int32)
    run_ptr = np.zeros(nr.value + 1, np.int64)
    pa = np.zeros(max(npr.value, 1), np.int64)
    pb = np.zeros(max(npr.value, 1), np.int64)
    _check(_lib.bsmm_inspect_stacks(A, B, C, ctypes.byref(nr), ctypes.byref(npr),
                                    run_cblk.ctypes.data_as(_i64p), run_class.ctypes.data_as(_i32p),
                                    run_ptr.ctypes.data_as(_i64p), pa.ctypes.data_as(_i64p),
                                    pb.ctypes.data_as(_i64p), _stream(stream)))
    n, p = nr.value, npr.value
    return {"run_cblk": run_cblk[:n], "run_class": run_class[:n], "run_ptr": run_ptr,
            "prod_ablk": pa[:p], "prod_bblk": pb[:p]}


def bsmm_kernel_times(reset=True):
    """(gemm_ms, gemm_launches, stack_ms, stack_launches) of the launches
    recorded while the option time_kernels is 1."""
    gm, gn, sm, sn = ctypes.c_double(), _i64(), ctypes.c_double(), _i64()
    _check(_lib.bsmm_kernel_times(ctypes.byref(gm), ctypes.byref(gn), ctypes.byref(sm),
                                  ctypes.byref(sn), 1 if reset else 0))
    return gm.value, gn.value, sm.value, sn.value


def bsmm_jit_stats():
    """(compiled, cache_hits, failures, compile_ms) of the run-time compiled
    kernels (option jit)."""
    c, h, f, ms = _i64(), _i64(), _i64(), ctypes.c_double()
    _check(_lib.bsmm_jit_stats(ctypes.byref(c), ctypes.byref(h), ctypes.byref(f), ctypes.byref(ms)))
    return c.value, h.value, f.value, ms.value


def bsmm_measure_peaks(copy_bytes=1 << 31, stream=None):
    """Measured device rates: dict of fp64_mfma, fp32_mfma (TFLOP/s),
    int8_mfma (TOP/s), bf16_mfma, fp64_valu (TFLOP/s), hbm_gbs (copy, read +
    write) and hbm_read_gbs (GB/s)."""
    v = [ctypes.c_double() for _ in range(7)]
    _check(_lib.bsmm_measure_peaks(*[ctypes.byref(x) for x in v], int(copy_bytes), _stream(stream)))
    return dict(zip(("fp64_mfma", "fp32_mfma", "int8_mfma", "bf16_mfma", "fp64_valu", "hbm_gbs",
                     "hbm_read_gbs"), (x.value for x in v)))


def bsmm_tune_candidates(m, n, k):
    """Legal parameter sets (tm, tn, kc, waves) of shape (m, n, k), as an
    int32 array of shape (count, 4)."""
    cnt = _i32(0)
    _check(_lib.bsmm_tune_candidates(m, n, k, ctypes.byref(cnt), None))
    out = np.zeros((max(cnt.value, 1), 4), np.int32)
    _check(_lib.bsmm_tune_candidates(m, n, k, ctypes.byref(cnt), out.ctypes.data_as(_i32p)))
    return out[:cnt.value]


def bsmm_tune_shape(m, n, k, cands, n_runs=3750, run_len=8, reps=5, stream=None):
    """Median microseconds of every candidate on a synthetic stack."""
    c = np.ascontiguousarray(cands, dtype=np.int32).reshape(-1, 4)
    out = np.zeros(max(len(c), 1), np.float64)
    _check(_lib.bsmm_tune_shape(m, n, k, n_runs, run_len, len(c), c.ctypes.data_as(_i32p), reps,
                                out.ctypes.data_as(_f64p), _stream(stream)))
    return out[:len(c)]


def bsmm_select_params(m, n, k, run_len=8):
    """Parameters of the tuned path for (m, n, k) in runs of about run_len
    products per C block."""
    p = np.zeros(4, np.int32)
    _check(_lib.bsmm_select_params(m, n, k, run_len, p.ctypes.data_as(_i32p)))
    return tuple(int(x) for x in p)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def bsmm_mlp_param_count(n_features):
    c = _i64()
    _check(_lib.bsmm_mlp_param_count(n_features, ctypes.byref(c)))
    return c.value


def bsmm_mlp_features(m, n, k, params4, run_len=8):
    p = np.ascontiguousarray(params4, dtype=np.int32)
    out = np.zeros(32, np.float32)
    nf = _i32()
    _check(_lib.bsmm_mlp_features(m, n, k, run_len, p.ctypes.data_as(_i32p), out.ctypes.data_as(_f32p),
                                  ctypes.byref(nf)))
    return out[:nf.value]


def bsmm_mlp_forward(params, x):
    x = _f32(x)
    P = _f32(params)
    y = np.zeros(max(len(x), 1), np.float32)
    _check(_lib.bsmm_mlp_forward(x.shape[1], P.ctypes.data_as(_f32p), len(x), x.ctypes.data_as(_f32p),
                                 y.ctypes.data_as(_f32p)))
    return y[:len(x)]


def bsmm_mlp_grad(params, x, t):
    x, t, P = _f32(x), _f32(t), _f32(params)
    g = np.zeros_like(P)
    loss = ctypes.c_float()
    _check(_lib.bsmm_mlp_grad(x.shape[1], P.ctypes.data_as(_f32p), len(x), x.ctypes.data_as(_f32p),
                              t.ctypes.data_as(_f32p), g.ctypes.data_as(_f32p), ctypes.byref(loss)))
    return g, loss.value


def bsmm_mlp_adam_step(n_features, params, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999,
                       eps=1e-8):
    """In-place update of params, m, v (float32 arrays)."""
    g = _f32(grad)
    for a in (params, m, v):
        assert a.dtype == np.float32 and a.flags.c_contiguous
    _check(_lib.bsmm_mlp_adam_step(n_features, params.ctypes.data_as(_f32p), g.ctypes.data_as(_f32p),
                                   m.ctypes.data_as(_f32p), v.ctypes.data_as(_f32p), step, lr, beta1,
                                   beta2, eps))


def bsmm_mlp_train(params, x, t, epochs=30, batch=256, lr=1e-3, seed=0):
    """Returns (trained params, final mean squared error)."""
    x, t = _f32(x), _f32(t)
    P = _f32(params).copy()
    loss = ctypes.c_float()
    _check(_lib.bsmm_mlp_train(x.shape[1], P.ctypes.data_as(_f32p), len(x), x.ctypes.data_as(_f32p),
                               t.ctypes.data_as(_f32p), epochs, batch, lr, seed, ctypes.byref(loss)))
    return P, loss.value


def use_default_tuning():
    """Points the tuned path at the shipped database and model (if present)."""
    if os.path.exists(DEFAULT_TUNE_DB):
        bsmm_set_option("tune_db", DEFAULT_TUNE_DB)
    if os.path.exists(DEFAULT_MLP):
        bsmm_set_option("mlp_weights", DEFAULT_MLP)


class HostBlockCSR:
    """Host copy of a matrix (numpy arrays)."""

    def __init__(self, rbs, cbs, row_ptr, col_ind, data):
        self.rbs, self.cbs, self.row_ptr, self.col_ind, self.data = rbs, cbs, row_ptr, col_ind, data


class Matrix:
    """Owning wrapper of a bsmm handle."""

    def __init__(self, handle, rbs, cbs, dtype="f64"):
        self.handle = handle
        self.rbs = np.asarray(rbs, dtype=np.int32)
        self.cbs = np.asarray(cbs, dtype=np.int32)
        self.dtype = dtype

    @classmethod
    def from_blocks(cls, M, stream=None, data=None, dtype="f64"):
        """From any object with rbs, cbs, row_ptr, col_ind, data attributes."""
        d = M.data if data is None else data
        h = bsmm_create_matrix(len(M.rbs), M.rbs, len(M.cbs), M.cbs, int(np.asarray(M.row_ptr)[-1]),
                               M.row_ptr, M.col_ind, d, stream=stream, dtype=dtype)
        return cls(h, M.rbs, M.cbs, dtype)

    @classmethod
    def empty(cls, rbs, cbs, stream=None, dtype="f64"):
        """A matrix with no stored blocks."""
        rp = np.zeros(len(rbs) + 1, dtype=np.int64)
        h = bsmm_create_matrix(len(rbs), rbs, len(cbs), cbs, 0, rp, np.zeros(0, np.int32), None,
                               stream=stream, dtype=dtype)
        return cls(h, rbs, cbs, dtype)

    def info(self):
        return bsmm_matrix_info(self.handle)

    def to_host(self, stream=None):
        rp, ci, data = bsmm_copy_out(self.handle, stream)
        return HostBlockCSR(self.rbs, self.cbs, rp, ci, data)

    def close(self):
        if self.handle:
            bsmm_destroy_matrix(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def multiply(alpha, A, B, beta, C, filter_eps=0.0, stream=None):
    """C <- filter_eps(beta*C + alpha*A*B) on Matrix objects."""
    bsmm_multiply(alpha, A.handle, B.handle, beta, C.handle, filter_eps, stream)


use_default_tuning()
