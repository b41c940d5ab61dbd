#!/usr/bin/env python3
"""Benchmark of the local block-sparse FP64 multiply on one MI355X.

Headline workload (one step = one full bsmm_multiply, inputs resident in HBM):
the banded product of uneven blocks, N ~ 50,000 with block-row and
block-column sizes drawn from {5, 13, 23, 32}, 30 % of the block positions
stored, magnitudes decaying as exp(-|I-J|/50), blocks whose magnitude
envelope falls below 1e-10 not stored, C = 1.0 * A * B with the result
filtered at eps = 1e-10.  `value` is the FP64-equivalent GFLOP/s (sum of
2 m n k over the block products per second) of the tuned stack path; the
plain stack path on the same inputs is reported beside it.

Further legs (extra JSON fields, each with a warm-up and median/min over
repeated multiplies): the dense N = 8192 product in 32-blocks (densified
GEMM, blocked plain and tuned, INT8 split-precision emulation), the
split-precision workload N = 16384 (native vs emulated), the banded product
at 1 % and 10 %, the 460 x 460 sparse case's latency, FP32 matrices (dense
and banded), and the learned model deciding for block sizes absent from the
tuning database.  The CPU
reference is timed on a bounded sample of the headline workload and checks
the GPU results on those rows.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FP64-equiv GFLOP/s of local C+=A·B, tuned/emulated vs plain, rel err≤1e-12"
PEAK_FP64_TFLOPS = 78.6       # MI355X FP64 matrix and vector peak
PEAK_HBM_GBS = 8000.0         # MI355X HBM3E bandwidth
PEAK_FP32_TFLOPS = 157.3      # MI355X FP32 matrix and vector peak
HEADLINE_OCC = 0.30
HEADLINE_EPS = 1e-10
HEADLINE_NAME = "banded_uneven_n50000_b5-13-23-32_occ30_eps1e-10"
SAMPLE_ROWS = 64              # CPU baseline: contiguous block rows of the headline C


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def set_opts(bsmm, **kw):
    for k, v in kw.items():
        bsmm.bsmm_set_option(k, str(v))


def timed(torch, fn, reps):
    """Wall time per call of fn (ms) over reps calls, bracketed by device syncs."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / reps


def timed_calls(torch, fn, warmup, reps):
    """Each call bracketed by device syncs: median, min, max and mean (ms)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t0) * 1e3)
    return {"median_ms": round(float(np.median(ts)), 4), "min_ms": round(min(ts), 4),
            "max_ms": round(max(ts), 4), "mean_ms": round(float(np.mean(ts)), 4),
            "reps": reps, "warmup": warmup}


def gflops(F, ms):
    return round(F / (ms * 1e-3) / 1e9, 1)


def profile_json(name, src, products_run=None):
    """A committed counter summary, valid only while the kernel source is
    unchanged since the counters were taken (and, when given, the launch ran
    the same number of block products)."""
    path = os.path.join(ROOT, "profiles", name)
    try:
        with open(path) as f:
            t = json.load(f)
        sha = hashlib.sha256(open(os.path.join(ROOT, src), "rb").read()).hexdigest()
        if t.get("source_sha256") != sha:
            return None
        if products_run is not None and t.get("products_run") != products_run:
            return None
        return t
    except (OSError, ValueError):
        return None


def mfma_padding(A, B):
    """Algorithmic flops F = sum 2 m n k over the block products, and the
    flops the small-block MFMA kernels issue for them: m and n rounded up to
    16-row / 16-column tiles, k to 16-deep steps.  Both sums factor over K:
    sum_K f(k_K) * (sum over A's blocks in column K of g(m_I)) * (sum over
    B's blocks in row K of h(n_J))."""
    rbs, kbs, cbs = (np.asarray(x, np.int64) for x in (A.rbs, A.cbs, B.cbs))
    a_rows = np.repeat(np.arange(len(rbs)), np.diff(A.row_ptr))
    a_m = np.bincount(A.col_ind, weights=rbs[a_rows], minlength=len(kbs))
    a_mp = np.bincount(A.col_ind, weights=16 * np.ceil(rbs[a_rows] / 16), minlength=len(kbs))
    b_rows = np.repeat(np.arange(len(kbs)), np.diff(B.row_ptr))
    b_n = np.bincount(b_rows, weights=cbs[B.col_ind], minlength=len(kbs))
    b_np = np.bincount(b_rows, weights=16 * np.ceil(cbs[B.col_ind] / 16), minlength=len(kbs))
    F = 2.0 * float(np.sum(kbs * a_m * b_n))
    issued = 2.0 * float(np.sum(16 * np.ceil(kbs / 16) * a_mp * b_np))
    return F, issued


def stream_bytes(A, B):
    """Bytes of the products' operands read once per product, with no reuse
    between products: sum over the block products of 8 (m k + k n), summed
    per K as in mfma_padding."""
    rbs, kbs, cbs = (np.asarray(x, np.int64) for x in (A.rbs, A.cbs, B.cbs))
    a_rows = np.repeat(np.arange(len(rbs)), np.diff(A.row_ptr))
    a_cnt = np.bincount(A.col_ind, minlength=len(kbs))
    a_m = np.bincount(A.col_ind, weights=rbs[a_rows], minlength=len(kbs))
    b_rows = np.repeat(np.arange(len(kbs)), np.diff(B.row_ptr))
    b_cnt = np.bincount(b_rows, minlength=len(kbs))
    b_n = np.bincount(b_rows, weights=cbs[B.col_ind], minlength=len(kbs))
    return 8.0 * float(np.sum(kbs * (a_m * b_cnt + a_cnt * b_n)))


def block_norms(M, chunk=1 << 26):
    """Frobenius norm of every block of a host block-CSR matrix (squares
    summed per block, in pieces of about `chunk` elements)."""
    sizes = np.asarray(M.rbs, np.int64)[np.repeat(np.arange(len(M.rbs)), np.diff(M.row_ptr))] * \
        np.asarray(M.cbs, np.int64)[np.asarray(M.col_ind)]
    start = np.concatenate([[0], np.cumsum(sizes)])
    out = np.empty(len(sizes))
    data = np.asarray(M.data)
    b0 = 0
    while b0 < len(sizes):
        b1 = int(np.searchsorted(start, start[b0] + chunk, side="right"))
        b1 = min(max(b1 - 1, b0 + 1), len(sizes))
        seg = data[start[b0]:start[b1]]
        out[b0:b1] = np.add.reduceat(seg * seg, start[b0:b1] - start[b0])
        b0 = b1
    return np.sqrt(out)


def screened_work(A, B, alpha, eps):
    """The work of the C blocks that the library's norm-bound screen keeps
    (option "prescreen": a block stays unless |alpha| sum_K ||A_IK||
    ||B_KJ|| grown by the rounding margin is below eps), estimated on the
    host with dense block-row x block-column matrices: products, flops,
    MFMA-issued flops (m, n, k rounded up to 16) and the no-reuse operand
    stream of those blocks, and the number of blocks screened."""
    nbr, nbk, nbc = len(A.rbs), len(A.cbs), len(B.cbs)
    a_rows = np.repeat(np.arange(nbr), np.diff(A.row_ptr))
    b_rows = np.repeat(np.arange(nbk), np.diff(B.row_ptr))
    MA = np.zeros((nbr, nbk))
    MA[a_rows, A.col_ind] = 1.0
    MB = np.zeros((nbk, nbc))
    MB[b_rows, B.col_ind] = 1.0
    NA = np.zeros((nbr, nbk))
    NA[a_rows, A.col_ind] = block_norms(A)
    NB = np.zeros((nbk, nbc))
    NB[b_rows, B.col_ind] = block_norms(B)
    bound = abs(alpha) * (NA @ NB)
    del NA, NB
    margin = max(1e-6, 4.0 * (float(np.sum(A.cbs)) + 4.0) * 2.0 ** -53)
    keep = ~((bound * (1.0 + margin) < eps) & (bound < 1e150))
    m, k, n = (np.asarray(x, np.float64) for x in (A.rbs, A.cbs, B.cbs))
    pad = lambda x: 16.0 * np.ceil(x / 16.0)
    P = MA @ MB
    KP = (MA * k) @ MB
    KPp = (MA * pad(k)) @ MB
    reached = P > 0
    return {"products_run": int(round(P[keep].sum())),
            "flops_run": 2.0 * float((np.outer(m, n) * KP)[keep].sum()),
            "issued_run": 2.0 * float((np.outer(pad(m), pad(n)) * KPp)[keep].sum()),
            "stream_run": 8.0 * float(((m[:, None] + n[None, :]) * KP)[keep].sum()),
            "screened_blocks": int((reached & ~keep).sum())}


def rows_slice(torch, M, r0, r1):
    """Block rows [r0, r1) of a matrix on the device as a host block-CSR
    (the data go through a device buffer, only the rows reach the host)."""
    from paper_1910_04796_amd import bsmm
    from synth import BlockCSR, block_elems
    nbr, nbc, nnzb, ne = M.info()
    tdt = torch.float32 if getattr(M, "dtype", "f64") == "f32" else torch.float64
    dev = torch.empty(max(ne, 1), dtype=tdt, device="cuda")
    rp, ci, _ = bsmm.bsmm_copy_out(M.handle, device_out=dev)
    sizes = block_elems(M.rbs, M.cbs, rp, ci)
    start = np.concatenate([[0], np.cumsum(sizes)])
    a0, a1 = int(rp[r0]), int(rp[r1])
    data = dev[int(start[a0]):int(start[a1])].cpu().numpy().astype(np.float64)
    del dev
    return BlockCSR(M.rbs[r0:r1], M.cbs, rp[r0:r1 + 1] - rp[r0], ci[a0:a1].astype(np.int32), data)


def rel_err_same_pattern(orc, X, R):
    """Relative error of X against R (inf if the block patterns differ)."""
    if not (np.array_equal(X.row_ptr, R.row_ptr) and np.array_equal(X.col_ind, R.col_ind)):
        return float("inf")
    return orc.rel_err(X.data, R.data)


def sampled_err(orc, torch, M, A, B, rows, threads, eps=0.0):
    """Largest relative error of the device matrix M against the reference
    on the given block rows (inf if a row's pattern differs)."""
    errs = []
    for r in rows:
        R = orc.multiply(1.0, A, B, 0.0, filter_eps=eps, rows=(r, r + 1), nthreads=threads)
        errs.append(rel_err_same_pattern(orc, rows_slice(torch, M, r, r + 1), R))
    return max(errs)


def sampled_err_host(orc, X, A, B, rows, threads, eps=0.0):
    """As sampled_err, for a host copy X of the whole result."""
    sizes = orc.block_sizes(X.rbs, X.cbs, X.row_ptr, X.col_ind)
    start = np.concatenate([[0], np.cumsum(sizes)])
    errs = []
    for r in rows:
        R = orc.multiply(1.0, A, B, 0.0, filter_eps=eps, rows=(r, r + 1), nthreads=threads)
        a0, a1 = int(X.row_ptr[r]), int(X.row_ptr[r + 1])
        if not np.array_equal(X.col_ind[a0:a1], R.col_ind):
            errs.append(float("inf"))
            continue
        errs.append(orc.rel_err(X.data[int(start[a0]):int(start[a1])], R.data))
    return max(errs)


def headline(bsmm, torch, stream, args):
    """The banded 30 % product: tuned stacks (timed as the contract says),
    plain stacks beside them, the stack kernels' device time, and the
    MFMA padding of the small-block kernels."""
    from synth import banded_uneven
    t0 = time.perf_counter()
    A, B = banded_uneven(seed=0, occupancy=HEADLINE_OCC, target=50000)
    log(f"headline inputs: {A.nnzb} + {B.nnzb} blocks ({time.perf_counter() - t0:.1f} s)")
    F, issued = mfma_padding(A, B)
    MA, MB = bsmm.Matrix.from_blocks(A), bsmm.Matrix.from_blocks(B)
    res = {}
    set_opts(bsmm, path="stack", stack_kernel="tuned")
    MC = bsmm.Matrix.empty(A.rbs, B.cbs)

    def step():
        bsmm.multiply(1.0, MA, MB, 0.0, MC, HEADLINE_EPS, stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"warmup done ({args.warmup} steps)")
    bsmm.bsmm_set_option("time_kernels", "1")
    bsmm.bsmm_kernel_times(reset=True)
    ms_per_step = timed(torch, step, args.steps)
    _, _, stack_ms, stack_n = bsmm.bsmm_kernel_times(reset=True)
    bsmm.bsmm_set_option("time_kernels", "0")
    st = bsmm.bsmm_last_stats()
    assert abs(st["flops"] - F) <= 1e-9 * F, (st["flops"], F)
    log(f"tuned: {ms_per_step:.3f} ms/step, {gflops(F, ms_per_step)} GFLOP/s")
    res["tuned"] = {"ms_per_step": round(ms_per_step, 4), "gflops": gflops(F, ms_per_step),
                    "stack_kernel_ms": round(stack_ms / max(stack_n, 1), 4),
                    "stack_launches": stack_n}
    res["stats"] = st
    res["C_tuned"] = MC
    set_opts(bsmm, stack_kernel="plain")
    MP = bsmm.Matrix.empty(A.rbs, B.cbs)
    t = timed_calls(torch, lambda: bsmm.multiply(1.0, MA, MB, 0.0, MP, HEADLINE_EPS, stream), 1,
                    args.plain_reps)
    res["plain"] = dict(t, gflops=gflops(F, t["median_ms"]))
    log(f"plain: {t['median_ms']:.3f} ms (median of {args.plain_reps})")
    res["C_plain"] = MP
    # The same tuned multiply with the norm-bound screen off: every block of
    # the product pattern is formed and the filter alone drops.
    if not args.no_unscreened:
        set_opts(bsmm, stack_kernel="tuned")
        bsmm.bsmm_set_option("prescreen", "0")
        MN = bsmm.Matrix.empty(A.rbs, B.cbs)
        t = timed_calls(torch, lambda: bsmm.multiply(1.0, MA, MB, 0.0, MN, HEADLINE_EPS, stream), 1,
                        args.plain_reps)
        bsmm.bsmm_set_option("prescreen", "1")
        res["tuned_without_prescreen"] = dict(t, gflops=gflops(F, t["median_ms"]))
        log(f"tuned without the screen: {t['median_ms']:.3f} ms (median of {args.plain_reps})")
        MN.close()
    set_opts(bsmm, path="auto", stack_kernel="plain")
    MA.close()
    MB.close()
    res["F"], res["issued"] = F, issued
    res["stream_bytes"] = stream_bytes(A, B)
    res["screen"] = screened_work(A, B, 1.0, HEADLINE_EPS)
    log(f"screen (host estimate): {res['screen']['screened_blocks']} blocks, "
        f"{res['screen']['products_run']} of {st['n_products']} products run (library: {st['n_products_run']})")
    # Algorithmic bytes: A and B read once, the filtered C written once.
    res["b_alg"] = 8.0 * (A.data.size + B.data.size + MC.info()[3])
    res["A"], res["B"] = A, B
    return res


def cpu_baseline(orc, torch, res, threads_all):
    """The reference on SAMPLE_ROWS contiguous block rows of the headline C
    (seeded start) on every core the process may use, and on fewer rows
    with one thread; the tuned and plain GPU results are checked on the
    sampled rows."""
    A, B = res["A"], res["B"]
    nbr = len(A.rbs)
    r0 = int(np.random.default_rng(12345).integers(0, nbr - SAMPLE_ROWS))
    r1 = r0 + SAMPLE_ROWS
    a_rows = np.repeat(np.arange(nbr), np.diff(A.row_ptr))
    flops_rows = None
    orc.multiply(1.0, A, B, 0.0, filter_eps=HEADLINE_EPS, rows=(r0, r0 + 2), nthreads=threads_all)
    c0 = time.perf_counter()
    R = orc.multiply(1.0, A, B, 0.0, filter_eps=HEADLINE_EPS, rows=(r0, r1), nthreads=threads_all)
    t_all = time.perf_counter() - c0
    # flops of the sampled rows: per A block (I, K) in the rows, 2 m k times
    # the columns of B's row K
    kbs = np.asarray(A.cbs, np.int64)
    cb = np.asarray(B.cbs, np.int64)
    b_rows = np.repeat(np.arange(len(kbs)), np.diff(B.row_ptr))
    b_n = np.bincount(b_rows, weights=cb[B.col_ind], minlength=len(kbs))
    sel = (a_rows >= r0) & (a_rows < r1)
    m = np.asarray(A.rbs, np.int64)[a_rows[sel]]
    k = kbs[A.col_ind[sel]]
    flops_rows = 2.0 * float(np.sum(m * k * b_n[A.col_ind[sel]]))
    one_rows = 4
    c0 = time.perf_counter()
    orc.multiply(1.0, A, B, 0.0, filter_eps=HEADLINE_EPS, rows=(r0, r0 + one_rows), nthreads=1)
    t_one = time.perf_counter() - c0
    sel1 = (a_rows >= r0) & (a_rows < r0 + one_rows)
    m1 = np.asarray(A.rbs, np.int64)[a_rows[sel1]]
    k1 = kbs[A.col_ind[sel1]]
    flops_one = 2.0 * float(np.sum(m1 * k1 * b_n[A.col_ind[sel1]]))
    cpu = {"value": round(flops_rows / t_all / 1e9, 3), "unit": "GFLOP/s", "cores": threads_all,
           "kind": "oracle",
           "sample": f"block rows {r0}..{r1 - 1} of {nbr} of the headline product "
                     f"({flops_rows:.3e} flop, {t_all:.1f} s on {threads_all} threads)",
           "value_1thread": round(flops_one / t_one / 1e9, 3),
           "sample_1thread": f"block rows {r0}..{r0 + one_rows - 1} ({flops_one:.3e} flop, {t_one:.1f} s)",
           "full_product_estimate_s": round(t_all * res["F"] / flops_rows, 1)}
    errs = {"tuned": rel_err_same_pattern(orc, rows_slice(torch, res["C_tuned"], r0, r1), R),
            "plain": rel_err_same_pattern(orc, rows_slice(torch, res["C_plain"], r0, r1), R)}
    return cpu, errs, (r0, r1)


def extras_dense(bsmm, torch, stream, args):
    """Dense N = 8192 in 32-blocks: densified GEMM (with the GEMM kernel's
    own roofline), blocked plain and tuned stacks (also with the run-time
    compiled kernel of the one 32 x 32 x 32 class), INT8 emulation."""
    from synth import dense_square
    N, BS = 8192, 32
    A, B = dense_square(seed=0, n=N, bs=BS)
    MA, MB = bsmm.Matrix.from_blocks(A), bsmm.Matrix.from_blocks(B)
    F = 2.0 * N ** 3
    out = {"N": N, "block": BS, "flops_per_multiply": F}
    keep = {}

    def leg(name, reps, **opts):
        set_opts(bsmm, **opts)
        MC = bsmm.Matrix.empty(A.rbs, B.cbs)
        bsmm.bsmm_set_option("time_kernels", "1")
        bsmm.bsmm_kernel_times(reset=True)
        t = timed_calls(torch, lambda: bsmm.multiply(1.0, MA, MB, 0.0, MC, 0.0, stream), 2, reps)
        g_ms, g_n, s_ms, s_n = bsmm.bsmm_kernel_times(reset=True)
        bsmm.bsmm_set_option("time_kernels", "0")
        r = dict(t, gflops=gflops(F, t["median_ms"]))
        if g_n:
            r["gemm_kernel_ms"] = round(g_ms / g_n, 4)
        if s_n:
            r["stack_kernel_ms"] = round(s_ms / s_n, 4)
        out[name] = r
        log(f"dense 8192 {name}: {t['median_ms']:.3f} ms")
        set_opts(bsmm, path="auto", stack_kernel="plain", dense_kb=16, jit=0)
        return MC

    keep["densified"] = leg("densified", args.reps * 2, path="dense")
    g = out["densified"]["gemm_kernel_ms"]
    out["densified"]["gemm_roofline"] = {
        "kernel": "k_dgemm_mfma", "achieved": round(F / (g * 1e-3) / 1e12, 3), "peak": PEAK_FP64_TFLOPS,
        "unit": "TFLOP/s", "frac": round(F / (g * 1e-3) / 1e12 / PEAK_FP64_TFLOPS, 4)}
    tr = profile_json("dgemm_dense_square_8192_traffic.json", "paper_1910_04796_amd/csrc/dense.hip")
    out["densified"]["gemm_roofline"]["traffic"] = tr.get("bytes_per_launch") if tr else None
    leg("densified_k32", args.reps, path="dense", dense_kb=32).close()
    for kern in ("plain", "tuned"):
        leg(f"blocked_{kern}", args.reps, path="stack", stack_kernel=kern).close()
        out[f"blocked_{kern}"]["t_blocked_over_t_densified"] = round(
            out[f"blocked_{kern}"]["median_ms"] / out["densified"]["median_ms"], 3)
    leg("blocked_tuned_jit", args.reps, path="stack", stack_kernel="tuned", jit=1).close()
    out["blocked_tuned_jit"]["t_blocked_over_t_densified"] = round(
        out["blocked_tuned_jit"]["median_ms"] / out["densified"]["median_ms"], 3)
    keep["emulated_int8_s7"] = leg("emulated_int8_s7", args.reps, path="emul", emul_slices=7)
    e = out["emulated_int8_s7"]
    e["speedup_vs_densified_fp64"] = round(out["densified"]["median_ms"] / e["median_ms"], 3)
    e["int8_tops_achieved"] = round(28 * F / (e["gemm_kernel_ms"] * 1e-3) / 1e12, 1)
    e["int8_peak_tops"] = 5000.0
    MA.close()
    MB.close()
    return out, keep, A, B


def extras_wide(bsmm, torch, stream, args, orc, threads):
    """Split-precision workload: N = 16384 in 32-blocks, entries
    sign * 10^U(-6, 2); native FP64 dense vs INT8 emulation (7 slices)."""
    from synth import wide_range_dense
    W1, W2 = wide_range_dense(seed=0, n=16384, bs=32)
    MW1, MW2 = bsmm.Matrix.from_blocks(W1), bsmm.Matrix.from_blocks(W2)
    F = 2.0 * 16384 ** 3
    out = {"N": 16384, "values": "sign * 10^U(-6,2)", "slices": 7, "flops_per_multiply": F}
    Xs = {}
    for name, opts in (("native_fp64", dict(path="dense")), ("emulated_int8", dict(path="emul", emul_slices=7))):
        set_opts(bsmm, **opts)
        MC = bsmm.Matrix.empty(W1.rbs, W2.cbs)
        t = timed_calls(torch, lambda: bsmm.multiply(1.0, MW1, MW2, 0.0, MC, 0.0, stream), 1, args.reps)
        out[name] = dict(t, gflops_fp64_equiv=gflops(F, t["median_ms"]))
        Xs[name] = MC.to_host()
        MC.close()
        log(f"wide-range 16384 {name}: {t['median_ms']:.3f} ms")
    set_opts(bsmm, path="auto")
    out["speedup_emulated_vs_native"] = round(out["native_fp64"]["median_ms"] /
                                              out["emulated_int8"]["median_ms"], 3)
    Xn, Xe = Xs["native_fp64"].data, Xs["emulated_int8"].data
    out["rel_err_emulated_vs_native"] = float(np.linalg.norm(Xe - Xn) / np.linalg.norm(Xn))
    if orc is not None:
        out["rel_err_emulated_rows_5_200_511"] = sampled_err_host(orc, Xs["emulated_int8"], W1, W2,
                                                                  (5, 200, 511), threads)
        out["rel_err_native_rows_5_200_511"] = sampled_err_host(orc, Xs["native_fp64"], W1, W2,
                                                                (5, 200, 511), threads)
    MW1.close()
    MW2.close()
    return out


def extras_banded(bsmm, torch, stream, args, orc, threads, occs=(0.01, 0.10)):
    """Banded uneven blocks at 1 % and 10 %: plain vs tuned stacks."""
    from synth import banded_uneven
    out = {}
    for occ in occs:
        U, V = banded_uneven(seed=0, occupancy=occ, target=50000)
        MU, MV = bsmm.Matrix.from_blocks(U), bsmm.Matrix.from_blocks(V)
        r = {"N": int(np.sum(U.rbs)), "blocks_A": int(U.nnzb)}
        scr = screened_work(U, V, 1.0, HEADLINE_EPS)
        sb = scr["stream_run"]
        r["no_reuse_stream_bytes"] = sb
        r["no_reuse_stream_bytes_all_products"] = stream_bytes(U, V)
        for kern in ("plain", "tuned"):
            set_opts(bsmm, path="stack", stack_kernel=kern)
            MW = bsmm.Matrix.empty(U.rbs, V.cbs)
            bsmm.bsmm_set_option("time_kernels", "1")
            bsmm.bsmm_kernel_times(reset=True)
            t = timed_calls(torch, lambda: bsmm.multiply(1.0, MU, MV, 0.0, MW, HEADLINE_EPS, stream), 2,
                            args.reps)
            _, _, s_ms, s_n = bsmm.bsmm_kernel_times(reset=True)
            bsmm.bsmm_set_option("time_kernels", "0")
            st = bsmm.bsmm_last_stats()
            r[kern] = dict(t, gflops=gflops(st["flops"], t["median_ms"]))
            # Stack kernel time per multiply (warm-up and timed calls alike)
            # and the operand stream it reads against the HBM bandwidth.
            k_ms = s_ms / (2 + args.reps)
            r[kern]["stack_kernel_ms"] = round(k_ms, 4)
            r[kern]["no_reuse_stream_frac"] = round(sb / (PEAK_HBM_GBS * 1e9) / (k_ms * 1e-3), 4)
            r["flops_per_multiply"] = st["flops"]
            r["products"] = st["n_products"]
            r["products_run"] = st["n_products_run"]
            r["screened_c_blocks"] = st["n_screened"]
            r["classes"] = st["n_classes"]
            if orc is not None and kern == "tuned":
                nb = len(U.rbs)
                r["tuned"]["rel_err_sampled_rows"] = sampled_err(orc, torch, MW, U, V,
                                                                 (3, nb // 2, nb - 4), threads, HEADLINE_EPS)
            MW.close()
        r["tuned_speedup"] = round(r["plain"]["median_ms"] / r["tuned"]["median_ms"], 3)
        out[f"banded_uneven_{int(round(occ * 100))}pct"] = r
        log(f"banded {occ}: plain {r['plain']['median_ms']} ms, tuned {r['tuned']['median_ms']} ms")
        MU.close()
        MV.close()
    set_opts(bsmm, path="auto", stack_kernel="plain")
    return out


HELDOUT_DB = os.path.join(ROOT, "paper_1910_04796_amd", "tune_db", "gfx950_heldout_sizes.txt")


def as_f32(M):
    """The same matrix with its values rounded to FP32 (held as float64,
    which represents them exactly): the reference's inputs for FP32 legs."""
    from synth import BlockCSR
    return BlockCSR(M.rbs, M.cbs, M.row_ptr, M.col_ind, np.asarray(M.data, np.float32).astype(np.float64))


def extras_f32(bsmm, torch, stream, args, orc, threads):
    """Single-precision matrices: the dense N = 8192 product in 32-blocks
    (densified, FP32 MFMA GEMM) and the banded 10 % product (plain and
    tuned stacks), checked against the FP64 reference of the FP32-rounded
    inputs on sampled block rows (tolerance 1e-5)."""
    from synth import banded_uneven, dense_square
    out = {}
    A, B = dense_square(seed=0, n=8192, bs=32)
    A, B = as_f32(A), as_f32(B)
    MA, MB = bsmm.Matrix.from_blocks(A, dtype="f32"), bsmm.Matrix.from_blocks(B, dtype="f32")
    F = 2.0 * 8192 ** 3
    set_opts(bsmm, path="dense")
    MC = bsmm.Matrix.empty(A.rbs, B.cbs, dtype="f32")
    bsmm.bsmm_set_option("time_kernels", "1")
    bsmm.bsmm_kernel_times(reset=True)
    t = timed_calls(torch, lambda: bsmm.multiply(1.0, MA, MB, 0.0, MC, 0.0, stream), 2, args.reps * 2)
    g_ms, g_n, _, _ = bsmm.bsmm_kernel_times(reset=True)
    bsmm.bsmm_set_option("time_kernels", "0")
    g = g_ms / max(g_n, 1)
    r = dict(t, gflops=gflops(F, t["median_ms"]), gemm_kernel_ms=round(g, 4),
             gemm_roofline={"kernel": "k_dgemm_mfma<float>", "achieved": round(F / (g * 1e-3) / 1e12, 3),
                            "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                            "frac": round(F / (g * 1e-3) / 1e12 / PEAK_FP32_TFLOPS, 4)})
    if orc is not None:
        r["rel_err_rows_0_127_255"] = sampled_err(orc, torch, MC, A, B, (0, 127, 255), threads)
    out["dense_square_8192_b32_f32"] = r
    log(f"f32 dense 8192: {t['median_ms']:.3f} ms (GEMM {g:.3f} ms)")
    for M in (MA, MB, MC):
        M.close()
    del A, B
    U, V = banded_uneven(seed=0, occupancy=0.10, target=50000)
    U, V = as_f32(U), as_f32(V)
    MU, MV = bsmm.Matrix.from_blocks(U, dtype="f32"), bsmm.Matrix.from_blocks(V, dtype="f32")
    r = {}
    for kern in ("plain", "tuned"):
        set_opts(bsmm, path="stack", stack_kernel=kern)
        MW = bsmm.Matrix.empty(U.rbs, V.cbs, dtype="f32")
        t = timed_calls(torch, lambda: bsmm.multiply(1.0, MU, MV, 0.0, MW, HEADLINE_EPS, stream), 2, args.reps)
        st = bsmm.bsmm_last_stats()
        r[kern] = dict(t, gflops=gflops(st["flops"], t["median_ms"]))
        if orc is not None:
            nb = len(U.rbs)
            r[kern]["rel_err_sampled_rows"] = sampled_err(orc, torch, MW, U, V, (3, nb // 2, nb - 4), threads,
                                                          HEADLINE_EPS)
        MW.close()
    r["tuned_speedup"] = round(r["plain"]["median_ms"] / r["tuned"]["median_ms"], 3)
    out["banded_uneven_10pct_f32"] = r
    log(f"f32 banded 10 %: plain {r['plain']['median_ms']} ms, tuned {r['tuned']['median_ms']} ms")
    MU.close()
    MV.close()
    set_opts(bsmm, path="auto", stack_kernel="plain")
    return out


def extras_learned(bsmm, torch, stream, args, orc, threads):
    """The learned model deciding: the banded 10 % product with block sizes
    {6, 14, 22, 30}, none of whose 64 shapes is in the shipped tuning
    database, so the tuned path takes the model's pick for every class.
    Timed against the plain rule and against the exhaustive choice of the
    tuner for those shapes (a database made offline by the tuner)."""
    from synth import banded_uneven
    U, V = banded_uneven(seed=0, occupancy=0.10, target=50000, choices=(6, 14, 22, 30))
    MU, MV = bsmm.Matrix.from_blocks(U), bsmm.Matrix.from_blocks(V)
    db = bsmm.bsmm_get_option("tune_db")
    r = {"block_sizes": [6, 14, 22, 30], "occupancy": 0.10}
    legs = [("plain", "plain", db), ("learned", "tuned", db)]
    if os.path.exists(HELDOUT_DB):
        legs.append(("exhaustive", "tuned", HELDOUT_DB))
    for name, kern, dbpath in legs:
        set_opts(bsmm, path="stack", stack_kernel=kern, tune_db=dbpath)
        MW = bsmm.Matrix.empty(U.rbs, V.cbs)
        t = timed_calls(torch, lambda: bsmm.multiply(1.0, MU, MV, 0.0, MW, HEADLINE_EPS, stream), 2, args.reps)
        st = bsmm.bsmm_last_stats()
        r[name] = dict(t, gflops=gflops(st["flops"], t["median_ms"]))
        if kern == "tuned":
            r[name]["picks_k22_R8"] = {f"{m}x{n}": list(bsmm.bsmm_select_params(m, n, 22, 8))
                                       for m in (6, 14, 22, 30) for n in (6, 14, 22, 30)}
        if orc is not None and name == "learned":
            nb = len(U.rbs)
            r[name]["rel_err_sampled_rows"] = sampled_err(orc, torch, MW, U, V, (3, nb // 2, nb - 4), threads,
                                                          HEADLINE_EPS)
        MW.close()
        log(f"learned-model leg {name}: {t['median_ms']:.3f} ms")
    set_opts(bsmm, path="auto", stack_kernel="plain", tune_db=db)
    r["learned_speedup_vs_plain"] = round(r["plain"]["median_ms"] / r["learned"]["median_ms"], 3)
    if "exhaustive" in r:
        r["exhaustive_over_learned_time"] = round(r["exhaustive"]["median_ms"] / r["learned"]["median_ms"], 4)
    MU.close()
    MV.close()
    return r


def extras_tiny(bsmm, torch, stream, args):
    """460 x 460 in 23-blocks, 10 %: latency of one multiply."""
    from synth import sparse_uniform
    S1, S2 = sparse_uniform(seed=0)
    M1, M2 = bsmm.Matrix.from_blocks(S1), bsmm.Matrix.from_blocks(S2)
    tiny = {}
    for kern in ("plain", "tuned"):
        set_opts(bsmm, path="stack", stack_kernel=kern)
        M3 = bsmm.Matrix.empty(S1.rbs, S2.cbs)
        run3 = lambda: bsmm.multiply(1.0, M1, M2, 0.0, M3, 0.0, stream)
        tiny[kern + "_us"] = round(1e3 * timed_calls(torch, run3, 3, 20)["median_ms"], 1)
        if kern == "tuned":
            # Repeated multiply into the same C with the plan cache: the
            # symbolic phase and stack build are skipped and the planned
            # hipGraph is replayed (same result, see the plan-cache tests).
            bsmm.bsmm_set_option("plan_cache", "1")
            tiny["tuned_plan_cache_us"] = round(1e3 * timed_calls(torch, run3, 3, 20)["median_ms"], 1)
            bsmm.bsmm_set_option("plan_cache", "0")
        M3.close()
    set_opts(bsmm, path="auto", stack_kernel="plain")
    M1.close()
    M2.close()
    return tiny


def all_configs(bsmm, torch, stream, args):
    """The remaining workloads of the evaluation set: rectangular dense
    (4096 x 65536 times 65536 x 4096) and the sparse split-precision case
    (1,424^2 blocks of 23, 20 %, entries sign * 10^U(-6,2)).  Returns the
    timings and, for the reference check, host copies of the results with
    their inputs."""
    from synth import dense_rect, wide_range_sparse
    res, keep = {}, {}

    def time_path(MA, MB, rbs, cbs, eps, reps, **opts):
        set_opts(bsmm, **opts)
        MC = bsmm.Matrix.empty(rbs, cbs)
        t = timed_calls(torch, lambda: bsmm.multiply(1.0, MA, MB, 0.0, MC, eps, stream), 1, reps)
        st = bsmm.bsmm_last_stats()
        set_opts(bsmm, path="auto", stack_kernel="plain")
        return MC, t, st

    A, B = dense_rect(seed=0)
    MA, MB = bsmm.Matrix.from_blocks(A), bsmm.Matrix.from_blocks(B)
    MC, t, st = time_path(MA, MB, A.rbs, B.cbs, 0.0, args.reps, path="auto")
    Fr = 2.0 * 4096 * 4096 * 65536
    res["dense_rect_4096x4096x65536"] = dict(t, path=st["path"], gflops=gflops(Fr, t["median_ms"]))
    keep["rect"] = (MC.to_host(), A, B, 0.0, (0, 61, 127))
    log(f"dense rect: {t['median_ms']:.3f} ms")
    for M in (MA, MB, MC):
        M.close()

    S1, S2 = wide_range_sparse(seed=0)
    M1, M2 = bsmm.Matrix.from_blocks(S1), bsmm.Matrix.from_blocks(S2)
    sp = {"N": int(np.sum(S1.rbs)), "block": 23, "occupancy": 0.2, "values": "sign * 10^U(-6,2)"}
    for name, opts in (("native_fp64_stack_plain", dict(path="stack", stack_kernel="plain")),
                       ("native_fp64_stack_tuned", dict(path="stack", stack_kernel="tuned")),
                       ("emulated_int8_densified", dict(path="emul", emul_slices=7))):
        MS, t, st = time_path(M1, M2, S1.rbs, S2.cbs, 0.0, args.reps, **opts)
        sp[name] = dict(t, gflops_fp64_equiv=gflops(st["flops"], t["median_ms"]))
        sp["flops_per_multiply"] = st["flops"]
        keep["sparse_" + name] = (MS.to_host(), S1, S2, 0.0, (3, 700, 1420))
        MS.close()
        log(f"sparse split-precision workload {name}: {t['median_ms']:.3f} ms")
    res["sparse_wide_range_32752_b23"] = sp
    M1.close()
    M2.close()
    return res, keep


PAPER_SHAPES = {"square_63360": (63360, 63360, 63360),
                "rect_1408x1408x1982464": (1408, 1408, 1982464),
                # the first tenth of the square product's C rows (every C row
                # of a dense product costs the same in both modes)
                "square_63360_rows_6336": (6336, 63360, 63360),
                # its first 176 C rows (44 block rows of 4, 8 of 22): the one
                # share of the product in blocks of 4 that the blocked mode
                # can hold (1.1e10 block products)
                "square_63360_rows_176": (176, 63360, 63360)}
# Blocked mode is skipped above this many block products (the square
# product in blocks of 22 has 2.4e10; its first tenth of rows took 3.7 s).
BLOCKED_MAX_PRODUCTS = 3e10


def paper_workloads(bsmm, torch, stream, names, threads, blocks=None):
    """The paper's own benchmark products (Sec. IV) on one GPU: square
    M = N = K = 63,360 and tall-and-skinny M = N = 1,408, K = 1,982,464, in
    square blocks of 22 or 64, every block present, values U[-1, 1].  Each
    is run densified (merged panels + one FP64 MFMA GEMM) and blocked (tuned
    stacks, built in row panels when the products exceed the stack cap);
    reported: time per multiply, T_blocked / T_densified per block size, and
    the densified time for blocks of 22 over that for 64.  One warm-up
    multiply and two timed ones per mode; a warm-up longer than 20 s is
    itself the timing.  The square product also runs in blocks of 4,
    densified only (the paper quotes that block size for its comparison
    with a dense library; blocked, it would hold about 4e12 block
    products); its first 176 rows run in blocks of 22 and 4 in both modes.
    Every result is checked against the reference on two sampled block
    rows."""
    from oracle import oracle as orc
    from synth import BlockCSR, pattern_full, rng_of, values_uniform
    out = {}
    for name in names:
        M, Nn, K = PAPER_SHAPES[name]
        rng = rng_of(0)
        log(f"{name}: drawing {M * K + K * Nn:.3e} values")
        a_vals = values_uniform(rng, M * K)
        b_vals = values_uniform(rng, K * Nn)
        F = 2.0 * M * Nn * K
        res = {"M": M, "N": Nn, "K": K, "flops_per_multiply": F}
        # The paper's square product also in blocks of 4 (its comparison with
        # a dense library); blocked mode there is far beyond the stack cap.
        sizes = {"square_63360": (64, 22, 4), "square_63360_rows_176": (22, 4)}.get(name, (64, 22))
        if blocks:
            sizes = tuple(b for b in sizes if b in blocks)
        for bs in sizes:
            ms_, ns_, ks_ = (np.full(x // bs, bs, np.int32) for x in (M, Nn, K))
            A = BlockCSR(ms_, ks_, *pattern_full(len(ms_), len(ks_)), a_vals)
            B = BlockCSR(ks_, ns_, *pattern_full(len(ks_), len(ns_)), b_vals)
            MA, MB = bsmm.Matrix.from_blocks(A), bsmm.Matrix.from_blocks(B)
            r = {"blocks_A": int(A.nnzb), "blocks_B": int(B.nnzb)}
            products = float(len(ms_)) * len(ks_) * len(ns_)
            for mode, opts in (("densified", dict(path="dense")),
                               ("blocked", dict(path="stack", stack_kernel="tuned", verbose=1))):
                if mode == "blocked" and products > BLOCKED_MAX_PRODUCTS:
                    r[mode] = {"skipped": f"{products:.3g} block products ({products * 16 / 1e9:.0f} GB "
                                          f"of stack entries) exceed {BLOCKED_MAX_PRODUCTS:.0e}"}
                    log(f"{name} b{bs} blocked skipped: {r[mode]['skipped']}")
                    continue
                set_opts(bsmm, **opts)
                MC = bsmm.Matrix.empty(ms_, ns_)

                def run(MC=MC):
                    bsmm.multiply(1.0, MA, MB, 0.0, MC, 0.0, stream)

                t_first = timed(torch, run, 1)
                st = bsmm.bsmm_last_stats()
                ms = t_first if t_first > 20e3 else timed(torch, run, 2)
                set_opts(bsmm, path="auto", stack_kernel="plain", verbose=0)
                r[mode] = {"ms": round(ms, 2), "gflops": round(F / (ms * 1e-3) / 1e9, 1),
                           "timed_runs": 1 if t_first > 20e3 else 2, "path": st["path"],
                           "products": st["n_products"], "row_panels": st["n_row_panels"]}
                log(f"{name} b{bs} {mode}: {ms:.1f} ms ({r[mode]['gflops']} GFLOP/s), "
                    f"{st['n_products']} products, {st['n_row_panels']} row panels")
                X = MC.to_host()
                MC.close()
                rows = (0, len(ms_) - 1)
                r[mode]["rel_err_sampled_rows"] = sampled_err_host(orc, X, A, B, rows, threads)
                r[mode]["sampled_block_rows"] = list(rows)
                log(f"{name} b{bs} {mode}: rel err {r[mode]['rel_err_sampled_rows']:.2e} on block rows {rows}")
                del X
            if "ms" in r["blocked"]:
                r["t_blocked_over_t_densified"] = round(r["blocked"]["ms"] / r["densified"]["ms"], 3)
            res[f"b{bs}"] = r
            MA.close()
            MB.close()
            del A, B
        if "b22" in res and "b64" in res:
            res["densified_b22_over_b64"] = round(res["b22"]["densified"]["ms"] / res["b64"]["densified"]["ms"],
                                                  4)
        if "b4" in res and "b64" in res:
            res["densified_b4_over_b64"] = round(res["b4"]["densified"]["ms"] / res["b64"]["densified"]["ms"], 4)
        if "b4" in res and "b22" in res:
            for mode in ("densified", "blocked"):
                if "ms" in res["b4"][mode] and "ms" in res["b22"][mode]:
                    res[f"{mode}_b4_over_b22"] = round(res["b4"][mode]["ms"] / res["b22"][mode]["ms"], 4)
        out[name] = res
        del a_vals, b_vals
    return out


EXTRA_LEGS = ("dense", "wide", "banded", "banded1", "banded10", "tiny", "f32", "learned", "all_configs")


def add_all_configs_errors(orc, out, keep, threads):
    """Reference check of the all-configs results on their sampled block rows."""
    for name, (X, Aref, Bref, eps, rows) in keep.items():
        e = sampled_err_host(orc, X, Aref, Bref, rows, threads, eps)
        d = out["dense_rect_4096x4096x65536"] if name == "rect" else \
            out["sparse_wide_range_32752_b23"][name[len("sparse_"):]]
        d["rel_err_sampled_rows"] = e
        d["sampled_block_rows"] = list(rows)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--reps", type=int, default=5, help="repetitions of every extra leg")
    ap.add_argument("--plain-reps", type=int, default=3, help="repetitions of the plain headline leg")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="only the headline workload")
    ap.add_argument("--no-unscreened", action="store_true",
                    help="skip the headline leg with the norm-bound screen off (counter runs)")
    ap.add_argument("--all-configs", action="store_true",
                    help="also run the rectangular dense and sparse split-precision workloads")
    ap.add_argument("--paper-workloads", default="",
                    help="only run the paper's products: comma list of " + ", ".join(PAPER_SHAPES))
    ap.add_argument("--paper-blocks", default="",
                    help="with --paper-workloads: only these block sizes (comma list of 64, 22, 4)")
    ap.add_argument("--extras-only", default="",
                    help="only run these extra legs, no headline (for profiling): comma list of "
                         + ", ".join(EXTRA_LEGS))
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this benchmark runs on exactly one GPU (the local multiply of one rank); "
              "--gpus N > 1 is not supported", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1910_04796_amd import bsmm

    torch.cuda.set_device(0)
    threads = len(os.sched_getaffinity(0))
    if args.calibrate_copy:
        # A plain copy of known size: 1 GiB read + 1 GiB written per launch.
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)  # elementwise kernel: 1 GiB in, 1 GiB out
        torch.cuda.synchronize()
        log("copy calibration: 3 launches of a 1 GiB elementwise copy kernel")
        return
    bsmm.use_torch_allocator(0)
    stream = torch.cuda.current_stream()
    bsmm.use_default_tuning()
    set_opts(bsmm, path="auto", stack_kernel="plain")
    if args.paper_workloads:
        names = [x for x in args.paper_workloads.split(",") if x]
        bad = [x for x in names if x not in PAPER_SHAPES]
        if bad:
            sys.exit(f"bench.py: unknown paper workload(s) {bad}")
        blocks = tuple(int(x) for x in args.paper_blocks.split(",") if x) or None
        res = paper_workloads(bsmm, torch, stream, names, threads, blocks)
        print(json.dumps({"paper_workloads": res, "dtype": "f64", "data": "synthetic", "n_gpus": 1}),
              flush=True)
        bsmm.bsmm_set_allocator()
        return

    if args.extras_only:
        names = [x for x in args.extras_only.split(",") if x]
        bad = [x for x in names if x not in EXTRA_LEGS]
        if bad:
            sys.exit(f"bench.py: unknown extra leg(s) {bad}")
        extras = {}
        for name in names:
            if name == "dense":
                extras["dense_square_8192_b32"], keep, _, _ = extras_dense(bsmm, torch, stream, args)
                for M in keep.values():
                    M.close()
            elif name == "wide":
                extras["emulated_wide_dense_16384"] = extras_wide(bsmm, torch, stream, args, None, threads)
            elif name == "banded":
                extras.update(extras_banded(bsmm, torch, stream, args, None, threads))
            elif name in ("banded1", "banded10"):
                occ = 0.01 if name == "banded1" else 0.10
                extras.update(extras_banded(bsmm, torch, stream, args, None, threads, (occ,)))
            elif name == "tiny":
                extras["sparse_460_b23_latency"] = extras_tiny(bsmm, torch, stream, args)
            elif name == "f32":
                extras.update(extras_f32(bsmm, torch, stream, args, None, threads))
            elif name == "learned":
                extras["learned_banded_10pct_b6-14-22-30"] = extras_learned(bsmm, torch, stream, args, None,
                                                                            threads)
            elif name == "all_configs":
                from oracle import oracle as orc
                extras["all_configs"], keep = all_configs(bsmm, torch, stream, args)
                add_all_configs_errors(orc, extras["all_configs"], keep, threads)
        print(json.dumps({"extras": extras, "dtype": "f64", "data": "synthetic", "n_gpus": 1}), flush=True)
        bsmm.bsmm_set_allocator()
        return

    res = headline(bsmm, torch, stream, args)
    F = res["F"]
    st = res["stats"]
    tuned = res["tuned"]
    k_ms = tuned["stack_kernel_ms"]
    scr = res["screen"]
    # The kernel's own rate counts the products it ran (the screen skips the
    # products of blocks that the filter would drop); `value` counts every
    # product of A*B, the work of the operation whose result it delivers.
    F_run = scr["flops_run"]
    achieved = F_run / (k_ms * 1e-3) / 1e12
    tr = profile_json("smm_sched_banded30_traffic.json", "paper_1910_04796_amd/csrc/smm.hip",
                      st["n_products_run"])
    roofline = {"bound": "mfma", "kernel": "k_smm_mfma_sched (tuned stack launch)",
                "achieved": round(achieved, 3), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP64_TFLOPS, 4), "kernel_ms": k_ms,
                "launches": tuned["stack_launches"],
                "traffic": tr.get("bytes_per_launch") if tr else None,
                "flops_run": F_run,
                "mfma_issued_over_algorithmic": round(scr["issued_run"] / F_run, 4),
                "mfma_issue_frac": round(scr["issued_run"] / (k_ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS, 4),
                # The roofline time max(F / FP64 peak, B_alg / HBM) with A and B
                # read once; and the streaming bound with no reuse between
                # products (operands read once per product), the bound this
                # kernel's design can reach.
                "b_alg_bytes": res["b_alg"],
                "t_roof_ms": round(max(F / (PEAK_FP64_TFLOPS * 1e12), res["b_alg"] / (PEAK_HBM_GBS * 1e9)) * 1e3,
                                   3),
                "no_reuse_stream_bytes": scr["stream_run"],
                "no_reuse_stream_bytes_all_products": res["stream_bytes"],
                "no_reuse_stream_tbs": round(scr["stream_run"] / (k_ms * 1e-3) / 1e12, 3),
                "no_reuse_stream_frac": round(scr["stream_run"] / (PEAK_HBM_GBS * 1e9) / (k_ms * 1e-3), 4)}

    peaks = bsmm.bsmm_measure_peaks()
    peaks = {"fp64_mfma_tflops": round(peaks["fp64_mfma"], 2), "fp32_mfma_tflops": round(peaks["fp32_mfma"], 2),
             "int8_mfma_tops": round(peaks["int8_mfma"], 1), "bf16_mfma_tflops": round(peaks["bf16_mfma"], 1),
             "fp64_valu_tflops": round(peaks["fp64_valu"], 2),
             "hbm_copy_gbs": round(peaks["hbm_gbs"], 1), "hbm_read_gbs": round(peaks["hbm_read_gbs"], 1),
             "vendor": {"fp64_tflops": PEAK_FP64_TFLOPS, "fp32_tflops": PEAK_FP32_TFLOPS, "int8_tops": 5000.0,
                        "bf16_tflops": 2500.0, "hbm_gbs": 8000.0}}
    log(f"measured peaks: {peaks}")
    roofline["frac_of_measured_fp64_mfma"] = round(achieved / peaks["fp64_mfma_tflops"], 4)

    orc = None
    cpu = None
    rel_errs = None
    sample = None
    if not args.no_cpu_baseline:
        from oracle import oracle as orc
        cpu, rel_errs, sample = cpu_baseline(orc, torch, res, threads)
        log(f"cpu baseline: {cpu['value']} GFLOP/s on {threads} threads, {cpu['value_1thread']} on 1; "
            f"rel err tuned {rel_errs['tuned']:.2e} plain {rel_errs['plain']:.2e}")

    res["C_tuned"].close()
    res["C_plain"].close()
    extras = {}
    if not args.no_extras:
        extras["dense_square_8192_b32"], keep, A2, B2 = extras_dense(bsmm, torch, stream, args)
        if orc is not None:
            for name, M in keep.items():
                extras["dense_square_8192_b32"][name]["rel_err_rows_0_127_255"] = sampled_err(
                    orc, torch, M, A2, B2, (0, 127, 255), threads)
        for M in keep.values():
            M.close()
        del A2, B2
        extras["emulated_wide_dense_16384"] = extras_wide(bsmm, torch, stream, args, orc, threads)
        extras.update(extras_banded(bsmm, torch, stream, args, orc, threads))
        extras["sparse_460_b23_latency"] = extras_tiny(bsmm, torch, stream, args)
        extras.update(extras_f32(bsmm, torch, stream, args, orc, threads))
        extras["learned_banded_10pct_b6-14-22-30"] = extras_learned(bsmm, torch, stream, args, orc, threads)
    if args.all_configs:
        extras["all_configs"], keep = all_configs(bsmm, torch, stream, args)
        if orc is not None:
            add_all_configs_errors(orc, extras["all_configs"], keep, threads)

    ms = tuned["ms_per_step"]
    out = {
        "metric": METRIC, "value": tuned["gflops"], "unit": "GFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": HEADLINE_NAME, "N": int(np.sum(res["A"].rbs)),
                   "block_sizes": [5, 13, 23, 32], "occupancy": HEADLINE_OCC,
                   "filter_eps": HEADLINE_EPS, "alpha": 1.0, "beta": 0.0,
                   "path": "tuned stacks: tuning database parameters, classes on the scheduled FP64 MFMA "
                           "small-block kernel in one hipGraph",
                   "flops_per_step": F, "products": st["n_products"], "runs": st["n_runs"],
                   "products_run": st["n_products_run"], "flops_run": F_run,
                   "screened_c_blocks": st["n_screened"],
                   "classes": st["n_classes"], "c_blocks_before_filter": st["c_nnzb_before"],
                   "c_blocks_after_filter": st["c_nnzb_after"]},
        "roofline": roofline,
        "peaks_measured": peaks,
        "cpu_baseline": cpu,
        "rel_err": rel_errs["tuned"] if rel_errs else None,
        "rel_err_mode": f"sampled: block rows {sample[0]}..{sample[1] - 1}" if sample else None,
        "plain": dict(res["plain"], rel_err=rel_errs["plain"] if rel_errs else None),
        "tuned_speedup_vs_plain": round(res["plain"]["median_ms"] / ms, 3),
        "tuned_without_prescreen": res.get("tuned_without_prescreen"),
        "extras": extras,
    }
    print(json.dumps(out), flush=True)
    bsmm.bsmm_set_allocator()


if __name__ == "__main__":
    main()
