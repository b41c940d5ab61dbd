/*
 * bsmm.h -- block-sparse FP64 / FP32 matrix multiply on one AMD MI355X
 * (gfx950).
 *
 * One rank's local step of a distributed block-CSR multiplication:
 *
 *     C <- filter_eps( beta * C + alpha * A * B )
 *
 * Matrices are kept in blocked compressed-sparse-row form (paper, Sec. II:
 * block-CSR storage; the local multiplication is a set of pairwise products
 * of small dense blocks, an A block m x k times a B block k x n).  The
 * library turns the block indices into stacks of block products grouped by
 * block shape and runs them as batched small-block GEMMs on the GPU
 * (Sec. II, Traversal / Generation / Scheduler phases); when both inputs are
 * fully occupied it instead merges the blocks into contiguous panels and
 * runs one large FP64 GEMM, then splits the result back into the original
 * blocks (Sec. III, densification and undensification, Eqs. (1)-(2) with a
 * single rank and a single panel).
 *
 * Conventions shared by every entry point
 *  - Block sizes are >= 1.  A matrix has nbr block rows (sizes
 *    row_blk_sizes[0..nbr)) and nbc block columns (col_blk_sizes[0..nbc)).
 *  - blk_row_ptr is int64[nbr+1] with blk_row_ptr[0] = 0 and
 *    blk_row_ptr[nbr] = nnzb, non-decreasing; blk_col_ind is int32[nnzb]
 *    with column indices in [0, nbc), strictly ascending inside each row.
 *  - Block data are FP64 (or FP32 for matrices created with
 *    bsmm_create_matrix_typed), packed in CSR order; every block is
 *    column-major with leading dimension equal to its number of rows.
 *  - "stream" is a hipStream_t (NULL = the legacy default stream).  All
 *    device work is ordered on that stream.
 *  - Every function returns a status code (below) and never throws across
 *    the ABI.  Validation failures leave every argument untouched.  The
 *    message of the last failure on the calling thread is returned by
 *    bsmm_last_error().
 *  - Handles are not thread-safe: a handle must not be used by two threads
 *    at once.
 */
#ifndef BSMM_H
#define BSMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bsmm_matrix_s *bsmm_matrix; /* opaque; owns its device memory */

/* Element type of a matrix's block data (paper, Sec. II: the library takes
 * single- and double-precision numbers). */
enum bsmm_dtype {
    BSMM_F64 = 0,  /* double */
    BSMM_F32 = 1   /* float  */
};

enum bsmm_status {
    BSMM_OK = 0,
    BSMM_EINVAL = -1,  /* null pointer, block size < 1, bad scalar, aliasing   */
    BSMM_ESHAPE = -2,  /* block sizes of A, B, C do not conform                 */
    BSMM_EINDEX = -3,  /* malformed row pointer or column indices               */
    BSMM_ENOMEM = -4,  /* the device allocator returned NULL                    */
    BSMM_EDEVICE = -5, /* a HIP runtime error; C's contents are unspecified     */
    BSMM_ERANGE = -6,  /* a size exceeds what the library can index             */
    BSMM_ENOTSUP = -7  /* a supported-but-not-implemented combination           */
};

/*
 * Creates a matrix from block-CSR arrays (paper, Sec. II: blocked CSR).
 *   nbr, row_blk_sizes   block-row count and sizes (host int32[nbr]).
 *   nbc, col_blk_sizes   block-column count and sizes (host int32[nbc]).
 *   nnzb, blk_row_ptr, blk_col_ind   the block pattern (host arrays).
 *   data                 FP64 block values, CSR order, column-major blocks;
 *                        host or device memory as data_on_device says, or
 *                        NULL for all-zero blocks.  Its length is the sum
 *                        of rows(I)*cols(J) over the stored blocks.
 *   stream               stream for the upload.
 *   out                  receives the handle.
 * Every array is copied: the caller may free its inputs on return.  Index
 * and data live in device memory obtained from the registered allocator.
 * Errors: EINVAL (null pointers, sizes < 1, nbr or nbc < 0), EINDEX
 * (malformed index), ERANGE (more than 2^47 elements or 2^31 - 1 blocks),
 * ENOMEM, EDEVICE.
 */
int bsmm_create_matrix(int32_t nbr, const int32_t *row_blk_sizes,
                       int32_t nbc, const int32_t *col_blk_sizes,
                       int64_t nnzb, const int64_t *blk_row_ptr,
                       const int32_t *blk_col_ind, const double *data,
                       int data_on_device, void *stream, bsmm_matrix *out);

/*
 * As bsmm_create_matrix, for block data of element type dtype (BSMM_F64 or
 * BSMM_F32; paper, Sec. II: the library takes single- and double-precision
 * numbers).  data points to dtype values (host or device, or NULL for
 * zeros).  A multiply takes A, B and C of one element type and computes in
 * it: FP32 matrices run the same stacks and kernels in FP32 (FP32 MFMA where
 * FP64 uses FP64 MFMA), with alpha, beta rounded to FP32 and the filter's
 * squared norms summed in FP64.  The split-precision emulation is FP64
 * only.  Errors: as bsmm_create_matrix, plus EINVAL for an unknown dtype.
 */
int bsmm_create_matrix_typed(int32_t nbr, const int32_t *row_blk_sizes,
                             int32_t nbc, const int32_t *col_blk_sizes,
                             int64_t nnzb, const int64_t *blk_row_ptr,
                             const int32_t *blk_col_ind, int32_t dtype,
                             const void *data, int data_on_device, void *stream,
                             bsmm_matrix *out);

/* Element type of a matrix (BSMM_F64 or BSMM_F32). */
int bsmm_matrix_dtype(bsmm_matrix m, int32_t *dtype);

/*
 * C <- filter_eps(beta*C + alpha*A*B) (paper, Sec. II local multiplication;
 * Sec. III densification for fully occupied inputs).
 *   A: nbr x nbk blocks, B: nbk x nbc blocks, C: nbr x nbc blocks; the
 *   block sizes must agree elementwise (A's column sizes = B's row sizes,
 *   C's row sizes = A's, C's column sizes = B's).
 *   beta == 0 overwrites C (NaN/Inf in the old C is ignored); alpha == 0
 *   skips the products (NaN/Inf in A and B is ignored).
 *   The new pattern of C is the old pattern united with every (I,J) for
 *   which some K has A(I,K) and B(K,J) stored.  Then, if filter_eps > 0,
 *   every C block whose squared Frobenius norm is strictly below
 *   filter_eps^2 is removed (a NaN norm keeps the block); blocks that a
 *   norm bound proves will be removed may be left out before their
 *   products are formed (option "prescreen"), with the same result.
 *   A == B is allowed; C must differ from both.
 * The call blocks the host to read the size of the new C pattern, on the
 * stack path the run and product counts of the shape classes, and, when
 * filter_eps > 0, the number of blocks the filter keeps; the rest is
 * stream-ordered.
 * Errors: EINVAL (nulls, C aliasing A or B, filter_eps < 0 or NaN, element
 * types that differ), ESHAPE, ERANGE, ENOMEM, ENOTSUP (incl. option "path"
 * "emul" on FP32 matrices), EDEVICE.  On EINVAL/ESHAPE nothing is modified.
 */
int bsmm_multiply(double alpha, bsmm_matrix A, bsmm_matrix B, double beta,
                  bsmm_matrix C, double filter_eps, void *stream);

/*
 * C <- beta*C + alpha*A*B without allocating device memory, for callers
 * that cannot allocate: code under stream capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arithmetic, paths and options as
 * bsmm_multiply, with these differences:
 *   - C's pattern must already contain every product block (e.g. C is the
 *     output of an earlier bsmm_multiply of the same patterns); C keeps its
 *     pattern and buffers.  Otherwise BSMM_EINDEX, C untouched.
 *   - No filter (filter_eps = 0) and no plan is kept for "plan_cache".
 *   - Every temporary (symbolic counts, product stacks, split-run partial
 *     blocks, dense panels, emulation slices) is carved from a fixed
 *     scratch array of 64 MiB in device memory, one per device, held from
 *     the first call on a device until the process ends.  A multiply whose
 *     temporaries exceed it fails with BSMM_ERANGE before C is written.
 *   - Stack classes are launched one by one (no hipGraph is instantiated).
 * The scratch array keeps the last call's contents and is shared by every
 * call on the device: calls that overlap on one device (two host threads,
 * or two streams not ordered with each other) race on it.  The call blocks
 * the host once to read the product counts, like bsmm_multiply.
 * Errors: as bsmm_multiply, plus EINDEX (pattern) and ERANGE (scratch).
 */
int bsmm_multiply_noalloc(double alpha, bsmm_matrix A, bsmm_matrix B, double beta,
                          bsmm_matrix C, void *stream);

/* Frees a matrix and its device memory (after synchronising the stream it
 * was last used on).  NULL is accepted and ignored. */
int bsmm_destroy_matrix(bsmm_matrix m);

/* Sizes of a matrix: block rows/columns, stored blocks, stored
 * elements.  Any output pointer may be NULL. */
int bsmm_matrix_info(bsmm_matrix m, int32_t *nbr, int32_t *nbc, int64_t *nnzb,
                     int64_t *nelems);

/*
 * Copies a matrix out: blk_row_ptr (host int64[nbr+1]), blk_col_ind (host
 * int32[nnzb]) and data (FP64[nelems], host or device as data_on_device
 * says), the blocks packed in CSR order, each column-major.  Any output
 * pointer may be NULL to skip that part.  Synchronous with respect to the
 * host for host outputs.  (Inside the library a filtered matrix may keep
 * its blocks at their old places with unused space between them; the copy
 * gathers them, through a temporary device buffer of nelems elements for
 * host outputs.)
 */
int bsmm_copy_out(bsmm_matrix m, int64_t *blk_row_ptr, int32_t *blk_col_ind,
                  double *data, int data_on_device, void *stream);

/* As bsmm_copy_out, with data in the matrix's own element type (the only
 * copy-out of FP32 matrices; bsmm_copy_out returns EINVAL for them). */
int bsmm_copy_out_typed(bsmm_matrix m, int64_t *blk_row_ptr, int32_t *blk_col_ind,
                        void *data, int data_on_device, void *stream);

/*
 * Device memory provider.  alloc(bytes, stream, ctx) returns device memory
 * usable on that stream or NULL; dealloc(ptr, bytes, stream, ctx) returns
 * it.  Passing alloc == NULL restores the built-in hipMalloc/hipFree
 * provider.  Memory cached by the library is released (after a device
 * synchronisation) before the provider changes; matrices created under one
 * provider are freed through that same provider.
 */
typedef void *(*bsmm_alloc_fn)(size_t bytes, void *stream, void *ctx);
typedef void (*bsmm_dealloc_fn)(void *ptr, size_t bytes, void *stream, void *ctx);
int bsmm_set_allocator(bsmm_alloc_fn alloc, bsmm_dealloc_fn dealloc, void *ctx);

/*
 * Library options (process-wide).  Keys and values:
 *   "path"        "auto" (default) | "stack" | "dense" | "emul"
 *                 auto takes the dense path iff A and B have every block
 *                 stored (paper, Sec. III: densify when the inputs are
 *                 dense); "dense" forces it (missing blocks read as zero);
 *                 "emul" runs the densified product as split-precision FP64
 *                 emulation on INT8 matrix cores (Ozaki scheme: S digit
 *                 slices of 7 bits per operand with power-of-two row/column
 *                 scales, exact INT32 sums of every digit pair s + t <= S + 1,
 *                 FP64 recombination and native FP64 beta*C)
 *   "emul_slices" S in [1, 8] (default 7)
 *   "emul_kernel" INT8 GEMM of the emulated path: "t128w8" (default; 128 x 64
 *                 outputs per 512-thread workgroup, 32x32x32 MFMA, k step
 *                 32, two LDS stages), "t128k32" (same with 256 threads),
 *                 "t128" (16x16x64 MFMA, k step 64, one stage) or "t64"
 *                 (64 x 64 tiles); every variant gives the same bits
 *   "stack_kernel" "plain" (default) | "tuned"
 *                 plain: one fixed parameter rule per shape, one launch per
 *                 shape class; tuned: parameters from the tuning database,
 *                 else the learned model, else the plain rule, and all shape
 *                 classes launched together as nodes of one hipGraph
 *   "stack_chunk" maximum products per stack launch, "0" = unlimited
 *                 (paper, Sec. II: batches of at most 30000 products)
 *   "stack_tile"  tuned path: "T" > 0 (default "32") runs every FP64 MFMA
                 class of blocks up to 32 x 32 whose runs need no splitting
                 in one launch, its runs ordered by tiles of T x T C blocks
                 (when those classes hold at least 4096 runs); "0" launches
                 every class on its own.  Results are the same bits.
   "jit"         tuned path: "1" compiles, at run time (hiprtc), an FP64 or
                 FP32 MFMA small-block kernel with m, n and k as compile-time
                 constants for every class whose products share one depth
                 k (A's block columns all of one size) and whose parameters
                 select the MFMA kernel; compiled kernels are cached for the
                 process; such classes are launched on their own (no
                 hipGraph).  Without hiprtc, or when a compilation fails,
                 the precompiled kernels run.  "0" (default): precompiled
                 kernels only
   "prescreen"   "1" (default): a filtering multiply (filter_eps >= 1e-150)
                 on the stack path leaves out of C's new pattern every
                 block whose norm bound |alpha| sum_K ||A_IK||_F ||B_KJ||_F
                 + |beta| ||C_IJ||_F, grown by a margin for rounding, lies
                 below filter_eps, and skips its products: such blocks
                 always fail the filter, so C is the same as with "0",
                 which forms every block of the product pattern first
   "stack_at"    scheduled launch: "1" reads A's blocks from row-major
                 copies made for the multiply (one vector load per four k
                 values), "0" reads them in place, "auto" (default) copies
                 for FP32 matrices only; the same bits either way (not in
                 bsmm_multiply_noalloc, which makes no copies)
   "stack_sched" order in which the scheduled launch's waves take runs:
                 "dynamic" (default; a run counter, several short runs per
                 update) or "static" (fixed strides, numbered XCD by XCD)
   "stack_panel" maximum products held in the stacks at once (default
 *                 "1073741824", 16 GiB of product entries; "0" = no
 *                 limit): a multiply with more products builds and runs
 *                 its stacks over panels of consecutive C block rows, one
 *                 panel after another on the stream (a row whose products
 *                 alone exceed the limit forms a panel of its own); such a
 *                 multiply leaves no plan for "plan_cache" to replay
 *   "verbose"     "1": one line on stderr per stack row panel as it is
 *                 queued (progress of long multiplies); "0" (default): quiet
 *   "tune_db"     path of a tuning database file ("" = none)
 *   "mlp_weights" path of a learned-model weight file ("" = none)
 *   "stack_params" "TM TN KC WAVES": the tuned path uses this parameter
 *                 set for every shape class ("" = select per shape)
 *   "dense_kb"    k step of the dense FP64 GEMM: "16" (default; 64 KB of
 *                 LDS, two workgroups per CU) or "32" (128 KB, one per CU)
 *   "plan_cache"  "1": a multiply into C keeps its plan (symbolic totals,
 *                 stacks, launches or instantiated hipGraph); the next
 *                 multiply into C with the same A and B handles, unchanged
 *                 patterns and buffers of A, B and C, the same alpha, beta
 *                 and options skips the symbolic phase and the stack build
 *                 and replays the launches (no host synchronisation unless
 *                 the filter drops blocks).  "0" (default) plans every call.
 *   "time_kernels" "1" brackets every dense-GEMM and stack-kernel launch
 *                 with HIP events on the launch stream (see
 *                 bsmm_kernel_times); "0" (default) records nothing
 * Errors: EINVAL for an unknown key or value.
 */
int bsmm_set_option(const char *key, const char *value);

/* Reads an option into buf (NUL-terminated, truncated to len). */
int bsmm_get_option(const char *key, char *buf, size_t len);

/* Message of the last failure on the calling thread ("" if none). */
const char *bsmm_last_error(void);

/*
 * Facts about the last bsmm_multiply on the calling thread, for tests and
 * benchmarks: which path ran, how many block products A*B has and how many
 * were computed, how many C-block runs the stacks held, how many shape
 * classes, the algorithmic FP64 flop count of A*B (sum of 2*m*n*k over its
 * block products), the C blocks the norm-bound screen left out, and the C
 * block count before and after the filter.
 */
typedef struct bsmm_multiply_stats {
    int32_t path;          /* 1 = stack, 2 = dense (merged panels)          */
    int32_t n_classes;     /* shape classes (m, n) holding at least one run */
    int64_t n_products;    /* block products (I, K, J) of A*B               */
    int64_t n_runs;        /* C blocks receiving at least one product       */
    int64_t c_nnzb_before; /* C blocks before the filter (after the screen) */
    int64_t c_nnzb_after;  /* C blocks after the filter                     */
    double flops;          /* sum of 2*m*n*k over the block products of A*B */
    int64_t n_row_panels;  /* stack path: C block-row panels the stacks were
                              built and run in (option "stack_panel"); 0 on
                              the other paths                               */
    int64_t n_sched_runs;  /* runs executed by the scheduled small-block
                              launch (tuned path, option "stack_tile")      */
    int64_t n_jit_classes; /* shape classes run on run-time compiled
                              kernels (tuned path, option "jit")            */
    int64_t n_screened;    /* C blocks left out by the norm-bound screen
                              (option "prescreen"); their products are
                              not computed                                  */
    int64_t n_products_run; /* block products computed (n_products less
                              those of screened blocks; 0 on path 0)        */
} bsmm_multiply_stats;
int bsmm_last_stats(bsmm_multiply_stats *out);

/*
 * Builds the product stacks of C = A*B (C's pattern must already contain
 * the product pattern, e.g. the output of an earlier multiply) and copies
 * them to the host, for inspection.  Runs are ordered by shape class, then
 * by C block index; the products of one run are ordered by ascending K.
 *   n_runs, n_products: in = capacity of the arrays, out = counts.
 *   run_cblk[r]   C block index of run r (CSR position in C)
 *   run_class[r]  class id of run r (index into the sorted distinct (m, n))
 *   run_ptr[r]    first product of run r; run_ptr[n_runs] = n_products
 *   prod_ablk[p], prod_bblk[p]  A and B block indices (CSR positions)
 * Arrays may be NULL to query the counts only.  Errors: as bsmm_multiply,
 * plus ERANGE when a capacity is too small, EINDEX when C's pattern misses
 * a product block.
 */
int bsmm_inspect_stacks(bsmm_matrix A, bsmm_matrix B, bsmm_matrix C,
                        int64_t *n_runs, int64_t *n_products,
                        int64_t *run_cblk, int32_t *run_class, int64_t *run_ptr,
                        int64_t *prod_ablk, int64_t *prod_bblk, void *stream);

/*
 * Run-time compiled kernels of option "jit", process-wide: kernels
 * compiled, launches served from the cache, compilations that failed (or
 * found no hiprtc), and the total compilation time.  Outputs may be NULL.
 */
int bsmm_jit_stats(int64_t *compiled, int64_t *cache_hits, int64_t *failures, double *compile_ms);

/*
 * Measured rates of the current device, for the rooflines (each output may
 * be NULL to skip that measurement): fp64_mfma, fp32_mfma (TFLOP/s),
 * int8_mfma (TOP/s) and bf16_mfma (TFLOP/s) from long loops of independent
 * v_mfma_f64_16x16x4, v_mfma_f32_16x16x4, v_mfma_i32_32x32x32_i8 and
 * v_mfma_f32_32x32x16_bf16 on register operands at 32 waves per CU;
 * fp64_valu (TFLOP/s) from independent v_fma_f64 chains;
 * hbm_gbs (GB/s, bytes read + written) from a 16-byte-vector copy between
 * two device buffers of copy_bytes each (taken from the registered
 * allocator), hbm_read_gbs (GB/s) from reading one of them.  Each figure
 * is one timed launch after an untimed one.
 * Errors: EINVAL (copy_bytes outside [0, 64 GiB]), ENOMEM, EDEVICE.
 */
int bsmm_measure_peaks(double *fp64_mfma, double *fp32_mfma, double *int8_mfma, double *bf16_mfma,
                       double *fp64_valu, double *hbm_gbs, double *hbm_read_gbs, int64_t copy_bytes,
                       void *stream);

/*
 * Device time of the recorded kernel launches (option "time_kernels"):
 * total milliseconds and launch counts of the dense GEMM and of the
 * small-block stack kernels.  Waits for the recorded events.  reset != 0
 * forgets the recorded launches afterwards.  Output pointers may be NULL.
 */
int bsmm_kernel_times(double *gemm_ms, int64_t *gemm_launches, double *stack_ms,
                      int64_t *stack_launches, int reset);

/*
 * Autotuning (paper, Sec. II: the small-matrix kernels are parametrised by
 * algorithm, work per thread block, elements per thread and tiling, and an
 * autotuner times the parameter sets of each (m, n, k)).
 *
 * A parameter set is 4 int32: register tile rows TM and columns TN per lane
 * (each in {1,2,3,4,5,6,8}) of the FP64 VALU kernel, k chunk staged per step
 * (0 = as large as LDS allows), waves per workgroup (1, 2 or 4; 0 = as many
 * as fit).  TM = TN = 16 selects the FP64 MFMA kernel instead (one wave per
 * C block, 16 x 16 tiles of v_mfma_f64_16x16x4, blocks up to 64 x 64; the k
 * chunk is ignored).
 *
 * The run length is the number of products per C block; short and long runs
 * favour different sets, so the database and the learned model are keyed by
 * it as well as by the shape.
 *
 * bsmm_tune_candidates: the legal candidate sets of shape (m, n, k).
 *   *n_cands: in = capacity (sets), out = count; cands may be NULL to query.
 * bsmm_tune_shape: times each candidate on a synthetic stack of n_runs C
 *   blocks of m x n, each receiving run_len products of k-deep blocks drawn
 *   from pools of 4096 A and 4096 B blocks; one warm-up launch, then reps
 *   timed launches (HIP events); out_us[c] = median microseconds, or -1 when
 *   the set cannot be launched.  1 <= m, n, k <= 256; n_runs * run_len <=
 *   2^26.  The library's own device memory holds the synthetic data.
 * bsmm_select_params: the parameters the tuned path uses for (m, n, k) in
 *   runs of about run_len products: the database entry of that shape timed
 *   at the run length nearest to run_len (log scale), else the learned
 *   model's choice for min(run_len, 32) (32: the longest run length the
 *   tuner times and the model is trained on), else the plain rule.  Database lines are
 *   "m n k R tm tn kc waves [best_us plain_us]"; lines without R
 *   ("m n k tm tn kc waves [best_us plain_us]") count as R = 8; lines of
 *   any other length are skipped.  run_len < 1: BSMM_EINVAL.
 */
int bsmm_tune_candidates(int32_t m, int32_t n, int32_t k, int32_t *n_cands, int32_t *cands);
int bsmm_tune_shape(int32_t m, int32_t n, int32_t k, int64_t n_runs, int32_t run_len,
                    int32_t n_cands, const int32_t *cands, int32_t reps, double *out_us,
                    void *stream);
int bsmm_select_params(int32_t m, int32_t n, int32_t k, int32_t run_len, int32_t *params4);

/*
 * Learned performance model (paper, Sec. II: a model learned from part of the
 * tuning data predicts performance for the whole shape set).  An FP32 MLP
 *     y = W3 relu(W2 relu(W1 x + b1) + b2) + b3,  hidden width 64,
 * maps the normalised features x of (shape, parameter set) to a predicted
 * (standardised) log kernel time.  Parameters are one float array of
 * bsmm_mlp_param_count() values: W1 [64 x F] row-major, b1 [64], W2 [64 x 64]
 * row-major, b2 [64], W3 [64], b3 [1].  Every array argument is host memory;
 * the work runs on the device (null stream) and the call returns when done.
 *
 * bsmm_mlp_features: the F raw features of (m, n, k, run_len, params4)
 *   (F = 11 here): log2 m, log2 n, log2 k, TM, TN, log2 effective k chunk,
 *   waves per workgroup, log2 lanes (or MFMA tiles) holding the block,
 *   fraction of the tiles that covers the block (times the k fill of 4-deep
 *   steps for the MFMA kernel), 1 for the MFMA kernel else 0, log2 run_len.
 *   Training and selection both use this definition; a weight file trained
 *   on another feature count is not used for selection.
 * bsmm_mlp_forward: y[i] for the n rows of x (n x F, row-major).
 * bsmm_mlp_grad: gradient of the mean squared error over the n samples
 *   (per-sample gradients summed in sample order) and the loss.
 * bsmm_mlp_adam_step: one Adam update (step >= 1) of params with moment
 *   arrays m, v (updated in place).
 * bsmm_mlp_train: epochs of minibatch Adam (batch size, learning rate; the
 *   sample order of every epoch is a Fisher-Yates shuffle driven by a 64-bit
 *   LCG seeded with seed); params are updated in place; final_loss = mean
 *   squared error over all samples afterwards.
 * The tuned path loads a model from the file named by option "mlp_weights"
 * (text: "bsmm-mlp features F mean ... std ... params COUNT ...") and, for a
 * shape missing from the tuning database, takes the candidate with the
 * lowest prediction.  Errors: EINVAL on bad arguments, ERANGE for more
 * than 4 (2^22 - 1) samples (forward, grad, train), ENOMEM, EDEVICE.
 */
int bsmm_mlp_param_count(int32_t n_features, int64_t *count);
int bsmm_mlp_features(int32_t m, int32_t n, int32_t k, int32_t run_len, const int32_t *params4,
                      float *features, int32_t *n_features);
int bsmm_mlp_forward(int32_t n_features, const float *params, int64_t n, const float *x, float *y);
int bsmm_mlp_grad(int32_t n_features, const float *params, int64_t n, const float *x,
                  const float *t, float *grad, float *loss);
int bsmm_mlp_adam_step(int32_t n_features, float *params, const float *grad, float *m, float *v,
                       int32_t step, float lr, float beta1, float beta2, float eps);
int bsmm_mlp_train(int32_t n_features, float *params, int64_t n, const float *x, const float *t,
                   int32_t epochs, int32_t batch, float lr, uint64_t seed, float *final_loss);

#ifdef __cplusplus
}
#endif

#endif /* BSMM_H */
