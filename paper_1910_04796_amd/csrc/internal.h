// internal.h -- shared declarations of the bsmm library (not installed).
//
// Layout of a matrix in device memory (one handle, all owned by the handle):
//   d_rbs/d_cbs        int32 block sizes
//   d_row_off/d_col_off int64 element offset of every block row / column
//   d_row_map/d_col_map int2 per element row / column: (block, index inside)
//   d_row_ptr/d_col_ind int64[nbr+1] / int32[nnzb] block-CSR pattern
//   d_blk_off          int64[nnzb+1] element offset of every block
//   d_data             FP64 blocks, CSR order, column-major inside a block
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/bsmm.h"

namespace bsmm {

// ------------------------------------------------------------------ errors
void set_error(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();
int last_code();

#define BSMM_HIP(call)                                                                   \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess) {                                                          \
            ::bsmm::set_error(BSMM_EDEVICE, "%s failed: %s (%s:%d)", #call,              \
                              hipGetErrorString(e_), __FILE__, __LINE__);                \
            return BSMM_EDEVICE;                                                         \
        }                                                                                \
    } while (0)

#define BSMM_TRY(expr)                  \
    do {                                \
        int s_ = (expr);                \
        if (s_ != BSMM_OK) return s_;   \
    } while (0)

// Checks the last kernel launch.
int launch_check(const char *what);

// --------------------------------------------------------------- options
struct Options {
    int path = 0;          // 0 auto, 1 stack, 2 dense, 3 emulated dense
    int emul_slices = 7;   // digit slices of the emulated path
    int stack_kernel = 0;  // 0 plain, 1 tuned
    int64_t stack_chunk = 0;
    int64_t stack_panel = int64_t(1) << 30;  // products of one row panel of stacks (0: no limit)
    int time_kernels = 0;
    int verbose = 0;       // one stderr line per stack row panel
    int dense_kb = 16;             // k step of the dense FP64 GEMM (16 or 32)
    int emul_kernel = 3;           // emulated GEMM: 0 t64, 1 t128, 2 t128k32, 3 t128w8
    int plan_cache = 0;            // reuse symbolic result + stacks + graph when patterns repeat
    std::string tune_db;
    std::string mlp_weights;
    int forced[4] = {0, 0, 0, 0};  // "stack_params": tm tn kc waves for every class
    int jit = 0;           // tuned path: run-time compiled kernels for classes of one product depth
    int stack_tile = 32;   // tuned path: > 0 runs MFMA classes in one launch, tiles of this many blocks
    int stack_sched = 1;   // scheduled kernel: 0 static XCD-aware striding, 1 dynamic run counter
    int prescreen = 1;     // stack path with eps > 0: leave out C blocks whose norm bound is below eps
    int stack_at = -1;     // scheduled launch reads A's blocks transposed: 1 on, 0 off, -1 FP32 only
};
Options &options();

// Brackets one kernel launch with HIP events when "time_kernels" is on.
// kind 0: dense GEMM, kind 1: small-block stack kernel.
class KernelTimer {
  public:
    KernelTimer(int kind, hipStream_t s);
    ~KernelTimer();

  private:
    int kind_;
    hipStream_t s_;
    void *a_ = nullptr, *b_ = nullptr;
};

// ------------------------------------------------------------ device pool
// Device memory comes from the registered provider (default hipMalloc) and
// is cached by the library; blocks are stream-ordered on the stream they
// were last used on.
void *dev_alloc(size_t bytes, hipStream_t s);
void dev_free(void *p, hipStream_t s);
int pool_release_all();

// A fixed region of device memory that temporaries are carved from (bump
// order, 256-byte aligned, never returned) while an allocation-free multiply
// runs on the calling thread.
struct ScratchArena {
    char *base = nullptr;
    size_t cap = 0, used = 0;
};
// The calling thread's active arena, or null (temporaries from the pool).
ScratchArena *&scratch_arena();

// A device buffer owned by RAII (freed back to the pool; a buffer carved
// from a scratch arena is only forgotten).
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    hipStream_t s = nullptr;
    bool borrowed = false;  // carved from a scratch arena
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept { *this = std::move(o); }
    DevBuf &operator=(DevBuf &&o) noexcept {
        if (this != &o) {
            reset();
            p = o.p; bytes = o.bytes; s = o.s; borrowed = o.borrowed;
            o.p = nullptr; o.bytes = 0; o.borrowed = false;
        }
        return *this;
    }
    ~DevBuf() { reset(); }
    void reset() {
        if (p && !borrowed) dev_free(p, s);
        p = nullptr;
        bytes = 0;
        borrowed = false;
    }
    // Ensures capacity >= n bytes (contents are not preserved).
    int reserve(size_t n, hipStream_t st) {
        s = st;
        if (n <= bytes && p) return BSMM_OK;
        reset();
        size_t want = n ? n : 1;
        if (ScratchArena *ar = scratch_arena()) {
            const size_t at = (ar->used + 255) & ~size_t(255);
            if (at > ar->cap || want > ar->cap - at) {
                set_error(BSMM_ERANGE, "temporaries exceed the %zu-byte scratch region (%zu more bytes)",
                          ar->cap, want);
                return BSMM_ERANGE;
            }
            p = ar->base + at;
            ar->used = at + want;
            bytes = want;
            borrowed = true;
            return BSMM_OK;
        }
        p = dev_alloc(want, st);
        if (!p) {
            set_error(BSMM_ENOMEM, "device allocation of %zu bytes failed", want);
            return BSMM_ENOMEM;
        }
        bytes = want;
        return BSMM_OK;
    }
    template <class T> T *as() const { return static_cast<T *>(p); }
};

}  // namespace bsmm

namespace bsmm {
struct Plan;
void free_plan(Plan *p);
uint64_t next_version();
}  // namespace bsmm

// ------------------------------------------------------------------ matrix
struct bsmm_matrix_s {
    int32_t nbr = 0, nbc = 0;
    std::vector<int32_t> rbs, cbs;          // host copies of the block sizes
    std::vector<int64_t> row_off, col_off;  // host element offsets (nbr+1, nbc+1)
    int64_t nnzb = 0, nelems = 0;        // nelems: elements of the stored blocks
    int32_t max_rbs = 0, max_cbs = 0;
    // Block b's data starts at blk_off[b] and holds rbs(row) * cbs(col)
    // elements, column-major; blocks are in CSR order.  The storage is
    // packed (blk_off[b + 1] - blk_off[b] is the block's size) except after
    // a filter that dropped blocks: their space stays behind as unused gaps
    // until the pattern next changes (holes = true; blk_off[nnzb] is then
    // the end of the storage, not nelems).
    int device = 0;
    int dtype = BSMM_F64;          // element type of the block data
    hipStream_t last_stream = nullptr;
    uint64_t version = 0;          // changes whenever the pattern or a buffer changes
    bsmm::Plan *plan = nullptr;    // cached multiply plan of which this matrix is C
    ~bsmm_matrix_s() { bsmm::free_plan(plan); }

    bsmm::DevBuf b_rbs, b_cbs, b_row_off, b_col_off, b_row_map, b_col_map;
    bsmm::DevBuf b_row_ptr, b_col_ind, b_blk_off, b_data;

    int32_t *d_rbs() const { return b_rbs.as<int32_t>(); }
    int32_t *d_cbs() const { return b_cbs.as<int32_t>(); }
    int64_t *d_row_off() const { return b_row_off.as<int64_t>(); }
    int64_t *d_col_off() const { return b_col_off.as<int64_t>(); }
    int2 *d_row_map() const { return b_row_map.as<int2>(); }
    int2 *d_col_map() const { return b_col_map.as<int2>(); }
    int64_t *d_row_ptr() const { return b_row_ptr.as<int64_t>(); }
    int32_t *d_col_ind() const { return b_col_ind.as<int32_t>(); }
    int64_t *d_blk_off() const { return b_blk_off.as<int64_t>(); }
    double *d_data() const { return b_data.as<double>(); }
    void *d_raw() const { return b_data.p; }
    size_t esize() const { return dtype == BSMM_F32 ? sizeof(float) : sizeof(double); }
    int64_t rows() const { return row_off.empty() ? 0 : row_off.back(); }
    int64_t cols() const { return col_off.empty() ? 0 : col_off.back(); }
    bool full() const { return nnzb == (int64_t)nbr * (int64_t)nbc; }
    bool holes = false;
    int64_t storage = 0;  // elements the data buffer holds (blk_off[nnzb])
};

namespace bsmm {

// ------------------------------------------------------- device utilities
// Exclusive prefix sum of n int64 values: out[0..n] with out[n] = total.
// in and out may alias.  Temporary storage comes from the pool.
int scan_exclusive_i64(const int64_t *in, int64_t *out, int64_t n, hipStream_t s);

// ---------------------------------------------------------------- index
// Builds d_blk_off (int64[nnzb+1]) of a pattern from per-row element totals
// (computed here when d_row_elems is null): scan, then per-row offsets.
int build_block_offsets(const int32_t *d_rbs, const int32_t *d_cbs, int32_t nbr,
                        const int64_t *d_row_ptr, const int32_t *d_col_ind, int64_t nnzb,
                        int64_t *d_blk_off, const int64_t *d_row_elems, hipStream_t s);

// Symbolic phase: per block row of C, the size of old-C united with the
// product pattern.  Outputs per row: block count, element count, product
// count and algorithmic flops.
struct SymbolicTotals {
    int64_t nnzb = 0, nelems = 0, nprod = 0;
    double flops = 0.0;
    bool screen = false;      // the norm-bound screen chose the pattern
    int64_t screened = 0;     // C blocks left out by the screen
    int64_t old_screened = 0; // of them, blocks of the old C pattern
};
// Inputs of the symbolic screen: per-block Frobenius norms of A, B and (for
// beta != 0) the old C, |alpha|, |beta|, the filter threshold and the
// relative margin left for rounding.
struct ScreenNorms {
    const double *a = nullptr, *b = nullptr, *c = nullptr;
    double alpha_abs = 0.0, beta_abs = 0.0, eps = 0.0, margin = 0.0;
};
// Widest C (block columns) the screen handles: a bound per column in LDS.
constexpr int32_t kScreenMaxCols = 7680;
int block_norms(const bsmm_matrix_s *M, double *d_out, hipStream_t s);
// Block row of every block (int32[nnzb]) of a matrix with gaps in its
// storage, where offsets do not give block sizes; out stays empty (null)
// for packed storage.
int block_rows(const bsmm_matrix_s *M, DevBuf &out, hipStream_t s);
int symbolic_count_screen(const bsmm_matrix_s *A, const bsmm_matrix_s *B, const bsmm_matrix_s *C,
                          const ScreenNorms &sn, uint32_t *d_bits, int64_t *d_row_nnz,
                          int64_t *d_row_elems, int64_t *d_row_prod, double *d_row_flops,
                          int64_t *d_row_screened, int64_t *d_row_old_screened, hipStream_t s);
int symbolic_fill_bits(int32_t nbr, int32_t nbc, const uint32_t *d_bits, const int64_t *d_new_row_ptr,
                       int32_t *d_new_col_ind, hipStream_t s);
int symbolic_count(const bsmm_matrix_s *A, const bsmm_matrix_s *B, const bsmm_matrix_s *C,
                   int64_t *d_row_nnz, int64_t *d_row_elems, int64_t *d_row_prod,
                   double *d_row_flops, hipStream_t s);
int symbolic_fill(const bsmm_matrix_s *A, const bsmm_matrix_s *B, const bsmm_matrix_s *C,
                  const int64_t *d_new_row_ptr, int32_t *d_new_col_ind, hipStream_t s);
// Every block present: row_ptr[i] = i*nbc, col_ind = 0..nbc-1 per row,
// row_elems[i] = rbs[i] * ncols.
int full_pattern(int32_t nbr, int32_t nbc, int64_t ncols, int64_t *d_row_ptr,
                 int32_t *d_col_ind, int64_t *d_row_elems, const int32_t *d_rbs, hipStream_t s);
// Copies old C blocks into the new layout (zeros for new blocks).
int relayout(const bsmm_matrix_s *Cold, const int64_t *d_new_rp, const int32_t *d_new_ci,
             const int64_t *d_new_off, void *d_new_data, hipStream_t s);
// data *= beta (beta == 0 writes zeros) over the blocks whose flag is zero
// (flags == nullptr: every block).
int scale_blocks(const bsmm_matrix_s *C, const int64_t *d_flags, double beta, hipStream_t s);
int fill_zero(double *p, int64_t n, hipStream_t s);
int fill_zero_bytes(void *p, size_t bytes, hipStream_t s);
int fill_value(double *p, int64_t n, double v, hipStream_t s);

// ---------------------------------------------------------------- stacks
// A product entry keeps A's element offset in 48 bits and k in 16 bits.
constexpr int kMaxStackK = 0xFFFF;
// Block columns of C the count and fill phases map in LDS (64 KB) at once;
// wider C rows are mapped in windows of kStackWin block columns, each B
// block row's share of every window found once per multiply.
constexpr int kMaxStackCols = 8192;
constexpr int kStackWin = 4096;
// Product stacks of C += A*B, grouped by shape class (m, n).
struct Stacks {
    int64_t n_runs = 0, n_prod = 0;
    int32_t n_classes = 0;            // distinct (m, n) classes (all, including empty)
    int32_t nrs = 0, ncs = 0;         // distinct row sizes / column sizes of C
    std::vector<int32_t> row_sizes;   // sorted distinct C block-row sizes
    std::vector<int32_t> col_sizes;   // sorted distinct C block-column sizes
    std::vector<int64_t> class_begin; // run range of class cl: [cb[cl], cb[cl+1])
    std::vector<int64_t> class_prod_begin;  // first product of class cl (ncl + 1 entries)
    DevBuf run_cblk;   // int64[n_runs]   C block index
    DevBuf run_coff;   // int64[n_runs]   C element offset
    DevBuf run_ptr;    // int64[n_runs+1] first product
    DevBuf run_class;  // int32[n_runs]
    DevBuf prods;      // ulonglong2[n_prod]: {a_off | k << 48, b_off}
    DevBuf c_count;    // int64[C.nnzb]   products per C block
    DevBuf c_row;      // int32[C.nnzb]   block row of every C block
    DevBuf run_of_c;   // int64[C.nnzb]   run of every C block in its panel, or -1
    DevBuf d_rsi, d_csi, missing;     // size-class index of rows / columns; pattern flag
    bool screened = false;            // C's pattern came from the screen: products of left-out blocks are skipped
    DevBuf a_t;                       // A's blocks transposed, for the scheduled launch (option stack_at)
    bool a_t_fresh = false;           // a_t holds this multiply's A (later row panels reuse it)
    int kparts = 1;                   // parts per A block row in count and fill
    DevBuf pcount;                    // int64[C.nnzb * kparts]: first position of each part (kparts > 1)
    int nwin = 0;                     // column windows of a C wider than kMaxStackCols (else 0)
    DevBuf b_split;                   // int64[B.nbr * (nwin + 1)]: first entry of each B row in each window
    DevBuf sched;                     // uint64[n_sched]: scheduled runs (run << 16 | m << 8 | n)
    int64_t n_sched = 0;
    DevBuf sched_next;                // uint64 run counter of the dynamic schedule
    int n_jit = 0;                    // classes on run-time compiled kernels
    std::vector<char> class_active;   // class holds runs (any panel so far)
    std::vector<int> run_len_hint;    // mean run length per class over every panel (else empty)
};
// Whole stacks: stack_count, then stack_rows over every C block row.
// st.n_prod must hold the product count of the symbolic phase on entry.
int build_stacks(const bsmm_matrix_s *A, const bsmm_matrix_s *B, const bsmm_matrix_s *C,
                 Stacks &st, hipStream_t s);
// Products per C block for every C block row (and the size classes).
int stack_count(const bsmm_matrix_s *A, const bsmm_matrix_s *B, const bsmm_matrix_s *C,
                Stacks &st, hipStream_t s);
// After stack_count: products and C blocks before every C block row
// (host vectors of nbr + 1 entries); EINDEX when C misses a product block.
int stack_row_bounds(const bsmm_matrix_s *C, const Stacks &st, std::vector<int64_t> *prod_before,
                     std::vector<int64_t> *blk_before, hipStream_t s);
// After stack_count: the mean run length (products per C block receiving
// any) of every class over all C block rows.
int stack_class_run_lengths(const bsmm_matrix_s *C, const Stacks &st, std::vector<int> *out,
                            hipStream_t s);
// The scheduled kernel's run order: the runs of the classes flagged in
// `eligible` (one flag per class), grouped by tiles of tile x tile C blocks
// (tiles in row-major order), with each entry's block shape.
int build_schedule(const bsmm_matrix_s *C, Stacks &st, const std::vector<char> &eligible, int tile,
                   hipStream_t s);
// After stack_count: the runs and products of C block rows [r0, r1) (C
// blocks [c0, c1), at most nprod products), replacing the previous panel's;
// st.n_prod is set to the count held.
int stack_rows(const bsmm_matrix_s *A, const bsmm_matrix_s *B, const bsmm_matrix_s *C,
               Stacks &st, int32_t r0, int32_t r1, int64_t c0, int64_t c1, int64_t nprod,
               hipStream_t s);

// --------------------------------------------------------- small blocks
// Parameters of the small-block kernel (the tuning space): register tile
// TM x TN per lane (TM, TN in {1,2,3,4,5,6,8}), k chunk staged per step
// (0 = as large as LDS allows), waves per workgroup (0 = as many as fit,
// at most 4).
struct SmmParams {
    int tm = 0, tn = 0, kc = 0, waves = 0;
};
// tm = tn = kMfmaTile selects the FP64 MFMA small-block kernel (kc unused).
constexpr int kMfmaTile = 16;
// Length of the learned model's feature vector (mlp_features).
constexpr int kMlpFeatures = 11;
// Compute units of the current device (cached per device; 256 if unknown).
int cu_count();
// Longest run length the tuner times (and the model is trained on); longer
// runs are presented to the model as runs of this length.
constexpr int kMlpMaxRunLen = 32;
// Kernel arguments of one small-block launch.
struct SmmArgs {
    const void *A;          // block data of the matrix's element type
    const void *B;
    void *C;
    const int64_t *run_coff;
    const int64_t *run_ptr;
    const ulonglong2 *prods;
    int64_t run_begin, run_end;
    int m, n;
    int tiles_m, tiles_n;   // register tiles covering the C block
    int L;                  // lanes per group (min(tiles, 64))
    int G;                  // groups per wave
    int passes;             // ceil(tiles / L)
    int region;             // doubles of LDS per group
    int kc_max;             // largest k chunk that fits the region
    double alpha, beta;
    // MFMA kernel only: each run's products are cut into `split` segments
    // handled by different waves; split > 1 writes unscaled partial blocks
    // to part[((r - run_begin) * split + segment) * m * n] (column-major)
    // and k_smm_split_reduce applies the epilogue.
    int split;
    void *part;
    // Scheduled MFMA kernel (one launch for every class with blocks up to
    // 32 x 32): entries run << 16 | m << 8 | n in tile order; mode 0 static
    // XCD-aware striding, 1 a run counter (*next, zeroed before the launch).
    const unsigned long long *sched;
    int64_t n_sched;
    unsigned long long *next;
    int sched_mode;
    int sched_chunk;        // schedule entries taken per wave at a time
    // Scheduled kernel, when the multiply filters: squared Frobenius norm of
    // every finished C block, norm2[run_cblk[r]] (run_cblk: C block of run r).
    double *norm2;
    const int64_t *run_cblk;
    // Scheduled kernel reading A's blocks transposed (row-major copies at
    // the same offsets), or null.
    const void *A_t;
};
// Squared block norms the scheduled kernel writes for the filter during the
// current multiply on this thread (nullptr: none); set around the numeric
// phase by the multiply.
void set_norm_sink(double *norm2);
double *norm_sink();
// A planned launch: kernel, shape-dependent arguments, block size, LDS.
struct SmmLaunch {
    void *fn = nullptr;
    SmmArgs args{};
    int waves = 1;
    size_t lds = 0;
    int dtype = BSMM_F64;   // element type the kernel was planned for
    hipFunction_t jit_fn = nullptr;  // run-time compiled kernel (then fn is unused)
};
// dtype: BSMM_F64 or BSMM_F32 (the kernel and the LDS budget follow it).
int plan_smm(const SmmParams &prm, int m, int n, int kmax, int dtype, SmmLaunch *out);
unsigned smm_grid(const SmmLaunch &L, int64_t nruns);
int launch_smm(SmmLaunch L, const void *A, const void *B, void *C, const int64_t *run_coff,
               const int64_t *run_ptr, const ulonglong2 *prods, int64_t rb, int64_t re,
               double alpha, double beta, hipStream_t s);
using LaunchList = std::vector<std::pair<SmmLaunch, std::pair<int64_t, int64_t>>>;
// Launches of one stack execution: per-class launches (plain) or one
// instantiated hipGraph holding every class (tuned).
// Hands an executable graph to the retire list: it is destroyed once `done`
// (recorded after its last launch) has completed, never while it may still
// run on the device.
void retire_graph(hipGraphExec_t exec, hipEvent_t done);
struct StackExec {
    LaunchList launches;
    std::vector<DevBuf> parts;  // partial blocks of split launches
    bool reads_a_t = false;     // a launch reads the stacks' transposed copy of A
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;  // recorded after every launch of exec
    StackExec() = default;
    StackExec(const StackExec &) = delete;
    StackExec &operator=(const StackExec &) = delete;
    ~StackExec() {
        if (exec) retire_graph(exec, done);
        else if (done) (void)hipEventDestroy(done);
    }
};
// Run-time specialised MFMA small-block kernel for products of one shape
// (m, n, k), compiled with hiprtc on first use and cached per device;
// nullptr when hiprtc or the compilation is unavailable.
hipFunction_t jit_smm_kernel(int dtype, int m, int n, int k);
int launch_jit_smm(hipFunction_t fn, unsigned grid, int waves, const void *A, const void *B, void *C,
                   const int64_t *run_coff, const int64_t *run_ptr, const ulonglong2 *prods,
                   int64_t rb, int64_t re, double alpha, double beta, hipStream_t s);
struct JitStats {
    int64_t compiled = 0, cache_hits = 0, failures = 0;
    double compile_ms = 0.0;
};
JitStats jit_stats();
SmmParams plain_params(int m, int n);
// Selected parameters for shape (m, n, k) in runs of about run_len products
// per C block: tuning database, then learned model, then the plain rule.
SmmParams select_params(int m, int n, int k, int run_len);
// Legal candidate parameter sets of a shape (the tuning space).
std::vector<SmmParams> candidate_params(int m, int n, int k);
// Learned model: ranks the candidates of (m, n, k) by predicted time; false
// when no model is loaded.
bool mlp_select(int m, int n, int k, int run_len, SmmParams *out);
// Plans and launches the stack kernels; the launches (and the instantiated
// graph of the tuned path) are kept in *ex for replay.
int run_stacks(const bsmm_matrix_s *A, const bsmm_matrix_s *B, bsmm_matrix_s *C, Stacks &st,
               double alpha, double beta, hipStream_t s, StackExec *ex);
int build_graph(const LaunchList &launches, const bsmm_matrix_s *A, const bsmm_matrix_s *B,
                bsmm_matrix_s *C, const Stacks &st, double alpha, double beta,
                hipGraphExec_t *out);
int replay_stacks(const StackExec &ex, const bsmm_matrix_s *A, const bsmm_matrix_s *B,
                  bsmm_matrix_s *C, const Stacks &st, double alpha, double beta, hipStream_t s);

// ----------------------------------------------------------------- dense
int dense_multiply(const bsmm_matrix_s *A, const bsmm_matrix_s *B, bsmm_matrix_s *C,
                   double alpha, double beta, hipStream_t s);

// Split-precision FP64 emulation of the dense product on INT8 matrix cores.
int emul_multiply(const bsmm_matrix_s *A, const bsmm_matrix_s *B, bsmm_matrix_s *C,
                  double alpha, double beta, int S, hipStream_t s);
int64_t emul_chunk(int S);

// ---------------------------------------------------------------- filter
// pre_norm2 (nullable): squared block norms already computed (negative:
// not computed), used in place of reading those blocks.
int filter_blocks(bsmm_matrix_s *C, double eps, int64_t *nnzb_after, hipStream_t s,
                  const double *pre_norm2 = nullptr);

// ------------------------------------------------------- fixed pattern
// C <- beta*C + alpha*A*B into C's existing pattern and buffers, with every
// temporary carved from the active scratch arena (no filter, no plan kept,
// stack classes launched one by one instead of through a hipGraph).
// EINDEX when C's pattern misses a product block (C untouched).
int multiply_fixed_pattern(double alpha, bsmm_matrix_s *A, bsmm_matrix_s *B, double beta,
                           bsmm_matrix_s *C, hipStream_t s);

// --------------------------------------------------------------- helpers
inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
// Largest one-dimensional grid in workgroups: a launch counts its grid in
// work-items with 32 bits, so gridDim.x * blockDim.x must stay below 2^32
// (past it the launch is refused, or wraps to a smaller grid); with up to
// 1024 threads per workgroup that allows 2^22 - 1 workgroups.  Every kernel
// launched with grid_of or grid_rows strides over its items by the grid.
constexpr int64_t kMaxGridBlocks = (int64_t(1) << 22) - 1;
inline unsigned grid_of(int64_t n, int64_t per, int64_t cap = kMaxGridBlocks) {
    int64_t g = ceil_div(n, per);
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    if (g > kMaxGridBlocks) g = kMaxGridBlocks;
    return (unsigned)g;
}
// One workgroup per row, up to the grid limit (the kernel strides over rows).
inline unsigned grid_rows(int64_t rows) { return grid_of(rows, 1); }

}  // namespace bsmm
