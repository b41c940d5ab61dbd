// stacks.hip -- the stack builder: block-CSR indices -> stacks of block
// products grouped by shape.
//
// Paper, Sec. II (Traversal and Generation phases): the local multiply walks
// the A block rows and, for each, the B block columns, and collects the
// pairwise block products in batches.  Here every product (I,K,J) becomes
// an entry {A offset, k, B offset} of the "run" of its C block (I,J): all
// products that update one C block are contiguous, in ascending K, and a
// run has exactly one owner during execution, so no two workers ever write
// the same C block (the paper's race-free static ownership, here per block
// instead of per block row).  Runs are grouped by the shape class (m, n) of
// their C block and, inside a class, kept in C's CSR order, which is the
// paper's traversal order (A row blocks outer, B column blocks inner).
//
// Phases (all on the GPU, one workgroup per C block row where a row is the
// unit):
//   1. count    products per C block, through an LDS map column -> slot
//               (for C wider than the map, in windows of block columns);
//   2. classify counting sort of the C blocks that receive products by
//               class, stable in CSR order (per-tile histograms, a scan,
//               wave-level ranking with ballots);
//   3. offsets  scan of the product counts in run order;
//   4. fill     products written per row, K ascending.
// Phase 1 covers every C block row; phases 2-4 cover one panel of
// consecutive C block rows, so a product count beyond what the stack
// buffers may hold is built and executed panel by panel (the paper's
// batches, at the granularity of block rows).
#include <algorithm>

#include "dev_util.h"
#include "internal.h"

namespace bsmm {

namespace {

constexpr int kTile = 1024;         // C blocks per classification tile
constexpr int kMaxClasses = 1024;   // distinct (m, n) shapes

// A block range [pa0, pa1) of part `part` of P of A's block row `row`.
__device__ __forceinline__ void a_part(const int64_t *a_rp, int32_t row, int part, int P, int64_t *pa0,
                                       int64_t *pa1) {
    const int64_t b = a_rp[row], len = a_rp[row + 1] - b;
    *pa0 = b + len * part / P;
    *pa1 = b + len * (part + 1) / P;
}

// Workgroup (row, part): products per C block of the row from the part's
// share of A's block row (P > 1 splits long A rows of few-row products;
// the part counts go to pcount[c * P + part], else straight to c_count).
// A product whose C block is not in the pattern sets *missing, unless
// missing is null (a pattern from the symbolic screen leaves such blocks
// out on purpose; their products are skipped here and in the fill).
__global__ __launch_bounds__(256) void k_stack_count(int32_t nbr, int32_t nbc, const int64_t *a_rp,
                                                     const int32_t *a_ci, const int64_t *b_rp,
                                                     const int32_t *b_ci, const int64_t *c_rp,
                                                     const int32_t *c_ci, int64_t *c_count,
                                                     int32_t *c_row, int32_t *missing, int P,
                                                     int64_t *pcount) {
    extern __shared__ int32_t lds[];
    int32_t *map = lds;          // nbc entries: column -> slot in the C row, or -1
    int32_t *cnt = lds + nbc;    // row length entries
    const int part = blockIdx.y;
    const int nw = blockDim.x / kWave;
    for (int32_t row = blockIdx.x; row < nbr; row += gridDim.x) {
        const int64_t p0 = c_rp[row];
        const int32_t len = (int32_t)(c_rp[row + 1] - p0);
        for (int j = threadIdx.x; j < nbc; j += blockDim.x) map[j] = -1;
        __syncthreads();
        for (int s = threadIdx.x; s < len; s += blockDim.x) {
            map[c_ci[p0 + s]] = s;
            cnt[s] = 0;
        }
        __syncthreads();
        int64_t pa0, pa1;
        a_part(a_rp, row, part, P, &pa0, &pa1);
        for (int64_t pa = pa0 + wave_id(); pa < pa1; pa += nw) {
            const int32_t kb = a_ci[pa];
            for (int64_t q = b_rp[kb] + lane_id(); q < b_rp[kb + 1]; q += kWave) {
                const int32_t s = map[b_ci[q]];
                if (s >= 0) atomicAdd(&cnt[s], 1);
                else if (missing) *missing = 1;
            }
        }
        __syncthreads();
        for (int s = threadIdx.x; s < len; s += blockDim.x) {
            if (P == 1) c_count[p0 + s] = cnt[s];
            else pcount[(p0 + s) * P + part] = cnt[s];
            c_row[p0 + s] = row;  // every part writes the same value
        }
        __syncthreads();  // map and counts are reset for the next row
    }
}

// First position in [lo, hi) of the sorted column indices ci whose column
// is at least j (hi if none).
__device__ __forceinline__ int64_t lower_col(const int32_t *ci, int64_t lo, int64_t hi, int64_t j) {
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if ((int64_t)ci[mid] < j) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// For C wider than the LDS map: split[k * (nwin + 1) + w] = first entry of
// B block row k whose block column is at least w * kStackWin (w = 0..nwin).
__global__ __launch_bounds__(256) void k_window_splits(int32_t nbk, int nwin, const int64_t *b_rp,
                                                       const int32_t *b_ci, int64_t *split) {
    const int64_t total = (int64_t)nbk * (nwin + 1);
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int32_t k = (int32_t)(t / (nwin + 1));
        const int w = (int)(t - (int64_t)k * (nwin + 1));
        split[t] = lower_col(b_ci, b_rp[k], b_rp[k + 1], (int64_t)w * kStackWin);
    }
}

// The slots of C block row [p0, p1) in column window [w0, w0 + kStackWin),
// found by the first thread and shared through LDS (a barrier follows).
__device__ __forceinline__ void window_slots(const int32_t *c_ci, int64_t p0, int64_t p1, int32_t w0,
                                             int64_t *s_cs) {
    if (threadIdx.x == 0) {
        s_cs[0] = lower_col(c_ci, p0, p1, w0);
        s_cs[1] = lower_col(c_ci, s_cs[0], p1, (int64_t)w0 + kStackWin);
    }
}

// k_stack_count for C with more block columns than the LDS map holds: the
// row is counted window by window, each window's columns mapped in LDS and
// each B row read only over its share of the window (split).
__global__ __launch_bounds__(256) void k_stack_count_win(int32_t nbr, int nwin, const int64_t *a_rp,
                                                         const int32_t *a_ci, const int64_t *split,
                                                         const int32_t *b_ci, const int64_t *c_rp,
                                                         const int32_t *c_ci, int64_t *c_count,
                                                         int32_t *c_row, int32_t *missing, int P,
                                                         int64_t *pcount) {
    __shared__ int32_t map[kStackWin];
    __shared__ int32_t cnt[kStackWin];
    __shared__ int64_t s_cs[2];
    const int part = blockIdx.y;
    const int nw = blockDim.x / kWave;
    for (int32_t row = blockIdx.x; row < nbr; row += gridDim.x) {
        const int64_t p0 = c_rp[row], p1 = c_rp[row + 1];
        for (int64_t c = p0 + threadIdx.x; c < p1; c += blockDim.x) c_row[c] = row;  // every part alike
        int64_t pa0, pa1;
        a_part(a_rp, row, part, P, &pa0, &pa1);
        for (int w = 0; w < nwin; ++w) {
            const int32_t w0 = w * kStackWin;
            window_slots(c_ci, p0, p1, w0, s_cs);
            for (int j = threadIdx.x; j < kStackWin; j += blockDim.x) map[j] = -1;
            __syncthreads();
            const int64_t cs0 = s_cs[0];
            const int32_t ns = (int32_t)(s_cs[1] - cs0);
            for (int s = threadIdx.x; s < ns; s += blockDim.x) {
                map[c_ci[cs0 + s] - w0] = s;
                cnt[s] = 0;
            }
            __syncthreads();
            for (int64_t pa = pa0 + wave_id(); pa < pa1; pa += nw) {
                const int64_t *sp = split + (int64_t)a_ci[pa] * (nwin + 1) + w;
                const int64_t q1 = sp[1];
                for (int64_t q = sp[0] + lane_id(); q < q1; q += kWave) {
                    const int32_t s = map[b_ci[q] - w0];
                    if (s >= 0) atomicAdd(&cnt[s], 1);
                    else if (missing) *missing = 1;
                }
            }
            __syncthreads();
            for (int s = threadIdx.x; s < ns; s += blockDim.x) {
                if (P == 1) c_count[cs0 + s] = cnt[s];
                else pcount[(cs0 + s) * P + part] = cnt[s];
            }
            __syncthreads();  // map, counts and the window's slot range are reused
        }
    }
}

// P > 1: per C block, the part counts become the part's first position in
// the run (exclusive prefix in part order) and c_count their total.
__global__ __launch_bounds__(256) void k_part_offsets(int64_t nnzb, int P, int64_t *pcount,
                                                      int64_t *c_count) {
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nnzb;
         c += (int64_t)gridDim.x * blockDim.x) {
        int64_t run = 0;
        for (int p = 0; p < P; ++p) {
            const int64_t v = pcount[c * P + p];
            pcount[c * P + p] = run;
            run += v;
        }
        c_count[c] = run;
    }
}

__device__ __forceinline__ int class_of(int64_t c, const int32_t *c_row, const int32_t *c_ci,
                                        const int32_t *rsi, const int32_t *csi, int ncs) {
    return rsi[c_row[c]] * ncs + csi[c_ci[c]];
}

// One wave per tile of kTile C blocks: per-class counts of the blocks that
// receive products and per-class sums of their products, written
// class-major (hist[cl * ntiles + tile], hist_p likewise).
__global__ __launch_bounds__(256) void k_class_hist(int64_t c_base, int64_t nnzb, int64_t ntiles,
                                                    const int64_t *c_count, const int32_t *c_row,
                                                    const int32_t *c_ci, const int32_t *rsi,
                                                    const int32_t *csi, int ncs, int ncl,
                                                    int64_t *hist, int64_t *hist_p) {
    extern __shared__ int64_t lds_h[];
    unsigned long long *psum = (unsigned long long *)lds_h + wave_id() * ncl;
    int32_t *cnt = (int32_t *)(lds_h + (blockDim.x / kWave) * ncl) + wave_id() * ncl;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
    for (int64_t tile = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave_id(); tile < ntiles;
         tile += waves) {
        for (int cl = lane_id(); cl < ncl; cl += kWave) {
            cnt[cl] = 0;
            psum[cl] = 0;
        }
        wave_lds_sync();
        const int64_t end = c_base + std::min<int64_t>(nnzb, (tile + 1) * kTile);
        for (int64_t c = c_base + tile * kTile + lane_id(); c < end; c += kWave) {
            const int64_t n = c_count[c];
            if (n > 0) {
                const int cl = class_of(c, c_row, c_ci, rsi, csi, ncs);
                atomicAdd(&cnt[cl], 1);
                atomicAdd(&psum[cl], (unsigned long long)n);
            }
        }
        wave_lds_sync();
        for (int cl = lane_id(); cl < ncl; cl += kWave) {
            hist[(int64_t)cl * ntiles + tile] = cnt[cl];
            hist_p[(int64_t)cl * ntiles + tile] = (int64_t)psum[cl];
        }
        wave_lds_sync();
    }
}

// Stable scatter of the runs into class-major order.
__global__ __launch_bounds__(256) void k_class_scatter(
    int64_t c_base, int64_t nnzb, int64_t ntiles, const int64_t *c_count, const int32_t *c_row,
    const int32_t *c_ci, const int64_t *c_blk_off, const int32_t *rsi, const int32_t *csi,
    int ncs, int ncl, const int64_t *hoff, int64_t *run_cblk, int32_t *run_class,
    int64_t *run_coff, int64_t *run_cnt, int64_t *run_of_c) {
    extern __shared__ int64_t lds64[];
    int64_t *next = lds64 + wave_id() * ncl;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
    for (int64_t tile = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave_id(); tile < ntiles;
         tile += waves) {
        for (int cl = lane_id(); cl < ncl; cl += kWave) next[cl] = hoff[(int64_t)cl * ntiles + tile];
        wave_lds_sync();
        const int64_t end = c_base + std::min<int64_t>(nnzb, (tile + 1) * kTile);
        for (int64_t base = c_base + tile * kTile; base < end; base += kWave) {
            const int64_t c = base + lane_id();
            const bool inb = c < end;
            const int64_t cnt = inb ? c_count[c] : 0;
            const bool valid = cnt > 0;
            const int cl = valid ? class_of(c, c_row, c_ci, rsi, csi, ncs) : -1;
            if (inb && !valid) run_of_c[c] = -1;
            uint64_t pending = __ballot(valid);
            while (pending) {
                const int leader = __ffsll((unsigned long long)pending) - 1;
                const int cl_lead = __shfl(cl, leader, kWave);
                const uint64_t mask = __ballot(valid && cl == cl_lead);
                if (valid && cl == cl_lead) {
                    const int64_t r = next[cl_lead] + __popcll(mask & lanemask_lt());
                    run_cblk[r] = c;
                    run_class[r] = cl;
                    run_coff[r] = c_blk_off[c];
                    run_cnt[r] = cnt;
                    run_of_c[c] = r;
                }
                wave_lds_sync();
                if (lane_id() == leader) next[cl_lead] += __popcll(mask);
                wave_lds_sync();
                pending &= ~mask;
            }
        }
    }
}

__global__ void k_zero_i32(int32_t *p) { *p = 0; }

// out[r] = scan[rp[r]] for r = 0..nbr: products before each C block row.
__global__ void k_gather_rows(const int64_t *scan, const int64_t *rp, int32_t nbr, int64_t *out) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r <= nbr;
         r += (int64_t)gridDim.x * blockDim.x)
        out[r] = scan[rp[r]];
}

// out[0..ncl]: first run of every class; out[ncl+1..2 ncl+1]: its first product.
__global__ void k_gather_class_begin(const int64_t *hoff, const int64_t *hoff_p, int64_t ntiles,
                                     int ncl, int64_t *out) {
    for (int cl = threadIdx.x; cl <= ncl; cl += blockDim.x) {
        out[cl] = hoff[(int64_t)cl * ntiles];
        out[ncl + 1 + cl] = hoff_p[(int64_t)cl * ntiles];
    }
}

// k_stack_fill for C with more block columns than the LDS map holds: the
// row is filled window by window (as in k_stack_count_win); each window's
// slots keep their next write position in LDS.  Within one K a slot is hit
// at most once, and a barrier separates consecutive K, so the runs stay in
// K order with no atomics.
__global__ __launch_bounds__(256) void k_stack_fill_win(int32_t row0, int32_t row1, int P,
                                                        const int64_t *poff, int nwin,
                                                        const int64_t *a_rp, const int32_t *a_ci,
                                                        const int64_t *a_off, const int64_t *split,
                                                        const int32_t *b_ci, const int64_t *b_off,
                                                        const int32_t *kbs, const int64_t *c_rp,
                                                        const int32_t *c_ci, const int64_t *run_of_c,
                                                        const int64_t *run_ptr, ulonglong2 *prods) {
    __shared__ int32_t map[kStackWin];
    __shared__ int64_t next[kStackWin];
    __shared__ int64_t s_cs[2];
    const int part = blockIdx.y;
    for (int32_t row = row0 + (int32_t)blockIdx.x; row < row1; row += gridDim.x) {
        const int64_t p0 = c_rp[row], p1 = c_rp[row + 1];
        int64_t pa0, pa1;
        a_part(a_rp, row, part, P, &pa0, &pa1);
        for (int w = 0; w < nwin; ++w) {
            const int32_t w0 = w * kStackWin;
            window_slots(c_ci, p0, p1, w0, s_cs);
            for (int j = threadIdx.x; j < kStackWin; j += blockDim.x) map[j] = -1;
            __syncthreads();
            const int64_t cs0 = s_cs[0];
            const int32_t ns = (int32_t)(s_cs[1] - cs0);
            for (int s = threadIdx.x; s < ns; s += blockDim.x) {
                const int64_t c = cs0 + s;
                map[c_ci[c] - w0] = s;
                const int64_t first = P == 1 ? 0 : poff[c * P + part];
                const int64_t r = run_of_c[c];
                next[s] = r >= 0 ? run_ptr[r] + first : 0;  // r < 0: the slot receives no product
            }
            __syncthreads();
            if (ns > 0) {  // a window without slots receives no product
                for (int64_t pa = pa0; pa < pa1; ++pa) {
                    const int32_t kb = a_ci[pa];
                    const uint64_t aw = (uint64_t)a_off[pa] | ((uint64_t)kbs[kb] << 48);
                    const int64_t *sp = split + (int64_t)kb * (nwin + 1) + w;
                    const int64_t q1 = sp[1];
                    for (int64_t q = sp[0] + threadIdx.x; q < q1; q += blockDim.x) {
                        const int32_t s = map[b_ci[q] - w0];
                        if (s < 0) continue;
                        const int64_t pos = next[s];
                        next[s] = pos + 1;
                        prods[pos] = make_ulonglong2(aw, (uint64_t)b_off[q]);
                    }
                    __syncthreads();
                }
            }
            __syncthreads();  // map, positions and the window's slot range are reused
        }
    }
}

// Products of one C block row, K ascending inside every run.  Within one K
// every C slot is hit at most once, so the per-slot write positions need no
// atomics; a barrier separates consecutive K.  When the row has at most
// `cap` slots, each slot's next position in the stacks is kept in LDS as a
// 64-bit index, so a product costs no global gather; longer rows keep a
// 32-bit count per slot and gather the run's first position per product.
__global__ __launch_bounds__(256) void k_stack_fill(int32_t row0, int32_t row1, int P, const int64_t *poff,
                                                    int32_t nbc, int32_t cap, const int64_t *a_rp,
                                                    const int32_t *a_ci, const int64_t *a_off,
                                                    const int64_t *b_rp, const int32_t *b_ci,
                                                    const int64_t *b_off, const int32_t *kbs,
                                                    const int64_t *c_rp, const int32_t *c_ci,
                                                    const int64_t *run_of_c, const int64_t *run_ptr,
                                                    ulonglong2 *prods) {
    extern __shared__ int32_t lds[];
    int32_t *map = lds;
    const int32_t nbc_pad = (nbc + 1) & ~1;
    int64_t *next = reinterpret_cast<int64_t *>(lds + nbc_pad);  // rows of at most cap slots
    int32_t *cur = lds + nbc_pad;                                // longer rows
    const int part = blockIdx.y;
    for (int32_t row = row0 + (int32_t)blockIdx.x; row < row1; row += gridDim.x) {
        const int64_t p0 = c_rp[row];
        const int32_t len = (int32_t)(c_rp[row + 1] - p0);
        const bool in_lds = len <= cap;
        for (int j = threadIdx.x; j < nbc; j += blockDim.x) map[j] = -1;
        __syncthreads();
        for (int s = threadIdx.x; s < len; s += blockDim.x) {
            map[c_ci[p0 + s]] = s;
            const int64_t first = P == 1 ? 0 : poff[(p0 + s) * P + part];
            if (in_lds) {
                const int64_t r = run_of_c[p0 + s];
                next[s] = r >= 0 ? run_ptr[r] + first : 0;  // r < 0: the slot receives no product
            } else {
                cur[s] = (int32_t)first;
            }
        }
        __syncthreads();
        int64_t pa0, pa1;
        a_part(a_rp, row, part, P, &pa0, &pa1);
        for (int64_t pa = pa0; pa < pa1; ++pa) {
            const int32_t kb = a_ci[pa];
            const uint64_t aw = (uint64_t)a_off[pa] | ((uint64_t)kbs[kb] << 48);
            for (int64_t q = b_rp[kb] + threadIdx.x; q < b_rp[kb + 1]; q += blockDim.x) {
                const int32_t s = map[b_ci[q]];
                if (s < 0) continue;
                int64_t pos;
                if (in_lds) {
                    pos = next[s];
                    next[s] = pos + 1;
                } else {
                    pos = run_ptr[run_of_c[p0 + s]] + cur[s];
                    cur[s] += 1;
                }
                prods[pos] = make_ulonglong2(aw, (uint64_t)b_off[q]);
            }
            __syncthreads();
        }
        __syncthreads();  // map and positions are reset for the next row
    }
}

// Tile of C block (I, J): tiles of `tile` x `tile` blocks in row-major order.
__device__ __forceinline__ int64_t tile_key(int32_t I, int32_t J, int tile, int64_t ntj) {
    return (int64_t)(I / tile) * ntj + J / tile;
}

// Runs per tile (runs of eligible classes only).
__global__ __launch_bounds__(256) void k_sched_hist(int64_t nruns, const int64_t *run_cblk,
                                                    const int32_t *run_class, const char *elig,
                                                    const int32_t *c_row, const int32_t *c_ci,
                                                    int tile, int64_t ntj, int64_t *hist) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < nruns;
         r += (int64_t)gridDim.x * blockDim.x) {
        if (!elig[run_class[r]]) continue;
        const int64_t c = run_cblk[r];
        atomicAdd((unsigned long long *)&hist[tile_key(c_row[c], c_ci[c], tile, ntj)], 1ull);
    }
}

// Every eligible run into its tile's range of the schedule (the order of
// the runs inside a tile is not fixed; it does not change any result).
__global__ __launch_bounds__(256) void k_sched_scatter(int64_t nruns, const int64_t *run_cblk,
                                                       const int32_t *run_class, const char *elig,
                                                       const int32_t *c_row, const int32_t *c_ci,
                                                       const int32_t *rbs, const int32_t *cbs,
                                                       int tile, int64_t ntj, int64_t *cursor,
                                                       unsigned long long *sched) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < nruns;
         r += (int64_t)gridDim.x * blockDim.x) {
        if (!elig[run_class[r]]) continue;
        const int64_t c = run_cblk[r];
        const int32_t I = c_row[c], J = c_ci[c];
        const int64_t pos =
            (int64_t)atomicAdd((unsigned long long *)&cursor[tile_key(I, J, tile, ntj)], 1ull);
        sched[pos] = ((unsigned long long)r << 16) | ((unsigned long long)rbs[I] << 8) |
                     (unsigned long long)cbs[J];
    }
}

}  // namespace

int build_schedule(const bsmm_matrix_s *C, Stacks &st, const std::vector<char> &eligible, int tile,
                   hipStream_t s) {
    st.n_sched = 0;
    for (int cl = 0; cl < st.n_classes; ++cl)
        if (eligible[cl]) st.n_sched += st.class_begin[cl + 1] - st.class_begin[cl];
    if (st.n_sched == 0) return BSMM_OK;
    tile = std::max(tile, 1);
    const int64_t nti = ceil_div(C->nbr, tile), ntj = ceil_div(C->nbc, tile);
    const int64_t ntiles = nti * ntj;
    DevBuf elig, hist, off;
    BSMM_TRY(elig.reserve(eligible.size(), s));
    BSMM_TRY(hist.reserve(sizeof(int64_t) * (ntiles + 1), s));
    BSMM_TRY(off.reserve(sizeof(int64_t) * (ntiles + 1), s));
    BSMM_TRY(st.sched.reserve(sizeof(unsigned long long) * st.n_sched, s));
    BSMM_TRY(st.sched_next.reserve(sizeof(unsigned long long), s));
    BSMM_HIP(hipMemcpyAsync(elig.p, eligible.data(), eligible.size(), hipMemcpyHostToDevice, s));
    BSMM_TRY(fill_zero(hist.as<double>(), ntiles + 1, s));
    const unsigned grid = grid_of(st.n_runs, 256, 8192);
    hipLaunchKernelGGL(k_sched_hist, dim3(grid), dim3(256), 0, s, st.n_runs,
                       (const int64_t *)st.run_cblk.as<int64_t>(),
                       (const int32_t *)st.run_class.as<int32_t>(), (const char *)elig.as<char>(),
                       (const int32_t *)st.c_row.as<int32_t>(), C->d_col_ind(), tile, ntj,
                       hist.as<int64_t>());
    BSMM_TRY(launch_check("sched_hist"));
    BSMM_TRY(scan_exclusive_i64(hist.as<int64_t>(), off.as<int64_t>(), ntiles, s));
    hipLaunchKernelGGL(k_sched_scatter, dim3(grid), dim3(256), 0, s, st.n_runs,
                       (const int64_t *)st.run_cblk.as<int64_t>(),
                       (const int32_t *)st.run_class.as<int32_t>(), (const char *)elig.as<char>(),
                       (const int32_t *)st.c_row.as<int32_t>(), C->d_col_ind(), C->d_rbs(),
                       C->d_cbs(), tile, ntj, off.as<int64_t>(),
                       st.sched.as<unsigned long long>());
    return launch_check("sched_scatter");
}

// Distinct sizes of a size vector and the index of every entry.
static void size_classes(const std::vector<int32_t> &sizes, std::vector<int32_t> &distinct,
                         std::vector<int32_t> &index) {
    distinct = sizes;
    std::sort(distinct.begin(), distinct.end());
    distinct.erase(std::unique(distinct.begin(), distinct.end()), distinct.end());
    index.resize(sizes.size());
    for (size_t i = 0; i < sizes.size(); ++i)
        index[i] = (int32_t)(std::lower_bound(distinct.begin(), distinct.end(), sizes[i]) -
                             distinct.begin());
}

// Phase 1 for every C block row: products per C block, the size classes,
// and the check that C's pattern holds every product block.
int stack_count(const bsmm_matrix_s *A, const bsmm_matrix_s *B, const bsmm_matrix_s *C,
                Stacks &st, hipStream_t s) {
    const int32_t nbr = C->nbr, nbc = C->nbc;
    const int64_t nnzb = C->nnzb;
    std::vector<int32_t> rsi, csi;
    size_classes(C->rbs, st.row_sizes, rsi);
    size_classes(C->cbs, st.col_sizes, csi);
    st.nrs = (int32_t)st.row_sizes.size();
    st.ncs = (int32_t)st.col_sizes.size();
    const int ncl = st.nrs * st.ncs;
    st.n_classes = ncl;
    if (ncl > kMaxClasses) {
        set_error(BSMM_ENOTSUP, "more than %d distinct block shapes", kMaxClasses);
        return BSMM_ENOTSUP;
    }
    st.class_begin.assign(ncl + 1, 0);
    st.class_prod_begin.assign(ncl + 1, 0);
    st.class_active.assign(ncl, 0);
    st.run_len_hint.clear();
    st.n_runs = 0;
    if (nbr == 0 || nnzb == 0) return BSMM_OK;

    BSMM_TRY(st.d_rsi.reserve(sizeof(int32_t) * nbr, s));
    BSMM_TRY(st.d_csi.reserve(sizeof(int32_t) * nbc, s));
    BSMM_TRY(st.c_row.reserve(sizeof(int32_t) * nnzb, s));
    BSMM_TRY(st.c_count.reserve(sizeof(int64_t) * nnzb, s));
    BSMM_TRY(st.missing.reserve(sizeof(int32_t), s));
    // Few C block rows with long A rows (tall-and-skinny products, or a
    // product whose stacks are built in row panels of few rows each): split
    // every A row into P parts so that about 1024 workgroups count and fill.
    // A panel holds about nbr * cap / n_prod rows when the products exceed
    // the cap; the per-part counts stay within 2^28 entries.
    st.kparts = 1;
    const int64_t cap = options().stack_panel;
    int64_t rows = nbr;
    if (cap > 0 && st.n_prod > cap)
        rows = std::max<int64_t>(1, (int64_t)((double)nbr * (double)cap / (double)st.n_prod));
    if (rows < 256 && A->nnzb > 0) {
        const int64_t per_row = A->nnzb / nbr;
        int64_t P = std::min<int64_t>(ceil_div(1024, rows), std::max<int64_t>(1, per_row / 64));
        P = std::min<int64_t>(P, std::max<int64_t>(1, (int64_t(1) << 28) / nnzb));
        st.kparts = (int)P;
    }
    if (st.kparts > 1) BSMM_TRY(st.pcount.reserve(sizeof(int64_t) * nnzb * st.kparts, s));
    BSMM_HIP(hipMemcpyAsync(st.d_rsi.p, rsi.data(), sizeof(int32_t) * nbr, hipMemcpyHostToDevice, s));
    BSMM_HIP(hipMemcpyAsync(st.d_csi.p, csi.data(), sizeof(int32_t) * nbc, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(1), 0, s, st.missing.as<int32_t>());
    BSMM_TRY(launch_check("zero_i32"));
    st.nwin = 0;
    if (nbc > kMaxStackCols) {
        st.nwin = (int)ceil_div(nbc, kStackWin);
        const int64_t nsplit = (int64_t)B->nbr * (st.nwin + 1);
        BSMM_TRY(st.b_split.reserve(sizeof(int64_t) * nsplit, s));
        hipLaunchKernelGGL(k_window_splits, dim3(grid_of(nsplit, 256)), dim3(256), 0, s, B->nbr, st.nwin,
                           B->d_row_ptr(), B->d_col_ind(), st.b_split.as<int64_t>());
        BSMM_TRY(launch_check("window_splits"));
        hipLaunchKernelGGL(k_stack_count_win, dim3(grid_rows(nbr), st.kparts), dim3(256), 0, s, nbr, st.nwin,
                           A->d_row_ptr(), A->d_col_ind(), (const int64_t *)st.b_split.as<int64_t>(),
                           B->d_col_ind(), C->d_row_ptr(), C->d_col_ind(), st.c_count.as<int64_t>(),
                           st.c_row.as<int32_t>(), st.screened ? nullptr : st.missing.as<int32_t>(), st.kparts,
                           st.pcount.as<int64_t>());
    } else {
        const size_t map_lds = sizeof(int32_t) * 2 * (size_t)nbc;
        hipLaunchKernelGGL(k_stack_count, dim3(grid_rows(nbr), st.kparts), dim3(256), map_lds, s, nbr,
                           nbc, A->d_row_ptr(), A->d_col_ind(), B->d_row_ptr(), B->d_col_ind(),
                           C->d_row_ptr(), C->d_col_ind(), st.c_count.as<int64_t>(),
                           st.c_row.as<int32_t>(), st.screened ? nullptr : st.missing.as<int32_t>(), st.kparts,
                           st.pcount.as<int64_t>());
    }
    BSMM_TRY(launch_check("stack_count"));
    if (st.kparts == 1) return BSMM_OK;
    hipLaunchKernelGGL(k_part_offsets, dim3(grid_of(nnzb, 256)), dim3(256), 0, s, nnzb, st.kparts,
                       st.pcount.as<int64_t>(), st.c_count.as<int64_t>());
    return launch_check("part_offsets");
}

// The flag of k_stack_count, read after a host synchronisation.
static int check_missing(int32_t miss) {
    if (!miss) return BSMM_OK;
    set_error(BSMM_EINDEX, "C pattern does not contain every product block");
    return BSMM_EINDEX;
}

int stack_row_bounds(const bsmm_matrix_s *C, const Stacks &st, std::vector<int64_t> *prod_before,
                     std::vector<int64_t> *blk_before, hipStream_t s) {
    const int32_t nbr = C->nbr;
    prod_before->assign(nbr + 1, 0);
    blk_before->assign(nbr + 1, 0);
    if (nbr == 0 || C->nnzb == 0) return BSMM_OK;
    DevBuf scan, out;
    BSMM_TRY(scan.reserve(sizeof(int64_t) * (C->nnzb + 1), s));
    BSMM_TRY(out.reserve(sizeof(int64_t) * (nbr + 1), s));
    BSMM_TRY(scan_exclusive_i64(st.c_count.as<int64_t>(), scan.as<int64_t>(), C->nnzb, s));
    hipLaunchKernelGGL(k_gather_rows, dim3(grid_of(nbr + 1, 256)), dim3(256), 0, s,
                       (const int64_t *)scan.as<int64_t>(), C->d_row_ptr(), nbr, out.as<int64_t>());
    BSMM_TRY(launch_check("gather_rows"));
    BSMM_HIP(hipMemcpyAsync(prod_before->data(), out.p, sizeof(int64_t) * (nbr + 1),
                            hipMemcpyDeviceToHost, s));
    BSMM_HIP(hipMemcpyAsync(blk_before->data(), C->d_row_ptr(), sizeof(int64_t) * (nbr + 1),
                            hipMemcpyDeviceToHost, s));
    int32_t miss = 0;
    BSMM_HIP(hipMemcpyAsync(&miss, st.missing.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    BSMM_HIP(hipStreamSynchronize(s));
    return check_missing(miss);
}

namespace {
struct ClassHist {
    DevBuf hist, hoff, hist_p, hoff_p, cb;
    int64_t ntiles = 0;
};

// Per-class histograms of the C blocks [c0, c0 + nblk) that receive products
// (blocks and products, per tile), their scans, and the class boundaries
// gathered into h.cb: first run of every class, then its first product
// (2 (ncl + 1) values).  Everything is queued on s.
int class_offsets(const bsmm_matrix_s *C, const Stacks &st, int64_t c0, int64_t nblk, ClassHist &h,
                  hipStream_t s) {
    const int ncl = st.n_classes;
    h.ntiles = ceil_div(nblk, kTile);
    const int64_t n = ncl * h.ntiles + 1;
    BSMM_TRY(h.hist.reserve(sizeof(int64_t) * n, s));
    BSMM_TRY(h.hoff.reserve(sizeof(int64_t) * n, s));
    BSMM_TRY(h.hist_p.reserve(sizeof(int64_t) * n, s));
    BSMM_TRY(h.hoff_p.reserve(sizeof(int64_t) * n, s));
    BSMM_TRY(h.cb.reserve(sizeof(int64_t) * 2 * (ncl + 1), s));
    hipLaunchKernelGGL(k_class_hist, dim3(grid_of(h.ntiles, 4)), dim3(256),
                       (sizeof(int32_t) + sizeof(int64_t)) * 4 * ncl, s, c0, nblk, h.ntiles,
                       (const int64_t *)st.c_count.as<int64_t>(),
                       (const int32_t *)st.c_row.as<int32_t>(), C->d_col_ind(),
                       (const int32_t *)st.d_rsi.as<int32_t>(),
                       (const int32_t *)st.d_csi.as<int32_t>(), st.ncs, ncl, h.hist.as<int64_t>(),
                       h.hist_p.as<int64_t>());
    BSMM_TRY(launch_check("class_hist"));
    BSMM_TRY(scan_exclusive_i64(h.hist.as<int64_t>(), h.hoff.as<int64_t>(), ncl * h.ntiles, s));
    BSMM_TRY(scan_exclusive_i64(h.hist_p.as<int64_t>(), h.hoff_p.as<int64_t>(), ncl * h.ntiles, s));
    hipLaunchKernelGGL(k_gather_class_begin, dim3(1), dim3(256), 0, s,
                       (const int64_t *)h.hoff.as<int64_t>(), (const int64_t *)h.hoff_p.as<int64_t>(),
                       h.ntiles, ncl, h.cb.as<int64_t>());
    return launch_check("gather_class_begin");
}
}  // namespace

int stack_class_run_lengths(const bsmm_matrix_s *C, const Stacks &st, std::vector<int> *out,
                            hipStream_t s) {
    const int ncl = st.n_classes;
    out->assign(ncl, 1);
    if (C->nnzb == 0 || ncl == 0) return BSMM_OK;
    ClassHist h;
    BSMM_TRY(class_offsets(C, st, 0, C->nnzb, h, s));
    std::vector<int64_t> both(2 * (ncl + 1));
    BSMM_HIP(hipMemcpyAsync(both.data(), h.cb.p, sizeof(int64_t) * 2 * (ncl + 1),
                            hipMemcpyDeviceToHost, s));
    BSMM_HIP(hipStreamSynchronize(s));
    for (int cl = 0; cl < ncl; ++cl) {
        const int64_t runs = both[cl + 1] - both[cl];
        const int64_t prods = both[ncl + 2 + cl] - both[ncl + 1 + cl];
        if (runs > 0) (*out)[cl] = (int)std::max<int64_t>(1, (prods + runs / 2) / runs);
    }
    return BSMM_OK;
}

int stack_rows(const bsmm_matrix_s *A, const bsmm_matrix_s *B, const bsmm_matrix_s *C,
               Stacks &st, int32_t r0, int32_t r1, int64_t c0, int64_t c1, int64_t nprod,
               hipStream_t s) {
    const int32_t nbc = C->nbc;
    const int ncl = st.n_classes;
    const int64_t nblk = c1 - c0;
    st.class_begin.assign(ncl + 1, 0);
    st.class_prod_begin.assign(ncl + 1, 0);
    st.n_runs = 0;
    st.n_prod = 0;
    if (r1 <= r0 || nblk <= 0) return BSMM_OK;

    DevBuf run_cnt;
    ClassHist h;
    BSMM_TRY(run_cnt.reserve(sizeof(int64_t) * (nblk + 1), s));
    BSMM_TRY(st.run_of_c.reserve(sizeof(int64_t) * C->nnzb, s));
    BSMM_TRY(st.run_cblk.reserve(sizeof(int64_t) * nblk, s));
    BSMM_TRY(st.run_coff.reserve(sizeof(int64_t) * nblk, s));
    BSMM_TRY(st.run_class.reserve(sizeof(int32_t) * nblk, s));
    BSMM_TRY(st.run_ptr.reserve(sizeof(int64_t) * (nblk + 1), s));
    BSMM_TRY(class_offsets(C, st, c0, nblk, h, s));
    hipLaunchKernelGGL(k_class_scatter, dim3(grid_of(h.ntiles, 4)), dim3(256), sizeof(int64_t) * 4 * ncl,
                       s, c0, nblk, h.ntiles, (const int64_t *)st.c_count.as<int64_t>(),
                       (const int32_t *)st.c_row.as<int32_t>(), C->d_col_ind(), C->d_blk_off(),
                       (const int32_t *)st.d_rsi.as<int32_t>(),
                       (const int32_t *)st.d_csi.as<int32_t>(), st.ncs, ncl,
                       (const int64_t *)h.hoff.as<int64_t>(), st.run_cblk.as<int64_t>(),
                       st.run_class.as<int32_t>(), st.run_coff.as<int64_t>(),
                       run_cnt.as<int64_t>(), st.run_of_c.as<int64_t>());
    BSMM_TRY(launch_check("class_scatter"));
    int32_t miss = 0;
    std::vector<int64_t> both(2 * (ncl + 1));
    BSMM_HIP(hipMemcpyAsync(both.data(), h.cb.p, sizeof(int64_t) * 2 * (ncl + 1),
                            hipMemcpyDeviceToHost, s));
    BSMM_HIP(hipMemcpyAsync(&miss, st.missing.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    BSMM_HIP(hipStreamSynchronize(s));
    BSMM_TRY(check_missing(miss));
    st.class_begin.assign(both.begin(), both.begin() + ncl + 1);
    st.class_prod_begin.assign(both.begin() + ncl + 1, both.end());
    st.n_runs = st.class_begin[ncl];
    st.n_prod = st.class_prod_begin[ncl];  // below nprod when the screen left blocks out
    for (int cl = 0; cl < ncl; ++cl)
        if (st.class_begin[cl + 1] > st.class_begin[cl]) st.class_active[cl] = 1;
    BSMM_TRY(scan_exclusive_i64(run_cnt.as<int64_t>(), st.run_ptr.as<int64_t>(), st.n_runs, s));
    if (st.n_prod > 0 && nbc > kMaxStackCols) {
        BSMM_TRY(st.prods.reserve(sizeof(ulonglong2) * st.n_prod, s));
        hipLaunchKernelGGL(k_stack_fill_win, dim3(grid_rows(r1 - r0), st.kparts), dim3(256), 0, s, r0, r1,
                           st.kparts, (const int64_t *)st.pcount.as<int64_t>(), st.nwin, A->d_row_ptr(),
                           A->d_col_ind(), A->d_blk_off(), (const int64_t *)st.b_split.as<int64_t>(),
                           B->d_col_ind(), B->d_blk_off(), B->d_rbs(), C->d_row_ptr(), C->d_col_ind(),
                           (const int64_t *)st.run_of_c.as<int64_t>(),
                           (const int64_t *)st.run_ptr.as<int64_t>(), st.prods.as<ulonglong2>());
        BSMM_TRY(launch_check("stack_fill_win"));
    } else if (st.n_prod > 0) {
        BSMM_TRY(st.prods.reserve(sizeof(ulonglong2) * st.n_prod, s));
        // LDS: the column map, then per slot a 64-bit next position (rows of
        // at most cap slots) or a 32-bit count; at most 64 KB.
        const int64_t nbc_pad = (nbc + 1) & ~1;
        const int32_t cap = (int32_t)std::min<int64_t>(nbc, (65536 - 4 * nbc_pad) / 8);
        const size_t fill_lds = 4 * nbc_pad + std::max<int64_t>(4 * (int64_t)nbc, 8 * (int64_t)cap);
        hipLaunchKernelGGL(k_stack_fill, dim3(grid_rows(r1 - r0), st.kparts), dim3(256), fill_lds, s, r0,
                           r1, st.kparts, (const int64_t *)st.pcount.as<int64_t>(), nbc, cap,
                           A->d_row_ptr(), A->d_col_ind(), A->d_blk_off(), B->d_row_ptr(),
                           B->d_col_ind(), B->d_blk_off(), B->d_rbs(), C->d_row_ptr(),
                           C->d_col_ind(), (const int64_t *)st.run_of_c.as<int64_t>(),
                           (const int64_t *)st.run_ptr.as<int64_t>(), st.prods.as<ulonglong2>());
        BSMM_TRY(launch_check("stack_fill"));
    }
    return BSMM_OK;
}

// st.n_prod must hold the product count of the symbolic phase on entry.
int build_stacks(const bsmm_matrix_s *A, const bsmm_matrix_s *B, const bsmm_matrix_s *C,
                 Stacks &st, hipStream_t s) {
    const int64_t nprod = st.n_prod;
    BSMM_TRY(stack_count(A, B, C, st, s));
    return stack_rows(A, B, C, st, 0, C->nbr, 0, C->nnzb, nprod, s);
}

}  // namespace bsmm
