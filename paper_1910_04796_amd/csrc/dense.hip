// dense.hip -- densification path: merge blocks into panels, one MFMA GEMM
// (FP64, or FP32 for single-precision matrices), split the result back into
// the blocks of C.
//
// Paper, Sec. III: when the inputs are dense, all blocks handled by a worker
// are coalesced into one large block by copying them into new buffers, the
// product becomes a single GEMM, and C is undensified at the end.  With one
// rank and one panel (Eqs. (1)-(2) with P~ = 1, t = 1) the panels are the
// whole matrices: A -> Ap (M x K), B -> Bp (K x N), both column-major and
// zero-padded to the GEMM tile.  The undensify step is fused into the GEMM
// epilogue, which writes C = beta*C + alpha*(Ap Bp) straight into C's
// blocks through per-row and per-column (block, offset) maps.
//
// GEMM: 128 x 128 output tile per 256-thread workgroup, k step 16 (or 32),
// LDS double buffered; each wave owns a 64 x 64 sub-tile as 4 x 4 MFMA tiles of
// v_mfma_f64_16x16x4 (FP64 in, FP64 accumulate).  Workgroup ids are remapped
// so that the tiles dispatched to one XCD form a contiguous band of
// 8 tile-rows (shared A panels stay in that XCD's L2).  When the output
// has too few tiles to fill the GPU (M = N = 1408 with K in the millions:
// 121 tiles for 256 CUs), k is split across workgroups; the partial tiles
// are summed in a fixed order by a second kernel that applies the epilogue.
#include <algorithm>
#include <atomic>

#include "dev_util.h"
#include "internal.h"
#include "mfma_util.h"

namespace bsmm {

namespace {

template <class T> struct Vec2;
template <> struct Vec2<double> { typedef double __attribute__((ext_vector_type(2))) t; };
template <> struct Vec2<float> { typedef float __attribute__((ext_vector_type(2))) t; };

constexpr int BM = 128, BN = 128;
constexpr int kGroupM = 8;

// Merge of blocks of 64 elements or more: one wave per block (block row
// found by binary search in the row pointer), copying the column-major
// block into the column-major panel (ld = panel rows); consecutive lanes
// write consecutive rows of a column.
template <class T>
__global__ __launch_bounds__(256) void k_merge_block(int32_t nbr, int64_t nnzb, const int32_t *rbs,
                                                     const int32_t *cbs, const int64_t *row_off,
                                                     const int64_t *col_off, const int64_t *rp,
                                                     const int32_t *ci, const int64_t *blk_off,
                                                     const T *data, T *panel, int64_t ld) {
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
    for (int64_t p = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave_id(); p < nnzb; p += waves) {
        int32_t lo = 0, hi = nbr;  // row = last lo with rp[lo] <= p
        while (hi - lo > 1) {
            const int32_t mid = (lo + hi) >> 1;
            if (rp[mid] <= p) lo = mid;
            else hi = mid;
        }
        const int32_t row = lo;
        const int m = rbs[row];
        const int64_t r0 = row_off[row];
        const int32_t j = ci[p];
        const int n = cbs[j];
        const int64_t c0 = col_off[j];
        const T *src = data + blk_off[p];
        const int64_t len = (int64_t)m * n;
        if (len < (1 << 20) && m < 4096) {
            const float rcp = 1.0f / (float)m;
            for (int e = lane_id(); e < len; e += kWave) {
                int ii;
                const int jj = divmod_small(e, m, rcp, &ii);
                panel[(c0 + jj) * ld + r0 + ii] = src[e];
            }
        } else {
            for (int64_t e = lane_id(); e < len; e += kWave)
                panel[(c0 + e / m) * ld + r0 + e % m] = src[e];
        }
    }
}

// Merge of blocks of fewer than 64 elements, where one wave per block would
// leave most lanes idle: one wave per chunk of 64 consecutive blocks.  Lane
// l takes block p0 + l (its block row by binary search in the row pointer,
// all lanes at once), and a running sum of the block lengths over the wave
// lays the chunk's elements out in one flat range; the wave walks that
// range 64 elements at a time, each lane stepping forward through the 64
// running sums in LDS to its block, and copies from the column-major block
// into the column-major panel (ld = panel rows).
constexpr int kMergeWaves = 4;
template <class T>
__global__ __launch_bounds__(kMergeWaves * kWave) void k_merge_chunk(
    int32_t nbr, int64_t nnzb, const int32_t *rbs, const int32_t *cbs, const int64_t *row_off,
    const int64_t *col_off, const int64_t *rp, const int32_t *ci, const int64_t *blk_off, const T *data,
    T *panel, int64_t ld) {
    __shared__ int64_t s_end[kMergeWaves][kWave], s_src[kMergeWaves][kWave], s_dst[kMergeWaves][kWave];
    __shared__ int32_t s_m[kMergeWaves][kWave];
    const int w = wave_id(), l = lane_id();
    const int64_t step = (int64_t)gridDim.x * kMergeWaves * kWave;
    for (int64_t p0 = ((int64_t)blockIdx.x * kMergeWaves + w) * kWave; p0 < nnzb; p0 += step) {
        const int64_t p = p0 + l;
        int64_t len = 0, src = 0, dst = 0;
        int m = 1;
        if (p < nnzb) {
            int32_t lo = 0, hi = nbr;  // row = last lo with rp[lo] <= p
            while (hi - lo > 1) {
                const int32_t mid = (lo + hi) >> 1;
                if (rp[mid] <= p) lo = mid;
                else hi = mid;
            }
            m = rbs[lo];
            const int32_t j = ci[p];
            len = (int64_t)m * cbs[j];
            src = blk_off[p];
            dst = col_off[j] * ld + row_off[lo];
        }
        int64_t end = len;  // inclusive running sum over the wave
        for (int d = 1; d < kWave; d <<= 1) {
            const int64_t v = __shfl_up(end, d, kWave);
            if (l >= d) end += v;
        }
        s_end[w][l] = end;
        s_src[w][l] = src;
        s_dst[w][l] = dst;
        s_m[w][l] = m;
        wave_lds_sync();
        const int64_t total = __shfl(end, kWave - 1, kWave);
        int b = 0;  // first block whose running sum exceeds e (e only grows)
        for (int64_t e = l; e < total; e += kWave) {
            while (s_end[w][b] <= e) ++b;
            const int64_t off = e - (b ? s_end[w][b - 1] : 0);
            const int mb = s_m[w][b];
            int64_t jj, ii;
            if (off < (1 << 20) && mb < 4096) {
                int r;
                jj = divmod_small((int)off, mb, 1.0f / (float)mb, &r);
                ii = r;
            } else {
                jj = off / mb;
                ii = off - jj * mb;
            }
            panel[s_dst[w][b] + jj * ld + ii] = data[s_src[w][b] + off];
        }
        wave_lds_sync();  // every lane has read the chunk before it is replaced
    }
}

struct GemmArgs {
    const void *Ap;     // M_pad x K_pad, column-major, ld = lda (element type of the matrices)
    const void *Bp;     // K_pad x N_pad, column-major, ld = ldb
    int64_t lda, ldb;
    int tiles_m, tiles_n, ktiles;
    int64_t M, N;       // true sizes (rows/cols of C)
    double alpha, beta;
    void *C;            // C block data
    const int64_t *c_blk_off;
    const int32_t *c_map;   // nbr*nbc block index map, or null when C is full
    int32_t c_nbc;
    const int32_t *c_rbs;
    const int2 *rmap, *cmap;
    // Split k (few output tiles): workgroup (tile, split) sums k tiles
    // [split * kt_per, (split + 1) * kt_per) into part[split] (row-major
    // M_pad x N_pad, unscaled); k_splitk_reduce applies the epilogue.
    int splits, kt_per;
    void *part;
};

// Global -> register loads of one k step of KB: A tile (128 rows x KB k) as
// KB * 64 double2 along the rows, B tile (KB k x 128 cols) along k.
template <class T, int KB>
__device__ __forceinline__ void gemm_gload(typename Vec2<T>::t (&ra)[KB / 4],
                                           typename Vec2<T>::t (&rb)[KB / 4], const T *Ablk,
                                           const T *Bblk, int64_t lda, int64_t ldb, int kt, int tid) {
    typedef typename Vec2<T>::t V2;
    const int64_t k0 = (int64_t)kt * KB;
#pragma unroll
    for (int i = 0; i < KB / 4; ++i) {
        const int e = tid + 256 * i;
        const int kk = e >> 6, r2 = e & 63;
        ra[i] = *reinterpret_cast<const V2 *>(Ablk + (k0 + kk) * lda + 2 * r2);
    }
#pragma unroll
    for (int i = 0; i < KB / 4; ++i) {
        const int e = tid + 256 * i;
        const int col = e / (KB / 2), k2 = e % (KB / 2);
        rb[i] = *reinterpret_cast<const V2 *>(Bblk + (int64_t)col * ldb + k0 + 2 * k2);
    }
}

// Register -> LDS stores: As[k][m]; Bs[n][k ^ (n & 15)] (XOR swizzle keeps
// the 16 lanes that read one k of 16 consecutive columns on distinct banks).
template <class T, int KB>
__device__ __forceinline__ void gemm_lstore(const typename Vec2<T>::t (&ra)[KB / 4],
                                            const typename Vec2<T>::t (&rb)[KB / 4], T *As, T *Bs,
                                            int tid) {
    typedef typename Vec2<T>::t V2;
#pragma unroll
    for (int i = 0; i < KB / 4; ++i) {
        const int e = tid + 256 * i;
        const int kk = e >> 6, r2 = e & 63;
        *reinterpret_cast<V2 *>(&As[kk * BM + 2 * r2]) = ra[i];
    }
#pragma unroll
    for (int i = 0; i < KB / 4; ++i) {
        const int e = tid + 256 * i;
        const int col = e / (KB / 2), k2 = e % (KB / 2);
        const int sw = col & 15;
        const int base = (2 * k2) ^ (sw & ~1);
        const V2 v = (sw & 1) ? rb[i].yx : rb[i];
        *reinterpret_cast<V2 *>(&Bs[col * KB + base]) = v;
    }
}

// KB = 16: 64 KB of LDS, two workgroups per CU; KB = 32: 128 KB, one
// workgroup per CU with twice the prefetch distance and half the barriers.
template <class T, int KB, int MINB, bool SPLIT>
__global__ __launch_bounds__(256, MINB) void k_dgemm_mfma(GemmArgs g) {
    __shared__ T As[2][KB * BM];  // [k][m]
    __shared__ T Bs[2][BN * KB];  // [n][k ^ swizzle(n)]

    // XCD-aware remap, then grouped row-major order inside the XCD's band
    // (split k: consecutive logical ids walk the tiles of one split).
    const int nwg = gridDim.x;
    int logical = blockIdx.x;
    if ((nwg & 7) == 0) logical = (blockIdx.x & 7) * (nwg >> 3) + (blockIdx.x >> 3);
    int split = 0, kt0 = 0, kt1 = g.ktiles;
    if (SPLIT) {
        const int tiles = g.tiles_m * g.tiles_n;
        split = logical / tiles;
        logical -= split * tiles;
        kt0 = split * g.kt_per;
        kt1 = min(g.ktiles, kt0 + g.kt_per);
    }
    const int per_group = kGroupM * g.tiles_n;
    const int group = logical / per_group;
    const int first_m = group * kGroupM;
    const int gsz = min(g.tiles_m - first_m, kGroupM);
    const int in_group = logical - group * per_group;
    const int tm = first_m + in_group % gsz;
    const int tn = in_group / gsz;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = tid >> 6;
    const int wm = w & 1, wn = w >> 1;
    const int l16 = lane & 15, lk = lane >> 4;

    const T *Ablk = static_cast<const T *>(g.Ap) + (int64_t)tm * BM;
    const T *Bblk = static_cast<const T *>(g.Bp) + (int64_t)tn * BN * g.ldb;

    typename Vec2<T>::t ra[KB / 4], rb[KB / 4];
    typename Mfma<T>::acc_t acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = Mfma<T>::zero();

    gemm_gload<T, KB>(ra, rb, Ablk, Bblk, g.lda, g.ldb, kt0, tid);
    gemm_lstore<T, KB>(ra, rb, As[0], Bs[0], tid);
    __syncthreads();
    for (int kt = kt0; kt < kt1; ++kt) {
        const int cur = (kt - kt0) & 1;
        if (kt + 1 < kt1) gemm_gload<T, KB>(ra, rb, Ablk, Bblk, g.lda, g.ldb, kt + 1, tid);
#pragma unroll
        for (int ks = 0; ks < KB / 4; ++ks) {
            const int k = ks * 4 + lk;
            T a[4], b[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) a[t] = As[cur][k * BM + wm * 64 + t * 16 + l16];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int col = wn * 64 + t * 16 + l16;
                b[t] = Bs[cur][col * KB + (k ^ (col & 15))];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = Mfma<T>::step(a[i], b[j], acc[i][j]);
        }
        if (kt + 1 < kt1) gemm_lstore<T, KB>(ra, rb, As[cur ^ 1], Bs[cur ^ 1], tid);
        __syncthreads();
    }

    // Epilogue: element e of lane l holds row Mfma<T>::row(e, l / 16),
    // column l % 16 of its 16 x 16 tile.
    const T alpha = (T)g.alpha, beta = (T)g.beta;
    if (SPLIT) {
        // Partial sums, row-major: 16 lanes store 16 consecutive columns.
        const int64_t ldp = (int64_t)g.tiles_n * BN;
        T *P = static_cast<T *>(g.part) + (int64_t)split * g.tiles_m * BM * ldp;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int64_t col = (int64_t)tn * BN + wn * 64 + j * 16 + l16;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int64_t row = (int64_t)tm * BM + wm * 64 + i * 16 + Mfma<T>::row(e, lk);
                    P[row * ldp + col] = acc[i][j][e];
                }
            }
        return;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t col = (int64_t)tn * BN + wn * 64 + j * 16 + l16;
            if (col >= g.N) continue;
            const int2 cm = g.cmap[col];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t row = (int64_t)tm * BM + wm * 64 + i * 16 + Mfma<T>::row(e, lk);
                if (row >= g.M) continue;
                const int2 rm = g.rmap[row];
                const int64_t bidx = (int64_t)rm.x * g.c_nbc + cm.x;
                const int32_t blk = g.c_map ? g.c_map[bidx] : (int32_t)bidx;
                if (blk < 0) continue;
                T *dst = static_cast<T *>(g.C) + g.c_blk_off[blk] + rm.y + (int64_t)g.c_rbs[rm.x] * cm.y;
                const T prod = alpha * acc[i][j][e];
                *dst = (beta == T(0)) ? prod : fma(beta, *dst, prod);
            }
        }
    }
}

// Split-k epilogue: C(row, col) = beta C + alpha * (sum of the partials in
// split order), written into C's blocks like the GEMM epilogue; one thread
// per element, consecutive threads on consecutive columns.
template <class T>
__global__ __launch_bounds__(256) void k_splitk_reduce(GemmArgs g) {
    const T alpha = (T)g.alpha, beta = (T)g.beta;
    const int64_t ldp = (int64_t)g.tiles_n * BN;
    const int64_t plane = (int64_t)g.tiles_m * BM * ldp;
    const int64_t n = g.M * g.N;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t row = t / g.N, col = t - row * g.N;
        const T *p = static_cast<const T *>(g.part) + row * ldp + col;
        T v = p[0];
        for (int sp = 1; sp < g.splits; ++sp) v += p[sp * plane];
        const int2 rm = g.rmap[row], cm = g.cmap[col];
        const int64_t bidx = (int64_t)rm.x * g.c_nbc + cm.x;
        const int32_t blk = g.c_map ? g.c_map[bidx] : (int32_t)bidx;
        if (blk < 0) continue;
        T *dst = static_cast<T *>(g.C) + g.c_blk_off[blk] + rm.y + (int64_t)g.c_rbs[rm.x] * cm.y;
        const T prod = alpha * v;
        *dst = (beta == T(0)) ? prod : fma(beta, *dst, prod);
    }
}

// c_map[I*nbc + J] = CSR position of block (I,J) in C, or -1.
__global__ __launch_bounds__(256) void k_block_map(int32_t nbr, int32_t nbc, const int64_t *rp,
                                                   const int32_t *ci, int32_t *map) {
    for (int32_t row = blockIdx.x; row < nbr; row += gridDim.x) {
        for (int j = threadIdx.x; j < nbc; j += blockDim.x) map[(int64_t)row * nbc + j] = -1;
        __syncthreads();
        for (int64_t p = rp[row] + threadIdx.x; p < rp[row + 1]; p += blockDim.x)
            map[(int64_t)row * nbc + ci[p]] = (int32_t)p;
        __syncthreads();
    }
}

}  // namespace

// Compute units of the current device (cached per device).
int cu_count() {
    static std::atomic<int> cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
        (void)hipGetLastError();
        return 256;
    }
    int n = cache[dev].load(std::memory_order_relaxed);
    if (n > 0) return n;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) {
        (void)hipGetLastError();
        return 256;
    }
    cache[dev].store(n, std::memory_order_relaxed);
    return n;
}


namespace {

// Merges M's blocks into a column-major panel (ld = panel rows): blocks of
// fewer than 64 elements in chunks of 64 blocks per wave, larger blocks one
// wave per block.
template <class T>
int merge_panel(const bsmm_matrix_s *M, T *panel, int64_t ld, const char *what, hipStream_t s) {
    if ((int64_t)M->max_rbs * M->max_cbs < kWave)
        hipLaunchKernelGGL(k_merge_chunk<T>, dim3(grid_of(M->nnzb, kMergeWaves * kWave)),
                           dim3(kMergeWaves * kWave), 0, s, M->nbr, M->nnzb, M->d_rbs(), M->d_cbs(),
                           M->d_row_off(), M->d_col_off(), M->d_row_ptr(), M->d_col_ind(), M->d_blk_off(),
                           (const T *)M->d_raw(), panel, ld);
    else
        hipLaunchKernelGGL(k_merge_block<T>, dim3(grid_of(M->nnzb, 4)), dim3(256), 0, s, M->nbr, M->nnzb,
                           M->d_rbs(), M->d_cbs(), M->d_row_off(), M->d_col_off(), M->d_row_ptr(),
                           M->d_col_ind(), M->d_blk_off(), (const T *)M->d_raw(), panel, ld);
    return launch_check(what);
}

template <class T>
int dense_multiply_t(const bsmm_matrix_s *A, const bsmm_matrix_s *B, bsmm_matrix_s *C,
                     double alpha, double beta, hipStream_t s) {
    const int64_t M = A->rows(), K = A->cols(), N = B->cols();
    if (M == 0 || N == 0 || C->nnzb == 0) return BSMM_OK;
    if (alpha == 0.0 || K == 0) return scale_blocks(C, nullptr, beta, s);
    const int KB = options().dense_kb == 32 ? 32 : 16;
    const int64_t Mp = ceil_div(M, BM) * BM, Np = ceil_div(N, BN) * BN, Kp = ceil_div(K, KB) * KB;
    const int64_t tiles = (Mp / BM) * (Np / BN);
    if (tiles > kMaxGridBlocks || Mp * Kp > (int64_t(1) << 47) || Kp * Np > (int64_t(1) << 47)) {
        set_error(BSMM_ERANGE, "dense panels too large");
        return BSMM_ERANGE;
    }
    DevBuf ap, bp, cmap;
    BSMM_TRY(ap.reserve(sizeof(T) * Mp * Kp, s));
    BSMM_TRY(bp.reserve(sizeof(T) * Kp * Np, s));
    // Panels need zeros where blocks are absent and in the padding.
    if (!A->full() || Mp != M || Kp != K) BSMM_TRY(fill_zero_bytes(ap.p, sizeof(T) * Mp * Kp, s));
    if (!B->full() || Kp != K || Np != N) BSMM_TRY(fill_zero_bytes(bp.p, sizeof(T) * Kp * Np, s));
    if (A->nnzb > 0) BSMM_TRY(merge_panel<T>(A, ap.as<T>(), Mp, "merge_A", s));
    if (B->nnzb > 0) BSMM_TRY(merge_panel<T>(B, bp.as<T>(), Kp, "merge_B", s));
    const int32_t *d_cmap = nullptr;
    if (!C->full()) {
        const int64_t cells = (int64_t)C->nbr * C->nbc;
        if (cells > (int64_t(1) << 30)) {
            set_error(BSMM_ENOTSUP, "dense path on a sparse C with more than 2^30 block cells");
            return BSMM_ENOTSUP;
        }
        BSMM_TRY(cmap.reserve(sizeof(int32_t) * cells, s));
        hipLaunchKernelGGL(k_block_map, dim3(grid_rows(C->nbr)), dim3(256), 0, s, C->nbr, C->nbc,
                           C->d_row_ptr(), C->d_col_ind(), cmap.as<int32_t>());
        BSMM_TRY(launch_check("block_map"));
        d_cmap = cmap.as<int32_t>();
    }
    GemmArgs g{};
    g.Ap = ap.p;
    g.Bp = bp.p;
    g.lda = Mp;
    g.ldb = Kp;
    g.tiles_m = (int)(Mp / BM);
    g.tiles_n = (int)(Np / BN);
    g.ktiles = (int)(Kp / KB);
    g.M = M;
    g.N = N;
    g.alpha = alpha;
    g.beta = beta;
    g.C = C->d_raw();
    g.c_blk_off = C->d_blk_off();
    g.c_map = d_cmap;
    g.c_nbc = C->nbc;
    g.c_rbs = C->d_rbs();
    g.rmap = C->d_row_map();
    g.cmap = C->d_col_map();
    // Split k when the output tiles cannot fill the GPU (tall-and-skinny
    // products): about two rounds of resident workgroups, each split at
    // least 16 k tiles deep, partials at most 2 GiB.
    const int64_t slots = (int64_t)cu_count() * (KB == 32 ? 1 : 2);
    int64_t splits = 1;
    if (tiles < slots) {
        splits = std::min<int64_t>(ceil_div(2 * slots, tiles), g.ktiles / 16);
        splits = std::min<int64_t>(splits, (int64_t(1) << 31) / (int64_t)(sizeof(T) * Mp * Np));
        splits = std::max<int64_t>(splits, 1);
    }
    DevBuf part;
    if (splits > 1) {
        g.kt_per = (int)ceil_div(g.ktiles, splits);
        splits = ceil_div(g.ktiles, g.kt_per);  // no empty split
        g.splits = (int)splits;
        BSMM_TRY(part.reserve(sizeof(T) * splits * Mp * Np, s));
        g.part = part.p;
    }
    {
        KernelTimer kt(0, s);
        const dim3 grid((unsigned)(tiles * splits));
        if (splits > 1) {
            if (KB == 32) hipLaunchKernelGGL((k_dgemm_mfma<T, 32, 1, true>), grid, dim3(256), 0, s, g);
            else hipLaunchKernelGGL((k_dgemm_mfma<T, 16, 2, true>), grid, dim3(256), 0, s, g);
        } else {
            if (KB == 32) hipLaunchKernelGGL((k_dgemm_mfma<T, 32, 1, false>), grid, dim3(256), 0, s, g);
            else hipLaunchKernelGGL((k_dgemm_mfma<T, 16, 2, false>), grid, dim3(256), 0, s, g);
        }
    }
    BSMM_TRY(launch_check("dgemm_mfma"));
    if (splits == 1) return BSMM_OK;
    hipLaunchKernelGGL(k_splitk_reduce<T>, dim3(grid_of(M * N, 256, 8192)), dim3(256), 0, s, g);
    return launch_check("splitk_reduce");
}

}  // namespace

int dense_multiply(const bsmm_matrix_s *A, const bsmm_matrix_s *B, bsmm_matrix_s *C,
                   double alpha, double beta, hipStream_t s) {
    if (C->dtype == BSMM_F32) return dense_multiply_t<float>(A, B, C, alpha, beta, s);
    return dense_multiply_t<double>(A, B, C, alpha, beta, s);
}

}  // namespace bsmm
