// emul.hip -- split-precision FP64 emulation of the dense product on INT8
// matrix cores.
//
// The Ozaki scheme (Ozaki, Ogita, Oishi, Rump, Numer. Algorithms 2012;
// integer form: Ootomo, Ozaki, Yokota, IJHPCA 2024), applied to the merged
// panels of the densified multiply (paper, Sec. III):
//   1. sigma_i = 2^e_i with max_k |a_ik| < 2^e_i per row of A, tau_j per
//      column of B (frexp exponents; zero rows get e = 0);
//   2. S digit slices per operand: r = a / sigma_i, d_s = trunc(128 r),
//      r <- 128 r - d_s (all exact in FP64), d_s in [-127, 127] stored as int8;
//   3. one INT8 MFMA GEMM over every digit pair with s + t <= S + 1,
//      accumulating G_d = sum_{s+t=d} A_s B_t exactly in INT32 (K chunks keep
//      K * 127^2 * S below 2^31; when K needs several chunks, each chunk adds
//      its INT32 sums into exact int64 partial sums, so G_d is the exact sum
//      over the whole K whatever the chunking);
//   4. FP64 recombination in the epilogue of the last chunk: Horner
//      h = G_{S+1}, h <- h 2^-7 + G_d down to d = 2, value =
//      h * 2^(e_i + e_j - 14) (exact scaling); C = beta C + alpha value with
//      separately rounded products (native FP64 for the recombination and
//      beta * C).
//
// Layout: A is merged transposed (rows of A contiguous in k) and B column-
// major (columns contiguous in k); the int8 slices are stored in k panels of
// 32 bytes ([slice][k / 32][row][k % 32]) so that every k step of a tile
// reads whole contiguous blocks.
// GEMM kernels (option "emul_kernel"), all with S INT32 accumulators (one per
// weight d) per output tile:
//   t64     64 x 64 outputs per 256-thread workgroup, each wave 2 x 2 tiles of
//           v_mfma_i32_16x16x64_i8, k step 64, two LDS stages;
//   t128    128 x 64 outputs, each wave 4 x 2 tiles of the same MFMA, k step
//           64, one LDS stage refilled from registers;
//   t128k32 128 x 64 outputs, each wave 2 x 1 tiles of
//           v_mfma_i32_32x32x32_i8, k step 32, two LDS stages;
//   t128w8  as t128k32 with 512 threads, each of the 8 waves one 32 x 32 tile
//           (two waves per SIMD; default).  Workgroup ids are remapped so that the
// tiles resident on one XCD form a compact group of tile rows and columns
// (their slices stay in that XCD's L2).
#include <algorithm>
#include <climits>

#include "dev_util.h"
#include "internal.h"

namespace bsmm {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int ET = 64;   // output tile edge
constexpr int EK = 64;   // k step
constexpr int ELD = 80;  // LDS row stride in bytes (64 + 16 padding)

// Operand layout of v_mfma_i32_16x16x64_i8 (16 bytes per lane): lane l holds
// row (l % 16) of A (column of B) and k = 16 * (l / 16) .. +15.
// Result layout: D(row, col) in lane col + 16 * (row / 4), element row % 4.
__device__ __forceinline__ int frag_k(int lane) { return 16 * (lane >> 4); }
__device__ __forceinline__ int out_row(int lane, int e) { return 4 * (lane >> 4) + e; }

constexpr int WTM = 128;  // wide tile: rows per workgroup
constexpr int WTN = 64;   // wide tile: columns per workgroup
constexpr int XK = 32;    // k step of the 32 x 32 x 32 variant
constexpr int XLD = 48;   // its LDS row stride in bytes (32 + 16 padding)

// v_mfma_i32_32x32x32_i8: lane l holds row (l % 32) of A (column of B) and
// 16 bytes of k at 16 * (l / 32); result element e of lane l is row
// 8 (e / 4) + 4 (l / 32) + e % 4, column l % 32.
__device__ __forceinline__ int out_row32(int lane, int e) {
    return 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
}

// Tile of this workgroup.  The hardware deals workgroups to the 8 XCDs round
// robin; the remap gives each XCD a contiguous range of logical ids, walked
// in groups of gm tile rows with the row index fastest, so concurrently
// resident workgroups of one XCD share A and B slices.  A bijection on
// [0, tiles_m * tiles_n) when the grid has exactly that many workgroups.
__device__ __forceinline__ void emul_tile_of(int tiles_m, int tiles_n, int gm, int &tm, int &tn) {
    const int nwg = gridDim.x;
    int logical = blockIdx.x;
    if ((nwg & 7) == 0) logical = (blockIdx.x & 7) * (nwg >> 3) + (blockIdx.x >> 3);
    const int per_group = gm * tiles_n;
    const int group = logical / per_group;
    const int first_m = group * gm;
    const int gsz = min(tiles_m - first_m, gm);
    const int in_group = logical - group * per_group;
    tm = first_m + in_group % gsz;
    tn = in_group / gsz;
}

// Exponent of a row holding an infinity or a NaN: digit slices cannot carry
// such values, so the row is sliced as zeros and every output element it
// touches becomes NaN.
constexpr int kNonFiniteExp = INT_MIN;

// Row exponents of a k-contiguous matrix (rows x ld): one wave per row.
__global__ __launch_bounds__(256) void k_row_exp(const double *X, int64_t rows, int64_t K,
                                                 int64_t ld, int *e) {
    for (int64_t r = (int64_t)blockIdx.x * 4 + wave_id(); r < rows; r += (int64_t)gridDim.x * 4) {
        double mx = 0.0;
        bool bad = false;
        for (int64_t k = lane_id(); k < K; k += kWave) {
            const double x = X[r * ld + k];
            bad |= !isfinite(x);
            mx = fmax(mx, fabs(x));
        }
        mx = wave_max(mx);
        const bool any_bad = __ballot(bad) != 0;
        if (lane_id() == 0) {
            int ex = 0;
            if (mx > 0.0) (void)frexp(mx, &ex);
            e[r] = any_bad ? kNonFiniteExp : ex;
        }
    }
}

// Digit slices of a k-contiguous matrix: each thread handles 8 consecutive k
// of one row and writes S 8-byte groups.  Slice layout: k panels of 32 bytes,
// [slice][k / 32][row][k % 32], so a tile's rows for one 32-deep k step are
// one contiguous block.
__global__ __launch_bounds__(256) void k_slice(const double *X, int64_t rows, int64_t ld, int S,
                                               const int *e, signed char *out) {
    // Thread -> (k panel p, row r, quarter q of the panel's 32 bytes):
    // consecutive threads write consecutive 8-byte groups of the output.
    const int64_t total = rows * (ld / 8);
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int q = (int)(idx & 3);
        const int64_t rp = idx >> 2;
        const int64_t p = rp / rows, r = rp - p * rows;
        const int64_t k = 32 * p + 8 * q;
        // Scaling by 2^-e in one step is exact also for subnormal rows (e
        // below -1022, where 2^-e itself would overflow).
        const int er = e[r];
        double v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = er == kNonFiniteExp ? 0.0 : ldexp(X[r * ld + k + j], -er);
        for (int s = 0; s < S; ++s) {
            unsigned long long w = 0;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const double t = v[j] * 128.0;
                const double d = trunc(t);
                v[j] = t - d;
                w |= (unsigned long long)(unsigned char)(signed char)(int)d << (8 * j);
            }
            *reinterpret_cast<unsigned long long *>(out + (int64_t)s * rows * ld + p * rows * 32 + r * 32 +
                                                    8 * q) = w;
        }
    }
}

struct EmulArgs {
    const signed char *As;  // S slices of Mp x Kp (row-major)
    const signed char *Bs;  // S slices of Np x Kp (column j contiguous in k)
    int64_t Mp, Np, Kp;
    int64_t k0, k1;         // k range of this chunk
    const int *ea, *eb;
    int mode;               // 1 first chunk, 2 later chunk, 4 last chunk (bit flags)
    long long *V;           // exact partial sums, S planes of Mp x Np (column-major), multi-chunk only
    int64_t M, N;
    double alpha, beta;
    double *C;
    const int64_t *c_blk_off;
    const int32_t *c_map;
    int32_t c_nbc;
    const int32_t *c_rbs;
    const int2 *rmap, *cmap;
};

// One output element from its S weight sums of this K chunk: exact int64
// accumulation over the chunks, then (last chunk) the FP64 recombination
// (Horner in 2^-7, exact power-of-two scaling) and the store
// C = beta C + alpha value into C's block (every operation rounded on its
// own: this file is compiled without contraction).  The int64 sums are
// exact (|G_d| <= S K 127^2 < 2^53), so converting them to FP64 is exact and
// the result does not depend on where K was split.
template <int S>
__device__ __forceinline__ void emul_out(const EmulArgs &g, const int (&vals)[S], int64_t row,
                                         int64_t col) {
    long long tot[S];
    const int64_t plane = g.Mp * g.Np, at = col * g.Mp + row;
#pragma unroll
    for (int d = 0; d < S; ++d) tot[d] = (g.mode & 1) ? (long long)vals[d] : g.V[d * plane + at] + vals[d];
    if (!(g.mode & 4)) {
#pragma unroll
        for (int d = 0; d < S; ++d) g.V[d * plane + at] = tot[d];
        return;
    }
    double h = (double)tot[S - 1];
#pragma unroll
    for (int d = S - 2; d >= 0; --d) h = h * (1.0 / 128.0) + (double)tot[d];
    // One power-of-two scaling (exponents lie in [-1073, 1024], so their sum
    // fits an int): the value is rounded at most once, on under- or overflow.
    const int ea = g.ea[row], eb = g.eb[col];
    const double v = (ea == kNonFiniteExp || eb == kNonFiniteExp) ? __builtin_nan("")
                                                                  : ldexp(h, ea + eb - 14);
    if (row >= g.M || col >= g.N) return;
    const int2 rm = g.rmap[row], cm = g.cmap[col];
    const int64_t bidx = (int64_t)rm.x * g.c_nbc + cm.x;
    const int32_t blk = g.c_map ? g.c_map[bidx] : (int32_t)bidx;
    if (blk < 0) return;
    double *dst = g.C + g.c_blk_off[blk] + rm.y + (int64_t)g.c_rbs[rm.x] * cm.y;
    const double prod = g.alpha * v;
    *dst = (g.beta == 0.0) ? prod : g.beta * *dst + prod;
}

template <int S>
__global__ __launch_bounds__(256) void k_emul_gemm(EmulArgs g) {
    // The recombination rounds every product and sum separately (no fused
    // multiply-add), matching the method's definition step by step.
#pragma clang fp contract(off)
    // Double-buffered LDS: slices of step k + 1 are fetched into registers
    // while the MFMAs of step k run, then stored to the other buffer.
    __shared__ __attribute__((aligned(16))) signed char lA[2][S][ET * ELD];
    __shared__ __attribute__((aligned(16))) signed char lB[2][S][ET * ELD];
    int tm, tn;
    emul_tile_of((int)(g.Mp / ET), (int)(g.Np / ET), 8, tm, tn);
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w & 1, wn = w >> 1;
    const int64_t row0 = (int64_t)tm * ET, col0 = (int64_t)tn * ET;

    v4i acc[S][2][2];
#pragma unroll
    for (int d = 0; d < S; ++d)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[d][i][j] = (v4i){0, 0, 0, 0};

    // global -> registers: 64 rows x 64 bytes per slice = 256 x 16 bytes
    const int lr = tid >> 2, lc = (tid & 3) * 16;
    const signed char *pa = g.As + ((lc >> 5) * g.Mp + row0 + lr) * 32 + (lc & 31);
    const signed char *pb = g.Bs + ((lc >> 5) * g.Np + col0 + lr) * 32 + (lc & 31);
    const int64_t sa = g.Mp * g.Kp, sb = g.Np * g.Kp, pA = g.Mp * 32, pB = g.Np * 32;
    v4i ra[S], rb[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
        ra[s] = *reinterpret_cast<const v4i *>(pa + s * sa + (g.k0 >> 5) * pA);
        rb[s] = *reinterpret_cast<const v4i *>(pb + s * sb + (g.k0 >> 5) * pB);
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
        *reinterpret_cast<v4i *>(&lA[0][s][lr * ELD + lc]) = ra[s];
        *reinterpret_cast<v4i *>(&lB[0][s][lr * ELD + lc]) = rb[s];
    }
    __syncthreads();
    int cur = 0;
    for (int64_t k = g.k0; k < g.k1; k += EK) {
        const bool more = k + EK < g.k1;
        if (more) {
#pragma unroll
            for (int s = 0; s < S; ++s) {
                ra[s] = *reinterpret_cast<const v4i *>(pa + s * sa + ((k + EK) >> 5) * pA);
                rb[s] = *reinterpret_cast<const v4i *>(pb + s * sb + ((k + EK) >> 5) * pB);
            }
        }
        v4i af[S][2], bf[S][2];
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                af[s][i] = *reinterpret_cast<const v4i *>(
                    &lA[cur][s][(wm * 32 + i * 16 + (lane & 15)) * ELD + frag_k(lane)]);
                bf[s][i] = *reinterpret_cast<const v4i *>(
                    &lB[cur][s][(wn * 32 + i * 16 + (lane & 15)) * ELD + frag_k(lane)]);
            }
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int t = 0; t < S - s; ++t)  // digit pair (s+1, t+1): weight d = s + t + 2
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        acc[s + t][i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(
                            af[s][i], bf[t][j], acc[s + t][i][j], 0, 0, 0);
        if (more) {
#pragma unroll
            for (int s = 0; s < S; ++s) {
                *reinterpret_cast<v4i *>(&lA[cur ^ 1][s][lr * ELD + lc]) = ra[s];
                *reinterpret_cast<v4i *>(&lB[cur ^ 1][s][lr * ELD + lc]) = rb[s];
            }
        }
        __syncthreads();
        cur ^= 1;
    }

    // Recombination (FP64) and store.
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                int vals[S];
#pragma unroll
                for (int d = 0; d < S; ++d) vals[d] = acc[d][i][j][e];
                emul_out<S>(g, vals, row0 + wm * 32 + i * 16 + out_row(lane, e),
                            col0 + wn * 32 + j * 16 + (lane & 15));
            }
}

// Wide variant: 128 x 64 outputs per workgroup, waves in 2 x 2, each wave
// 64 x 32 outputs (4 x 2 MFMA tiles).  One LDS stage (S x 192 rows of 64
// bytes, padded stride): the slices of step k + 1 are fetched into registers
// while the MFMAs of step k run and stored after a barrier.
template <int S>
__global__ __launch_bounds__(256, 1) void k_emul_gemm_w(EmulArgs g) {
#pragma clang fp contract(off)
    __shared__ __attribute__((aligned(16))) signed char lA[S][WTM * ELD];
    __shared__ __attribute__((aligned(16))) signed char lB[S][WTN * ELD];
    int tm, tn;
    emul_tile_of((int)(g.Mp / WTM), (int)(g.Np / WTN), 4, tm, tn);
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w & 1, wn = w >> 1;
    const int64_t row0 = (int64_t)tm * WTM, col0 = (int64_t)tn * WTN;

    v4i acc[S][4][2];
#pragma unroll
    for (int d = 0; d < S; ++d)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[d][i][j] = (v4i){0, 0, 0, 0};

    // global -> registers: per slice, A rows lr and lr + 64, B row lr
    // (16 bytes each at byte lc of the k step).
    const int lr = tid >> 2, lc = (tid & 3) * 16;
    const signed char *pa = g.As + ((lc >> 5) * g.Mp + row0 + lr) * 32 + (lc & 31);
    const signed char *pb = g.Bs + ((lc >> 5) * g.Np + col0 + lr) * 32 + (lc & 31);
    const int64_t sa = g.Mp * g.Kp, sb = g.Np * g.Kp, pA = g.Mp * 32, pB = g.Np * 32;
    const int64_t half = 64 * 32;
    v4i ra0[S], ra1[S], rb[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
        ra0[s] = *reinterpret_cast<const v4i *>(pa + s * sa + (g.k0 >> 5) * pA);
        ra1[s] = *reinterpret_cast<const v4i *>(pa + s * sa + half + (g.k0 >> 5) * pA);
        rb[s] = *reinterpret_cast<const v4i *>(pb + s * sb + (g.k0 >> 5) * pB);
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
        *reinterpret_cast<v4i *>(&lA[s][lr * ELD + lc]) = ra0[s];
        *reinterpret_cast<v4i *>(&lA[s][(lr + 64) * ELD + lc]) = ra1[s];
        *reinterpret_cast<v4i *>(&lB[s][lr * ELD + lc]) = rb[s];
    }
    __syncthreads();
    for (int64_t k = g.k0; k < g.k1; k += EK) {
        const bool more = k + EK < g.k1;
        if (more) {
#pragma unroll
            for (int s = 0; s < S; ++s) {
                ra0[s] = *reinterpret_cast<const v4i *>(pa + s * sa + ((k + EK) >> 5) * pA);
                ra1[s] = *reinterpret_cast<const v4i *>(pa + s * sa + half + ((k + EK) >> 5) * pA);
                rb[s] = *reinterpret_cast<const v4i *>(pb + s * sb + ((k + EK) >> 5) * pB);
            }
        }
        v4i bf[S][2];
#pragma unroll
        for (int t = 0; t < S; ++t)
#pragma unroll
            for (int j = 0; j < 2; ++j)
                bf[t][j] = *reinterpret_cast<const v4i *>(
                    &lB[t][(wn * 32 + j * 16 + (lane & 15)) * ELD + frag_k(lane)]);
#pragma unroll
        for (int s = 0; s < S; ++s) {
            v4i af[4];
#pragma unroll
            for (int i = 0; i < 4; ++i)
                af[i] = *reinterpret_cast<const v4i *>(
                    &lA[s][(wm * 64 + i * 16 + (lane & 15)) * ELD + frag_k(lane)]);
#pragma unroll
            for (int t = 0; t < S - s; ++t)  // digit pair (s+1, t+1): weight d = s + t + 2
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        acc[s + t][i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(
                            af[i], bf[t][j], acc[s + t][i][j], 0, 0, 0);
        }
        __syncthreads();
        if (more) {
#pragma unroll
            for (int s = 0; s < S; ++s) {
                *reinterpret_cast<v4i *>(&lA[s][lr * ELD + lc]) = ra0[s];
                *reinterpret_cast<v4i *>(&lA[s][(lr + 64) * ELD + lc]) = ra1[s];
                *reinterpret_cast<v4i *>(&lB[s][lr * ELD + lc]) = rb[s];
            }
        }
        __syncthreads();
    }

#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                int vals[S];
#pragma unroll
                for (int d = 0; d < S; ++d) vals[d] = acc[d][i][j][e];
                emul_out<S>(g, vals, row0 + wm * 64 + i * 16 + out_row(lane, e),
                            col0 + wn * 32 + j * 16 + (lane & 15));
            }
}

// 32 x 32 x 32 variant: 128 x 64 outputs per workgroup, waves in 2 x 2, each
// wave 64 x 32 outputs (2 x 1 tiles of v_mfma_i32_32x32x32_i8).  The k step
// of 32 halves an LDS stage (S x 192 rows of 32 bytes, padded stride), so two
// stages fit.  Slices travel global -> registers -> LDS two steps ahead of
// their use; one barrier per step; scheduling fences keep the order of the
// fragment reads, the stage stores and the fetches.
template <int S>
__global__ __launch_bounds__(256, 1) void k_emul_gemm_x(EmulArgs g) {
#pragma clang fp contract(off)
    constexpr int NB = (S + 1) / 2;  // B chunks per thread and step
    __shared__ __attribute__((aligned(16))) signed char lA[2][S][WTM * XLD];
    __shared__ __attribute__((aligned(16))) signed char lB[2][S][WTN * XLD];
    int tm, tn;
    emul_tile_of((int)(g.Mp / WTM), (int)(g.Np / WTN), 4, tm, tn);
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w & 1, wn = w >> 1;
    const int64_t row0 = (int64_t)tm * WTM, col0 = (int64_t)tn * WTN;

    v16i acc[S][2];
#pragma unroll
    for (int d = 0; d < S; ++d)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[d][i][e] = 0;

    // Staging.  Chunk c of a slice's 32-deep step (16 bytes) is row
    // 32 (c / 64) + l % 16 + 16 (l / 32), half (l / 16) % 2 with l = c % 64:
    // each wave reads one contiguous KB of the k panel, and every 16 lanes
    // write 16 consecutive rows of one half (no LDS bank conflicts).  A
    // chunk c = tid of every slice; B chunk j = tid + 256 q is chunk j % 128
    // of slice min(j / 128, S - 1).  For odd S the upper 128 threads of the
    // last round repeat the lower ones (same loads, same bytes stored), which
    // keeps the loop body free of branches.
    const int sl = tid & 63;
    const int ar = 32 * (tid >> 6) + (sl & 15) + 16 * (sl >> 5), ah = 16 * ((sl >> 4) & 1);
    const signed char *pa = g.As + (row0 + ar) * 32 + ah;
    const signed char *pb[NB];
    int lb[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const int j = tid + 256 * q;
        const int bs = min(j / 128, S - 1), c = j % 128;
        const int br = 32 * (c >> 6) + (sl & 15) + 16 * (sl >> 5);
        pb[q] = g.Bs + bs * g.Np * g.Kp + (col0 + br) * 32 + ah;
        lb[q] = bs * (WTN * XLD) + br * XLD + ah;
    }
    const int64_t sa = g.Mp * g.Kp, pA = g.Mp * 32, pB = g.Np * 32;
    const int64_t klast = g.k1 - XK;  // last step of the chunk; later fetches re-read it
    v4i ra[S], rb[NB];
#define BSMM_EMUL_FETCH(kk)                                                                    \
    do {                                                                                      \
        const int64_t kf_ = ((kk) < klast ? (kk) : klast) >> 5;                               \
        _Pragma("unroll") for (int s_ = 0; s_ < S; ++s_) ra[s_] =                             \
            *reinterpret_cast<const v4i *>(pa + s_ * sa + kf_ * pA);                          \
        _Pragma("unroll") for (int q_ = 0; q_ < NB; ++q_) rb[q_] =                            \
            *reinterpret_cast<const v4i *>(pb[q_] + kf_ * pB);                                \
    } while (0)
#define BSMM_EMUL_STAGE(st)                                                                   \
    do {                                                                                      \
        _Pragma("unroll") for (int s_ = 0; s_ < S; ++s_)                                      \
            *reinterpret_cast<v4i *>(&lA[st][s_][ar * XLD + ah]) = ra[s_];                    \
        _Pragma("unroll") for (int q_ = 0; q_ < NB; ++q_)                                     \
            *reinterpret_cast<v4i *>(&lB[st][0][0] + lb[q_]) = rb[q_];                        \
    } while (0)
    // Prologue: step k0 into stage 0, step k0 + 1 into registers.
    BSMM_EMUL_FETCH(g.k0);
    BSMM_EMUL_STAGE(0);
    BSMM_EMUL_FETCH(g.k0 + XK);
    __syncthreads();
    const int fr = (lane & 31) * XLD + 16 * (lane >> 5);  // fragment offset within a 32-row tile
    const int fa = wm * 64 * XLD + fr, fb = wn * 32 * XLD + fr;
    constexpr int kStageAfter = S > 2 ? 1 : 0;  // slice after whose MFMAs the stage is stored
    int cur = 0;
    for (int64_t k = g.k0; k < g.k1; k += XK) {
        // Software pipeline within the step: B fragments and slice 0 of A up
        // front; slice s + 1 of A is read while slice s's MFMAs run; after
        // slice kStageAfter, step k + 1 (fetched during the previous step)
        // goes to the other stage and step k + 2 is fetched.  The other stage
        // was last read before the previous barrier.
        v4i bf[S], af[S][2];
#pragma unroll
        for (int t = 0; t < S; ++t) bf[t] = *reinterpret_cast<const v4i *>(&lB[cur][t][fb]);
#pragma unroll
        for (int i = 0; i < 2; ++i)
            af[0][i] = *reinterpret_cast<const v4i *>(&lA[cur][0][fa + i * 32 * XLD]);
        __builtin_amdgcn_sched_group_barrier(0x100, S + 2, 0);  // DS reads: B, A slice 0
#pragma unroll
        for (int s = 0; s < S; ++s) {
            if (s + 1 < S) {
#pragma unroll
                for (int i = 0; i < 2; ++i)
                    af[s + 1][i] = *reinterpret_cast<const v4i *>(&lA[cur][s + 1][fa + i * 32 * XLD]);
                __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);  // DS reads: A slice s + 1
            }
#pragma unroll
            for (int t = 0; t < S - s; ++t) {  // digit pair (s+1, t+1): weight d = s + t + 2
#pragma unroll
                for (int i = 0; i < 2; ++i)
                    acc[s + t][i] = __builtin_amdgcn_mfma_i32_32x32x32_i8(af[s][i], bf[t],
                                                                          acc[s + t][i], 0, 0, 0);
                __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);  // the pair's MFMAs
            }
            if (s == kStageAfter) {
                // The registers hold step k + 1 until stored; only then are
                // they refilled with step k + 2.
                BSMM_EMUL_STAGE(cur ^ 1);
                __builtin_amdgcn_sched_group_barrier(0x200, S + NB, 0);  // DS writes: next stage
                BSMM_EMUL_FETCH(k + 2 * XK);
                __builtin_amdgcn_sched_group_barrier(0x020, S + NB, 0);  // global reads
            }
        }
        __syncthreads();
        cur ^= 1;
    }
#undef BSMM_EMUL_FETCH
#undef BSMM_EMUL_STAGE

#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            int vals[S];
#pragma unroll
            for (int d = 0; d < S; ++d) vals[d] = acc[d][i][e];
            emul_out<S>(g, vals, row0 + wm * 64 + i * 32 + out_row32(lane, e),
                        col0 + wn * 32 + (lane & 31));
        }
}

// Eight-wave variant of the 32 x 32 x 32 kernel: 512 threads per workgroup,
// the same 128 x 64 tile, waves in 4 x 2, each wave one 32 x 32 tile (S
// accumulators of 16 registers), so that two waves share each SIMD and hide
// each other's LDS and barrier waits.  Stages, slice layout and pipeline as
// in k_emul_gemm_x.
template <int S>
__global__ __launch_bounds__(512, 1) void k_emul_gemm_x8(EmulArgs g) {
#pragma clang fp contract(off)
    constexpr int NA = (S + 1) / 2;  // A chunks per thread and step
    constexpr int NB = (S + 3) / 4;  // B chunks per thread and step
    __shared__ __attribute__((aligned(16))) signed char lA[2][S][WTM * XLD];
    __shared__ __attribute__((aligned(16))) signed char lB[2][S][WTN * XLD];
    int tm, tn;
    emul_tile_of((int)(g.Mp / WTM), (int)(g.Np / WTN), 4, tm, tn);
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w & 3, wn = w >> 2;
    const int64_t row0 = (int64_t)tm * WTM, col0 = (int64_t)tn * WTN;

    v16i acc[S];
#pragma unroll
    for (int d = 0; d < S; ++d)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[d][e] = 0;

    // Staging (chunk -> row/half map as in k_emul_gemm_x).  A: chunk tid %
    // 256 of slices tid / 256 + 2 m; B: chunk j % 128 of slice j / 128 for
    // j = tid + 512 q.  Slice indices past S - 1 are clamped: those threads
    // repeat another thread's load and store the same bytes, which keeps the
    // loop body free of branches.
    const int sl = tid & 63;
    const int crow = (sl & 15) + 16 * (sl >> 5), ah = 16 * ((sl >> 4) & 1);
    const int ar = 32 * ((tid & 255) >> 6) + crow;
    const signed char *pa[NA];
    int la[NA];
#pragma unroll
    for (int m = 0; m < NA; ++m) {
        const int as = min((tid >> 8) + 2 * m, S - 1);
        pa[m] = g.As + as * g.Mp * g.Kp + (row0 + ar) * 32 + ah;
        la[m] = as * (WTM * XLD) + ar * XLD + ah;
    }
    const signed char *pb[NB];
    int lb[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const int j = tid + 512 * q;
        const int bs = min(j / 128, S - 1), c = j % 128;
        const int br = 32 * (c >> 6) + crow;
        pb[q] = g.Bs + bs * g.Np * g.Kp + (col0 + br) * 32 + ah;
        lb[q] = bs * (WTN * XLD) + br * XLD + ah;
    }
    const int64_t pA = g.Mp * 32, pB = g.Np * 32;
    const int64_t klast = g.k1 - XK;  // last step of the chunk; later fetches re-read it
    v4i ra[NA], rb[NB];
#define BSMM_EMUL_FETCH(kk)                                                                    \
    do {                                                                                      \
        const int64_t kf_ = ((kk) < klast ? (kk) : klast) >> 5;                               \
        _Pragma("unroll") for (int m_ = 0; m_ < NA; ++m_) ra[m_] =                            \
            *reinterpret_cast<const v4i *>(pa[m_] + kf_ * pA);                                \
        _Pragma("unroll") for (int q_ = 0; q_ < NB; ++q_) rb[q_] =                            \
            *reinterpret_cast<const v4i *>(pb[q_] + kf_ * pB);                                \
    } while (0)
#define BSMM_EMUL_STAGE(st)                                                                   \
    do {                                                                                      \
        _Pragma("unroll") for (int m_ = 0; m_ < NA; ++m_)                                     \
            *reinterpret_cast<v4i *>(&lA[st][0][0] + la[m_]) = ra[m_];                        \
        _Pragma("unroll") for (int q_ = 0; q_ < NB; ++q_)                                     \
            *reinterpret_cast<v4i *>(&lB[st][0][0] + lb[q_]) = rb[q_];                        \
    } while (0)
    BSMM_EMUL_FETCH(g.k0);
    BSMM_EMUL_STAGE(0);
    BSMM_EMUL_FETCH(g.k0 + XK);
    __syncthreads();
    const int fr = (lane & 31) * XLD + 16 * (lane >> 5);
    const int fa = wm * 32 * XLD + fr, fb = wn * 32 * XLD + fr;
    constexpr int kStageAfter = S > 2 ? 1 : 0;
    int cur = 0;
    for (int64_t k = g.k0; k < g.k1; k += XK) {
        v4i bf[S], af[S];
#pragma unroll
        for (int t = 0; t < S; ++t) bf[t] = *reinterpret_cast<const v4i *>(&lB[cur][t][fb]);
        af[0] = *reinterpret_cast<const v4i *>(&lA[cur][0][fa]);
        __builtin_amdgcn_sched_group_barrier(0x100, S + 1, 0);  // DS reads: B, A slice 0
#pragma unroll
        for (int s = 0; s < S; ++s) {
            if (s + 1 < S) {
                af[s + 1] = *reinterpret_cast<const v4i *>(&lA[cur][s + 1][fa]);
                __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // DS read: A slice s + 1
            }
#pragma unroll
            for (int t = 0; t < S - s; ++t) {  // digit pair (s+1, t+1): weight d = s + t + 2
                acc[s + t] = __builtin_amdgcn_mfma_i32_32x32x32_i8(af[s], bf[t], acc[s + t], 0, 0, 0);
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
            }
            if (s == kStageAfter) {
                BSMM_EMUL_STAGE(cur ^ 1);
                __builtin_amdgcn_sched_group_barrier(0x200, NA + NB, 0);  // DS writes: next stage
                BSMM_EMUL_FETCH(k + 2 * XK);
                __builtin_amdgcn_sched_group_barrier(0x020, NA + NB, 0);  // global reads
            }
        }
        __syncthreads();
        cur ^= 1;
    }
#undef BSMM_EMUL_FETCH
#undef BSMM_EMUL_STAGE

#pragma unroll
    for (int e = 0; e < 16; ++e) {
        int vals[S];
#pragma unroll
        for (int d = 0; d < S; ++d) vals[d] = acc[d][e];
        emul_out<S>(g, vals, row0 + wm * 32 + out_row32(lane, e), col0 + wn * 32 + (lane & 31));
    }
}

// Transposing merge (one wave per block): block (I,K) of A lands at rows
// r0.. of the row-major panel At[i][k] (ld = panel columns).
__global__ __launch_bounds__(256) void k_merge_t(int32_t nbr, int64_t nnzb, const int32_t *rbs,
                                                 const int32_t *cbs, const int64_t *row_off,
                                                 const int64_t *col_off, const int64_t *rp,
                                                 const int32_t *ci, const int64_t *blk_off,
                                                 const double *data, double *panel, int64_t ld) {
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
    for (int64_t p = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave_id(); p < nnzb; p += waves) {
        int32_t lo = 0, hi = nbr;  // block row: rp[lo] <= p < rp[lo + 1]
        while (hi - lo > 1) {
            const int32_t mid = (lo + hi) >> 1;
            if (rp[mid] <= p) lo = mid;
            else hi = mid;
        }
        const int m = rbs[lo];
        const int64_t r0 = row_off[lo];
        const int32_t j = ci[p];
        const int n = cbs[j];
        const int64_t c0 = col_off[j];
        const double *src = data + blk_off[p];
        const int64_t len = (int64_t)m * n;
        // Consecutive lanes write consecutive columns of one panel row
        // (reads stride through the block, which stays in cache).
        for (int64_t e = lane_id(); e < len; e += kWave) {
            const int64_t ii = e / n, jj = e - ii * n;
            panel[(r0 + ii) * ld + c0 + jj] = src[jj * m + ii];
        }
    }
}

__global__ __launch_bounds__(256) void k_merge_c(int32_t nbr, int64_t nnzb, const int32_t *rbs,
                                                 const int32_t *cbs, const int64_t *row_off,
                                                 const int64_t *col_off, const int64_t *rp,
                                                 const int32_t *ci, const int64_t *blk_off,
                                                 const double *data, double *panel, int64_t ld) {
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
    for (int64_t p = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave_id(); p < nnzb; p += waves) {
        int32_t lo = 0, hi = nbr;  // block row: rp[lo] <= p < rp[lo + 1]
        while (hi - lo > 1) {
            const int32_t mid = (lo + hi) >> 1;
            if (rp[mid] <= p) lo = mid;
            else hi = mid;
        }
        const int m = rbs[lo];
        const int64_t r0 = row_off[lo];
        const int32_t j = ci[p];
        const int n = cbs[j];
        const int64_t c0 = col_off[j];
        const double *src = data + blk_off[p];
        const int64_t len = (int64_t)m * n;
        for (int64_t e = lane_id(); e < len; e += kWave) {
            const int64_t jj = e / m, ii = e - jj * m;
            panel[(c0 + jj) * ld + r0 + ii] = src[e];
        }
    }
}

__global__ __launch_bounds__(256) void k_block_map_e(int32_t nbr, int32_t nbc, const int64_t *rp,
                                                     const int32_t *ci, int32_t *map) {
    for (int32_t row = blockIdx.x; row < nbr; row += gridDim.x) {
        for (int j = threadIdx.x; j < nbc; j += blockDim.x) map[(int64_t)row * nbc + j] = -1;
        __syncthreads();
        for (int64_t p = rp[row] + threadIdx.x; p < rp[row + 1]; p += blockDim.x)
            map[(int64_t)row * nbc + ci[p]] = (int32_t)p;
        __syncthreads();
    }
}

using EmulKernel = void (*)(EmulArgs);
template <int S>
EmulKernel emul_kernel_s(int variant) {
    return variant == 0 ? k_emul_gemm<S>
         : variant == 1 ? k_emul_gemm_w<S>
         : variant == 2 ? k_emul_gemm_x<S>
                        : k_emul_gemm_x8<S>;
}
// variant 0: 64 x 64 tiles; 1: 128 x 64, 16x16x64 MFMA, one stage; 2: 128 x 64,
// 32x32x32 MFMA, two stages; 3: as 2 with eight waves per workgroup.
EmulKernel emul_kernel(int S, int variant) {
    switch (S) {
    case 1: return emul_kernel_s<1>(variant);
    case 2: return emul_kernel_s<2>(variant);
    case 3: return emul_kernel_s<3>(variant);
    case 4: return emul_kernel_s<4>(variant);
    case 5: return emul_kernel_s<5>(variant);
    case 6: return emul_kernel_s<6>(variant);
    case 7: return emul_kernel_s<7>(variant);
    case 8: return emul_kernel_s<8>(variant);
    default: return nullptr;
    }
}

}  // namespace

// Largest k chunk (multiple of 64, hence of every variant's k step) with
// K * 127^2 * S < 2^31.
int64_t emul_chunk(int S) {
    int64_t k = (int64_t(2147483647)) / (127 * 127 * (int64_t)S);
    return std::max<int64_t>(EK, k / EK * EK);
}

int emul_multiply(const bsmm_matrix_s *A, const bsmm_matrix_s *B, bsmm_matrix_s *C,
                  double alpha, double beta, int S, hipStream_t s) {
    const int64_t M = A->rows(), K = A->cols(), N = B->cols();
    if (M == 0 || N == 0 || C->nnzb == 0) return BSMM_OK;
    if (alpha == 0.0 || K == 0) return scale_blocks(C, nullptr, beta, s);
    const int variant = options().emul_kernel;
    const bool wide = variant != 0;
    EmulKernel fn = emul_kernel(S, variant);
    if (!fn) {
        set_error(BSMM_EINVAL, "emulation slices must be in [1, 8]");
        return BSMM_EINVAL;
    }
    const int64_t tile_m = wide ? WTM : ET, tile_n = wide ? WTN : ET;
    const int64_t Mp = ceil_div(M, tile_m) * tile_m, Np = ceil_div(N, tile_n) * tile_n;
    const int64_t Kp = ceil_div(K, EK) * EK;
    DevBuf at, bp, ea, eb, as, bs, V, cmap;
    BSMM_TRY(at.reserve(sizeof(double) * Mp * Kp, s));
    BSMM_TRY(bp.reserve(sizeof(double) * Kp * Np, s));
    BSMM_TRY(ea.reserve(sizeof(int) * Mp, s));
    BSMM_TRY(eb.reserve(sizeof(int) * Np, s));
    BSMM_TRY(as.reserve((size_t)S * Mp * Kp, s));
    BSMM_TRY(bs.reserve((size_t)S * Np * Kp, s));
    // Panels need zeros where no block lands: padding and missing blocks.
    if (!(A->full() && Mp == M && Kp == K)) BSMM_TRY(fill_zero(at.as<double>(), Mp * Kp, s));
    if (!(B->full() && Np == N && Kp == K)) BSMM_TRY(fill_zero(bp.as<double>(), Kp * Np, s));
    if (A->nnzb > 0) {
        hipLaunchKernelGGL(k_merge_t, dim3(grid_of(A->nnzb, 4)), dim3(256), 0, s, A->nbr, A->nnzb,
                           A->d_rbs(), A->d_cbs(),
                           A->d_row_off(), A->d_col_off(), A->d_row_ptr(), A->d_col_ind(),
                           A->d_blk_off(), A->d_data(), at.as<double>(), Kp);
        BSMM_TRY(launch_check("emul merge A"));
    }
    if (B->nnzb > 0) {
        hipLaunchKernelGGL(k_merge_c, dim3(grid_of(B->nnzb, 4)), dim3(256), 0, s, B->nbr, B->nnzb,
                           B->d_rbs(), B->d_cbs(),
                           B->d_row_off(), B->d_col_off(), B->d_row_ptr(), B->d_col_ind(),
                           B->d_blk_off(), B->d_data(), bp.as<double>(), Kp);
        BSMM_TRY(launch_check("emul merge B"));
    }
    hipLaunchKernelGGL(k_row_exp, dim3(grid_of(Mp, 4)), dim3(256), 0, s,
                       (const double *)at.as<double>(), Mp, K, Kp, ea.as<int>());
    hipLaunchKernelGGL(k_row_exp, dim3(grid_of(Np, 4)), dim3(256), 0, s,
                       (const double *)bp.as<double>(), Np, K, Kp, eb.as<int>());
    BSMM_TRY(launch_check("emul exponents"));
    hipLaunchKernelGGL(k_slice, dim3(grid_of(Mp * (Kp / 8), 256)), dim3(256), 0, s,
                       (const double *)at.as<double>(), Mp, Kp, S, (const int *)ea.as<int>(),
                       as.as<signed char>());
    hipLaunchKernelGGL(k_slice, dim3(grid_of(Np * (Kp / 8), 256)), dim3(256), 0, s,
                       (const double *)bp.as<double>(), Np, Kp, S, (const int *)eb.as<int>(),
                       bs.as<signed char>());
    BSMM_TRY(launch_check("emul slices"));
    const int32_t *d_cmap = nullptr;
    if (!C->full()) {
        const int64_t cells = (int64_t)C->nbr * C->nbc;
        if (cells > (int64_t(1) << 30)) {
            set_error(BSMM_ENOTSUP, "emulated path on a sparse C with more than 2^30 block cells");
            return BSMM_ENOTSUP;
        }
        BSMM_TRY(cmap.reserve(sizeof(int32_t) * cells, s));
        hipLaunchKernelGGL(k_block_map_e, dim3(grid_rows(C->nbr)), dim3(256), 0, s, C->nbr, C->nbc,
                           C->d_row_ptr(),
                           C->d_col_ind(), cmap.as<int32_t>());
        BSMM_TRY(launch_check("emul block map"));
        d_cmap = cmap.as<int32_t>();
    }
    const int64_t chunk = emul_chunk(S);
    const int64_t nchunks = ceil_div(Kp, chunk);
    if (nchunks > 1) BSMM_TRY(V.reserve(sizeof(long long) * S * Mp * Np, s));
    const int64_t tiles = (Mp / tile_m) * (Np / tile_n);
    if (tiles > kMaxGridBlocks) {
        set_error(BSMM_ERANGE, "emulated product too large");
        return BSMM_ERANGE;
    }
    for (int64_t c = 0; c < nchunks; ++c) {
        EmulArgs g{};
        g.As = as.as<signed char>();
        g.Bs = bs.as<signed char>();
        g.Mp = Mp;
        g.Np = Np;
        g.Kp = Kp;
        g.k0 = c * chunk;
        g.k1 = std::min(Kp, (c + 1) * chunk);
        g.ea = ea.as<int>();
        g.eb = eb.as<int>();
        g.mode = (c == 0 ? 1 : 2) | (c == nchunks - 1 ? 4 : 0);
        g.V = V.as<long long>();
        g.M = M;
        g.N = N;
        g.alpha = alpha;
        g.beta = beta;
        g.C = C->d_data();
        g.c_blk_off = C->d_blk_off();
        g.c_map = d_cmap;
        g.c_nbc = C->nbc;
        g.c_rbs = C->d_rbs();
        g.rmap = C->d_row_map();
        g.cmap = C->d_col_map();
        KernelTimer kt(0, s);
        hipLaunchKernelGGL(fn, dim3((unsigned)tiles), dim3(variant == 3 ? 512 : 256), 0, s, g);
        BSMM_TRY(launch_check("emul gemm"));
    }
    return BSMM_OK;
}

}  // namespace bsmm
