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
//      K * 127^2 * S below 2^31);
//   4. FP64 recombination in the epilogue: Horner h = G_{S+1}, h <- h 2^-7 + G_d
//      down to d = 2, value = h * 2^(e_i + e_j - 14) (exact scaling); chunk
//      values summed in FP64 in chunk order; C = beta C + alpha value with
//      separately rounded products (native FP64 for the recombination and
//      beta * C).
//
// Layout: A is merged transposed (rows of A contiguous in k) and B column-
// major (columns contiguous in k); slices keep those layouts as int8.
// GEMM tile: 64 x 64 outputs per 256-thread workgroup, k step 64; each wave
// owns 32 x 32 outputs = 2 x 2 tiles of v_mfma_i32_16x16x64_i8, with S INT32
// accumulators (one per weight d) per tile.
#include <algorithm>

#include "dev_util.h"
#include "internal.h"

namespace bsmm {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int ET = 64;   // output tile edge
constexpr int EK = 64;   // k step
constexpr int ELD = 80;  // LDS row stride in bytes (64 + 16 padding)

// Operand layout of v_mfma_i32_16x16x64_i8 (16 bytes per lane): lane l holds
// row (l % 16) of A (column of B) and k = 16 * (l / 16) .. +15.
// Result layout: D(row, col) in lane col + 16 * (row / 4), element row % 4.
__device__ __forceinline__ int frag_k(int lane) { return 16 * (lane >> 4); }
__device__ __forceinline__ int out_row(int lane, int e) { return 4 * (lane >> 4) + e; }

// Row exponents of a k-contiguous matrix (rows x ld): one wave per row.
__global__ __launch_bounds__(256) void k_row_exp(const double *X, int64_t rows, int64_t K,
                                                 int64_t ld, int *e) {
    const int64_t r = (int64_t)blockIdx.x * 4 + wave_id();
    if (r >= rows) return;
    double mx = 0.0;
    for (int64_t k = lane_id(); k < K; k += kWave) mx = fmax(mx, fabs(X[r * ld + k]));
    mx = wave_max(mx);
    if (lane_id() == 0) {
        int ex = 0;
        if (mx > 0.0) (void)frexp(mx, &ex);
        e[r] = ex;
    }
}

// Digit slices of a k-contiguous matrix: each thread handles 8 consecutive k
// of one row and writes S 8-byte groups.
__global__ __launch_bounds__(256) void k_slice(const double *X, int64_t rows, int64_t ld, int S,
                                               const int *e, signed char *out) {
    const int64_t per_row = ld / 8;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= rows * per_row) return;
    const int64_t r = idx / per_row, k8 = idx - r * per_row;
    const double sc = ldexp(1.0, -e[r]);
    double v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = X[r * ld + 8 * k8 + j] * sc;
    for (int s = 0; s < S; ++s) {
        unsigned long long w = 0;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const double t = v[j] * 128.0;
            const double d = trunc(t);
            v[j] = t - d;
            w |= (unsigned long long)(unsigned char)(signed char)(int)d << (8 * j);
        }
        *reinterpret_cast<unsigned long long *>(out + (int64_t)s * rows * ld + r * ld + 8 * k8) = w;
    }
}

struct EmulArgs {
    const signed char *As;  // S slices of Mp x Kp (row-major)
    const signed char *Bs;  // S slices of Np x Kp (column j contiguous in k)
    int64_t Mp, Np, Kp;
    int64_t k0, k1;         // k range of this chunk
    const int *ea, *eb;
    int mode;               // 1 first chunk, 2 later chunk, 4 last chunk (bit flags)
    double *V;              // FP64 partial values (Mp x Np, column-major), multi-chunk only
    int64_t M, N;
    double alpha, beta;
    double *C;
    const int64_t *c_blk_off;
    const int32_t *c_map;
    int32_t c_nbc;
    const int32_t *c_rbs;
    const int2 *rmap, *cmap;
};

template <int S>
__global__ __launch_bounds__(256) void k_emul_gemm(EmulArgs g) {
    // The recombination rounds every product and sum separately (no fused
    // multiply-add), matching the method's definition step by step.
#pragma clang fp contract(off)
    // Double-buffered LDS: slices of step k + 1 are fetched into registers
    // while the MFMAs of step k run, then stored to the other buffer.
    __shared__ __attribute__((aligned(16))) signed char lA[2][S][ET * ELD];
    __shared__ __attribute__((aligned(16))) signed char lB[2][S][ET * ELD];
    const int tiles_n = (int)(g.Np / ET);
    const int tm = blockIdx.x / tiles_n, tn = blockIdx.x % tiles_n;
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
    const signed char *pa = g.As + (row0 + lr) * g.Kp + lc;
    const signed char *pb = g.Bs + (col0 + lr) * g.Kp + lc;
    const int64_t sa = g.Mp * g.Kp, sb = g.Np * g.Kp;
    v4i ra[S], rb[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
        ra[s] = *reinterpret_cast<const v4i *>(pa + s * sa + g.k0);
        rb[s] = *reinterpret_cast<const v4i *>(pb + s * sb + g.k0);
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
                ra[s] = *reinterpret_cast<const v4i *>(pa + s * sa + k + EK);
                rb[s] = *reinterpret_cast<const v4i *>(pb + s * sb + k + EK);
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
                const int64_t row = row0 + wm * 32 + i * 16 + out_row(lane, e);
                const int64_t col = col0 + wn * 32 + j * 16 + (lane & 15);
                double h = (double)acc[S - 1][i][j][e];
#pragma unroll
                for (int d = S - 2; d >= 0; --d) h = h * (1.0 / 128.0) + (double)acc[d][i][j][e];
                double v = ldexp(h, g.ea[row] + g.eb[col] - 14);
                if (!(g.mode & 1)) v = g.V[col * g.Mp + row] + v;
                if (!(g.mode & 4)) {
                    g.V[col * g.Mp + row] = v;
                    continue;
                }
                if (row >= g.M || col >= g.N) continue;
                const int2 rm = g.rmap[row], cm = g.cmap[col];
                const int64_t bidx = (int64_t)rm.x * g.c_nbc + cm.x;
                const int32_t blk = g.c_map ? g.c_map[bidx] : (int32_t)bidx;
                if (blk < 0) continue;
                double *dst = g.C + g.c_blk_off[blk] + rm.y + (int64_t)g.c_rbs[rm.x] * cm.y;
                const double prod = g.alpha * v;
                *dst = (g.beta == 0.0) ? prod : g.beta * *dst + prod;
            }
}

// Transposing merge (one wave per block): block (I,K) of A lands at rows
// r0.. of the row-major panel At[i][k] (ld = panel columns).
__global__ __launch_bounds__(256) void k_merge_t(int32_t nbr, int64_t nnzb, const int32_t *rbs,
                                                 const int32_t *cbs, const int64_t *row_off,
                                                 const int64_t *col_off, const int64_t *rp,
                                                 const int32_t *ci, const int64_t *blk_off,
                                                 const double *data, double *panel, int64_t ld) {
    const int64_t p = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave_id();
    if (p >= nnzb) return;
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
        panel[(r0 + ii) * ld + c0 + jj] = src[e];
    }
}

__global__ __launch_bounds__(256) void k_merge_c(int32_t nbr, int64_t nnzb, const int32_t *rbs,
                                                 const int32_t *cbs, const int64_t *row_off,
                                                 const int64_t *col_off, const int64_t *rp,
                                                 const int32_t *ci, const int64_t *blk_off,
                                                 const double *data, double *panel, int64_t ld) {
    const int64_t p = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave_id();
    if (p >= nnzb) return;
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

__global__ __launch_bounds__(256) void k_block_map_e(int32_t nbc, const int64_t *rp,
                                                     const int32_t *ci, int32_t *map) {
    const int32_t row = blockIdx.x;
    for (int j = threadIdx.x; j < nbc; j += blockDim.x) map[(int64_t)row * nbc + j] = -1;
    __syncthreads();
    for (int64_t p = rp[row] + threadIdx.x; p < rp[row + 1]; p += blockDim.x)
        map[(int64_t)row * nbc + ci[p]] = (int32_t)p;
}

using EmulKernel = void (*)(EmulArgs);
EmulKernel emul_kernel(int S) {
    switch (S) {
    case 1: return k_emul_gemm<1>;
    case 2: return k_emul_gemm<2>;
    case 3: return k_emul_gemm<3>;
    case 4: return k_emul_gemm<4>;
    case 5: return k_emul_gemm<5>;
    case 6: return k_emul_gemm<6>;
    case 7: return k_emul_gemm<7>;
    case 8: return k_emul_gemm<8>;
    default: return nullptr;
    }
}

}  // namespace

// Largest k chunk (multiple of 64) with K * 127^2 * S < 2^31.
int64_t emul_chunk(int S) {
    int64_t k = (int64_t(2147483647)) / (127 * 127 * (int64_t)S);
    return std::max<int64_t>(EK, k / EK * EK);
}

int emul_multiply(const bsmm_matrix_s *A, const bsmm_matrix_s *B, bsmm_matrix_s *C,
                  double alpha, double beta, int S, hipStream_t s) {
    const int64_t M = A->rows(), K = A->cols(), N = B->cols();
    if (M == 0 || N == 0 || C->nnzb == 0) return BSMM_OK;
    if (alpha == 0.0 || K == 0) return scale_blocks(C, nullptr, beta, s);
    EmulKernel fn = emul_kernel(S);
    if (!fn) {
        set_error(BSMM_EINVAL, "emulation slices must be in [1, 8]");
        return BSMM_EINVAL;
    }
    const int64_t Mp = ceil_div(M, ET) * ET, Np = ceil_div(N, ET) * ET, Kp = ceil_div(K, EK) * EK;
    DevBuf at, bp, ea, eb, as, bs, V, cmap;
    BSMM_TRY(at.reserve(sizeof(double) * Mp * Kp, s));
    BSMM_TRY(bp.reserve(sizeof(double) * Kp * Np, s));
    BSMM_TRY(ea.reserve(sizeof(int) * Mp, s));
    BSMM_TRY(eb.reserve(sizeof(int) * Np, s));
    BSMM_TRY(as.reserve((size_t)S * Mp * Kp, s));
    BSMM_TRY(bs.reserve((size_t)S * Np * Kp, s));
    BSMM_TRY(fill_zero(at.as<double>(), Mp * Kp, s));
    BSMM_TRY(fill_zero(bp.as<double>(), Kp * Np, s));
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
        hipLaunchKernelGGL(k_block_map_e, dim3(C->nbr), dim3(256), 0, s, C->nbc, C->d_row_ptr(),
                           C->d_col_ind(), cmap.as<int32_t>());
        BSMM_TRY(launch_check("emul block map"));
        d_cmap = cmap.as<int32_t>();
    }
    const int64_t chunk = emul_chunk(S);
    const int64_t nchunks = ceil_div(Kp, chunk);
    if (nchunks > 1) BSMM_TRY(V.reserve(sizeof(double) * Mp * Np, s));
    const int64_t tiles = (Mp / ET) * (Np / ET);
    if (tiles > INT32_MAX) {
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
        g.V = V.as<double>();
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
        hipLaunchKernelGGL(fn, dim3((unsigned)tiles), dim3(256), 0, s, g);
        BSMM_TRY(launch_check("emul gemm"));
    }
    return BSMM_OK;
}

}  // namespace bsmm
