// smm.hip -- batched small-block GEMM over the product stacks (FP64).
//
// Paper, Sec. II: the stacks of small block products are processed by
// dedicated small-matrix kernels (LIBCUSMM on NVIDIA GPUs, parametrised by
// the amount of work per thread block, the elements computed per thread and
// the tiling).  This is the gfx950 counterpart, written for wave64:
//
//  * a wavefront is split into G groups of L lanes; a group owns one run
//    (all products of one C block) at a time, so C stays in registers for
//    the whole run and is read-modified-written exactly once;
//  * every lane holds a TM x TN register tile of C (FP64 VALU FMAs: on
//    MI355X the FP64 vector rate equals the FP64 matrix rate, so small
//    blocks need no padding to MFMA shapes);
//  * each product's A block (m x k) and B block (k x n), contiguous in
//    memory, are staged into the group's LDS region with coalesced loads
//    and read back per k step, A as TM consecutive values, B as TN values
//    of one row;
//  * long k is split into chunks that fit the region; tile sets larger than
//    one wavefront are covered in passes;
//  * for blocks of about 16 x 16 and more, a variant runs each C block on
//    FP64 matrix cores (register tile "16 x 16" in the parameter space).
//
// The epilogue applies C = beta*C + alpha*acc (beta == 0 overwrites).
#include <algorithm>
#include <mutex>

#include "dev_util.h"
#include "internal.h"
#include "mfma_util.h"

namespace bsmm {

namespace {

template <class T, int TM, int TN>
__global__ __launch_bounds__(256) void k_smm_valu(SmmArgs p) {
    extern __shared__ double lds_raw[];
    T *lds = reinterpret_cast<T *>(lds_raw);
    const T *A = static_cast<const T *>(p.A);
    const T *B = static_cast<const T *>(p.B);
    T *C = static_cast<T *>(p.C);
    const T alpha = (T)p.alpha, beta = (T)p.beta;
    const int lane = lane_id();
    const int g = lane / p.L;
    const int gl = lane - g * p.L;
    const bool in_group = g < p.G;
    T *reg = lds + (size_t)(wave_id() * p.G + (in_group ? g : 0)) * p.region;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
    const int64_t wid = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave_id();
    const int m = p.m, n = p.n;
    const int tiles = p.tiles_m * p.tiles_n;

    for (int64_t rb = p.run_begin + wid * p.G; rb < p.run_end; rb += waves * p.G) {
        const int64_t r = rb + g;
        const bool has = in_group && r < p.run_end;
        const int64_t q0 = has ? p.run_ptr[r] : 0;
        const int64_t q1 = has ? p.run_ptr[r + 1] : 0;
        const int64_t nq = wave_max(q1 - q0);
        for (int pass = 0; pass < p.passes; ++pass) {
            const int t = pass * p.L + gl;
            const bool tile_ok = has && t < tiles;
            const int it = tile_ok ? t % p.tiles_m : 0;
            const int jt = tile_ok ? t / p.tiles_m : 0;
            const int i0 = it * TM, j0 = jt * TN;
            T acc[TM][TN];
#pragma unroll
            for (int a = 0; a < TM; ++a)
#pragma unroll
                for (int b = 0; b < TN; ++b) acc[a][b] = T(0);

            for (int64_t qi = 0; qi < nq; ++qi) {
                const bool act = has && qi < q1 - q0;
                ulonglong2 pr = make_ulonglong2(0ull, 0ull);
                if (act) pr = p.prods[q0 + qi];
                const int64_t a_off = (int64_t)(pr.x & ((1ull << 48) - 1));
                const int k = act ? (int)(pr.x >> 48) : 0;
                const int64_t b_off = (int64_t)pr.y;
                const int kmax = wave_max(k);
                for (int kc0 = 0; kc0 < kmax; kc0 += p.kc_max) {
                    const int kc = act ? std::min(p.kc_max, k - kc0) : 0;
                    // stage A(:, kc0:kc0+kc) (contiguous) and B(kc0:kc0+kc, :)
                    if (kc > 0) {
                        const T *ga = A + a_off + (int64_t)m * kc0;
                        const int na = m * kc;
                        for (int e = gl; e < na; e += p.L) reg[e] = ga[e];
                        T *rbuf = reg + na;
                        const T *gb = B + b_off + kc0;
                        if (kc == k) {
                            const int nb = k * n;
                            for (int e = gl; e < nb; e += p.L) rbuf[e] = gb[e];
                        } else {
                            const int nb = kc * n;
                            const float rcp = 1.0f / (float)kc;
                            for (int e = gl; e < nb; e += p.L) {
                                int kk;
                                const int j = divmod_small(e, kc, rcp, &kk);
                                rbuf[e] = gb[(int64_t)j * k + kk];
                            }
                        }
                    }
                    wave_lds_sync();
                    if (tile_ok && kc > 0) {
                        const T *As = reg + i0;
                        const T *Bs = reg + m * kc + (int64_t)j0 * kc;
                        for (int kk = 0; kk < kc; ++kk) {
                            T av[TM], bv[TN];
#pragma unroll
                            for (int a = 0; a < TM; ++a) av[a] = As[kk * m + a];
#pragma unroll
                            for (int b = 0; b < TN; ++b) bv[b] = Bs[b * kc + kk];
#pragma unroll
                            for (int a = 0; a < TM; ++a)
#pragma unroll
                                for (int b = 0; b < TN; ++b) acc[a][b] = fma(av[a], bv[b], acc[a][b]);
                        }
                    }
                    wave_lds_sync();
                }
            }
            if (tile_ok) {
                T *c = C + p.run_coff[r];
#pragma unroll
                for (int b = 0; b < TN; ++b) {
                    const int j = j0 + b;
                    if (j >= n) break;
#pragma unroll
                    for (int a = 0; a < TM; ++a) {
                        const int i = i0 + a;
                        if (i < m) {
                            T *dst = c + (int64_t)j * m + i;
                            const T prod = alpha * acc[a][b];
                            *dst = (beta == T(0)) ? prod : fma(beta, *dst, prod);
                        }
                    }
                }
            }
        }
    }
}

// MFMA variant for blocks of at least about 16 x 16 (parameter set
// tm = tn = 16): one wave owns one run at a time and keeps the C block as
// MT x NT tiles of 16 x 16 x 4 MFMA accumulators (m <= 16 MT, n <= 16 NT):
// v_mfma_f64_16x16x4 for FP64, v_mfma_f32_16x16x4 for FP32.  Operands come
// straight from the contiguous A and B blocks (each product's blocks are a
// few KB and stay in L1/L2), zero outside the block, so 23- or 13-sized
// blocks are padded in registers only.  Both instructions take lane l's
// operands at row (or column) l % 16 and k = l / 16 of the step.
// Products [q0, q1) of one run into the MT x NT accumulator tiles of an
// m x n C block.
template <class T, int MT, int NT, bool AT = false>
__device__ __forceinline__ void mfma_products(const SmmArgs &p, int m, int n, int64_t q0, int64_t q1,
                                              typename Mfma<T>::acc_t (&acc)[MT][NT]) {
    const int lane = lane_id();
    const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[i][j] = Mfma<T>::zero();
    const T *A = static_cast<const T *>(AT ? p.A_t : p.A);
    const T *B = static_cast<const T *>(p.B);
    // The next product's descriptor is loaded one product ahead.
    ulonglong2 nxt = q0 < q1 ? p.prods[q0] : make_ulonglong2(0ull, 0ull);
    for (int64_t q = q0; q < q1; ++q) {
        const ulonglong2 pr = nxt;
        if (q + 1 < q1) nxt = p.prods[q + 1];
        const T *a = A + (int64_t)(pr.x & ((1ull << 48) - 1));
        const int k = (int)(pr.x >> 48);
        const T *b = B + (int64_t)pr.y;
        for (int k0 = 0; k0 < k; k0 += 16) {
            // Four k steps of fragments, then their MFMAs.  Lane group
            // g = l / 16 supplies k = k0 + 4 g + s to step s (any
            // assignment of k to steps is valid when A and B agree), so a
            // lane's B operands are four consecutive values of a column.
            T af[4][MT], bf[4][NT];
            const int kb = k0 + 4 * lk;
#pragma unroll
            for (int i = 0; i < MT; ++i) {
                const int row = 16 * i + lr;
                if (AT) {
                    // Row-major copy: the four k values of a row are adjacent.
                    const T *ar = a + (int64_t)row * k + kb;
                    if (row < m && kb + 3 < k) {
                        T v[4];
                        Mfma<T>::load4(ar, v);
#pragma unroll
                        for (int s = 0; s < 4; ++s) af[s][i] = v[s];
                    } else {
#pragma unroll
                        for (int s = 0; s < 4; ++s) af[s][i] = (row < m && kb + s < k) ? ar[s] : T(0);
                    }
                } else {
#pragma unroll
                    for (int s = 0; s < 4; ++s)
                        af[s][i] = (row < m && kb + s < k) ? a[(int64_t)(kb + s) * m + row] : T(0);
                }
            }
#pragma unroll
            for (int j = 0; j < NT; ++j) {
                const int col = 16 * j + lr;
                const T *bc = b + (int64_t)col * k + kb;
                if (col < n && kb + 3 < k) {
                    T v[4];
                    Mfma<T>::load4(bc, v);
#pragma unroll
                    for (int s = 0; s < 4; ++s) bf[s][j] = v[s];
                } else {
#pragma unroll
                    for (int s = 0; s < 4; ++s) bf[s][j] = (col < n && kb + s < k) ? bc[s] : T(0);
                }
            }
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int i = 0; i < MT; ++i)
#pragma unroll
                    for (int j = 0; j < NT; ++j) acc[i][j] = Mfma<T>::step(af[s][i], bf[s][j], acc[i][j]);
        }
    }
}

// C block (column-major, ld = m) <- beta C + alpha acc, or the unscaled
// accumulators into a partial block when alpha is not applied here.
template <class T, int MT, int NT>
__device__ __forceinline__ void mfma_store(T *c, int m, int n,
                                           const typename Mfma<T>::acc_t (&acc)[MT][NT],
                                           bool partial, T alpha, T beta) {
    const int lane = lane_id();
    const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = 16 * i + Mfma<T>::row(e, lk), col = 16 * j + lr;
                if (row < m && col < n) {
                    T *dst = c + (int64_t)col * m + row;
                    if (partial) {
                        *dst = acc[i][j][e];
                    } else {
                        const T prod = alpha * acc[i][j][e];
                        *dst = (beta == T(0)) ? prod : fma(beta, *dst, prod);
                    }
                }
            }
}

// mfma_store (C = beta C + alpha acc) that also returns, on every lane,
// the squared Frobenius norm of the stored block (summed in FP64: each
// lane's elements in order, then across the wave in a fixed order).
template <class T, int MT, int NT>
__device__ __forceinline__ double mfma_store_sumsq(T *c, int m, int n,
                                                   const typename Mfma<T>::acc_t (&acc)[MT][NT],
                                                   T alpha, T beta) {
    const int lane = lane_id();
    const int lr = lane & 15, lk = lane >> 4;
    double ss = 0.0;
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = 16 * i + Mfma<T>::row(e, lk), col = 16 * j + lr;
                if (row < m && col < n) {
                    T *dst = c + (int64_t)col * m + row;
                    const T prod = alpha * acc[i][j][e];
                    const T v = (beta == T(0)) ? prod : fma(beta, *dst, prod);
                    *dst = v;
                    ss = fma((double)v, (double)v, ss);
                }
            }
    return wave_sum(ss);
}

template <class T, int MT, int NT>
__global__ __launch_bounds__(256) void k_smm_mfma(SmmArgs p) {
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
    const int64_t wid = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave_id();
    const int m = p.m, n = p.n;
    const int S = p.split > 1 ? p.split : 1;
    const int64_t items = (p.run_end - p.run_begin) * S;
    for (int64_t it = wid; it < items; it += waves) {
        // Item = (run, segment): segment sg of S takes products
        // [len sg / S, len (sg + 1) / S) of the run.
        const int64_t r = p.run_begin + it / S;
        const int sg = (int)(it % S);
        const int64_t rq0 = p.run_ptr[r], len = p.run_ptr[r + 1] - rq0;
        const int64_t q0 = rq0 + len * sg / S, q1 = rq0 + len * (sg + 1) / S;
        typename Mfma<T>::acc_t acc[MT][NT];
        mfma_products<T, MT, NT>(p, m, n, q0, q1, acc);
        if (S > 1)
            mfma_store<T, MT, NT>(static_cast<T *>(p.part) + it * (int64_t)m * n, m, n, acc, true, T(0),
                                  T(0));
        else
            mfma_store<T, MT, NT>(static_cast<T *>(p.C) + p.run_coff[r], m, n, acc, false, (T)p.alpha,
                                  (T)p.beta);
    }
}

// Runs of every class with C blocks up to 32 x 32 in one launch, in the
// order of a schedule that groups the runs by 2-D tiles of C blocks: the
// waves in flight then work on nearby block rows and block columns and
// share their A and B blocks in the caches.  Schedule entry: run << 16 |
// m << 8 | n.  Static mode: wave slots are numbered XCD by XCD (workgroup g
// runs on XCD g % 8), so each XCD takes a contiguous part of every window
// of in-flight runs; dynamic mode: waves take the next run from a counter.
template <class T, int MT, int NT, bool AT>
__device__ __forceinline__ void sched_run(const SmmArgs &p, int64_t r, int m, int n) {
    typename Mfma<T>::acc_t acc[MT][NT];
    mfma_products<T, MT, NT, AT>(p, m, n, p.run_ptr[r], p.run_ptr[r + 1], acc);
    // One store path: the norm is summed whether or not the filter wants it.
    const double ss = mfma_store_sumsq<T, MT, NT>(static_cast<T *>(p.C) + p.run_coff[r], m, n, acc,
                                                  (T)p.alpha, (T)p.beta);
    if (p.norm2 && lane_id() == 0) p.norm2[p.run_cblk[r]] = ss;
}

constexpr int kXcds = 8;
// Fewest runs for which the MFMA classes go through the scheduled launch.
constexpr int64_t kSchedMinRuns = 4096;

template <class T, bool AT>
__device__ __forceinline__ void sched_loop(const SmmArgs &p) {
    const int wpw = blockDim.x / kWave;
    const int64_t waves = (int64_t)gridDim.x * wpw;
    // A wave takes `chunk` consecutive entries at a time (short runs: fewer
    // counter updates).
    const int64_t chunk = p.sched_chunk > 1 ? p.sched_chunk : 1;
    int64_t it;
    if (p.sched_mode == 0) {
        const int G = gridDim.x, xcd = blockIdx.x % kXcds, loc = blockIdx.x / kXcds;
        const int before = xcd * (G / kXcds) + min(xcd, G % kXcds);
        it = ((int64_t)(before + loc) * wpw + wave_id()) * chunk;
    } else {
        unsigned long long t = 0;
        if (lane_id() == 0) t = atomicAdd(p.next, (unsigned long long)chunk);
        it = (int64_t)__shfl(t, 0, kWave);
    }
    while (it < p.n_sched) {
        const int64_t end = min(it + chunk, p.n_sched);
        for (int64_t i = it; i < end; ++i) {
            const unsigned long long e = p.sched[i];
            const int64_t r = (int64_t)(e >> 16);
            const int m = (int)((e >> 8) & 255), n = (int)(e & 255);
            if (m > 16) {
                if (n > 16) sched_run<T, 2, 2, AT>(p, r, m, n);
                else sched_run<T, 2, 1, AT>(p, r, m, n);
            } else {
                if (n > 16) sched_run<T, 1, 2, AT>(p, r, m, n);
                else sched_run<T, 1, 1, AT>(p, r, m, n);
            }
        }
        if (p.sched_mode == 0) {
            it += waves * chunk;
        } else {
            unsigned long long t = 0;
            if (lane_id() == 0) t = atomicAdd(p.next, (unsigned long long)chunk);
            it = (int64_t)__shfl(t, 0, kWave);
        }
    }
}

template <class T>
__global__ __launch_bounds__(256, 4) void k_smm_mfma_sched(SmmArgs p) {
    sched_loop<T, false>(p);
}

// The scheduled launch reading A's blocks from their row-major copies.
template <class T>
__global__ __launch_bounds__(256, 4) void k_smm_mfma_sched_at(SmmArgs p) {
    sched_loop<T, true>(p);
}

// Row-major copies of A's blocks at the blocks' own offsets: one workgroup
// per block row, consecutive lanes write consecutive elements of a row.
template <class T>
__global__ __launch_bounds__(256) void k_transpose_blocks(int32_t nbr, const int64_t *rp, const int32_t *ci,
                                                          const int32_t *rbs, const int32_t *cbs,
                                                          const int64_t *blk_off, const T *src, T *dst) {
    for (int32_t r = blockIdx.x; r < nbr; r += gridDim.x) {
        const int m = rbs[r];
        for (int64_t p = rp[r]; p < rp[r + 1]; ++p) {
            const int k = cbs[ci[p]];
            const T *sb = src + blk_off[p];
            T *db = dst + blk_off[p];
            for (int e = threadIdx.x; e < m * k; e += blockDim.x) {
                const int i = e / k, j = e - i * k;
                db[e] = sb[(int64_t)j * m + i];
            }
        }
    }
}

__global__ void k_zero_u64(unsigned long long *p) { *p = 0ull; }

// Epilogue of split runs: C block of run r = beta C + alpha * (sum of its
// segments' partial blocks in segment order); one thread per element.
template <class T>
__global__ __launch_bounds__(256) void k_smm_split_reduce(SmmArgs p) {
    const int64_t mn = (int64_t)p.m * p.n;
    const int64_t total = (p.run_end - p.run_begin) * mn;
    const T *part = static_cast<const T *>(p.part);
    T *C = static_cast<T *>(p.C);
    const T alpha = (T)p.alpha, beta = (T)p.beta;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t rl = t / mn, e = t - rl * mn;
        const T *w = part + rl * p.split * mn + e;
        T v = w[0];
        for (int sg = 1; sg < p.split; ++sg) v += w[sg * mn];
        T *dst = C + p.run_coff[p.run_begin + rl] + e;
        const T prod = alpha * v;
        *dst = (beta == T(0)) ? prod : fma(beta, *dst, prod);
    }
}

using SmmKernel = void (*)(SmmArgs);

template <class T, int MT> SmmKernel pick_mfma_nt(int nt) {
    switch (nt) {
    case 1: return k_smm_mfma<T, MT, 1>;
    case 2: return k_smm_mfma<T, MT, 2>;
    case 3: return k_smm_mfma<T, MT, 3>;
    case 4: return k_smm_mfma<T, MT, 4>;
    default: return nullptr;
    }
}

// MFMA kernels for C blocks up to 64 x 64 (MT, NT in 1..4).
template <class T> SmmKernel mfma_kernel_for(int mt, int nt) {
    switch (mt) {
    case 1: return pick_mfma_nt<T, 1>(nt);
    case 2: return pick_mfma_nt<T, 2>(nt);
    case 3: return pick_mfma_nt<T, 3>(nt);
    case 4: return pick_mfma_nt<T, 4>(nt);
    default: return nullptr;
    }
}

// Register-tile shapes with a compiled kernel: TM, TN in {1,2,3,4,5,6,8}.
template <class T, int TM> SmmKernel pick_tn(int tn) {
    switch (tn) {
    case 1: return k_smm_valu<T, TM, 1>;
    case 2: return k_smm_valu<T, TM, 2>;
    case 3: return k_smm_valu<T, TM, 3>;
    case 4: return k_smm_valu<T, TM, 4>;
    case 5: return k_smm_valu<T, TM, 5>;
    case 6: return k_smm_valu<T, TM, 6>;
    case 8: return k_smm_valu<T, TM, 8>;
    default: return nullptr;
    }
}

template <class T> SmmKernel kernel_for(int tm, int tn) {
    switch (tm) {
    case 1: return pick_tn<T, 1>(tn);
    case 2: return pick_tn<T, 2>(tn);
    case 3: return pick_tn<T, 3>(tn);
    case 4: return pick_tn<T, 4>(tn);
    case 5: return pick_tn<T, 5>(tn);
    case 6: return pick_tn<T, 6>(tn);
    case 8: return pick_tn<T, 8>(tn);
    default: return nullptr;
    }
}

thread_local double *t_norm_sink = nullptr;

bool is_sched_kernel(const void *fn) {
    return fn == (const void *)k_smm_mfma_sched<double> || fn == (const void *)k_smm_mfma_sched<float> ||
           fn == (const void *)k_smm_mfma_sched_at<double> || fn == (const void *)k_smm_mfma_sched_at<float>;
}

constexpr int kLdsBudget = 64 * 1024;  // bytes of LDS per workgroup

}  // namespace

void set_norm_sink(double *norm2) { t_norm_sink = norm2; }
double *norm_sink() { return t_norm_sink; }


// Plain parameter rule: the smallest square register tile T (1..8) for
// which ceil(m/T) * ceil(n/T) <= 64 lanes (blocks above 64 use T = 8 and
// passes), the largest k chunk that fits, and as many waves per workgroup
// (up to 4) as 64 KB of LDS allow.
SmmParams plain_params(int m, int n) {
    int t = 8;
    for (int c = 1; c < 8; ++c)
        if (c != 7 && ceil_div(m, c) * ceil_div(n, c) <= kWave) {
            t = c;
            break;
        }
    return SmmParams{t, t, 0, 0};
}

int plan_smm(const SmmParams &prm, int m, int n, int kmax, int dtype, SmmLaunch *out) {
    const bool f32 = dtype == BSMM_F32;
    const size_t esize = f32 ? sizeof(float) : sizeof(double);
    out->dtype = dtype;
    if (prm.tm == kMfmaTile && prm.tn == kMfmaTile) {
        const int mt = (int)ceil_div(m, 16), nt = (int)ceil_div(n, 16);
        SmmKernel fn = f32 ? mfma_kernel_for<float>(mt, nt) : mfma_kernel_for<double>(mt, nt);
        if (!fn) {
            set_error(BSMM_ENOTSUP, "MFMA small-block kernel covers blocks up to 64 x 64, not %dx%d", m, n);
            return BSMM_ENOTSUP;
        }
        SmmArgs a{};
        a.m = m;
        a.n = n;
        a.tiles_m = mt;
        a.tiles_n = nt;
        a.L = kWave;
        a.G = 1;
        a.passes = 1;
        out->fn = (void *)fn;
        out->args = a;
        out->waves = prm.waves > 0 ? std::min(prm.waves, 4) : 4;
        out->lds = 0;
        return BSMM_OK;
    }
    const int TM = prm.tm, TN = prm.tn;
    SmmKernel fn = f32 ? kernel_for<float>(TM, TN) : kernel_for<double>(TM, TN);
    if (!fn) {
        set_error(BSMM_EINVAL, "no small-block kernel for register tile %dx%d", TM, TN);
        return BSMM_EINVAL;
    }
    SmmArgs a{};
    a.m = m;
    a.n = n;
    a.tiles_m = (int)ceil_div(m, TM);
    a.tiles_n = (int)ceil_div(n, TN);
    const int tiles = a.tiles_m * a.tiles_n;
    a.L = std::min(tiles, kWave);
    a.G = kWave / a.L;
    a.passes = (int)ceil_div(tiles, a.L);
    // LDS region per group: A chunk (m x kc) + B chunk (n_pad x kc) + slack
    // for the tail reads of the last register tile.
    const int n_pad = a.tiles_n * TN;
    const int waves_req = prm.waves > 0 ? std::min(prm.waves, 4) : 1;
    const int max_group_elems = (int)(kLdsBudget / esize / a.G / waves_req);
    int kc = (max_group_elems - TM - 3) / (m + n_pad);
    kc = std::min(kc, std::max(1, kmax));
    if (prm.kc > 0) kc = std::min(kc, prm.kc);
    if (kc < 1) {
        set_error(BSMM_ENOTSUP, "block shape %dx%d with tile %dx%d does not fit in LDS", m, n, TM, TN);
        return BSMM_ENOTSUP;
    }
    a.kc_max = kc;
    a.region = (m + n_pad) * kc + TM + 2;
    a.region = (a.region + 1) & ~1;
    const size_t wave_bytes = esize * (size_t)a.G * a.region;
    int waves = prm.waves > 0 ? waves_req
                              : (int)std::max<int64_t>(1, std::min<int64_t>(4, kLdsBudget / wave_bytes));
    if (wave_bytes * waves > (size_t)kLdsBudget) {
        set_error(BSMM_ENOTSUP, "small-block launch needs more than 64 KB of LDS");
        return BSMM_ENOTSUP;
    }
    out->fn = (void *)fn;
    out->args = a;
    out->waves = waves;
    out->lds = wave_bytes * waves;
    return BSMM_OK;
}

static unsigned split_reduce_grid(const SmmArgs &a) {
    return grid_of((a.run_end - a.run_begin) * (int64_t)a.m * a.n, 256, 8192);
}

unsigned smm_grid(const SmmLaunch &L, int64_t nruns) {
    const int64_t waves_needed = ceil_div(nruns * std::max(L.args.split, 1), L.args.G);
    // At most 32 waves per CU (256 CUs) in the grid, whatever the waves per
    // workgroup; the kernels stride over the remaining runs.
    const int64_t wg_cap = 256 * 32 / std::max(L.waves, 1);
    return grid_of(waves_needed, L.waves, wg_cap);
}

int launch_smm(SmmLaunch L, const void *A, const void *B, void *C, const int64_t *run_coff,
               const int64_t *run_ptr, const ulonglong2 *prods, int64_t rb, int64_t re,
               double alpha, double beta, hipStream_t s) {
    SmmArgs a = L.args;
    a.A = A;
    a.B = B;
    a.C = C;
    a.run_coff = run_coff;
    a.run_ptr = run_ptr;
    a.prods = prods;
    a.run_begin = rb;
    a.run_end = re;
    a.alpha = alpha;
    a.beta = beta;
    if (L.jit_fn)
        return launch_jit_smm(L.jit_fn, smm_grid(L, re - rb), L.waves, A, B, C, run_coff, run_ptr, prods,
                              rb, re, alpha, beta, s);
    if (is_sched_kernel(L.fn) && a.sched_mode == 1) {
        hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, s, a.next);
        BSMM_TRY(launch_check("zero_u64"));
    }
    {
        KernelTimer kt(1, s);
        hipLaunchKernelGGL((SmmKernel)L.fn, dim3(smm_grid(L, re - rb)), dim3(64 * L.waves), L.lds, s,
                           a);
    }
    BSMM_TRY(launch_check("smm_valu"));
    if (a.split <= 1) return BSMM_OK;
    if (L.dtype == BSMM_F32)
        hipLaunchKernelGGL(k_smm_split_reduce<float>, dim3(split_reduce_grid(a)), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(k_smm_split_reduce<double>, dim3(split_reduce_grid(a)), dim3(256), 0, s, a);
    return launch_check("smm_split_reduce");
}

// Average products per run of every class (tuned path: the run length is
// part of the parameter lookup), from the per-class run and product counts
// the stack builder read back.
static void class_run_lengths(const Stacks &st, std::vector<int> *out) {
    out->assign(st.n_classes, 1);
    if ((int)st.class_prod_begin.size() != st.n_classes + 1) return;
    for (int cl = 0; cl < st.n_classes; ++cl) {
        const int64_t runs = st.class_begin[cl + 1] - st.class_begin[cl];
        const int64_t prods = st.class_prod_begin[cl + 1] - st.class_prod_begin[cl];
        if (runs > 0) (*out)[cl] = (int)std::max<int64_t>(1, (prods + runs / 2) / runs);
    }
}

// The k under which tuned parameters are looked up: a run mixes the k of
// A's block columns, and a product's work grows with k, so the key is the
// block-column size k carrying the most work (count of columns of size k,
// times k; ties: the smaller k).
static int representative_k(const bsmm_matrix_s *A) {
    std::vector<int32_t> v = A->cbs;
    if (v.empty()) return 1;
    std::sort(v.begin(), v.end());
    int best = v[0];
    int64_t bestw = 0;
    for (size_t i = 0; i < v.size();) {
        size_t j = i;
        while (j < v.size() && v[j] == v[i]) ++j;
        const int64_t w = (int64_t)(j - i) * v[i];
        if (w > bestw) {
            bestw = w;
            best = v[i];
        }
        i = j;
    }
    return best;
}

// Segments per run for a class of `runs` runs holding `prods` products on
// the one-wave-per-run MFMA kernel: enough (run, segment) items for about
// 16 waves per CU when the runs alone are fewer, each segment at least 16
// products long, at most 64 segments and 1 GiB of partial blocks.
static int split_for(int64_t runs, int64_t prods, int m, int n, size_t esize) {
    const int64_t target = (int64_t)cu_count() * 16;
    if (runs <= 0 || runs >= target) return 1;
    int64_t S = ceil_div(target, runs);
    S = std::min<int64_t>(S, prods / runs / 16);
    S = std::min<int64_t>(S, 64);
    S = std::min<int64_t>(S, (int64_t(1) << 30) / (runs * (int64_t)m * n * (int64_t)esize));
    return (int)std::max<int64_t>(S, 1);
}

// Row-major copies of A's blocks into st.a_t (the A data of this call: a
// replayed plan copies again, since A's values may have changed).
static int transpose_a(const bsmm_matrix_s *A, const Stacks &st, hipStream_t s) {
    BSMM_TRY(const_cast<DevBuf &>(st.a_t).reserve(A->esize() * (size_t)(A->storage + 1), s));
    if (A->nnzb == 0) return BSMM_OK;
    if (A->dtype == BSMM_F32)
        hipLaunchKernelGGL(k_transpose_blocks<float>, dim3(grid_rows(A->nbr)), dim3(256), 0, s, A->nbr,
                           A->d_row_ptr(), A->d_col_ind(), A->d_rbs(), A->d_cbs(), A->d_blk_off(),
                           (const float *)A->d_raw(), st.a_t.as<float>());
    else
        hipLaunchKernelGGL(k_transpose_blocks<double>, dim3(grid_rows(A->nbr)), dim3(256), 0, s, A->nbr,
                           A->d_row_ptr(), A->d_col_ind(), A->d_rbs(), A->d_cbs(), A->d_blk_off(),
                           (const double *)A->d_raw(), st.a_t.as<double>());
    return launch_check("transpose_blocks");
}

int run_stacks(const bsmm_matrix_s *A, const bsmm_matrix_s *B, bsmm_matrix_s *C, Stacks &st,
               double alpha, double beta, hipStream_t s, StackExec *ex) {
    ex->launches.clear();
    ex->parts.clear();
    st.n_sched = 0;
    st.n_jit = 0;
    if (st.n_runs == 0) return BSMM_OK;
    const int kmax = std::max(1, A->max_cbs);
    const int64_t chunk = options().stack_chunk;
    const bool tuned = options().stack_kernel == 1;
    const int krep = representative_k(A);
    // Every product has the same depth when A's block columns share one size.
    const int uniform_k = !A->cbs.empty() &&
                                  *std::min_element(A->cbs.begin(), A->cbs.end()) == A->max_cbs
                              ? A->max_cbs
                              : 0;
    std::vector<int64_t> run_ptr_h;
    if (chunk > 0) {
        run_ptr_h.resize(st.n_runs + 1);
        BSMM_HIP(hipMemcpyAsync(run_ptr_h.data(), st.run_ptr.p, sizeof(int64_t) * (st.n_runs + 1),
                                hipMemcpyDeviceToHost, s));
        BSMM_HIP(hipStreamSynchronize(s));
    }
    std::vector<int> rlen;
    if (tuned) {
        // Row panels share the whole multiply's run lengths, so every panel
        // picks the same parameters as one whole stack would.
        if ((int)st.run_len_hint.size() == st.n_classes) rlen = st.run_len_hint;
        else class_run_lengths(st, &rlen);
    }
    LaunchList &launches = ex->launches;
    // Tuned path with a tile size: the MFMA classes of blocks up to 32 x 32
    // whose runs need no splitting go to one scheduled launch.
    const bool sched_on = tuned && chunk <= 0 && options().stack_tile > 0 &&
                          (int)st.class_prod_begin.size() == st.n_classes + 1;
    std::vector<char> eligible(st.n_classes, 0);
    for (int cl = 0; cl < st.n_classes; ++cl) {
        const int64_t rb = st.class_begin[cl], re = st.class_begin[cl + 1];
        if (re <= rb) continue;
        const int m = st.row_sizes[cl / st.ncs], n = st.col_sizes[cl % st.ncs];
        SmmParams prm = tuned ? select_params(m, n, krep, rlen[cl]) : plain_params(m, n);
        SmmLaunch L;
        BSMM_TRY(plan_smm(prm, m, n, kmax, C->dtype, &L));
        if (chunk <= 0 && prm.tm == kMfmaTile && (int)st.class_prod_begin.size() == st.n_classes + 1) {
            const int S = split_for(re - rb, st.class_prod_begin[cl + 1] - st.class_prod_begin[cl], m, n,
                                    C->esize());
            if (tuned && options().jit && S == 1 && uniform_k > 0) {
                // One product depth: a kernel compiled for this (m, n, k).
                if (hipFunction_t f = jit_smm_kernel(C->dtype, m, n, uniform_k)) {
                    L.jit_fn = f;
                    launches.push_back({L, {rb, re}});
                    ++st.n_jit;
                    continue;
                }
            }
            if (sched_on && S == 1 && m <= 32 && n <= 32) {
                eligible[cl] = 1;
                continue;
            }
            if (S > 1) {
                DevBuf part;
                BSMM_TRY(part.reserve(C->esize() * (size_t)(re - rb) * S * m * n, s));
                L.args.split = S;
                L.args.part = part.as<double>();
                ex->parts.push_back(std::move(part));
            }
        }
        if (chunk <= 0) {
            launches.push_back({L, {rb, re}});
            continue;
        }
        // Batches of at most `chunk` products; a run is never split.
        int64_t b0 = rb;
        while (b0 < re) {
            int64_t b1 = b0 + 1;
            while (b1 < re && run_ptr_h[b1 + 1] - run_ptr_h[b0] <= chunk) ++b1;
            launches.push_back({L, {b0, b1}});
            b0 = b1;
        }
    }
    int64_t sched_runs = 0, sched_prods = 0;
    for (int cl = 0; cl < st.n_classes; ++cl)
        if (eligible[cl]) {
            sched_runs += st.class_begin[cl + 1] - st.class_begin[cl];
            sched_prods += st.class_prod_begin[cl + 1] - st.class_prod_begin[cl];
        }
    if (sched_on && sched_runs > 0 && sched_runs < kSchedMinRuns) {
        // Too few runs for the scheduling passes to pay off: those classes
        // take their own launches after all.
        for (int cl = 0; cl < st.n_classes; ++cl) {
            if (!eligible[cl]) continue;
            const int m = st.row_sizes[cl / st.ncs], n = st.col_sizes[cl % st.ncs];
            SmmLaunch L;
            BSMM_TRY(plan_smm(select_params(m, n, krep, rlen[cl]), m, n, kmax, C->dtype, &L));
            launches.push_back({L, {st.class_begin[cl], st.class_begin[cl + 1]}});
            eligible[cl] = 0;
        }
        sched_runs = 0;
    }
    if (sched_on && sched_runs > 0) {
        BSMM_TRY(build_schedule(C, st, eligible, options().stack_tile, s));
        SmmLaunch L;
        // FP32 loads are instruction-bound: A's blocks are read from
        // row-major copies (one 16-byte load for four k values instead of
        // four 4-byte loads; banded 10 % FP32 kernel 54.5 -> 51.8 ms).  FP64
        // is bound by the fabric, where the copies' strided rows coalesce
        // worse (headline kernel 669 -> 718 ms), so it reads A in place.
        const int at_opt = options().stack_at;
        // (Not with a scratch arena: the copy is as large as A.)
        const bool at = (at_opt == 1 || (at_opt < 0 && C->dtype == BSMM_F32)) && !scratch_arena();
        if (at && !st.a_t_fresh) {
            BSMM_TRY(transpose_a(A, st, s));
            st.a_t_fresh = true;
        }
        ex->reads_a_t = at;
        if (C->dtype == BSMM_F32)
            L.fn = at ? (void *)k_smm_mfma_sched_at<float> : (void *)k_smm_mfma_sched<float>;
        else
            L.fn = at ? (void *)k_smm_mfma_sched_at<double> : (void *)k_smm_mfma_sched<double>;
        L.args.A_t = at ? st.a_t.p : nullptr;
        L.dtype = C->dtype;
        L.args.L = kWave;
        L.args.G = 1;
        L.args.passes = 1;
        L.args.sched = st.sched.as<unsigned long long>();
        L.args.n_sched = st.n_sched;
        L.args.next = st.sched_next.as<unsigned long long>();
        L.args.sched_mode = options().stack_sched;
        L.args.norm2 = norm_sink();
        L.args.run_cblk = st.run_cblk.as<int64_t>();
        // About 32 products per counter update: runs of one product go
        // 16 at a time, runs of 32 or more one at a time.
        const int64_t mean_len = std::max<int64_t>(1, sched_prods / sched_runs);
        L.args.sched_chunk = (int)std::min<int64_t>(16, std::max<int64_t>(1, 32 / mean_len));
        L.waves = 4;
        L.lds = 0;
        launches.push_back({L, {0, st.n_sched}});
    }
    // Instantiating a graph may allocate device memory: a multiply running
    // on a scratch arena launches its classes one by one instead, and so
    // does one with run-time compiled kernels (module functions, which a
    // graph kernel node does not take).
    if (tuned && chunk <= 0 && launches.size() > 1 && !scratch_arena() && st.n_jit == 0) {
        BSMM_TRY(build_graph(launches, A, B, C, st, alpha, beta, &ex->exec));
        BSMM_HIP(hipEventCreateWithFlags(&ex->done, hipEventDisableTiming));
    }
    return replay_stacks(*ex, A, B, C, st, alpha, beta, s);
}

namespace {
std::mutex g_retire_mu;
std::vector<std::pair<hipGraphExec_t, hipEvent_t>> g_retired;

// Destroys the retired graphs whose last launch has completed.
void reap_retired_locked() {
    std::vector<std::pair<hipGraphExec_t, hipEvent_t>> keep;
    for (auto &r : g_retired) {
        const hipError_t q = r.second ? hipEventQuery(r.second) : hipSuccess;
        if (q == hipErrorNotReady) {
            if (hipPeekAtLastError() == hipErrorNotReady) (void)hipGetLastError();
            keep.push_back(r);
            continue;
        }
        (void)hipGraphExecDestroy(r.first);
        if (r.second) (void)hipEventDestroy(r.second);
    }
    g_retired.swap(keep);
}
}  // namespace

void retire_graph(hipGraphExec_t exec, hipEvent_t done) {
    std::lock_guard<std::mutex> lk(g_retire_mu);
    g_retired.push_back({exec, done});
    reap_retired_locked();
    // Bounded backlog: wait for the oldest retired graph when many are pending.
    while (g_retired.size() > 64) {
        if (g_retired.front().second) (void)hipEventSynchronize(g_retired.front().second);
        reap_retired_locked();
    }
}

int replay_stacks(const StackExec &ex, const bsmm_matrix_s *A, const bsmm_matrix_s *B,
                  bsmm_matrix_s *C, const Stacks &st, double alpha, double beta, hipStream_t s) {
    // Same buffer (the launches hold its address), this call's A values.
    if (ex.reads_a_t) BSMM_TRY(transpose_a(A, st, s));
    if (ex.exec) {
        {
            KernelTimer kt(1, s);
            BSMM_HIP(hipGraphLaunch(ex.exec, s));
        }
        if (ex.done) BSMM_HIP(hipEventRecord(ex.done, s));
        return BSMM_OK;
    }
    for (auto &l : ex.launches)
        BSMM_TRY(launch_smm(l.first, A->d_raw(), B->d_raw(), C->d_raw(),
                            st.run_coff.as<int64_t>(), st.run_ptr.as<int64_t>(),
                            st.prods.as<ulonglong2>(), l.second.first, l.second.second, alpha, beta,
                            s));
    return BSMM_OK;
}

// Tuned path: all shape classes as independent kernel nodes of one hipGraph
// (launched once, classes run concurrently).  The kernel arguments are
// copied into the graph when the nodes are added.
int build_graph(const LaunchList &launches, const bsmm_matrix_s *A, const bsmm_matrix_s *B,
                bsmm_matrix_s *C, const Stacks &st, double alpha, double beta,
                hipGraphExec_t *out) {
    hipGraph_t graph = nullptr;
    BSMM_HIP(hipGraphCreate(&graph, 0));
    int status = BSMM_OK;
    for (size_t i = 0; i < launches.size() && status == BSMM_OK; ++i) {
        const SmmLaunch &L = launches[i].first;
        SmmArgs a = L.args;
        a.A = A->d_raw();
        a.B = B->d_raw();
        a.C = C->d_raw();
        a.run_coff = st.run_coff.as<int64_t>();
        a.run_ptr = st.run_ptr.as<int64_t>();
        a.prods = st.prods.as<ulonglong2>();
        a.run_begin = launches[i].second.first;
        a.run_end = launches[i].second.second;
        a.alpha = alpha;
        a.beta = beta;
        void *argp = &a;
        hipKernelNodeParams kp{};
        kp.func = L.fn;
        kp.gridDim = dim3(smm_grid(L, a.run_end - a.run_begin));
        kp.blockDim = dim3(64 * L.waves);
        kp.sharedMemBytes = (unsigned)L.lds;
        kp.kernelParams = &argp;
        kp.extra = nullptr;
        hipGraphNode_t node, zero;
        const bool counter = is_sched_kernel(L.fn) && a.sched_mode == 1;
        void *zargp = &a.next;
        if (counter) {
            // The dynamic schedule's run counter starts at zero every replay
            // (a kernel node: memset nodes are not used in the graph).
            hipKernelNodeParams zp{};
            zp.func = (void *)k_zero_u64;
            zp.gridDim = dim3(1);
            zp.blockDim = dim3(1);
            zp.sharedMemBytes = 0;
            zp.kernelParams = &zargp;
            zp.extra = nullptr;
            if (hipGraphAddKernelNode(&zero, graph, nullptr, 0, &zp) != hipSuccess) {
                set_error(BSMM_EDEVICE, "hipGraphAddKernelNode failed");
                status = BSMM_EDEVICE;
                break;
            }
        }
        if (hipGraphAddKernelNode(&node, graph, counter ? &zero : nullptr, counter ? 1 : 0, &kp) !=
            hipSuccess) {
            set_error(BSMM_EDEVICE, "hipGraphAddKernelNode failed");
            status = BSMM_EDEVICE;
        } else if (a.split > 1) {
            // The class's split-run epilogue runs after its kernel.
            hipKernelNodeParams rp{};
            rp.func = L.dtype == BSMM_F32 ? (void *)k_smm_split_reduce<float>
                                          : (void *)k_smm_split_reduce<double>;
            rp.gridDim = dim3(split_reduce_grid(a));
            rp.blockDim = dim3(256);
            rp.sharedMemBytes = 0;
            rp.kernelParams = &argp;
            rp.extra = nullptr;
            hipGraphNode_t rnode;
            if (hipGraphAddKernelNode(&rnode, graph, &node, 1, &rp) != hipSuccess) {
                set_error(BSMM_EDEVICE, "hipGraphAddKernelNode failed");
                status = BSMM_EDEVICE;
            }
        }
    }
    if (status == BSMM_OK && hipGraphInstantiate(out, graph, nullptr, nullptr, 0) != hipSuccess) {
        set_error(BSMM_EDEVICE, "hipGraphInstantiate failed");
        *out = nullptr;
        status = BSMM_EDEVICE;
    }
    (void)hipGraphDestroy(graph);
    (void)hipGetLastError();
    return status;
}

}  // namespace bsmm
