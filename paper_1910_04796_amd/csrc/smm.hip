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
//    one wavefront are covered in passes.
//
// The epilogue applies C = beta*C + alpha*acc (beta == 0 overwrites).
#include <algorithm>

#include "dev_util.h"
#include "internal.h"

namespace bsmm {

namespace {

struct SmmArgs {
    const double *A;
    const double *B;
    double *C;
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
};

template <int TM, int TN>
__global__ __launch_bounds__(256) void k_smm_valu(SmmArgs p) {
    extern __shared__ double lds[];
    const int lane = lane_id();
    const int g = lane / p.L;
    const int gl = lane - g * p.L;
    const bool in_group = g < p.G;
    double *reg = lds + (size_t)(wave_id() * p.G + (in_group ? g : 0)) * p.region;
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
            double acc[TM][TN];
#pragma unroll
            for (int a = 0; a < TM; ++a)
#pragma unroll
                for (int b = 0; b < TN; ++b) acc[a][b] = 0.0;

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
                        const double *ga = p.A + a_off + (int64_t)m * kc0;
                        const int na = m * kc;
                        for (int e = gl; e < na; e += p.L) reg[e] = ga[e];
                        double *rbuf = reg + na;
                        const double *gb = p.B + b_off + kc0;
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
                        const double *As = reg + i0;
                        const double *Bs = reg + m * kc + (int64_t)j0 * kc;
                        for (int kk = 0; kk < kc; ++kk) {
                            double av[TM], bv[TN];
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
                double *c = p.C + p.run_coff[r];
#pragma unroll
                for (int b = 0; b < TN; ++b) {
                    const int j = j0 + b;
                    if (j >= n) break;
#pragma unroll
                    for (int a = 0; a < TM; ++a) {
                        const int i = i0 + a;
                        if (i < m) {
                            double *dst = c + (int64_t)j * m + i;
                            const double prod = p.alpha * acc[a][b];
                            *dst = (p.beta == 0.0) ? prod : fma(p.beta, *dst, prod);
                        }
                    }
                }
            }
        }
    }
}

using SmmKernel = void (*)(SmmArgs);

template <int T> SmmKernel pick_square() { return k_smm_valu<T, T>; }

SmmKernel kernel_for(int tm) {
    switch (tm) {
    case 1: return pick_square<1>();
    case 2: return pick_square<2>();
    case 3: return pick_square<3>();
    case 4: return pick_square<4>();
    case 5: return pick_square<5>();
    case 6: return pick_square<6>();
    case 7: return pick_square<7>();
    default: return pick_square<8>();
    }
}

constexpr int kLdsBudget = 64 * 1024;  // bytes of LDS per workgroup

}  // namespace

// Plain parameter rule: the smallest square register tile T (1..8) for
// which ceil(m/T) * ceil(n/T) <= 64 lanes; blocks above 64 use T = 8 and
// passes.
static int plain_tile(int m, int n) {
    for (int t = 1; t < 8; ++t)
        if (ceil_div(m, t) * ceil_div(n, t) <= kWave) return t;
    return 8;
}

static int launch_class(const bsmm_matrix_s *A, const bsmm_matrix_s *B, bsmm_matrix_s *C,
                        const Stacks &st, int cl, int64_t rb, int64_t re, int kmax, double alpha,
                        double beta, hipStream_t s) {
    SmmArgs a{};
    a.A = A->d_data();
    a.B = B->d_data();
    a.C = C->d_data();
    a.run_coff = st.run_coff.as<int64_t>();
    a.run_ptr = st.run_ptr.as<int64_t>();
    a.prods = st.prods.as<ulonglong2>();
    a.run_begin = rb;
    a.run_end = re;
    a.m = st.row_sizes[cl / st.ncs];
    a.n = st.col_sizes[cl % st.ncs];
    const int T = plain_tile(a.m, a.n);
    a.tiles_m = (int)ceil_div(a.m, T);
    a.tiles_n = (int)ceil_div(a.n, T);
    const int tiles = a.tiles_m * a.tiles_n;
    a.L = std::min(tiles, kWave);
    a.G = kWave / a.L;
    a.passes = (int)ceil_div(tiles, a.L);
    // LDS region per group: A chunk (m x kc) + B chunk (n_pad x kc) + slack
    // for the tail reads of the last register tile.
    const int n_pad = a.tiles_n * T;
    const int max_group_doubles = kLdsBudget / 8 / a.G;
    int kc = std::min(kmax, (max_group_doubles - T - 3) / (a.m + n_pad));
    if (kc < 1) {
        set_error(BSMM_ENOTSUP, "block shape %dx%d too large for the small-block kernel", a.m, a.n);
        return BSMM_ENOTSUP;
    }
    a.kc_max = kc;
    a.region = (a.m + n_pad) * kc + T + 2;
    a.region = (a.region + 1) & ~1;
    a.alpha = alpha;
    a.beta = beta;
    const int64_t per_wave = a.G;
    const int64_t nruns = re - rb;
    const size_t wave_bytes = sizeof(double) * (size_t)a.G * a.region;
    int waves_per_wg = (int)std::max<int64_t>(1, std::min<int64_t>(4, kLdsBudget / wave_bytes));
    const int64_t waves_needed = ceil_div(nruns, per_wave);
    const int64_t wg_cap = 256 * 8;  // enough resident work for 256 CUs
    const unsigned grid = grid_of(waves_needed, waves_per_wg, wg_cap);
    KernelTimer kt(1, s);
    hipLaunchKernelGGL(kernel_for(T), dim3(grid), dim3(64 * waves_per_wg),
                       wave_bytes * waves_per_wg, s, a);
    return launch_check("smm_valu");
}

int run_stacks(const bsmm_matrix_s *A, const bsmm_matrix_s *B, bsmm_matrix_s *C,
               const Stacks &st, double alpha, double beta, hipStream_t s) {
    if (st.n_runs == 0) return BSMM_OK;
    const int kmax = std::max(1, A->max_cbs);
    const int64_t chunk = options().stack_chunk;
    std::vector<int64_t> run_ptr_h;
    if (chunk > 0) {
        run_ptr_h.resize(st.n_runs + 1);
        BSMM_HIP(hipMemcpyAsync(run_ptr_h.data(), st.run_ptr.p, sizeof(int64_t) * (st.n_runs + 1),
                                hipMemcpyDeviceToHost, s));
        BSMM_HIP(hipStreamSynchronize(s));
    }
    for (int cl = 0; cl < st.n_classes; ++cl) {
        const int64_t rb = st.class_begin[cl], re = st.class_begin[cl + 1];
        if (re <= rb) continue;
        if (chunk <= 0) {
            BSMM_TRY(launch_class(A, B, C, st, cl, rb, re, kmax, alpha, beta, s));
            continue;
        }
        // Batches of at most `chunk` products; a run is never split.
        int64_t b0 = rb;
        while (b0 < re) {
            int64_t b1 = b0 + 1;
            while (b1 < re && run_ptr_h[b1 + 1] - run_ptr_h[b0] <= chunk) ++b1;
            BSMM_TRY(launch_class(A, B, C, st, cl, b0, b1, kmax, alpha, beta, s));
            b0 = b1;
        }
    }
    return BSMM_OK;
}

}  // namespace bsmm
