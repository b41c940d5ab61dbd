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

namespace bsmm {

namespace {

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

// FP64 MFMA variant for blocks of at least about 16 x 16 (parameter set
// tm = tn = 16): one wave owns one run at a time and keeps the C block as
// MT x NT tiles of v_mfma_f64_16x16x4 accumulators (m <= 16 MT, n <= 16 NT).
// Operands come straight from the contiguous A and B blocks (each product's
// blocks are a few KB and stay in L1/L2), zero outside the block, so 23- or
// 13-sized blocks are padded in registers only.
// Result element e of lane l is row 4 e + l / 16, column l % 16 of a tile.
typedef double v4d_t __attribute__((ext_vector_type(4)));
typedef double v2d_t __attribute__((ext_vector_type(2)));

template <int MT, int NT>
__global__ __launch_bounds__(256) void k_smm_mfma(SmmArgs p) {
    const int lane = lane_id();
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
    const int64_t wid = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave_id();
    const int m = p.m, n = p.n;
    const int lr = lane & 15, lk = lane >> 4;
    const int S = p.split > 1 ? p.split : 1;
    const int64_t items = (p.run_end - p.run_begin) * S;
    for (int64_t it = wid; it < items; it += waves) {
        // Item = (run, segment): segment sg of S takes products
        // [len sg / S, len (sg + 1) / S) of the run.
        const int64_t r = p.run_begin + it / S;
        const int sg = (int)(it % S);
        const int64_t rq0 = p.run_ptr[r], len = p.run_ptr[r + 1] - rq0;
        const int64_t q0 = rq0 + len * sg / S, q1 = rq0 + len * (sg + 1) / S;
        v4d_t acc[MT][NT];
#pragma unroll
        for (int i = 0; i < MT; ++i)
#pragma unroll
            for (int j = 0; j < NT; ++j) acc[i][j] = (v4d_t){0.0, 0.0, 0.0, 0.0};
        // The next product's descriptor is loaded one product ahead.
        ulonglong2 nxt = q0 < q1 ? p.prods[q0] : make_ulonglong2(0ull, 0ull);
        for (int64_t q = q0; q < q1; ++q) {
            const ulonglong2 pr = nxt;
            if (q + 1 < q1) nxt = p.prods[q + 1];
            const double *a = p.A + (int64_t)(pr.x & ((1ull << 48) - 1));
            const int k = (int)(pr.x >> 48);
            const double *b = p.B + (int64_t)pr.y;
            for (int k0 = 0; k0 < k; k0 += 16) {
                // Four k steps of fragments, then their MFMAs.  Lane group
                // g = l / 16 supplies k = k0 + 4 g + s to step s (any
                // assignment of k to steps is valid when A and B agree), so a
                // lane's B operands are four consecutive doubles of a column.
                double af[4][MT], bf[4][NT];
                const int kb = k0 + 4 * lk;
#pragma unroll
                for (int i = 0; i < MT; ++i) {
                    const int row = 16 * i + lr;
#pragma unroll
                    for (int s = 0; s < 4; ++s)
                        af[s][i] = (row < m && kb + s < k) ? a[(int64_t)(kb + s) * m + row] : 0.0;
                }
#pragma unroll
                for (int j = 0; j < NT; ++j) {
                    const int col = 16 * j + lr;
                    const double *bc = b + (int64_t)col * k + kb;
                    if (col < n && kb + 3 < k) {
                        // 16-byte loads at 8-byte alignment (dword alignment
                        // is all the vector loads need).
                        v2d_t lo, hi;
                        __builtin_memcpy(&lo, bc, sizeof lo);
                        __builtin_memcpy(&hi, bc + 2, sizeof hi);
                        bf[0][j] = lo[0];
                        bf[1][j] = lo[1];
                        bf[2][j] = hi[0];
                        bf[3][j] = hi[1];
                    } else {
#pragma unroll
                        for (int s = 0; s < 4; ++s) bf[s][j] = (col < n && kb + s < k) ? bc[s] : 0.0;
                    }
                }
#pragma unroll
                for (int s = 0; s < 4; ++s)
#pragma unroll
                    for (int i = 0; i < MT; ++i)
#pragma unroll
                        for (int j = 0; j < NT; ++j)
                            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[s][i], bf[s][j], acc[i][j],
                                                                             0, 0, 0);
            }
        }
        if (S > 1) {
            double *w = p.part + it * (int64_t)m * n;
#pragma unroll
            for (int i = 0; i < MT; ++i)
#pragma unroll
                for (int j = 0; j < NT; ++j)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int row = 16 * i + 4 * e + lk, col = 16 * j + lr;
                        if (row < m && col < n) w[(int64_t)col * m + row] = acc[i][j][e];
                    }
            continue;
        }
        double *c = p.C + p.run_coff[r];
#pragma unroll
        for (int i = 0; i < MT; ++i)
#pragma unroll
            for (int j = 0; j < NT; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int row = 16 * i + 4 * e + lk, col = 16 * j + lr;
                    if (row < m && col < n) {
                        double *dst = c + (int64_t)col * m + row;
                        const double prod = p.alpha * acc[i][j][e];
                        *dst = (p.beta == 0.0) ? prod : fma(p.beta, *dst, prod);
                    }
                }
    }
}

// Epilogue of split runs: C block of run r = beta C + alpha * (sum of its
// segments' partial blocks in segment order); one thread per element.
__global__ __launch_bounds__(256) void k_smm_split_reduce(SmmArgs p) {
    const int64_t mn = (int64_t)p.m * p.n;
    const int64_t total = (p.run_end - p.run_begin) * mn;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t rl = t / mn, e = t - rl * mn;
        const double *w = p.part + rl * p.split * mn + e;
        double v = w[0];
        for (int sg = 1; sg < p.split; ++sg) v += w[sg * mn];
        double *dst = p.C + p.run_coff[p.run_begin + rl] + e;
        const double prod = p.alpha * v;
        *dst = (p.beta == 0.0) ? prod : fma(p.beta, *dst, prod);
    }
}

using SmmKernel = void (*)(SmmArgs);

template <int MT> SmmKernel pick_mfma_nt(int nt) {
    switch (nt) {
    case 1: return k_smm_mfma<MT, 1>;
    case 2: return k_smm_mfma<MT, 2>;
    case 3: return k_smm_mfma<MT, 3>;
    case 4: return k_smm_mfma<MT, 4>;
    default: return nullptr;
    }
}

// MFMA kernels for C blocks up to 64 x 64 (MT, NT in 1..4).
SmmKernel mfma_kernel_for(int mt, int nt) {
    switch (mt) {
    case 1: return pick_mfma_nt<1>(nt);
    case 2: return pick_mfma_nt<2>(nt);
    case 3: return pick_mfma_nt<3>(nt);
    case 4: return pick_mfma_nt<4>(nt);
    default: return nullptr;
    }
}

// Register-tile shapes with a compiled kernel: TM, TN in {1,2,3,4,5,6,8}.
template <int TM> SmmKernel pick_tn(int tn) {
    switch (tn) {
    case 1: return k_smm_valu<TM, 1>;
    case 2: return k_smm_valu<TM, 2>;
    case 3: return k_smm_valu<TM, 3>;
    case 4: return k_smm_valu<TM, 4>;
    case 5: return k_smm_valu<TM, 5>;
    case 6: return k_smm_valu<TM, 6>;
    case 8: return k_smm_valu<TM, 8>;
    default: return nullptr;
    }
}

SmmKernel kernel_for(int tm, int tn) {
    switch (tm) {
    case 1: return pick_tn<1>(tn);
    case 2: return pick_tn<2>(tn);
    case 3: return pick_tn<3>(tn);
    case 4: return pick_tn<4>(tn);
    case 5: return pick_tn<5>(tn);
    case 6: return pick_tn<6>(tn);
    case 8: return pick_tn<8>(tn);
    default: return nullptr;
    }
}

constexpr int kLdsBudget = 64 * 1024;  // bytes of LDS per workgroup

}  // namespace

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

int plan_smm(const SmmParams &prm, int m, int n, int kmax, SmmLaunch *out) {
    if (prm.tm == kMfmaTile && prm.tn == kMfmaTile) {
        const int mt = (int)ceil_div(m, 16), nt = (int)ceil_div(n, 16);
        SmmKernel fn = mfma_kernel_for(mt, nt);
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
    SmmKernel fn = kernel_for(TM, TN);
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
    const int max_group_doubles = kLdsBudget / 8 / a.G / waves_req;
    int kc = (max_group_doubles - TM - 3) / (m + n_pad);
    kc = std::min(kc, std::max(1, kmax));
    if (prm.kc > 0) kc = std::min(kc, prm.kc);
    if (kc < 1) {
        set_error(BSMM_ENOTSUP, "block shape %dx%d with tile %dx%d does not fit in LDS", m, n, TM, TN);
        return BSMM_ENOTSUP;
    }
    a.kc_max = kc;
    a.region = (m + n_pad) * kc + TM + 2;
    a.region = (a.region + 1) & ~1;
    const size_t wave_bytes = sizeof(double) * (size_t)a.G * a.region;
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

int launch_smm(SmmLaunch L, const double *A, const double *B, double *C, const int64_t *run_coff,
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
    {
        KernelTimer kt(1, s);
        hipLaunchKernelGGL((SmmKernel)L.fn, dim3(smm_grid(L, re - rb)), dim3(64 * L.waves), L.lds, s,
                           a);
    }
    BSMM_TRY(launch_check("smm_valu"));
    if (a.split <= 1) return BSMM_OK;
    hipLaunchKernelGGL(k_smm_split_reduce, dim3(split_reduce_grid(a)), dim3(256), 0, s, a);
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
static int split_for(int64_t runs, int64_t prods, int m, int n) {
    const int64_t target = (int64_t)cu_count() * 16;
    if (runs <= 0 || runs >= target) return 1;
    int64_t S = ceil_div(target, runs);
    S = std::min<int64_t>(S, prods / runs / 16);
    S = std::min<int64_t>(S, 64);
    S = std::min<int64_t>(S, (int64_t(1) << 30) / (runs * (int64_t)m * n * (int64_t)sizeof(double)));
    return (int)std::max<int64_t>(S, 1);
}

int run_stacks(const bsmm_matrix_s *A, const bsmm_matrix_s *B, bsmm_matrix_s *C,
               const Stacks &st, double alpha, double beta, hipStream_t s, StackExec *ex) {
    ex->launches.clear();
    ex->parts.clear();
    if (st.n_runs == 0) return BSMM_OK;
    const int kmax = std::max(1, A->max_cbs);
    const int64_t chunk = options().stack_chunk;
    const bool tuned = options().stack_kernel == 1;
    const int krep = representative_k(A);
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
    for (int cl = 0; cl < st.n_classes; ++cl) {
        const int64_t rb = st.class_begin[cl], re = st.class_begin[cl + 1];
        if (re <= rb) continue;
        const int m = st.row_sizes[cl / st.ncs], n = st.col_sizes[cl % st.ncs];
        SmmParams prm = tuned ? select_params(m, n, krep, rlen[cl]) : plain_params(m, n);
        SmmLaunch L;
        BSMM_TRY(plan_smm(prm, m, n, kmax, &L));
        if (chunk <= 0 && prm.tm == kMfmaTile && (int)st.class_prod_begin.size() == st.n_classes + 1) {
            const int S = split_for(re - rb, st.class_prod_begin[cl + 1] - st.class_prod_begin[cl], m, n);
            if (S > 1) {
                DevBuf part;
                BSMM_TRY(part.reserve(sizeof(double) * (size_t)(re - rb) * S * m * n, s));
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
    // Instantiating a graph may allocate device memory: a multiply running
    // on a scratch arena launches its classes one by one instead.
    if (tuned && chunk <= 0 && launches.size() > 1 && !scratch_arena()) {
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
    if (ex.exec) {
        {
            KernelTimer kt(1, s);
            BSMM_HIP(hipGraphLaunch(ex.exec, s));
        }
        if (ex.done) BSMM_HIP(hipEventRecord(ex.done, s));
        return BSMM_OK;
    }
    for (auto &l : ex.launches)
        BSMM_TRY(launch_smm(l.first, A->d_data(), B->d_data(), C->d_data(),
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
        a.A = A->d_data();
        a.B = B->d_data();
        a.C = C->d_data();
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
        hipGraphNode_t node;
        if (hipGraphAddKernelNode(&node, graph, nullptr, 0, &kp) != hipSuccess) {
            set_error(BSMM_EDEVICE, "hipGraphAddKernelNode failed");
            status = BSMM_EDEVICE;
        } else if (a.split > 1) {
            // The class's split-run epilogue runs after its kernel.
            hipKernelNodeParams rp{};
            rp.func = (void *)k_smm_split_reduce;
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
