// multiply.hip -- orchestration of C <- filter_eps(beta*C + alpha*A*B).
//
// Order of the phases (paper, Sec. II: Traversal, Generation, Scheduler;
// Sec. III: densification):
//   1. symbolic: new C pattern = old pattern U product pattern; one host
//      read of the totals; new C storage with the old blocks moved in;
//   2. numeric: dense inputs -> merged panels + one FP64 MFMA GEMM with the
//      undensify step fused into its epilogue; otherwise stacks of block
//      products grouped by shape -> batched small-block kernels;
//   3. filter.
#include <algorithm>
#include <cmath>
#include <cstdio>

#include "dev_util.h"
#include "internal.h"

namespace bsmm {
int validate_multiply(bsmm_matrix_s *A, bsmm_matrix_s *B, bsmm_matrix_s *C, double eps);
int adopt_stream(bsmm_matrix_s *M, hipStream_t s);
bsmm_multiply_stats &stats();

namespace {

// Sums of the per-row symbolic counts: out_i[0..4] (nnz, elems, products,
// and with the screen the screened blocks and screened old blocks), out_d[0]
// (flops).
__global__ __launch_bounds__(256) void k_row_totals(int32_t nbr, const int64_t *nnz,
                                                    const int64_t *elems, const int64_t *prod,
                                                    const double *flops, const int64_t *scr,
                                                    const int64_t *old_scr, int64_t *out_i,
                                                    double *out_d) {
    __shared__ int64_t ri[16];
    __shared__ double rd[16];
    int64_t a = 0, b = 0, c = 0, e = 0, f = 0;
    double d = 0.0;
    for (int64_t i = threadIdx.x; i < nbr; i += blockDim.x) {
        a += nnz[i];
        b += elems[i];
        c += prod[i];
        d += flops[i];
        if (scr) {
            e += scr[i];
            f += old_scr[i];
        }
    }
    a = block_sum(a, ri);
    b = block_sum(b, ri);
    c = block_sum(c, ri);
    e = block_sum(e, ri);
    f = block_sum(f, ri);
    d = block_sum(d, rd);
    if (threadIdx.x == 0) {
        out_i[0] = a;
        out_i[1] = b;
        out_i[2] = c;
        out_i[3] = e;
        out_i[4] = f;
        out_d[0] = d;
    }
}

struct NewPattern {
    DevBuf rp, ci, off, data;
};

// Symbolic phase with the norm-bound screen: block norms of A, B and (beta
// != 0) the old C, the count with the screen, then the fill from its
// bitmap.  The new pattern is (old pattern U product pattern) minus the
// screened blocks, so it may also lose old blocks.
int symbolic_screened(bsmm_matrix_s *A, bsmm_matrix_s *B, bsmm_matrix_s *C, const ScreenNorms &req,
                      SymbolicTotals *tot, bool *changed, NewPattern &np, DevBuf &row_elems,
                      hipStream_t s) {
    const int32_t nbr = A->nbr, nbc = B->nbc;
    const int64_t nwords = (nbc + 31) / 32;
    ScreenNorms sn = req;
    DevBuf an, bn, cn, bits, rnnz, rprod, rflops, rscr, rold, sums_i, sums_d;
    BSMM_TRY(an.reserve(sizeof(double) * (A->nnzb + 1), s));
    BSMM_TRY(bn.reserve(sizeof(double) * (B->nnzb + 1), s));
    BSMM_TRY(block_norms(A, an.as<double>(), s));
    BSMM_TRY(block_norms(B, bn.as<double>(), s));
    sn.a = an.as<double>();
    sn.b = bn.as<double>();
    sn.c = nullptr;
    if (sn.beta_abs != 0.0 && C->nnzb > 0) {
        BSMM_TRY(cn.reserve(sizeof(double) * (C->nnzb + 1), s));
        BSMM_TRY(block_norms(C, cn.as<double>(), s));
        sn.c = cn.as<double>();
    }
    BSMM_TRY(row_elems.reserve(sizeof(int64_t) * (nbr + 1), s));
    BSMM_TRY(bits.reserve(sizeof(uint32_t) * nbr * nwords, s));
    BSMM_TRY(rnnz.reserve(sizeof(int64_t) * (nbr + 1), s));
    BSMM_TRY(rprod.reserve(sizeof(int64_t) * (nbr + 1), s));
    BSMM_TRY(rflops.reserve(sizeof(double) * (nbr + 1), s));
    BSMM_TRY(rscr.reserve(sizeof(int64_t) * (nbr + 1), s));
    BSMM_TRY(rold.reserve(sizeof(int64_t) * (nbr + 1), s));
    BSMM_TRY(sums_i.reserve(sizeof(int64_t) * 6, s));
    BSMM_TRY(sums_d.reserve(sizeof(double) * 2, s));
    BSMM_TRY(symbolic_count_screen(A, B, C, sn, bits.as<uint32_t>(), rnnz.as<int64_t>(),
                                   row_elems.as<int64_t>(), rprod.as<int64_t>(), rflops.as<double>(),
                                   rscr.as<int64_t>(), rold.as<int64_t>(), s));
    hipLaunchKernelGGL(k_row_totals, dim3(1), dim3(256), 0, s, nbr,
                       (const int64_t *)rnnz.as<int64_t>(), (const int64_t *)row_elems.as<int64_t>(),
                       (const int64_t *)rprod.as<int64_t>(), (const double *)rflops.as<double>(),
                       (const int64_t *)rscr.as<int64_t>(), (const int64_t *)rold.as<int64_t>(),
                       sums_i.as<int64_t>(), sums_d.as<double>());
    BSMM_TRY(launch_check("row_totals"));
    int64_t hi[5];
    double hd[1];
    BSMM_HIP(hipMemcpyAsync(hi, sums_i.p, sizeof(hi), hipMemcpyDeviceToHost, s));
    BSMM_HIP(hipMemcpyAsync(hd, sums_d.p, sizeof(hd), hipMemcpyDeviceToHost, s));
    BSMM_HIP(hipStreamSynchronize(s));
    tot->nnzb = hi[0];
    tot->nelems = hi[1];
    tot->nprod = hi[2];
    tot->flops = hd[0];
    tot->screen = true;
    tot->screened = hi[3];
    tot->old_screened = hi[4];
    if (tot->nnzb > (int64_t)INT32_MAX || tot->nelems >= (int64_t(1) << 47)) {
        set_error(BSMM_ERANGE, "result too large (%lld blocks, %lld elements)",
                  (long long)tot->nnzb, (long long)tot->nelems);
        return BSMM_ERANGE;
    }
    // Unchanged exactly when no old block was screened (the new pattern then
    // contains the old one) and the counts agree.
    if (tot->old_screened == 0 && tot->nnzb == C->nnzb) return BSMM_OK;
    *changed = true;
    BSMM_TRY(np.rp.reserve(sizeof(int64_t) * (nbr + 1), s));
    BSMM_TRY(np.ci.reserve(sizeof(int32_t) * (tot->nnzb + 1), s));
    BSMM_TRY(scan_exclusive_i64(rnnz.as<int64_t>(), np.rp.as<int64_t>(), nbr, s));
    return symbolic_fill_bits(nbr, nbc, bits.as<uint32_t>(), np.rp.as<int64_t>(), np.ci.as<int32_t>(), s);
}

// Symbolic phase.  On return *tot holds the new C sizes, the product count
// and the algorithmic flops of A*B; if the pattern changes, np holds the new
// index (and row element totals in row_elems).  With `screen` (filtering
// stack multiplies), C blocks whose norm bound lies below eps are left out
// of the new pattern.
int symbolic(bsmm_matrix_s *A, bsmm_matrix_s *B, bsmm_matrix_s *C, SymbolicTotals *tot,
             bool *changed, NewPattern &np, DevBuf &row_elems, hipStream_t s,
             const ScreenNorms *screen = nullptr) {
    const int32_t nbr = A->nbr, nbk = A->nbc, nbc = B->nbc;
    *changed = false;
    if (nbr == 0 || nbc == 0) return BSMM_OK;
    const bool closed_form = A->full() && B->full() && nbk > 0;
    // The screen's bitmap: one bit per (I, J), at most 256 MB.
    const int64_t nwords = (nbc + 31) / 32;
    if (screen && !closed_form && nbc <= kScreenMaxCols && (int64_t)nbr * nwords <= (int64_t(1) << 26))
        return symbolic_screened(A, B, C, *screen, tot, changed, np, row_elems, s);
    BSMM_TRY(row_elems.reserve(sizeof(int64_t) * (nbr + 1), s));
    if (closed_form) {
        // Every (I,K,J) is a product: the new pattern is every block.
        const double M = (double)A->rows(), K = (double)A->cols(), N = (double)B->cols();
        tot->nnzb = (int64_t)nbr * nbc;
        tot->nelems = A->rows() * B->cols();
        tot->nprod = (int64_t)nbr * nbk * nbc;
        tot->flops = 2.0 * M * N * K;
        if (tot->nnzb > (int64_t)INT32_MAX || tot->nelems >= (int64_t(1) << 47)) {
            set_error(BSMM_ERANGE, "result too large (%lld blocks, %lld elements)",
                      (long long)tot->nnzb, (long long)tot->nelems);
            return BSMM_ERANGE;
        }
        if (tot->nnzb == C->nnzb) return BSMM_OK;
        *changed = true;
        BSMM_TRY(np.rp.reserve(sizeof(int64_t) * (nbr + 1), s));
        BSMM_TRY(np.ci.reserve(sizeof(int32_t) * (tot->nnzb + 1), s));
        BSMM_TRY(full_pattern(nbr, nbc, B->cols(), np.rp.as<int64_t>(), np.ci.as<int32_t>(),
                              row_elems.as<int64_t>(), C->d_rbs(), s));
        return BSMM_OK;
    }
    DevBuf rnnz, rprod, rflops, sums_i, sums_d;
    BSMM_TRY(rnnz.reserve(sizeof(int64_t) * (nbr + 1), s));
    BSMM_TRY(rprod.reserve(sizeof(int64_t) * (nbr + 1), s));
    BSMM_TRY(rflops.reserve(sizeof(double) * (nbr + 1), s));
    BSMM_TRY(sums_i.reserve(sizeof(int64_t) * 6, s));
    BSMM_TRY(sums_d.reserve(sizeof(double) * 2, s));
    BSMM_TRY(symbolic_count(A, B, C, rnnz.as<int64_t>(), row_elems.as<int64_t>(),
                            rprod.as<int64_t>(), rflops.as<double>(), s));
    hipLaunchKernelGGL(k_row_totals, dim3(1), dim3(256), 0, s, nbr,
                       (const int64_t *)rnnz.as<int64_t>(), (const int64_t *)row_elems.as<int64_t>(),
                       (const int64_t *)rprod.as<int64_t>(), (const double *)rflops.as<double>(),
                       (const int64_t *)nullptr, (const int64_t *)nullptr, sums_i.as<int64_t>(),
                       sums_d.as<double>());
    BSMM_TRY(launch_check("row_totals"));
    int64_t hi[3];
    double hd[1];
    BSMM_HIP(hipMemcpyAsync(hi, sums_i.p, sizeof(hi), hipMemcpyDeviceToHost, s));
    BSMM_HIP(hipMemcpyAsync(hd, sums_d.p, sizeof(hd), hipMemcpyDeviceToHost, s));
    BSMM_HIP(hipStreamSynchronize(s));
    tot->nnzb = hi[0];
    tot->nelems = hi[1];
    tot->nprod = hi[2];
    tot->flops = hd[0];
    if (tot->nnzb > (int64_t)INT32_MAX || tot->nelems >= (int64_t(1) << 47)) {
        set_error(BSMM_ERANGE, "result too large (%lld blocks, %lld elements)",
                  (long long)tot->nnzb, (long long)tot->nelems);
        return BSMM_ERANGE;
    }
    // The new pattern contains the old one, so equal counts mean equal sets.
    if (tot->nnzb == C->nnzb) return BSMM_OK;
    *changed = true;
    BSMM_TRY(np.rp.reserve(sizeof(int64_t) * (nbr + 1), s));
    BSMM_TRY(np.ci.reserve(sizeof(int32_t) * (tot->nnzb + 1), s));
    BSMM_TRY(scan_exclusive_i64(rnnz.as<int64_t>(), np.rp.as<int64_t>(), nbr, s));
    return symbolic_fill(A, B, C, np.rp.as<int64_t>(), np.ci.as<int32_t>(), s);
}

// Installs a grown pattern into C, moving the old blocks in when beta != 0.
int install_pattern(bsmm_matrix_s *C, const SymbolicTotals &tot, NewPattern &np,
                    const DevBuf &row_elems, double beta, hipStream_t s) {
    BSMM_TRY(np.off.reserve(sizeof(int64_t) * (tot.nnzb + 1), s));
    BSMM_TRY(np.data.reserve(C->esize() * (tot.nelems + 1), s));
    BSMM_TRY(build_block_offsets(C->d_rbs(), C->d_cbs(), C->nbr, np.rp.as<int64_t>(),
                                 np.ci.as<int32_t>(), tot.nnzb, np.off.as<int64_t>(),
                                 row_elems.as<int64_t>(), s));
    // beta != 0 reads the old values: move the old blocks in (new blocks get
    // zeros), or zero everything when there were no old blocks.  beta == 0
    // never reads C, so the new storage is left as is.
    if (beta != 0.0) {
        if (C->nnzb > 0)
            BSMM_TRY(relayout(C, np.rp.as<int64_t>(), np.ci.as<int32_t>(), np.off.as<int64_t>(),
                              np.data.p, s));
        else
            BSMM_TRY(fill_zero_bytes(np.data.p, C->esize() * tot.nelems, s));
    }
    C->b_row_ptr = std::move(np.rp);
    C->b_col_ind = std::move(np.ci);
    C->b_blk_off = std::move(np.off);
    C->b_data = std::move(np.data);
    C->nnzb = tot.nnzb;
    C->nelems = tot.nelems;
    C->storage = tot.nelems;
    C->holes = false;
    C->version = next_version();
    return BSMM_OK;
}

int active_classes(const Stacks &st) {
    int nc = 0;
    for (char a : st.class_active) nc += a != 0;
    return nc;
}

// Options that change what a plan computes.
std::string plan_key(const Options &o) {
    char buf[160];
    snprintf(buf, sizeof buf, "%d %d %lld %lld %d %d %d %d %d %d %d %d %d %d|", o.path, o.stack_kernel,
             (long long)o.stack_chunk, (long long)o.stack_panel, o.emul_slices, o.forced[0],
             o.forced[1], o.forced[2], o.forced[3], o.stack_tile, o.stack_sched, o.jit, o.prescreen,
             o.stack_at);
    return std::string(buf) + o.tune_db + "|" + o.mlp_weights;
}

}  // namespace

// A cached multiply: the symbolic totals, the stacks and their launches (or
// instantiated graph), valid while A, B and C keep the versions recorded.
struct Plan {
    const bsmm_matrix_s *A = nullptr, *B = nullptr;
    uint64_t va = 0, vb = 0, vc = 0;
    std::string key;
    double alpha = 0.0, beta = 0.0;
    double eps = 0.0;  // filter threshold the screen used (tot.screen)
    SymbolicTotals tot;
    int path = 0;
    Stacks st;
    StackExec ex;
    DevBuf norm2;  // squared block norms the planned launches write (filtering multiplies)
};
void free_plan(Plan *p) { delete p; }

// Sets the norm sink for the numeric phase of one multiply and clears it
// again on every way out.
struct NormSinkScope {
    explicit NormSinkScope(double *p) { set_norm_sink(p); }
    ~NormSinkScope() { set_norm_sink(nullptr); }
};

// Whether a multiply screens its new C pattern by the norm bound (filtering
// stack multiplies with option "prescreen"), and with which inputs.  The
// margin bounds the rounding of a computed block relative to the bound:
// at most about n u for n accumulated terms (n at most A's column count),
// taken four times over and never below 1e-6.  Thresholds below 1e-150
// are left alone (their square, which the filter compares with, loses
// precision), and so are margins above 1/4 (FP32 sums of very long rows).
bool screen_request(const bsmm_matrix_s *A, const bsmm_matrix_s *B, const bsmm_matrix_s *C,
                    double alpha, double beta, double eps, const Options &o, ScreenNorms *sn) {
    const bool stack = o.path == 1 || (o.path == 0 && !(A->full() && B->full()));
    if (!o.prescreen || !stack || !(eps >= 1e-150) || alpha == 0.0 || !std::isfinite(alpha) ||
        !std::isfinite(beta))
        return false;
    const double u = C->dtype == BSMM_F32 ? 0x1p-24 : 0x1p-53;
    const double margin = std::max(1e-6, 4.0 * ((double)A->cols() + 4.0) * u);
    if (margin > 0.25) return false;
    sn->alpha_abs = std::fabs(alpha);
    sn->beta_abs = std::fabs(beta);
    sn->eps = eps;
    sn->margin = margin;
    return true;
}

// Limits of the stack path, checked on the host before any work is queued:
// a product entry carries k in 16 bits and the count and fill phases map
// C's block columns in LDS.
int check_stack_limits(const bsmm_matrix_s *A, const bsmm_matrix_s *B, const bsmm_matrix_s *C,
                       const Options &o) {
    if (o.path == 3 && C->dtype != BSMM_F64) {
        set_error(BSMM_ENOTSUP, "the split-precision emulation computes FP64 products only");
        return BSMM_ENOTSUP;
    }
    const bool dense = o.path == 2 || (o.path == 0 && A->full() && B->full());
    if (o.path == 3 || dense) return BSMM_OK;
    if (A->max_cbs > kMaxStackK) {
        set_error(BSMM_ENOTSUP, "stack path: block columns of A hold at most %d columns (found %d)",
                  kMaxStackK, A->max_cbs);
        return BSMM_ENOTSUP;
    }
    return BSMM_OK;
}

namespace {

// Stack path over panels of consecutive C block rows whose products fit
// the stack buffers (option "stack_panel"); each panel's stacks are built,
// executed and then replaced by the next panel's, in stream order.
int stacks_by_panels(bsmm_matrix_s *A, bsmm_matrix_s *B, bsmm_matrix_s *C, double alpha,
                     double beta, int64_t cap, Stacks &st, int64_t *n_panels, hipStream_t s) {
    std::vector<int64_t> pb, cb;
    BSMM_TRY(stack_row_bounds(C, st, &pb, &cb, s));
    if (options().stack_kernel == 1) BSMM_TRY(stack_class_run_lengths(C, st, &st.run_len_hint, s));
    int64_t runs = 0, sched = 0;
    int jit = 0;
    for (int32_t r0 = 0; r0 < C->nbr;) {
        int32_t r1 = r0 + 1;
        while (r1 < C->nbr && pb[r1 + 1] - pb[r0] <= cap) ++r1;
        if (pb[r1] > pb[r0]) {
            BSMM_TRY(stack_rows(A, B, C, st, r0, r1, cb[r0], cb[r1], pb[r1] - pb[r0], s));
            StackExec ex;  // a graph is retired only after its launch has completed
            BSMM_TRY(run_stacks(A, B, C, st, alpha, beta, s, &ex));
            runs += st.n_runs;
            sched += st.n_sched;
            jit = std::max(jit, st.n_jit);
            ++*n_panels;
            if (options().verbose) {
                // Host progress of a long multiply (the panel is queued, not finished).
                fprintf(stderr, "[bsmm] stack panel %lld: block rows %d..%d of %d, %lld products\n",
                        (long long)*n_panels, r0, r1 - 1, C->nbr, (long long)(pb[r1] - pb[r0]));
                fflush(stderr);
            }
        }
        r0 = r1;
    }
    st.n_runs = runs;
    st.n_sched = sched;
    st.n_jit = jit;
    st.n_prod = pb[C->nbr];
    return BSMM_OK;
}

int numeric(int path, bsmm_matrix_s *A, bsmm_matrix_s *B, bsmm_matrix_s *C, double alpha,
            double beta, const Options &o, Stacks &st, StackExec &ex, bool replay,
            int64_t *n_panels, hipStream_t s) {
    *n_panels = 0;
    switch (path) {
    case 0:
        if (beta != 1.0) BSMM_TRY(scale_blocks(C, nullptr, beta, s));
        return BSMM_OK;
    case 3:
        return emul_multiply(A, B, C, alpha, beta, o.emul_slices, s);
    case 2:
        return dense_multiply(A, B, C, alpha, beta, s);
    default:
        st.a_t_fresh = false;  // A's transposed copy, if any, is made anew
        if (replay) {
            BSMM_TRY(replay_stacks(ex, A, B, C, st, alpha, beta, s));
            *n_panels = 1;
        } else if (o.stack_panel > 0 && st.n_prod > o.stack_panel) {
            BSMM_TRY(stack_count(A, B, C, st, s));
            BSMM_TRY(stacks_by_panels(A, B, C, alpha, beta, o.stack_panel, st, n_panels, s));
        } else {
            BSMM_TRY(build_stacks(A, B, C, st, s));
            BSMM_TRY(run_stacks(A, B, C, st, alpha, beta, s, &ex));
            *n_panels = 1;
        }
        if (beta != 1.0 && st.n_runs < C->nnzb)
            BSMM_TRY(scale_blocks(C, st.c_count.as<int64_t>(), beta, s));
        return BSMM_OK;
    }
}

int multiply_impl(double alpha, bsmm_matrix_s *A, bsmm_matrix_s *B, double beta,
                  bsmm_matrix_s *C, double eps, hipStream_t s) {
    bsmm_multiply_stats &stt = stats();
    stt = bsmm_multiply_stats{};
    const Options &o = options();
    Plan *pl = C->plan;
    // A screened pattern holds only for the threshold it was screened with.
    const bool hit = o.plan_cache && pl && pl->A == A && pl->B == B && pl->va == A->version &&
                     pl->vb == B->version && pl->vc == C->version && pl->alpha == alpha &&
                     pl->beta == beta && pl->key == plan_key(o) &&
                     (!pl->tot.screen || pl->eps == eps);
    // Filtering stack multiplies: the scheduled kernel writes the squared
    // norms of the blocks it finishes, the filter reads the rest.
    const double *pre_norm2 = nullptr;
    if (hit) {
        // Same patterns, buffers and options as the planned multiply: C's
        // pattern already holds the product, the stacks are still valid.
        if (eps > 0.0 && pl->norm2.p) {
            BSMM_TRY(fill_value(pl->norm2.as<double>(), C->nnzb, -1.0, s));
            pre_norm2 = pl->norm2.as<double>();
        }
        BSMM_TRY(numeric(pl->path, A, B, C, alpha, beta, o, pl->st, pl->ex, true,
                         &stt.n_row_panels, s));
        stt.path = pl->path;
        stt.c_nnzb_before = C->nnzb;
        stt.n_screened = pl->tot.screened;
        stt.n_products_run = pl->st.n_prod;
        stt.n_products = pl->tot.nprod;
        stt.flops = pl->tot.flops;
        stt.n_runs = pl->st.n_runs;
        stt.n_sched_runs = pl->st.n_sched;
        stt.n_jit_classes = pl->st.n_jit;
        stt.n_classes = active_classes(pl->st);
    } else {
        free_plan(C->plan);
        C->plan = nullptr;
        SymbolicTotals tot;
        bool changed = false;
        NewPattern np;
        DevBuf row_elems;
        ScreenNorms sn;
        const bool screen = screen_request(A, B, C, alpha, beta, eps, o, &sn);
        BSMM_TRY(symbolic(A, B, C, &tot, &changed, np, row_elems, s, screen ? &sn : nullptr));
        if (changed) BSMM_TRY(install_pattern(C, tot, np, row_elems, beta, s));
        stt.c_nnzb_before = C->nnzb;
        stt.n_screened = tot.screened;
        stt.n_products = tot.nprod;
        stt.flops = tot.flops;
        const bool dense = o.path == 2 || (o.path == 0 && A->full() && B->full());
        const int path = (alpha == 0.0 || tot.nprod == 0) ? 0 : o.path == 3 ? 3 : dense ? 2 : 1;
        auto *p = new Plan();
        p->st.n_prod = tot.nprod;
        p->st.screened = tot.screen;
        if (eps > 0.0 && path == 1 && C->nnzb > 0) {
            int st = p->norm2.reserve(sizeof(double) * (size_t)C->nnzb, s);
            if (st == BSMM_OK) st = fill_value(p->norm2.as<double>(), C->nnzb, -1.0, s);
            if (st != BSMM_OK) {
                delete p;
                return st;
            }
            pre_norm2 = p->norm2.as<double>();
        }
        int status;
        {
            NormSinkScope sink(const_cast<double *>(pre_norm2));
            status = numeric(path, A, B, C, alpha, beta, o, p->st, p->ex, false, &stt.n_row_panels, s);
        }
        if (status != BSMM_OK) {
            delete p;
            return status;
        }
        stt.path = path;
        stt.n_runs = p->st.n_runs;
        stt.n_products_run = path == 1 ? p->st.n_prod : path == 0 ? 0 : tot.nprod;
        stt.n_sched_runs = p->st.n_sched;
        stt.n_jit_classes = p->st.n_jit;
        stt.n_classes = active_classes(p->st);
        // A multiply built in several row panels keeps no stacks to replay.
        if (o.plan_cache && stt.n_row_panels <= 1) {
            p->A = A;
            p->B = B;
            p->va = A->version;
            p->vb = B->version;
            p->vc = C->version;
            p->key = plan_key(o);
            p->alpha = alpha;
            p->beta = beta;
            p->eps = eps;
            p->tot = tot;
            p->path = path;
            C->plan = p;
        } else {
            // The norms outlive the plan until the filter has read them.
            DevBuf norms = std::move(p->norm2);
            delete p;
            int64_t after = C->nnzb;
            BSMM_TRY(filter_blocks(C, eps, &after, s, pre_norm2));
            stt.c_nnzb_after = after;
            return BSMM_OK;
        }
    }
    int64_t after = C->nnzb;
    BSMM_TRY(filter_blocks(C, eps, &after, s, pre_norm2));
    stt.c_nnzb_after = after;
    return BSMM_OK;
}

}  // namespace

int multiply_fixed_pattern(double alpha, bsmm_matrix_s *A, bsmm_matrix_s *B, double beta,
                           bsmm_matrix_s *C, hipStream_t s) {
    bsmm_multiply_stats &stt = stats();
    stt = bsmm_multiply_stats{};
    Options o = options();
    SymbolicTotals tot;
    bool changed = false;
    NewPattern np;
    DevBuf row_elems;
    BSMM_TRY(symbolic(A, B, C, &tot, &changed, np, row_elems, s));
    if (changed) {
        set_error(BSMM_EINDEX, "C's pattern misses product blocks (%lld blocks needed, %lld stored)",
                  (long long)tot.nnzb, (long long)C->nnzb);
        return BSMM_EINDEX;
    }
    const bool dense = o.path == 2 || (o.path == 0 && A->full() && B->full());
    const int path = (alpha == 0.0 || tot.nprod == 0) ? 0 : o.path == 3 ? 3 : dense ? 2 : 1;
    // Whole stacks in one piece: row panels would reserve again per panel,
    // after earlier panels have already written C.
    o.stack_panel = 0;
    Stacks st;
    st.n_prod = tot.nprod;
    StackExec ex;
    BSMM_TRY(numeric(path, A, B, C, alpha, beta, o, st, ex, false, &stt.n_row_panels, s));
    stt.path = path;
    stt.c_nnzb_before = stt.c_nnzb_after = C->nnzb;
    stt.n_products = tot.nprod;
    stt.n_products_run = path == 1 ? st.n_prod : path == 0 ? 0 : tot.nprod;
    stt.flops = tot.flops;
    stt.n_runs = st.n_runs;
    stt.n_sched_runs = st.n_sched;
    stt.n_jit_classes = st.n_jit;
    stt.n_classes = active_classes(st);
    return BSMM_OK;
}

}  // namespace bsmm

using namespace bsmm;

extern "C" int bsmm_multiply(double alpha, bsmm_matrix A, bsmm_matrix B, double beta,
                             bsmm_matrix C, double filter_eps, void *stream) {
    clear_error();
    BSMM_TRY(validate_multiply(A, B, C, filter_eps));
    BSMM_TRY(check_stack_limits(A, B, C, options()));
    hipStream_t s = (hipStream_t)stream;
    BSMM_TRY(adopt_stream(A, s));
    if (B != A) BSMM_TRY(adopt_stream(B, s));
    BSMM_TRY(adopt_stream(C, s));
    const int st = multiply_impl(alpha, A, B, beta, C, filter_eps, s);
    A->last_stream = B->last_stream = C->last_stream = s;
    return st;
}

extern "C" int bsmm_inspect_stacks(bsmm_matrix A, bsmm_matrix B, bsmm_matrix C, int64_t *n_runs,
                                   int64_t *n_products, int64_t *run_cblk, int32_t *run_class,
                                   int64_t *run_ptr, int64_t *prod_ablk, int64_t *prod_bblk,
                                   void *stream) {
    clear_error();
    if (!n_runs || !n_products) {
        set_error(BSMM_EINVAL, "count pointers are NULL");
        return BSMM_EINVAL;
    }
    BSMM_TRY(validate_multiply(A, B, C, 0.0));
    hipStream_t s = (hipStream_t)stream;
    SymbolicTotals tot;
    bool changed = false;
    NewPattern np;
    DevBuf row_elems;
    BSMM_TRY(symbolic(A, B, C, &tot, &changed, np, row_elems, s));
    if (changed) {
        set_error(BSMM_EINDEX, "C pattern does not contain every product block");
        return BSMM_EINDEX;
    }
    Stacks st;
    st.n_prod = tot.nprod;
    BSMM_TRY(build_stacks(A, B, C, st, s));
    const int64_t cap_r = *n_runs, cap_p = *n_products;
    *n_runs = st.n_runs;
    *n_products = st.n_prod;
    if (!run_cblk && !run_class && !run_ptr && !prod_ablk && !prod_bblk) return BSMM_OK;
    if (cap_r < st.n_runs || cap_p < st.n_prod) {
        set_error(BSMM_ERANGE, "output capacity too small");
        return BSMM_ERANGE;
    }
    std::vector<ulonglong2> prods(st.n_prod);
    std::vector<int64_t> a_off(A->nnzb + 1), b_off(B->nnzb + 1);
    if (st.n_runs > 0) {
        if (run_cblk)
            BSMM_HIP(hipMemcpyAsync(run_cblk, st.run_cblk.p, sizeof(int64_t) * st.n_runs,
                                    hipMemcpyDeviceToHost, s));
        if (run_class)
            BSMM_HIP(hipMemcpyAsync(run_class, st.run_class.p, sizeof(int32_t) * st.n_runs,
                                    hipMemcpyDeviceToHost, s));
        if (run_ptr)
            BSMM_HIP(hipMemcpyAsync(run_ptr, st.run_ptr.p, sizeof(int64_t) * (st.n_runs + 1),
                                    hipMemcpyDeviceToHost, s));
    } else if (run_ptr) {
        run_ptr[0] = 0;
    }
    if (st.n_prod > 0)
        BSMM_HIP(hipMemcpyAsync(prods.data(), st.prods.p, sizeof(ulonglong2) * st.n_prod,
                                hipMemcpyDeviceToHost, s));
    BSMM_HIP(hipMemcpyAsync(a_off.data(), A->d_blk_off(), sizeof(int64_t) * (A->nnzb + 1),
                            hipMemcpyDeviceToHost, s));
    BSMM_HIP(hipMemcpyAsync(b_off.data(), B->d_blk_off(), sizeof(int64_t) * (B->nnzb + 1),
                            hipMemcpyDeviceToHost, s));
    BSMM_HIP(hipStreamSynchronize(s));
    // Element offsets back to block indices (offsets are strictly increasing
    // because every block holds at least one element).
    for (int64_t p = 0; p < st.n_prod; ++p) {
        const int64_t ao = (int64_t)(prods[p].x & ((1ull << 48) - 1));
        const int64_t bo = (int64_t)prods[p].y;
        if (prod_ablk)
            prod_ablk[p] = std::lower_bound(a_off.begin(), a_off.end() - 1, ao) - a_off.begin();
        if (prod_bblk)
            prod_bblk[p] = std::lower_bound(b_off.begin(), b_off.end() - 1, bo) - b_off.begin();
    }
    return BSMM_OK;
}
