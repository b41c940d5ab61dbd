/*
 * bsmm_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU reference for one rank's local
 * block-sparse multiply  C <- filter_eps( beta*C + alpha*A*B )  over matrices
 * stored in blocked compressed-sparse-row form (paper, Sec. II: matrices are
 * kept as block CSR; the local step is a set of pairwise products of small
 * dense blocks, an A block being m x k and a B block k x n).
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  The GPU library shares no code, header, table or
 * helper with it.
 *
 * Conventions (the readings used where the paper is silent):
 *  - a matrix has nbr block rows of sizes rbs[] and nbc block columns of
 *    sizes cbs[]; row_ptr is int64[nbr+1], col_ind int32[nnzb], columns
 *    strictly ascending inside a row;
 *  - block data are packed in CSR order, every block column-major with
 *    leading dimension equal to its row count;
 *  - the output pattern is the union of the old C pattern and every (I,J)
 *    for which some K has A(I,K) and B(K,J) stored;
 *  - BLAS-style scalars: beta == 0 overwrites (old C ignored), alpha == 0
 *    skips the products;
 *  - the filter drops a block iff eps > 0 and its squared Frobenius norm,
 *    summed in column-major order, is strictly below eps*eps.
 *
 * Floating point: FP64 throughout, no FMA contraction (built with
 * -ffp-contract=off).  The compensated mode replaces every block dot
 * product by the Dot2 algorithm of Ogita, Rump and Oishi ("Accurate sum and
 * dot product", SIAM J. Sci. Comput. 26(6), 2005): TwoProduct through an
 * explicit fma() and TwoSum, which returns the dot product as if computed
 * in twice the working precision.
 *
 * Build-time mutants (-DORC_MUTANT=n) plant one deliberate mistake each;
 * the test suite builds them to show that its pins catch such mistakes.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef ORC_MUTANT
#define ORC_MUTANT 0
#endif

/* Element offset of every block of a block-CSR matrix, in CSR order. */
static int64_t *block_offsets(int32_t nbr, const int32_t *rbs, const int32_t *cbs,
                              const int64_t *rp, const int32_t *ci)
{
    int64_t nnzb = rp[nbr];
    int64_t *off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nnzb + 1));
    if (!off) return NULL;
    int64_t acc = 0;
    for (int32_t i = 0; i < nbr; ++i)
        for (int64_t b = rp[i]; b < rp[i + 1]; ++b) {
            off[b] = acc;
            acc += (int64_t)rbs[i] * (int64_t)cbs[ci[b]];
        }
    off[nnzb] = acc;
    return off;
}

/* Position of column j in the sorted list ci[lo..hi), or -1. */
static int64_t find_col(const int32_t *ci, int64_t lo, int64_t hi, int32_t j)
{
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (ci[mid] < j) lo = mid + 1;
        else if (ci[mid] > j) hi = mid;
        else return mid;
    }
    return -1;
}

/*
 * Output pattern: old C pattern united with the symbolic product pattern.
 * out_rp (int64[nbr+1]) is always written.  out_ci may be NULL, in which
 * case only the counts are produced; otherwise it receives the ascending
 * column list of every row.  c_rp/c_ci may be NULL (no old C).
 * Returns 0, or -4 when scratch memory cannot be obtained.
 */
int orc_pattern(int32_t nbr, int32_t nbc,
                const int64_t *a_rp, const int32_t *a_ci,
                const int64_t *b_rp, const int32_t *b_ci,
                const int64_t *c_rp, const int32_t *c_ci,
                int64_t *out_rp, int32_t *out_ci)
{
    unsigned char *mark = (unsigned char *)calloc((size_t)(nbc > 0 ? nbc : 1), 1);
    if (!mark) return -4;
    out_rp[0] = 0;
    for (int32_t i = 0; i < nbr; ++i) {
        memset(mark, 0, (size_t)nbc);
#if ORC_MUTANT != 6
        if (c_rp)
            for (int64_t p = c_rp[i]; p < c_rp[i + 1]; ++p) mark[c_ci[p]] = 1;
#endif
        for (int64_t p = a_rp[i]; p < a_rp[i + 1]; ++p) {
            int32_t k = a_ci[p];
            for (int64_t q = b_rp[k]; q < b_rp[k + 1]; ++q) mark[b_ci[q]] = 1;
        }
        int64_t cnt = 0;
        for (int32_t j = 0; j < nbc; ++j)
            if (mark[j]) {
                if (out_ci) out_ci[out_rp[i] + cnt] = j;
                ++cnt;
            }
        out_rp[i + 1] = out_rp[i] + cnt;
    }
    free(mark);
    return 0;
}

/* Dot2 building blocks (Ogita, Rump, Oishi 2005). */
static inline void two_sum(double a, double b, double *s, double *e)
{
    double x = a + b;
    double z = x - a;
    *e = (a - (x - z)) + (b - z);
    *s = x;
}

/*
 * Numeric phase.  For every output block (I,J) of rows [row_begin,row_end):
 *   acc = sum over K ascending in row I of A, with B(K,J) stored, of
 *         A(I,K) * B(K,J)             (plain triple loop, column-major)
 *   out = (beta == 0 ? 0 : beta*Cin(I,J)) + (alpha == 0 ? 0 : alpha*acc)
 * with an absent Cin block read as zero.  o_data points at the data of the
 * first block of row row_begin (offsets are taken relative to it), so a
 * caller that samples rows only allocates the sampled part.
 * compensated != 0 selects the Dot2 accumulation.  nthreads <= 0 uses the
 * OpenMP default.  Returns 0, or -4 on allocation failure.
 */
int orc_multiply(double alpha, double beta,
                 int32_t nbr, int32_t nbk, int32_t nbc,
                 const int32_t *rbs, const int32_t *kbs, const int32_t *cbs,
                 const int64_t *a_rp, const int32_t *a_ci, const double *a_data,
                 const int64_t *b_rp, const int32_t *b_ci, const double *b_data,
                 const int64_t *c_rp, const int32_t *c_ci, const double *c_data,
                 const int64_t *o_rp, const int32_t *o_ci, double *o_data,
                 int32_t row_begin, int32_t row_end, int32_t compensated,
                 int32_t nthreads)
{
    (void)nbk;
    (void)nbc;
    int64_t *a_off = block_offsets(nbr, rbs, kbs, a_rp, a_ci);
    int64_t *b_off = block_offsets(nbk, kbs, cbs, b_rp, b_ci);
    int64_t *c_off = c_rp ? block_offsets(nbr, rbs, cbs, c_rp, c_ci) : NULL;
    int64_t *o_off = block_offsets(nbr, rbs, cbs, o_rp, o_ci);
    int status = 0;
    if (!a_off || !b_off || !o_off || (c_rp && !c_off)) {
        status = -4;
        goto done;
    }
    {
        int64_t base = o_off[o_rp[row_begin]];
#ifdef _OPENMP
        if (nthreads > 0) omp_set_num_threads(nthreads);
#else
        (void)nthreads;
#endif
        int failed = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : failed)
        for (int32_t i = row_begin; i < row_end; ++i) {
            const int32_t m = rbs[i];
            double *acc = NULL, *cmp = NULL;
            int64_t maxn = 0;
            for (int64_t p = o_rp[i]; p < o_rp[i + 1]; ++p)
                if (cbs[o_ci[p]] > maxn) maxn = cbs[o_ci[p]];
            acc = (double *)malloc(sizeof(double) * (size_t)(m * maxn + 1));
            cmp = (double *)malloc(sizeof(double) * (size_t)(m * maxn + 1));
            if (!acc || !cmp) {
                failed = 1;
                free(acc);
                free(cmp);
                continue;
            }
            for (int64_t p = o_rp[i]; p < o_rp[i + 1]; ++p) {
                const int32_t j = o_ci[p];
                const int32_t n = cbs[j];
                const int64_t mn = (int64_t)m * n;
                for (int64_t e = 0; e < mn; ++e) acc[e] = 0.0, cmp[e] = 0.0;
                if (alpha != 0.0) {
                    int64_t pend = a_rp[i + 1];
#if ORC_MUTANT == 4
                    if (pend > a_rp[i]) --pend; /* mutant: last K dropped */
#endif
                    for (int64_t pa = a_rp[i]; pa < pend; ++pa) {
                        const int32_t kb = a_ci[pa];
                        const int64_t pb = find_col(b_ci, b_rp[kb], b_rp[kb + 1], j);
                        if (pb < 0) continue;
                        const int32_t k = kbs[kb];
                        const double *a = a_data + a_off[pa];
                        const double *b = b_data + b_off[pb];
                        for (int32_t jj = 0; jj < n; ++jj)
                            for (int32_t kk = 0; kk < k; ++kk)
                                for (int32_t ii = 0; ii < m; ++ii) {
#if ORC_MUTANT == 1
                                    /* mutant: square A blocks read transposed */
                                    const double av = (m == k) ? a[kk + (int64_t)m * ii]
                                                               : a[ii + (int64_t)m * kk];
#else
                                    const double av = a[ii + (int64_t)m * kk];
#endif
                                    const double bv = b[kk + (int64_t)k * jj];
                                    if (compensated) {
                                        double h = av * bv;
                                        double r = fma(av, bv, -h);
                                        double s, q;
                                        two_sum(acc[ii + m * jj], h, &s, &q);
                                        acc[ii + m * jj] = s;
                                        cmp[ii + m * jj] += q + r;
                                    } else {
                                        acc[ii + (int64_t)m * jj] += av * bv;
                                    }
                                }
                    }
                }
                double *out = o_data + (o_off[p] - base);
                const double *cin = NULL;
                if (c_rp && beta != 0.0) {
                    const int64_t pc = find_col(c_ci, c_rp[i], c_rp[i + 1], j);
                    if (pc >= 0) cin = c_data + c_off[pc];
                }
                for (int64_t e = 0; e < mn; ++e) {
                    const double dot = compensated ? acc[e] + cmp[e] : acc[e];
#if ORC_MUTANT == 3
                    const double prod = (alpha == 0.0) ? 0.0 : -alpha * dot;
#else
                    const double prod = (alpha == 0.0) ? 0.0 : alpha * dot;
#endif
#if ORC_MUTANT == 2
                    const double old = 0.0 * (cin ? 1.0 : 0.0); /* mutant: beta term dropped */
#else
                    const double old = (beta == 0.0 || !cin) ? 0.0 : beta * cin[e];
#endif
                    out[e] = old + prod;
                }
            }
            free(acc);
            free(cmp);
        }
        if (failed) status = -4;
    }
done:
    free(a_off);
    free(b_off);
    free(c_off);
    free(o_off);
    return status;
}

/*
 * Squared Frobenius norm of every block, summed plainly in column-major
 * order: out_sumsq[b] = sum_e data_b[e]^2.  The caller drops block b iff
 * eps > 0 and out_sumsq[b] < eps*eps (a NaN norm is therefore kept).
 */
int orc_block_sumsq(int32_t nbr, const int32_t *rbs, const int32_t *cbs,
                    const int64_t *rp, const int32_t *ci, const double *data,
                    double *out_sumsq)
{
    int64_t *off = block_offsets(nbr, rbs, cbs, rp, ci);
    if (!off) return -4;
    for (int32_t i = 0; i < nbr; ++i)
        for (int64_t b = rp[i]; b < rp[i + 1]; ++b) {
            const int64_t len = off[b + 1] - off[b];
            double s = 0.0;
            for (int64_t e = 0; e < len; ++e) s += data[off[b] + e] * data[off[b] + e];
            out_sumsq[b] = s;
        }
    free(off);
    return 0;
}

/* Keep rule of the filter, applied to n block norms: keep[b] = 1 unless
 * eps > 0 and sumsq[b] < eps*eps. */
int orc_filter_keep(int64_t n, const double *sumsq, double eps, unsigned char *keep)
{
    for (int64_t b = 0; b < n; ++b) {
#if ORC_MUTANT == 5
        keep[b] = !(eps > 0.0 && sumsq[b] <= eps * eps); /* mutant: ties dropped */
#else
        keep[b] = !(eps > 0.0 && sumsq[b] < eps * eps);
#endif
    }
    return 0;
}
