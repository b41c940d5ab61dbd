// index.hip -- block offsets, the symbolic C pattern, relayout and scaling.
//
// Symbolic phase (paper, Sec. II, start of the Generation phase): the new C
// pattern is the old one united with {(I,J) : some K has A(I,K) and B(K,J)}.
// One workgroup owns one block row I of C (the paper's race-free row
// ownership) and builds the row's column set as a bitmap in LDS.
#include "dev_util.h"
#include "internal.h"

namespace bsmm {

namespace {

constexpr int kRowThreads = 256;
constexpr int kMaxBitmapWords = 16384;  // 64 KB of LDS: up to 524288 block columns

// ------------------------------------------------------------ offsets
// One wave per block row: blk_off[p] = row_base[I] + m_I * (sum of the
// column sizes of the earlier blocks of the row).
__global__ __launch_bounds__(256) void k_block_offsets(const int32_t *rbs, const int32_t *cbs,
                                                       int32_t nbr, const int64_t *rp,
                                                       const int32_t *ci, const int64_t *row_base,
                                                       int64_t *blk_off) {
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
    for (int64_t row = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave_id(); row < nbr; row += waves) {
        const int64_t m = rbs[row];
        int64_t base = row_base[row];
        const int64_t p0 = rp[row], p1 = rp[row + 1];
        for (int64_t c = p0; c < p1; c += kWave) {
            const int64_t p = c + lane_id();
            const int64_t v = p < p1 ? m * cbs[ci[p]] : 0;
            const int64_t inc = wave_inclusive_scan(v);
            if (p < p1) blk_off[p] = base + inc - v;
            base += __shfl(inc, kWave - 1, kWave);
        }
        if (row == nbr - 1 && lane_id() == 0) blk_off[p1] = row_base[nbr];
    }
}

__global__ void k_set_i64(int64_t *p, int64_t v) { *p = v; }

// --------------------------------------------------------- row totals
__global__ __launch_bounds__(256) void k_row_elems(const int32_t *rbs, const int32_t *cbs,
                                                   int32_t nbr, const int64_t *rp,
                                                   const int32_t *ci, int64_t *row_elems) {
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
    for (int64_t row = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave_id(); row < nbr; row += waves) {
        int64_t s = 0;
        for (int64_t p = rp[row] + lane_id(); p < rp[row + 1]; p += kWave) s += cbs[ci[p]];
        s = wave_sum(s);
        if (lane_id() == 0) row_elems[row] = s * rbs[row];
    }
}

// --------------------------------------------------------- symbolic
// Marks the old-C columns and every column J reached through A(I,K) B(K,J)
// in the LDS bitmap of row I.  Returns (through the accumulators) the
// number of block products and their algorithmic flop count / (2 m_I).
__device__ void mark_row(uint32_t *bm, int nwords, int32_t row, const int64_t *a_rp,
                         const int32_t *a_ci, const int64_t *b_rp, const int32_t *b_ci,
                         const int64_t *c_rp, const int32_t *c_ci, const int32_t *kbs,
                         const int32_t *cbs, int64_t *nprod, double *kn_sum) {
    for (int w = threadIdx.x; w < nwords; w += blockDim.x) bm[w] = 0u;
    __syncthreads();
    if (c_rp)
        for (int64_t p = c_rp[row] + threadIdx.x; p < c_rp[row + 1]; p += blockDim.x) {
            const int32_t j = c_ci[p];
            atomicOr(&bm[j >> 5], 1u << (j & 31));
        }
    const int nw = blockDim.x / kWave;
    int64_t np = 0;
    double kn = 0.0;
    for (int64_t pa = a_rp[row] + wave_id(); pa < a_rp[row + 1]; pa += nw) {
        const int32_t kb = a_ci[pa];
        const int64_t q0 = b_rp[kb], q1 = b_rp[kb + 1];
        const double k = (double)kbs[kb];
        for (int64_t q = q0 + lane_id(); q < q1; q += kWave) {
            const int32_t j = b_ci[q];
            atomicOr(&bm[j >> 5], 1u << (j & 31));
            np += 1;
            kn += k * (double)cbs[j];
        }
    }
    *nprod = np;
    *kn_sum = kn;
    __syncthreads();
}

__global__ __launch_bounds__(kRowThreads) void k_symbolic_count(
    int32_t nbr, int32_t nbc, const int64_t *a_rp, const int32_t *a_ci, const int64_t *b_rp,
    const int32_t *b_ci, const int64_t *c_rp, const int32_t *c_ci, const int32_t *rbs,
    const int32_t *kbs, const int32_t *cbs, int64_t *row_nnz, int64_t *row_elems,
    int64_t *row_prod, double *row_flops) {
    extern __shared__ uint32_t bm[];
    __shared__ int64_t red_i[16];
    __shared__ double red_d[16];
    const int nwords = (nbc + 31) >> 5;
    for (int32_t row = blockIdx.x; row < nbr; row += gridDim.x) {
        int64_t np;
        double kn;
        mark_row(bm, nwords, row, a_rp, a_ci, b_rp, b_ci, c_rp, c_ci, kbs, cbs, &np, &kn);
        int64_t cnt = 0, cols = 0;
        for (int w = threadIdx.x; w < nwords; w += blockDim.x) {
            uint32_t bits = bm[w];
            cnt += __popc(bits);
            while (bits) {
                const int b = __ffs(bits) - 1;
                bits &= bits - 1;
                cols += cbs[(w << 5) + b];
            }
        }
        cnt = block_sum(cnt, red_i);
        cols = block_sum(cols, red_i);
        np = block_sum(np, red_i);
        kn = block_sum(kn, red_d);
        if (threadIdx.x == 0) {
            const int64_t m = rbs[row];
            row_nnz[row] = cnt;
            row_elems[row] = m * cols;
            row_prod[row] = np;
            row_flops[row] = 2.0 * (double)m * kn;
        }
        __syncthreads();  // the bitmap is cleared for the next row
    }
}

__global__ __launch_bounds__(kRowThreads) void k_symbolic_fill(
    int32_t nbr, int32_t nbc, const int64_t *a_rp, const int32_t *a_ci, const int64_t *b_rp,
    const int32_t *b_ci, const int64_t *c_rp, const int32_t *c_ci, const int32_t *kbs,
    const int32_t *cbs, const int64_t *new_rp, int32_t *new_ci) {
    extern __shared__ uint32_t bm[];
    __shared__ int64_t red[16];
    const int nwords = (nbc + 31) >> 5;
    for (int32_t row = blockIdx.x; row < nbr; row += gridDim.x) {
        int64_t np;
        double kn;
        mark_row(bm, nwords, row, a_rp, a_ci, b_rp, b_ci, c_rp, c_ci, kbs, cbs, &np, &kn);
        int64_t out = new_rp[row];
        for (int w0 = 0; w0 < nwords; w0 += blockDim.x) {
            const int w = w0 + threadIdx.x;
            const uint32_t bits = w < nwords ? bm[w] : 0u;
            int64_t total;
            const int64_t pos = out + block_exclusive_scan((int64_t)__popc(bits), red, &total);
            uint32_t b = bits;
            int64_t k = 0;
            while (b) {
                const int bit = __ffs(b) - 1;
                b &= b - 1;
                new_ci[pos + k] = (w << 5) + bit;
                ++k;
            }
            out += total;
        }
        __syncthreads();  // the bitmap is cleared for the next row
    }
}

// ------------------------------------------------------ symbolic screen
// A C block whose norm bound |alpha| sum_K ||A_IK|| ||B_KJ|| + |beta| ||C_IJ||
// (Frobenius norms: triangle inequality and ||X Y|| <= ||X|| ||Y||) lies
// below eps is certain to fail the filter, so it is left out of the pattern
// and its products are never formed.  grow = 1 + margin, the margin
// covering the rounding of the computed block (at most about n u relative
// to the bound for n accumulated terms), of the norms and of the bound.
// Bounds of 1e150 and above are kept (their squared norm could overflow),
// and so are NaN and infinite ones.
__device__ __forceinline__ bool screened_out(double bound, double eps, double grow) {
    return bound * grow < eps && bound < 1e150;
}

// k_symbolic_count with the screen: per block row, the column bitmap and
// the bound of every column in LDS; the kept columns go to bits (nwords
// 32-bit words per row) for the fill, with the counts of the kept blocks,
// of the screened ones and of the old C blocks screened.  Products and
// flops count every (I,K,J) of A*B.
__global__ __launch_bounds__(kRowThreads) void k_symbolic_count_screen(
    int32_t nbr, int32_t nbc, const int64_t *a_rp, const int32_t *a_ci, const int64_t *b_rp,
    const int32_t *b_ci, const int64_t *c_rp, const int32_t *c_ci, const int32_t *rbs,
    const int32_t *kbs, const int32_t *cbs, const double *a_nrm, const double *b_nrm,
    const double *c_nrm, double alpha_abs, double beta_abs, double eps, double grow, uint32_t *bits,
    int64_t *row_nnz, int64_t *row_elems, int64_t *row_prod, double *row_flops,
    int64_t *row_screened, int64_t *row_old_screened) {
    extern __shared__ double bnd[];  // nbc bounds, then the bitmap
    uint32_t *bm = reinterpret_cast<uint32_t *>(bnd + nbc);
    __shared__ int64_t red_i[16];
    __shared__ double red_d[16];
    const int nwords = (nbc + 31) >> 5;
    const int nw = blockDim.x / kWave;
    for (int32_t row = blockIdx.x; row < nbr; row += gridDim.x) {
        for (int w = threadIdx.x; w < nwords; w += blockDim.x) bm[w] = 0u;
        for (int j = threadIdx.x; j < nbc; j += blockDim.x) bnd[j] = 0.0;
        __syncthreads();
        if (c_rp)
            for (int64_t p = c_rp[row] + threadIdx.x; p < c_rp[row + 1]; p += blockDim.x) {
                const int32_t j = c_ci[p];
                atomicOr(&bm[j >> 5], 1u << (j & 31));
                if (c_nrm) atomicAdd(&bnd[j], beta_abs * c_nrm[p]);
            }
        int64_t np = 0;
        double kn = 0.0;
        for (int64_t pa = a_rp[row] + wave_id(); pa < a_rp[row + 1]; pa += nw) {
            const int32_t kb = a_ci[pa];
            const double k = (double)kbs[kb], na = alpha_abs * a_nrm[pa];
            for (int64_t q = b_rp[kb] + lane_id(); q < b_rp[kb + 1]; q += kWave) {
                const int32_t j = b_ci[q];
                atomicOr(&bm[j >> 5], 1u << (j & 31));
                atomicAdd(&bnd[j], na * b_nrm[q]);
                np += 1;
                kn += k * (double)cbs[j];
            }
        }
        __syncthreads();
        int64_t cnt = 0, cols = 0, scr = 0, old_scr = 0;
        for (int w = threadIdx.x; w < nwords; w += blockDim.x) {
            const uint32_t all = bm[w];
            uint32_t keep = all, rest = all;
            while (rest) {
                const int b = __ffs(rest) - 1;
                rest &= rest - 1;
                const int j = (w << 5) + b;
                if (screened_out(bnd[j], eps, grow)) keep &= ~(1u << b);
                else cols += cbs[j];
            }
            cnt += __popc(keep);
            scr += __popc(all) - __popc(keep);
            bits[(int64_t)row * nwords + w] = keep;
        }
        if (c_rp)
            for (int64_t p = c_rp[row] + threadIdx.x; p < c_rp[row + 1]; p += blockDim.x)
                if (screened_out(bnd[c_ci[p]], eps, grow)) old_scr += 1;
        cnt = block_sum(cnt, red_i);
        cols = block_sum(cols, red_i);
        scr = block_sum(scr, red_i);
        old_scr = block_sum(old_scr, red_i);
        np = block_sum(np, red_i);
        kn = block_sum(kn, red_d);
        if (threadIdx.x == 0) {
            const int64_t m = rbs[row];
            row_nnz[row] = cnt;
            row_elems[row] = m * cols;
            row_prod[row] = np;
            row_flops[row] = 2.0 * (double)m * kn;
            row_screened[row] = scr;
            row_old_screened[row] = old_scr;
        }
        __syncthreads();  // bounds and bitmap are cleared for the next row
    }
}

// The kept columns of every row (bits of k_symbolic_count_screen), in
// ascending order.
__global__ __launch_bounds__(kRowThreads) void k_symbolic_fill_bits(int32_t nbr, int32_t nwords,
                                                                    const uint32_t *bits,
                                                                    const int64_t *new_rp,
                                                                    int32_t *new_ci) {
    __shared__ int64_t red[16];
    for (int32_t row = blockIdx.x; row < nbr; row += gridDim.x) {
        int64_t out = new_rp[row];
        for (int w0 = 0; w0 < nwords; w0 += blockDim.x) {
            const int w = w0 + threadIdx.x;
            const uint32_t word = w < nwords ? bits[(int64_t)row * nwords + w] : 0u;
            int64_t total;
            const int64_t pos = out + block_exclusive_scan((int64_t)__popc(word), red, &total);
            uint32_t b = word;
            int64_t k = 0;
            while (b) {
                const int bit = __ffs(b) - 1;
                b &= b - 1;
                new_ci[pos + k] = (w << 5) + bit;
                ++k;
            }
            out += total;
        }
    }
}

__global__ __launch_bounds__(256) void k_full_pattern(int32_t nbr, int32_t nbc, int64_t *rp,
                                                      int32_t *ci, int64_t *row_elems,
                                                      const int32_t *rbs, int64_t ncols) {
    const int64_t total = (int64_t)nbr * nbc;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x)
        ci[e] = (int32_t)(e % nbc);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= nbr;
         i += (int64_t)gridDim.x * blockDim.x) {
        rp[i] = i * nbc;
        if (i < nbr) row_elems[i] = (int64_t)rbs[i] * ncols;
    }
}

// ---------------------------------------------------------- relayout
// One workgroup per new block row; each wave copies whole blocks: the old
// block (found by binary search in the old row) or zeros.
template <class T>
__global__ __launch_bounds__(256) void k_relayout(int32_t nbr, const int32_t *rbs, const int32_t *cbs,
                                                  const int64_t *o_rp, const int32_t *o_ci,
                                                  const int64_t *o_off, const T *o_data,
                                                  const int64_t *n_rp, const int32_t *n_ci,
                                                  const int64_t *n_off, T *n_data) {
    const int nw = blockDim.x / kWave;
    for (int32_t row = blockIdx.x; row < nbr; row += gridDim.x) {
        const int64_t m = rbs[row];
        for (int64_t p = n_rp[row] + wave_id(); p < n_rp[row + 1]; p += nw) {
            const int32_t j = n_ci[p];
            int64_t lo = o_rp[row], hi = o_rp[row + 1], found = -1;
            while (lo < hi) {
                const int64_t mid = lo + (hi - lo) / 2;
                const int32_t c = o_ci[mid];
                if (c < j) lo = mid + 1;
                else if (c > j) hi = mid;
                else { found = mid; break; }
            }
            const int64_t len = m * cbs[j];
            T *dst = n_data + n_off[p];
            if (found >= 0) {
                const T *src = o_data + o_off[found];
                for (int64_t e = lane_id(); e < len; e += kWave) dst[e] = src[e];
            } else {
                for (int64_t e = lane_id(); e < len; e += kWave) dst[e] = T(0);
            }
        }
    }
}

// Block row of every block: one workgroup per block row.
__global__ __launch_bounds__(256) void k_block_rows(int32_t nbr, const int64_t *rp, int32_t *row) {
    for (int32_t r = blockIdx.x; r < nbr; r += gridDim.x)
        for (int64_t p = rp[r] + threadIdx.x; p < rp[r + 1]; p += blockDim.x) row[p] = r;
}

// One wave per block: data *= beta, or zeros when beta == 0, for the blocks
// whose flag is zero.  With gaps in the storage (blk_row non-null) a block's
// size comes from its block sizes, else from the offsets.
template <class T>
__global__ __launch_bounds__(256) void k_scale_blocks(int64_t nnzb, const int64_t *blk_off,
                                                      const int32_t *blk_row, const int32_t *rbs,
                                                      const int32_t *cbs, const int32_t *ci,
                                                      const int64_t *flags, T beta, T *data) {
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
    for (int64_t b = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave_id(); b < nnzb; b += waves) {
        if (flags && flags[b] != 0) continue;
        T *d = data + blk_off[b];
        const int64_t len = blk_row ? (int64_t)rbs[blk_row[b]] * cbs[ci[b]] : blk_off[b + 1] - blk_off[b];
        if (beta == T(0))
            for (int64_t e = lane_id(); e < len; e += kWave) d[e] = T(0);
        else
            for (int64_t e = lane_id(); e < len; e += kWave) d[e] *= beta;
    }
}

__global__ __launch_bounds__(256) void k_fill_zero(double *p, int64_t n) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x)
        p[e] = 0.0;
}

__global__ __launch_bounds__(256) void k_fill_value(double *p, int64_t n, double v) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x)
        p[e] = v;
}

__global__ __launch_bounds__(256) void k_fill_zero_u32(uint32_t *p, int64_t n) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x)
        p[e] = 0u;
}

}  // namespace

// ------------------------------------------------------------- host side
int build_block_offsets(const int32_t *d_rbs, const int32_t *d_cbs, int32_t nbr,
                        const int64_t *d_row_ptr, const int32_t *d_col_ind, int64_t nnzb,
                        int64_t *d_blk_off, const int64_t *d_row_elems, hipStream_t s) {
    (void)nnzb;
    if (nbr == 0) {
        hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(1), 0, s, d_blk_off, (int64_t)0);
        return launch_check("set_i64");
    }
    DevBuf row_elems, row_base;
    BSMM_TRY(row_base.reserve(sizeof(int64_t) * (nbr + 1), s));
    if (!d_row_elems) {
        BSMM_TRY(row_elems.reserve(sizeof(int64_t) * (nbr + 1), s));
        hipLaunchKernelGGL(k_row_elems, dim3(grid_of(nbr, 4)), dim3(256), 0, s, d_rbs, d_cbs, nbr,
                           d_row_ptr, d_col_ind, row_elems.as<int64_t>());
        BSMM_TRY(launch_check("row_elems"));
        d_row_elems = row_elems.as<int64_t>();
    }
    BSMM_TRY(scan_exclusive_i64(d_row_elems, row_base.as<int64_t>(), nbr, s));
    hipLaunchKernelGGL(k_block_offsets, dim3(grid_of(nbr, 4)), dim3(256), 0, s, d_rbs, d_cbs, nbr,
                       d_row_ptr, d_col_ind, (const int64_t *)row_base.as<int64_t>(), d_blk_off);
    return launch_check("block_offsets");
}

static int bitmap_lds_bytes(int32_t nbc, size_t *bytes) {
    const int64_t nwords = (nbc + 31) / 32;
    if (nwords > kMaxBitmapWords) {
        set_error(BSMM_ENOTSUP, "more than %d block columns in C", kMaxBitmapWords * 32);
        return BSMM_ENOTSUP;
    }
    *bytes = (size_t)(nwords > 0 ? nwords : 1) * sizeof(uint32_t);
    return BSMM_OK;
}

int symbolic_count(const bsmm_matrix_s *A, const bsmm_matrix_s *B, const bsmm_matrix_s *C,
                   int64_t *d_row_nnz, int64_t *d_row_elems, int64_t *d_row_prod,
                   double *d_row_flops, hipStream_t s) {
    if (A->nbr == 0) return BSMM_OK;
    size_t lds;
    BSMM_TRY(bitmap_lds_bytes(B->nbc, &lds));
    const bool has_c = C && C->nnzb > 0;
    hipLaunchKernelGGL(k_symbolic_count, dim3(grid_rows(A->nbr)), dim3(kRowThreads), lds, s, A->nbr, B->nbc,
                       A->d_row_ptr(), A->d_col_ind(), B->d_row_ptr(), B->d_col_ind(),
                       has_c ? C->d_row_ptr() : nullptr, has_c ? C->d_col_ind() : nullptr,
                       A->d_rbs(), B->d_rbs(), B->d_cbs(), d_row_nnz, d_row_elems, d_row_prod,
                       d_row_flops);
    return launch_check("symbolic_count");
}

int symbolic_fill(const bsmm_matrix_s *A, const bsmm_matrix_s *B, const bsmm_matrix_s *C,
                  const int64_t *d_new_row_ptr, int32_t *d_new_col_ind, hipStream_t s) {
    if (A->nbr == 0) return BSMM_OK;
    size_t lds;
    BSMM_TRY(bitmap_lds_bytes(B->nbc, &lds));
    const bool has_c = C && C->nnzb > 0;
    hipLaunchKernelGGL(k_symbolic_fill, dim3(grid_rows(A->nbr)), dim3(kRowThreads), lds, s, A->nbr, B->nbc,
                       A->d_row_ptr(), A->d_col_ind(), B->d_row_ptr(), B->d_col_ind(),
                       has_c ? C->d_row_ptr() : nullptr, has_c ? C->d_col_ind() : nullptr,
                       B->d_rbs(), B->d_cbs(), d_new_row_ptr, d_new_col_ind);
    return launch_check("symbolic_fill");
}

int symbolic_count_screen(const bsmm_matrix_s *A, const bsmm_matrix_s *B, const bsmm_matrix_s *C,
                          const ScreenNorms &sn, uint32_t *d_bits, int64_t *d_row_nnz,
                          int64_t *d_row_elems, int64_t *d_row_prod, double *d_row_flops,
                          int64_t *d_row_screened, int64_t *d_row_old_screened, hipStream_t s) {
    if (A->nbr == 0) return BSMM_OK;
    const int32_t nbc = B->nbc;
    if (nbc > kScreenMaxCols) {
        set_error(BSMM_ENOTSUP, "symbolic screen: more than %d block columns", kScreenMaxCols);
        return BSMM_ENOTSUP;
    }
    const size_t lds = sizeof(double) * (size_t)nbc + sizeof(uint32_t) * (size_t)((nbc + 31) / 32 + 1);
    const bool has_c = C && C->nnzb > 0;
    hipLaunchKernelGGL(k_symbolic_count_screen, dim3(grid_rows(A->nbr)), dim3(kRowThreads), lds, s,
                       A->nbr, nbc, A->d_row_ptr(), A->d_col_ind(), B->d_row_ptr(), B->d_col_ind(),
                       has_c ? C->d_row_ptr() : nullptr, has_c ? C->d_col_ind() : nullptr,
                       A->d_rbs(), B->d_rbs(), B->d_cbs(), sn.a, sn.b, has_c ? sn.c : nullptr,
                       sn.alpha_abs, sn.beta_abs, sn.eps, 1.0 + sn.margin, d_bits, d_row_nnz, d_row_elems,
                       d_row_prod, d_row_flops, d_row_screened, d_row_old_screened);
    return launch_check("symbolic_count_screen");
}

int symbolic_fill_bits(int32_t nbr, int32_t nbc, const uint32_t *d_bits, const int64_t *d_new_row_ptr,
                       int32_t *d_new_col_ind, hipStream_t s) {
    if (nbr == 0) return BSMM_OK;
    hipLaunchKernelGGL(k_symbolic_fill_bits, dim3(grid_rows(nbr)), dim3(kRowThreads), 0, s, nbr,
                       (nbc + 31) / 32, d_bits, d_new_row_ptr, d_new_col_ind);
    return launch_check("symbolic_fill_bits");
}

int full_pattern(int32_t nbr, int32_t nbc, int64_t ncols, int64_t *d_row_ptr,
                 int32_t *d_col_ind, int64_t *d_row_elems, const int32_t *d_rbs, hipStream_t s) {
    const int64_t total = (int64_t)nbr * nbc;
    hipLaunchKernelGGL(k_full_pattern, dim3(grid_of(std::max<int64_t>(total, nbr + 1), 256, 8192)),
                       dim3(256), 0, s, nbr, nbc, d_row_ptr, d_col_ind, d_row_elems, d_rbs, ncols);
    return launch_check("full_pattern");
}

int relayout(const bsmm_matrix_s *Cold, const int64_t *d_new_rp, const int32_t *d_new_ci,
             const int64_t *d_new_off, void *d_new_data, hipStream_t s) {
    if (Cold->nbr == 0) return BSMM_OK;
    if (Cold->dtype == BSMM_F32)
        hipLaunchKernelGGL(k_relayout<float>, dim3(grid_rows(Cold->nbr)), dim3(256), 0, s, Cold->nbr,
                           Cold->d_rbs(),
                           Cold->d_cbs(), Cold->d_row_ptr(), Cold->d_col_ind(), Cold->d_blk_off(),
                           (const float *)Cold->d_raw(), d_new_rp, d_new_ci, d_new_off,
                           (float *)d_new_data);
    else
        hipLaunchKernelGGL(k_relayout<double>, dim3(grid_rows(Cold->nbr)), dim3(256), 0, s, Cold->nbr,
                           Cold->d_rbs(),
                           Cold->d_cbs(), Cold->d_row_ptr(), Cold->d_col_ind(), Cold->d_blk_off(),
                           (const double *)Cold->d_raw(), d_new_rp, d_new_ci, d_new_off,
                           (double *)d_new_data);
    return launch_check("relayout");
}

int block_rows(const bsmm_matrix_s *M, DevBuf &out, hipStream_t s) {
    if (!M->holes || M->nnzb == 0) return BSMM_OK;
    BSMM_TRY(out.reserve(sizeof(int32_t) * M->nnzb, s));
    hipLaunchKernelGGL(k_block_rows, dim3(grid_rows(M->nbr)), dim3(256), 0, s, M->nbr, M->d_row_ptr(),
                       out.as<int32_t>());
    return launch_check("block_rows");
}

int scale_blocks(const bsmm_matrix_s *C, const int64_t *d_flags, double beta, hipStream_t s) {
    if (C->nnzb == 0) return BSMM_OK;
    DevBuf rows;
    BSMM_TRY(block_rows(C, rows, s));
    const int32_t *r = rows.as<int32_t>();
    if (C->dtype == BSMM_F32)
        hipLaunchKernelGGL(k_scale_blocks<float>, dim3(grid_of(C->nnzb, 4)), dim3(256), 0, s, C->nnzb,
                           C->d_blk_off(), r, C->d_rbs(), C->d_cbs(), C->d_col_ind(), d_flags,
                           (float)beta, (float *)C->d_raw());
    else
        hipLaunchKernelGGL(k_scale_blocks<double>, dim3(grid_of(C->nnzb, 4)), dim3(256), 0, s,
                           C->nnzb, C->d_blk_off(), r, C->d_rbs(), C->d_cbs(), C->d_col_ind(), d_flags,
                           beta, (double *)C->d_raw());
    return launch_check("scale_blocks");
}

int fill_zero(double *p, int64_t n, hipStream_t s) {
    if (n <= 0) return BSMM_OK;
    hipLaunchKernelGGL(k_fill_zero, dim3(grid_of(n, 256, 16384)), dim3(256), 0, s, p, n);
    return launch_check("fill_zero");
}

int fill_value(double *p, int64_t n, double v, hipStream_t s) {
    if (n <= 0) return BSMM_OK;
    hipLaunchKernelGGL(k_fill_value, dim3(grid_of(n, 256, 16384)), dim3(256), 0, s, p, n, v);
    return launch_check("fill_value");
}

int fill_zero_bytes(void *p, size_t bytes, hipStream_t s) {
    if (bytes == 0) return BSMM_OK;
    if (bytes % sizeof(double) == 0) return fill_zero((double *)p, (int64_t)(bytes / sizeof(double)), s);
    hipLaunchKernelGGL(k_fill_zero_u32, dim3(grid_of((int64_t)(bytes / 4), 256, 16384)), dim3(256), 0, s,
                       (uint32_t *)p, (int64_t)(bytes / 4));
    return launch_check("fill_zero_u32");
}

}  // namespace bsmm
