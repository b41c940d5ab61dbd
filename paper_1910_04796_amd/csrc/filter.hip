// filter.hip -- post-multiply block filter: drop every C block whose squared
// Frobenius norm is strictly below eps^2 (a NaN norm keeps the block), then
// compact C's index; the kept blocks' data stay in place (the dropped
// blocks leave gaps) unless most of the storage would be gaps.
#include "dev_util.h"
#include "internal.h"

namespace bsmm {

namespace {

// Elements of block b: from the offsets of packed storage, else (blk_row
// non-null) from the block's row and column sizes.
__device__ __forceinline__ int64_t block_len(int64_t b, const int64_t *blk_off, const int32_t *blk_row,
                                             const int32_t *rbs, const int32_t *cbs, const int32_t *ci) {
    return blk_row ? (int64_t)rbs[blk_row[b]] * cbs[ci[b]] : blk_off[b + 1] - blk_off[b];
}

// Keep flag and kept element count of every block.  A wave takes 64
// consecutive blocks, one per lane: a block whose squared norm the
// small-block kernel handed over (pre[b] >= 0, or NaN) is decided by its
// lane; the others are summed by the whole wave, one block at a time
// (squares summed in FP64 for either element type).
template <class T>
__global__ __launch_bounds__(256) void k_norm_keep(int64_t nnzb, const int64_t *blk_off,
                                                   const int32_t *blk_row, const int32_t *rbs,
                                                   const int32_t *cbs, const int32_t *ci,
                                                   const T *data, const double *pre, double eps2,
                                                   int64_t *keep, int64_t *keep_elems) {
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
    for (int64_t base = ((int64_t)blockIdx.x * (blockDim.x / kWave) + wave_id()) * kWave; base < nnzb;
         base += waves * kWave) {
        const int64_t b = base + lane_id();
        const bool in = b < nnzb;
        const int64_t len = in ? block_len(b, blk_off, blk_row, rbs, cbs, ci) : 0;
        double ss = in && pre ? pre[b] : -1.0;
        uint64_t need = __ballot(in && ss < 0.0);
        while (need) {
            const int l = __ffsll((unsigned long long)need) - 1;
            need &= need - 1;
            const int64_t bb = base + l;
            const int64_t o = blk_off[bb], n = block_len(bb, blk_off, blk_row, rbs, cbs, ci);
            // Four independent partial sums per lane keep four loads in flight.
            double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
            int64_t e = lane_id();
            for (; e + 3 * kWave < n; e += 4 * kWave) {
                const double x0 = (double)data[o + e], x1 = (double)data[o + e + kWave];
                const double x2 = (double)data[o + e + 2 * kWave], x3 = (double)data[o + e + 3 * kWave];
                s0 = fma(x0, x0, s0);
                s1 = fma(x1, x1, s1);
                s2 = fma(x2, x2, s2);
                s3 = fma(x3, x3, s3);
            }
            for (; e < n; e += kWave) {
                const double x = (double)data[o + e];
                s0 = fma(x, x, s0);
            }
            const double sum = wave_sum((s0 + s1) + (s2 + s3));
            if (lane_id() == l) ss = sum;
        }
        if (in) {
            const int64_t k = (ss < eps2) ? 0 : 1;  // a NaN norm keeps the block
            keep[b] = k;
            keep_elems[b] = k ? len : 0;
        }
    }
}

__global__ __launch_bounds__(256) void k_new_row_ptr(int32_t nbr, int64_t nnzb, const int64_t *rp,
                                                     const int64_t *kpos, int64_t *new_rp,
                                                     int64_t *new_off, int64_t total_elems) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= nbr;
         i += (int64_t)gridDim.x * blockDim.x) {
        new_rp[i] = kpos[rp[i]];
        if (i == 0) new_off[kpos[nnzb]] = total_elems;
    }
}

// One thread per old block: the kept blocks' column indices and data
// offsets move to their new index positions; the data stay in place.
__global__ __launch_bounds__(256) void k_keep_index(int64_t nnzb, const int32_t *ci,
                                                    const int64_t *blk_off, const int64_t *kpos,
                                                    int32_t *new_ci, int64_t *new_off) {
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nnzb;
         b += (int64_t)gridDim.x * blockDim.x) {
        if (kpos[b + 1] == kpos[b]) continue;  // dropped
        new_ci[kpos[b]] = ci[b];
        new_off[kpos[b]] = blk_off[b];
    }
}

// One wave per old block: kept blocks move to their packed place (len:
// kept element counts, zero for dropped blocks).
template <class T>
__global__ __launch_bounds__(256) void k_compact(int64_t nnzb, const int32_t *ci,
                                                 const int64_t *blk_off, const int64_t *kept_len,
                                                 const T *data, const int64_t *kpos,
                                                 const int64_t *epos, int32_t *new_ci,
                                                 int64_t *new_off, T *new_data) {
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
    for (int64_t b = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave_id(); b < nnzb; b += waves) {
        if (kpos[b + 1] == kpos[b]) continue;  // dropped
        const int64_t nb = kpos[b];
        const int64_t o = blk_off[b], len = kept_len[b], no = epos[b];
        if (lane_id() == 0) {
            new_ci[nb] = ci[b];
            new_off[nb] = no;
        }
        int64_t e = lane_id();
        for (; e + 3 * kWave < len; e += 4 * kWave) {
            const T x0 = data[o + e], x1 = data[o + e + kWave];
            const T x2 = data[o + e + 2 * kWave], x3 = data[o + e + 3 * kWave];
            new_data[no + e] = x0;
            new_data[no + e + kWave] = x1;
            new_data[no + e + 2 * kWave] = x2;
            new_data[no + e + 3 * kWave] = x3;
        }
        for (; e < len; e += kWave) new_data[no + e] = data[o + e];
    }
}

// One wave per block: the block's Frobenius norm in FP64, for the norm
// bound of the symbolic screen.  One pass sums the squares and finds
// max|x|; when max|x| lies in [2^-500, 2^500] no square overflows and the
// ones that underflow are negligible beside max|x|^2, so sqrt(sum) stands
// (relative rounding error below len * 2^-52).  Otherwise a second pass
// sums (x / max|x|)^2, and for max|x| below 2^-900 or above 2^900 the
// upper bound sqrt(len) * max|x| is taken.  A NaN element gives NaN, an
// infinite one infinity.
template <class T>
__global__ __launch_bounds__(256) void k_block_norm(int64_t nnzb, const int64_t *blk_off,
                                                    const int32_t *blk_row, const int32_t *rbs,
                                                    const int32_t *cbs, const int32_t *ci,
                                                    const T *data, double *out) {
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
    for (int64_t b = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave_id(); b < nnzb; b += waves) {
        const int64_t o = blk_off[b], len = block_len(b, blk_off, blk_row, rbs, cbs, ci);
        double mx = 0.0, ss = 0.0;
        int nan = 0;
        for (int64_t e = lane_id(); e < len; e += kWave) {
            const double x = (double)data[o + e], v = fabs(x);
            nan |= v != v;
            mx = v > mx ? v : mx;
            ss = fma(x, x, ss);
        }
        mx = wave_max(mx);
        nan = __any(nan);
        double nrm;
        if (nan) {
            nrm = __builtin_nan("");
        } else if (mx >= 0x1p-500 && mx <= 0x1p500) {
            nrm = sqrt(wave_sum(ss));
        } else if (mx == 0.0 || mx > 0x1p900 || mx < 0x1p-900) {
            nrm = mx * sqrt((double)len);  // also 0 and infinity
        } else {
            const double r = 1.0 / mx;
            double sc = 0.0;
            for (int64_t e = lane_id(); e < len; e += kWave) {
                const double v = (double)data[o + e] * r;
                sc = fma(v, v, sc);
            }
            nrm = mx * sqrt(wave_sum(sc));
        }
        if (lane_id() == 0) out[b] = nrm;
    }
}

}  // namespace

int block_norms(const bsmm_matrix_s *M, double *d_out, hipStream_t s) {
    if (M->nnzb == 0) return BSMM_OK;
    DevBuf rows;
    BSMM_TRY(block_rows(M, rows, s));
    const int32_t *r = rows.as<int32_t>();
    if (M->dtype == BSMM_F32)
        hipLaunchKernelGGL(k_block_norm<float>, dim3(grid_of(M->nnzb, 4)), dim3(256), 0, s, M->nnzb,
                           M->d_blk_off(), r, M->d_rbs(), M->d_cbs(), M->d_col_ind(),
                           (const float *)M->d_raw(), d_out);
    else
        hipLaunchKernelGGL(k_block_norm<double>, dim3(grid_of(M->nnzb, 4)), dim3(256), 0, s, M->nnzb,
                           M->d_blk_off(), r, M->d_rbs(), M->d_cbs(), M->d_col_ind(),
                           (const double *)M->d_raw(), d_out);
    return launch_check("block_norm");
}

int filter_blocks(bsmm_matrix_s *C, double eps, int64_t *nnzb_after, hipStream_t s,
                  const double *pre_norm2) {
    *nnzb_after = C->nnzb;
    if (!(eps > 0.0) || C->nnzb == 0) return BSMM_OK;
    const int64_t nnzb = C->nnzb;
    DevBuf keep, kel, kpos, epos, rows;
    BSMM_TRY(keep.reserve(sizeof(int64_t) * (nnzb + 1), s));
    BSMM_TRY(kel.reserve(sizeof(int64_t) * (nnzb + 1), s));
    BSMM_TRY(kpos.reserve(sizeof(int64_t) * (nnzb + 1), s));
    BSMM_TRY(epos.reserve(sizeof(int64_t) * (nnzb + 1), s));
    BSMM_TRY(block_rows(C, rows, s));
    const int32_t *r = rows.as<int32_t>();
    if (C->dtype == BSMM_F32)
        hipLaunchKernelGGL(k_norm_keep<float>, dim3(grid_of(ceil_div(nnzb, kWave), 4)), dim3(256), 0, s, nnzb,
                           C->d_blk_off(), r, C->d_rbs(), C->d_cbs(), C->d_col_ind(),
                           (const float *)C->d_raw(), pre_norm2, eps * eps, keep.as<int64_t>(),
                           kel.as<int64_t>());
    else
        hipLaunchKernelGGL(k_norm_keep<double>, dim3(grid_of(ceil_div(nnzb, kWave), 4)), dim3(256), 0, s, nnzb,
                           C->d_blk_off(), r, C->d_rbs(), C->d_cbs(), C->d_col_ind(),
                           (const double *)C->d_raw(), pre_norm2, eps * eps, keep.as<int64_t>(),
                           kel.as<int64_t>());
    BSMM_TRY(launch_check("norm_keep"));
    BSMM_TRY(scan_exclusive_i64(keep.as<int64_t>(), kpos.as<int64_t>(), nnzb, s));
    BSMM_TRY(scan_exclusive_i64(kel.as<int64_t>(), epos.as<int64_t>(), nnzb, s));
    int64_t tot[2];
    BSMM_HIP(hipMemcpyAsync(&tot[0], kpos.as<int64_t>() + nnzb, sizeof(int64_t),
                            hipMemcpyDeviceToHost, s));
    BSMM_HIP(hipMemcpyAsync(&tot[1], epos.as<int64_t>() + nnzb, sizeof(int64_t),
                            hipMemcpyDeviceToHost, s));
    BSMM_HIP(hipStreamSynchronize(s));
    const int64_t new_nnzb = tot[0], new_elems = tot[1];
    *nnzb_after = new_nnzb;
    if (new_nnzb == nnzb) return BSMM_OK;

    // The index always shrinks; the data move only when the gaps would be
    // most of the storage (memory back), otherwise they stay in place.
    const bool pack = new_elems < C->storage / 2;
    DevBuf n_rp, n_ci, n_off, n_data;
    BSMM_TRY(n_rp.reserve(sizeof(int64_t) * (C->nbr + 1), s));
    BSMM_TRY(n_ci.reserve(sizeof(int32_t) * (new_nnzb + 1), s));
    BSMM_TRY(n_off.reserve(sizeof(int64_t) * (new_nnzb + 1), s));
    if (pack) BSMM_TRY(n_data.reserve(C->esize() * (new_elems + 1), s));
    hipLaunchKernelGGL(k_new_row_ptr, dim3(grid_of(C->nbr + 1, 256)), dim3(256), 0, s, C->nbr,
                       nnzb, C->d_row_ptr(), (const int64_t *)kpos.as<int64_t>(), n_rp.as<int64_t>(),
                       n_off.as<int64_t>(), pack ? new_elems : C->storage);
    BSMM_TRY(launch_check("new_row_ptr"));
    if (!pack) {
        hipLaunchKernelGGL(k_keep_index, dim3(grid_of(nnzb, 256)), dim3(256), 0, s, nnzb,
                           C->d_col_ind(), C->d_blk_off(), (const int64_t *)kpos.as<int64_t>(),
                           n_ci.as<int32_t>(), n_off.as<int64_t>());
        BSMM_TRY(launch_check("keep_index"));
    } else if (C->dtype == BSMM_F32) {
        hipLaunchKernelGGL(k_compact<float>, dim3(grid_of(nnzb, 4)), dim3(256), 0, s, nnzb,
                           C->d_col_ind(), C->d_blk_off(), (const int64_t *)kel.as<int64_t>(),
                           (const float *)C->d_raw(), (const int64_t *)kpos.as<int64_t>(),
                           (const int64_t *)epos.as<int64_t>(), n_ci.as<int32_t>(), n_off.as<int64_t>(),
                           n_data.as<float>());
    } else {
        hipLaunchKernelGGL(k_compact<double>, dim3(grid_of(nnzb, 4)), dim3(256), 0, s, nnzb,
                           C->d_col_ind(), C->d_blk_off(), (const int64_t *)kel.as<int64_t>(),
                           (const double *)C->d_raw(), (const int64_t *)kpos.as<int64_t>(),
                           (const int64_t *)epos.as<int64_t>(), n_ci.as<int32_t>(), n_off.as<int64_t>(),
                           n_data.as<double>());
    }
    if (pack) BSMM_TRY(launch_check("compact"));
    C->b_row_ptr = std::move(n_rp);
    C->b_col_ind = std::move(n_ci);
    C->b_blk_off = std::move(n_off);
    if (pack) {
        C->b_data = std::move(n_data);
        C->storage = new_elems;
    }
    C->holes = !pack;
    C->nnzb = new_nnzb;
    C->nelems = new_elems;
    C->version = next_version();
    return BSMM_OK;
}

}  // namespace bsmm
