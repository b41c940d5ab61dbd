// scan.hip -- device exclusive prefix sums (three-phase, recursive).
#include "dev_util.h"
#include "internal.h"

namespace bsmm {

namespace {
constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;

// Each workgroup scans one tile of 1024 values; tile totals go to sums[].
__global__ __launch_bounds__(kScanThreads) void k_scan_tile(const int64_t *in, int64_t *out,
                                                              int64_t n, int64_t *sums,
                                                              int write_total) {
    __shared__ int64_t lds[16];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t v[kScanItems];
    int64_t local = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        v[i] = (base + i < n) ? in[base + i] : 0;
        local += v[i];
    }
    int64_t total;
    int64_t run = block_exclusive_scan(local, lds, &total);
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        if (base + i < n) out[base + i] = run;
        run += v[i];
    }
    if (threadIdx.x == 0) {
        if (sums) sums[blockIdx.x] = total;
        if (write_total) out[n] = total;
    }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_add(int64_t *out, int64_t n,
                                                             const int64_t *offs) {
    const int64_t add = offs[blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    for (int i = threadIdx.x; i < kScanTile; i += kScanThreads)
        if (base + i < n) out[base + i] += add;
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = offs[gridDim.x];
}

__global__ void k_set_zero_i64(int64_t *p) { *p = 0; }
}  // namespace

int scan_exclusive_i64(const int64_t *in, int64_t *out, int64_t n, hipStream_t s) {
    if (n <= 0) {
        hipLaunchKernelGGL(k_set_zero_i64, dim3(1), dim3(1), 0, s, out);
        return launch_check("scan_zero");
    }
    const int64_t tiles = ceil_div(n, kScanTile);
    if (tiles == 1) {
        hipLaunchKernelGGL(k_scan_tile, dim3(1), dim3(kScanThreads), 0, s, in, out, n,
                           (int64_t *)nullptr, 1);
        return launch_check("scan_tile");
    }
    DevBuf sums;
    BSMM_TRY(sums.reserve(sizeof(int64_t) * (tiles + 1), s));
    hipLaunchKernelGGL(k_scan_tile, dim3((unsigned)tiles), dim3(kScanThreads), 0, s, in, out, n,
                       sums.as<int64_t>(), 0);
    BSMM_TRY(launch_check("scan_tile"));
    BSMM_TRY(scan_exclusive_i64(sums.as<int64_t>(), sums.as<int64_t>(), tiles, s));
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)tiles), dim3(kScanThreads), 0, s, out, n,
                       (const int64_t *)sums.as<int64_t>());
    return launch_check("scan_add");
}

}  // namespace bsmm
