// peaks.hip -- microbenchmarks of the device rates the rooflines are
// measured against: FP64, FP32, INT8 and BF16 matrix-core throughput on
// register operands, FP64 vector FMA throughput, and HBM copy bandwidth.
//
// Each compute kernel runs a long loop of independent accumulation chains
// per wave (no memory traffic inside the loop) on 32 waves per CU, and
// writes its accumulators once at the end (to a buffer the host never
// reads) so that the loop is not removed.  The copy and read kernels
// stream 16-byte loads (four in flight per thread) over buffers of
// copy_bytes each.
#include "dev_util.h"
#include "internal.h"
#include "mfma_util.h"

namespace bsmm {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int kChains = 16;  // independent accumulators per wave (FP64 / FP32 MFMA)

// At least two workgroups per CU: with one, the compiler keeps the loop's
// accumulators in VGPRs but runs the MFMAs on AGPR copies, moving all of
// them back and forth every iteration (about half the rate).
__global__ __launch_bounds__(256, 2) void k_peak_f64_mfma(int iters, double seed, double *out) {
    v4d_t acc[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc[c] = (v4d_t){0.0, 0.0, 0.0, 0.0};
    const double a = seed + lane_id(), b = seed - lane_id();
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int c = 0; c < kChains; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_peak_f32_mfma(int iters, float seed, float *out) {
    v4f_t acc[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc[c] = (v4f_t){0.0f, 0.0f, 0.0f, 0.0f};
    const float a = seed + lane_id(), b = seed - lane_id();
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int c = 0; c < kChains; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[c], 0, 0, 0);
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_peak_i8_mfma(int iters, int seed, int *out) {
    v16i acc[2];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[c][e] = 0;
    const v4i a = (v4i){seed, seed + lane_id(), seed - 1, lane_id()};
    const v4i b = (v4i){lane_id(), seed, seed + 2, seed - lane_id()};
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int c = 0; c < 2; ++c) acc[c] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, acc[c], 0, 0, 0);
    int s = 0;
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int e = 0; e < 16; ++e) s += acc[c][e];
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_peak_bf16_mfma(int iters, float seed, float *out) {
    v16f acc[2];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[c][e] = 0.0f;
    v8bf a, b;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        a[e] = (__bf16)(seed + e + lane_id());
        b[e] = (__bf16)(seed - e);
    }
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int c = 0; c < 2; ++c) acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[c], 0, 0, 0);
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int e = 0; e < 16; ++e) s += acc[c][e];
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

constexpr int kFmaChains = 8;

__global__ __launch_bounds__(256) void k_peak_f64_valu(int iters, double seed, double *out) {
    double acc[kFmaChains];
#pragma unroll
    for (int c = 0; c < kFmaChains; ++c) acc[c] = seed + c;
    const double a = 1.0 - 1e-9 * lane_id(), b = 1e-9;
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int c = 0; c < kFmaChains; ++c) acc[c] = fma(acc[c], a, b);
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < kFmaChains; ++c) s += acc[c];
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// Four 16-byte loads in flight per thread and round.
__global__ __launch_bounds__(256) void k_peak_copy(const v4i *src, v4i *dst, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
        const v4i a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
        dst[i] = a;
        dst[i + stride] = b;
        dst[i + 2 * stride] = c;
        dst[i + 3 * stride] = d;
    }
    for (; i < n; i += stride) dst[i] = src[i];
}

// Reads only: four 16-byte loads in flight per thread and round, folded
// into one value per thread.
__global__ __launch_bounds__(256) void k_peak_read(const v4i *src, int64_t n, int *out) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    v4i x = (v4i){0, 0, 0, 0};
    for (; i + 3 * stride < n; i += 4 * stride)
        x ^= src[i] ^ src[i + stride] ^ src[i + 2 * stride] ^ src[i + 3 * stride];
    for (; i < n; i += stride) x ^= src[i];
    out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = x[0] ^ x[1] ^ x[2] ^ x[3];
}

// Device time (ms) of one launch, after one untimed launch.
template <class F> int time_ms(hipStream_t s, F launch, float *ms) {
    hipEvent_t e0, e1;
    BSMM_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        set_error(BSMM_EDEVICE, "hipEventCreate failed");
        return BSMM_EDEVICE;
    }
    launch();
    (void)hipEventRecord(e0, s);
    launch();
    (void)hipEventRecord(e1, s);
    const hipError_t e = hipEventSynchronize(e1);
    if (e == hipSuccess) (void)hipEventElapsedTime(ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess || hipPeekAtLastError() != hipSuccess) {
        set_error(BSMM_EDEVICE, "peak microbenchmark failed: %s", hipGetErrorString(hipGetLastError()));
        return BSMM_EDEVICE;
    }
    return BSMM_OK;
}

}  // namespace

}  // namespace bsmm

using namespace bsmm;

extern "C" int bsmm_measure_peaks(double *fp64_mfma, double *fp32_mfma, double *int8_mfma,
                                  double *bf16_mfma, double *fp64_valu, double *hbm_gbs,
                                  double *hbm_read_gbs, int64_t copy_bytes, void *stream) {
    clear_error();
    if (copy_bytes < 0 || copy_bytes > (int64_t(64) << 30)) {
        set_error(BSMM_EINVAL, "copy_bytes must be in [0, 64 GiB]");
        return BSMM_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    const int cus = cu_count();
    const unsigned grid = (unsigned)cus * 8;  // 8 workgroups of 4 waves: 32 waves per CU
    const double waves = (double)grid * 4;
    DevBuf out;
    BSMM_TRY(out.reserve(sizeof(double) * grid * 256, s));
    float ms = 0.0f;
    const int it = 20000;
    if (fp64_mfma) {
        BSMM_TRY(time_ms(s, [&] { hipLaunchKernelGGL(k_peak_f64_mfma, dim3(grid), dim3(256), 0, s, it, 1.0,
                                                     out.as<double>()); }, &ms));
        *fp64_mfma = waves * it * kChains * 2.0 * 16 * 16 * 4 / (ms * 1e-3) / 1e12;
    }
    if (fp32_mfma) {
        BSMM_TRY(time_ms(s, [&] { hipLaunchKernelGGL(k_peak_f32_mfma, dim3(grid), dim3(256), 0, s, it, 1.0f,
                                                     out.as<float>()); }, &ms));
        *fp32_mfma = waves * it * kChains * 2.0 * 16 * 16 * 4 / (ms * 1e-3) / 1e12;
    }
    if (int8_mfma) {
        BSMM_TRY(time_ms(s, [&] { hipLaunchKernelGGL(k_peak_i8_mfma, dim3(grid), dim3(256), 0, s, it, 1,
                                                     out.as<int>()); }, &ms));
        *int8_mfma = waves * it * 2 * 2.0 * 32 * 32 * 32 / (ms * 1e-3) / 1e12;
    }
    if (bf16_mfma) {
        BSMM_TRY(time_ms(s, [&] { hipLaunchKernelGGL(k_peak_bf16_mfma, dim3(grid), dim3(256), 0, s, it, 1.0f,
                                                     out.as<float>()); }, &ms));
        *bf16_mfma = waves * it * 2 * 2.0 * 32 * 32 * 16 / (ms * 1e-3) / 1e12;
    }
    if (fp64_valu) {
        BSMM_TRY(time_ms(s, [&] { hipLaunchKernelGGL(k_peak_f64_valu, dim3(grid), dim3(256), 0, s, it, 1.0,
                                                     out.as<double>()); }, &ms));
        *fp64_valu = waves * 64.0 * it * kFmaChains * 2.0 / (ms * 1e-3) / 1e12;
    }
    if ((hbm_gbs || hbm_read_gbs) && copy_bytes >= 16) {
        const int64_t n = copy_bytes / 16;
        DevBuf a, b;
        BSMM_TRY(a.reserve(16 * (size_t)n, s));
        BSMM_TRY(b.reserve(16 * (size_t)n, s));
        BSMM_TRY(fill_zero_bytes(a.p, 16 * (size_t)n, s));
        const unsigned cgrid = grid_of(n, 256 * 4, (int64_t)cus * 32);
        if (hbm_gbs) {
            BSMM_TRY(time_ms(s, [&] { hipLaunchKernelGGL(k_peak_copy, dim3(cgrid), dim3(256), 0, s,
                                                         (const v4i *)a.p, (v4i *)b.p, n); }, &ms));
            *hbm_gbs = 2.0 * 16 * (double)n / (ms * 1e-3) / 1e9;
        }
        if (hbm_read_gbs) {
            DevBuf sink;
            BSMM_TRY(sink.reserve(sizeof(int) * (size_t)cgrid * 256, s));
            BSMM_TRY(time_ms(s, [&] { hipLaunchKernelGGL(k_peak_read, dim3(cgrid), dim3(256), 0, s,
                                                         (const v4i *)a.p, n, sink.as<int>()); }, &ms));
            *hbm_read_gbs = 16 * (double)n / (ms * 1e-3) / 1e9;
        }
    }
    return BSMM_OK;
}
