// mfma_util.h -- element-type traits of the 16 x 16 x 4 MFMA instructions
// used by the small-block and dense kernels (FP64 and FP32 block data).
#pragma once

#include <hip/hip_runtime.h>

namespace bsmm {

typedef double v4d_t __attribute__((ext_vector_type(4)));
typedef double v2d_t __attribute__((ext_vector_type(2)));
typedef float v4f_t __attribute__((ext_vector_type(4)));

// Both instructions take lane l's operands at row (or column) l % 16 and
// k = l / 16 of the step and return four results per lane.
template <class T> struct Mfma;
template <> struct Mfma<double> {
    typedef v4d_t acc_t;
    static __device__ __forceinline__ acc_t zero() { return (v4d_t){0.0, 0.0, 0.0, 0.0}; }
    static __device__ __forceinline__ acc_t step(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // Result element e of lane l: row 4 e + l / 16, column l % 16.
    static __device__ __forceinline__ int row(int e, int lk) { return 4 * e + lk; }
    // Four consecutive values (16-byte loads at 8-byte alignment: dword
    // alignment is all the vector loads need).
    static __device__ __forceinline__ void load4(const double *p, double (&v)[4]) {
        v2d_t lo, hi;
        __builtin_memcpy(&lo, p, sizeof lo);
        __builtin_memcpy(&hi, p + 2, sizeof hi);
        v[0] = lo[0];
        v[1] = lo[1];
        v[2] = hi[0];
        v[3] = hi[1];
    }
};
template <> struct Mfma<float> {
    typedef v4f_t acc_t;
    static __device__ __forceinline__ acc_t zero() { return (v4f_t){0.0f, 0.0f, 0.0f, 0.0f}; }
    static __device__ __forceinline__ acc_t step(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // Result element e of lane l: row 4 (l / 16) + e, column l % 16.
    static __device__ __forceinline__ int row(int e, int lk) { return 4 * lk + e; }
    static __device__ __forceinline__ void load4(const float *p, float (&v)[4]) {
        v4f_t x;
        __builtin_memcpy(&x, p, sizeof x);
        v[0] = x[0];
        v[1] = x[1];
        v[2] = x[2];
        v[3] = x[3];
    }
};

}  // namespace bsmm
