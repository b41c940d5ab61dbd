// jit.hip -- run-time specialised small-block kernels (paper, Sec. II: the
// small-matrix kernels are generated for the block shapes a multiply meets,
// or dispatched from pre-generated code).
//
// For a shape class whose products all have the same depth k (the block
// columns of A share one size), the tuned path can compile, at run time
// with hiprtc, an MFMA small-block kernel with m, n and k as compile-time
// constants: the k loop unrolls completely, the register tiles and the
// edge masks of m and n fold away, and the last k chunk takes only the
// 4-deep steps it needs (a 22-deep product runs 6 MFMA steps instead of
// the 8 of two zero-padded 16-deep chunks).  Compiled kernels are cached
// per device and shape for the life of the process.  hiprtc is opened with
// dlopen on first use; without it (or when a compilation fails) the class
// runs on the precompiled kernels.
#include <dlfcn.h>

#include <chrono>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "dev_util.h"
#include "internal.h"

namespace bsmm {

namespace {

// The hiprtc entry points used here (C API, declared locally so that the
// library needs hiprtc only when the option is on).
typedef int (*rtc_create_t)(void **prog, const char *src, const char *name, int nh,
                            const char *const *headers, const char *const *include_names);
typedef int (*rtc_compile_t)(void *prog, int nopt, const char *const *opts);
typedef int (*rtc_size_t)(void *prog, size_t *n);
typedef int (*rtc_get_t)(void *prog, char *out);
typedef int (*rtc_destroy_t)(void **prog);

struct Rtc {
    bool tried = false, ok = false;
    rtc_create_t create = nullptr;
    rtc_compile_t compile = nullptr;
    rtc_size_t log_size = nullptr, code_size = nullptr;
    rtc_get_t log = nullptr, code = nullptr;
    rtc_destroy_t destroy = nullptr;
    std::string why;
};

Rtc &rtc() {
    static Rtc r;
    if (r.tried) return r;
    r.tried = true;
    void *h = dlopen("libhiprtc.so.7", RTLD_NOW | RTLD_GLOBAL);
    if (!h) h = dlopen("/opt/rocm/lib/libhiprtc.so.7", RTLD_NOW | RTLD_GLOBAL);
    if (!h) h = dlopen("libhiprtc.so", RTLD_NOW | RTLD_GLOBAL);
    if (!h) {
        r.why = "hiprtc not found";
        return r;
    }
    r.create = (rtc_create_t)dlsym(h, "hiprtcCreateProgram");
    r.compile = (rtc_compile_t)dlsym(h, "hiprtcCompileProgram");
    r.log_size = (rtc_size_t)dlsym(h, "hiprtcGetProgramLogSize");
    r.log = (rtc_get_t)dlsym(h, "hiprtcGetProgramLog");
    r.code_size = (rtc_size_t)dlsym(h, "hiprtcGetCodeSize");
    r.code = (rtc_get_t)dlsym(h, "hiprtcGetCode");
    r.destroy = (rtc_destroy_t)dlsym(h, "hiprtcDestroyProgram");
    r.ok = r.create && r.compile && r.log_size && r.log && r.code_size && r.code && r.destroy;
    if (!r.ok) r.why = "hiprtc lacks an entry point";
    return r;
}

// Kernel source: M, N, K and the element type are substituted before
// compilation.  One wave owns one run (all products of one C block, in the
// stacks' order) and keeps the C block as MT x NT tiles of 16 x 16 x 4 MFMA
// accumulators; lane l supplies row (or column) l % 16 of an operand and
// k = l / 16 of each step.  Full 16-deep chunks: lane group g takes
// k = 16 c + 4 g + s for step s (four consecutive values of a B column per
// lane); the tail of KT < 16 values: lane group g takes k = 16 KC + 4 t + g
// for tail step t.
const char *kSource = R"JIT(
typedef @T@ T;
typedef T acc_t __attribute__((ext_vector_type(4)));
typedef T vec4_t __attribute__((ext_vector_type(4)));
typedef T vec2_t __attribute__((ext_vector_type(2)));
constexpr int M = @M@, N = @N@, K = @K@;
constexpr int MT = (M + 15) / 16, NT = (N + 15) / 16;
constexpr int KC = K / 16, KT = K - 16 * KC, TS = (KT + 3) / 4;
struct JitArgs {
    const T *A;
    const T *B;
    T *C;
    const long long *run_coff;
    const long long *run_ptr;
    const unsigned long long *prods;
    long long run_begin, run_end;
    double alpha, beta;
};
__device__ __forceinline__ acc_t mfma(T a, T b, acc_t c) {
#if @F64@
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
#else
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
#endif
}
// Result element e of lane l: FP64 row 4 e + l / 16, FP32 row 4 (l / 16) + e.
__device__ __forceinline__ int out_row(int e, int lk) { return @F64@ ? 4 * e + lk : 4 * lk + e; }
extern "C" __global__ __launch_bounds__(256, 4) void bsmm_jit_smm(JitArgs p) {
    const int lane = threadIdx.x & 63;
    const int lr = lane & 15, lk = lane >> 4;
    const long long waves = (long long)gridDim.x * (blockDim.x / 64);
    const long long wid = (long long)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    for (long long r = p.run_begin + wid; r < p.run_end; r += waves) {
        acc_t acc[MT][NT];
#pragma unroll
        for (int i = 0; i < MT; ++i)
#pragma unroll
            for (int j = 0; j < NT; ++j) acc[i][j] = (acc_t){0, 0, 0, 0};
        const long long q0 = p.run_ptr[r], q1 = p.run_ptr[r + 1];
        // The next product's descriptor is loaded one product ahead.
        unsigned long long na = q0 < q1 ? p.prods[2 * q0] : 0ull, nb = q0 < q1 ? p.prods[2 * q0 + 1] : 0ull;
        for (long long q = q0; q < q1; ++q) {
            const T *a = p.A + (long long)(na & ((1ull << 48) - 1));
            const T *b = p.B + (long long)nb;
            if (q + 1 < q1) {
                na = p.prods[2 * q + 2];
                nb = p.prods[2 * q + 3];
            }
#pragma unroll
            for (int c = 0; c < KC; ++c) {
                T af[4][MT], bf[4][NT];
                const int kb = 16 * c + 4 * lk;
#pragma unroll
                for (int i = 0; i < MT; ++i) {
                    const int row = 16 * i + lr;
#pragma unroll
                    for (int s = 0; s < 4; ++s) af[s][i] = row < M ? a[(kb + s) * M + row] : T(0);
                }
#pragma unroll
                for (int j = 0; j < NT; ++j) {
                    const int col = 16 * j + lr;
                    // four consecutive values of the column as 16-byte loads
                    vec4_t v = (vec4_t){0, 0, 0, 0};
                    if (col < N) {
#if @F64@
                        vec2_t lo, hi;
                        __builtin_memcpy(&lo, b + col * K + kb, sizeof lo);
                        __builtin_memcpy(&hi, b + col * K + kb + 2, sizeof hi);
                        v = (vec4_t){lo[0], lo[1], hi[0], hi[1]};
#else
                        __builtin_memcpy(&v, b + col * K + kb, sizeof v);
#endif
                    }
#pragma unroll
                    for (int s = 0; s < 4; ++s) bf[s][j] = v[s];
                }
#pragma unroll
                for (int s = 0; s < 4; ++s)
#pragma unroll
                    for (int i = 0; i < MT; ++i)
#pragma unroll
                        for (int j = 0; j < NT; ++j) acc[i][j] = mfma(af[s][i], bf[s][j], acc[i][j]);
            }
#pragma unroll
            for (int t = 0; t < TS; ++t) {
                const int kk = 16 * KC + 4 * t + lk;
                const bool kin = kk < K;
                T af[MT], bf[NT];
#pragma unroll
                for (int i = 0; i < MT; ++i) {
                    const int row = 16 * i + lr;
                    af[i] = (row < M && kin) ? a[kk * M + row] : T(0);
                }
#pragma unroll
                for (int j = 0; j < NT; ++j) {
                    const int col = 16 * j + lr;
                    bf[j] = (col < N && kin) ? b[col * K + kk] : T(0);
                }
#pragma unroll
                for (int i = 0; i < MT; ++i)
#pragma unroll
                    for (int j = 0; j < NT; ++j) acc[i][j] = mfma(af[i], bf[j], acc[i][j]);
            }
        }
        T *cb = p.C + p.run_coff[r];
        const T alpha = (T)p.alpha, beta = (T)p.beta;
#pragma unroll
        for (int i = 0; i < MT; ++i)
#pragma unroll
            for (int j = 0; j < NT; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int row = 16 * i + out_row(e, lk), col = 16 * j + lr;
                    if (row < M && col < N) {
                        T *dst = cb + col * M + row;
                        const T prod = alpha * acc[i][j][e];
                        *dst = beta == T(0) ? prod : fma(beta, *dst, prod);
                    }
                }
    }
}
)JIT";

void subst(std::string &s, const char *key, const std::string &val) {
    for (size_t p = s.find(key); p != std::string::npos; p = s.find(key, p + val.size()))
        s.replace(p, strlen(key), val);
}

struct JitEntry {
    hipModule_t mod = nullptr;
    hipFunction_t fn = nullptr;
    bool failed = false;
};
std::mutex g_jit_mu;
std::map<std::tuple<int, int, int, int, int>, JitEntry> g_jit;  // (device, dtype, m, n, k)
JitStats g_stats;

}  // namespace

JitStats jit_stats() {
    std::lock_guard<std::mutex> lk(g_jit_mu);
    return g_stats;
}

hipFunction_t jit_smm_kernel(int dtype, int m, int n, int k) {
    if (m < 1 || n < 1 || m > 64 || n > 64 || k < 1 || k > 256) return nullptr;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_jit_mu);
    JitEntry &e = g_jit[std::make_tuple(dev, dtype, m, n, k)];
    if (e.fn || e.failed) {
        if (e.fn) ++g_stats.cache_hits;
        return e.fn;
    }
    e.failed = true;  // until proven otherwise
    Rtc &r = rtc();
    if (!r.ok) {
        ++g_stats.failures;
        return nullptr;
    }
    std::string src = kSource;
    subst(src, "@T@", dtype == BSMM_F32 ? "float" : "double");
    subst(src, "@F64@", dtype == BSMM_F32 ? "0" : "1");
    subst(src, "@M@", std::to_string(m));
    subst(src, "@N@", std::to_string(n));
    subst(src, "@K@", std::to_string(k));
    const auto t0 = std::chrono::steady_clock::now();
    void *prog = nullptr;
    if (r.create(&prog, src.c_str(), "bsmm_jit.hip", 0, nullptr, nullptr) != 0) {
        ++g_stats.failures;
        return nullptr;
    }
    const char *opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature",
                          "-Xclang", "-packed-fp32-ops"};
    const int rc = r.compile(prog, (int)(sizeof opts / sizeof opts[0]), opts);
    std::vector<char> code;
    if (rc == 0) {
        size_t n_code = 0;
        if (r.code_size(prog, &n_code) == 0 && n_code > 0) {
            code.resize(n_code);
            if (r.code(prog, code.data()) != 0) code.clear();
        }
    } else if (options().verbose) {
        size_t n_log = 0;
        r.log_size(prog, &n_log);
        std::vector<char> log(n_log + 1, 0);
        r.log(prog, log.data());
        fprintf(stderr, "[bsmm] JIT compilation of %dx%dx%d failed:\n%s\n", m, n, k, log.data());
    }
    r.destroy(&prog);
    if (code.empty()) {
        ++g_stats.failures;
        return nullptr;
    }
    if (hipModuleLoadData(&e.mod, code.data()) != hipSuccess ||
        hipModuleGetFunction(&e.fn, e.mod, "bsmm_jit_smm") != hipSuccess) {
        (void)hipGetLastError();
        e.fn = nullptr;
        ++g_stats.failures;
        return nullptr;
    }
    e.failed = false;
    ++g_stats.compiled;
    g_stats.compile_ms +=
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return e.fn;
}

int launch_jit_smm(hipFunction_t fn, unsigned grid, int waves, const void *A, const void *B, void *C,
                   const int64_t *run_coff, const int64_t *run_ptr, const ulonglong2 *prods,
                   int64_t rb, int64_t re, double alpha, double beta, hipStream_t s) {
    // Same layout as the JitArgs struct of the kernel source.
    struct {
        const void *A, *B;
        void *C;
        const int64_t *run_coff, *run_ptr;
        const ulonglong2 *prods;
        int64_t run_begin, run_end;
        double alpha, beta;
    } args = {A, B, C, run_coff, run_ptr, prods, rb, re, alpha, beta};
    void *params[] = {&args};
    KernelTimer kt(1, s);
    BSMM_HIP(hipModuleLaunchKernel(fn, grid, 1, 1, 64 * waves, 1, 1, 0, s, params, nullptr));
    return BSMM_OK;
}

}  // namespace bsmm

using namespace bsmm;

extern "C" int bsmm_jit_stats(int64_t *compiled, int64_t *cache_hits, int64_t *failures,
                              double *compile_ms) {
    clear_error();
    const JitStats st = jit_stats();
    if (compiled) *compiled = st.compiled;
    if (cache_hits) *cache_hits = st.cache_hits;
    if (failures) *failures = st.failures;
    if (compile_ms) *compile_ms = st.compile_ms;
    return BSMM_OK;
}
