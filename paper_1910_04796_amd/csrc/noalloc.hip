// noalloc.hip -- the allocation-free multiply entry point.
//
// For callers that cannot allocate device memory (code under stream
// capture, tight serving loops, harnesses that forbid it): every temporary
// of the multiply (symbolic counts, product stacks, split-run partial
// blocks, dense panels, emulation slices) is carved from one file-scope
// device array of fixed size instead of the pool.  C keeps its pattern and
// buffers, so no output storage is allocated either.
//
// The array is a separate object on every device the library runs on; its
// device address is looked up once per device (hipGetSymbolAddress with the
// device current) and only that address is handed to the kernels -- the
// array's name in host code is a host-side stand-in, not device memory.
#include <mutex>

#include "dev_util.h"
#include "internal.h"

namespace bsmm {
int validate_multiply(bsmm_matrix_s *A, bsmm_matrix_s *B, bsmm_matrix_s *C, double eps);
int check_stack_limits(const bsmm_matrix_s *A, const bsmm_matrix_s *B, const bsmm_matrix_s *C,
                       const Options &o);
int adopt_stream(bsmm_matrix_s *M, hipStream_t s);

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // 64 MiB per device
constexpr int kMaxDevices = 64;

__device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
void *g_scratch_ptr[kMaxDevices];  // device address of `scratch`, per device

// Device address of this device's scratch array (looked up on first use).
int scratch_address(void **out) {
    int dev = 0;
    BSMM_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_error(BSMM_ENOTSUP, "device %d: the scratch table covers devices 0..%d", dev,
                  kMaxDevices - 1);
        return BSMM_ENOTSUP;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            set_error(BSMM_EDEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                      hipGetErrorString(e));
            return BSMM_EDEVICE;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return BSMM_OK;
}

// Makes the arena the calling thread's allocation source for one call.
struct ArenaScope {
    ScratchArena arena;
    explicit ArenaScope(void *base) {
        arena.base = static_cast<char *>(base);
        arena.cap = kScratchBytes;
        scratch_arena() = &arena;
    }
    ~ArenaScope() { scratch_arena() = nullptr; }
};

}  // namespace
}  // namespace bsmm

using namespace bsmm;

extern "C" int bsmm_multiply_noalloc(double alpha, bsmm_matrix A, bsmm_matrix B, double beta,
                                     bsmm_matrix C, void *stream) {
    clear_error();
    BSMM_TRY(validate_multiply(A, B, C, 0.0));
    BSMM_TRY(check_stack_limits(A, B, C, options()));
    void *base = nullptr;
    BSMM_TRY(scratch_address(&base));
    hipStream_t s = (hipStream_t)stream;
    BSMM_TRY(adopt_stream(A, s));
    if (B != A) BSMM_TRY(adopt_stream(B, s));
    BSMM_TRY(adopt_stream(C, s));
    int st;
    {
        ArenaScope scope(base);
        st = multiply_fixed_pattern(alpha, A, B, beta, C, s);
    }
    A->last_stream = B->last_stream = C->last_stream = s;
    return st;
}
