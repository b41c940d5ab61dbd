// timing.hip -- optional HIP-event timing of the hot kernels.
//
// While the option "time_kernels" is "1", every launch of the dense GEMM
// and of the small-block stack kernels is bracketed by two events recorded
// on the launch stream; bsmm_kernel_times() sums the elapsed times.
#include <mutex>
#include <vector>

#include "internal.h"

namespace bsmm {

namespace {
struct Span {
    int kind;
    hipEvent_t a, b;
};
std::mutex g_tmu;
std::vector<Span> g_spans;
std::vector<hipEvent_t> g_free_events;

hipEvent_t get_event() {
    if (!g_free_events.empty()) {
        hipEvent_t e = g_free_events.back();
        g_free_events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}
}  // namespace

KernelTimer::KernelTimer(int kind, hipStream_t s) : kind_(kind), s_(s) {
    if (!options().time_kernels) return;
    std::lock_guard<std::mutex> lk(g_tmu);
    a_ = get_event();
    b_ = get_event();
    if (a_ && b_) (void)hipEventRecord((hipEvent_t)a_, s_);
}

KernelTimer::~KernelTimer() {
    if (!a_ || !b_) return;
    (void)hipEventRecord((hipEvent_t)b_, s_);
    std::lock_guard<std::mutex> lk(g_tmu);
    g_spans.push_back(Span{kind_, (hipEvent_t)a_, (hipEvent_t)b_});
}

}  // namespace bsmm

extern "C" int bsmm_kernel_times(double *gemm_ms, int64_t *gemm_launches, double *stack_ms,
                                 int64_t *stack_launches, int reset) {
    using namespace bsmm;
    clear_error();
    std::lock_guard<std::mutex> lk(g_tmu);
    double t[2] = {0.0, 0.0};
    int64_t n[2] = {0, 0};
    for (const Span &sp : g_spans) {
        if (hipEventSynchronize(sp.b) != hipSuccess) {
            set_error(BSMM_EDEVICE, "event synchronisation failed");
            return BSMM_EDEVICE;
        }
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, sp.a, sp.b) != hipSuccess) {
            set_error(BSMM_EDEVICE, "event timing failed");
            return BSMM_EDEVICE;
        }
        t[sp.kind] += ms;
        n[sp.kind] += 1;
    }
    if (gemm_ms) *gemm_ms = t[0];
    if (gemm_launches) *gemm_launches = n[0];
    if (stack_ms) *stack_ms = t[1];
    if (stack_launches) *stack_launches = n[1];
    if (reset) {
        for (const Span &sp : g_spans) {
            g_free_events.push_back(sp.a);
            g_free_events.push_back(sp.b);
        }
        g_spans.clear();
    }
    return BSMM_OK;
}
