// params.hip -- kernel-parameter selection and the autotuning harness.
//
// Paper, Sec. II: the small-matrix kernels are parametrised (algorithm,
// work and threads per block, elements per thread, tiling), an autotuner
// times the parameter sets of each requested (m, n, k), and a performance
// model learned from a subset of the tuning data predicts parameters for
// the rest.  Here:
//   * bsmm_tune_shape times candidate parameter sets on a synthetic stack
//     of one shape (the exhaustive tuner; its driver writes the database);
//   * select_params looks a shape up in the database, then asks the learned
//     model (mlp.hip) to rank the legal candidates, then falls back to the
//     plain rule.  Both are keyed by the run length (products per C block)
//     as well as the shape: short and long runs favour different kernels.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <tuple>

#include "internal.h"

namespace bsmm {

namespace {
std::mutex g_db_mu;
std::string g_db_path;
bool g_db_loaded = false;
// (m, n, k) -> run length -> best parameter set.
std::map<std::tuple<int, int, int>, std::map<int, SmmParams>> g_db;

// Database lines: "m n k R tm tn kc waves [best_us plain_us]" (eight or ten
// fields; R = run length the set was timed at).  Lines without R ("m n k tm
// tn kc waves [best_us plain_us]", seven or nine fields) count as R = 8.
void load_db_locked(const std::string &path) {
    g_db.clear();
    g_db_path = path;
    g_db_loaded = true;
    if (path.empty()) return;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        if (line.empty() || line[0] == '#') continue;
        std::istringstream is(line);
        std::vector<double> v;
        double x;
        while (is >> x) v.push_back(x);
        SmmParams p;
        int m, n, k, R;
        if (v.size() == 10 || v.size() == 8) {
            m = (int)v[0], n = (int)v[1], k = (int)v[2], R = (int)v[3];
            p = SmmParams{(int)v[4], (int)v[5], (int)v[6], (int)v[7]};
        } else if (v.size() == 9 || v.size() == 7) {
            m = (int)v[0], n = (int)v[1], k = (int)v[2], R = 8;
            p = SmmParams{(int)v[3], (int)v[4], (int)v[5], (int)v[6]};
        } else {
            continue;
        }
        if (R >= 1) g_db[{m, n, k}][R] = p;
    }
}

// Entry whose run length is nearest to R on a log scale (ties: the shorter).
bool db_lookup_locked(int m, int n, int k, int R, SmmParams *out) {
    auto it = g_db.find({m, n, k});
    if (it == g_db.end() || it->second.empty()) return false;
    double best = 1e300;
    for (auto &e : it->second) {
        const double d = std::fabs(std::log2((double)e.first) - std::log2((double)std::max(R, 1)));
        if (d < best - 1e-12) {
            best = d;
            *out = e.second;
        }
    }
    return true;
}
}  // namespace

// Candidate parameter sets of a shape: every compiled register tile whose
// lane count fits a wavefront (or the largest tile when none does), k
// chunks {4, 8, 16, 32, whole}, 1, 2 or 4 waves per workgroup.
std::vector<SmmParams> candidate_params(int m, int n, int k) {
    static const int tiles[] = {1, 2, 3, 4, 5, 6, 8};
    static const int kcs[] = {4, 8, 16, 32, 0};
    static const int waves[] = {1, 2, 4};
    std::vector<SmmParams> out;
    for (int tm : tiles)
        for (int tn : tiles) {
            const int64_t lanes = ceil_div(m, tm) * ceil_div(n, tn);
            const bool fits = lanes <= 64;
            const bool biggest = tm == 8 && tn == 8;
            if (!fits && !biggest) continue;
            // skip tiles that leave most of the tile empty
            if (tm > 1 && ceil_div(m, tm) == ceil_div(m, tm - (tm == 8 ? 2 : 1))) continue;
            if (tn > 1 && ceil_div(n, tn) == ceil_div(n, tn - (tn == 8 ? 2 : 1))) continue;
            if (lanes < 4 && !(tm == 1 && tn == 1)) continue;
            for (int kc : kcs) {
                if (kc > 0 && kc >= k) continue;
                for (int w : waves) out.push_back(SmmParams{tm, tn, kc, w});
            }
        }
    // FP64 MFMA kernel (16 x 16 tiles, zero padding in registers) for every
    // block up to 64 x 64: even 5-sized blocks can gain on long runs.
    if (m <= 64 && n <= 64)
        for (int w : waves) out.push_back(SmmParams{kMfmaTile, kMfmaTile, 0, w});
    return out;
}

SmmParams select_params(int m, int n, int k, int run_len) {
    const Options &o = options();
    if (o.forced[0] > 0) return SmmParams{o.forced[0], o.forced[1], o.forced[2], o.forced[3]};
    {
        std::lock_guard<std::mutex> lk(g_db_mu);
        const std::string &want = options().tune_db;
        if (!g_db_loaded || want != g_db_path) load_db_locked(want);
        SmmParams p;
        if (db_lookup_locked(m, n, k, run_len, &p)) return p;
    }
    // The model is only asked within the run lengths it was trained on: its
    // run-length feature is not extrapolated past the tuner's longest runs.
    SmmParams p;
    if (mlp_select(m, n, k, std::min(run_len, kMlpMaxRunLen), &p)) return p;
    return plain_params(m, n);
}

}  // namespace bsmm

using namespace bsmm;

namespace {
__global__ void k_fill_const(double *p, int64_t n, double v) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x)
        p[e] = v;
}
}  // namespace

extern "C" int bsmm_tune_shape(int32_t m, int32_t n, int32_t k, int64_t n_runs, int32_t run_len,
                               int32_t n_cands, const int32_t *cands, int32_t reps,
                               double *out_us, void *stream) {
    clear_error();
    if (m < 1 || n < 1 || k < 1 || m > 256 || n > 256 || k > 256 || n_runs < 1 || run_len < 1 ||
        n_runs * (int64_t)run_len > (int64_t(1) << 26) || n_cands < 0 ||
        (n_cands > 0 && (!cands || !out_us)) || reps < 1) {
        set_error(BSMM_EINVAL, "bad tuning arguments");
        return BSMM_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    // Synthetic stack with the paper's batch size in mind: pools of A and B
    // blocks, runs of run_len products each drawn from the pools by a fixed
    // linear congruential sequence.
    const int64_t pool = 4096;
    const int64_t na = pool * m * (int64_t)k, nb = pool * (int64_t)k * n, nc = n_runs * m * (int64_t)n;
    const int64_t np = n_runs * run_len;
    DevBuf A, B, C, coff, rptr, prods;
    BSMM_TRY(A.reserve(sizeof(double) * na, s));
    BSMM_TRY(B.reserve(sizeof(double) * nb, s));
    BSMM_TRY(C.reserve(sizeof(double) * nc, s));
    BSMM_TRY(coff.reserve(sizeof(int64_t) * n_runs, s));
    BSMM_TRY(rptr.reserve(sizeof(int64_t) * (n_runs + 1), s));
    BSMM_TRY(prods.reserve(sizeof(ulonglong2) * np, s));
    std::vector<int64_t> hc(n_runs), hr(n_runs + 1);
    std::vector<ulonglong2> hp(np);
    uint64_t x = 88172645463325252ull;
    for (int64_t r = 0; r < n_runs; ++r) {
        hc[r] = r * m * (int64_t)n;
        hr[r] = r * run_len;
        for (int32_t q = 0; q < run_len; ++q) {
            x = x * 6364136223846793005ull + 1442695040888963407ull;
            const int64_t ia = (int64_t)((x >> 33) % pool), ib = (int64_t)((x >> 13) % pool);
            hp[r * run_len + q] = make_ulonglong2((uint64_t)(ia * m * k) | ((uint64_t)k << 48),
                                                  (uint64_t)(ib * k * n));
        }
    }
    hr[n_runs] = np;
    BSMM_HIP(hipMemcpyAsync(coff.p, hc.data(), sizeof(int64_t) * n_runs, hipMemcpyHostToDevice, s));
    BSMM_HIP(hipMemcpyAsync(rptr.p, hr.data(), sizeof(int64_t) * (n_runs + 1), hipMemcpyHostToDevice, s));
    BSMM_HIP(hipMemcpyAsync(prods.p, hp.data(), sizeof(ulonglong2) * np, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_fill_const, dim3(1024), dim3(256), 0, s, A.as<double>(), na, 0.5);
    hipLaunchKernelGGL(k_fill_const, dim3(1024), dim3(256), 0, s, B.as<double>(), nb, 0.25);
    hipLaunchKernelGGL(k_fill_const, dim3(1024), dim3(256), 0, s, C.as<double>(), nc, 0.0);
    BSMM_TRY(launch_check("tune fill"));
    BSMM_HIP(hipStreamSynchronize(s));

    hipEvent_t e0, e1;
    BSMM_HIP(hipEventCreate(&e0));
    BSMM_HIP(hipEventCreate(&e1));
    int status = BSMM_OK;
    std::vector<float> t(reps);
    for (int32_t c = 0; c < n_cands && status == BSMM_OK; ++c) {
        SmmParams prm{cands[4 * c], cands[4 * c + 1], cands[4 * c + 2], cands[4 * c + 3]};
        SmmLaunch L;
        if (plan_smm(prm, m, n, k, BSMM_F64, &L) != BSMM_OK) {
            out_us[c] = -1.0;
            clear_error();
            continue;
        }
        auto go = [&]() {
            return launch_smm(L, A.as<double>(), B.as<double>(), C.as<double>(), coff.as<int64_t>(),
                              rptr.as<int64_t>(), prods.as<ulonglong2>(), 0, n_runs, 1.0, 0.0, s);
        };
        if ((status = go()) != BSMM_OK) break;
        for (int32_t i = 0; i < reps && status == BSMM_OK; ++i) {
            if (hipEventRecord(e0, s) != hipSuccess) status = BSMM_EDEVICE;
            if (status == BSMM_OK) status = go();
            if (status == BSMM_OK && hipEventRecord(e1, s) != hipSuccess) status = BSMM_EDEVICE;
            if (status == BSMM_OK && hipEventSynchronize(e1) != hipSuccess) status = BSMM_EDEVICE;
            if (status == BSMM_OK && hipEventElapsedTime(&t[i], e0, e1) != hipSuccess)
                status = BSMM_EDEVICE;
        }
        if (status != BSMM_OK) break;
        std::vector<float> u = t;
        std::sort(u.begin(), u.end());
        out_us[c] = 1000.0 * u[reps / 2];
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (status == BSMM_EDEVICE && last_code() == BSMM_OK)
        set_error(BSMM_EDEVICE, "event timing failed");
    return status;
}

extern "C" int bsmm_tune_candidates(int32_t m, int32_t n, int32_t k, int32_t *n_cands,
                                    int32_t *cands) {
    clear_error();
    if (!n_cands || m < 1 || n < 1 || k < 1) {
        set_error(BSMM_EINVAL, "bad arguments");
        return BSMM_EINVAL;
    }
    std::vector<SmmParams> v = candidate_params(m, n, k);
    const int32_t cap = *n_cands;
    *n_cands = (int32_t)v.size();
    if (!cands) return BSMM_OK;
    if (cap < (int32_t)v.size()) {
        set_error(BSMM_ERANGE, "capacity too small");
        return BSMM_ERANGE;
    }
    for (size_t i = 0; i < v.size(); ++i) {
        cands[4 * i] = v[i].tm;
        cands[4 * i + 1] = v[i].tn;
        cands[4 * i + 2] = v[i].kc;
        cands[4 * i + 3] = v[i].waves;
    }
    return BSMM_OK;
}

extern "C" int bsmm_select_params(int32_t m, int32_t n, int32_t k, int32_t run_len,
                                  int32_t *params4) {
    clear_error();
    if (!params4 || m < 1 || n < 1 || k < 1 || run_len < 1) {
        set_error(BSMM_EINVAL, "bad arguments");
        return BSMM_EINVAL;
    }
    SmmParams p = select_params(m, n, k, run_len);
    params4[0] = p.tm;
    params4[1] = p.tn;
    params4[2] = p.kc;
    params4[3] = p.waves;
    return BSMM_OK;
}
