// mlp.hip -- learned performance model of the small-block kernels.
//
// Paper, Sec. II: a model learned from a subset of the tuning data predicts
// kernel performance over the whole (m, n, k) set, so that untuned shapes
// still get good parameters (the paper uses regression trees on engineered
// features).  Here the model is a small FP32 MLP,
//     y = W3 relu(W2 relu(W1 x + b1) + b2) + b3,
// hidden width 64, whose input x is a normalised feature vector of a shape
// and a parameter set and whose output is the standardised log of the
// kernel time.  Training (forward, per-sample gradients, a fixed-order batch
// reduction, Adam) and inference run in the kernels below; the feature
// function is the single definition shared by training (through the C ABI)
// and by parameter selection.
//
// Parameter layout (one float array): W1 [64 x F] row-major, b1 [64],
// W2 [64 x 64] row-major, b2 [64], W3 [64], b3 [1].
#include <algorithm>
#include <cmath>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <tuple>

#include "dev_util.h"
#include "internal.h"

namespace bsmm {

namespace {

constexpr int H = 64;
constexpr int kMaxF = 32;

__host__ __device__ inline int64_t param_count(int F) { return (int64_t)H * F + H + H * H + H + H + 1; }

struct Views {
    const float *W1, *b1, *W2, *b2, *W3, *b3;
};
__device__ __forceinline__ Views views(const float *P, int F) {
    Views v;
    v.W1 = P;
    v.b1 = v.W1 + H * F;
    v.W2 = v.b1 + H;
    v.b2 = v.W2 + H * H;
    v.W3 = v.b2 + H;
    v.b3 = v.W3 + H;
    return v;
}

// One wave per sample, lane j = hidden unit j.  Stores the hidden
// activations for the backward pass when H1/H2 are given.
__global__ __launch_bounds__(256) void k_mlp_fwd(int F, const float *P, int64_t n, const float *X,
                                                 const int64_t *perm, float *Y, float *H1, float *H2) {
    __shared__ float h1s[4][H];
    const int64_t smp = (int64_t)blockIdx.x * 4 + wave_id();
    if (smp >= n) return;
    const int64_t src = perm ? perm[smp] : smp;
    const int j = lane_id();
    const Views v = views(P, F);
    const float *x = X + src * F;
    float a = v.b1[j];
    for (int f = 0; f < F; ++f) a = fmaf(v.W1[j * F + f], x[f], a);
    const float h1 = fmaxf(a, 0.0f);
    h1s[wave_id()][j] = h1;
    wave_lds_sync();
    float c = v.b2[j];
    for (int i = 0; i < H; ++i) c = fmaf(v.W2[j * H + i], h1s[wave_id()][i], c);
    const float h2 = fmaxf(c, 0.0f);
    const float y = wave_sum(v.W3[j] * h2) + v.b3[0];
    if (j == 0) Y[smp] = y;
    if (H1) H1[smp * H + j] = h1;
    if (H2) H2[smp * H + j] = h2;
}

// Per-sample gradients of the mean squared error over a batch of nb samples
// into G[sample][param].
__global__ __launch_bounds__(256) void k_mlp_bwd(int F, const float *P, int64_t nb, const float *X,
                                                 const int64_t *perm, const float *T, const float *Y,
                                                 const float *H1, const float *H2, float *G) {
    __shared__ float h1s[4][H];
    __shared__ float d2s[4][H];
    const int64_t smp = (int64_t)blockIdx.x * 4 + wave_id();
    if (smp >= nb) return;
    const int64_t src = perm ? perm[smp] : smp;
    const int j = lane_id();
    const int w = wave_id();
    const Views v = views(P, F);
    const int64_t np = param_count(F);
    float *g = G + smp * np;
    float *gW1 = g, *gb1 = gW1 + H * F, *gW2 = gb1 + H, *gb2 = gW2 + H * H, *gW3 = gb2 + H,
          *gb3 = gW3 + H;
    const float dy = 2.0f * (Y[smp] - T[src]) / (float)nb;
    const float h1 = H1[smp * H + j], h2 = H2[smp * H + j];
    gW3[j] = dy * h2;
    if (j == 0) gb3[0] = dy;
    const float d2 = h2 > 0.0f ? dy * v.W3[j] : 0.0f;
    h1s[w][j] = h1;
    d2s[w][j] = d2;
    wave_lds_sync();
    for (int i = 0; i < H; ++i) gW2[j * H + i] = d2 * h1s[w][i];
    gb2[j] = d2;
    float s = 0.0f;
    for (int jj = 0; jj < H; ++jj) s = fmaf(v.W2[jj * H + j], d2s[w][jj], s);
    const float d1 = h1 > 0.0f ? s : 0.0f;
    const float *x = X + src * F;
    for (int f = 0; f < F; ++f) gW1[j * F + f] = d1 * x[f];
    gb1[j] = d1;
}

// Fixed-order sum of the per-sample gradients: grad[p] = sum_s G[s][p].
__global__ __launch_bounds__(256) void k_reduce(int64_t np, int64_t nb, const float *G, float *grad) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    float s = 0.0f;
    for (int64_t i = 0; i < nb; ++i) s += G[i * np + p];
    grad[p] = s;
}

// Adam (Kingma & Ba, 2015) with bias correction; step t starts at 1.
__global__ __launch_bounds__(256) void k_adam(int64_t np, float *P, const float *grad, float *M,
                                              float *V, float lr, float b1, float b2, float eps,
                                              float c1, float c2) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const float g = grad[p];
    const float m = b1 * M[p] + (1.0f - b1) * g;
    const float v = b2 * V[p] + (1.0f - b2) * g * g;
    M[p] = m;
    V[p] = v;
    const float mh = m / c1, vh = v / c2;
    P[p] -= lr * mh / (sqrtf(vh) + eps);
}

__global__ void k_sq_err(int64_t n, const float *Y, const float *T, float *E) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) E[i] = (Y[i] - T[i]) * (Y[i] - T[i]);
}

template <class T> int upload(DevBuf &b, const T *h, int64_t n, hipStream_t s) {
    BSMM_TRY(b.reserve(sizeof(T) * (n > 0 ? n : 1), s));
    if (n > 0) BSMM_HIP(hipMemcpyAsync(b.p, h, sizeof(T) * n, hipMemcpyHostToDevice, s));
    return BSMM_OK;
}

int check_f(int F) {
    if (F < 1 || F > kMaxF) {
        set_error(BSMM_EINVAL, "feature count must be in [1, %d]", kMaxF);
        return BSMM_EINVAL;
    }
    return BSMM_OK;
}

int forward(int F, const float *dP, int64_t n, const float *dX, const int64_t *perm, float *dY,
            float *dH1, float *dH2, hipStream_t s) {
    if (n <= 0) return BSMM_OK;
    hipLaunchKernelGGL(k_mlp_fwd, dim3(grid_of(n, 4)), dim3(256), 0, s, F, dP, n, dX, perm, dY,
                       dH1, dH2);
    return launch_check("mlp_fwd");
}

}  // namespace

// Features of a shape and a parameter set (before normalisation):
// log2 m, log2 n, log2 k, TM, TN, log2 of the effective k chunk, waves per
// workgroup (0 = as many as fit -> 4), log2 of the lanes (or MFMA tiles)
// holding tiles, the fraction of the tiles that covers the block (times the
// k fill of 4-deep steps for the MFMA kernel), 1 for the MFMA kernel, and
// log2 of the run length (products per C block).
int mlp_features(int m, int n, int k, int run_len, const SmmParams &p, float *f) {
    const bool mfma = p.tm == kMfmaTile && p.tn == kMfmaTile;
    const int kc = (!mfma && p.kc > 0 && p.kc < k) ? p.kc : k;
    const double lanes = (double)ceil_div(m, p.tm) * (double)ceil_div(n, p.tn);
    double cover = (double)m * n / (lanes * p.tm * p.tn);
    if (mfma) cover *= (double)k / (4.0 * (double)ceil_div(k, 4));
    f[0] = (float)std::log2((double)m);
    f[1] = (float)std::log2((double)n);
    f[2] = (float)std::log2((double)k);
    f[3] = (float)p.tm;
    f[4] = (float)p.tn;
    f[5] = (float)std::log2((double)kc);
    f[6] = (float)(p.waves > 0 ? p.waves : 4);
    f[7] = (float)std::log2(lanes);
    f[8] = (float)cover;
    f[9] = mfma ? 1.0f : 0.0f;
    f[10] = (float)std::log2((double)std::max(run_len, 1));
    return kMlpFeatures;
}

namespace {
struct Model {
    bool loaded = false;
    std::string path;
    int F = 0;
    std::vector<float> mean, stdev, params;
    std::map<std::tuple<int, int, int, int>, SmmParams> cache;
};
std::mutex g_mlp_mu;
Model g_model;

bool load_model_locked(const std::string &path) {
    g_model = Model{};
    g_model.path = path;
    g_model.loaded = true;
    if (path.empty()) return false;
    std::ifstream f(path);
    std::string tag;
    int F = 0;
    int64_t np = 0;
    if (!(f >> tag) || tag != "bsmm-mlp" || !(f >> tag) || tag != "features" || !(f >> F) ||
        F < 1 || F > kMaxF)
        return false;
    std::vector<float> mean(F), sd(F);
    if (!(f >> tag) || tag != "mean") return false;
    for (auto &x : mean) f >> x;
    if (!(f >> tag) || tag != "std") return false;
    for (auto &x : sd) f >> x;
    if (!(f >> tag) || tag != "params" || !(f >> np) || np != param_count(F)) return false;
    std::vector<float> P(np);
    for (auto &x : P) f >> x;
    if (!f) return false;
    g_model.F = F;
    g_model.mean = mean;
    g_model.stdev = sd;
    g_model.params = P;
    return true;
}
}  // namespace

bool mlp_select(int m, int n, int k, int run_len, SmmParams *out) {
    std::lock_guard<std::mutex> lk(g_mlp_mu);
    const std::string &want = options().mlp_weights;
    if (!g_model.loaded || g_model.path != want) load_model_locked(want);
    if (g_model.params.empty()) return false;
    auto it = g_model.cache.find({m, n, k, run_len});
    if (it != g_model.cache.end()) {
        *out = it->second;
        return true;
    }
    std::vector<SmmParams> cands = candidate_params(m, n, k);
    if (cands.empty()) return false;
    const int F = g_model.F;
    if (F != kMlpFeatures) return false;  // weights trained on another feature set
    std::vector<float> X(cands.size() * F), Y(cands.size());
    float tmp[kMaxF];
    for (size_t c = 0; c < cands.size(); ++c) {
        mlp_features(m, n, k, run_len, cands[c], tmp);
        for (int f = 0; f < F; ++f) X[c * F + f] = (tmp[f] - g_model.mean[f]) / g_model.stdev[f];
    }
    // Inference on the device, on the null stream, outside any caller stream.
    DevBuf dP, dX, dY;
    hipStream_t s = nullptr;
    if (upload(dP, g_model.params.data(), (int64_t)g_model.params.size(), s) != BSMM_OK ||
        upload(dX, X.data(), (int64_t)X.size(), s) != BSMM_OK || dY.reserve(sizeof(float) * Y.size(), s) ||
        forward(F, dP.as<float>(), (int64_t)cands.size(), dX.as<float>(), nullptr, dY.as<float>(),
                nullptr, nullptr, s) != BSMM_OK ||
        hipMemcpy(Y.data(), dY.p, sizeof(float) * Y.size(), hipMemcpyDeviceToHost) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    const size_t best = (size_t)(std::min_element(Y.begin(), Y.end()) - Y.begin());
    g_model.cache[{m, n, k, run_len}] = cands[best];
    *out = cands[best];
    return true;
}

}  // namespace bsmm

using namespace bsmm;

extern "C" int bsmm_mlp_param_count(int32_t n_features, int64_t *count) {
    clear_error();
    BSMM_TRY(check_f(n_features));
    if (!count) {
        set_error(BSMM_EINVAL, "count is NULL");
        return BSMM_EINVAL;
    }
    *count = param_count(n_features);
    return BSMM_OK;
}

extern "C" int bsmm_mlp_features(int32_t m, int32_t n, int32_t k, int32_t run_len,
                                 const int32_t *params4, float *features, int32_t *n_features) {
    clear_error();
    if (!params4 || !features || m < 1 || n < 1 || k < 1 || run_len < 1 || params4[0] < 1 ||
        params4[1] < 1) {
        set_error(BSMM_EINVAL, "bad arguments");
        return BSMM_EINVAL;
    }
    const int F = mlp_features(m, n, k, run_len,
                               SmmParams{params4[0], params4[1], params4[2], params4[3]}, features);
    if (n_features) *n_features = F;
    return BSMM_OK;
}

// The sample kernels run one wave per sample over at most kMaxGridBlocks
// workgroups of four waves.
static int check_samples(int64_t n) {
    if (n > 4 * kMaxGridBlocks) {
        set_error(BSMM_ERANGE, "more than %lld samples", (long long)(4 * kMaxGridBlocks));
        return BSMM_ERANGE;
    }
    return BSMM_OK;
}

extern "C" int bsmm_mlp_forward(int32_t n_features, const float *params, int64_t n, const float *x,
                                float *y) {
    clear_error();
    BSMM_TRY(check_f(n_features));
    BSMM_TRY(check_samples(n));
    if (!params || (n > 0 && (!x || !y)) || n < 0) {
        set_error(BSMM_EINVAL, "bad arguments");
        return BSMM_EINVAL;
    }
    hipStream_t s = nullptr;
    DevBuf dP, dX, dY;
    BSMM_TRY(upload(dP, params, param_count(n_features), s));
    BSMM_TRY(upload(dX, x, n * n_features, s));
    BSMM_TRY(dY.reserve(sizeof(float) * (n > 0 ? n : 1), s));
    BSMM_TRY(forward(n_features, dP.as<float>(), n, dX.as<float>(), nullptr, dY.as<float>(), nullptr,
                     nullptr, s));
    if (n > 0) BSMM_HIP(hipMemcpy(y, dY.p, sizeof(float) * n, hipMemcpyDeviceToHost));
    return BSMM_OK;
}

extern "C" int bsmm_mlp_grad(int32_t n_features, const float *params, int64_t n, const float *x,
                             const float *t, float *grad, float *loss) {
    clear_error();
    BSMM_TRY(check_f(n_features));
    BSMM_TRY(check_samples(n));
    if (!params || !x || !t || !grad || n < 1) {
        set_error(BSMM_EINVAL, "bad arguments");
        return BSMM_EINVAL;
    }
    const int F = n_features;
    const int64_t np = param_count(F);
    hipStream_t s = nullptr;
    DevBuf dP, dX, dT, dY, dH1, dH2, dG, dgrad, dE;
    BSMM_TRY(upload(dP, params, np, s));
    BSMM_TRY(upload(dX, x, n * F, s));
    BSMM_TRY(upload(dT, t, n, s));
    BSMM_TRY(dY.reserve(sizeof(float) * n, s));
    BSMM_TRY(dH1.reserve(sizeof(float) * n * H, s));
    BSMM_TRY(dH2.reserve(sizeof(float) * n * H, s));
    BSMM_TRY(dG.reserve(sizeof(float) * n * np, s));
    BSMM_TRY(dgrad.reserve(sizeof(float) * np, s));
    BSMM_TRY(dE.reserve(sizeof(float) * n, s));
    BSMM_TRY(forward(F, dP.as<float>(), n, dX.as<float>(), nullptr, dY.as<float>(), dH1.as<float>(),
                     dH2.as<float>(), s));
    hipLaunchKernelGGL(k_mlp_bwd, dim3(grid_of(n, 4)), dim3(256), 0, s, F,
                       (const float *)dP.as<float>(), n, (const float *)dX.as<float>(),
                       (const int64_t *)nullptr, (const float *)dT.as<float>(),
                       (const float *)dY.as<float>(), (const float *)dH1.as<float>(),
                       (const float *)dH2.as<float>(), dG.as<float>());
    BSMM_TRY(launch_check("mlp_bwd"));
    hipLaunchKernelGGL(k_reduce, dim3(grid_of(np, 256)), dim3(256), 0, s, np, n,
                       (const float *)dG.as<float>(), dgrad.as<float>());
    BSMM_TRY(launch_check("mlp_reduce"));
    hipLaunchKernelGGL(k_sq_err, dim3(grid_of(n, 256)), dim3(256), 0, s, n,
                       (const float *)dY.as<float>(), (const float *)dT.as<float>(), dE.as<float>());
    BSMM_TRY(launch_check("mlp_sq_err"));
    BSMM_HIP(hipMemcpy(grad, dgrad.p, sizeof(float) * np, hipMemcpyDeviceToHost));
    if (loss) {
        std::vector<float> e(n);
        BSMM_HIP(hipMemcpy(e.data(), dE.p, sizeof(float) * n, hipMemcpyDeviceToHost));
        double acc = 0.0;
        for (float v : e) acc += v;
        *loss = (float)(acc / (double)n);
    }
    return BSMM_OK;
}

extern "C" int bsmm_mlp_adam_step(int32_t n_features, float *params, const float *grad, float *m,
                                  float *v, int32_t step, float lr, float beta1, float beta2,
                                  float eps) {
    clear_error();
    BSMM_TRY(check_f(n_features));
    if (!params || !grad || !m || !v || step < 1) {
        set_error(BSMM_EINVAL, "bad arguments");
        return BSMM_EINVAL;
    }
    const int64_t np = param_count(n_features);
    hipStream_t s = nullptr;
    DevBuf dP, dg, dM, dV;
    BSMM_TRY(upload(dP, params, np, s));
    BSMM_TRY(upload(dg, grad, np, s));
    BSMM_TRY(upload(dM, m, np, s));
    BSMM_TRY(upload(dV, v, np, s));
    const float c1 = 1.0f - std::pow(beta1, (float)step), c2 = 1.0f - std::pow(beta2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3(grid_of(np, 256)), dim3(256), 0, s, np, dP.as<float>(),
                       (const float *)dg.as<float>(), dM.as<float>(), dV.as<float>(), lr, beta1, beta2,
                       eps, c1, c2);
    BSMM_TRY(launch_check("mlp_adam"));
    BSMM_HIP(hipMemcpy(params, dP.p, sizeof(float) * np, hipMemcpyDeviceToHost));
    BSMM_HIP(hipMemcpy(m, dM.p, sizeof(float) * np, hipMemcpyDeviceToHost));
    BSMM_HIP(hipMemcpy(v, dV.p, sizeof(float) * np, hipMemcpyDeviceToHost));
    return BSMM_OK;
}

extern "C" int bsmm_mlp_train(int32_t n_features, float *params, int64_t n, const float *x,
                              const float *t, int32_t epochs, int32_t batch, float lr, uint64_t seed,
                              float *final_loss) {
    clear_error();
    BSMM_TRY(check_f(n_features));
    BSMM_TRY(check_samples(n));
    if (!params || !x || !t || n < 1 || epochs < 0 || batch < 1 || !(lr > 0.0f)) {
        set_error(BSMM_EINVAL, "bad arguments");
        return BSMM_EINVAL;
    }
    const int F = n_features;
    const int64_t np = param_count(F);
    const int64_t nb_max = std::min<int64_t>(batch, n);
    hipStream_t s = nullptr;
    DevBuf dP, dX, dT, dY, dH1, dH2, dG, dgrad, dM, dV, dperm, dE;
    std::vector<float> zeros(np, 0.0f);
    BSMM_TRY(upload(dP, params, np, s));
    BSMM_TRY(upload(dX, x, n * F, s));
    BSMM_TRY(upload(dT, t, n, s));
    BSMM_TRY(upload(dM, zeros.data(), np, s));
    BSMM_TRY(upload(dV, zeros.data(), np, s));
    BSMM_TRY(dY.reserve(sizeof(float) * n, s));
    BSMM_TRY(dH1.reserve(sizeof(float) * nb_max * H, s));
    BSMM_TRY(dH2.reserve(sizeof(float) * nb_max * H, s));
    BSMM_TRY(dG.reserve(sizeof(float) * nb_max * np, s));
    BSMM_TRY(dgrad.reserve(sizeof(float) * np, s));
    BSMM_TRY(dperm.reserve(sizeof(int64_t) * n, s));
    BSMM_TRY(dE.reserve(sizeof(float) * n, s));
    std::vector<int64_t> perm(n);
    uint64_t state = seed * 6364136223846793005ull + 1442695040888963407ull;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    int32_t step = 0;
    for (int32_t ep = 0; ep < epochs; ++ep) {
        for (int64_t i = 0; i < n; ++i) perm[i] = i;
        for (int64_t i = n - 1; i > 0; --i) {  // Fisher-Yates with a 64-bit LCG
            state = state * 6364136223846793005ull + 1442695040888963407ull;
            const int64_t j = (int64_t)((state >> 11) % (uint64_t)(i + 1));
            std::swap(perm[i], perm[j]);
        }
        BSMM_HIP(hipMemcpy(dperm.p, perm.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice));
        for (int64_t b0 = 0; b0 < n; b0 += batch) {
            const int64_t nb = std::min<int64_t>(batch, n - b0);
            const int64_t *pp = dperm.as<int64_t>() + b0;
            BSMM_TRY(forward(F, dP.as<float>(), nb, dX.as<float>(), pp, dY.as<float>(),
                             dH1.as<float>(), dH2.as<float>(), s));
            hipLaunchKernelGGL(k_mlp_bwd, dim3(grid_of(nb, 4)), dim3(256), 0, s, F,
                               (const float *)dP.as<float>(), nb, (const float *)dX.as<float>(), pp,
                               (const float *)dT.as<float>(), (const float *)dY.as<float>(),
                               (const float *)dH1.as<float>(), (const float *)dH2.as<float>(),
                               dG.as<float>());
            BSMM_TRY(launch_check("mlp_bwd"));
            hipLaunchKernelGGL(k_reduce, dim3(grid_of(np, 256)), dim3(256), 0, s, np, nb,
                               (const float *)dG.as<float>(), dgrad.as<float>());
            BSMM_TRY(launch_check("mlp_reduce"));
            ++step;
            const float c1 = 1.0f - std::pow(b1, (float)step), c2 = 1.0f - std::pow(b2, (float)step);
            hipLaunchKernelGGL(k_adam, dim3(grid_of(np, 256)), dim3(256), 0, s, np, dP.as<float>(),
                               (const float *)dgrad.as<float>(), dM.as<float>(), dV.as<float>(), lr,
                               b1, b2, eps, c1, c2);
            BSMM_TRY(launch_check("mlp_adam"));
        }
    }
    BSMM_TRY(forward(F, dP.as<float>(), n, dX.as<float>(), nullptr, dY.as<float>(), nullptr, nullptr, s));
    hipLaunchKernelGGL(k_sq_err, dim3(grid_of(n, 256)), dim3(256), 0, s, n,
                       (const float *)dY.as<float>(), (const float *)dT.as<float>(), dE.as<float>());
    BSMM_TRY(launch_check("mlp_sq_err"));
    std::vector<float> e(n);
    BSMM_HIP(hipMemcpy(e.data(), dE.p, sizeof(float) * n, hipMemcpyDeviceToHost));
    BSMM_HIP(hipMemcpy(params, dP.p, sizeof(float) * np, hipMemcpyDeviceToHost));
    if (final_loss) {
        double acc = 0.0;
        for (float v : e) acc += v;
        *final_loss = (float)(acc / (double)n);
    }
    return BSMM_OK;
}
