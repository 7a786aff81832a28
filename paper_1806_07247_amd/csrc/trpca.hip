// Tensor robust PCA, the problem the paper names as the use of the prox of
// Theorem 2.3:  min ||L||_* + lam ||S||_1  s.t.  L + S = X  (||.||_* the TNN
// of Definition 2.9), by the inexact augmented Lagrangian method.  Each
// iteration is one prox call (tp_prox_tnn, or the learned-rank prox chained
// from call to call) and one fused pass over the entries that does the rest
// of the iteration: the soft threshold for S, the residual, the multiplier
// step, the next prox input and the three maxima of the stopping test.
#include <cmath>
#include <utility>

#include "tp_internal.h"

namespace tp {
namespace {

constexpr int kThreads = 256;
constexpr int kMaxBlocks = 2048;  // partial maxima per pass

// NaN-propagating maximum, NaN in either argument wins (a NaN entry must fail
// the stopping test, whichever operand order the reductions use)
__device__ __forceinline__ float nmax(float m, float v) { return (m != m || v <= m) ? m : v; }

// block maximum of up to 3 values per thread, written to part[3 * block + c]
template <int C>
__device__ __forceinline__ void block_max(float (&v)[C], float* part)
{
    __shared__ float red[C][kThreads / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < C; ++c) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v[c] = nmax(v[c], __shfl_xor(v[c], o, 64));
        if (lane == 0) red[c][wave] = v[c];
    }
    __syncthreads();
    if (threadIdx.x < C) {
        float m = red[threadIdx.x][0];
#pragma unroll
        for (int w = 1; w < kThreads / 64; ++w) m = nmax(m, red[threadIdx.x][w]);
        part[C * blockIdx.x + threadIdx.x] = m;
    }
}

struct UpdateArgs {
    const float* x;
    const float* lold;
    const float* lnew;
    float* s;
    float* lam;
    float* yin;
    long long n;
    float mu, thr, mu_next;  // penalty, lam / mu, next penalty
    float* part;
    int vec;                 // all six arrays 16-byte aligned: float4 main loop
};

// One entry of the iteration (FP32):
//   r = X - L' - Lam/mu;  S' = sign(r) max(|r| - lam/mu, 0);  R = L' + S' - X
//   Lam' = Lam + mu R;    Yin = X - S' - Lam'/mu_next
__device__ __forceinline__ void update_one(const UpdateArgs& a, float x, float lo, float ln, float& s, float& lm,
                                           float& yin, float& dl, float& ds, float& dr)
{
    const float r = x - ln - lm / a.mu;
    const float sh = fabsf(r) - a.thr;
    const float sn = sh > 0.0f ? copysignf(sh, r) : 0.0f;
    const float res = ln + sn - x;
    dl = nmax(dl, fabsf(ln - lo));
    ds = nmax(ds, fabsf(sn - s));
    dr = nmax(dr, fabsf(res));
    lm = lm + a.mu * res;
    s = sn;
    yin = x - sn - lm / a.mu_next;
}

__global__ __launch_bounds__(kThreads) void k_trpca_update(UpdateArgs a)
{
    float d[3] = {0.0f, 0.0f, 0.0f};
    const long long stride = (long long)gridDim.x * kThreads;
    const long long n4 = a.vec ? a.n / 4 : 0;
    for (long long q = (long long)blockIdx.x * kThreads + threadIdx.x; q < n4; q += stride) {
        const float4 x = reinterpret_cast<const float4*>(a.x)[q];
        const float4 lo = reinterpret_cast<const float4*>(a.lold)[q];
        const float4 ln = reinterpret_cast<const float4*>(a.lnew)[q];
        float4 s = reinterpret_cast<const float4*>(a.s)[q];
        float4 lm = reinterpret_cast<const float4*>(a.lam)[q];
        float4 y;
        update_one(a, x.x, lo.x, ln.x, s.x, lm.x, y.x, d[0], d[1], d[2]);
        update_one(a, x.y, lo.y, ln.y, s.y, lm.y, y.y, d[0], d[1], d[2]);
        update_one(a, x.z, lo.z, ln.z, s.z, lm.z, y.z, d[0], d[1], d[2]);
        update_one(a, x.w, lo.w, ln.w, s.w, lm.w, y.w, d[0], d[1], d[2]);
        reinterpret_cast<float4*>(a.s)[q] = s;
        reinterpret_cast<float4*>(a.lam)[q] = lm;
        reinterpret_cast<float4*>(a.yin)[q] = y;
    }
    // tail (n not a multiple of 4)
    for (long long e = n4 * 4 + (long long)blockIdx.x * kThreads + threadIdx.x; e < a.n; e += stride) {
        float s = a.s[e], lm = a.lam[e], y;
        update_one(a, a.x[e], a.lold[e], a.lnew[e], s, lm, y, d[0], d[1], d[2]);
        a.s[e] = s;
        a.lam[e] = lm;
        a.yin[e] = y;
    }
    block_max<3>(d, a.part);
}

// partial maxima of |x| (the scale of the stopping test)
__global__ __launch_bounds__(kThreads) void k_absmax(const float* __restrict__ x, long long n, float* part)
{
    float d[1] = {0.0f};
    for (long long e = (long long)blockIdx.x * kThreads + threadIdx.x; e < n; e += (long long)gridDim.x * kThreads)
        d[0] = nmax(d[0], fabsf(x[e]));
    block_max<1>(d, part);
}

// out[c] = max over the nb partials of component c (one workgroup)
__global__ __launch_bounds__(kThreads) void k_max_reduce(const float* __restrict__ part, int nb, int C,
                                                         float* out)
{
    __shared__ float red[kThreads];
    for (int c = 0; c < C; ++c) {
        float m = 0.0f;
        for (int b = threadIdx.x; b < nb; b += kThreads) m = nmax(m, part[C * b + c]);
        red[threadIdx.x] = m;
        __syncthreads();
        for (int w = kThreads / 2; w > 0; w >>= 1) {
            if (threadIdx.x < w) red[threadIdx.x] = nmax(red[threadIdx.x], red[threadIdx.x + w]);
            __syncthreads();
        }
        if (threadIdx.x == 0) out[c] = red[0];
        __syncthreads();
    }
}

int blocks_for_n(long long n)
{
    const long long b = (n / 4 + kThreads - 1) / kThreads;
    return (int)(b < 1 ? 1 : (b > kMaxBlocks ? kMaxBlocks : b));
}

}  // namespace

hipError_t launch_trpca_update(const float* x, const float* lold, const float* lnew, float* s, float* lam,
                               float* yin, long long n, float mu, float thr, float mu_next, float* part,
                               float* dmax, hipStream_t st)
{
    const int nb = blocks_for_n(n);
    trace_work(0.0, 32.0 * (double)n);  // reads X, L, L', S, Lam; writes S, Lam, Yin
    const unsigned long long al = reinterpret_cast<unsigned long long>(x) | reinterpret_cast<unsigned long long>(lold) |
                                  reinterpret_cast<unsigned long long>(lnew) | reinterpret_cast<unsigned long long>(s) |
                                  reinterpret_cast<unsigned long long>(lam) | reinterpret_cast<unsigned long long>(yin);
    k_trpca_update<<<nb, kThreads, 0, st>>>(
        UpdateArgs{x, lold, lnew, s, lam, yin, n, mu, thr, mu_next, part, (al & 15) == 0 ? 1 : 0});
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_max_reduce<<<1, kThreads, 0, st>>>(part, nb, 3, dmax);
    return hipGetLastError();
}

hipError_t launch_absmax(const float* x, long long n, float* part, float* out, hipStream_t st)
{
    const int nb = blocks_for_n(n);
    k_absmax<<<nb, kThreads, 0, st>>>(x, n, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_max_reduce<<<1, kThreads, 0, st>>>(part, nb, 1, out);
    return hipGetLastError();
}

size_t trpca_part_bytes() { return align_up((size_t)3 * kMaxBlocks * sizeof(float)); }

}  // namespace tp

namespace {

struct TrpcaLayout {
    float *lam, *yin, *lalt, *part, *dmax;
    // learned-rank prox chaining (two of each, alternating between calls)
    int* rank[2];
    float* sigma[2];
    float* basis[2];
    int* bcols[2];
    int* fallback;
    void* prox_ws;
    size_t prox_bytes;
    void* feat_ws;  // tp_slice_features workspace when features are recorded
    size_t feat_bytes;
};

tp::Arena trpca_arena(void* ws, size_t bytes, int n1, int n2, int n3, const tp_trpca_opts* o, bool own_lam,
                      TrpcaLayout* out)
{
    const size_t n = (size_t)n1 * n2 * n3, h = (size_t)tp::half_slices(n3);
    tp::Arena ar(ws, bytes);
    TrpcaLayout t{};
    t.lam = own_lam ? ar.take<float>(n) : nullptr;
    t.yin = ar.take<float>(n);
    t.lalt = ar.take<float>(n);
    t.part = reinterpret_cast<float*>(ar.take<char>(tp::trpca_part_bytes()));
    t.dmax = ar.take<float>(4);
    if (o->learned) {
        const int mr = o->learned->max_rank;
        for (int b = 0; b < 2; ++b) {
            t.rank[b] = ar.take<int>(h);
            t.sigma[b] = ar.take<float>(h * TP_SIGMA_KEEP);
            t.basis[b] = ar.take<float>(2 * h * n2 * (size_t)mr);
            t.bcols[b] = ar.take<int>(h);
        }
        t.fallback = ar.take<int>(h);
        t.prox_bytes = tp_prox_tnn_learned_workspace_size(n1, n2, n3, mr);
    } else {
        t.prox_bytes = tp_prox_tnn_workspace_size(n1, n2, n3);
    }
    t.prox_ws = t.prox_bytes ? ar.take<char>(t.prox_bytes) : nullptr;
    if (o->learned && t.prox_bytes == 0) ar.ok = false;  // max_rank or shape rejected by the prox
    if (o->record && o->record->features) {
        t.feat_bytes = tp_slice_features_workspace_size(n1, n2, n3);
        t.feat_ws = t.feat_bytes ? ar.take<char>(t.feat_bytes) : nullptr;
    }
    if (out) *out = t;
    return ar;
}

bool bad_opts(const tp_trpca_opts* o)
{
    return !o || !(o->mu > 0.0f) || !(o->rho >= 1.0f) || !(o->mu_max >= o->mu) || !(o->tol >= 0.0f) ||
           o->max_iter < 1 || std::isnan(o->lambda) || std::isinf(o->mu_max) ||
           (o->learned && (o->learned->max_rank < 1 || o->learned->max_rank > tp::kMaxL)) ||
           (o->record && o->record->max_calls < 0);
}

}  // namespace

extern "C" {

size_t tp_trpca_workspace_size(int n1, int n2, int n3, const tp_trpca_opts* opts)
{
    if (n1 <= 0 || n2 <= 0 || n3 <= 0 || bad_opts(opts)) return 0;
    return trpca_arena(nullptr, 0, n1, n2, n3, opts, true, nullptr).used;
}

int tp_trpca(const float* X, float* L, float* S, int n1, int n2, int n3, const tp_trpca_opts* opts, float* Lam,
             int* iters, int* converged, void* workspace, size_t workspace_bytes, void* stream)
{
    if (!X || !L || !S || bad_opts(opts)) return TP_ERR_ARG;
    if (n1 <= 0 || n2 <= 0 || n3 <= 0) return TP_ERR_SHAPE;
    TrpcaLayout W;
    tp::Arena ar = trpca_arena(workspace, workspace_bytes, n1, n2, n3, opts, Lam == nullptr, &W);
    if (!ar.ok) return TP_ERR_WORKSPACE;
    if (Lam) W.lam = Lam;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const long long n = (long long)n1 * n2 * n3, h = tp::half_slices(n3);
    const double lam = opts->lambda > 0.0f ? (double)opts->lambda : 1.0 / std::sqrt((double)std::max(n1, n2) * n3);

    TP_TRY(hipMemsetAsync(L, 0, n * sizeof(float), s));
    TP_TRY(hipMemsetAsync(S, 0, n * sizeof(float), s));
    TP_TRY(hipMemsetAsync(W.lam, 0, n * sizeof(float), s));
    float hd[3] = {0.0f, 0.0f, 0.0f};
    TP_LAUNCH(tp::K_TRPCA, s, tp::launch_absmax(X, n, W.part, W.dmax, s));
    TP_TRY(hipMemcpyAsync(hd, W.dmax, sizeof(float), hipMemcpyDeviceToHost, s));
    TP_TRY(hipStreamSynchronize(s));
    if (std::isnan(hd[0])) return TP_ERR_ARG;  // non-finite input
    const double scale = std::max(1.0, (double)hd[0]);

    float* lold = L;      // the current L (zero)
    float* lnew = W.lalt;  // the prox writes L' here
    double mu = opts->mu;
    int it = 0;
    bool done = false;
    while (it < opts->max_iter && !done) {
        const float* yin = it == 0 ? X : W.yin;  // X - S - Lam/mu = X while S = Lam = 0
        const tp_trpca_record* rec = (opts->record && it < opts->record->max_calls) ? opts->record : nullptr;
        const int cur = it & 1, prv = cur ^ 1;
        if (rec && rec->inputs)
            TP_TRY(hipMemcpyAsync(rec->inputs + (long long)it * n, yin, n * sizeof(float), hipMemcpyDeviceToDevice, s));
        if (rec && rec->features) {
            const bool chain = opts->learned && it > 0;
            const int fs = tp_slice_features(yin, n1, n2, n3, (float)(1.0 / mu), chain ? W.rank[prv] : nullptr,
                                             chain ? W.sigma[prv] : nullptr,
                                             rec->features + (long long)it * h * TP_MLP_INPUTS, W.feat_ws, W.feat_bytes,
                                             stream);
            if (fs != TP_OK) return fs;
        }
        int st;
        if (opts->learned) {
            tp_learned_opts lo = *opts->learned;
            lo.prev_rank = it > 0 ? W.rank[prv] : nullptr;
            lo.prev_sigma = it > 0 ? W.sigma[prv] : nullptr;
            lo.warm_basis = it > 0 ? W.basis[prv] : nullptr;
            lo.warm_cols = it > 0 ? W.bcols[prv] : nullptr;
            lo.basis_out = W.basis[cur];
            lo.basis_cols_out = W.bcols[cur];
            lo.seed = opts->learned->seed + (unsigned long long)it;
            st = tp_prox_tnn_learned(yin, lnew, n1, n2, n3, (float)(1.0 / mu), &lo, W.rank[cur], W.fallback,
                                     nullptr, W.sigma[cur], W.prox_ws, W.prox_bytes, stream);
        } else {
            st = tp_prox_tnn(yin, lnew, n1, n2, n3, (float)(1.0 / mu), nullptr, nullptr, W.prox_ws, W.prox_bytes,
                             stream);
        }
        if (st != TP_OK) return st;
        if (rec && opts->learned) {
            const long long mr = opts->learned->max_rank;
            if (rec->counts)
                TP_TRY(hipMemcpyAsync(rec->counts + (long long)it * h, W.rank[cur], h * sizeof(int),
                                      hipMemcpyDeviceToDevice, s));
            if (rec->sigmas)
                TP_TRY(hipMemcpyAsync(rec->sigmas + (long long)it * h * TP_SIGMA_KEEP, W.sigma[cur],
                                      h * TP_SIGMA_KEEP * sizeof(float), hipMemcpyDeviceToDevice, s));
            if (rec->bases)
                TP_TRY(hipMemcpyAsync(rec->bases + (long long)it * 2 * h * n2 * mr, W.basis[cur],
                                      2 * h * n2 * mr * sizeof(float), hipMemcpyDeviceToDevice, s));
            if (rec->basis_cols)
                TP_TRY(hipMemcpyAsync(rec->basis_cols + (long long)it * h, W.bcols[cur], h * sizeof(int),
                                      hipMemcpyDeviceToDevice, s));
        }
        const double mu_next = std::min(opts->rho * mu, (double)opts->mu_max);
        TP_LAUNCH(tp::K_TRPCA, s,
                  tp::launch_trpca_update(X, lold, lnew, S, W.lam, W.yin, n, (float)mu, (float)(lam / mu),
                                          (float)mu_next, W.part, W.dmax, s));
        TP_TRY(hipMemcpyAsync(hd, W.dmax, 3 * sizeof(float), hipMemcpyDeviceToHost, s));
        TP_TRY(hipStreamSynchronize(s));
        std::swap(lold, lnew);
        mu = mu_next;
        ++it;
        const double dm = std::max((double)hd[0], std::max((double)hd[1], (double)hd[2]));
        done = dm <= opts->tol * scale;  // false for NaN
    }
    if (lold != L) TP_TRY(hipMemcpyAsync(L, lold, n * sizeof(float), hipMemcpyDeviceToDevice, s));
    if (iters) *iters = it;
    if (converged) *converged = done ? 1 : 0;
    return TP_OK;
}

}  // extern "C"
