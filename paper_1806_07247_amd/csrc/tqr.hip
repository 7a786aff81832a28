// Tensor inverse (Definition 2.4) and T-QR (Theorem 2.4) through the same
// slice pipeline as the other operations: the real DFT along the tubes, a
// dense operation on each of the floor(n3/2)+1 leading Fourier slices, the
// inverse DFT (the conjugate-symmetric rest is implicit).  A * B = I holds
// slice by slice in the Fourier domain, where I's slices are identities, so
// the inverse is a matrix inverse per slice; A = Q * R likewise becomes a QR
// factorisation per slice, upper triangular R-slices giving an f-upper
// triangular R.
//
// Per slice one workgroup, the working matrices in the workspace (FP32
// planar complex, reused from L2), FP64 for norms, dot products and pivot
// moduli:
//   inverse: Gauss-Jordan with partial pivoting on [A | I] (largest modulus,
//            first row on ties);
//   QR:      Householder reflectors H = I - 2 v v^* / (v^* v), v = x + phi |x| e1
//            (phi the phase of x's first entry), Q = H_0 H_1 ... formed on the
//            identity in reverse order, then row i of R and column i of Q
//            rephased so that R(i,i) is real and >= 0 (unique R for
//            full-rank slices).
#include <cmath>

#include "tp_internal.h"

namespace tp {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ double abs2d(float r, float i) { return (double)r * r + (double)i * i; }

// --------------------------------------------------------------- inverse --
// w: n x 2n per slice (planar), b: n x n per slice (planar, output)
__global__ __launch_bounds__(kThreads) void k_slice_inv(const float* __restrict__ ar, const float* __restrict__ ai,
                                                        float* __restrict__ wr, float* __restrict__ wi,
                                                        float* __restrict__ br, float* __restrict__ bi, int n,
                                                        int* __restrict__ info)
{
    __shared__ double red_v[kThreads];
    __shared__ int red_i[kThreads];
    __shared__ float fr[1024], fi[1024];  // elimination factors of the step (n <= 1024)
    const int s = blockIdx.x, tid = threadIdx.x, w2 = 2 * n;
    const long long so = (long long)s * n * n, wo = (long long)s * n * w2;
    float* Wr = wr + wo;
    float* Wi = wi + wo;
    for (long long e = tid; e < (long long)n * w2; e += kThreads) {
        const int i = (int)(e / w2), c = (int)(e % w2);
        const bool left = c < n;
        Wr[e] = left ? ar[so + (long long)i * n + c] : (c - n == i ? 1.0f : 0.0f);
        Wi[e] = left ? ai[so + (long long)i * n + c] : 0.0f;
    }
    __syncthreads();
    int bad = 0;
    for (int j = 0; j < n; ++j) {
        // pivot: largest modulus in column j from row j down, first on ties
        double best = -1.0;
        int arg = n;
        for (int i = j + tid; i < n; i += kThreads) {
            const double v = abs2d(Wr[(long long)i * w2 + j], Wi[(long long)i * w2 + j]);
            if (v > best) {
                best = v;
                arg = i;
            }
        }
        red_v[tid] = best;
        red_i[tid] = arg;
        __syncthreads();
        for (int h = kThreads / 2; h > 0; h >>= 1) {
            if (tid < h) {
                const double v2 = red_v[tid + h];
                const int i2 = red_i[tid + h];
                if (v2 > red_v[tid] || (v2 == red_v[tid] && i2 < red_i[tid])) {
                    red_v[tid] = v2;
                    red_i[tid] = i2;
                }
            }
            __syncthreads();
        }
        const int p = red_i[0];
        const bool zero = !(red_v[0] > 0.0);
        // the pivot is read by every thread before the barrier, ahead of the swap
        const float pr = zero ? 1.0f : Wr[(long long)p * w2 + j], pi = zero ? 0.0f : Wi[(long long)p * w2 + j];
        __syncthreads();
        if (zero) {  // singular slice: record the step and leave the rest
            bad = j + 1;
            break;
        }
        // swap rows j and p, then scale row j by 1 / pivot
        const double pm = (double)pr * pr + (double)pi * pi;
        const float qr = (float)(pr / pm), qi = (float)(-pi / pm);  // 1 / pivot
        for (int c = tid; c < w2; c += kThreads) {
            const long long oj = (long long)j * w2 + c, op = (long long)p * w2 + c;
            const float xr = Wr[op], xi = Wi[op];
            if (p != j) {
                Wr[op] = Wr[oj];
                Wi[op] = Wi[oj];
            }
            Wr[oj] = xr * qr - xi * qi;
            Wi[oj] = xr * qi + xi * qr;
        }
        __syncthreads();
        // factors of column j (read before any row changes)
        for (int i = tid; i < n; i += kThreads) {
            fr[i] = i == j ? 0.0f : Wr[(long long)i * w2 + j];
            fi[i] = i == j ? 0.0f : Wi[(long long)i * w2 + j];
        }
        __syncthreads();
        // row i -= f_i row j, i != j
        for (long long e = tid; e < (long long)n * w2; e += kThreads) {
            const int i = (int)(e / w2), c = (int)(e % w2);
            if (i == j) continue;
            const float f_r = fr[i], f_i = fi[i];
            if (f_r == 0.0f && f_i == 0.0f) continue;
            const float yr = Wr[(long long)j * w2 + c], yi = Wi[(long long)j * w2 + c];
            Wr[e] -= f_r * yr - f_i * yi;
            Wi[e] -= f_r * yi + f_i * yr;
        }
        __syncthreads();
    }
    for (long long e = tid; e < (long long)n * n; e += kThreads) {
        const int i = (int)(e / n), c = (int)(e % n);
        br[so + e] = Wr[(long long)i * w2 + n + c];
        bi[so + e] = Wi[(long long)i * w2 + n + c];
    }
    if (tid == 0 && info) info[s] = bad;
}

// -------------------------------------------------------------------- QR --
// w: m x n working copy of the slice; v: m x k reflectors; beta: k; q: m x m;
// r: m x n (all per slice, planar)
__global__ __launch_bounds__(kThreads) void k_slice_qr(const float* __restrict__ ar, const float* __restrict__ ai,
                                                       float* __restrict__ wr, float* __restrict__ wi,
                                                       float* __restrict__ vr, float* __restrict__ vi,
                                                       double* __restrict__ beta, float* __restrict__ qr,
                                                       float* __restrict__ qi, float* __restrict__ rr,
                                                       float* __restrict__ ri, int m, int n)
{
    __shared__ double red[kThreads];
    __shared__ double sh_beta;
    const int s = blockIdx.x, tid = threadIdx.x, k = m < n ? m : n;
    const long long mn = (long long)m * n, mk = (long long)m * k, mm = (long long)m * m;
    float* Wr = wr + s * mn;
    float* Wi = wi + s * mn;
    float* Vr = vr + s * mk;
    float* Vi = vi + s * mk;
    double* B = beta + (long long)s * k;
    for (long long e = tid; e < mn; e += kThreads) {
        Wr[e] = ar[s * mn + e];
        Wi[e] = ai[s * mn + e];
    }
    __syncthreads();
    for (int j = 0; j < k; ++j) {
        double part = 0.0;
        for (int i = j + tid; i < m; i += kThreads) part += abs2d(Wr[(long long)i * n + j], Wi[(long long)i * n + j]);
        red[tid] = part;
        __syncthreads();
        for (int h = kThreads / 2; h > 0; h >>= 1) {
            if (tid < h) red[tid] += red[tid + h];
            __syncthreads();
        }
        const double s2 = red[0];
        __syncthreads();
        if (!(s2 > 0.0)) {  // zero column below the diagonal: H = I
            if (tid == 0) B[j] = 0.0;
            for (int i = tid; i < m; i += kThreads) {
                Vr[(long long)i * k + j] = 0.0f;
                Vi[(long long)i * k + j] = 0.0f;
            }
            __syncthreads();
            continue;
        }
        // v = x + phi |x| e1 (x = column j from row j), beta = 2 / v^* v
        if (tid == 0) {
            const double sn = sqrt(s2);
            const double al_r = Wr[(long long)j * n + j], al_i = Wi[(long long)j * n + j];
            const double aa = sqrt(al_r * al_r + al_i * al_i);
            const double ph_r = aa > 0.0 ? al_r / aa : 1.0, ph_i = aa > 0.0 ? al_i / aa : 0.0;
            const double v0r = al_r + ph_r * sn, v0i = al_i + ph_i * sn;
            Vr[(long long)j * k + j] = (float)v0r;
            Vi[(long long)j * k + j] = (float)v0i;
            // v^* v = |v0|^2 + (s2 - |alpha|^2)
            const double vv = v0r * v0r + v0i * v0i + (s2 - aa * aa);
            sh_beta = 2.0 / vv;
            B[j] = sh_beta;
        }
        for (int i = tid; i < m; i += kThreads) {
            if (i == j) continue;
            Vr[(long long)i * k + j] = i > j ? Wr[(long long)i * n + j] : 0.0f;
            Vi[(long long)i * k + j] = i > j ? Wi[(long long)i * n + j] : 0.0f;
        }
        __syncthreads();
        const double bt = sh_beta;
        // columns c >= j: w_c -= beta v (v^* w_c), one thread per column
        for (int c = j + tid; c < n; c += kThreads) {
            double tr = 0.0, ti = 0.0;
            for (int i = j; i < m; ++i) {
                const double xr = Vr[(long long)i * k + j], xi = Vi[(long long)i * k + j];
                const double yr = Wr[(long long)i * n + c], yi = Wi[(long long)i * n + c];
                tr += xr * yr + xi * yi;  // conj(v_i) w_ic
                ti += xr * yi - xi * yr;
            }
            tr *= bt;
            ti *= bt;
            for (int i = j; i < m; ++i) {
                const double xr = Vr[(long long)i * k + j], xi = Vi[(long long)i * k + j];
                Wr[(long long)i * n + c] -= (float)(xr * tr - xi * ti);
                Wi[(long long)i * n + c] -= (float)(xr * ti + xi * tr);
            }
        }
        __syncthreads();
    }
    // Q = H_0 ... H_{k-1} I, the reflectors applied in reverse order
    float* Qr = qr + s * mm;
    float* Qi = qi + s * mm;
    for (long long e = tid; e < mm; e += kThreads) {
        Qr[e] = (e / m == e % m) ? 1.0f : 0.0f;
        Qi[e] = 0.0f;
    }
    __syncthreads();
    for (int j = k - 1; j >= 0; --j) {
        const double bt = B[j];
        if (bt != 0.0)
            for (int c = j + tid; c < m; c += kThreads) {
                double tr = 0.0, ti = 0.0;
                for (int i = j; i < m; ++i) {
                    const double xr = Vr[(long long)i * k + j], xi = Vi[(long long)i * k + j];
                    const double yr = Qr[(long long)i * m + c], yi = Qi[(long long)i * m + c];
                    tr += xr * yr + xi * yi;
                    ti += xr * yi - xi * yr;
                }
                tr *= bt;
                ti *= bt;
                for (int i = j; i < m; ++i) {
                    const double xr = Vr[(long long)i * k + j], xi = Vi[(long long)i * k + j];
                    Qr[(long long)i * m + c] -= (float)(xr * tr - xi * ti);
                    Qi[(long long)i * m + c] -= (float)(xr * ti + xi * tr);
                }
            }
        __syncthreads();
    }
    // R (upper part of W), rephased with Q so that R(i,i) = |R(i,i)| >= 0
    float* Rr = rr + s * mn;
    float* Ri = ri + s * mn;
    for (long long e = tid; e < mn; e += kThreads) {
        const int i = (int)(e / n), c = (int)(e % n);
        float xr = 0.0f, xi = 0.0f;
        if (c >= i) {
            xr = Wr[e];
            xi = Wi[e];
            if (i < k) {
                const double dr = Wr[(long long)i * n + i], di = Wi[(long long)i * n + i];
                const double ad = sqrt(dr * dr + di * di);
                if (ad > 0.0) {  // times conj(d) / |d|
                    const double pr = dr / ad, pi = -di / ad;
                    const double yr = xr * pr - xi * pi, yi = xr * pi + xi * pr;
                    xr = c == i ? (float)ad : (float)yr;
                    xi = c == i ? 0.0f : (float)yi;
                }
            }
        }
        Rr[e] = xr;
        Ri[e] = xi;
    }
    for (long long e = tid; e < mm; e += kThreads) {
        const int c = (int)(e % m);
        if (c >= k) continue;
        const double dr = Wr[(long long)c * n + c], di = Wi[(long long)c * n + c];
        const double ad = sqrt(dr * dr + di * di);
        if (!(ad > 0.0)) continue;
        const double pr = dr / ad, pi = di / ad;  // column c times d / |d|
        const double xr = Qr[e], xi = Qi[e];
        Qr[e] = (float)(xr * pr - xi * pi);
        Qi[e] = (float)(xr * pi + xi * pr);
    }
}

}  // namespace

hipError_t launch_slice_inv(const float* ar, const float* ai, float* wr, float* wi, float* br, float* bi, int n,
                            int nslices, int* info, hipStream_t st)
{
    k_slice_inv<<<nslices, kThreads, 0, st>>>(ar, ai, wr, wi, br, bi, n, info);
    return hipGetLastError();
}

hipError_t launch_slice_qr(const float* ar, const float* ai, float* wr, float* wi, float* vr, float* vi,
                           double* beta, float* qr, float* qi, float* rr, float* ri, int m, int n, int nslices,
                           hipStream_t st)
{
    k_slice_qr<<<nslices, kThreads, 0, st>>>(ar, ai, wr, wi, vr, vi, beta, qr, qi, rr, ri, m, n);
    return hipGetLastError();
}

}  // namespace tp

namespace {

constexpr int kMaxInvN = 1024;  // the factor staging of the inverse

struct InvLayout {
    tp::Planes a, w, b;
};
tp::Arena inv_arena(void* ws, size_t bytes, int n, int n3, InvLayout* out)
{
    const size_t h = (size_t)tp::half_slices(n3), nn = (size_t)n * n;
    tp::Arena ar(ws, bytes);
    InvLayout t;
    t.a.re = ar.take<float>(h * nn);
    t.a.im = ar.take<float>(h * nn);
    t.w.re = ar.take<float>(2 * h * nn);
    t.w.im = ar.take<float>(2 * h * nn);
    t.b.re = ar.take<float>(h * nn);
    t.b.im = ar.take<float>(h * nn);
    if (out) *out = t;
    return ar;
}

struct QrLayout {
    tp::Planes a, w, v, q, r;
    double* beta;
};
tp::Arena qr_arena(void* ws, size_t bytes, int m, int n, int n3, QrLayout* out)
{
    const size_t h = (size_t)tp::half_slices(n3), k = (size_t)(m < n ? m : n);
    tp::Arena ar(ws, bytes);
    QrLayout t;
    t.a.re = ar.take<float>(h * m * n);
    t.a.im = ar.take<float>(h * m * n);
    t.w.re = ar.take<float>(h * m * n);
    t.w.im = ar.take<float>(h * m * n);
    t.v.re = ar.take<float>(h * m * k);
    t.v.im = ar.take<float>(h * m * k);
    t.q.re = ar.take<float>(h * m * m);
    t.q.im = ar.take<float>(h * m * m);
    t.r.re = ar.take<float>(h * m * n);
    t.r.im = ar.take<float>(h * m * n);
    t.beta = ar.take<double>(h * k);
    if (out) *out = t;
    return ar;
}

bool bad_tensor(int a, int b, int n3) { return a <= 0 || b <= 0 || n3 <= 0 || n3 > 1024 || (long long)a * b >= (1LL << 31); }

}  // namespace

extern "C" {

size_t tp_tinv_workspace_size(int n, int n3)
{
    if (bad_tensor(n, n, n3) || n > kMaxInvN) return 0;
    return inv_arena(nullptr, 0, n, n3, nullptr).used;
}

int tp_tinv(const float* A, float* B, int n, int n3, int* info, void* workspace, size_t workspace_bytes,
            void* stream)
{
    if (!A || !B) return TP_ERR_ARG;
    if (bad_tensor(n, n, n3) || n > kMaxInvN) return TP_ERR_SHAPE;
    InvLayout W;
    tp::Arena ar = inv_arena(workspace, workspace_bytes, n, n3, &W);
    if (!ar.ok) return TP_ERR_WORKSPACE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int h = tp::half_slices(n3);
    const long long ntubes = (long long)n * n;
    TP_LAUNCH(tp::K_RFFT, s, tp::launch_rfft(A, W.a.re, W.a.im, ntubes, n3, s));
    TP_LAUNCH(tp::K_TENSOR_OP, s, tp::launch_slice_inv(W.a.re, W.a.im, W.w.re, W.w.im, W.b.re, W.b.im, n, h, info, s));
    TP_LAUNCH(tp::K_IRFFT, s, tp::launch_irfft(W.b.re, W.b.im, B, ntubes, n3, s));
    return TP_OK;
}

size_t tp_tqr_workspace_size(int n1, int n2, int n3)
{
    if (bad_tensor(n1, n2, n3) || bad_tensor(n1, n1, n3)) return 0;
    return qr_arena(nullptr, 0, n1, n2, n3, nullptr).used;
}

int tp_tqr(const float* A, float* Q, float* R, int n1, int n2, int n3, void* workspace, size_t workspace_bytes,
           void* stream)
{
    if (!A || !Q || !R) return TP_ERR_ARG;
    if (bad_tensor(n1, n2, n3) || bad_tensor(n1, n1, n3)) return TP_ERR_SHAPE;
    QrLayout W;
    tp::Arena ar = qr_arena(workspace, workspace_bytes, n1, n2, n3, &W);
    if (!ar.ok) return TP_ERR_WORKSPACE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int h = tp::half_slices(n3);
    TP_LAUNCH(tp::K_RFFT, s, tp::launch_rfft(A, W.a.re, W.a.im, (long long)n1 * n2, n3, s));
    TP_LAUNCH(tp::K_TENSOR_OP, s,
              tp::launch_slice_qr(W.a.re, W.a.im, W.w.re, W.w.im, W.v.re, W.v.im, W.beta, W.q.re, W.q.im, W.r.re,
                                  W.r.im, n1, n2, h, s));
    TP_LAUNCH(tp::K_IRFFT, s, tp::launch_irfft(W.q.re, W.q.im, Q, (long long)n1 * n1, n3, s));
    TP_LAUNCH(tp::K_IRFFT, s, tp::launch_irfft(W.r.re, W.r.im, R, (long long)n1 * n2, n3, s));
    return TP_OK;
}

}  // extern "C"
