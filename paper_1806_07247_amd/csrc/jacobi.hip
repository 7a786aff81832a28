// Per-slice SVD by one-sided (Hestenes) Jacobi, the "SVD" of Algorithms 2 and
// 3 (step 2), and the singular value shrinkage of Theorem 2.3 / eq (21).
//
// One workgroup owns one Fourier slice.  The slice (or its conjugate
// transpose when it is wide, so that the work matrix is R x P with R >= P) is
// held column-major as float2 (re, im), in LDS when it fits and otherwise in a
// workspace buffer.  A sweep visits all P(P-1)/2 column pairs in P'-1 steps of
// P'/2 disjoint pairs (round-robin "circle" order, P' = P rounded up to even);
// a barrier separates steps.  A group of G lanes handles one pair: each lane
// holds RPL rows of both columns in registers, accumulates
//   alpha = ||x||^2, beta = ||y||^2, gamma = x^* y
// in FP64 (products of FP32 values are exact in FP64), reduces them with an
// xor butterfly (every lane ends with bitwise identical sums, so all lanes
// take the same decision), and when |gamma| > tol sqrt(alpha beta) applies
// the rotation that zeroes gamma.  The rotation (zeta, t, c, s and the phase
// of gamma) is computed in FP64 and applied to the FP32 columns.  The
// iteration stops after a sweep without rotations (info = sweeps used), or at
// max_sweeps (info = -max_sweeps).
//
// Real slices stay real: with zero imaginary parts gamma is real, its phase
// is +-1 and every update keeps the imaginary parts at zero.
//
// Outputs: the rotated columns w_j = (Y V)_j (row-major R x P, planar) and
// sigma_j = ||w_j|| in FP64, unsorted.
#include "tp_internal.h"

namespace tp {
namespace {

// Column index at position `pos` of step `step` of the circle order over np
// (even) columns: position 0 is fixed, the others rotate.
__device__ __forceinline__ int rr_col(int pos, int step, int np)
{
    return pos == 0 ? 0 : 1 + (pos - 1 + step) % (np - 1);
}

template <int G>
__device__ __forceinline__ double group_sum(double v)
{
#pragma unroll
    for (int m = G / 2; m >= 1; m >>= 1) v += __shfl_xor(v, m, G);
    return v;
}

template <int G, int RPL, bool LDS>
__global__ __launch_bounds__(256) void k_jacobi(JacobiArgs a, float2* __restrict__ gwork)
{
    extern __shared__ float2 lwork[];
    __shared__ int rotated;
    const int s = blockIdx.x;
    const int R = a.transpose ? a.n : a.m;
    const int P = a.transpose ? a.m : a.n;
    const int ldr = R;
    float2* work = LDS ? lwork : gwork + (long long)s * R * P;
    const long long so = (long long)s * a.m * a.n;
    const float* yr = a.yr + so;
    const float* yi = a.yi + so;
    const int tid = threadIdx.x, nthr = blockDim.x;

    // load the work matrix, column-major
    const int total = R * P;
    if (!a.transpose) {
        for (int e = tid; e < total; e += nthr) {  // Y is row-major m x n: e = i*n + j
            const int i = e / P, j = e % P;
            work[j * ldr + i] = make_float2(yr[e], yi[e]);
        }
    } else {
        for (int e = tid; e < total; e += nthr) {  // column j of Y^* is conj(row j of Y)
            const int j = e / R, i = e % R;
            work[j * ldr + i] = make_float2(yr[e], -yi[e]);
        }
    }
    if (tid == 0) rotated = 0;
    __syncthreads();

    const int np = P + (P & 1);
    const int group = tid / G, gl = tid % G, ngroups = nthr / G;
    const double tol = a.tol;
    int sweep = 0;
    bool converged = (P < 2);
    while (!converged && sweep < a.max_sweeps) {
        for (int step = 0; step < np - 1; ++step) {
            for (int pair = group; pair < np / 2; pair += ngroups) {
                const int p = rr_col(pair, step, np);
                const int q = rr_col(np - 1 - pair, step, np);
                if (p >= P || q >= P) continue;
                float2* xc = work + p * ldr;
                float2* yc = work + q * ldr;
                float2 x[RPL], y[RPL];
                double al = 0.0, be = 0.0, gr = 0.0, gi = 0.0;
#pragma unroll
                for (int t = 0; t < RPL; ++t) {
                    const int i = gl + G * t;
                    if (i < R) {
                        x[t] = xc[i];
                        y[t] = yc[i];
                    } else {
                        x[t] = make_float2(0.f, 0.f);
                        y[t] = make_float2(0.f, 0.f);
                    }
                    const double xr = x[t].x, xi = x[t].y, yr_ = y[t].x, yi_ = y[t].y;
                    al = fma(xr, xr, fma(xi, xi, al));
                    be = fma(yr_, yr_, fma(yi_, yi_, be));
                    gr = fma(xr, yr_, fma(xi, yi_, gr));
                    gi = fma(xr, yi_, fma(-xi, yr_, gi));
                }
                al = group_sum<G>(al);
                be = group_sum<G>(be);
                gr = group_sum<G>(gr);
                gi = group_sum<G>(gi);
                const double g = sqrt(gr * gr + gi * gi);
                if (g > 0.0 && g > tol * sqrt(al) * sqrt(be)) {
                    // x' = c x - s conj(e) y,  y' = s e x + c y,  e = gamma/|gamma|
                    const double zeta = (be - al) / (2.0 * g);
                    const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                    const double c = 1.0 / sqrt(1.0 + t * t);
                    const double sn = c * t;
                    const double er = gr / g, ei = gi / g;
                    const float cf = (float)c;
                    const float sr = (float)(sn * er), si = (float)(sn * ei);  // s e
#pragma unroll
                    for (int t2 = 0; t2 < RPL; ++t2) {
                        const int i = gl + G * t2;
                        if (i < R) {
                            const float2 xv = x[t2], yv = y[t2];
                            // s conj(e) y = (sr*yr + si*yi, sr*yi - si*yr)
                            xc[i] = make_float2(cf * xv.x - (sr * yv.x + si * yv.y), cf * xv.y - (sr * yv.y - si * yv.x));
                            // s e x = (sr*xr - si*xi, sr*xi + si*xr)
                            yc[i] = make_float2((sr * xv.x - si * xv.y) + cf * yv.x, (sr * xv.y + si * xv.x) + cf * yv.y);
                        }
                    }
                    if (gl == 0) rotated = 1;
                }
            }
            __syncthreads();
        }
        ++sweep;
        converged = (rotated == 0);
        __syncthreads();
        if (tid == 0) rotated = 0;
        __syncthreads();
    }

    // column norms in FP64 and the rotated columns, row-major R x P
    double* sig = a.sigma + (long long)s * P;
    for (int j = tid / G; j < P; j += ngroups) {
        double acc = 0.0;
        for (int i = gl; i < R; i += G) {
            const float2 v = work[j * ldr + i];
            acc = fma((double)v.x, (double)v.x, fma((double)v.y, (double)v.y, acc));
        }
        acc = group_sum<G>(acc);
        if (gl == 0) sig[j] = sqrt(acc);
    }
    if (a.wr) {
        float* wr = a.wr + (long long)s * R * P;
        float* wi = a.wi + (long long)s * R * P;
        for (int e = tid; e < total; e += nthr) {
            const int i = e / P, j = e % P;
            const float2 v = work[j * ldr + i];
            wr[e] = v.x;
            wi[e] = v.y;
        }
    }
    if (a.info && tid == 0) a.info[s] = converged ? (sweep > 0 ? sweep : 1) : -sweep;
}

constexpr size_t kMaxLds = 160 * 1024 - 1024;

template <int G, int RPL>
hipError_t launch_rpl(const JacobiArgs& a, void* scratch, int R, int P, hipStream_t st)
{
    const size_t lds = (size_t)R * P * sizeof(float2);
    if (lds <= kMaxLds) {
        auto kern = k_jacobi<G, RPL, true>;
        static bool attr = false;
        if (!attr) {
            hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds);
            if (e != hipSuccess) return e;
            attr = true;
        }
        kern<<<a.nslices, 256, lds, st>>>(a, nullptr);
    } else {
        k_jacobi<G, RPL, false><<<a.nslices, 256, 0, st>>>(a, static_cast<float2*>(scratch));
    }
    return hipGetLastError();
}

}  // namespace

size_t jacobi_scratch_bytes(int m, int n, int nslices)
{
    const size_t lds = (size_t)m * n * sizeof(float2);
    return lds <= kMaxLds ? 0 : lds * nslices;
}

hipError_t launch_jacobi(const JacobiArgs& a, void* scratch, size_t scratch_bytes, hipStream_t st)
{
    if (a.nslices <= 0) return hipSuccess;
    const int R = a.transpose ? a.n : a.m;
    const int P = a.transpose ? a.m : a.n;
    if (jacobi_scratch_bytes(a.m, a.n, a.nslices) > scratch_bytes) return hipErrorInvalidValue;
    if (R <= 32) return launch_rpl<16, 2>(a, scratch, R, P, st);
    if (R <= 64) return launch_rpl<16, 4>(a, scratch, R, P, st);
    if (R <= 128) return launch_rpl<16, 8>(a, scratch, R, P, st);
    if (R <= 256) return launch_rpl<16, 16>(a, scratch, R, P, st);
    if (R <= 512) return launch_rpl<64, 8>(a, scratch, R, P, st);
    if (R <= 1024) return launch_rpl<64, 16>(a, scratch, R, P, st);
    if (R <= 2048) return launch_rpl<64, 32>(a, scratch, R, P, st);
    return hipErrorInvalidValue;
}

// ------------------------------------------------------------------ shrink --
namespace {

// w_j <- w_j * sqrt(d_j) / sigma_j with d_j = (1 - tau/sigma_j)_+ (eq (21));
// keep[s] = #{j : sigma_j > tau}.
__global__ __launch_bounds__(256) void k_shrink(float* __restrict__ wr, float* __restrict__ wi,
                                                const double* __restrict__ sigma, int* __restrict__ keep, int R,
                                                int P, long long total, double tau)
{
    const long long e0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long per = (long long)R * P;
    for (long long e = e0; e < total; e += (long long)gridDim.x * blockDim.x) {
        const long long s = e / per;
        const int j = (int)(e % P);
        const double sg = sigma[s * P + j];
        float f = 0.0f;
        if (sg > tau) f = (float)(sqrt(1.0 - tau / sg) / sg);
        wr[e] *= f;
        wi[e] *= f;
    }
    if (keep && e0 < total / per) {
        const long long s = e0;
        int k = 0;
        for (int j = 0; j < P; ++j) k += sigma[s * P + j] > tau ? 1 : 0;
        keep[s] = k;
    }
}

// tnn = (1/n3) sum_k w_k sum_j sigma_kj, w_k = 1 for real slices, 2 otherwise
// (Definition 2.9 with eq (14), using the conjugate symmetry of eq (8)).
__global__ __launch_bounds__(256) void k_tnn_reduce(const double* __restrict__ sigma, int nslices, int P, int n3,
                                                    double* __restrict__ out)
{
    __shared__ double part[256];
    double acc = 0.0;
    for (int s = 0; s < nslices; ++s) {  // fixed order: deterministic
        const bool real = (s == 0) || (n3 % 2 == 0 && s == n3 / 2);
        double v = 0.0;
        for (int j = threadIdx.x; j < P; j += blockDim.x) v += sigma[(long long)s * P + j];
        acc += real ? v : 2.0 * v;
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = part[0] / (double)n3;
}

}  // namespace

hipError_t launch_shrink(float* wr, float* wi, const double* sigma, int* keep, int R, int P, int nslices, double tau,
                         hipStream_t st)
{
    const long long total = (long long)R * P * nslices;
    if (total <= 0) return hipSuccess;
    long long blocks = (total + 255) / 256;
    if (blocks > 256 * 32) blocks = 256 * 32;
    if (blocks * 256 < nslices) blocks = (nslices + 255) / 256;
    k_shrink<<<(int)blocks, 256, 0, st>>>(wr, wi, sigma, keep, R, P, total, tau);
    return hipGetLastError();
}

hipError_t launch_tnn_reduce(const double* sigma, int nslices, int P, int n3, double* out, hipStream_t st)
{
    k_tnn_reduce<<<1, 256, 0, st>>>(sigma, nslices, P, n3, out);
    return hipGetLastError();
}

}  // namespace tp
