// Real DFT along the mode-3 tubes (Section 2.2, eq (2); fft(A,[],3) of
// Algorithms 1-3, step 1) and its inverse (step 3), for gfx950.
//
// Layout: the tensor is tube-major (n1, n2, n3), so a block of consecutive
// tubes is one contiguous span of memory.  A workgroup of one wavefront takes
// 64 tubes and each lane transforms one tube in registers.  The forward
// transform reads each lane's tube with 16-byte loads (the lines a wavefront
// touches are consumed from L1 over its next loads; no LDS, so more
// wavefronts fit a compute unit), or stages the 64-tube span through LDS with
// coalesced loads; the inverse stages its output through LDS and writes the
// span coalesced.  The Fourier side is slice-major planar
// complex: bin k of tube q is re[k*ntubes + q], im[k*ntubes + q], so the
// per-bin stores of a wavefront are 64 consecutive floats; the transpose from
// tube-major to slice-major costs no extra pass.
//
// Only the floor(n3/2)+1 leading bins are produced (Lemma 2.1 / eq (8)): the
// others are the conjugates of these.  The inverse reads the same half
// spectrum and forms the conjugate fill of step 2 implicitly.
//
// Power-of-two n3 (4..128): a complex FFT of length n3/2 on the packed
// sequence z_t = x_2t + i x_2t+1 (radix-2, fully unrolled in registers), then
// the even/odd split, with compile-time twiddles.  Other n3: a direct DFT
// per lane, with twiddles computed per workgroup in double precision
// (sincospi) and rounded once.
#include "tp_internal.h"

namespace tp {
namespace {

constexpr int kTubes = 64;  // tubes per workgroup (one wavefront)

__device__ void fill_twiddles(float2* tw, int n)
{
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        double s, c;
        sincospi(-2.0 * (double)j / (double)n, &s, &c);  // W_n^j = exp(-2 pi i j / n)
        tw[j] = make_float2((float)c, (float)s);
    }
}

// Twiddles of the power-of-two lengths as compile-time constants,
// W_N^j = exp(-2 pi i j / N): cos and sin of 2 pi j / N in double (reduction
// to an octant, Taylor series on [0, pi/4), exact octant rotations), rounded
// once to float.  The fully unrolled transforms index them with constants,
// so they become instruction literals and take no registers or LDS.
constexpr double kCxPi = 3.14159265358979323846264338327950288;
constexpr double cx_sin_small(double x)
{
    double t = x, s = x;
    for (int k = 1; k < 14; ++k) {
        t *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
        s += t;
    }
    return s;
}
constexpr double cx_cos_small(double x)
{
    double t = 1.0, s = 1.0;
    for (int k = 1; k < 14; ++k) {
        t *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
        s += t;
    }
    return s;
}
template <int N>
struct TwTab {
    float re[N], im[N];
};
template <int N>
constexpr TwTab<N> make_twiddles()
{
    TwTab<N> t{};
    for (int j = 0; j < N; ++j) {
        const long o = (8L * j) / N, r = 8L * j - o * N;  // angle = (pi/4)(o + r/N)
        const double x = (kCxPi / 4.0) * (double)r / (double)N;
        double c = cx_cos_small(x), sn = cx_sin_small(x);
        const double h = 0.70710678118654752440084436210484903;
        for (long q = 0; q < o; ++q) {
            const double nc = (c - sn) * h, ns = (sn + c) * h;
            c = nc;
            sn = ns;
        }
        t.re[j] = (float)c;
        t.im[j] = (float)(-sn);
    }
    return t;
}
template <int N>
__device__ __forceinline__ float2 twc(int j)
{
    constexpr TwTab<N> T = make_twiddles<N>();
    return make_float2(T.re[j], T.im[j]);
}

template <int M>
__device__ constexpr int bitrev(int t)
{
    int r = 0;
    for (int b = 1; b < M; b <<= 1) {
        r = (r << 1) | (t & 1);
        t >>= 1;
    }
    return r;
}

// In-place radix-2 DIT FFT of length M = N/2 on bit-reversed input.  The
// twiddle W_len^j is W_N^(j*N/len) from the length-N table; INV conjugates it.
template <int N, bool INV>
__device__ __forceinline__ void cfft_half(float (&zr)[N / 2], float (&zi)[N / 2])
{
    constexpr int M = N / 2;
#pragma unroll
    for (int len = 2; len <= M; len <<= 1) {
#pragma unroll
        for (int b = 0; b < M; b += len) {
#pragma unroll
            for (int j = 0; j < len / 2; ++j) {
                const int i0 = b + j, i1 = i0 + len / 2;
                float tr, ti;
                if (j == 0) {
                    tr = zr[i1];
                    ti = zi[i1];
                } else {
                    float2 w = twc<N>(j * (N / len));
                    if (INV) w.y = -w.y;
                    tr = zr[i1] * w.x - zi[i1] * w.y;
                    ti = zr[i1] * w.y + zi[i1] * w.x;
                }
                zr[i1] = zr[i0] - tr;
                zi[i1] = zi[i0] - ti;
                zr[i0] += tr;
                zi[i0] += ti;
            }
        }
    }
}

// coalesced copy of nt*n floats from global into the padded LDS tile (row per tube)
__device__ __forceinline__ void load_tile(const float* __restrict__ src, float* buf, int nt, int n, int ld)
{
    const int total = nt * n;
    if ((n & 3) == 0 && (reinterpret_cast<uintptr_t>(src) & 15) == 0) {
        for (int e = threadIdx.x * 4; e < total; e += blockDim.x * 4) {
            const float4 v = *reinterpret_cast<const float4*>(src + e);
            float* d = buf + (e / n) * ld + (e % n);
            d[0] = v.x;
            d[1] = v.y;
            d[2] = v.z;
            d[3] = v.w;
        }
    } else {
        for (int e = threadIdx.x; e < total; e += blockDim.x) buf[(e / n) * ld + (e % n)] = src[e];
    }
}

__device__ __forceinline__ void store_tile(float* __restrict__ dst, const float* buf, int nt, int n, int ld)
{
    const int total = nt * n;
    if ((n & 3) == 0 && (reinterpret_cast<uintptr_t>(dst) & 15) == 0) {
        for (int e = threadIdx.x * 4; e < total; e += blockDim.x * 4) {
            const float* s = buf + (e / n) * ld + (e % n);
            *reinterpret_cast<float4*>(dst + e) = make_float4(s[0], s[1], s[2], s[3]);
        }
    } else {
        for (int e = threadIdx.x; e < total; e += blockDim.x) dst[e] = buf[(e / n) * ld + (e % n)];
    }
}

// coalesced copy of the LDS tile (nt rows of `cols` floats, leading dimension
// ld) to global rows `gstride` floats apart (a column block of nt tubes)
__device__ __forceinline__ void store_tile_cols(float* __restrict__ dst, const float* buf, int nt, int cols, int ld,
                                                int gstride)
{
    const int total = nt * cols;
    if ((cols & 3) == 0 && (gstride & 3) == 0 && (reinterpret_cast<uintptr_t>(dst) & 15) == 0) {
        for (int e = threadIdx.x * 4; e < total; e += blockDim.x * 4) {
            const int r = e / cols, c = e % cols;
            const float* sp = buf + r * ld + c;
            *reinterpret_cast<float4*>(dst + (long long)r * gstride + c) = make_float4(sp[0], sp[1], sp[2], sp[3]);
        }
    } else {
        for (int e = threadIdx.x; e < total; e += blockDim.x) dst[(long long)(e / cols) * gstride + e % cols] =
            buf[(e / cols) * ld + e % cols];
    }
}

// Bins 0 .. N/2 of the real length-N input from the length-N/2 transform Z of
// its packed pairs: X_k = E_k + W_N^k O_k with E = (Z_k + conj Z_{M-k})/2,
// O = -i (Z_k - conj Z_{M-k})/2; put(k, re, im) takes each bin.
template <int N, class Put>
__device__ __forceinline__ void rfft_bins(const float (&zr)[N / 2], const float (&zi)[N / 2], Put&& put)
{
    constexpr int M = N / 2;
    put(0, zr[0] + zi[0], 0.0f);
    put(M, zr[0] - zi[0], 0.0f);
#pragma unroll
    for (int k = 1; k < M; ++k) {
        const float ar = zr[k], ai = zi[k], br = zr[M - k], bi = -zi[M - k];
        const float er = 0.5f * (ar + br), ei = 0.5f * (ai + bi);
        const float dr = 0.5f * (ar - br), di = 0.5f * (ai - bi);
        const float orr = di, oi = -dr;
        const float2 w = twc<N>(k);
        put(k, er + (w.x * orr - w.y * oi), ei + (w.x * oi + w.y * orr));
    }
}

// Forward transform of the nt (<= 64) tubes starting at tube `base` of a
// tensor with `ntubes` tubes; tw holds W_N^j, buf 64 x (N+1) floats.
template <int N>
__device__ __forceinline__ void rfft_tile(const float* __restrict__ x, float* __restrict__ re, float* __restrict__ im,
                                          long long ntubes, long long base, int nt, const float2* tw, float* buf)
{
    constexpr int M = N / 2, LD = N + 1;
    const int tid = threadIdx.x;
    load_tile(x + base * N, buf, nt, N, LD);
    __syncthreads();
    if (tid < nt) {
        float zr[M], zi[M];
        const float* xt = buf + tid * LD;
#pragma unroll
        for (int t = 0; t < M; ++t) {
            zr[bitrev<M>(t)] = xt[2 * t];
            zi[bitrev<M>(t)] = xt[2 * t + 1];
        }
        cfft_half<N, false>(zr, zi);
        const long long q = base + tid;
        rfft_bins<N>(zr, zi, [&](int k, float vr, float vi) {
            re[(long long)k * ntubes + q] = vr;
            im[(long long)k * ntubes + q] = vi;
        });
    }
}

template <int N>
__global__ __launch_bounds__(kTubes) void k_rfft_pow2(const float* __restrict__ x, float* __restrict__ re,
                                                       float* __restrict__ im, long long ntubes)
{
    __shared__ float buf[kTubes * (N + 1)];
    for (long long base = (long long)blockIdx.x * kTubes; base < ntubes; base += (long long)gridDim.x * kTubes) {
        const int nt = (int)min<long long>(kTubes, ntubes - base);
        __syncthreads();
        rfft_tile<N>(x, re, im, ntubes, base, nt, nullptr, buf);
    }
}

// The same transform with each lane loading its own tube straight from
// global memory (16-byte loads, no LDS staging): less LDS per wavefront, so
// more wavefronts per compute unit; the lines a wavefront touches are reused
// from the L1 cache over its next loads.
template <int N>
__global__ __launch_bounds__(kTubes) void k_rfft_pow2_direct(const float* __restrict__ x, float* __restrict__ re,
                                                              float* __restrict__ im, long long ntubes)
{
    constexpr int M = N / 2;
    const int tid = threadIdx.x;
    for (long long base = (long long)blockIdx.x * kTubes; base < ntubes; base += (long long)gridDim.x * kTubes) {
        const long long q = base + tid;
        if (q >= ntubes) continue;
        float zr[M], zi[M];
        const float4* xt = reinterpret_cast<const float4*>(x + q * N);
#pragma unroll
        for (int t = 0; t < M / 2; ++t) {
            const float4 v = xt[t];
            zr[bitrev<M>(2 * t)] = v.x;
            zi[bitrev<M>(2 * t)] = v.y;
            zr[bitrev<M>(2 * t + 1)] = v.z;
            zi[bitrev<M>(2 * t + 1)] = v.w;
        }
        cfft_half<N, false>(zr, zi);
        rfft_bins<N>(zr, zi, [&](int k, float vr, float vi) {
            re[(long long)k * ntubes + q] = vr;
            im[(long long)k * ntubes + q] = vi;
        });
    }
}

// ------------------------------------------------- bf16 plane output --
// Element t of a plane slice in storage order (k-blocked, see SplitOut):
// its tube, or -1 for padding.  Consecutive lanes write consecutive
// elements of a plane.
__device__ __forceinline__ long long split_tube(const SplitOut& o, long long t)
{
    const long long panel = (long long)o.outer * o.bkl;
    const long long kb = t / panel, rem = t - kb * panel;
    const long long r = rem / o.bkl, i = kb * o.bkl + (rem - r * o.bkl);
    return i < o.inner ? r * o.q_outer + i * o.q_inner : -1;
}

__device__ __forceinline__ unsigned short bf16_bits(float v) { return __builtin_bit_cast(unsigned short, (__bf16)v); }

// bin k of one tube: hi = bf16(v) (round to nearest even), lo = bf16(v - hi)
__device__ __forceinline__ void put_split(const SplitOut& o, long long pos, int k, float vr, float vi)
{
    unsigned short* d = o.p + (long long)k * o.slice + pos;
    const __bf16 hr = (__bf16)vr, hi = (__bf16)vi;
    d[0] = __builtin_bit_cast(unsigned short, hr);
    d[o.plane] = __builtin_bit_cast(unsigned short, hi);
    if (o.split) {
        d[2 * o.plane] = bf16_bits(vr - (float)hr);
        d[3 * o.plane] = bf16_bits(vi - (float)hi);
    }
}

__device__ __forceinline__ void put_zero(const SplitOut& o, long long pos, int h)
{
    for (int k = 0; k < h; ++k) put_split(o, pos, k, 0.0f, 0.0f);
}

// Power-of-two N: each lane transforms one tube read with 16-byte loads (as
// k_rfft_pow2_direct) and writes its bins to the planes.
template <int N>
__global__ __launch_bounds__(kTubes) void k_rfft_split(const float* __restrict__ x, SplitOut o)
{
    constexpr int M = N / 2;
    const long long total = (long long)o.outer * o.ld;
    for (long long t = (long long)blockIdx.x * kTubes + threadIdx.x; t < total; t += (long long)gridDim.x * kTubes) {
        const long long q = split_tube(o, t);
        if (q < 0) {
            put_zero(o, t, M + 1);
            continue;
        }
        float zr[M], zi[M];
        const float4* xt = reinterpret_cast<const float4*>(x + q * N);
#pragma unroll
        for (int u = 0; u < M / 2; ++u) {
            const float4 v = xt[u];
            zr[bitrev<M>(2 * u)] = v.x;
            zi[bitrev<M>(2 * u)] = v.y;
            zr[bitrev<M>(2 * u + 1)] = v.z;
            zi[bitrev<M>(2 * u + 1)] = v.w;
        }
        cfft_half<N, false>(zr, zi);
        rfft_bins<N>(zr, zi, [&](int k, float vr, float vi) { put_split(o, t, k, vr, vi); });
    }
}

// Any n: direct DFT per lane on its tube staged in LDS (blockDim.x x (n+1)
// floats after the n twiddles), as rdft_tile.
__global__ void k_rdft_split_any(const float* __restrict__ x, SplitOut o, int n)
{
    extern __shared__ float smem[];
    float2* tw = reinterpret_cast<float2*>(smem);
    float* xt = smem + 2 * n + threadIdx.x * (n + 1);
    fill_twiddles(tw, n);
    __syncthreads();
    const int h = n / 2 + 1;
    const long long total = (long long)o.outer * o.ld;
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (long long)gridDim.x * blockDim.x) {
        const long long q = split_tube(o, t);
        if (q < 0) {
            put_zero(o, t, h);
            continue;
        }
        for (int u = 0; u < n; ++u) xt[u] = x[q * n + u];
        for (int k = 0; k < h; ++k) {
            float sr = 0.0f, si = 0.0f;
            int e = 0;
            for (int u = 0; u < n; ++u) {
                const float v = xt[u];
                const float2 w = tw[e];
                sr += v * w.x;
                si += v * w.y;
                e += k;
                if (e >= n) e -= n;
            }
            put_split(o, t, k, sr, (k == 0 || 2 * k == n) ? 0.0f : si);
        }
    }
}

// Inverse transform of the nt tubes starting at `base` (see rfft_tile).
// HALF: the output goes through a half-width LDS tile (N/2 + 1 floats per
// tube) in two passes, for more wavefronts per compute unit at large N.  All
// barriers are reached by every lane.
template <int N, bool HALF = false>
__device__ __forceinline__ void irfft_tile(const float* __restrict__ re, const float* __restrict__ im,
                                           float* __restrict__ x, long long ntubes, long long base, int nt,
                                           const float2* tw, float* buf)
{
    constexpr int M = N / 2, LD = N + 1;
    const int tid = threadIdx.x;
    const bool act = tid < nt;
    const float scale = 1.0f / (float)N;
    float zr[M], zi[M];
    if (act) {
        const long long q = base + tid;
        // 2 Z_k = (X_k + conj X_{M-k}) + i W_N^{-k} (X_k - conj X_{M-k}).  Bins k
        // and M-k feed both Z_k and Z_{M-k}: they are loaded as a pair and
        // consumed at once (a few pairs in flight), so the M+1 bins are never
        // all live in registers.
#pragma unroll
        for (int k = 0; k <= M / 2; ++k) {
            const int k2 = M - k;  // partner bin (M for k = 0)
            const float xr_a = re[(long long)k * ntubes + q];
            const float xi_a = (k == 0) ? 0.0f : im[(long long)k * ntubes + q];
            const float xr_b = (k2 == k) ? xr_a : re[(long long)k2 * ntubes + q];
            const float xi_b = (k2 == M || k2 == k) ? ((k2 == k) ? xi_a : 0.0f) : im[(long long)k2 * ntubes + q];
            auto zk = [&](int kk, float ar, float ai, float br, float bi) {
                const float sr = ar + br, si = ai + bi, dr = ar - br, di = ai - bi;
                const float2 w = twc<N>(kk);  // conj applied below
                const float tr = w.x * dr + w.y * di;
                const float ti = w.x * di - w.y * dr;
                zr[bitrev<M>(kk)] = sr - ti;
                zi[bitrev<M>(kk)] = si + tr;
            };
            zk(k, xr_a, xi_a, xr_b, -xi_b);
            if (k > 0 && k2 != k) zk(k2, xr_b, xi_b, xr_a, -xi_a);
            if ((k & 7) == 7) __builtin_amdgcn_sched_barrier(0);
        }
        cfft_half<N, true>(zr, zi);
    }
    if (!HALF) {
        if (act) {
            float* xt = buf + tid * LD;
#pragma unroll
            for (int t = 0; t < M; ++t) {
                xt[2 * t] = zr[t] * scale;
                xt[2 * t + 1] = zi[t] * scale;
            }
        }
        __syncthreads();
        store_tile(x + base * N, buf, nt, N, LD);
    } else {
        float* xt = buf + tid * (M + 1);
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            if (half) __syncthreads();  // the first half has been stored
            if (act) {
#pragma unroll
                for (int t = 0; t < M / 2; ++t) {
                    xt[2 * t] = zr[t + half * M / 2] * scale;
                    xt[2 * t + 1] = zi[t + half * M / 2] * scale;
                }
            }
            __syncthreads();
            store_tile_cols(x + base * N + half * M, buf, nt, M, M + 1, N);
        }
    }
}

template <int N>
__global__ __launch_bounds__(kTubes) void k_irfft_pow2(const float* __restrict__ re, const float* __restrict__ im,
                                                        float* __restrict__ x, long long ntubes)
{
    constexpr bool HALF = N >= 64;  // half-width staging tile at the larger lengths
    __shared__ float buf[kTubes * (HALF ? N / 2 + 1 : N + 1)];
    for (long long base = (long long)blockIdx.x * kTubes; base < ntubes; base += (long long)gridDim.x * kTubes) {
        const int nt = (int)min<long long>(kTubes, ntubes - base);
        __syncthreads();
        irfft_tile<N, HALF>(re, im, x, ntubes, base, nt, nullptr, buf);
    }
}

// direct DFT of any length n: X_k = sum_t x_t W_n^(k t), k < n/2+1, for the
// nt (<= blockDim.x) tubes starting at `base`; buf holds blockDim.x x (n+1)
__device__ __forceinline__ void rdft_tile(const float* __restrict__ x, float* __restrict__ re, float* __restrict__ im,
                                          long long ntubes, long long base, int nt, int n, const float2* tw,
                                          float* buf)
{
    const int ld = n + 1, h = n / 2 + 1, tid = threadIdx.x;
    load_tile(x + base * n, buf, nt, n, ld);
    __syncthreads();
    if (tid < nt) {
        const long long q = base + tid;
        const float* xt = buf + tid * ld;
        for (int k = 0; k < h; ++k) {
            float sr = 0.0f, si = 0.0f;
            int e = 0;
            for (int t = 0; t < n; ++t) {
                const float v = xt[t];
                const float2 w = tw[e];
                sr += v * w.x;
                si += v * w.y;
                e += k;
                if (e >= n) e -= n;
            }
            re[(long long)k * ntubes + q] = sr;
            im[(long long)k * ntubes + q] = (k == 0 || 2 * k == n) ? 0.0f : si;
        }
    }
}

// x_t = (1/n) [X_0 + (-1)^t X_{n/2} + 2 sum_{0<k<n/2} Re(X_k W_n^(-k t))]
__device__ __forceinline__ void irdft_tile(const float* __restrict__ re, const float* __restrict__ im,
                                           float* __restrict__ x, long long ntubes, long long base, int nt, int n,
                                           const float2* tw, float* buf)
{
    const int ld = n + 1, kmax = (n - 1) / 2, tid = threadIdx.x;
    const float scale = 1.0f / (float)n;
    if (tid < nt) {
        const long long q = base + tid;
        float* xt = buf + tid * ld;
        const float x0 = re[q];
        const float xn = (n % 2 == 0) ? re[(long long)(n / 2) * ntubes + q] : 0.0f;
        for (int t = 0; t < n; ++t) xt[t] = x0 + ((t & 1) ? -xn : xn);
        for (int k = 1; k <= kmax; ++k) {
            const float a = 2.0f * re[(long long)k * ntubes + q];
            const float b = 2.0f * im[(long long)k * ntubes + q];
            int e = 0;
            for (int t = 0; t < n; ++t) {
                const float2 w = tw[e];
                xt[t] += a * w.x + b * w.y;
                e += k;
                if (e >= n) e -= n;
            }
        }
        for (int t = 0; t < n; ++t) xt[t] *= scale;
    }
    __syncthreads();
    store_tile(x + base * n, buf, nt, n, ld);
}

__global__ void k_rdft_any(const float* __restrict__ x, float* __restrict__ re, float* __restrict__ im,
                           long long ntubes, int n)
{
    extern __shared__ float smem[];
    float2* tw = reinterpret_cast<float2*>(smem);
    float* buf = smem + 2 * n;
    const int tpb = blockDim.x;
    fill_twiddles(tw, n);
    for (long long base = (long long)blockIdx.x * tpb; base < ntubes; base += (long long)gridDim.x * tpb) {
        const int nt = (int)min<long long>(tpb, ntubes - base);
        __syncthreads();
        rdft_tile(x, re, im, ntubes, base, nt, n, tw, buf);
    }
}

__global__ void k_irdft_any(const float* __restrict__ re, const float* __restrict__ im, float* __restrict__ x,
                            long long ntubes, int n)
{
    extern __shared__ float smem[];
    float2* tw = reinterpret_cast<float2*>(smem);
    float* buf = smem + 2 * n;
    const int tpb = blockDim.x;
    fill_twiddles(tw, n);
    for (long long base = (long long)blockIdx.x * tpb; base < ntubes; base += (long long)gridDim.x * tpb) {
        const int nt = (int)min<long long>(tpb, ntubes - base);
        __syncthreads();
        irdft_tile(re, im, x, ntubes, base, nt, n, tw, buf);
    }
}

// Batched transforms: one persistent grid walks a list of units (64 tubes
// of one tensor each; tensors of any n3 <= kBatchMaxN3).  The twiddle table
// is refilled when a workgroup moves to a unit of another length.
template <int MAXN>
__global__ __launch_bounds__(kTubes) void k_fft_batch(const FftUnit* __restrict__ units, int nunits, int inverse)
{
    __shared__ float2 tw[MAXN];
    __shared__ float buf[kTubes * (MAXN + 1)];
    int cur = 0;
    for (int u = blockIdx.x; u < nunits; u += gridDim.x) {
        const FftUnit w = units[u];
        __syncthreads();
        if (w.n3 != cur) {
            fill_twiddles(tw, w.n3);
            cur = w.n3;
            __syncthreads();
        }
        if (!inverse) {
            switch (w.n3) {
#define TP_RB(N) \
    case N: rfft_tile<N>(w.src, w.re, w.im, w.ntubes, w.base, w.nt, tw, buf); break;
                TP_RB(4) TP_RB(8) TP_RB(16) TP_RB(32) TP_RB(64)
                case 128:
                    if constexpr (MAXN >= 128) rfft_tile<128>(w.src, w.re, w.im, w.ntubes, w.base, w.nt, tw, buf);
                    break;
#undef TP_RB
                default: rdft_tile(w.src, w.re, w.im, w.ntubes, w.base, w.nt, w.n3, tw, buf); break;
            }
        } else {
            switch (w.n3) {
#define TP_IB(N) \
    case N: irfft_tile<N>(w.re, w.im, w.dst, w.ntubes, w.base, w.nt, tw, buf); break;
                TP_IB(4) TP_IB(8) TP_IB(16) TP_IB(32) TP_IB(64)
                case 128:
                    if constexpr (MAXN >= 128) irfft_tile<128>(w.re, w.im, w.dst, w.ntubes, w.base, w.nt, tw, buf);
                    break;
#undef TP_IB
                default: irdft_tile(w.re, w.im, w.dst, w.ntubes, w.base, w.nt, w.n3, tw, buf); break;
            }
        }
    }
}

// ------------------------------------------------------ order-p tensors --
// Complex DFT along one axis of planar complex data laid out [outer][n][inner]:
// y[o][k][i] = scale * sum_t x[o][t][i] W_n^(+-k t) (direct, twiddles computed
// per workgroup in double precision and rounded once, as k_rdft_any).  One
// output per thread, inner index fastest, so reads of a row are shared by
// neighbouring threads.
__global__ __launch_bounds__(256) void k_cdft_axis(const float* __restrict__ xr, const float* __restrict__ xi,
                                                   float* __restrict__ yr, float* __restrict__ yi, long long outer,
                                                   int n, long long inner, int inverse)
{
    extern __shared__ float2 tws[];
    fill_twiddles(tws, n);
    __syncthreads();
    const float sgn = inverse ? -1.0f : 1.0f, scale = inverse ? 1.0f / (float)n : 1.0f;
    const long long total = outer * n * inner;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const long long i = e % inner, ok = e / inner;
        const int k = (int)(ok % n);
        const long long base = (ok / n) * n * inner + i;
        float sr = 0.0f, si = 0.0f;
        int idx = 0;
        for (int t = 0; t < n; ++t) {
            const float a = xr[base + (long long)t * inner], b = xi[base + (long long)t * inner];
            const float2 w = tws[idx];
            const float wi = sgn * w.y;
            sr += a * w.x - b * wi;
            si += a * wi + b * w.x;
            idx += k;
            if (idx >= n) idx -= n;
        }
        yr[e] = sr * scale;
        yi[e] = si * scale;
    }
}

// Planar complex batched transpose [P][M][R] -> [P][R][M] through 32 x 32
// LDS tiles (coalesced on both sides); tiles walked by a persistent grid.
__global__ __launch_bounds__(256) void k_transpose_planes(const float* __restrict__ xr, const float* __restrict__ xi,
                                                          float* __restrict__ yr, float* __restrict__ yi, long long P,
                                                          long long M, long long R)
{
    __shared__ float tr[32][33], ti[32][33];
    const long long tm = (M + 31) / 32, tn = (R + 31) / 32, ntiles = P * tm * tn;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (long long t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const long long p = t / (tm * tn), rem = t % (tm * tn), m0 = (rem / tn) * 32, r0 = (rem % tn) * 32;
        const float* sr = xr + p * M * R;
        const float* si = xi + p * M * R;
        __syncthreads();
        for (int yy = ty; yy < 32; yy += 8) {
            const long long m = m0 + yy, r = r0 + tx;
            if (m < M && r < R) {
                tr[yy][tx] = sr[m * R + r];
                ti[yy][tx] = si[m * R + r];
            }
        }
        __syncthreads();
        float* dr = yr + p * M * R;
        float* di = yi + p * M * R;
        for (int yy = ty; yy < 32; yy += 8) {
            const long long r = r0 + yy, m = m0 + tx;
            if (m < M && r < R) {
                dr[r * M + m] = tr[tx][yy];
                di[r * M + m] = ti[tx][yy];
            }
        }
    }
}

inline int grid_for(long long ntubes, int tpb)
{
    long long g = (ntubes + tpb - 1) / tpb;
    const long long cap = 256LL * param(TP_PARAM_FFT_GRID);  // persistent: the rest loops
    return (int)(g < cap ? (g > 0 ? g : 1) : cap);
}

int any_tubes_per_block(int n)
{
    int tpb = 64;
    while (tpb > 8 && (size_t)(4 * tpb * (n + 1) + 8 * n) > 64 * 1024) tpb /= 2;
    return tpb;
}

}  // namespace

hipError_t launch_rfft(const float* x, float* re, float* im, long long ntubes, int n3, hipStream_t s)
{
    if (ntubes <= 0) return hipSuccess;
    trace_work(0.0, (double)ntubes * (4.0 * n3 + 8.0 * (n3 / 2 + 1)));
    const int g = grid_for(ntubes, kTubes);
    const bool direct = param(TP_PARAM_FFT_DIRECT) == 1 && (reinterpret_cast<uintptr_t>(x) & 15) == 0;
    switch (n3) {
#define TP_RFFT_CASE(N)                                                       \
    case N:                                                                   \
        if (direct && N >= 8)                                                 \
            k_rfft_pow2_direct<N><<<g, kTubes, 0, s>>>(x, re, im, ntubes);    \
        else                                                                  \
            k_rfft_pow2<N><<<g, kTubes, 0, s>>>(x, re, im, ntubes);           \
        return hipGetLastError();
        TP_RFFT_CASE(4)
        TP_RFFT_CASE(8)
        TP_RFFT_CASE(16)
        TP_RFFT_CASE(32)
        TP_RFFT_CASE(64)
        TP_RFFT_CASE(128)
#undef TP_RFFT_CASE
        default: break;
    }
    const int tpb = any_tubes_per_block(n3);
    const size_t lds = (size_t)(4 * tpb * (n3 + 1) + 8 * n3);
    k_rdft_any<<<grid_for(ntubes, tpb), tpb, lds, s>>>(x, re, im, ntubes, n3);
    return hipGetLastError();
}

hipError_t launch_irfft(const float* re, const float* im, float* x, long long ntubes, int n3, hipStream_t s)
{
    if (ntubes <= 0) return hipSuccess;
    trace_work(0.0, (double)ntubes * (4.0 * n3 + 8.0 * (n3 / 2 + 1)));
    const int g = grid_for(ntubes, kTubes);
    switch (n3) {
#define TP_IRFFT_CASE(N) \
    case N: k_irfft_pow2<N><<<g, kTubes, 0, s>>>(re, im, x, ntubes); return hipGetLastError();
        TP_IRFFT_CASE(4)
        TP_IRFFT_CASE(8)
        TP_IRFFT_CASE(16)
        TP_IRFFT_CASE(32)
        TP_IRFFT_CASE(64)
        TP_IRFFT_CASE(128)
#undef TP_IRFFT_CASE
        default: break;
    }
    const int tpb = any_tubes_per_block(n3);
    const size_t lds = (size_t)(4 * tpb * (n3 + 1) + 8 * n3);
    k_irdft_any<<<grid_for(ntubes, tpb), tpb, lds, s>>>(re, im, x, ntubes, n3);
    return hipGetLastError();
}

hipError_t launch_rfft_split(const float* x, const SplitOut& o, int n3, hipStream_t s)
{
    const long long total = (long long)o.outer * o.ld;
    if (total <= 0) return hipSuccess;
    if (o.inner > o.ld || o.bkl <= 0 || o.ld % o.bkl) return hipErrorInvalidValue;
    const int h = n3 / 2 + 1;
    trace_work(0.0, (double)o.outer * o.inner * 4.0 * n3 + (double)total * (o.split ? 8.0 : 4.0) * h);
    const bool vec = (reinterpret_cast<uintptr_t>(x) & 15) == 0;
    if (vec) {
        const int g = grid_for(total, kTubes);
        switch (n3) {
#define TP_RSPLIT_CASE(N) \
    case N: k_rfft_split<N><<<g, kTubes, 0, s>>>(x, o); return hipGetLastError();
            TP_RSPLIT_CASE(4)
            TP_RSPLIT_CASE(8)
            TP_RSPLIT_CASE(16)
            TP_RSPLIT_CASE(32)
            TP_RSPLIT_CASE(64)
            TP_RSPLIT_CASE(128)
#undef TP_RSPLIT_CASE
            default: break;
        }
    }
    const int tpb = any_tubes_per_block(n3);
    const size_t lds = (size_t)(4 * tpb * (n3 + 1) + 8 * n3);
    k_rdft_split_any<<<grid_for(total, tpb), tpb, lds, s>>>(x, o, n3);
    return hipGetLastError();
}

namespace {
hipError_t launch_cdft(Planes x, Planes y, long long outer, int n, long long inner, int inverse, hipStream_t s)
{
    const long long total = outer * n * inner;
    if (total <= 0) return hipSuccess;
    trace_work(8.0 * total * n, 16.0 * total);
    const long long g = (total + 255) / 256, cap = 256LL * 64;
    k_cdft_axis<<<(unsigned)(g < cap ? g : cap), 256, (size_t)n * sizeof(float2), s>>>(x.re, x.im, y.re, y.im,
                                                                                      outer, n, inner, inverse);
    return hipGetLastError();
}

hipError_t launch_transpose(Planes x, Planes y, long long P, long long M, long long R, hipStream_t s)
{
    const long long tiles = P * ((M + 31) / 32) * ((R + 31) / 32);
    if (tiles <= 0) return hipSuccess;
    trace_work(0.0, 16.0 * P * M * R);
    const long long cap = 256LL * 32;
    k_transpose_planes<<<(unsigned)(tiles < cap ? tiles : cap), 256, 0, s>>>(x.re, x.im, y.re, y.im, P, M, R);
    return hipGetLastError();
}

long long prod_dims(const int* dims, int from, int to)
{
    long long p = 1;
    for (int a = from; a < to; ++a) p *= dims[a];
    return p;
}
}  // namespace

hipError_t launch_rfft_nd(const float* x, long long mrow, int nd, const int* dims, Planes dst, Planes tmp,
                          hipStream_t s)
{
    const int N = dims[nd - 1], hp = N / 2 + 1;
    const long long r = prod_dims(dims, 0, nd - 1);
    if (nd == 1) return launch_rfft(x, dst.re, dst.im, mrow, N, s);
    // nd passes follow the real transform (nd - 1 complex DFTs, one transpose)
    Planes cur = (nd % 2 == 0) ? dst : tmp, oth = (nd % 2 == 0) ? tmp : dst;
    hipError_t e = launch_rfft(x, cur.re, cur.im, mrow * r, N, s);  // [kp][e][rest]
    if (e != hipSuccess) return e;
    for (int a = 0; a < nd - 1; ++a) {
        const long long outer = (long long)hp * mrow * prod_dims(dims, 0, a), inner = prod_dims(dims, a + 1, nd - 1);
        if ((e = launch_cdft(cur, oth, outer, dims[a], inner, 0, s)) != hipSuccess) return e;
        const Planes t = cur;
        cur = oth;
        oth = t;
    }
    return launch_transpose(cur, oth, hp, mrow, r, s);  // [kp][rest][e] in dst
}

hipError_t launch_irfft_nd(Planes src, Planes tmp, float* x, long long mrow, int nd, const int* dims, hipStream_t s)
{
    const int N = dims[nd - 1], hp = N / 2 + 1;
    const long long r = prod_dims(dims, 0, nd - 1);
    if (nd == 1) return launch_irfft(src.re, src.im, x, mrow, N, s);
    hipError_t e = launch_transpose(src, tmp, hp, r, mrow, s);  // [kp][e][rest]
    if (e != hipSuccess) return e;
    Planes cur = tmp, oth = src;
    for (int a = nd - 2; a >= 0; --a) {
        const long long outer = (long long)hp * mrow * prod_dims(dims, 0, a), inner = prod_dims(dims, a + 1, nd - 1);
        if ((e = launch_cdft(cur, oth, outer, dims[a], inner, 1, s)) != hipSuccess) return e;
        const Planes t = cur;
        cur = oth;
        oth = t;
    }
    return launch_irfft(cur.re, cur.im, x, mrow * r, N, s);
}

size_t max_fft_length() { return 1024; }

hipError_t launch_fft_batch(const FftUnit* units, int nunits, int inverse, int max_n3, int grid, hipStream_t s)
{
    if (nunits <= 0) return hipSuccess;
    if (max_n3 > kBatchMaxN3) return hipErrorInvalidValue;
    const int g = grid < nunits ? grid : nunits;
    if (max_n3 <= 64)
        k_fft_batch<64><<<g, kTubes, 0, s>>>(units, nunits, inverse);
    else
        k_fft_batch<128><<<g, kTubes, 0, s>>>(units, nunits, inverse);
    return hipGetLastError();
}

}  // namespace tp
