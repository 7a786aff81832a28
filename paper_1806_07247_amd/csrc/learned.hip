// Learned-rank prox_tnn: per-slice features, a small MLP that predicts the
// number of singular values above tau, a randomized range finder sized by
// that prediction (Halko, Martinsson, Tropp 2011) with FP64 CholeskyQR2
// re-orthonormalisation, the check sigma_(k+1) < tau, and the MLP's training
// kernels.  The exact operation it approximates is Theorem 2.3.
//
// Sizes: L is the padded sketch width (l_max, <= kMaxL); each slice uses its
// own l = lact[s] <= L leading columns, the others are kept at zero.
#include <cmath>

#include "tp_internal.h"

namespace tp {
namespace {

// ------------------------------------------------------------------ Philox --
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).
__device__ __forceinline__ void philox4x32_10(unsigned int c[4], unsigned int k0, unsigned int k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const unsigned long long p0 = (unsigned long long)0xD2511F53u * c[0];
        const unsigned long long p1 = (unsigned long long)0xCD9E8D57u * c[2];
        const unsigned int n0 = (unsigned int)(p1 >> 32) ^ c[1] ^ k0;
        const unsigned int n2 = (unsigned int)(p0 >> 32) ^ c[3] ^ k1;
        c[1] = (unsigned int)p1;
        c[3] = (unsigned int)p0;
        c[0] = n0;
        c[2] = n2;
    }
}

__device__ __forceinline__ bool is_real_slice(int s, int n3) { return s == 0 || (n3 % 2 == 0 && s == n3 / 2); }

// Om (n x L per slice, planar row-major): entry (i, j) from Philox on counter
// {i, j, slice, 0}, key {seed lo, seed hi}; Box-Muller in FP64 on
// u = (x + 0.5) 2^-32; complex slices (z0 + i z1)/sqrt(2), real slices z0;
// zero for j >= lact[slice].
__global__ __launch_bounds__(256) void k_sketch(float* __restrict__ omr, float* __restrict__ omi, int n, int L,
                                                const int* __restrict__ lact, int nslices, int n3,
                                                unsigned long long seed, WarmBasis warm, const int* __restrict__ gate)
{
    if (gate && *gate == 0) return;
    const long long total = (long long)nslices * n * L;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const int s = (int)(e / ((long long)n * L));
        const int rem = (int)(e % ((long long)n * L));
        const int i = rem / L, j = rem % L;
        float vr = 0.0f, vi = 0.0f;
        if (j < lact[s] && warm.re && j < min(warm.cols[s], warm.ld)) {  // column j of the previous basis
            const long long o = ((long long)s * n + i) * warm.ld + j;
            vr = warm.re[o];
            vi = warm.im[o];
        } else if (j < lact[s]) {
            unsigned int c[4] = {(unsigned int)i, (unsigned int)j, (unsigned int)s, 0u};
            philox4x32_10(c, (unsigned int)seed, (unsigned int)(seed >> 32));
            const double u0 = ((double)c[0] + 0.5) * 0x1p-32, u1 = ((double)c[1] + 0.5) * 0x1p-32;
            const double rad = sqrt(-2.0 * log(u0));
            double sn, cs;
            sincospi(2.0 * u1, &sn, &cs);
            if (is_real_slice(s, n3)) {
                vr = (float)(rad * cs);
            } else {
                vr = (float)(rad * cs * 0.70710678118654752440);
                vi = (float)(rad * sn * 0.70710678118654752440);
            }
        }
        omr[e] = vr;
        omi[e] = vi;
    }
}

// ------------------------------------------------------------ CholeskyQR --
constexpr int kMaxGramSplit = 16;  // row bands of the Gram (partials summed by k_chol)

// Partial Gram G_w = Y_w^* Y_w (FP64) of the rows handled by workgroup w of
// nsplit, for the lact leading columns; Y is m x L planar row-major.  Only the
// upper triangle is formed (the Cholesky reads nothing else): thread t owns
// the B x B block (ta, tb), ta <= tb, the t-th block of the upper triangle
// of the nb x nb block grid (nb = ceil(L / B), nb (nb + 1) / 2 <= 256).
// Rows are staged in LDS in chunks; every product of two FP32 values is exact
// in FP64 and the sums are FP64.
constexpr int kGramChunk = 32;                        // rows per LDS chunk
constexpr int kGramLoads = kGramChunk * kMaxL / 256;  // chunk elements per thread (at most)
constexpr int kMaxParts = 4;                          // split parts summed by k_reduce_gram

// the B x B block (ta, tb) of the Gram that thread tid of the workgroup owns
struct GramBlock {
    int a0, b0;
    bool has, work;  // has: a block of the grid; work: inside the active columns
};
template <int B>
__device__ __forceinline__ GramBlock gram_block(int tid, int L, int la)
{
    const int nb = (L + B - 1) / B;
    // row ta holds nb - ta blocks (tb = ta .. nb-1)
    int ta = 0, t = tid;
    while (ta < nb && t >= nb - ta) {
        t -= nb - ta;
        ++ta;
    }
    GramBlock gb;
    gb.a0 = ta * B;
    gb.b0 = (ta + t) * B;
    gb.has = ta < nb;
    gb.work = gb.has && gb.a0 < la && gb.b0 < la;
    return gb;
}

// accumulate conj(x_a) y_b over the nr staged rows of tile (row stride W)
template <int B, int W>
__device__ __forceinline__ void gram_rows(const float2* tile, int nr, int a0, int b0, double (&gr)[B][B],
                                          double (&gi)[B][B])
{
    for (int i = 0; i < nr; ++i) {
        double xr[B], xi[B], vr[B], vi[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const float2 x = tile[i * W + a0 + u], y = tile[i * W + b0 + u];
            xr[u] = x.x;
            xi[u] = x.y;
            vr[u] = y.x;
            vi[u] = y.y;
        }
#pragma unroll
        for (int u = 0; u < B; ++u)
#pragma unroll
            for (int v = 0; v < B; ++v) {  // conj(x_a) y_b
                gr[u][v] = fma(xr[u], vr[v], fma(xi[u], vi[v], gr[u][v]));
                gi[u][v] = fma(xr[u], vi[v], fma(-xi[u], vr[v], gi[u][v]));
            }
    }
}

// the thread's block of partial Gram w of slice s
template <int B>
__device__ __forceinline__ void gram_store(const GramBlock& gb, int L, int s, int w, int nsplit, double2* part,
                                           const double (&gr)[B][B], const double (&gi)[B][B])
{
    if (!gb.has) return;
    double2* out = part + ((long long)s * nsplit + w) * L * L;
#pragma unroll
    for (int u = 0; u < B; ++u)
#pragma unroll
        for (int v = 0; v < B; ++v) {
            const int a = gb.a0 + u, b = gb.b0 + v;
            if (a < L && b < L) out[a * L + b] = gb.work ? make_double2(gr[u][v], gi[u][v]) : make_double2(0.0, 0.0);
        }
}

// block edge of the Gram blocks for la live columns: the upper triangle of
// ceil(la / B) blocks fits the 256 threads
__device__ __forceinline__ int gram_edge(int la) { return la <= 22 ? 1 : (la <= 44 ? 2 : 3); }
constexpr int kGramW = kMaxL + 3;  // staged row stride (room for the widest edge's last block)

template <int B>
__device__ __forceinline__ void gram_body(const float* __restrict__ yr, const float* __restrict__ yi, int m, int L,
                                          int la, double2* __restrict__ part, int nsplit, float2* tile)
{
    constexpr int W = kGramW;
    const int s = blockIdx.y, w = blockIdx.x, tid = threadIdx.x;
    const int lc = min(la, L);
    const GramBlock gb = gram_block<B>(tid, lc, lc);  // blocks of the live columns only
    const int r0 = (int)((long long)m * w / nsplit), r1 = (int)((long long)m * (w + 1) / nsplit);
    const float* Yr = yr + (long long)s * m * L;
    const float* Yi = yi + (long long)s * m * L;
    double gr[B][B], gi[B][B];
#pragma unroll
    for (int u = 0; u < B; ++u)
#pragma unroll
        for (int v = 0; v < B; ++v) gr[u][v] = gi[u][v] = 0.0;
    const int lw = min(L, (lc + B - 1) / B * B);  // staged columns: the live ones, zero to the block edge
    for (int c0 = r0; c0 < r1; c0 += kGramChunk) {
        // every load of the thread is issued before any is used
        const int nr = min(kGramChunk, r1 - c0), nf = nr * lw;
        float xr[kGramLoads], xi[kGramLoads];
#pragma unroll
        for (int q = 0; q < kGramLoads; ++q) {
            const int f = tid + 256 * q;
            const int i = f / lw, j = f % lw;
            const bool ok = f < nf && j < lc;
            const long long o = (long long)(c0 + i) * L + j;
            xr[q] = ok ? Yr[o] : 0.0f;
            xi[q] = ok ? Yi[o] : 0.0f;
        }
        __syncthreads();  // the previous chunk is read
#pragma unroll
        for (int q = 0; q < kGramLoads; ++q) {
            const int f = tid + 256 * q;
            if (f < nf) tile[(f / lw) * W + f % lw] = make_float2(xr[q], xi[q]);
        }
        __syncthreads();
        if (gb.work) gram_rows<B, W>(tile, nr, gb.a0, gb.b0, gr, gi);
    }
    gram_store<B>(gb, L, s, w, nsplit, part, gr, gi);
}

// Partial Gram of the live columns (lact) of every slice; only their block
// of the L x L layout is written.
__global__ __launch_bounds__(256) void k_gram(const float* __restrict__ yr, const float* __restrict__ yi, int m,
                                              int L, const int* __restrict__ lact, double2* __restrict__ part,
                                              int nsplit, const int* __restrict__ gate)
{
    if (gate && *gate == 0) return;
    __shared__ float2 tile[kGramChunk * kGramW];
    const int la = lact[blockIdx.y];
    switch (gram_edge(la)) {
        case 1: gram_body<1>(yr, yi, m, L, la, part, nsplit, tile); break;
        case 2: gram_body<2>(yr, yi, m, L, la, part, nsplit, tile); break;
        default: gram_body<3>(yr, yi, m, L, la, part, nsplit, tile); break;
    }
}

// The split parts of a narrow slice product summed into Y (the fixed order
// kp = 0, 1, ... of the plain reduction) and, from the same staged rows,
// the partial Grams of k_gram: one pass over Y instead of a write and a
// read back.
template <int B>
__device__ __forceinline__ void reduce_gram_body(const float* __restrict__ parts, int ksplit, int m, int L, int ny,
                                                 int nslices, int real_first, int real_last, float* __restrict__ yr,
                                                 float* __restrict__ yi, int la, double2* __restrict__ part,
                                                 int nsplit, float2* tile)
{
    constexpr int W = kGramW;
    const int s = blockIdx.y, w = blockIdx.x, tid = threadIdx.x;
    const int lc = min(la, L);
    const GramBlock gb = gram_block<B>(tid, lc, lc);
    const int r0 = (int)((long long)m * w / nsplit), r1 = (int)((long long)m * (w + 1) / nsplit);
    const long long mn = (long long)m * L, total = (long long)nslices * mn, plane = (long long)ksplit * total;
    const bool real = (real_first && s == 0) || (real_last && s == nslices - 1);
    const float* P = parts + s * mn;
    float* Yr = yr + s * mn;
    float* Yi = yi + s * mn;
    double gr[B][B], gi[B][B];
#pragma unroll
    for (int u = 0; u < B; ++u)
#pragma unroll
        for (int v = 0; v < B; ++v) gr[u][v] = gi[u][v] = 0.0;
    for (int c0 = r0; c0 < r1; c0 += kGramChunk) {
        // all loads of the thread in flight at once: unconditional loads of
        // in-range addresses (an element past the chunk reads the chunk's
        // first, a part past ksplit the last part), the unused values
        // dropped where they are summed (a load under a condition would make
        // the merge wait for it before the next one is issued)
        const int nr = min(kGramChunk, r1 - c0), nf = nr * ny;
        float pr[kGramLoads][kMaxParts], pim[kGramLoads][kMaxParts];
#pragma unroll
        for (int q = 0; q < kGramLoads; ++q) {
            const int f = tid + 256 * q;
            const long long o = f < nf ? (long long)(c0 + f / ny) * L + f % ny : (long long)c0 * L;
#pragma unroll
            for (int kp = 0; kp < kMaxParts; ++kp) {
                const long long kc = min(kp, ksplit - 1);
                pr[q][kp] = P[kc * total + o];
                pim[q][kp] = P[plane + kc * total + o];
            }
        }
        __syncthreads();  // the previous chunk is read
#pragma unroll
        for (int q = 0; q < kGramLoads; ++q) {
            const int f = tid + 256 * q;
            if (f < nf) {
                float sr = 0.0f, si = 0.0f;  // the parts in order, as the plain reduction
#pragma unroll
                for (int kp = 0; kp < kMaxParts; ++kp)
                    if (kp < ksplit) {
                        sr += pr[q][kp];
                        si += pim[q][kp];
                    }
                if (real) si = 0.0f;
                const int i = f / ny, j = f % ny;
                const long long o = (long long)(c0 + i) * L + j;
                Yr[o] = sr;
                Yi[o] = si;
                if (j < W) tile[i * W + j] = j < lc ? make_float2(sr, si) : make_float2(0.f, 0.f);
            }
        }
        __syncthreads();
        if (gb.work) gram_rows<B, W>(tile, nr, gb.a0, gb.b0, gr, gi);
    }
    gram_store<B>(gb, L, s, w, nsplit, part, gr, gi);
}

// The split parts of a narrow product summed into Y (columns below the
// device width `width`, or all L) and the partial Grams of its live columns.
__global__ __launch_bounds__(256) void k_reduce_gram(const float* __restrict__ parts, int ksplit, int m, int L,
                                                     int nslices, int real_first, int real_last,
                                                     float* __restrict__ yr, float* __restrict__ yi,
                                                     const int* __restrict__ lact, double2* __restrict__ part,
                                                     int nsplit, const int* __restrict__ gate,
                                                     const int* __restrict__ width)
{
    if (gate && *gate == 0) return;
    __shared__ float2 tile[kGramChunk * kGramW];
    const int la = lact[blockIdx.y];
    const int ny = width ? max(min(*width, L), min(la, L)) : L;  // columns of Y written
    switch (gram_edge(la)) {
        case 1:
            reduce_gram_body<1>(parts, ksplit, m, L, ny, nslices, real_first, real_last, yr, yi, la, part, nsplit,
                                tile);
            break;
        case 2:
            reduce_gram_body<2>(parts, ksplit, m, L, ny, nslices, real_first, real_last, yr, yi, la, part, nsplit,
                                tile);
            break;
        default:
            reduce_gram_body<3>(parts, ksplit, m, L, ny, nslices, real_first, real_last, yr, yi, la, part, nsplit,
                                tile);
            break;
    }
}

// Per slice: G = sum of the partial Grams (fixed order, upper triangle); in
// pass 0 a diagonal shift 1e-13 trace(G)/lact; then one elimination sweep on
// the augmented pair [G | I] (FP64): step j scales row j by 1/sqrt(pivot) and
// subtracts conj(R_ja) times it from every later row a.  On the G side this
// is the right-looking Cholesky G = R^* R; the same row operations turn I
// into M = R^{-*} (they are the E with E G = R), so Rinv = M^* is formed in
// the same L steps.  The entries stay in registers (the upper triangle of G
// and the strict lower triangle of M share one slot per (a, b)).  The sweep
// is blocked by panels of kPanel rows, one panel per wavefront: the owner
// takes its panel's steps alone (the pivot row is broadcast across the
// wavefront with readlane, no barrier), publishes the normalized panel rows
// to LDS, and after one barrier every later wavefront applies those steps to
// its rows in step order (the same operations, in the same order, as the
// unblocked sweep).  Rinv is written as FP32 planar (identity on the
// inactive columns); optionally Rtot <- R Rtot (FP64) and R2^* (FP32 planar,
// zero outside the active block).
constexpr int kCholThreads = 1024;
constexpr int kCholEntries = kMaxL * kMaxL / kCholThreads;  // entries per thread (rows per wavefront)
constexpr int kPanel = kCholEntries;                          // rows of one panel = rows of one wavefront
static_assert(kMaxL == 64 && kCholThreads / 64 * kCholEntries == kMaxL, "one lane per column, 16 waves x 4 rows");

// sqrt(p) and 1/sqrt(p), p > 0 normal: the hardware reciprocal square root
// refined by two Newton steps, then one Newton step on sqrt(p) = p / sqrt(p)
__device__ __forceinline__ void sqrt_and_rsqrt(double p, double& r, double& inv)
{
    double y = __builtin_amdgcn_rsq(p);
    double h = p * y;
    y = fma(0.5 * y, fma(-h, y, 1.0), y);
    h = p * y;
    y = fma(0.5 * y, fma(-h, y, 1.0), y);
    const double q = p * y;
    r = fma(0.5 * y, fma(-q, q, p), q);
    inv = y;
}

// value of v in lane l (l wavefront-uniform; every lane computed v)
__device__ __forceinline__ double read_lane(double v, int l)
{
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__global__ __launch_bounds__(kCholThreads) void k_chol(const double2* __restrict__ part, int nsplit, int L,
                                                       const int* __restrict__ lact, int pass, float* __restrict__ rir,
                                                       float* __restrict__ rii, double2* __restrict__ rtot,
                                                       float* __restrict__ rhr, float* __restrict__ rhi,
                                                       int* __restrict__ status, const int* __restrict__ gate)
{
    if (gate && *gate == 0) return;
    extern __shared__ double2 sh[];
    double2* R = sh;            // L x L (R, for the Rtot product)
    double2* X = sh + L * L;    // L x L (Rtot)
    __shared__ double2 pan[2][kPanel][kMaxL];  // the published normalized panel rows, two buffers
    const int s = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
    const int la = lact[s];
    const double2* P = part + (long long)s * nsplit * L * L;

    // One value per entry (a, b), held by lane b of wavefront w for the rows
    // a = kPanel w + u: the G side for b >= a, the M side for b < a (the two
    // share a slot: M_ab is zero until column b is eliminated, and the slot is
    // reset at that step); the slot of (a, a) holds R_aa once row a is
    // eliminated (M_aa = 1 / R_aa).  Plain doubles, so that the values stay
    // in registers.
    // G = the sum of the partials in the fixed order w = 0, 1, ... (upper
    // triangle; one entry per thread with all of its partials in flight),
    // staged in R
    // (only the la x la live block: the rest of the layout stays unread)
    const int nup = la * (la + 1) / 2;
    for (int e = tid; e < nup; e += nt) {
        int a = 0, r = e;
        while (r >= la - a) {
            r -= la - a;
            ++a;
        }
        const int o = a * L + a + r;
        double pr[kMaxGramSplit], pi[kMaxGramSplit];
#pragma unroll
        for (int w = 0; w < kMaxGramSplit; ++w) {
            const double2 v = w < nsplit ? P[(long long)w * L * L + o] : make_double2(0.0, 0.0);
            pr[w] = v.x;
            pi[w] = v.y;
        }
        double gr = 0.0, gi = 0.0;
#pragma unroll
        for (int w = 0; w < kMaxGramSplit; ++w) {
            if (w < nsplit) {
                gr += pr[w];
                gi += pi[w];
            }
        }
        R[o] = make_double2(gr, gi);
    }
    __syncthreads();
    const int lane = tid & 63, wave = tid >> 6;
    int ea[kCholEntries];
    double vr[kCholEntries], vi[kCholEntries];
    const int b = lane;
    // diagonal shift (pass 0): every thread sums the same values in the same order
    double sd = 0.0;
    if (pass == 0 && la > 0) {
        double tr = 0.0;
        for (int k = 0; k < la; ++k) tr += R[k * L + k].x;
        sd = 1e-13 * tr / la;
    }
#pragma unroll
    for (int u = 0; u < kCholEntries; ++u) {
        const int a0 = kPanel * wave + u;
        ea[u] = (a0 < L && b < L) ? a0 : L;  // L: no entry
        vr[u] = vi[u] = 0.0;
        if (ea[u] < la && b < la && b >= ea[u]) {
            const double2 g = R[ea[u] * L + b];
            vr[u] = g.x + (ea[u] == b && b < la ? sd : 0.0);
            vi[u] = g.y;
        }
    }

    bool broke = false;
    // steps j = kPanel p .. of panel p by its owner (all 64 lanes take part,
    // so that readlane sees computed values); writes pan[buf]
    auto factor = [&](int p, int buf) {
#pragma unroll
        for (int t = 0; t < kPanel; ++t) {
            const int j = kPanel * p + t;
            if (j >= L) break;
            const bool act = j < la;
            // pivot of step j (inactive rows: pivot 1)
            double pv = act ? read_lane(vr[t], j) : 1.0;
            if (!(pv > 0.0)) {
                pv = 1e-300;
                broke = true;
            }
            double rjj, inv;
            sqrt_and_rsqrt(pv, rjj, inv);
            // y_b: R_jb (b > j; zero outside the active block), M'_jb (b < j), M'_jj = 1 / R_jj
            double yr = inv, yi = 0.0;
            if (b != j) {
                const bool keep = b < j || (act && b < la);
                yr = keep ? vr[t] * inv : 0.0;
                yi = keep ? vi[t] * inv : 0.0;
            }
            vr[t] = b == j ? rjj : yr;
            vi[t] = b == j ? 0.0 : yi;
            pan[buf][t][b] = make_double2(yr, yi);
#pragma unroll
            for (int u = t + 1; u < kPanel; ++u) {
                const int a = kPanel * p + u;
                if (a >= L) break;
                const double xr = read_lane(yr, a), xi = read_lane(yi, a);  // R_ja (zero unless active)
                // v_ab -= conj(R_ja) y_b; column j enters the M side from zero
                const double br = b == j ? 0.0 : vr[u], bi = b == j ? 0.0 : vi[u];
                vr[u] = br - (xr * yr + xi * yi);
                vi[u] = bi - (xr * yi - xi * yr);
            }
        }
    };
    // the steps of panel p (published in pan[buf]) on this wavefront's rows
    auto apply = [&](int p, int buf) {
#pragma unroll
        for (int t = 0; t < kPanel; ++t) {
            const int j = kPanel * p + t;
            if (j >= L) break;
            const double2 y = pan[buf][t][b];
#pragma unroll
            for (int u = 0; u < kPanel; ++u) {
                const int a = kPanel * wave + u;
                if (a >= L) break;
                const double2 x = pan[buf][t][a];  // R_ja
                const double br = b == j ? 0.0 : vr[u], bi = b == j ? 0.0 : vi[u];
                vr[u] = br - (x.x * y.x + x.y * y.y);
                vi[u] = bi - (x.x * y.y - x.y * y.x);
            }
        }
    };
    // panels past the live block are not swept: their rows end as the identity
    const int npan = (la + kPanel - 1) / kPanel;
    if (wave == 0 && npan > 0) factor(0, 0);
    __syncthreads();
    for (int p = 0; p + 1 < npan; ++p) {
        if (wave > p && wave < npan) {
            apply(p, p & 1);
            if (wave == p + 1) factor(p + 1, (p + 1) & 1);
        }
        __syncthreads();
    }
    if (broke && status) status[s] = 1;  // by the owners of the failed pivots
    // Rinv = M^*: entry (a, b), b <= a, of M gives Rinv(b, a); Rinv(b, a) = 0 for b > a
#pragma unroll
    for (int u = 0; u < kCholEntries; ++u) {
        const int a = ea[u];
        if (a < L) {
            const long long o = (long long)s * L * L + b * L + a;
            double mr = vr[u], mi = vi[u];
            if (a >= la) {  // outside the live block: the identity
                mr = b == a ? 1.0 : 0.0;
                mi = 0.0;
                vr[u] = b == a ? 1.0 : 0.0;
                vi[u] = 0.0;
            } else if (b == a) {  // M_aa = 1 / R_aa (R_aa real)
                mr = 1.0 / vr[u];
                mi = 0.0;
            }
            rir[o] = b <= a ? (float)mr : 0.0f;
            rii[o] = b <= a ? (float)(-mi) : 0.0f;
            R[a * L + b] = b >= a ? make_double2(vr[u], vi[u]) : make_double2(0.0, 0.0);
        }
    }
    if (rtot) {
        double2* T = rtot + (long long)s * L * L;
        __syncthreads();  // R complete
        if (pass == 0) {
            for (int e = tid; e < L * L; e += nt) X[e] = R[e];
        } else {
            for (int e = tid; e < L * L; e += nt) X[e] = T[e];
            __syncthreads();
            // R Rtot of two upper triangular factors
            double cr[kCholEntries], ci[kCholEntries];
#pragma unroll
            for (int u = 0; u < kCholEntries; ++u) {
                const int a = ea[u];
                cr[u] = ci[u] = 0.0;
                if (a < L)
                    for (int k = a; k <= b; ++k) {
                        const double2 x = R[a * L + k], y = X[k * L + b];
                        cr[u] += x.x * y.x - x.y * y.y;
                        ci[u] += x.x * y.y + x.y * y.x;
                    }
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < kCholEntries; ++u)
                if (ea[u] < L) X[ea[u] * L + b] = make_double2(cr[u], ci[u]);
        }
        __syncthreads();
        for (int e = tid; e < L * L; e += nt) T[e] = X[e];
        if (rhr && pass == 1) {  // R2^* restricted to the active block
            for (int e = tid; e < L * L; e += nt) {
                const int a = e / L, b = e % L;
                const bool in = a < la && b < la;
                const double2 v = X[b * L + a];
                rhr[(long long)s * L * L + e] = in ? (float)v.x : 0.0f;
                rhi[(long long)s * L * L + e] = in ? (float)(-v.y) : 0.0f;
            }
        }
    }
}

// ------------------------------------------------------ check and core T --
// sigma_j, C_r (cols, column-major L x L), V_r (column-major L x L) from the
// Jacobi SVD of R2^*.  fallback[s] = 1 when #{sigma_j >= tau} > kpred[s]
// (the check sigma_(k+1) < tau fails) or when the slice was already sent to
// the full SVD; T = C_r diag((sigma - tau)_+ / sigma) V_r^* (planar, L x L).
// With vp / cp given, V_r and C_r are also written planar row-major (L x L,
// the operands of the a posteriori check's products).
__global__ __launch_bounds__(256) void k_rsvd_check(const float2* __restrict__ cols, const double* __restrict__ sigma,
                                                    const float2* __restrict__ vr, const int* __restrict__ kpred,
                                                    const int* __restrict__ lact, const int* __restrict__ prefb,
                                                    const int* __restrict__ status, int L, double tau,
                                                    float* __restrict__ tr, float* __restrict__ ti,
                                                    int* __restrict__ fallback, int* __restrict__ rank, const int* __restrict__ gate,
                                                    float* __restrict__ vpr, float* __restrict__ vpi,
                                                    float* __restrict__ cpr, float* __restrict__ cpi)
{
    if (gate && *gate == 0) return;
    __shared__ double scale[64];
    __shared__ int above;
    const int s = blockIdx.x, tid = threadIdx.x;
    const double* sg = sigma + (long long)s * L;
    if (tid < kMaxL) {  // wavefront 0: one singular value per lane (L <= kMaxL = 64)
        const int la_ = lact[s];
        const bool live = tid < la_ && tid < L;
        const double sj = live ? sg[tid] : 0.0;
        // counted NaN-safe: a NaN singular value counts as not below tau, so
        // a broken basis fails the check instead of passing it
        const int ge = __popcll(__ballot(live && !(sj < tau)));
        const int gt = __popcll(__ballot(live && sj > tau));
        scale[tid] = (live && sj > tau) ? (sj - tau) / sj : 0.0;
        if (tid == 0) {
            above = gt;
            // a CholeskyQR breakdown on any basis of this slice (status) also sends it to the full SVD
            const int fb = (prefb[s] || (status && status[s]) || (ge > kpred[s] && la_ > 0)) ? 1 : 0;
            fallback[s] = fb;
            if (fb == 0 && rank) rank[s] = gt;
        }
    }
    __syncthreads();
    (void)above;
    // C and V of the slice staged in LDS (column-major, L x L each); T is
    // formed on the live la x la block and zero elsewhere
    const int la = min(lact[s], L);
    __shared__ float2 sC[kMaxL * kMaxL], sV[kMaxL * kMaxL];
    // (every load of a thread issued before any is stored: unconditional
    // loads of in-range elements, the extra ones not stored)
    constexpr int kPer = kMaxL * kMaxL / 256;  // elements per thread (blockDim 256)
    {
        float2 c[kPer], v[kPer];
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int e = tid + 256 * u;
            const long long o = (long long)s * L * L + (e < L * la ? e : 0);
            c[u] = cols[o];
            v[u] = vr[o];
        }
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int e = tid + 256 * u;
            if (e < L * la) {
                sC[e] = c[u];
                sV[e] = v[u];
            }
        }
    }
    __syncthreads();
    for (int e = tid; e < L * L; e += blockDim.x) {
        const int a = e / L, b = e % L;
        double vr_ = 0.0, vi_ = 0.0;
        const int nj = (a < la && b < la) ? la : 0;  // zero outside the live block
        for (int j = 0; j < nj; ++j) {
            if (scale[j] == 0.0) continue;
            const float2 c = sC[j * L + a], v = sV[j * L + b];  // C(a,j) conj(V(b,j))
            vr_ += scale[j] * ((double)c.x * v.x + (double)c.y * v.y);
            vi_ += scale[j] * ((double)c.y * v.x - (double)c.x * v.y);
        }
        tr[(long long)s * L * L + e] = (float)vr_;
        ti[(long long)s * L * L + e] = (float)vi_;
    }
    if (vpr) {  // column-major to planar row-major, as k_cm_to_planar (loads first, as above)
        float2 c[kPer], v[kPer];
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int e = tid + 256 * u, ec = e < L * L ? e : 0;
            const long long o = (long long)s * L * L + (long long)(ec % L) * L + ec / L;
            v[u] = vr[o];
            c[u] = cols[o];
        }
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int e = tid + 256 * u;
            if (e < L * L) {
                const long long d = (long long)s * L * L + e;
                vpr[d] = v[u].x;
                vpi[d] = v[u].y;
                cpr[d] = c[u].x;
                cpi[d] = c[u].y;
            }
        }
    }
}

// ---------------------------------------------------- a posteriori check --
// column-major L x L (float2) to planar row-major L x L, per slice
// (and a second pair src2 -> re2, im2 in the same launch when src2 is given)
__global__ __launch_bounds__(256) void k_cm_to_planar(const float2* __restrict__ src, float* __restrict__ re,
                                                      float* __restrict__ im, int L, int nslices, const int* __restrict__ gate,
                                                      const float2* __restrict__ src2, float* __restrict__ re2,
                                                      float* __restrict__ im2)
{
    if (gate && *gate == 0) return;
    const long long total = (long long)nslices * L * L;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const long long s = e / ((long long)L * L);
        const int r = (int)(e % ((long long)L * L));
        const int i = r / L, j = r % L;
        const long long o = s * L * L + (long long)j * L + i;
        const float2 v = src[o];
        re[e] = v.x;
        im[e] = v.y;
        if (src2) {
            const float2 w = src2[o];
            re2[e] = w.x;
            im2[e] = w.y;
        }
    }
}

// Per slice: the kept Ritz triplets (sigma_j > tau) have right residuals
// r_j = Ybar v_j - sigma_j u_j = T1 e_j - T2 e_j (T1 = Ybar Q2 V_r,
// T2 = Q U_r S); the slice is inaccurate when
//   sum_J ||r_j||^2 > delta^2 sum_J (sigma_j - tau)^2,
// i.e. the residuals are not small against the thresholded part it keeps.
constexpr int kAccSplit = 16;  // row bands of the residual sums (partials summed in order)

// Partial residual sums over the rows of band w of kAccSplit:
// sum over kept columns j (sigma_j > tau, j < lact) of |t1 - t2|^2, FP64
__global__ __launch_bounds__(256) void k_accuracy_part(const float* __restrict__ t1r, const float* __restrict__ t1i,
                                                       const float* __restrict__ t2r, const float* __restrict__ t2i,
                                                       const double* __restrict__ sigma,
                                                       const int* __restrict__ lact, int m, int L, double tau,
                                                       double* __restrict__ part, const int* __restrict__ gate)
{
    if (gate && *gate == 0) return;
    __shared__ double red[256];
    __shared__ unsigned char keep[kMaxL];
    const int w = blockIdx.x, s = blockIdx.y, tid = threadIdx.x;
    const double* sg = sigma + (long long)s * L;
    if (tid < L) keep[tid] = (tid < lact[s] && sg[tid] > tau) ? 1 : 0;
    __syncthreads();
    const long long r0 = (long long)m * w / kAccSplit, r1 = (long long)m * (w + 1) / kAccSplit;
    const long long off = (long long)s * m * L;
    const long long e0 = r0 * L, e1 = r1 * L;
    const int step = (int)(blockDim.x % L);
    int j = (int)((e0 + tid) % L);  // column of element e, advanced without a division
    double num = 0.0;
    for (long long e = e0 + tid; e < e1; e += blockDim.x) {
        if (keep[j]) {
            const double dr = (double)t1r[off + e] - t2r[off + e], di = (double)t1i[off + e] - t2i[off + e];
            num += dr * dr + di * di;
        }
        j += step;
        if (j >= L) j -= L;
    }
    red[tid] = num;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if (tid < h) red[tid] += red[tid + h];
        __syncthreads();
    }
    if (tid == 0) part[(long long)s * kAccSplit + w] = red[0];
}

// Per slice: the partial sums in band order, and the test against the kept
// shrunk energy (or the slice's Frobenius norm squared with fro2)
__device__ __forceinline__ int slice_inaccurate(const double* __restrict__ part, const double* __restrict__ sigma,
                                                const int* __restrict__ lact, const double* __restrict__ fro2, int L,
                                                double tau, double delta, int s)
{
    double num = 0.0;
    for (int w = 0; w < kAccSplit; ++w) num += part[(long long)s * kAccSplit + w];
    const double* sg = sigma + (long long)s * L;
    double den = 0.0;
    for (int j = 0; j < lact[s]; ++j)
        if (sg[j] > tau) den += (sg[j] - tau) * (sg[j] - tau);
    if (fro2 && den > 0.0) den = fmax(den, fro2[s]);
    // NaN-safe: anything but a finite residual within the bound fails
    // (num is 0 when no triplet is kept, and 0 <= 0 passes)
    return !(num <= delta * delta * den) ? 1 : 0;
}

__global__ __launch_bounds__(64) void k_accuracy(const double* __restrict__ part, const double* __restrict__ sigma,
                                                 const int* __restrict__ lact, const double* __restrict__ fro2, int L,
                                                 double tau, double delta, int* __restrict__ bad, int nslices,
                                                 const int* __restrict__ gate)
{
    if (gate && *gate == 0) return;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nslices) return;
    bad[s] = slice_inaccurate(part, sigma, lact, fro2, L, tau, delta, s);
}

// ---------------------------------------------------------------- features --
// Per slice: f = [log(tau/rms sigma), log(max column norm / tau), prev/p,
// has_prev, frequency, real, log(p)/8, log(max(m,n)/p), and from the previous
// call's leading singular values s: #{s > tau}/p, #{s > tau/1.25}/p,
// log(s_1/tau), [s_c > tau]], logarithms clamped to [-30, 30].
// Squared column norms of each slice over one band of rows: block (c, s)
// writes part[(s * nsplit + c) * n + j] for every column j (FP64 sums of
// the FP32 entries; rows read whole, coalesced across the columns).
__global__ __launch_bounds__(256) void k_features_part(const float* __restrict__ yr, const float* __restrict__ yi,
                                                       int m, int n, int nsplit, double* __restrict__ part)
{
    const int c = blockIdx.x, s = blockIdx.y, tid = threadIdx.x;
    const int rows = (m + nsplit - 1) / nsplit, i0 = c * rows, i1 = min(m, i0 + rows);
    const float* Yr = yr + (long long)s * m * n;
    const float* Yi = yi + (long long)s * m * n;
    double* out = part + ((long long)s * nsplit + c) * n;
    if ((n & 3) == 0) {  // 16-byte loads of 4 neighbouring columns
        constexpr int U = 8;  // rows in flight per thread (loaded before any is summed)
        for (int j = 4 * tid; j < n; j += 4 * blockDim.x) {
            double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
            for (int i = i0; i < i1; i += U) {
                float4 r[U], q[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {  // rows past the band re-read its last row (not summed)
                    const long long o = (long long)min(i + u, i1 - 1) * n + j;
                    r[u] = *reinterpret_cast<const float4*>(Yr + o);
                    q[u] = *reinterpret_cast<const float4*>(Yi + o);
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {  // rows in order, as one row at a time
                    if (i + u < i1) {
                        a0 += (double)r[u].x * r[u].x + (double)q[u].x * q[u].x;
                        a1 += (double)r[u].y * r[u].y + (double)q[u].y * q[u].y;
                        a2 += (double)r[u].z * r[u].z + (double)q[u].z * q[u].z;
                        a3 += (double)r[u].w * r[u].w + (double)q[u].w * q[u].w;
                    }
                }
            }
            out[j] = a0;
            out[j + 1] = a1;
            out[j + 2] = a2;
            out[j + 3] = a3;
        }
        return;
    }
    for (int j = tid; j < n; j += blockDim.x) {
        double acc = 0.0;
        for (int i = i0; i < i1; ++i) {
            const double a = Yr[(long long)i * n + j], b = Yi[(long long)i * n + j];
            acc += a * a + b * b;
        }
        out[j] = acc;
    }
}

constexpr int kFeatSplit = 16;  // row bands of the column norms (partials summed by k_features)

__global__ __launch_bounds__(256) void k_features(const double* __restrict__ part, int m, int n, int nsplit, int n3,
                                                  int nslices, double tau, const int* __restrict__ prev,
                                                  const float* __restrict__ psig, float* __restrict__ feats,
                                                  double* __restrict__ fro2)
{
    __shared__ double red[4], redm[4];
    const int s = blockIdx.x, tid = threadIdx.x;
    double tot = 0.0, cmax = 0.0;
    for (int j = tid; j < n; j += blockDim.x) {
        // the column's partial sums all in flight, then added in the fixed order b = 0, 1, ...
        double v[kFeatSplit];
#pragma unroll
        for (int b = 0; b < kFeatSplit; ++b) v[b] = b < nsplit ? part[((long long)s * nsplit + b) * n + j] : 0.0;
        double c = 0.0;
#pragma unroll
        for (int b = 0; b < kFeatSplit; ++b) c += v[b];
        tot += c;
        cmax = fmax(cmax, c);
    }
    // wavefront butterflies (every lane ends with the same bits), then the four wavefronts in order
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        tot += __shfl_xor(tot, o);
        cmax = fmax(cmax, __shfl_xor(cmax, o));
    }
    if ((tid & 63) == 0) {
        red[tid >> 6] = tot;
        redm[tid >> 6] = cmax;
    }
    __syncthreads();
    if (tid == 0) {
        const int p = m < n ? m : n;
        const double nrm2 = ((red[0] + red[1]) + red[2]) + red[3], t2 = tau * tau;
        const double cm = fmax(fmax(redm[0], redm[1]), fmax(redm[2], redm[3]));
        if (fro2) fro2[s] = nrm2;
        auto clampf = [](double v) { return (float)fmin(30.0, fmax(-30.0, v)); };
        float* f = feats + (long long)s * TP_MLP_INPUTS;
        // a zero slice (or tau = 0) takes the clamped limit of the logarithm
        f[0] = nrm2 > 0.0 ? (t2 > 0.0 ? clampf(0.5 * log(t2 * p / nrm2)) : -30.0f) : 30.0f;
        f[1] = (cm > 0.0 && t2 > 0.0) ? clampf(0.5 * log(cm / t2)) : (cm > 0.0 ? 30.0f : -30.0f);
        f[2] = prev ? (float)prev[s] / (float)p : 0.0f;
        f[3] = prev ? 1.0f : 0.0f;
        f[4] = n3 > 1 ? (float)s / (float)(n3 / 2 > 0 ? n3 / 2 : 1) : 0.0f;
        f[5] = is_real_slice(s, n3) ? 1.0f : 0.0f;
        f[6] = (float)(log((double)p) / 8.0);
        f[7] = (float)log((double)(m > n ? m : n) / (double)p);
        float f8 = 0.0f, f9 = 0.0f, f10 = 0.0f, f11 = 0.0f;
        if (psig) {
            const float* sv = psig + (long long)s * TP_SIGMA_KEEP;
            int a = 0, b = 0, c = 0;
            for (int j = 0; j < TP_SIGMA_KEEP; ++j) {
                const double v = sv[j];
                c += v > 0.0 ? 1 : 0;
                a += v > tau ? 1 : 0;
                b += v > tau / 1.25 ? 1 : 0;
            }
            f8 = (float)a / (float)p;
            f9 = (float)b / (float)p;
            f10 = (sv[0] > 0.0f && tau > 0.0) ? clampf(log((double)sv[0] / tau)) : (sv[0] > 0.0f ? 30.0f : -30.0f);
            f11 = (c > 0 && (double)sv[c - 1] > tau) ? 1.0f : 0.0f;
        }
        f[8] = f8;
        f[9] = f9;
        f[10] = f10;
        f[11] = f11;
    }
}

// Leading singular values of each slice, sorted decreasing, TP_SIGMA_KEEP per
// slice (zero-padded): row r of `out` (slice map[r], or r) from the P
// unsorted values sig[r*P ..], of which the first lact[r] are valid (or all);
// rows with skip[r] != 0 are left alone.
__global__ __launch_bounds__(256) void k_sigma_top(const double* __restrict__ sig, int P, const int* __restrict__ lact,
                                                   const int* __restrict__ map, const int* __restrict__ skip,
                                                   float* __restrict__ out, const int* __restrict__ count)
{
    const int r = blockIdx.x;
    if (count && r >= *count) return;
    if (skip && skip[r]) return;
    const int valid = lact ? min(lact[r], P) : P;
    const double* sv = sig + (long long)r * P;
    float* o = out + (long long)(map ? map[r] : r) * TP_SIGMA_KEEP;
    for (int j = threadIdx.x; j < TP_SIGMA_KEEP; j += blockDim.x) o[j] = 0.0f;
    __syncthreads();
    for (int j = threadIdx.x; j < valid; j += blockDim.x) {
        int rank = 0;
        for (int i = 0; i < valid; ++i) rank += (sv[i] > sv[j] || (sv[i] == sv[j] && i < j)) ? 1 : 0;
        if (rank < TP_SIGMA_KEEP) o[rank] = (float)sv[j];
    }
}

// --------------------------------------------------------------------- MLP --
constexpr int D = TP_MLP_INPUTS, H = TP_MLP_HIDDEN;

struct MlpOffsets {
    static constexpr int W1 = 0, B1 = W1 + H * D, W2 = B1 + H, B2 = W2 + H * H, W3 = B2 + H, B3 = W3 + H * H,
                         W4 = B3 + H, B4 = W4 + H, COUNT = B4 + 1;
};

__device__ __forceinline__ float mlp_eval(const float* p, const float* x, float* z1, float* z2, float* z3)
{
    using O = MlpOffsets;
    for (int i = 0; i < H; ++i) {
        float v = p[O::B1 + i];
        for (int j = 0; j < D; ++j) v = fmaf(p[O::W1 + i * D + j], x[j], v);
        z1[i] = v;
    }
    for (int i = 0; i < H; ++i) {
        float v = p[O::B2 + i];
        for (int j = 0; j < H; ++j) v = fmaf(p[O::W2 + i * H + j], fmaxf(z1[j], 0.0f), v);
        z2[i] = v;
    }
    for (int i = 0; i < H; ++i) {
        float v = p[O::B3 + i];
        for (int j = 0; j < H; ++j) v = fmaf(p[O::W3 + i * H + j], fmaxf(z2[j], 0.0f), v);
        z3[i] = v;
    }
    float y = p[O::B4];
    for (int j = 0; j < H; ++j) y = fmaf(p[O::W4 + j], fmaxf(z3[j], 0.0f), y);
    return y;
}

// y[s] = MLP(x[s]) for a batch (one thread per sample; weights in LDS)
__global__ __launch_bounds__(64) void k_mlp_forward(const float* __restrict__ params, const float* __restrict__ x,
                                                    float* __restrict__ y, int batch)
{
    __shared__ float p[MlpOffsets::COUNT];
    for (int e = threadIdx.x; e < MlpOffsets::COUNT; e += blockDim.x) p[e] = params[e];
    __syncthreads();
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= batch) return;
    float z[3 * H];
    y[s] = mlp_eval(p, x + (long long)s * D, z, z + H, z + 2 * H);
}

// Rank prediction: kpred = round(expm1(y log1p(p))) clipped to [0, p] (or the
// fixed rank), lact = min(kpred + oversample, p); slices with lact > L go to
// the full SVD (fallback = 1, lact = 0).  One wavefront per slice, lane i
// computing hidden unit i of each layer (each unit's sum in the same order as
// mlp_eval, so y is bit-identical to tp_mlp_forward).
__global__ __launch_bounds__(H) void k_predict(const float* __restrict__ params, const float* __restrict__ feats,
                                               int nslices, int p, int fixed_rank, int oversample, int L,
                                               int* __restrict__ kpred, int* __restrict__ lact,
                                               int* __restrict__ fallback, int* __restrict__ rank)
{
    using O = MlpOffsets;
    __shared__ float x[D];
    __shared__ float za[H], zb[H];
    const int s = blockIdx.x, i = threadIdx.x;
    float yv = 0.0f;
    if (params) {
        if (i < D) x[i] = feats[(long long)s * D + i];
        __syncthreads();
        float v = params[O::B1 + i];
        for (int j = 0; j < D; ++j) v = fmaf(params[O::W1 + i * D + j], x[j], v);
        za[i] = v;
        __syncthreads();
        v = params[O::B2 + i];
        for (int j = 0; j < H; ++j) v = fmaf(params[O::W2 + i * H + j], fmaxf(za[j], 0.0f), v);
        zb[i] = v;
        __syncthreads();
        v = params[O::B3 + i];
        for (int j = 0; j < H; ++j) v = fmaf(params[O::W3 + i * H + j], fmaxf(zb[j], 0.0f), v);
        __syncthreads();
        za[i] = v;
        __syncthreads();
        if (i == 0) {
            yv = params[O::B4];
            for (int j = 0; j < H; ++j) yv = fmaf(params[O::W4 + j], fmaxf(za[j], 0.0f), yv);
        }
    }
    if (i != 0) return;
    int k = fixed_rank;
    if (params) {
        const double kk = expm1((double)yv * log1p((double)p));
        k = (int)fmin((double)p, fmax(0.0, rint(kk)));
    }
    k = k < 0 ? 0 : (k > p ? p : k);
    int l = k + oversample;
    if (l > p) l = p;
    kpred[s] = k;
    fallback[s] = 0;
    if (rank) rank[s] = 0;
    if (l > L) {
        fallback[s] = 1;
        l = 0;
    }
    lact[s] = l;
}

// Training: per sample forward and backward deltas of the asymmetric squared
// loss c(e) e^2 / N (c = 1 for e >= 0, `under` for e < 0); stores the
// pre-activations z1..z3, the deltas d1..d3 and the loss term.
__global__ __launch_bounds__(64) void k_mlp_fwd_bwd(const float* __restrict__ params, const float* __restrict__ x,
                                                    const float* __restrict__ t, int batch, float under,
                                                    float* __restrict__ zs, float* __restrict__ ds,
                                                    float* __restrict__ lterm)
{
    using O = MlpOffsets;
    __shared__ float p[O::COUNT];
    for (int e = threadIdx.x; e < O::COUNT; e += blockDim.x) p[e] = params[e];
    __syncthreads();
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= batch) return;
    float z[3 * H], d[3 * H];
    float *z1 = z, *z2 = z + H, *z3 = z + 2 * H, *d1 = d, *d2 = d + H, *d3 = d + 2 * H;
    const float y = mlp_eval(p, x + (long long)s * D, z1, z2, z3);
    const float e = y - t[s];
    const float c = e >= 0.0f ? 1.0f : under;
    const float dy = 2.0f * c * e / (float)batch;
    lterm[s] = c * e * e;
    for (int j = 0; j < H; ++j) d3[j] = z3[j] > 0.0f ? dy * p[O::W4 + j] : 0.0f;
    for (int j = 0; j < H; ++j) {
        float v = 0.0f;
        for (int i = 0; i < H; ++i) v = fmaf(p[O::W3 + i * H + j], d3[i], v);
        d2[j] = z2[j] > 0.0f ? v : 0.0f;
    }
    for (int j = 0; j < H; ++j) {
        float v = 0.0f;
        for (int i = 0; i < H; ++i) v = fmaf(p[O::W2 + i * H + j], d2[i], v);
        d1[j] = z1[j] > 0.0f ? v : 0.0f;
    }
    float* zo = zs + (long long)s * 3 * H;
    float* dd = ds + (long long)s * 4 * H;
    for (int j = 0; j < 3 * H; ++j) zo[j] = z[j];
    for (int j = 0; j < 3 * H; ++j) dd[j] = d[j];
    dd[3 * H] = dy;
}

// grad[param] = sum over samples in index order (deterministic, no atomics)
__global__ __launch_bounds__(256) void k_mlp_grad(const float* __restrict__ x, const float* __restrict__ zs,
                                                  const float* __restrict__ ds, const float* __restrict__ lterm,
                                                  int batch, float* __restrict__ grad, float* __restrict__ loss)
{
    using O = MlpOffsets;
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q == O::COUNT) {
        float acc = 0.0f;
        for (int s = 0; s < batch; ++s) acc += lterm[s];
        *loss = acc / (float)batch;
        return;
    }
    if (q > O::COUNT) return;
    float acc = 0.0f;
    // locate parameter q: delta index di (layer l, unit i) and activation source
    for (int s = 0; s < batch; ++s) {
        const float* z = zs + (long long)s * 3 * H;
        const float* d = ds + (long long)s * 4 * H;
        float v;
        if (q < O::B1) {
            const int i = (q - O::W1) / D, j = (q - O::W1) % D;
            v = d[i] * x[(long long)s * D + j];
        } else if (q < O::W2) {
            v = d[q - O::B1];
        } else if (q < O::B2) {
            const int i = (q - O::W2) / H, j = (q - O::W2) % H;
            v = d[H + i] * fmaxf(z[j], 0.0f);
        } else if (q < O::W3) {
            v = d[H + (q - O::B2)];
        } else if (q < O::B3) {
            const int i = (q - O::W3) / H, j = (q - O::W3) % H;
            v = d[2 * H + i] * fmaxf(z[H + j], 0.0f);
        } else if (q < O::W4) {
            v = d[2 * H + (q - O::B3)];
        } else if (q < O::B4) {
            v = d[3 * H] * fmaxf(z[2 * H + (q - O::W4)], 0.0f);
        } else {
            v = d[3 * H];
        }
        acc += v;
    }
    grad[q] = acc;
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                                              float* __restrict__ v, int count, float lr, float b1, float b2,
                                              float eps, float c1, float c2)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= count) return;
    const float gq = g[q];
    const float mq = b1 * m[q] + (1.0f - b1) * gq;
    const float vq = b2 * v[q] + (1.0f - b2) * gq * gq;
    m[q] = mq;
    v[q] = vq;
    p[q] -= lr * (mq / c1) / (sqrtf(vq / c2) + eps);
}

// copy slices idx[0..cnt) of a planar stack into / out of a compact stack
__global__ __launch_bounds__(256) void k_gather(const float* __restrict__ sr, const float* __restrict__ si,
                                                float* __restrict__ dr, float* __restrict__ di,
                                                const int* __restrict__ idx, int cnt, long long per, int scatter,
                                                const int* __restrict__ count)
{
    const long long total = (long long)(count ? min(*count, cnt) : cnt) * per;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const long long c = e / per, o = e % per;
        const long long full = (long long)idx[c] * per + o;
        if (scatter) {
            dr[full] = sr[e];
            di[full] = si[e];
        } else {
            dr[e] = sr[full];
            di[e] = si[full];
        }
    }
}

// ------------------------------------------------- device-side control --
// The decisions of the learned prox that depend on device data are taken by
// these single-workgroup kernels; later launches read their results (gates,
// widths, counts), so a call never waits for the host.

// OR of v over the workgroup (every thread gets it)
__device__ __forceinline__ int block_or(int v) { return __syncthreads_or(v); }

// Common sketch width of an attempt: L = the widest l over the slices not
// already sent to the full SVD, rounded up to 8, at most max_rank (0: none);
// every such slice then uses l = min(L, p) columns and kpred = max(kpred,
// l - oversample).  set_fb: fallback starts as the pre-sent slices (all
// slices when L = 0).
// gate_in (optional) = 0 leaves L = 0 and the attempt's gate closed.
__global__ __launch_bounds__(256) void k_width(int* __restrict__ kpred, int* __restrict__ lact,
                                               const int* __restrict__ prefb, int* __restrict__ fb, int nslices,
                                               int p, int oversample, int max_rank, const int* __restrict__ gate_in,
                                               int* __restrict__ ctl_L, int* __restrict__ ctl_gate, int set_fb)
{
    __shared__ int red[256];
    const int tid = threadIdx.x;
    const bool open = !gate_in || *gate_in != 0;
    int m = 0;
    for (int q = tid; q < nslices; q += blockDim.x) {
        if (set_fb) fb[q] = prefb[q];
        if (!prefb[q]) m = max(m, lact[q]);
    }
    red[tid] = m;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (tid < w) red[tid] = max(red[tid], red[tid + w]);
        __syncthreads();
    }
    const int lmax = red[0];
    const int L = (open && lmax > 0) ? min(((lmax + 7) / 8) * 8, max_rank) : 0;
    if (set_fb && L == 0)  // no sketch at all: every slice takes the full SVD
        for (int q = tid; q < nslices; q += blockDim.x) fb[q] = 1;
    if (L > 0)
        for (int q = tid; q < nslices; q += blockDim.x)
            if (!prefb[q]) {
                lact[q] = min(L, p);
                kpred[q] = max(kpred[q], lact[q] - oversample);
            }
    if (tid == 0) {
        *ctl_L = L;
        *ctl_gate = L > 0 ? 1 : 0;
    }
}

// Wide retry: slices whose count check failed below the widest sketch get
// kpred = max_rank - oversample, l = kpred + oversample (at most p); the
// retry gate opens when there is one and the first attempt ran.
__global__ __launch_bounds__(256) void k_retry(const int* __restrict__ fb, const int* __restrict__ prefb,
                                               int* __restrict__ kpred, int* __restrict__ lact, int nslices, int p,
                                               int oversample, int max_rank, const int* __restrict__ gate_in,
                                               int* __restrict__ ctl_retry)
{
    const int kwide = min(max(max_rank - oversample, 0), p), lwide = min(kwide + oversample, p);
    const bool open = *gate_in != 0;
    int any = 0;
    for (int q = threadIdx.x; q < nslices; q += blockDim.x)
        if (open && fb[q] && !prefb[q] && lact[q] < lwide && kpred[q] < kwide) {
            kpred[q] = kwide;
            lact[q] = lwide;
            any = 1;
        }
    any = block_or(any);
    if (threadIdx.x == 0) *ctl_retry = any;
}

// End of an accuracy round (when it ran): next = some slice still inaccurate
// and not sent to the full SVD, unless this was the last round, whose
// inaccurate slices join the fallback set.
// The verdict of each slice (bad: see k_accuracy) is formed here from the
// partial residual sums when part is given.
__global__ __launch_bounds__(256) void k_round(int* __restrict__ bad, int* __restrict__ fb, int nslices,
                                               const int* __restrict__ cur, int* __restrict__ next, int last,
                                               const double* __restrict__ part, const double* __restrict__ sigma,
                                               const int* __restrict__ lact, const double* __restrict__ fro2, int L,
                                               double tau, double delta)
{
    if (*cur == 0) {
        if (next && threadIdx.x == 0) *next = 0;
        return;
    }
    if (part)
        for (int q = threadIdx.x; q < nslices; q += blockDim.x) bad[q] = slice_inaccurate(part, sigma, lact, fro2, L, tau,
                                                                                          delta, q);
    __syncthreads();
    int any = 0;
    for (int q = threadIdx.x; q < nslices; q += blockDim.x) any |= (bad[q] && !fb[q]) ? 1 : 0;
    any = block_or(any);
    if (last && any)
        for (int q = threadIdx.x; q < nslices; q += blockDim.x)
            if (bad[q]) fb[q] = 1;
    if (next && threadIdx.x == 0) *next = (!last && any) ? 1 : 0;
}

// idx[0..count) = the fallback slices in increasing order; count to *count
__global__ __launch_bounds__(64) void k_compact(const int* __restrict__ fb, int nslices, int* __restrict__ idx,
                                                int* __restrict__ count)
{
    if (threadIdx.x != 0) return;
    int c = 0;
    for (int q = 0; q < nslices; ++q)
        if (fb[q]) idx[c++] = q;
    *count = c;
}

// the full-SVD counts and sweeps of the compact fallback slices back to
// their slices (info: 0 for the others)
__global__ __launch_bounds__(256) void k_fb_results(const int* __restrict__ idx, const int* __restrict__ count,
                                                    const int* __restrict__ crank, const int* __restrict__ cinfo,
                                                    const int* __restrict__ fb, int* __restrict__ rank,
                                                    int* __restrict__ info, int nslices)
{
    const int c = *count;
    for (int q = threadIdx.x; q < nslices; q += blockDim.x)
        if (info && !fb[q]) info[q] = 0;
    __syncthreads();
    for (int j = threadIdx.x; j < c; j += blockDim.x) {
        rank[idx[j]] = crank[j];
        if (info) info[idx[j]] = cinfo[j];
    }
}

// dst = src (planar, n floats per plane) when the gate is open
__global__ __launch_bounds__(256) void k_copy_planes(const float* __restrict__ sr, const float* __restrict__ si,
                                                     float* __restrict__ dr, float* __restrict__ di, long long n,
                                                     const int* __restrict__ gate)
{
    if (gate && *gate == 0) return;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
        dr[e] = sr[e];
        di[e] = si[e];
    }
}

__global__ __launch_bounds__(256) void k_fill_int(int* __restrict__ p, long long n, int v)
{
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
        p[e] = v;
}

inline int blocks_for(long long n, int tpb, int cap = 8192)
{
    long long b = (n + tpb - 1) / tpb;
    return (int)(b < 1 ? 1 : (b > cap ? cap : b));
}

}  // namespace

int mlp_param_count() { return MlpOffsets::COUNT; }

hipError_t launch_sketch(float* omr, float* omi, int n, int L, const int* lact, int nslices, int n3,
                         unsigned long long seed, WarmBasis warm, hipStream_t st, const int* gate)
{
    k_sketch<<<blocks_for((long long)nslices * n * L, 256), 256, 0, st>>>(omr, omi, n, L, lact, nslices, n3, seed,
                                                                          warm, gate);
    return hipGetLastError();
}

// The range basis Q2 (n x L per slice, planar) into the caller's basis
// buffer (n x ld per slice), zero beyond the slice's valid columns, and the
// valid count per slice (0 for fallback slices, whose basis failed).
__global__ __launch_bounds__(256) void k_store_basis(const float* __restrict__ zr, const float* __restrict__ zi, int n,
                                                     int L, const int* __restrict__ lact, const int* __restrict__ fb,
                                                     int nslices, float* __restrict__ outr, float* __restrict__ outi,
                                                     int ld, int* __restrict__ cols, const int* __restrict__ gate)
{
    if (gate && *gate == 0) return;
    const long long total = (long long)nslices * n * ld;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const int s = (int)(e / ((long long)n * ld));
        const int rem = (int)(e % ((long long)n * ld));
        const int i = rem / ld, j = rem % ld;
        const int valid = fb[s] ? 0 : min(lact[s], L);
        float vr = 0.0f, vi = 0.0f;
        if (j < valid) {
            const long long o = ((long long)s * n + i) * L + j;
            vr = zr[o];
            vi = zi[o];
        }
        outr[e] = vr;
        outi[e] = vi;
        if (rem == 0) cols[s] = valid;
    }
}

hipError_t launch_store_basis(const float* zr, const float* zi, int n, int L, const int* lact, const int* fb,
                              int nslices, float* outr, float* outi, int ld, int* cols, hipStream_t st,
                              const int* gate)
{
    k_store_basis<<<blocks_for((long long)nslices * n * ld, 256), 256, 0, st>>>(zr, zi, n, L, lact, fb, nslices,
                                                                                outr, outi, ld, cols, gate);
    return hipGetLastError();
}

int gram_split(int m) { return m >= 1024 ? kMaxGramSplit : (m >= 256 ? 8 : 1); }

hipError_t launch_reduce_gram(const float* parts, int ksplit, int m, int L, int nslices, int real_first, int real_last,
                              float* yr, float* yi, const int* lact, double2* part, hipStream_t st,
                              const int* gate, const int* width)
{
    if (L > kMaxL || ksplit < 1 || ksplit > kMaxParts) return hipErrorInvalidValue;
    const int ns = gram_split(m);
    k_reduce_gram<<<dim3(ns, nslices), 256, 0, st>>>(parts, ksplit, m, L, nslices, real_first, real_last, yr, yi, lact,
                                                     part, ns, gate, width);
    return hipGetLastError();
}

hipError_t launch_cholqr_pass(const float* yr, const float* yi, int m, int L, const int* lact, int nslices,
                              int pass, double2* part, float* rir, float* rii, double2* rtot, float* rhr,
                              float* rhi, int* status, hipStream_t st, bool gram_ready, const int* gate)
{
    if (L > kMaxL) return hipErrorInvalidValue;
    const int ns = gram_split(m);
    if (!gram_ready) k_gram<<<dim3(ns, nslices), 256, 0, st>>>(yr, yi, m, L, lact, part, ns, gate);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t lds = 2 * (size_t)L * L * sizeof(double2);
    if (lds + 16 * 1024 > 64 * 1024) {  // dynamic + the static panel buffers
        e = hipFuncSetAttribute((const void*)k_chol, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    k_chol<<<nslices, kCholThreads, lds, st>>>(part, ns, L, lact, pass, rir, rii, rtot, rhr, rhi, status, gate);
    return hipGetLastError();
}

size_t cholqr_part_bytes(int m, int L, int nslices)
{
    return align_up((size_t)gram_split(m) * nslices * L * L * sizeof(double2));
}

hipError_t launch_rsvd_check(const float2* cols, const double* sigma, const float2* vr, const int* kpred,
                             const int* lact, const int* prefb, const int* status, int L, double tau, Planes T,
                             int* fallback, int* rank, int nslices, hipStream_t st, const int* gate, Planes vp,
                             Planes cp)
{
    k_rsvd_check<<<nslices, 256, 0, st>>>(cols, sigma, vr, kpred, lact, prefb, status, L, tau, T.re, T.im, fallback,
                                          rank, gate, vp.re, vp.im, cp.re, cp.im);
    return hipGetLastError();
}

hipError_t launch_cm_to_planar(const float2* src, Planes dst, int L, int nslices, hipStream_t st, const int* gate,
                               const float2* src2, Planes dst2)
{
    k_cm_to_planar<<<blocks_for((long long)nslices * L * L, 256), 256, 0, st>>>(src, dst.re, dst.im, L, nslices,
                                                                                gate, src2, dst2.re, dst2.im);
    return hipGetLastError();
}

size_t accuracy_part_bytes(int nslices) { return align_up((size_t)nslices * kAccSplit * sizeof(double)); }

hipError_t launch_accuracy(Planes t1, Planes t2, const double* sigma, const int* lact, const double* fro2, int m,
                           int L, double tau, double delta, int* bad, int nslices, double* part, hipStream_t st,
                           const int* gate)
{
    // part: nslices x kAccSplit doubles (accuracy_part_bytes)
    k_accuracy_part<<<dim3(kAccSplit, nslices), 256, 0, st>>>(t1.re, t1.im, t2.re, t2.im, sigma, lact, m, L, tau,
                                                              part, gate);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_accuracy<<<(nslices + 63) / 64, 64, 0, st>>>(part, sigma, lact, fro2, L, tau, delta, bad, nslices, gate);
    return hipGetLastError();
}

int features_split(int m) { return m < kFeatSplit * 32 ? (m + 31) / 32 : kFeatSplit; }

size_t features_part_bytes(int m, int n, int nslices)
{
    return align_up((size_t)nslices * features_split(m) * n * sizeof(double));
}

hipError_t launch_features(const float* yr, const float* yi, int m, int n, int n3, int nslices, double tau,
                           const int* prev, const float* prev_sigma, float* feats, double* part, double* fro2,
                           hipStream_t st)
{
    const int ns = features_split(m);
    k_features_part<<<dim3(ns, nslices), 256, 0, st>>>(yr, yi, m, n, ns, part);
    k_features<<<nslices, 256, 0, st>>>(part, m, n, ns, n3, nslices, tau, prev, prev_sigma, feats, fro2);
    return hipGetLastError();
}

hipError_t launch_sigma_top(const double* sig, int P, const int* lact, const int* map, const int* skip, int rows,
                            float* out, hipStream_t st, const int* count)
{
    if (rows <= 0) return hipSuccess;
    k_sigma_top<<<rows, 256, 0, st>>>(sig, P, lact, map, skip, out, count);
    return hipGetLastError();
}

hipError_t launch_predict(const float* params, const float* feats, int nslices, int p, int fixed_rank,
                          int oversample, int L, int* kpred, int* lact, int* fallback, int* rank, hipStream_t st)
{
    k_predict<<<nslices, H, 0, st>>>(params, feats, nslices, p, fixed_rank, oversample, L, kpred, lact, fallback,
                                     rank);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const float* params, const float* x, float* y, int batch, hipStream_t st)
{
    k_mlp_forward<<<(batch + 63) / 64, 64, 0, st>>>(params, x, y, batch);
    return hipGetLastError();
}

size_t mlp_train_bytes(int batch)
{
    return align_up((size_t)batch * 3 * H * sizeof(float)) + align_up((size_t)batch * 4 * H * sizeof(float)) +
           align_up((size_t)batch * sizeof(float));
}

hipError_t launch_mlp_loss_grad(const float* params, const float* x, const float* t, int batch, float under,
                                float* grad, float* loss, void* ws, hipStream_t st)
{
    char* b = static_cast<char*>(ws);
    float* zs = reinterpret_cast<float*>(b);
    float* ds = reinterpret_cast<float*>(b + align_up((size_t)batch * 3 * H * sizeof(float)));
    float* lt = reinterpret_cast<float*>(b + align_up((size_t)batch * 3 * H * sizeof(float)) +
                                         align_up((size_t)batch * 4 * H * sizeof(float)));
    k_mlp_fwd_bwd<<<(batch + 63) / 64, 64, 0, st>>>(params, x, t, batch, under, zs, ds, lt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_mlp_grad<<<(MlpOffsets::COUNT + 1 + 255) / 256, 256, 0, st>>>(x, zs, ds, lt, batch, grad, loss);
    return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int count, int step, float lr, float b1, float b2,
                       float eps, hipStream_t st)
{
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    k_adam<<<(count + 255) / 256, 256, 0, st>>>(p, g, m, v, count, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_width(int* kpred, int* lact, const int* prefb, int* fb, int nslices, int p, int oversample,
                        int max_rank, const int* gate_in, int* ctl_L, int* ctl_gate, bool set_fb, hipStream_t st)
{
    k_width<<<1, 256, 0, st>>>(kpred, lact, prefb, fb, nslices, p, oversample, max_rank, gate_in, ctl_L, ctl_gate,
                               set_fb ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_retry(const int* fb, const int* prefb, int* kpred, int* lact, int nslices, int p, int oversample,
                        int max_rank, const int* gate_in, int* ctl_retry, hipStream_t st)
{
    k_retry<<<1, 256, 0, st>>>(fb, prefb, kpred, lact, nslices, p, oversample, max_rank, gate_in, ctl_retry);
    return hipGetLastError();
}

hipError_t launch_round(int* bad, int* fb, int nslices, const int* cur, int* next, bool last, hipStream_t st)
{
    k_round<<<1, 256, 0, st>>>(bad, fb, nslices, cur, next, last ? 1 : 0, nullptr, nullptr, nullptr, nullptr, 0, 0.0,
                               0.0);
    return hipGetLastError();
}

hipError_t launch_accuracy_round(Planes t1, Planes t2, const double* sigma, const int* lact, const double* fro2, int m,
                                 int L, double tau, double delta, int* bad, int nslices, double* part, int* fb,
                                 const int* cur, int* next, bool last, hipStream_t st)
{
    k_accuracy_part<<<dim3(kAccSplit, nslices), 256, 0, st>>>(t1.re, t1.im, t2.re, t2.im, sigma, lact, m, L, tau,
                                                              part, cur);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_round<<<1, 256, 0, st>>>(bad, fb, nslices, cur, next, last ? 1 : 0, part, sigma, lact, fro2, L, tau, delta);
    return hipGetLastError();
}

hipError_t launch_compact(const int* fb, int nslices, int* idx, int* count, hipStream_t st)
{
    k_compact<<<1, 64, 0, st>>>(fb, nslices, idx, count);
    return hipGetLastError();
}

hipError_t launch_fb_results(const int* idx, const int* count, const int* crank, const int* cinfo, const int* fb,
                             int* rank, int* info, int nslices, hipStream_t st)
{
    k_fb_results<<<1, 256, 0, st>>>(idx, count, crank, cinfo, fb, rank, info, nslices);
    return hipGetLastError();
}

hipError_t launch_copy_planes(const float* sr, const float* si, float* dr, float* di, long long n, const int* gate,
                              hipStream_t st)
{
    k_copy_planes<<<blocks_for(n, 256), 256, 0, st>>>(sr, si, dr, di, n, gate);
    return hipGetLastError();
}

hipError_t launch_fill_int(int* p, long long n, int v, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    k_fill_int<<<blocks_for(n, 256), 256, 0, st>>>(p, n, v);
    return hipGetLastError();
}

hipError_t launch_gather(const float* sr, const float* si, float* dr, float* di, const int* idx, int cnt,
                         long long per, bool scatter, hipStream_t st, const int* count)
{
    if (cnt <= 0) return hipSuccess;
    k_gather<<<blocks_for((long long)cnt * per, 256), 256, 0, st>>>(sr, si, dr, di, idx, cnt, per, scatter ? 1 : 0,
                                                                    count);
    return hipGetLastError();
}

}  // namespace tp
