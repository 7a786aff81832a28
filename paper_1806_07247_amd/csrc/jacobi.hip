// Per-slice SVD by one-sided (Hestenes) Jacobi, the "SVD" of Algorithms 2 and
// 3 (step 2), and the singular value shrinkage of Theorem 2.3 / eq (21).
//
// One workgroup owns one Fourier slice.  The slice (or its conjugate
// transpose when it is wide, so that the work matrix is R x P with R >= P) is
// held column-major as float2 (re, im), in LDS when it fits and otherwise in a
// workspace buffer.  A sweep visits all P(P-1)/2 column pairs in P'-1 steps of
// P'/2 disjoint pairs (round-robin "circle" order, P' = P rounded up to even);
// a barrier separates steps.  A group of G lanes handles one pair: each lane
// holds RPL rows of both columns in registers, accumulates its part of
//   alpha = ||x||^2, beta = ||y||^2, gamma = x^* y
// in FP32, and the group sums the parts in FP64 with a butterfly of DPP moves
// (every lane ends with bitwise identical sums, so all lanes take the same
// decision); when |gamma| > tol sqrt(alpha beta) it applies
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
    if (pos == 0) return 0;
    int c = pos - 1 + step;  // < 2 (np - 1)
    if (c >= np - 1) c -= np - 1;
    return 1 + c;
}

// 1/sqrt(x) and 1/x for normal x > 0 (x != 0): the hardware estimate and two
// Newton steps, each doubling the correct bits
__device__ __forceinline__ double rsqrt_f64(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    double h = x * y;
    y = fma(0.5 * y, fma(-h, y, 1.0), y);
    h = x * y;
    return fma(0.5 * y, fma(-h, y, 1.0), y);
}
__device__ __forceinline__ double rcp_f64(double x)
{
    double y = __builtin_amdgcn_rcp(x);
    y = fma(y, fma(-x, y, 1.0), y);
    return fma(y, fma(-x, y, 1.0), y);
}

// DPP move of a double within a row of 16 lanes
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v)
{
    const long long u = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(u & 0xffffffff), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(u >> 32), CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the G lanes of a group.  Each level adds a partner's value with a
// commutative add, so every lane of the group ends with the same bits.
// Partners: lane^1, lane^2 (quad permutations), the mirror within 8 lanes and
// within 16 lanes (DPP), then lane^16, lane^32 for wider groups.
template <int G>
__device__ __forceinline__ double group_sum(double v)
{
    if (G >= 2) v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
    if (G >= 4) v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
    if (G >= 8) v += dpp_f64<0x141>(v);  // row_half_mirror
    if (G >= 16) v += dpp_f64<0x140>(v); // row_mirror
#pragma unroll
    for (int m = 16; m < G; m <<= 1) v += __shfl_xor(v, m, G);
    return v;
}

// One Jacobi rotation of columns p and q (each R long, stride ldr in `work`)
// by the G lanes of a group; gl is the lane within the group.  Returns true
// when the pair was rotated (identically in every lane of the group).
template <int G, int RPL, bool WITHV>
__device__ __forceinline__ bool jacobi_pair(float2* work, int ldr, int p, int q, int R, int gl, double tol2,
                                            float2* vw, int ldv, int P)
{
    float2* xc = work + (long long)p * ldr;
    float2* yc = work + (long long)q * ldr;
    float2 x[RPL], y[RPL];
    double al, be, gr, gi;
    float pa = 0.f, pb = 0.f, pr = 0.f, pi = 0.f;
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
        pa = fmaf(x[t].x, x[t].x, fmaf(x[t].y, x[t].y, pa));
        pb = fmaf(y[t].x, y[t].x, fmaf(y[t].y, y[t].y, pb));
        pr = fmaf(x[t].x, y[t].x, fmaf(x[t].y, y[t].y, pr));
        pi = fmaf(x[t].x, y[t].y, fmaf(-x[t].y, y[t].x, pi));
    }
    // per-lane partial sums of RPL rows in FP32 (relative error ~RPL u32, far
    // below the rotation threshold); the cross-lane sums and everything after
    // them in FP64
    al = group_sum<G>((double)pa);
    be = group_sum<G>((double)pb);
    gr = group_sum<G>((double)pr);
    gi = group_sum<G>((double)pi);
    const double g2 = gr * gr + gi * gi;
    // rotate when |gamma| > tol sqrt(alpha beta)
    if (!(g2 > 0.0 && g2 > tol2 * al * be)) return false;
    // x' = c x - s conj(e) y,  y' = s e x + c y,  e = gamma/|gamma|,
    // t = s/c the smaller root of t^2 + 2 zeta t - 1 = 0, zeta = (beta - alpha)/(2|gamma|)
    // the chain of square roots and reciprocals from the hardware estimates
    // refined by Newton steps (relative error ~1e-15, far below the FP32
    // columns' rounding; a fraction of the IEEE sequences' latency)
    const double ig = rsqrt_f64(g2);
    const double zeta = 0.5 * (be - al) * ig;
    const double z2 = fma(zeta, zeta, 1.0);
    const double t = copysign(rcp_f64(fabs(zeta) + z2 * rsqrt_f64(z2)), zeta);
    const double c = rsqrt_f64(fma(t, t, 1.0));
    const double sn = c * t;
    const float cf = (float)c;
    const float sr = (float)(sn * gr * ig), si = (float)(sn * gi * ig);  // s e
#pragma unroll
    for (int t2 = 0; t2 < RPL; ++t2) {
        const int i = gl + G * t2;
        if (i < R) {
            const float2 xv = x[t2], yv = y[t2];
            // s conj(e) y = (sr yr + si yi, sr yi - si yr);  s e x = (sr xr - si xi, sr xi + si xr)
            xc[i] = make_float2(cf * xv.x - (sr * yv.x + si * yv.y), cf * xv.y - (sr * yv.y - si * yv.x));
            yc[i] = make_float2((sr * xv.x - si * xv.y) + cf * yv.x, (sr * xv.y + si * xv.x) + cf * yv.y);
        }
    }
    if (WITHV) {  // the same rotation on columns p, q of V (P rows)
        float2* vx = vw + (long long)p * ldv;
        float2* vy = vw + (long long)q * ldv;
#pragma unroll
        for (int t2 = 0; t2 < RPL; ++t2) {
            const int i = gl + G * t2;
            if (i < P) {
                const float2 xv = vx[i], yv = vy[i];
                vx[i] = make_float2(cf * xv.x - (sr * yv.x + si * yv.y), cf * xv.y - (sr * yv.y - si * yv.x));
                vy[i] = make_float2((sr * xv.x - si * xv.y) + cf * yv.x, (sr * xv.y + si * xv.x) + cf * yv.y);
            }
        }
    }
    return true;
}

__device__ __forceinline__ void set_identity(float2* v, int P, int w, int nw)
{
    for (int e = w; e < P * P; e += nw) v[e] = make_float2((e / P) == (e % P) ? 1.0f : 0.0f, 0.0f);
}

// Copies slice s of the planar row-major input into the column-major work
// matrix (conjugate transpose when a.transpose); worker w of nw.
__device__ __forceinline__ void load_work(const JacobiArgs& a, int s, float2* work, int R, int P, int w, int nw)
{
    const long long so = (long long)s * a.m * a.n;
    const float* yr = a.yr + so;
    const float* yi = a.yi + so;
    const int total = R * P;
    if (!a.transpose) {
        for (int e = w; e < total; e += nw) {  // Y row-major m x n: e = i*n + j
            const int i = e / P, j = e % P;
            work[(long long)j * R + i] = make_float2(yr[e], yi[e]);
        }
    } else {
        for (int e = w; e < total; e += nw) {  // column j of Y^* = conj(row j of Y)
            const int j = e / R, i = e % R;
            work[(long long)j * R + i] = make_float2(yr[e], -yi[e]);
        }
    }
}

// Column norms (FP64) and the rotated columns (row-major R x P, planar), by
// workgroup wg of nwg working on slice s.
template <int G>
__device__ __forceinline__ void store_result(const JacobiArgs& a, int s, const float2* work, int R, int P, int wg,
                                             int nwg)
{
    const int gl = threadIdx.x % G, ngroups = blockDim.x / G;
    double* sig = a.sigma + (long long)s * P;
    for (int j = wg * ngroups + threadIdx.x / G; j < P; j += nwg * ngroups) {
        double acc = 0.0;
        for (int i = gl; i < R; i += G) {
            const float2 v = work[(long long)j * R + i];
            acc = fma((double)v.x, (double)v.x, fma((double)v.y, (double)v.y, acc));
        }
        acc = group_sum<G>(acc);
        if (gl == 0) sig[j] = sqrt(acc);
    }
    if (a.wr) {
        float* wr = a.wr + (long long)s * R * P;
        float* wi = a.wi + (long long)s * R * P;
        const int total = R * P;
        for (int e = wg * blockDim.x + threadIdx.x; e < total; e += nwg * blockDim.x) {
            const int i = e / P, j = e % P;
            const float2 v = work[(long long)j * R + i];
            wr[e] = v.x;
            wi[e] = v.y;
        }
    }
    if (a.cols) {
        float2* c = a.cols + (long long)s * R * P;
        for (int e = wg * blockDim.x + threadIdx.x; e < R * P; e += nwg * blockDim.x) c[e] = work[e];
    }
}

__device__ __forceinline__ void store_q(const JacobiArgs& a, int s, const float2* q, int P, int wg, int nwg)
{
    float2* o = a.qout + (long long)s * P * P;
    for (int e = wg * blockDim.x + threadIdx.x; e < P * P; e += nwg * blockDim.x) o[e] = q[e];
}

// ---- whole slice in one workgroup (LDS when it fits, else workspace) ----
// Sweeps over the first Ps columns, touching the first Rs rows of the work
// matrix (stride R) and the first Pv rows of V (stride P): RPL rows per lane
// cover Rs and Pv.
template <int G, int RPL, bool WITHV>
__device__ __forceinline__ void sweeps_whole(const JacobiArgs& a, float2* work, float2* vw, int R, int P, int Ps,
                                             int Rs, int Pv, int& rotated, int& sweep, bool& converged)
{
    const int np = Ps + (Ps & 1);
    const int tid = threadIdx.x, group = tid / G, gl = tid % G, ngroups = blockDim.x / G;
    const double tol2 = a.tol * a.tol;
    while (!converged && sweep < a.max_sweeps) {
        for (int step = 0; step < np - 1; ++step) {
            for (int pair = group; pair < np / 2; pair += ngroups) {
                const int p = rr_col(pair, step, np);
                const int q = rr_col(np - 1 - pair, step, np);
                if (p >= Ps || q >= Ps) continue;
                if (jacobi_pair<G, RPL, WITHV>(work, R, p, q, Rs, gl, tol2, vw, P, Pv) && gl == 0)
                    rotated = 1;
            }
            __syncthreads();
        }
        ++sweep;
        converged = (rotated == 0);
        __syncthreads();
        if (tid == 0) rotated = 0;
        __syncthreads();
    }
}

// Slice s of a, held in `work` (R x P, then P x P rotations with WITHV);
// `rotated` is a workgroup-shared flag.  With a.pdyn the first *pdyn columns
// are swept and the rows from *pdyn on are zero (the caller's contract), so
// the rotations touch the first *pdyn rows only (of the work matrix and of
// V), with 2 or 3 rows per lane when that covers them.
template <int G, int RPL, bool WITHV>
__device__ __forceinline__ void jacobi_whole(const JacobiArgs& a, int s, float2* work, int& rotated)
{
    const int R = a.transpose ? a.n : a.m;
    const int P = a.transpose ? a.m : a.n;
    float2* vw = work + (long long)R * P;
    const int tid = threadIdx.x;
    load_work(a, s, work, R, P, tid, blockDim.x);
    if (WITHV) set_identity(vw, P, tid, blockDim.x);
    if (tid == 0) rotated = 0;
    __syncthreads();

    const int Ps = a.pdyn ? min(P, *a.pdyn) : P;  // columns swept
    const int Rs = a.pdyn ? min(R, Ps) : R;       // rows of the work matrix touched
    const int Pv = a.pdyn ? Ps : P;               // rows of V touched (Ps <= P <= R)
    int sweep = 0;
    bool converged = (Ps < 2);
    if (RPL > 2 && Rs <= 2 * G)
        sweeps_whole<G, (RPL > 2 ? 2 : RPL), WITHV>(a, work, vw, R, P, Ps, Rs, Pv, rotated, sweep, converged);
    else if (RPL > 3 && Rs <= 3 * G)
        sweeps_whole<G, (RPL > 3 ? 3 : RPL), WITHV>(a, work, vw, R, P, Ps, Rs, Pv, rotated, sweep, converged);
    else
        sweeps_whole<G, RPL, WITHV>(a, work, vw, R, P, Ps, Rs, Pv, rotated, sweep, converged);
    store_result<G>(a, s, work, R, P, 0, 1);
    if (WITHV) store_q(a, s, vw, P, 0, 1);
    if (a.info && tid == 0) a.info[s] = converged ? (sweep > 0 ? sweep : 1) : -sweep;
}

// largest workgroup of the whole-slice kernel: 1024 threads, 512 when each
// lane holds 32 rows per column (register budget)
constexpr int whole_max_threads(int rpl) { return rpl >= 32 ? 512 : 1024; }

template <int G, int RPL, bool LDS, bool WITHV>
__global__ __launch_bounds__(whole_max_threads(RPL)) void k_jacobi(JacobiArgs a, float2* __restrict__ gwork)
{
    extern __shared__ float2 lwork[];
    __shared__ int rotated;
    const int s = blockIdx.x;
    if ((a.gate && *a.gate == 0) || (a.count && s >= *a.count)) return;
    const int R = a.transpose ? a.n : a.m;
    const int P = a.transpose ? a.m : a.n;
    const long long per = (long long)R * P + (WITHV ? (long long)P * P : 0);
    float2* work = LDS ? lwork : gwork + (long long)s * per;
    jacobi_whole<G, RPL, WITHV>(a, s, work, rotated);
}

// Batched slices of uneven shapes (R <= 128, LDS-resident): a persistent
// grid walks (item, slice) units; each item has its own JacobiArgs.
__global__ __launch_bounds__(1024) void k_jacobi_batch(const JacobiArgs* __restrict__ items,
                                                      const SliceUnit* __restrict__ units, int nunits)
{
    extern __shared__ float2 lwork[];
    __shared__ int rotated;
    for (int u = blockIdx.x; u < nunits; u += gridDim.x) {
        const SliceUnit w = units[u];
        const JacobiArgs a = items[w.item];
        const int R = a.transpose ? a.n : a.m;
        __syncthreads();
        if (R <= 32)
            jacobi_whole<16, 2, false>(a, w.slice, lwork, rotated);
        else if (R <= 64)
            jacobi_whole<16, 4, false>(a, w.slice, lwork, rotated);
        else
            jacobi_whole<16, 8, false>(a, w.slice, lwork, rotated);
    }
}

// ---- block Jacobi: several workgroups per slice, one launch per block step ----
// The P columns are cut into nb (even) blocks of width b.  A sweep is nb-1
// block steps of the circle order over blocks; in a block step, workgroup bp
// of a slice stages its two blocks in LDS and rotates their pairs: at block
// step 0 every pair among its 2b columns (this covers the pairs inside each
// block once per sweep), later only the b x b pairs across the two blocks, so
// a sweep visits every column pair exactly once.  Per-slice rotation flags in
// three rotating buffers tell, at the start of sweep k, whether sweep k-1 had
// any rotation; a slice without is converged and its workgroups return.
struct BlockArgs {
    const int* count;  // optional device count of live slices
    float2* work;   // [nslices][P][R] column-major
    float2* v;      // [nslices][P][P] column-major (accumulated rotations) or null
    int* rot;       // [3][nslices]
    int* done;      // [nslices]: sweeps used, 0 while running
    int R, P, nslices, nb, b, sweep, bstep;
    double tol2;
};

__device__ __forceinline__ int block_cols(int beta, int b, int P)
{
    const int lo = beta * b;
    return lo >= P ? 0 : min(b, P - lo);
}

template <int G, int RPL, bool WITHV>
__global__ __launch_bounds__(512) void k_jacobi_block(BlockArgs a)
{
    extern __shared__ float2 lds[];
    __shared__ int rotated;
    const int s = blockIdx.y, bp = blockIdx.x, tid = threadIdx.x;
    if (a.count && s >= *a.count) return;
    const int ns = a.nslices;
    if (bp == 0 && a.bstep == 0 && tid == 0) a.rot[((a.sweep + 1) % 3) * ns + s] = 0;
    if (a.sweep > 0 && a.rot[((a.sweep - 1) % 3) * ns + s] == 0) {
        if (bp == 0 && tid == 0 && a.done[s] == 0) a.done[s] = a.sweep;
        return;
    }
    const int b1 = rr_col(bp, a.bstep, a.nb), b2 = rr_col(a.nb - 1 - bp, a.bstep, a.nb);
    const int c1 = block_cols(b1, a.b, a.P), c2 = block_cols(b2, a.b, a.P);
    const int R = a.R, L = c1 + c2;
    const int P = a.P;
    float2* slice = a.work + (long long)s * P * R;
    float2* vslice = a.v + (long long)s * P * P;
    float2* vl = lds + 2 * a.b * R;  // staged columns of V, P rows each
    // stage the two blocks: local columns 0..c1-1 and c1..L-1
    for (int e = tid; e < L * R; e += blockDim.x) {
        const int lj = e / R, i = e % R;
        const int j = lj < c1 ? b1 * a.b + lj : b2 * a.b + (lj - c1);
        lds[e] = slice[(long long)j * R + i];
    }
    if (WITHV)
        for (int e = tid; e < L * P; e += blockDim.x) {
            const int lj = e / P, i = e % P;
            const int j = lj < c1 ? b1 * a.b + lj : b2 * a.b + (lj - c1);
            vl[e] = vslice[(long long)j * P + i];
        }
    if (tid == 0) rotated = 0;
    __syncthreads();
    const int group = tid / G, gl = tid % G, ngroups = blockDim.x / G;
    if (a.bstep == 0) {
        const int np = L + (L & 1);
        for (int step = 0; step < np - 1; ++step) {
            for (int pair = group; pair < np / 2; pair += ngroups) {
                const int p = rr_col(pair, step, np), q = rr_col(np - 1 - pair, step, np);
                if (p >= L || q >= L) continue;
                if (jacobi_pair<G, RPL, WITHV>(lds, R, p, q, R, gl, a.tol2, vl, P, P) && gl == 0) rotated = 1;
            }
            __syncthreads();
        }
    } else {
        const int w = max(c1, c2);
        for (int step = 0; step < w; ++step) {
            for (int i = group; i < w; i += ngroups) {
                const int j = (i + step) < w ? i + step : i + step - w;
                if (i >= c1 || j >= c2) continue;
                if (jacobi_pair<G, RPL, WITHV>(lds, R, i, c1 + j, R, gl, a.tol2, vl, P, P) && gl == 0) rotated = 1;
            }
            __syncthreads();
        }
    }
    for (int e = tid; e < L * R; e += blockDim.x) {
        const int lj = e / R, i = e % R;
        const int j = lj < c1 ? b1 * a.b + lj : b2 * a.b + (lj - c1);
        slice[(long long)j * R + i] = lds[e];
    }
    if (WITHV)
        for (int e = tid; e < L * P; e += blockDim.x) {
            const int lj = e / P, i = e % P;
            const int j = lj < c1 ? b1 * a.b + lj : b2 * a.b + (lj - c1);
            vslice[(long long)j * P + i] = vl[e];
        }
    if (rotated && tid == 0) atomicOr(&a.rot[(a.sweep % 3) * ns + s], 1);
}

__global__ __launch_bounds__(256) void k_jacobi_block_init(JacobiArgs a, float2* work, float2* v, int* rot, int* done)
{
    const int s = blockIdx.y;
    if (a.count && s >= *a.count) return;
    const int R = a.transpose ? a.n : a.m;
    const int P = a.transpose ? a.m : a.n;
    const int w = blockIdx.x * blockDim.x + threadIdx.x, nw = gridDim.x * blockDim.x;
    load_work(a, s, work + (long long)s * R * P, R, P, w, nw);
    if (v) set_identity(v + (long long)s * P * P, P, w, nw);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        rot[s] = 0;
        rot[a.nslices + s] = 0;
        rot[2 * a.nslices + s] = 0;
        done[s] = 0;
    }
}

template <int G>
__global__ __launch_bounds__(256) void k_jacobi_block_finish(JacobiArgs a, const float2* work, const float2* v,
                                                             const int* rot, const int* done, int sweeps_run,
                                                             int ring = 3)
{
    const int s = blockIdx.y;
    if (a.count && s >= *a.count) return;
    const int R = a.transpose ? a.n : a.m;
    const int P = a.transpose ? a.m : a.n;
    store_result<G>(a, s, work + (long long)s * R * P, R, P, blockIdx.x, gridDim.x);
    if (v) store_q(a, s, v + (long long)s * P * P, P, blockIdx.x, gridDim.x);
    if (a.info && blockIdx.x == 0 && threadIdx.x == 0) {
        int d = done[s];
        if (d == 0 && sweeps_run > 0 && rot[((sweeps_run - 1) % ring) * a.nslices + s] == 0) d = sweeps_run;
        a.info[s] = d > 0 ? d : -sweeps_run;
    }
}

// ---- block sweep: one launch per sweep, column pairs held in registers ----
// The same block circle order as k_jacobi_block, for slices without V.  An
// item is one block pair (b1, b2) at one block step of one slice; items are
// numbered step-major (step, slice, pair) and workgroups take them in that
// order from a per-sweep ticket counter.  An item at step t waits for the two
// items of step t-1 that last wrote its blocks, and those hold smaller
// tickets, so they were taken by workgroups that are already running: the
// waits always end, whatever the number of workgroups resident at once.
//
// In an item the b groups of G lanes (b = blockDim / G, also the block width)
// hold columns in registers (RPL rows per lane, R <= G RPL).  Cross pairs:
// group g keeps column g of block b1 and meets the b2 columns in turn, the
// b2 columns passing one group down through LDS each round (b rounds).  At
// block step 0 the pairs inside each block come first: groups [0, b/2) take
// block b1 and [b/2, b) block b2, two columns per group, in the circle order
// over b positions (b - 1 rounds; the columns move one position per round,
// through LDS, one block at a time).  Completion is published with an
// agent-scope release after the columns are stored; the waiter acquires
// before it loads them (the L2s of the XCDs are not coherent).
struct SweepArgs {
    float2* work;           // [nslices][P][R] column-major
    int* rot;               // [3][nslices]
    int* done;              // [nslices]
    int* flags;             // [nslices][nb - 1][nb / 2] completion stamps (sweep + 1)
    unsigned int* tickets;  // [4] ticket counters: sweep k takes tickets from k mod 4
    int* err;               // set when a wait hit its spin limit (never expected)
    const int* count;       // optional device count of live slices (<= nslices)
    int R, P, nslices, nb, b, sweep, nitems;
    double tol2;
    int nsw;                // Gram sweep: sweeps per launch (sweep .. sweep + nsw - 1; nitems covers them)
};

// Gram sweep: sweeps per launch.  Its rotation flags have one row per sweep
// (max_sweeps rows, zeroed once), so no row is reused within a call.
constexpr int kGramSweepsPerLaunch = 3;

// position of block beta in step t of the circle order over nb blocks
__device__ __forceinline__ int rr_pos(int beta, int t, int nb)
{
    if (beta == 0) return 0;
    int p = beta - 1 - t;
    while (p < 0) p += nb - 1;
    return p + 1;
}

// rotation of the pair (x, y) held by the G lanes of a group: the same
// arithmetic as jacobi_pair on register-resident columns
template <int G, int RPL>
__device__ __forceinline__ bool rotate_regs(float2 (&x)[RPL], float2 (&y)[RPL], double tol2)
{
    float pa = 0.f, pb = 0.f, pr = 0.f, pi = 0.f;
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
        pa = fmaf(x[t].x, x[t].x, fmaf(x[t].y, x[t].y, pa));
        pb = fmaf(y[t].x, y[t].x, fmaf(y[t].y, y[t].y, pb));
        pr = fmaf(x[t].x, y[t].x, fmaf(x[t].y, y[t].y, pr));
        pi = fmaf(x[t].x, y[t].y, fmaf(-x[t].y, y[t].x, pi));
    }
    const double al = group_sum<G>((double)pa);
    const double be = group_sum<G>((double)pb);
    const double gr = group_sum<G>((double)pr);
    const double gi = group_sum<G>((double)pi);
    const double g2 = gr * gr + gi * gi;
    if (!(g2 > 0.0 && g2 > tol2 * al * be)) return false;
    const double ig = rsqrt_f64(g2);
    const double zeta = 0.5 * (be - al) * ig;
    const double z2 = fma(zeta, zeta, 1.0);
    const double t = copysign(rcp_f64(fabs(zeta) + z2 * rsqrt_f64(z2)), zeta);
    const double c = rsqrt_f64(fma(t, t, 1.0));
    const double sn = c * t;
    const float cf = (float)c;
    const float sr = (float)(sn * gr * ig), si = (float)(sn * gi * ig);
#pragma unroll
    for (int t2 = 0; t2 < RPL; ++t2) {
        const float2 xv = x[t2], yv = y[t2];
        x[t2] = make_float2(cf * xv.x - (sr * yv.x + si * yv.y), cf * xv.y - (sr * yv.y - si * yv.x));
        y[t2] = make_float2((sr * xv.x - si * xv.y) + cf * yv.x, (sr * xv.y + si * xv.x) + cf * yv.y);
    }
    return true;
}

// Column i/o of the block sweep.  Lane gl of a group holds, in its slot t,
// row rowof(gl, t) = 2 (gl + G (t / 2)) + (t % 2) of a column: two adjacent
// rows per pair of slots, so every access moves 16 bytes and a group's
// accesses are contiguous.  The same mapping serves LDS and global memory.
// The slice's columns in global memory, which other workgroups (on any XCD)
// wrote in this launch, move with buffer loads and stores at device scope
// (SC1): such accesses are coherent across the XCDs' L2 caches by their
// scope, with no cache-wide writeback or invalidation.
typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v2i __attribute__((ext_vector_type(2)));
constexpr int kDeviceScope = 16;  // cache policy: SC1 (device scope)

template <int G>
__device__ __forceinline__ int rowof(int gl, int t) { return 2 * (gl + G * (t >> 1)) + (t & 1); }

template <int G, int RPL>
__device__ __forceinline__ void col_load(float2 (&v)[RPL], const float2* src, int R, int gl, bool live)
{
#pragma unroll
    for (int t = 0; t < RPL; t += 2) {
        const int r = rowof<G>(gl, t);
        if (live && r + 1 < R) {
            const float4 q = *reinterpret_cast<const float4*>(src + r);
            v[t] = make_float2(q.x, q.y);
            v[t + 1] = make_float2(q.z, q.w);
        } else {
            v[t] = (live && r < R) ? src[r] : make_float2(0.f, 0.f);
            v[t + 1] = make_float2(0.f, 0.f);
        }
    }
}

template <int G, int RPL>
__device__ __forceinline__ void col_store(const float2 (&v)[RPL], float2* dst, int R, int gl)
{
#pragma unroll
    for (int t = 0; t < RPL; t += 2) {
        const int r = rowof<G>(gl, t);
        if (r + 1 < R)
            *reinterpret_cast<float4*>(dst + r) = make_float4(v[t].x, v[t].y, v[t + 1].x, v[t + 1].y);
        else if (r < R)
            dst[r] = v[t];
    }
}

// raw buffer access (the LLVM intrinsics; the resource is one slice, uniform
// across the workgroup)
typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v2f __attribute__((ext_vector_type(2)));
__device__ v4f raw_buffer_load_v4(v4i rsrc, int voffset, int soffset, int aux) __asm("llvm.amdgcn.raw.buffer.load.v4f32");
__device__ v2f raw_buffer_load_v2(v4i rsrc, int voffset, int soffset, int aux) __asm("llvm.amdgcn.raw.buffer.load.v2f32");
__device__ void raw_buffer_store_v4(v4i data, v4i rsrc, int voffset, int soffset,
                                    int aux) __asm("llvm.amdgcn.raw.buffer.store.v4i32");
__device__ void raw_buffer_store_v2(v2i data, v4i rsrc, int voffset, int soffset,
                                    int aux) __asm("llvm.amdgcn.raw.buffer.store.v2i32");

// buffer resource over `bytes` bytes at p (stride 0: the range is in bytes;
// accesses past it read zeros and write nothing)
__device__ __forceinline__ v4i slice_rsrc(const void* p, unsigned int bytes)
{
    const unsigned long long a = reinterpret_cast<unsigned long long>(p);
    v4i r;
    r.x = (int)(unsigned int)(a & 0xffffffffu);
    r.y = (int)(unsigned int)((a >> 32) & 0xffffu);
    r.z = (int)bytes;
    r.w = 0x00020000;
    return r;
}

// column `col` (R rows, column-major, byte offset col * 8 R in the slice
// resource rs of `limit` bytes); live = false reads zeros
template <int G, int RPL>
__device__ __forceinline__ void col_load_shared(float2 (&v)[RPL], v4i rs, int limit, int col, int R, int gl, bool live)
{
    const int base = col * R * 8;
#pragma unroll
    for (int t = 0; t < RPL; t += 2) {
        const int r = rowof<G>(gl, t);
        const v4f q = raw_buffer_load_v4(rs, (live && r + 1 < R) ? base + r * 8 : limit, 0, kDeviceScope);
        v[t] = make_float2(q.x, q.y);
        v[t + 1] = make_float2(q.z, q.w);
        if ((R & 1) && live && r == R - 1) {  // the last row of an odd height
            const v2f q2 = raw_buffer_load_v2(rs, base + r * 8, 0, kDeviceScope);
            v[t] = make_float2(q2.x, q2.y);
        }
    }
}

template <int G, int RPL>
__device__ __forceinline__ void col_store_shared(const float2 (&v)[RPL], v4i rs, int col, int R, int gl)
{
    const int base = col * R * 8;
#pragma unroll
    for (int t = 0; t < RPL; t += 2) {
        const int r = rowof<G>(gl, t);
        if (r + 1 < R) {
            v4i q;
            q.x = __builtin_bit_cast(int, v[t].x);
            q.y = __builtin_bit_cast(int, v[t].y);
            q.z = __builtin_bit_cast(int, v[t + 1].x);
            q.w = __builtin_bit_cast(int, v[t + 1].y);
            raw_buffer_store_v4(q, rs, base + r * 8, 0, kDeviceScope);
        } else if (r < R) {
            v2i q;
            q.x = __builtin_bit_cast(int, v[t].x);
            q.y = __builtin_bit_cast(int, v[t].y);
            raw_buffer_store_v2(q, rs, base + r * 8, 0, kDeviceScope);
        }
    }
}

// spin (bounded) until *f >= want; one lane
__device__ __forceinline__ void wait_stamp(const int* f, int want, int* err)
{
    for (long long it = 0; it < (1LL << 26); ++it) {
        if (__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= want) return;
        __builtin_amdgcn_s_sleep(2);
    }
    atomicExch(err, 1);
}

template <int G, int RPL, int MAXT>
__global__ __launch_bounds__(MAXT) void k_jacobi_sweep(SweepArgs a)
{
    extern __shared__ float2 xch[];  // b columns of R rows (stride ldr)
    __shared__ int sh_item, sh_rot;
    __shared__ int sh_id[64], sh_yid[64];
    const int tid = threadIdx.x, g = tid / G, gl = tid % G, b = a.b, R = a.R;
    const int ldr = (R + 1) & ~1;  // LDS column stride (even: 16-byte aligned columns)
    const int npairs = a.nb / 2, per_step = a.nslices * npairs, half = b / 2;
    const int live_slices = a.count ? min(*a.count, a.nslices) : a.nslices;
    if (live_slices <= 0) return;
    const int ns = a.nslices, stamp = a.sweep + 1;
    if (a.sweep > 0) {  // every live slice converged: the launch has nothing to do
        int busy = 0;
        for (int q = tid; q < live_slices; q += blockDim.x) busy |= a.rot[((a.sweep - 1) % 3) * ns + q];
        if (!__syncthreads_or(busy)) {
            // the bookkeeping the slices' first items would have done
            if (blockIdx.x == 0)
                for (int q = tid; q < live_slices; q += blockDim.x) {
                    a.rot[((a.sweep + 1) % 3) * ns + q] = 0;
                    if (a.done[q] == 0) a.done[q] = a.sweep;
                }
            return;
        }
    }
    float2 x[RPL], y[RPL];
    for (;;) {
        if (tid == 0) {
            const unsigned int tk = atomicAdd(a.tickets + (a.sweep & 3), 1u);
            // the counter of sweep + 2 was last used by sweep - 2, which has ended
            if (tk == 0) a.tickets[(a.sweep + 2) & 3] = 0;
            sh_item = (int)tk;
            sh_rot = 0;
        }
        __syncthreads();
        const int item = sh_item;
        if (item >= a.nitems) return;
        const int step = item / per_step, rem = item - step * per_step, s = rem / npairs, bp = rem - s * npairs;
        if (s >= live_slices) {
            __syncthreads();
            continue;
        }
        // the flag of the next sweep is cleared every sweep, converged or not
        if (step == 0 && bp == 0 && tid == 0) a.rot[((a.sweep + 1) % 3) * ns + s] = 0;
        if (a.sweep > 0 && a.rot[((a.sweep - 1) % 3) * ns + s] == 0) {  // converged in the previous sweep
            if (step == 0 && bp == 0 && tid == 0 && a.done[s] == 0) a.done[s] = a.sweep;
            __syncthreads();
            continue;
        }
        const int b1 = rr_col(bp, step, a.nb), b2 = rr_col(a.nb - 1 - bp, step, a.nb);
        const int c1 = block_cols(b1, b, a.P), c2 = block_cols(b2, b, a.P);
        int* fl = a.flags + (long long)s * (a.nb - 1) * npairs;
        if (step > 0 && tid == 0) {
            const int q1 = rr_pos(b1, step - 1, a.nb), q2 = rr_pos(b2, step - 1, a.nb);
            wait_stamp(fl + (step - 1) * npairs + min(q1, a.nb - 1 - q1), stamp, a.err);
            wait_stamp(fl + (step - 1) * npairs + min(q2, a.nb - 1 - q2), stamp, a.err);
        }
        // the column loads below are issued after the stamps were seen (the
        // barrier) and read at device scope
        __syncthreads();
        // the slice as one buffer resource; columns by index
        const int limit = a.P * R * (int)sizeof(float2);
        const v4i rs = slice_rsrc(a.work + (long long)s * a.P * R, (unsigned int)limit);
        const int col1 = b1 * b, col2 = b2 * b;
        bool rotated = false;
        int xid = g, yid = g;  // local column ids held in x (block b1) and y (block b2)
        if (step == 0) {
            // pairs inside each block: group (blk, u) holds positions u and
            // b - 1 - u of its block; position p holds local column cid[p]
            const int blk = g < half ? 0 : 1, u = g - blk * half, cb = blk ? c2 : c1;
            const int cbase = blk ? col2 : col1;
            int px = u, py = b - 1 - u, cx = px, cy = py;
            col_load_shared<G, RPL>(x, rs, limit, cbase + cx, R, gl, cx < cb);
            col_load_shared<G, RPL>(y, rs, limit, cbase + cy, R, gl, cy < cb);
            for (int r = 0; r < b - 1; ++r) {
                if (cx < cb && cy < cb) rotated |= rotate_regs<G, RPL>(x, y, a.tol2);
                // every position but 0 moves down one (1 wraps to b - 1), one block at a time
                const int nx = px == 0 ? 0 : (px == 1 ? b - 1 : px - 1);
                const int ny = py == 1 ? b - 1 : py - 1;
                for (int k = 0; k < 2; ++k) {
                    if (blk == k) {
                        col_store<G, RPL>(x, xch + (long long)nx * ldr, R, gl);
                        col_store<G, RPL>(y, xch + (long long)ny * ldr, R, gl);
                        if (gl == 0) {
                            sh_id[nx] = cx;
                            sh_id[ny] = cy;
                        }
                    }
                    __syncthreads();
                    if (blk == k) {
                        col_load<G, RPL>(x, xch + (long long)px * ldr, R, gl, true);
                        col_load<G, RPL>(y, xch + (long long)py * ldr, R, gl, true);
                        cx = sh_id[px];
                        cy = sh_id[py];
                    }
                    __syncthreads();
                }
            }
            // to the cross layout (one b1 and one b2 column per group): group
            // u of b1 swaps its second column for the first of group u of b2
            if (blk == 0) {
                col_store<G, RPL>(y, xch + (long long)u * ldr, R, gl);
                if (gl == 0) sh_id[u] = cy;
            } else {
                col_store<G, RPL>(x, xch + (long long)(half + u) * ldr, R, gl);
                if (gl == 0) sh_id[half + u] = cx;
            }
            __syncthreads();
            if (blk == 0) {
                col_load<G, RPL>(y, xch + (long long)(half + u) * ldr, R, gl, true);
                xid = cx;
                yid = sh_id[half + u];
            } else {
                col_load<G, RPL>(x, xch + (long long)u * ldr, R, gl, true);
                xid = sh_id[u];
                yid = cy;
            }
            __syncthreads();
        } else {
            col_load_shared<G, RPL>(x, rs, limit, col1 + g, R, gl, g < c1);
            col_load_shared<G, RPL>(y, rs, limit, col2 + g, R, gl, g < c2);
        }
        // cross pairs: the b2 columns pass one group down per round, so group
        // g meets in round r the column group (g + r) mod b started with
        if (gl == 0) sh_yid[g] = yid;
        __syncthreads();
        for (int r = 0; r < b; ++r) {
            yid = sh_yid[g + r < b ? g + r : g + r - b];
            if (xid < c1 && yid < c2) rotated |= rotate_regs<G, RPL>(x, y, a.tol2);
            if (r == b - 1) break;
            col_store<G, RPL>(y, xch + (long long)g * ldr, R, gl);
            __syncthreads();
            col_load<G, RPL>(y, xch + (long long)(g + 1 < b ? g + 1 : 0) * ldr, R, gl, true);
            __syncthreads();
        }
        if (xid < c1) col_store_shared<G, RPL>(x, rs, col1 + xid, R, gl);
        if (yid < c2) col_store_shared<G, RPL>(y, rs, col2 + yid, R, gl);
        if (rotated && gl == 0) sh_rot = 1;
        // every wave's device-scope stores acknowledged before the stamp is written
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (tid == 0) {
            if (sh_rot) atomicOr(&a.rot[(a.sweep % 3) * ns + s], 1);
            __hip_atomic_store(fl + step * npairs + bp, stamp, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// ---- Gram block sweep: block pairs through MFMA Gram matrices ----
// The item order and stamps of k_jacobi_sweep (here three sweeps per launch,
// with one row of rotation flags per sweep), with blocks of b = 8 NT columns,
// so that an item holds W = 16 NT columns X (R x W).  An item
//  1. forms G = X^* X with FP32 MFMA (16x16x4) over groups of 8 rows, two
//     accumulator sets per wave (one per row of a row pair), the partial sums
//     added in FP64 in LDS;
//  2. takes the scalar sweep's pair rotations (all W(W-1)/2 pairs in the
//     circle order at block step 0, the b x b cross pairs later) on G instead
//     of on the columns: a rotation J of positions (p, q) chosen from G_pp,
//     G_qq and G_pq turns G into J^* G J and the accumulated V into V J, in
//     FP64 (J^* G J is the Gram matrix of X J, so each decision is the one the
//     column rotations would take up to the rounding of G);
//  3. when anything rotated, replaces X by X V with FP32 MFMA (V rounded to
//     FP32), rows in tiles of 16.
// The columns are read from memory once when they fit in LDS (copied there by
// step 1, read back by step 3), else twice; loads run one batch ahead.
// The R-long column work of the W(W-1)/2 (or b^2) rotations becomes two
// R x W x W complex products on the matrix cores; the dependent chain of an
// item is W - 1 (or b) steps on W x W matrices in LDS.
template <int NT>
struct GramSmem {
    static constexpr int W = 16 * NT, B = 8 * NT;
    static constexpr int NREG = NT == 1 ? 4 : 2;  // partial-sum regions (one per wave, or per wave pair)
    double2 g[2][W][W + 1];  // G, double-buffered across the steps of the rotation chain
    union {
        double part[NREG][2][W][W];  // [region][re, T][i][j]: partial sums of the waves
        double2 v[W][W + 1];         // accumulated rotations V
    } u;
    double rc[B], rsr[B], rsi[B];  // rotations of the current step (two-pass chain)
    int item;
};

// the rotation of the scalar sweep from alpha = ||x||^2, beta = ||y||^2 and
// gamma = x^* y (FP64): x' = c x - s conj(e) y, y' = s e x + c y, e =
// gamma/|gamma|; (sr, si) = s e.  False (and the identity) below the threshold.
__device__ __forceinline__ bool pair_rotation(double al, double be, double gr, double gi, double tol2, double& c,
                                              double& sr, double& si)
{
    c = 1.0;
    sr = 0.0;
    si = 0.0;
    const double g2 = gr * gr + gi * gi;
    if (!(g2 > 0.0 && g2 > tol2 * al * be)) return false;
    // e = gamma / |gamma| and c = 1/sqrt(1 + t^2) to FP64 accuracy keep J
    // unitary to FP64 rounding for any t; t itself (which only sets how
    // closely gamma is annihilated) comes from the FP32 hardware estimates
    const double ig = rsqrt_f64(g2);
    const float zeta = (float)(0.5 * (be - al) * ig);
    const float az = fabsf(zeta);
    const float tf = az < 1e18f ? copysignf(__builtin_amdgcn_rcpf(az + __builtin_amdgcn_sqrtf(fmaf(az, az, 1.0f))), zeta)
                                : 0.5f * __builtin_amdgcn_rcpf(zeta);
    // an angle that underflows (norms some 10^12 apart) is no rotation: the
    // pair counts as converged rather than as rotated without change
    if (tf == 0.0f) return false;
    const double t = (double)tf;
    c = rsqrt_f64(fma(t, t, 1.0));
    const double sn = c * t;
    sr = sn * gr * ig;
    si = sn * gi * ig;
    return true;
}

// positions of pair k at inner step st: the circle order over all W positions
// at block step 0, else position k of the first block against position
// (k + st) mod b of the second
template <int W>
__device__ __forceinline__ void gram_pair(bool all, int k, int st, int& p, int& q)
{
    constexpr int B = W / 2;
    if (all) {
        p = rr_col(k, st, W);
        q = rr_col(W - 1 - k, st, W);
    } else {
        p = k;
        q = B + (k + st < B ? k + st : k + st - B);
    }
}

// the bits of a float taken by value: a bit cast applied directly to an
// element of an ext_vector_type value reads element 0 with this compiler
__device__ __forceinline__ int f32_bits(float f) { return __builtin_bit_cast(int, f); }

// rows r and r + 1 of a column (16 bytes), zeros where absent
__device__ __forceinline__ v4f gram_rows2(v4i rs, int limit, int base, int r, int R, bool live)
{
    if (live && r + 1 < R) return raw_buffer_load_v4(rs, base + r * 8, 0, kDeviceScope);
    v4f z = {0.f, 0.f, 0.f, 0.f};
    if (live && r < R) {
        const v2f q = raw_buffer_load_v2(rs, base + r * 8, 0, kDeviceScope);
        z.x = q.x;
        z.y = q.y;
    }
    return z;
}

// column stride (float2) of the item's columns staged in LDS: even, and 16 mod
// 32, so that the two columns a half-wave reads in the update fall in
// different halves of the banks
__host__ __device__ constexpr int gram_ldx(int R) { return R + ((16 - R) % 32 + 32) % 32; }

// whether the W columns of an item are staged in LDS (read once from memory)
constexpr bool gram_stage_fits(int nt, int R)
{
    return (size_t)gram_ldx(R) * 16 * nt * sizeof(float2) <= (nt == 1 ? 64 : 90) * 1024;
}

template <int NT, bool STAGE>
__global__ __launch_bounds__(256) void k_gram_sweep(SweepArgs a)
{
    constexpr int W = 16 * NT, B = 8 * NT;
    constexpr int PF = NT == 1 ? 8 : 4;  // row groups per load batch
    extern __shared__ __align__(16) char gram_raw[];
    GramSmem<NT>& sm = *reinterpret_cast<GramSmem<NT>*>(gram_raw);
    float2* xs = reinterpret_cast<float2*>(gram_raw + ((sizeof(GramSmem<NT>) + 15) & ~(size_t)15));
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int j16 = lane & 15, k4 = lane >> 4;
    const int R = a.R, ldx = gram_ldx(R);
    const int npairs = a.nb / 2, per_step = a.nslices * npairs;
    const int live_slices = a.count ? min(*a.count, a.nslices) : a.nslices;
    if (live_slices <= 0) return;
    // The launch covers sweeps a.sweep .. a.sweep + nsw - 1, items numbered
    // sweep-major (sweep, step, slice, pair).  A slice whose previous sweep
    // (the last of the previous launch) rotated nothing is converged and its
    // items return; within a launch every sweep runs (one that rotates
    // nothing stores nothing), and the next launch sees the last one's flag.
    // Rotation flags: rot[sweep * ns + slice].
    const int ns = a.nslices, per_sweep = (a.nb - 1) * per_step, launch = a.sweep / max(a.nsw, 1);
    if (a.sweep > 0) {  // every live slice converged: the launch has nothing to do
        int busy = 0;
        for (int q = tid; q < live_slices; q += blockDim.x) busy |= a.rot[(a.sweep - 1) * ns + q];
        if (!__syncthreads_or(busy)) {
            if (blockIdx.x == 0)
                for (int q = tid; q < live_slices; q += blockDim.x)
                    if (a.done[q] == 0) a.done[q] = a.sweep;
            return;
        }
    }
    for (;;) {
        if (tid == 0) {
            const unsigned int tk = atomicAdd(a.tickets + (launch & 3), 1u);
            // the counter of launch + 2 was last used by launch - 2, which has ended
            if (tk == 0) a.tickets[(launch + 2) & 3] = 0;
            sm.item = (int)tk;
        }
        __syncthreads();
        const int item = sm.item;
        if (item >= a.nitems) return;
        const int ls = item / per_sweep, irem = item - ls * per_sweep;
        const int sweep = a.sweep + ls, stamp = sweep + 1;
        const int step = irem / per_step, rem = irem - step * per_step, s = rem / npairs, bp = rem - s * npairs;
        if (s >= live_slices) {
            __syncthreads();
            continue;
        }
        if (a.sweep > 0 && a.rot[(a.sweep - 1) * ns + s] == 0) {  // converged before this launch
            if (ls == 0 && step == 0 && bp == 0 && tid == 0 && a.done[s] == 0) a.done[s] = a.sweep;
            __syncthreads();
            continue;
        }
        const int b1 = rr_col(bp, step, a.nb), b2 = rr_col(a.nb - 1 - bp, step, a.nb);
        const int c1 = block_cols(b1, B, a.P), c2 = block_cols(b2, B, a.P);
        int* fl = a.flags + (long long)s * (a.nb - 1) * npairs;
        // wait for the items that last wrote the two blocks: at the previous
        // step, or at the last step of the previous sweep when it ran in this
        // launch (smaller tickets: workgroups already running)
        if (tid == 0 && (step > 0 || ls > 0)) {
            const int ps = step > 0 ? step - 1 : a.nb - 2, want = step > 0 ? stamp : stamp - 1;
            const int q1 = rr_pos(b1, ps, a.nb), q2 = rr_pos(b2, ps, a.nb);
            wait_stamp(fl + ps * npairs + min(q1, a.nb - 1 - q1), want, a.err);
            wait_stamp(fl + ps * npairs + min(q2, a.nb - 1 - q2), want, a.err);
        }
        __syncthreads();
        const int limit = a.P * R * (int)sizeof(float2);
        const v4i rs = slice_rsrc(a.work + (long long)s * a.P * R, (unsigned int)limit);
        // local column i of the item: block b1 for i < b, else block b2
        auto col_base = [&](int i) { return (i < B ? b1 * B + i : b2 * B + i - B) * R * 8; };
        auto col_live = [&](int i) { return i < B ? i < c1 : i - B < c2; };

        // 1. Gram matrix: lane (j16, k4) feeds rows 8t + 2 k4 (set 0) and + 1
        // (set 1) of column 16 g + j16 as both MFMA operands
        {
            v4f accR[NT][NT][2], accT[NT][NT][2];
#pragma unroll
            for (int ti = 0; ti < NT; ++ti)
#pragma unroll
                for (int tj = 0; tj < NT; ++tj)
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        accR[ti][tj][h] = v4f{0.f, 0.f, 0.f, 0.f};
                        accT[ti][tj][h] = v4f{0.f, 0.f, 0.f, 0.f};
                    }
            int base[NT];
            bool live[NT];
#pragma unroll
            for (int g = 0; g < NT; ++g) {
                base[g] = col_base(16 * g + j16);
                live[g] = col_live(16 * g + j16);
            }
            // wave wv takes the row groups wv + 4 i, i < nw, in batches of PF:
            // 16 columns load a whole batch at once (8 groups, every group of
            // a 256-row slice), 32 columns issue the loads one batch ahead
            const int ngroups = (R + 7) / 8;
            const int nw = wv < ngroups ? (ngroups - wv + 3) / 4 : 0;
            auto load_batch = [&](int i0, v4f (&dst)[PF][NT]) {
#pragma unroll
                for (int b = 0; b < PF; ++b) {
                    const int r = 8 * (wv + 4 * (i0 + b)) + 2 * k4;
#pragma unroll
                    for (int g = 0; g < NT; ++g) dst[b][g] = gram_rows2(rs, limit, base[g], r, R, live[g]);
                }
            };
            auto use_batch = [&](int i0, const v4f (&cur)[PF][NT]) {
#pragma unroll
                for (int b = 0; b < PF; ++b) {
                    const v4f* x = cur[b];
                    if (STAGE) {
                        const int r = 8 * (wv + 4 * (i0 + b)) + 2 * k4;
                        if (r < R)
#pragma unroll
                            for (int g = 0; g < NT; ++g)
                                *reinterpret_cast<v4f*>(xs + (16 * g + j16) * ldx + r) = x[g];
                    }
#pragma unroll
                    for (int ti = 0; ti < NT; ++ti)
#pragma unroll
                        for (int tj = 0; tj < NT; ++tj) {
                            v4f& r0 = accR[ti][tj][0];
                            v4f& r1 = accR[ti][tj][1];
                            r0 = __builtin_amdgcn_mfma_f32_16x16x4f32(x[ti].x, x[tj].x, r0, 0, 0, 0);
                            r0 = __builtin_amdgcn_mfma_f32_16x16x4f32(x[ti].y, x[tj].y, r0, 0, 0, 0);
                            accT[ti][tj][0] =
                                __builtin_amdgcn_mfma_f32_16x16x4f32(x[ti].x, x[tj].y, accT[ti][tj][0], 0, 0, 0);
                            r1 = __builtin_amdgcn_mfma_f32_16x16x4f32(x[ti].z, x[tj].z, r1, 0, 0, 0);
                            r1 = __builtin_amdgcn_mfma_f32_16x16x4f32(x[ti].w, x[tj].w, r1, 0, 0, 0);
                            accT[ti][tj][1] =
                                __builtin_amdgcn_mfma_f32_16x16x4f32(x[ti].z, x[tj].w, accT[ti][tj][1], 0, 0, 0);
                        }
                }
            };
            if constexpr (NT == 1) {
                for (int i0 = 0; i0 < nw; i0 += PF) {
                    v4f cur[PF][NT];
                    load_batch(i0, cur);
                    use_batch(i0, cur);
                }
            } else {
                v4f cur[PF][NT], nxt[PF][NT];
                if (nw > 0) load_batch(0, cur);
                for (int i0 = 0; i0 < nw; i0 += PF) {
                    if (i0 + PF < nw) load_batch(i0 + PF, nxt);
                    use_batch(i0, cur);
#pragma unroll
                    for (int b = 0; b < PF; ++b)
#pragma unroll
                        for (int g = 0; g < NT; ++g) cur[b][g] = nxt[b][g];
                }
            }
            // partial sums: one region per wave (16 columns), or waves 0, 1
            // store and waves 2, 3 add theirs (32 columns); fixed order
            constexpr int NREG = GramSmem<NT>::NREG;
            for (int pass = 0; pass < 4 / NREG; ++pass) {
                if (wv / NREG == pass) {
                    double (*pr)[W] = sm.u.part[wv % NREG][0];
                    double (*pt)[W] = sm.u.part[wv % NREG][1];
#pragma unroll
                    for (int ti = 0; ti < NT; ++ti)
#pragma unroll
                        for (int tj = 0; tj < NT; ++tj)
#pragma unroll
                            for (int e = 0; e < 4; ++e) {
                                const int i = 16 * ti + 4 * k4 + e, jj = 16 * tj + j16;
                                const double dr = (double)accR[ti][tj][0][e] + (double)accR[ti][tj][1][e];
                                const double dt = (double)accT[ti][tj][0][e] + (double)accT[ti][tj][1][e];
                                if (pass == 0) {
                                    pr[i][jj] = dr;
                                    pt[i][jj] = dt;
                                } else {
                                    pr[i][jj] += dr;
                                    pt[i][jj] += dt;
                                }
                            }
                }
                __syncthreads();
            }
        }
        // G = (Xr^T Xr + Xi^T Xi) + i (T - T^T), T = Xr^T Xi; the real part
        // symmetrised so that G is exactly Hermitian
        for (int e = tid; e < W * W; e += 256) {
            const int i = e / W, jj = e - i * W;
            double rij = 0.0, rji = 0.0, tij = 0.0, tji = 0.0;
#pragma unroll
            for (int q = 0; q < GramSmem<NT>::NREG; ++q) {
                rij += sm.u.part[q][0][i][jj];
                rji += sm.u.part[q][0][jj][i];
                tij += sm.u.part[q][1][i][jj];
                tji += sm.u.part[q][1][jj][i];
            }
            sm.g[0][i][jj] = make_double2(0.5 * (rij + rji), tij - tji);
        }
        __syncthreads();
        const bool all = step == 0;
        int need = 0;
        for (int e = tid; e < W * W; e += 256) {
            const int i = e / W, jj = e - i * W;
            sm.u.v[i][jj] = make_double2(i == jj ? 1.0 : 0.0, 0.0);
            if (i < jj && (all || (i < B && jj >= B))) {
                const double2 g = sm.g[0][i][jj];
                const double g2 = g.x * g.x + g.y * g.y;
                need |= (g2 > 0.0 && g2 > a.tol2 * sm.g[0][i][i].x * sm.g[0][jj][jj].x) ? 1 : 0;
            }
        }
        // 2. the pair rotations on G (none when no visited pair is above the
        // threshold: then none would ever rotate)
        bool rotated = false;
        if (__syncthreads_or(need)) {
            const int nsteps = all ? W - 1 : B;
            if constexpr (NT == 1) {
                // 16 columns, two passes per step over all threads: thread k =
                // tid mod b takes pair k's rotation; G J into the second
                // buffer and V J in place, then J^* (G J) back (rows p, q)
                const int k = tid % B;
                double2 (*ga)[W + 1] = sm.g[0];
                double2 (*gb)[W + 1] = sm.g[1];
                for (int st = 0; st < nsteps; ++st) {
                    int p, q;
                    gram_pair<W>(all, k, st, p, q);
                    double c, sr, si;
                    const bool r = pair_rotation(ga[p][p].x, ga[q][q].x, ga[p][q].x, ga[p][q].y, a.tol2, c, sr, si);
                    if (tid < B) {
                        sm.rc[k] = c;
                        sm.rsr[k] = sr;
                        sm.rsi[k] = si;
                    }
                    for (int u = tid / B; u < 2 * W; u += 256 / B) {
                        double2* row = u < W ? &ga[u][0] : &sm.u.v[u - W][0];
                        double2* out = u < W ? &gb[u][0] : row;
                        const double2 x = row[p], y = row[q];
                        out[p] = make_double2(c * x.x - (sr * y.x + si * y.y), c * x.y - (sr * y.y - si * y.x));
                        out[q] = make_double2((sr * x.x - si * x.y) + c * y.x, (sr * x.y + si * x.x) + c * y.y);
                    }
                    if (!__syncthreads_or(r ? 1 : 0)) continue;  // no rotation: G (ga) unchanged
                    rotated = true;
                    for (int u = tid; u < B * W; u += 256) {
                        const int kk = u / W, cc = u - kk * W;
                        int pp, qq;
                        gram_pair<W>(all, kk, st, pp, qq);
                        const double c2 = sm.rc[kk], sr2 = sm.rsr[kk], si2 = sm.rsi[kk];
                        const double2 x = gb[pp][cc], y = gb[qq][cc];
                        ga[pp][cc] = make_double2(c2 * x.x - (sr2 * y.x - si2 * y.y), c2 * x.y - (sr2 * y.y + si2 * y.x));
                        ga[qq][cc] = make_double2((sr2 * x.x + si2 * x.y) + c2 * y.x, (sr2 * x.y - si2 * x.x) + c2 * y.y);
                    }
                    __syncthreads();
                }
            } else {
                // 32 columns, one pass per step: thread (kr, kc) owns the 2 x 2
                // block of G in the rows of pair kr and the columns of pair kc,
                // and rows 2 kr, 2 kr + 1 of V in the columns of pair kc; it
                // takes both rotations itself, so that a step reads G from one
                // buffer, writes the other and ends with one barrier: block <-
                // J_kr^* block J_kc, V <- V J_kc, with J_k = [c, z; -conj(z), c]
                // on positions (p_k, q_k), z = s e
                const int kr = tid / B, kc = tid % B;
                for (int st = 0; st < nsteps; ++st) {
                    const double2 (*g0)[W + 1] = sm.g[st & 1];
                    double2 (*g1)[W + 1] = sm.g[(st & 1) ^ 1];
                    int pr, qr, pc, qc;
                    gram_pair<W>(all, kr, st, pr, qr);
                    gram_pair<W>(all, kc, st, pc, qc);
                    double cr, zr, wr, cc, zc, wc;  // c, Re z, Im z of pairs kr, kc
                    const bool rr = pair_rotation(g0[pr][pr].x, g0[qr][qr].x, g0[pr][qr].x, g0[pr][qr].y, a.tol2, cr,
                                                  zr, wr);
                    const bool rcb = pair_rotation(g0[pc][pc].x, g0[qc][qc].x, g0[pc][qc].x, g0[pc][qc].y, a.tol2,
                                                   cc, zc, wc);
                    const double2 a00 = g0[pr][pc], a01 = g0[pr][qc], a10 = g0[qr][pc], a11 = g0[qr][qc];
                    // M = block J_kc: M0 = c a0 - conj(z) a1, M1 = z a0 + c a1 (per row)
                    auto col_rot = [&](double2 x, double2 y, double2& o0, double2& o1) {
                        o0 = make_double2(cc * x.x - (zc * y.x + wc * y.y), cc * x.y - (zc * y.y - wc * y.x));
                        o1 = make_double2((zc * x.x - wc * x.y) + cc * y.x, (zc * x.y + wc * x.x) + cc * y.y);
                    };
                    // J_kr^* M: row p = c M_p - z M_q, row q = conj(z) M_p + c M_q
                    auto row_rot = [&](double2 x, double2 y, double2& o0, double2& o1) {
                        o0 = make_double2(cr * x.x - (zr * y.x - wr * y.y), cr * x.y - (zr * y.y + wr * y.x));
                        o1 = make_double2((zr * x.x + wr * x.y) + cr * y.x, (zr * x.y - wr * x.x) + cr * y.y);
                    };
                    double2 m00, m01, m10, m11, n00, n01, n10, n11;
                    col_rot(a00, a01, m00, m01);
                    col_rot(a10, a11, m10, m11);
                    row_rot(m00, m10, n00, n10);
                    row_rot(m01, m11, n01, n11);
                    g1[pr][pc] = n00;
                    g1[pr][qc] = n01;
                    g1[qr][pc] = n10;
                    g1[qr][qc] = n11;
                    if (rcb) {
#pragma unroll
                        for (int h = 0; h < 2; ++h) {
                            double2* vrow = &sm.u.v[2 * kr + h][0];
                            double2 o0, o1;
                            col_rot(vrow[pc], vrow[qc], o0, o1);
                            vrow[pc] = o0;
                            vrow[qc] = o1;
                        }
                    }
                    if (__syncthreads_or((rr || rcb) ? 1 : 0)) rotated = true;
                }
            }
        }
        // 3. X <- X V: lane (j16, k4) feeds row 16 rt + j16 of column 4 kq + k4
        // (A) and V(4 kq + k4, 16 gn + j16) (B); the output tile holds rows
        // 16 rt + 4 k4 + e of column 16 gn + j16
        if (rotated) {
            float vr[W / 4][NT], vi[W / 4][NT];
#pragma unroll
            for (int kq = 0; kq < W / 4; ++kq)
#pragma unroll
                for (int gn = 0; gn < NT; ++gn) {
                    const double2 v = sm.u.v[4 * kq + k4][16 * gn + j16];
                    vr[kq][gn] = (float)v.x;
                    vi[kq][gn] = (float)v.y;
                }
            // the A operand of a row tile: from the LDS stage, or from memory
            // one tile ahead
            auto load_tile = [&](int rt, v2f (&dst)[W / 4]) {
                const int row = 16 * rt + j16;
#pragma unroll
                for (int kq = 0; kq < W / 4; ++kq) {
                    const int lc = 4 * kq + k4;
                    const bool lv = col_live(lc) && row < R;
                    if (STAGE) {
                        const float2 v = lv ? xs[lc * ldx + row] : make_float2(0.f, 0.f);
                        dst[kq] = v2f{v.x, v.y};
                    } else {
                        dst[kq] = raw_buffer_load_v2(rs, lv ? col_base(lc) + row * 8 : limit, 0, kDeviceScope);
                    }
                }
            };
            v2f xc[W / 4], xn[W / 4];
            if (wv * 16 < R) load_tile(wv, xc);
            for (int rt = wv; 16 * rt < R; rt += 4) {
                if (16 * (rt + 4) < R) load_tile(rt + 4, xn);
                v4f ar[NT], ai[NT];
#pragma unroll
                for (int gn = 0; gn < NT; ++gn) {
                    ar[gn] = v4f{0.f, 0.f, 0.f, 0.f};
                    ai[gn] = v4f{0.f, 0.f, 0.f, 0.f};
                }
#pragma unroll
                for (int kq = 0; kq < W / 4; ++kq) {
                    const v2f x = xc[kq];
#pragma unroll
                    for (int gn = 0; gn < NT; ++gn) {
                        ar[gn] = __builtin_amdgcn_mfma_f32_16x16x4f32(x.x, vr[kq][gn], ar[gn], 0, 0, 0);
                        ar[gn] = __builtin_amdgcn_mfma_f32_16x16x4f32(-x.y, vi[kq][gn], ar[gn], 0, 0, 0);
                        ai[gn] = __builtin_amdgcn_mfma_f32_16x16x4f32(x.x, vi[kq][gn], ai[gn], 0, 0, 0);
                        ai[gn] = __builtin_amdgcn_mfma_f32_16x16x4f32(x.y, vr[kq][gn], ai[gn], 0, 0, 0);
                    }
                }
                const int r0 = 16 * rt + 4 * k4;
#pragma unroll
                for (int gn = 0; gn < NT; ++gn) {
                    const int lc = 16 * gn + j16;
                    if (!col_live(lc)) continue;
                    const int base = col_base(lc);
#pragma unroll
                    for (int e = 0; e < 4; e += 2) {
                        const int r = r0 + e;
                        if (r + 1 < R) {
                            v4i q;
                            q.x = f32_bits(ar[gn][e]);
                            q.y = f32_bits(ai[gn][e]);
                            q.z = f32_bits(ar[gn][e + 1]);
                            q.w = f32_bits(ai[gn][e + 1]);
                            raw_buffer_store_v4(q, rs, base + r * 8, 0, kDeviceScope);
                        } else if (r < R) {
                            v2i q;
                            q.x = f32_bits(ar[gn][e]);
                            q.y = f32_bits(ai[gn][e]);
                            raw_buffer_store_v2(q, rs, base + r * 8, 0, kDeviceScope);
                        }
                    }
                }
#pragma unroll
                for (int kq = 0; kq < W / 4; ++kq) xc[kq] = xn[kq];
            }
        }
        // every wave's device-scope stores acknowledged before the stamp
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (tid == 0) {
            if (rotated) atomicOr(&a.rot[sweep * ns + s], 1);
            __hip_atomic_store(fl + step * npairs + bp, stamp, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

__global__ __launch_bounds__(256) void k_zero_ints(int* p, long long n)
{
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
        p[e] = 0;
}

constexpr size_t kMaxLds = 160 * 1024 - 1024;
constexpr size_t kBlockLds = 80 * 1024;  // two workgroups per CU

template <class K>
hipError_t allow_lds(K kern, size_t bytes)
{
    if (bytes <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds);
}

// bytes of one slice's work matrix (R x P) and, with V, its P x P rotations
size_t whole_bytes(int R, int P, bool withv)
{
    return ((size_t)R * P + (withv ? (size_t)P * P : 0)) * sizeof(float2);
}

// one group of G lanes per column pair of a step (at most `cap` threads)
int whole_threads(int G, int P, int cap = 1024)
{
    const int t = G * ((P + 1) / 2);
    return t >= cap ? cap : (t <= 64 ? 64 : ((t + 63) / 64) * 64);
}

template <int G, int RPL, bool WITHV>
hipError_t launch_whole(const JacobiArgs& a, void* scratch, int R, int P, hipStream_t st)
{
    const size_t lds = whole_bytes(R, P, WITHV);
    const int threads = whole_threads(G, P, whole_max_threads(RPL));
    if (lds <= kMaxLds) {
        auto kern = k_jacobi<G, RPL, true, WITHV>;
        hipError_t e = allow_lds(kern, lds);
        if (e != hipSuccess) return e;
        kern<<<a.nslices, threads, lds, st>>>(a, nullptr);
    } else {
        k_jacobi<G, RPL, false, WITHV><<<a.nslices, threads, 0, st>>>(a, static_cast<float2*>(scratch));
    }
    return hipGetLastError();
}

// block width: the two staged blocks (work columns, plus V columns when
// accumulating) fit kBlockLds, at most 32 pairs per step (or the tuned width)
int block_width(int R, int P, bool withv)
{
    const size_t col = (size_t)(R + (withv ? P : 0)) * sizeof(float2);
    const int bmax = (int)(kMaxLds / (2 * col));
    int b = (int)(kBlockLds / (2 * col));
    if (b > 32) b = 32;
    const int tuned = param(TP_PARAM_JACOBI_BLOCK);
    if (tuned > 0) b = tuned < bmax ? tuned : bmax;
    if (b < 1) b = 1;
    const int nb = (P + b - 1) / b;
    if (nb < 2) return 0;
    return b;
}

struct BlockPlan {
    int b, nb;
    size_t work_bytes, v_bytes, flag_bytes;
};

BlockPlan block_plan(int R, int P, int nslices, bool withv)
{
    BlockPlan pl{};
    pl.b = block_width(R, P, withv);
    if (pl.b == 0) return pl;
    pl.nb = (P + pl.b - 1) / pl.b;
    pl.nb += pl.nb & 1;
    pl.work_bytes = align_up((size_t)R * P * nslices * sizeof(float2));
    pl.v_bytes = withv ? align_up((size_t)P * P * nslices * sizeof(float2)) : 0;
    pl.flag_bytes = align_up(4 * (size_t)nslices * sizeof(int));
    return pl;
}

// one launch per sweep (column pairs in registers) or per block step (blocks
// staged in LDS): by measurement the sweep form is faster on slices taller
// than 256 rows (64-lane groups) and slower below
bool use_sweeps(int R)
{
    const int m = param(TP_PARAM_JACOBI_STEPWISE);
    if (m == 1) return false;
    if (m == 2) return true;
    return R > 256;
}

// Block sweep plan (slices without V): groups of G lanes, block width b (the
// groups per workgroup, even, at most 64 and 1024 / G threads), reduced
// towards 8 until a block step has enough items to fill the GPU.
struct SweepPlan {
    int b, nb, threads, grid, nitems;
    size_t lds, work_bytes, flag_bytes;
};

SweepPlan sweep_plan(int G, int rpl, int R, int P, int nslices)
{
    SweepPlan sp{};
    // workgroup size: 1024 threads, 512 with 32 rows per lane (registers)
    const int maxthreads = rpl >= 32 ? 512 : 1024;
    int b = maxthreads / G;
    if (b > 64) b = 64;
    const int tuned = param(TP_PARAM_JACOBI_BLOCK);
    if (tuned > 0) {
        b = tuned < b ? tuned : b;
        b &= ~1;
        if (b < 4) b = 4;
    } else {
        auto nbof = [&](int bb) { int n = (P + bb - 1) / bb; return n + (n & 1); };
        while (b > 8 && (long long)(nbof(b) / 2) * nslices < 512) b /= 2;
    }
    sp.b = b;
    sp.nb = (P + b - 1) / b;
    sp.nb += sp.nb & 1;
    if (sp.nb < 2) sp.nb = 2;
    sp.threads = b * G;
    sp.lds = (size_t)b * ((R + 1) & ~1) * sizeof(float2);
    sp.nitems = (sp.nb - 1) * nslices * (sp.nb / 2);
    int per_cu = (int)((160 * 1024) / (sp.lds + 1024));
    const int by_threads = 2048 / sp.threads;
    if (per_cu > by_threads) per_cu = by_threads;
    if (per_cu > 8) per_cu = 8;
    if (per_cu < 1) per_cu = 1;
    sp.grid = 256 * per_cu < sp.nitems ? 256 * per_cu : sp.nitems;
    sp.work_bytes = align_up((size_t)R * P * nslices * sizeof(float2));
    // rot [3][ns], done [ns], flags [ns][nb-1][nb/2], tickets [4], err
    sp.flag_bytes = align_up((4 * (size_t)nslices + (size_t)nslices * (sp.nb - 1) * (sp.nb / 2) + 5) * sizeof(int));
    return sp;
}

// the lane-group shape of a slice height (the instantiations launch_jacobi picks)
void group_shape(int R, int* G, int* rpl)
{
    if (R <= 32) { *G = 16; *rpl = 2; }
    else if (R <= 64) { *G = 16; *rpl = 4; }
    else if (R <= 128) { *G = 16; *rpl = 8; }
    else if (R <= 256) { *G = 16; *rpl = 16; }
    else if (R <= 512) { *G = 64; *rpl = 8; }
    else if (R <= 1024) { *G = 64; *rpl = 16; }
    else { *G = 64; *rpl = 32; }
}

template <int G, int RPL>
hipError_t launch_sweeps(const JacobiArgs& a, void* scratch, int R, int P, hipStream_t st)
{
    const SweepPlan sp = sweep_plan(G, RPL, R, P, a.nslices);
    char* base = static_cast<char*>(scratch);
    float2* work = reinterpret_cast<float2*>(base);
    int* ints = reinterpret_cast<int*>(base + sp.work_bytes);
    const int ns = a.nslices;
    int* rot = ints;
    int* done = rot + 3 * ns;
    int* flags = done + ns;
    const long long nflags = (long long)ns * (sp.nb - 1) * (sp.nb / 2);
    unsigned int* tickets = reinterpret_cast<unsigned int*>(flags + nflags);
    int* err = reinterpret_cast<int*>(tickets + 4);
    const long long nints = 4LL * ns + nflags + 5;
    k_zero_ints<<<(int)((nints + 255) / 256 < 1024 ? (nints + 255) / 256 : 1024), 256, 0, st>>>(ints, nints);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t per = (size_t)R * P;
    const int chunks = (int)(per / (256 * 8) + 1) < 64 ? (int)(per / (256 * 8) + 1) : 64;
    k_jacobi_block_init<<<dim3(chunks, ns), 256, 0, st>>>(a, work, nullptr, rot, done);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    // the 512-thread instantiation has twice the registers per lane
    auto kern = k_jacobi_sweep<G, RPL, 512>;
    if constexpr (RPL < 32)
        if (sp.threads > 512) kern = k_jacobi_sweep<G, RPL, 1024>;
    e = allow_lds(kern, sp.lds);
    if (e != hipSuccess) return e;
    SweepArgs sa{work, rot, done, flags, tickets, err, a.count, R, P, ns, sp.nb, sp.b, 0, sp.nitems, a.tol * a.tol};
    for (int sw = 0; sw < a.max_sweeps; ++sw) {
        sa.sweep = sw;
        kern<<<sp.grid, sp.threads, sp.lds, st>>>(sa);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    k_jacobi_block_finish<G><<<dim3(chunks, ns), 256, 0, st>>>(a, work, nullptr, rot, done, a.max_sweeps);
    return hipGetLastError();
}

// Gram block sweep: items of 16 NT columns (NT = 1 up to 256 rows, else 2;
// TP_PARAM_JACOBI_GRAM 2 / 3 force 1 / 2, 1 turns the form off)
int gram_nt(int R, int P)
{
    const int m = param(TP_PARAM_JACOBI_GRAM);
    if (m == 1 || P < 16) return 0;
    if (m == 2) return 1;
    if (m == 3) return 2;
    return R <= 256 ? 1 : 2;
}

// rows of the Gram sweep's rotation flags: one per sweep of the cap (at least
// the three rows the shared initialisation kernel clears)
int gram_flag_rows() { return std::max(3, param(TP_PARAM_JACOBI_SWEEPS)); }

SweepPlan gram_plan(int nt, int R, int P, int nslices)
{
    SweepPlan sp{};
    sp.b = 8 * nt;
    sp.nb = (P + sp.b - 1) / sp.b;
    sp.nb += sp.nb & 1;
    if (sp.nb < 2) sp.nb = 2;
    sp.threads = 256;
    sp.lds = nt == 1 ? sizeof(GramSmem<1>) : sizeof(GramSmem<2>);
    sp.lds = (sp.lds + 15) & ~(size_t)15;
    if (gram_stage_fits(nt, R)) sp.lds += (size_t)gram_ldx(R) * 16 * nt * sizeof(float2);
    sp.nitems = (sp.nb - 1) * nslices * (sp.nb / 2);
    int per_cu = (int)((160 * 1024) / (sp.lds + 1024));
    if (per_cu > 8) per_cu = 8;
    if (per_cu < 1) per_cu = 1;
    sp.grid = 256 * per_cu < sp.nitems ? 256 * per_cu : sp.nitems;
    sp.work_bytes = align_up((size_t)R * P * nslices * sizeof(float2));
    // rot [max_sweeps][ns] (one row per sweep), done [ns], flags, tickets [4], err
    const size_t rows = (size_t)gram_flag_rows();
    sp.flag_bytes = align_up(((rows + 1) * nslices + (size_t)nslices * (sp.nb - 1) * (sp.nb / 2) + 5) * sizeof(int));
    return sp;
}

template <int NT>
hipError_t launch_gram_sweeps(const JacobiArgs& a, void* scratch, int R, int P, hipStream_t st)
{
    const SweepPlan sp = gram_plan(NT, R, P, a.nslices);
    const int rows = gram_flag_rows();
    if (a.max_sweeps > rows) return hipErrorInvalidValue;  // the flags are sized for the sweep cap
    char* base = static_cast<char*>(scratch);
    float2* work = reinterpret_cast<float2*>(base);
    int* ints = reinterpret_cast<int*>(base + sp.work_bytes);
    const int ns = a.nslices;
    int* rot = ints;
    int* done = rot + (long long)rows * ns;
    int* flags = done + ns;
    const long long nflags = (long long)ns * (sp.nb - 1) * (sp.nb / 2);
    unsigned int* tickets = reinterpret_cast<unsigned int*>(flags + nflags);
    int* err = reinterpret_cast<int*>(tickets + 4);
    const long long nints = (long long)(rows + 1) * ns + nflags + 5;
    k_zero_ints<<<(int)((nints + 255) / 256 < 1024 ? (nints + 255) / 256 : 1024), 256, 0, st>>>(ints, nints);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t per = (size_t)R * P;
    const int chunks = (int)(per / (256 * 8) + 1) < 64 ? (int)(per / (256 * 8) + 1) : 64;
    k_jacobi_block_init<<<dim3(chunks, ns), 256, 0, st>>>(a, work, nullptr, rot, done);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    auto kern = gram_stage_fits(NT, R) ? k_gram_sweep<NT, true> : k_gram_sweep<NT, false>;
    e = allow_lds(kern, sp.lds);
    if (e != hipSuccess) return e;
    SweepArgs sa{work, rot, done, flags, tickets, err, a.count, R, P, ns, sp.nb, sp.b, 0, 0, a.tol * a.tol,
                 kGramSweepsPerLaunch};
    const int per_sweep = sp.nitems;  // (nb - 1) steps x slices x pairs
    for (int sw = 0; sw < a.max_sweeps; sw += kGramSweepsPerLaunch) {
        sa.sweep = sw;
        sa.nitems = std::min(kGramSweepsPerLaunch, a.max_sweeps - sw) * per_sweep;
        kern<<<sp.grid, sp.threads, sp.lds, st>>>(sa);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    k_jacobi_block_finish<16><<<dim3(chunks, ns), 256, 0, st>>>(a, work, nullptr, rot, done, a.max_sweeps, rows);
    return hipGetLastError();
}

template <int G, int RPL, bool WITHV>
hipError_t launch_blocked(const JacobiArgs& a, void* scratch, int R, int P, const BlockPlan& pl, hipStream_t st)
{
    if (!WITHV) {
        const int nt = gram_nt(R, P);
        if (nt == 1) return launch_gram_sweeps<1>(a, scratch, R, P, st);
        if (nt == 2) return launch_gram_sweeps<2>(a, scratch, R, P, st);
    }
    if (!WITHV && R <= G * RPL && use_sweeps(R)) return launch_sweeps<G, RPL>(a, scratch, R, P, st);
    char* base = static_cast<char*>(scratch);
    float2* work = reinterpret_cast<float2*>(base);
    float2* v = WITHV ? reinterpret_cast<float2*>(base + pl.work_bytes) : nullptr;
    int* rot = reinterpret_cast<int*>(base + pl.work_bytes + pl.v_bytes);
    int* done = rot + 3 * a.nslices;
    const size_t per = (size_t)R * P;
    const int chunks = (int)(per / (256 * 8) + 1) < 64 ? (int)(per / (256 * 8) + 1) : 64;
    k_jacobi_block_init<<<dim3(chunks, a.nslices), 256, 0, st>>>(a, work, v, rot, done);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    BlockArgs b{a.count, work, v, rot, done, R, P, a.nslices, pl.nb, pl.b, 0, 0, a.tol * a.tol};
    const int threads = min(512, ((pl.b * G + 63) / 64) * 64);
    const size_t lds = (size_t)2 * pl.b * (R + (WITHV ? P : 0)) * sizeof(float2);
    auto kern = k_jacobi_block<G, RPL, WITHV>;
    e = allow_lds(kern, lds);
    if (e != hipSuccess) return e;
    dim3 grid(pl.nb / 2, a.nslices);
    for (int sw = 0; sw < a.max_sweeps; ++sw) {
        b.sweep = sw;
        for (int bs = 0; bs < pl.nb - 1; ++bs) {
            b.bstep = bs;
            kern<<<grid, threads, lds, st>>>(b);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
    }
    k_jacobi_block_finish<G><<<dim3(chunks, a.nslices), 256, 0, st>>>(a, work, v, rot, done, a.max_sweeps);
    return hipGetLastError();
}

// slices too large for LDS, or too few of them to fill the GPU, go blocked
bool use_blocked(int R, int P, int nslices, bool withv)
{
    if (block_width(R, P, withv) == 0) return false;
    if (whole_bytes(R, P, withv) > kMaxLds) return true;
    const int mode = param(TP_PARAM_JACOBI_MODE);
    if (mode == 1) return false;
    if (mode == 2) return true;
    return nslices < param(TP_PARAM_JACOBI_BLOCKED_BELOW) && P >= 64;
}

template <int G, int RPL>
hipError_t launch_rpl(const JacobiArgs& a, void* scratch, int R, int P, hipStream_t st)
{
    const bool withv = a.qout != nullptr;
    if (!(a.whole && whole_bytes(R, P, withv) <= kMaxLds) && use_blocked(R, P, a.nslices, withv)) {
        const BlockPlan pl = block_plan(R, P, a.nslices, withv);
        return withv ? launch_blocked<G, RPL, true>(a, scratch, R, P, pl, st)
                     : launch_blocked<G, RPL, false>(a, scratch, R, P, pl, st);
    }
    return withv ? launch_whole<G, RPL, true>(a, scratch, R, P, st) : launch_whole<G, RPL, false>(a, scratch, R, P, st);
}

}  // namespace

size_t jacobi_scratch_bytes(int m, int n, int nslices, bool withv)
{
    const int R = m >= n ? m : n, P = m >= n ? n : m;
    if (use_blocked(R, P, nslices, withv)) {  // (an upper bound when a call forces one workgroup per slice)
        const BlockPlan pl = block_plan(R, P, nslices, withv);
        size_t bytes = pl.work_bytes + pl.v_bytes + pl.flag_bytes;
        if (!withv && use_sweeps(R)) {
            int G, rpl;
            group_shape(R, &G, &rpl);
            const SweepPlan sp = sweep_plan(G, rpl, R, P, nslices);
            if (sp.work_bytes + sp.flag_bytes > bytes) bytes = sp.work_bytes + sp.flag_bytes;
        }
        if (!withv && gram_nt(R, P) > 0) {
            const SweepPlan sp = gram_plan(gram_nt(R, P), R, P, nslices);
            if (sp.work_bytes + sp.flag_bytes > bytes) bytes = sp.work_bytes + sp.flag_bytes;
        }
        return bytes;
    }
    const size_t b = whole_bytes(R, P, withv);
    return b <= kMaxLds ? 0 : b * nslices;
}

size_t jacobi_batch_lds(int max_r, int max_p) { return (size_t)max_r * max_p * sizeof(float2); }

hipError_t launch_jacobi_batch(const JacobiArgs* items, const SliceUnit* units, int nunits, int max_r, int max_p,
                               int grid, hipStream_t st)
{
    if (nunits <= 0) return hipSuccess;
    if (max_r > 128) return hipErrorInvalidValue;
    const size_t lds = jacobi_batch_lds(max_r, max_p);
    hipError_t e = allow_lds(k_jacobi_batch, lds);
    if (e != hipSuccess) return e;
    k_jacobi_batch<<<grid < nunits ? grid : nunits, whole_threads(16, max_p), lds, st>>>(items, units, nunits);
    return hipGetLastError();
}

hipError_t launch_jacobi(const JacobiArgs& a, void* scratch, size_t scratch_bytes, hipStream_t st)
{
    if (a.nslices <= 0) return hipSuccess;
    const int R = a.transpose ? a.n : a.m;
    const int P = a.transpose ? a.m : a.n;
    const bool withv = a.qout != nullptr;
    const bool whole_fits = a.whole && whole_bytes(R, P, withv) <= kMaxLds;
    if (!whole_fits && jacobi_scratch_bytes(a.m, a.n, a.nslices, withv) > scratch_bytes) return hipErrorInvalidValue;
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
// Shrinkage of the rotated columns (eq (21)): column j of slice s is scaled
// by sqrt(1 - tau/sigma_j)/sigma_j where sigma_j > tau, else 0.  A
// workgroup takes a block of rows of one slice: the P column scales of the
// slice go to LDS once, then the rows stream through with 16-byte accesses
// (P a multiple of 4 and 16-byte aligned planes) or element by element.
// keep[s] = #{sigma_j > tau}.  Only the first *count slices when count is
// given.
__global__ __launch_bounds__(256) void k_shrink(float* __restrict__ wr, float* __restrict__ wi,
                                                const double* __restrict__ sigma, int* __restrict__ keep, int R,
                                                int P, int nslices, int rows, double tau,
                                                const int* __restrict__ count, int vec)
{
    extern __shared__ float fsc[];
    const int nb = (R + rows - 1) / rows;
    const int ns = count ? min(nslices, *count) : nslices;
    for (long long b = blockIdx.x; b < (long long)ns * nb; b += gridDim.x) {
        const int s = (int)(b / nb), rb = (int)(b % nb);
        __syncthreads();  // the previous block's scales are no longer read
        int kept = 0;     // #{sigma_j > tau}, counted across the workgroup
        for (int j0 = 0; j0 < P; j0 += blockDim.x) {
            const int j = j0 + threadIdx.x;
            bool above = false;
            if (j < P) {
                const double sg = sigma[(long long)s * P + j];
                above = sg > tau;
                fsc[j] = above ? (float)(sqrt(1.0 - tau / sg) / sg) : 0.0f;
            }
            kept += __syncthreads_count(above);
        }
        if (keep && rb == 0 && threadIdx.x == 0) keep[s] = kept;
        __syncthreads();
        const int r0 = rb * rows, nr = min(rows, R - r0);
        const long long base = ((long long)s * R + r0) * P;
        if (vec) {
            float4* pr = reinterpret_cast<float4*>(wr + base);
            float4* pi = reinterpret_cast<float4*>(wi + base);
            const int q4 = P / 4, n4 = nr * q4;
#pragma unroll 4
            for (int q = threadIdx.x; q < n4; q += blockDim.x) {
                const int j = (q % q4) * 4;
                float4 a = pr[q], c = pi[q];
                a.x *= fsc[j]; a.y *= fsc[j + 1]; a.z *= fsc[j + 2]; a.w *= fsc[j + 3];
                c.x *= fsc[j]; c.y *= fsc[j + 1]; c.z *= fsc[j + 2]; c.w *= fsc[j + 3];
                pr[q] = a;
                pi[q] = c;
            }
        } else {
            const int n1 = nr * P;
            for (int q = threadIdx.x; q < n1; q += blockDim.x) {
                const float f = fsc[q % P];
                wr[base + q] *= f;
                wi[base + q] *= f;
            }
        }
    }
}

// Batched shrinkage: unit (item, slice) scales the slice's rotated columns
// by sqrt(d_j)/sigma_j with the item's tau; with tau_rel the item's tau is
// tau_rel * max over its slices of sigma_1 (= tau_rel * tsn), computed here
// from the singular values of all its slices.
__global__ __launch_bounds__(256) void k_shrink_batch(const ShrinkItem* __restrict__ items,
                                                      const SliceUnit* __restrict__ units, int nunits)
{
    __shared__ double red[256];
    for (int u = blockIdx.x; u < nunits; u += gridDim.x) {
        const SliceUnit w = units[u];
        const ShrinkItem it = items[w.item];
        double tau = it.tau;
        if (it.rel) {
            double mx = 0.0;
            for (int e = threadIdx.x; e < it.h * it.P; e += blockDim.x) mx = fmax(mx, it.sigma[e]);
            __syncthreads();
            red[threadIdx.x] = mx;
            __syncthreads();
            for (int st = blockDim.x / 2; st > 0; st >>= 1) {
                if (threadIdx.x < st) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + st]);
                __syncthreads();
            }
            tau = it.tau * red[0];
        }
        const double* sg = it.sigma + (long long)w.slice * it.P;
        const long long per = (long long)it.R * it.P;
        float* wr = it.wr + w.slice * per;
        float* wi = it.wi + w.slice * per;
        for (long long e = threadIdx.x; e < per; e += blockDim.x) {
            const double sv = sg[e % it.P];
            const float f = sv > tau ? (float)(sqrt(1.0 - tau / sv) / sv) : 0.0f;
            wr[e] *= f;
            wi[e] *= f;
        }
        if (threadIdx.x == 0) {
            if (it.keep) {
                int k = 0;
                for (int j = 0; j < it.P; ++j) k += sg[j] > tau ? 1 : 0;
                it.keep[w.slice] = k;
            }
            if (it.tau_out && w.slice == 0) *it.tau_out = (float)tau;
        }
    }
}

// tnn = (1/n3) sum_k w_k sum_j sigma_kj, w_k = 1 for real slices, 2 otherwise
// (Definition 2.9 with eq (14), using the conjugate symmetry of eq (8)).
// slice s has last-mode bin s / period (period = 1 for p = 3); the bins 0 and,
// for even n3, n3/2 are their own conjugates, the others stand for two
__global__ __launch_bounds__(256) void k_tnn_reduce(const double* __restrict__ sigma, int nslices, int P, int n3,
                                                    int period, double* __restrict__ out)
{
    __shared__ double part[256];
    double acc = 0.0;
    for (int s = 0; s < nslices; ++s) {  // fixed order: deterministic
        const int kp = s / period;
        const bool real = (kp == 0) || (n3 % 2 == 0 && kp == n3 / 2);
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
    if (threadIdx.x == 0) *out = part[0] / ((double)n3 * period);
}

}  // namespace

hipError_t launch_shrink(float* wr, float* wi, const double* sigma, int* keep, int R, int P, int nslices, double tau,
                         hipStream_t st, const int* count)
{
    const long long total = (long long)R * P * nslices;
    if (total <= 0) return hipSuccess;
    // read and write both planes, read the singular values (slices the
    // device-side count excludes are not known here)
    if (!count) trace_work(0.0, 16.0 * total + 8.0 * (double)P * nslices);
    const int rows = std::max(1, std::min(R, 8192 / P));  // about 32 KB of each plane per block
    const long long blocks = (long long)nslices * ((R + rows - 1) / rows);
    const int grid = (int)std::min<long long>(blocks, 256LL * 16);
    const int vec = (P % 4 == 0 && ((reinterpret_cast<uintptr_t>(wr) | reinterpret_cast<uintptr_t>(wi)) & 15) == 0)
                        ? 1 : 0;
    k_shrink<<<grid, 256, (size_t)P * sizeof(float), st>>>(wr, wi, sigma, keep, R, P, nslices, rows, tau, count, vec);
    return hipGetLastError();
}

hipError_t launch_shrink_batch(const ShrinkItem* items, const SliceUnit* units, int nunits, int grid, hipStream_t st)
{
    if (nunits <= 0) return hipSuccess;
    k_shrink_batch<<<grid < nunits ? grid : nunits, 256, 0, st>>>(items, units, nunits);
    return hipGetLastError();
}


namespace {

// max over all slices and columns (the column norms are the singular values)
__global__ __launch_bounds__(256) void k_tsn_reduce(const double* __restrict__ sigma, long long total,
                                                    double* __restrict__ out)
{
    __shared__ double part[256];
    double m = 0.0;
    for (long long e = threadIdx.x; e < total; e += blockDim.x) m = fmax(m, sigma[e]);
    part[threadIdx.x] = m;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) part[threadIdx.x] = fmax(part[threadIdx.x], part[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = part[0];
}

// per slice (one workgroup): the P values in decreasing order, ties by index
__global__ __launch_bounds__(256) void k_sort_sigma(const double* __restrict__ sigma, double* __restrict__ sorted,
                                                    int P)
{
    const double* sg = sigma + (long long)blockIdx.x * P;
    double* out = sorted + (long long)blockIdx.x * P;
    for (int j = threadIdx.x; j < P; j += blockDim.x) {
        const double v = sg[j];
        int r = 0;
        for (int i = 0; i < P; ++i) {
            const double u = sg[i];
            r += (u > v || (u == v && i < j)) ? 1 : 0;
        }
        out[r] = v;
    }
}

// S(i,i,1) = (1/n3) sum over all n3 slices of the i-th largest singular value
// (the h leading slices, the non-real ones counted twice by conjugate
// symmetry); rank = #{i : S(i,i,1) > tol}, tol < 0: tol_scale * S(1,1,1)
__global__ __launch_bounds__(256) void k_tubal_rank(const double* __restrict__ sorted, int nslices, int P, int n3,
                                                    double tol, double tol_scale, int* __restrict__ out)
{
    __shared__ int cnt[256];
    __shared__ double s0;
    auto mean_at = [&](int i) {
        double acc = 0.0;
        for (int s = 0; s < nslices; ++s) {
            const bool real = (s == 0) || (n3 % 2 == 0 && s == n3 / 2);
            acc += (real ? 1.0 : 2.0) * sorted[(long long)s * P + i];
        }
        return acc / n3;
    };
    if (threadIdx.x == 0) s0 = P > 0 ? mean_at(0) : 0.0;
    __syncthreads();
    const double t = tol >= 0.0 ? tol : tol_scale * s0;
    int c = 0;
    for (int i = threadIdx.x; i < P; i += blockDim.x) c += mean_at(i) > t ? 1 : 0;
    cnt[threadIdx.x] = c;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) cnt[threadIdx.x] += cnt[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = cnt[0];
}

}  // namespace

hipError_t launch_tsn_reduce(const double* sigma, int nslices, int P, double* out, hipStream_t st)
{
    k_tsn_reduce<<<1, 256, 0, st>>>(sigma, (long long)nslices * P, out);
    return hipGetLastError();
}

hipError_t launch_tubal_rank(const double* sigma, double* sorted, int nslices, int P, int n3, double tol,
                             double tol_scale, int* out, hipStream_t st)
{
    k_sort_sigma<<<nslices, 256, 0, st>>>(sigma, sorted, P);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_tubal_rank<<<1, 256, 0, st>>>(sorted, nslices, P, n3, tol, tol_scale, out);
    return hipGetLastError();
}

hipError_t launch_tnn_reduce(const double* sigma, int nslices, int P, int n3, double* out, hipStream_t st,
                             int period)
{
    k_tnn_reduce<<<1, 256, 0, st>>>(sigma, nslices, P, n3, period, out);
    return hipGetLastError();
}

}  // namespace tp

// ------------------------------------------------------------- t-SVD out --
namespace tp {
namespace {

// Per slice (one workgroup): sort the singular values in decreasing order
// (ties by index), and write the full bases and the diagonal of S^(k):
//   L (R x R): column r = w_perm(r) / sigma_perm(r) for sigma > 0, the rest
//              completed to an orthonormal basis: each missing column is the
//              unit vector e_c with the largest component outside the span so
//              far, orthogonalised twice (classical Gram-Schmidt) and
//              normalised;
//   Q (P x P): column r = v_perm(r);
//   S (m x n): S(r, r) = sigma_perm(r), zero elsewhere.
// All outputs are row-major planar slices.
__global__ __launch_bounds__(256) void k_tsvd_finish(const float2* __restrict__ cols, const double* __restrict__ sigma,
                                                     const float2* __restrict__ q, float* __restrict__ lr,
                                                     float* __restrict__ li, float* __restrict__ qr,
                                                     float* __restrict__ qi, float* __restrict__ sr,
                                                     float* __restrict__ si, int R, int P, int m, int n)
{
    extern __shared__ char smem[];
    int* perm = reinterpret_cast<int*>(smem);                               // P
    double2* w = reinterpret_cast<double2*>(smem + align_up(P * sizeof(int)));  // R
    double2* coef = w + R;                                                  // R
    __shared__ double red[256];
    __shared__ int redi[256];
    const int s = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
    const double* sg = sigma + (long long)s * P;
    const float2* cs = cols + (long long)s * R * P;
    const float2* qs = q + (long long)s * P * P;
    float* Lr = lr + (long long)s * R * R;
    float* Li = li + (long long)s * R * R;

    for (int j = tid; j < P; j += nt) {
        int rank = 0;
        for (int i = 0; i < P; ++i) rank += (sg[i] > sg[j] || (sg[i] == sg[j] && i < j)) ? 1 : 0;
        perm[rank] = j;
    }
    __syncthreads();
    // Q columns and S diagonal
    for (int e = tid; e < P * P; e += nt) {
        const int i = e / P, r = e % P;
        const float2 v = qs[(long long)perm[r] * P + i];
        qr[(long long)s * P * P + e] = v.x;
        qi[(long long)s * P * P + e] = v.y;
    }
    for (int e = tid; e < m * n; e += nt) {
        const int i = e / n, j = e % n;
        sr[(long long)s * m * n + e] = (i == j) ? (float)sg[perm[i]] : 0.0f;
        si[(long long)s * m * n + e] = 0.0f;
    }
    // leading columns of L
    int rank = 0;
    for (int r = 0; r < P; ++r) rank += sg[perm[r]] > 0.0 ? 1 : 0;
    for (int e = tid; e < R * R; e += nt) {
        const int i = e / R, r = e % R;
        float vr = 0.0f, vi = 0.0f;
        if (r < rank) {
            const float2 v = cs[(long long)perm[r] * R + i];
            const double inv = 1.0 / sg[perm[r]];
            vr = (float)(v.x * inv);
            vi = (float)(v.y * inv);
        }
        Lr[e] = vr;
        Li[e] = vi;
    }
    __syncthreads();
    // completion
    for (int r = rank; r < R; ++r) {
        double best = -1.0;
        int bi = 0;
        for (int c = tid; c < R; c += nt) {
            double in = 0.0;
            for (int qq = 0; qq < r; ++qq) {
                const double a = Lr[(long long)c * R + qq], b = Li[(long long)c * R + qq];
                in += a * a + b * b;
            }
            if (1.0 - in > best) {
                best = 1.0 - in;
                bi = c;
            }
        }
        red[tid] = best;
        redi[tid] = bi;
        __syncthreads();
        for (int h = nt / 2; h > 0; h >>= 1) {
            if (tid < h) {
                const double o = red[tid + h];
                const int oi = redi[tid + h];
                if (o > red[tid] || (o == red[tid] && oi < redi[tid])) {
                    red[tid] = o;
                    redi[tid] = oi;
                }
            }
            __syncthreads();
        }
        const int c = redi[0];
        for (int i = tid; i < R; i += nt) w[i] = make_double2(i == c ? 1.0 : 0.0, 0.0);
        __syncthreads();
        for (int pass = 0; pass < 2; ++pass) {
            for (int qq = tid; qq < r; qq += nt) {  // coef_q = L(:,q)^* w
                double ar = 0.0, ai = 0.0;
                for (int i = 0; i < R; ++i) {
                    const double lr_ = Lr[(long long)i * R + qq], li_ = Li[(long long)i * R + qq];
                    ar += lr_ * w[i].x + li_ * w[i].y;
                    ai += lr_ * w[i].y - li_ * w[i].x;
                }
                coef[qq] = make_double2(ar, ai);
            }
            __syncthreads();
            for (int i = tid; i < R; i += nt) {  // w -= sum_q coef_q L(:,q)
                double ar = w[i].x, ai = w[i].y;
                for (int qq = 0; qq < r; ++qq) {
                    const double lr_ = Lr[(long long)i * R + qq], li_ = Li[(long long)i * R + qq];
                    ar -= coef[qq].x * lr_ - coef[qq].y * li_;
                    ai -= coef[qq].x * li_ + coef[qq].y * lr_;
                }
                w[i] = make_double2(ar, ai);
            }
            __syncthreads();
        }
        double nrm = 0.0;
        for (int i = tid; i < R; i += nt) nrm += w[i].x * w[i].x + w[i].y * w[i].y;
        red[tid] = nrm;
        __syncthreads();
        for (int h = nt / 2; h > 0; h >>= 1) {
            if (tid < h) red[tid] += red[tid + h];
            __syncthreads();
        }
        const double inv = 1.0 / sqrt(red[0]);
        for (int i = tid; i < R; i += nt) {
            Lr[(long long)i * R + r] = (float)(w[i].x * inv);
            Li[(long long)i * R + r] = (float)(w[i].y * inv);
        }
        __syncthreads();
    }
}

}  // namespace

size_t tsvd_finish_lds(int R, int P) { return align_up(P * sizeof(int)) + 2 * (size_t)R * sizeof(double2); }

hipError_t launch_tsvd_finish(const float2* cols, const double* sigma, const float2* q, Planes L, Planes Q, Planes S,
                              int R, int P, int m, int n, int nslices, hipStream_t st)
{
    const size_t lds = tsvd_finish_lds(R, P);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void*)k_tsvd_finish, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           160 * 1024 - 1024);
        if (e != hipSuccess) return e;
    }
    k_tsvd_finish<<<nslices, 256, lds, st>>>(cols, sigma, q, L.re, L.im, Q.re, Q.im, S.re, S.im, R, P, m, n);
    return hipGetLastError();
}

}  // namespace tp
