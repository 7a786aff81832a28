// Batched planar-complex slice GEMM on the gfx950 matrix cores:
//   C^(s) = op(A^(s)) op(B^(s)),  s = 0 .. nslices-1,
// the dense per-slice step of Algorithm 1 (Cbar^(i) = Abar^(i) Bbar^(i) for the
// ceil((n3+1)/2) leading slices, eq (10)), also used for the reconstruction
// products of the singular value thresholding and the randomized range finder.
//
// Complex products use the 4-real-product form  Cr = ArBr - AiBi,
// Ci = ArBi + AiBr.  Real slices (the DC slice and, for even n3, the middle
// one) only issue the ArBr product and write Ci = 0.
//
// Precisions (all accumulate in FP32):
//   FP32   v_mfma_f32_16x16x4f32
//   BF16X3 every operand split as x = hi + lo, hi = bf16(x), lo = bf16(x - hi)
//          (round to nearest even), products hi*hi + hi*lo + lo*hi on
//          v_mfma_f32_16x16x32_bf16
//   BF16   hi*hi only
//
// Tiling: 256 threads = 4 wavefronts; a workgroup tile of BM x BN (complex)
// outputs is split WGM x WGN over the wavefronts, each wavefront owning
// TM x TN MFMA tiles of 16 x 16.  Operand panels (BM x BK of op(A), BN x BK of
// op(B)) are staged through LDS, double buffered, with k contiguous so that
// each lane reads its MFMA operands with 16-byte LDS loads.  Tile shapes from
// 64 x 64 to 256 x 16 cover square products; FP32 products with at most 64
// output columns (the range-finder products of the randomized SVD) take a
// dedicated kernel that streams op(A) straight into registers, and FP32
// products with an inner dimension of at most 48 and whole 64 x 256 output
// tiles (the reconstruction of the randomized SVT) one that keeps A in
// registers and streams the output.
#include "tp_internal.h"

namespace tp {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef short shortx8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <int BM_, int BN_, int WGM_, int WGN_>
struct Tile {
    static constexpr int BM = BM_, BN = BN_, WGM = WGM_, WGN = WGN_;
    static constexpr int WM = BM / WGM, WN = BN / WGN;
    static constexpr int TM = WM / 16, TN = WN / 16;
    static_assert(WGM * WGN == 4, "four wavefronts");
    static_assert(TM >= 1 && TN >= 1 && WM % 16 == 0 && WN % 16 == 0, "16 x 16 MFMA tiles");
};
using T64x64 = Tile<64, 64, 2, 2>;
using T128x128 = Tile<128, 128, 2, 2>;
using T128x64 = Tile<128, 64, 2, 2>;
using T128x32 = Tile<128, 32, 4, 1>;
using T256x16 = Tile<256, 16, 4, 1>;
using T32x32 = Tile<32, 32, 2, 2>;
using T64x48 = Tile<64, 48, 4, 1>;

struct SliceView {
    const float *ar, *ai, *br, *bi;
    float *cr, *ci;
    long long ldc;
    int K0, K;  // inner-dimension range [K0, K) of this workgroup
    bool real;
};

// Slice s, inner-dimension part kp of p.ksplit (output to the partial buffer
// when the product is split).
__device__ __forceinline__ SliceView slice_view(const CgemmArgs& p, int s, int kp = 0)
{
    SliceView v;
    v.ar = p.ar + s * p.sa;
    v.ai = p.ai + s * p.sa;
    v.br = p.br + s * p.sb;
    v.bi = p.bi + s * p.sb;
    const int K = p.kdyn ? min(p.kdyn[s], p.k) : p.k;
    v.real = (p.real_first && s == 0) || (p.real_last && s == p.nslices - 1);
    if (p.ksplit > 1) {
        const long long mn = (long long)p.m * p.n;
        const int chunk = ((p.k + p.ksplit - 1) / p.ksplit + 15) / 16 * 16;
        v.K0 = min(K, kp * chunk);
        v.K = min(K, v.K0 + chunk);
        v.cr = p.part + ((long long)kp * p.nslices + s) * mn;
        v.ci = v.cr + (long long)p.ksplit * p.nslices * mn;
        v.ldc = p.n;
    } else {
        v.K0 = 0;
        v.K = K;
        v.cr = p.cr + s * p.sc;
        v.ci = p.ci + s * p.sc;
        v.ldc = p.ldc;
    }
    return v;
}

// The device-side values of a launch (see CgemmArgs): false when its gate is
// 0 or a live size is 0.  A capped k replaces k; m and n keep the layout of
// the output and of the split parts, and m_live / n_live give the rows and
// columns that are computed (tiles past them do nothing).
__device__ __forceinline__ int m_live(const CgemmArgs& p) { return p.dyn_m ? min(p.m, *p.dyn_m) : p.m; }
__device__ __forceinline__ int n_live(const CgemmArgs& p) { return p.dyn_n ? min(p.n, *p.dyn_n) : p.n; }
__device__ __forceinline__ bool apply_dyn(CgemmArgs& p)
{
    if (p.gate && *p.gate == 0) return false;
    if (p.dyn_k) p.k = min(p.k, *p.dyn_k);
    return m_live(p) > 0 && n_live(p) > 0 && p.k > 0;
}
__device__ __forceinline__ bool slice_live(const CgemmArgs& p, int s) { return !p.dyn_ns || s < *p.dyn_ns; }

// Four source elements contiguous in memory at off (valid of them in bounds):
// one 16-byte load per plane when all four are valid and the planes allow
// it, else element by element with zero fill.  neg negates the imaginary
// part (conjugated operands).
struct Quad {
    float4 r, i;
};
__device__ __forceinline__ Quad load4(const float* pr, const float* pi, long long off, int valid, bool vec, bool neg)
{
    Quad q;
    if (vec && valid == 4) {
        q.r = *reinterpret_cast<const float4*>(pr + off);
        q.i = *reinterpret_cast<const float4*>(pi + off);
    } else {
        q.r.x = valid > 0 ? pr[off] : 0.0f;
        q.r.y = valid > 1 ? pr[off + 1] : 0.0f;
        q.r.z = valid > 2 ? pr[off + 2] : 0.0f;
        q.r.w = valid > 3 ? pr[off + 3] : 0.0f;
        q.i.x = valid > 0 ? pi[off] : 0.0f;
        q.i.y = valid > 1 ? pi[off + 1] : 0.0f;
        q.i.z = valid > 2 ? pi[off + 2] : 0.0f;
        q.i.w = valid > 3 ? pi[off + 3] : 0.0f;
    }
    if (neg) q.i = -q.i;
    return q;
}

// true when 16-byte loads of 4-aligned groups are aligned in both planes
__device__ __forceinline__ bool vec_ok(const float* pr, const float* pi, long long ld)
{
    return ((reinterpret_cast<unsigned long long>(pr) | reinterpret_cast<unsigned long long>(pi)) & 15) == 0 &&
           (ld & 3) == 0;
}

// Register staging of one BM x BK panel of op(A) and BN x BK panel of op(B):
// the panels are cut in groups of 4 consecutive elements along the
// contiguous direction of the source, groups spread over the 256 threads.
//   A, OP_N: group -> (row, 4 k)    A, OP_C: group -> (k, 4 rows)
//   B, OP_N: group -> (k, 4 cols)   B, OP_C: group -> (col, 4 k)
// Tile origins and inner-dimension stages are multiples of 4, so every
// group starts 4-aligned in its source.
template <int OPA, int OPB, int BM, int BN, int BK>
struct PanelLoader {
    static constexpr int KQ = BK / 4;
    static constexpr int GA = BM * BK / 4, GB = BN * BK / 4;
    static constexpr int NA = (GA + 255) / 256, NB = (GB + 255) / 256;
    Quad a[NA], b[NB];

    __device__ __forceinline__ void load(const SliceView& v, const CgemmArgs& p, int m0, int n0, int k0, int tid)
    {
        const bool va = vec_ok(v.ar, v.ai, p.lda), vb = vec_ok(v.br, v.bi, p.ldb);
#pragma unroll
        for (int u = 0; u < NA; ++u) {
            const int g = tid + u * 256;
            int valid;
            long long off;
            if (OPA == OP_N) {
                const int row = m0 + g / KQ, kk = k0 + (g % KQ) * 4;
                valid = (g < GA && row < p.m) ? max(0, min(4, v.K - kk)) : 0;
                off = (long long)row * p.lda + kk;
            } else {
                const int kk = k0 + g / (BM / 4), row = m0 + (g % (BM / 4)) * 4;
                valid = (g < GA && kk < v.K) ? max(0, min(4, p.m - row)) : 0;
                off = (long long)kk * p.lda + row;
            }
            a[u] = load4(v.ar, v.ai, off, valid, va, OPA == OP_C);
        }
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int g = tid + u * 256;
            int valid;
            long long off;
            if (OPB == OP_N) {
                const int kk = k0 + g / (BN / 4), col = n0 + (g % (BN / 4)) * 4;
                valid = (g < GB && kk < v.K) ? max(0, min(4, p.n - col)) : 0;
                off = (long long)kk * p.ldb + col;
            } else {
                const int col = n0 + g / KQ, kk = k0 + (g % KQ) * 4;
                valid = (g < GB && col < p.n) ? max(0, min(4, v.K - kk)) : 0;
                off = (long long)col * p.ldb + kk;
            }
            b[u] = load4(v.br, v.bi, off, valid, vb, OPB == OP_C);
        }
    }

    // writes the panels to LDS.  Row-major panels are sA[row][k], sB[col][k]
    // (leading dimension LDK); with KA (KB) the A (B) panel is k-major,
    // sA[k][row] (sB[k][col]) with leading dimension BM + 4 (BN + 4), chosen
    // where the source groups run along rows (columns), so that every group
    // is one contiguous 16-byte LDS write.
    template <int LDK, bool KA, bool KB, class Store>
    __device__ __forceinline__ void store(int tid, Store&& st) const
    {
        constexpr int LDM = BM + 4, LDN = BN + 4;
#pragma unroll
        for (int u = 0; u < NA; ++u) {
            const int g = tid + u * 256;
            if (g >= GA) continue;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                int idx;
                if (OPA == OP_N)
                    idx = KA ? ((g % KQ) * 4 + e) * LDM + g / KQ : (g / KQ) * LDK + (g % KQ) * 4 + e;
                else
                    idx = KA ? (g / (BM / 4)) * LDM + (g % (BM / 4)) * 4 + e
                             : ((g % (BM / 4)) * 4 + e) * LDK + g / (BM / 4);
                st.a(idx, (&a[u].r.x)[e], (&a[u].i.x)[e]);
            }
        }
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int g = tid + u * 256;
            if (g >= GB) continue;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                int idx;
                if (OPB == OP_N)
                    idx = KB ? (g / (BN / 4)) * LDN + (g % (BN / 4)) * 4 + e
                             : ((g % (BN / 4)) * 4 + e) * LDK + g / (BN / 4);
                else
                    idx = KB ? ((g % KQ) * 4 + e) * LDN + g / KQ : (g / KQ) * LDK + (g % KQ) * 4 + e;
                st.b(idx, (&b[u].r.x)[e], (&b[u].i.x)[e]);
            }
        }
    }
};

template <class T>
__device__ __forceinline__ void write_tile(const SliceView& v, const CgemmArgs& p, int m0, int n0, int wr, int wc,
                                           int lane, const floatx4 (&accr)[T::TM][T::TN],
                                           const floatx4 (&acci)[T::TM][T::TN])
{
    const int g = lane >> 4, c16 = lane & 15;
#pragma unroll
    for (int ti = 0; ti < T::TM; ++ti)
#pragma unroll
        for (int tj = 0; tj < T::TN; ++tj)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int row = m0 + wr + 16 * ti + 4 * g + j;
                const int col = n0 + wc + 16 * tj + c16;
                if (row < p.m && col < p.n) {
                    const long long off = (long long)row * v.ldc + col;
                    v.cr[off] = accr[ti][tj][j];
                    v.ci[off] = v.real ? 0.0f : acci[ti][tj][j];
                }
            }
}

// ------------------------------------------------------------------ FP32 --
struct StoreF32 {
    float *ar, *ai, *br, *bi;
    __device__ __forceinline__ void a(int i, float r, float im) const { ar[i] = r; ai[i] = im; }
    __device__ __forceinline__ void b(int i, float r, float im) const { br[i] = r; bi[i] = im; }
};

// Tile of workgroup blockIdx, XCD-aware: the hardware deals consecutive
// workgroup ids round-robin to the 8 XCDs, each with its own L2; renumbering
// gives every XCD one contiguous run of tiles (same slice, neighbouring
// row/column blocks), so the panels those tiles share stay in one L2.
__device__ __forceinline__ void xcd_tile(int& x, int& y, int& z)
{
    const int nx = gridDim.x, ny = gridDim.y, nz = gridDim.z;
    const int total = nx * ny * nz;
    const int i = blockIdx.x + nx * (blockIdx.y + ny * blockIdx.z);
    int t = i;
    if (total >= 64 && total % 8 == 0) t = (i % 8) * (total / 8) + i / 8;
    x = t % nx;
    y = (t / nx) % ny;
    z = t / (nx * ny);
}

// FP32 LDS footprint of one workgroup tile: double-buffered re/im panels of
// BK columns of the inner dimension
template <int R, int BK>
constexpr int panel_floats()  // one plane of an R x BK panel, row-major or k-major
{
    return R * (BK + 4) > BK * (R + 4) ? R * (BK + 4) : BK * (R + 4);
}
template <class T, int BK = 16>
constexpr int f32_smem_floats()
{
    return 2 * 2 * (panel_floats<T::BM, BK>() + panel_floats<T::BN, BK>());
}

// One BM x BN output tile of slice s at (m0, n0); smem holds
// f32_smem_floats<T, BK>() floats.  BK (16 or 32) inner-dimension columns
// per LDS stage.
template <int OPA, int OPB, class T, int BK = 16>
__device__ __forceinline__ void cgemm_f32_tile(const CgemmArgs& p, int slice, int m0, int n0, float* smem, int kp = 0)
{
    constexpr int BM = T::BM, BN = T::BN, TM = T::TM, TN = T::TN;
    constexpr int LDK = BK + 4;
    // k-major panels where the source runs along the output dimension
    constexpr bool KA = OPA == OP_C, KB = OPB == OP_N;
    constexpr int LDM = BM + 4, LDN = BN + 4;
    static_assert(BK % 16 == 0, "16-column MFMA k groups");
    typedef float PanelA[panel_floats<BM, BK>()];
    typedef float PanelB[panel_floats<BN, BK>()];
    PanelA* sAr = reinterpret_cast<PanelA*>(smem);
    PanelA* sAi = sAr + 2;
    PanelB* sBr = reinterpret_cast<PanelB*>(smem + 4 * panel_floats<BM, BK>());
    PanelB* sBi = sBr + 2;

    const SliceView v = slice_view(p, slice, kp);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = (wave / T::WGN) * T::WM, wc = (wave % T::WGN) * T::WN;
    const int g = lane >> 4, r16 = lane & 15;

    // Complex products: tiles with few MFMA sub-tiles per wavefront use the
    // three-product form p1 = Ar Br, p2 = Ai Bi, p3 = (Ar + Ai)(Br + Bi),
    // Cr = p1 - p2, Ci = p3 - p1 - p2 (3 real MFMAs per step instead of 4);
    // larger tiles, whose accumulators would not fit the registers three
    // times, keep the four-product form (p1 = Cr, p3 = Ci, p2 unused).
    // Real slices: p1 only.
    constexpr bool M3 = TM * TN <= 4;
    floatx4 p1[TM][TN], p2[TM][TN], p3[TM][TN];
#pragma unroll
    for (int ti = 0; ti < TM; ++ti)
#pragma unroll
        for (int tj = 0; tj < TN; ++tj) {
            p1[ti][tj] = floatx4{0.f, 0.f, 0.f, 0.f};
            p2[ti][tj] = floatx4{0.f, 0.f, 0.f, 0.f};
            p3[ti][tj] = floatx4{0.f, 0.f, 0.f, 0.f};
        }

    PanelLoader<OPA, OPB, BM, BN, BK> ld;
    const int nk = (v.K - v.K0 + BK - 1) / BK;
    if (nk > 0) {
        ld.load(v, p, m0, n0, v.K0, tid);
        ld.template store<LDK, KA, KB>(tid, StoreF32{sAr[0], sAi[0], sBr[0], sBi[0]});
    }
    __syncthreads();
    for (int c = 0; c < nk; ++c) {
        const int cur = c & 1;
        if (c + 1 < nk) ld.load(v, p, m0, n0, v.K0 + (c + 1) * BK, tid);
#pragma unroll
        for (int kh = 0; kh < BK / 16; ++kh) {
        // lane (g, r16) of MFMA step s uses k = 16 kh + 4g + s: one 16-byte LDS read per operand
        float4 fa_r[TM], fa_i[TM], fb_r[TN], fb_i[TN];
#pragma unroll
        for (int t = 0; t < TM; ++t) {
            if (KA) {  // four reads of 16 consecutive rows each
                const int o = (16 * kh + 4 * g) * LDM + wr + 16 * t + r16;
                fa_r[t] = float4{sAr[cur][o], sAr[cur][o + LDM], sAr[cur][o + 2 * LDM], sAr[cur][o + 3 * LDM]};
                fa_i[t] = float4{sAi[cur][o], sAi[cur][o + LDM], sAi[cur][o + 2 * LDM], sAi[cur][o + 3 * LDM]};
            } else {
                fa_r[t] = *reinterpret_cast<const float4*>(&sAr[cur][(wr + 16 * t + r16) * LDK + 16 * kh + 4 * g]);
                fa_i[t] = *reinterpret_cast<const float4*>(&sAi[cur][(wr + 16 * t + r16) * LDK + 16 * kh + 4 * g]);
            }
        }
#pragma unroll
        for (int t = 0; t < TN; ++t) {
            if (KB) {
                const int o = (16 * kh + 4 * g) * LDN + wc + 16 * t + r16;
                fb_r[t] = float4{sBr[cur][o], sBr[cur][o + LDN], sBr[cur][o + 2 * LDN], sBr[cur][o + 3 * LDN]};
                fb_i[t] = float4{sBi[cur][o], sBi[cur][o + LDN], sBi[cur][o + 2 * LDN], sBi[cur][o + 3 * LDN]};
            } else {
                fb_r[t] = *reinterpret_cast<const float4*>(&sBr[cur][(wc + 16 * t + r16) * LDK + 16 * kh + 4 * g]);
                fb_i[t] = *reinterpret_cast<const float4*>(&sBi[cur][(wc + 16 * t + r16) * LDK + 16 * kh + 4 * g]);
            }
        }
        if (v.real) {
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int ti = 0; ti < TM; ++ti)
#pragma unroll
                    for (int tj = 0; tj < TN; ++tj)
                        p1[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                            (&fa_r[ti].x)[s], (&fb_r[tj].x)[s], p1[ti][tj], 0, 0, 0);
        } else if (M3) {
            // three passes over the tiles: the products into one accumulator
            // are TM TN independent MFMAs apart
#pragma unroll
            for (int s = 0; s < 4; ++s) {
#pragma unroll
                for (int ti = 0; ti < TM; ++ti)
#pragma unroll
                    for (int tj = 0; tj < TN; ++tj)
                        p1[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x4f32((&fa_r[ti].x)[s], (&fb_r[tj].x)[s],
                                                                          p1[ti][tj], 0, 0, 0);
#pragma unroll
                for (int ti = 0; ti < TM; ++ti)
#pragma unroll
                    for (int tj = 0; tj < TN; ++tj)
                        p2[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x4f32((&fa_i[ti].x)[s], (&fb_i[tj].x)[s],
                                                                          p2[ti][tj], 0, 0, 0);
#pragma unroll
                for (int ti = 0; ti < TM; ++ti) {
                    const float as = (&fa_r[ti].x)[s] + (&fa_i[ti].x)[s];
#pragma unroll
                    for (int tj = 0; tj < TN; ++tj)
                        p3[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                            as, (&fb_r[tj].x)[s] + (&fb_i[tj].x)[s], p3[ti][tj], 0, 0, 0);
                }
            }
        } else {
            // four-product form in two passes over the tiles (2 TM TN
            // independent MFMAs between the products into one accumulator)
#pragma unroll
            for (int s = 0; s < 4; ++s) {
#pragma unroll
                for (int ti = 0; ti < TM; ++ti)
#pragma unroll
                    for (int tj = 0; tj < TN; ++tj) {
                        const float ar = (&fa_r[ti].x)[s];
                        p1[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, (&fb_r[tj].x)[s], p1[ti][tj], 0, 0, 0);
                        p3[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, (&fb_i[tj].x)[s], p3[ti][tj], 0, 0, 0);
                    }
#pragma unroll
                for (int ti = 0; ti < TM; ++ti)
#pragma unroll
                    for (int tj = 0; tj < TN; ++tj) {
                        const float ai = (&fa_i[ti].x)[s];
                        p1[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x4f32(-ai, (&fb_i[tj].x)[s], p1[ti][tj], 0, 0, 0);
                        p3[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai, (&fb_r[tj].x)[s], p3[ti][tj], 0, 0, 0);
                    }
            }
        }
        }
        if (c + 1 < nk) ld.template store<LDK, KA, KB>(tid, StoreF32{sAr[cur ^ 1], sAi[cur ^ 1], sBr[cur ^ 1], sBi[cur ^ 1]});
        __syncthreads();
    }
    floatx4 accr[TM][TN], acci[TM][TN];
#pragma unroll
    for (int ti = 0; ti < TM; ++ti)
#pragma unroll
        for (int tj = 0; tj < TN; ++tj) {
            accr[ti][tj] = M3 ? p1[ti][tj] - p2[ti][tj] : p1[ti][tj];
            acci[ti][tj] = M3 ? p3[ti][tj] - p1[ti][tj] - p2[ti][tj] : p3[ti][tj];
        }
    write_tile<T>(v, p, m0, n0, wr, wc, lane, accr, acci);
}

template <int OPA, int OPB, class T, int BK>
__global__ __launch_bounds__(256) void k_cgemm_f32(CgemmArgs p)
{
    __shared__ __attribute__((aligned(16))) float smem[f32_smem_floats<T, BK>()];
    if (!apply_dyn(p)) return;
    int x, y, z;
    xcd_tile(x, y, z);  // z = kp * nslices + slice
    if (!slice_live(p, z % p.nslices) || y * T::BM >= m_live(p) || x * T::BN >= n_live(p)) return;
    cgemm_f32_tile<OPA, OPB, T, BK>(p, z % p.nslices, y * T::BM, x * T::BN, smem, z / p.nslices);
}

// C = sum over the ksplit partial products, in a fixed order
__global__ __launch_bounds__(256) void k_splitk_reduce(CgemmArgs p)
{
    if (!apply_dyn(p)) return;
    const long long mn = (long long)p.m * p.n, total = (long long)p.nslices * mn;
    const long long plane = (long long)p.ksplit * total;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const int s = (int)(e / mn);
        if (!slice_live(p, s)) continue;
        const long long r = e % mn;
        const int i = (int)(r / p.n), j = (int)(r % p.n);
        if (i >= m_live(p) || j >= n_live(p)) continue;  // not computed: left alone
        float vr = 0.0f, vi = 0.0f;
        for (int kp = 0; kp < p.ksplit; ++kp) {
            vr += p.part[kp * total + e];
            vi += p.part[plane + kp * total + e];
        }
        const bool real = (p.real_first && s == 0) || (p.real_last && s == p.nslices - 1);
        const long long off = s * p.sc + (long long)i * p.ldc + j;
        p.cr[off] = vr;
        p.ci[off] = real ? 0.0f : vi;
    }
}

// ------------------------------------------------------------ skinny FP32 --
// Narrow outputs with a long inner dimension: op(A) (m x k) B (k x n),
// n <= 64 and a multiple of 4, B not transposed (the range-finder
// products).  A workgroup of four wavefronts computes 64 output rows x all
// n columns over one inner-dimension part.  Each wavefront loads its 16 rows
// of op(A) straight from global memory into registers, already in the MFMA
// operand layout, with the next two 32-deep stages in flight while one is
// multiplied; B goes through LDS (one 32 x n stage, row-major with rows
// padded to 16 TN + 4 floats, shared by the four wavefronts,
// double-buffered): 16-byte stores, and the four 4-byte fragment reads of a
// lane fall in distinct banks.  3M complex form.  The MFMAs take
// the B fragment as their first operand, so that they accumulate the
// transposed 16 x 16 tile: lane (r, g) ends with output row r and the four
// columns 4g .. 4g+3 (one 16-byte store per plane).
//
// Operand layout of one 32-deep stage at k0, for lane (r, g) = (lane % 16,
// lane / 16): MFMA step (h, s), h = 0, 1 and s = 0 .. 3, takes inner index
// k0 + 16 h + 4 g + s, which is op(A)(row r, .) and B(., column r of the
// column tile); over the 8 steps each of the 32 inner indices enters once.
constexpr int kSkBK = 32;
template <int TN>
constexpr int sk_ldb()  // padded row of the B stage: 4 (16 TN + 4) = 16 mod 64 banks
{
    return 16 * TN + 4;
}
constexpr int kSkRows = 64;

struct AStage {
    float4 r[2], i[2];
};

// FAST: the whole stage lies inside the part and the row exists, and (OP_N)
// the planes allow 16-byte loads; no masks, so that no load sits behind a
// branch (a divergent load would make the compiler wait for every load in
// flight where the paths merge)
template <int OPA, bool FAST>
__device__ __forceinline__ void sk_load_a(AStage& a, const SliceView& v, const CgemmArgs& p, int row, int k0, int g,
                                          bool vec)
{
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int kb = k0 + 16 * h + 4 * g;
        if (OPA == OP_N) {
            const long long off = (long long)row * p.lda + kb;
            if (FAST) {
                a.r[h] = *reinterpret_cast<const float4*>(v.ar + off);
                a.i[h] = *reinterpret_cast<const float4*>(v.ai + off);
            } else {
                const int valid = row < p.m ? max(0, min(4, v.K - kb)) : 0;
                const Quad q = load4(v.ar, v.ai, off, valid, vec, false);
                a.r[h] = q.r;
                a.i[h] = q.i;
            }
        } else {  // A(k, row), A stored k x m; the conjugation of op(A) enters the arithmetic
            const int valid = FAST ? 4 : (row < p.m ? max(0, min(4, v.K - kb)) : 0);
            float xr[4], xi[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const long long off = (long long)(kb + s) * p.lda + row;
                xr[s] = FAST || s < valid ? v.ar[off] : 0.0f;
                xi[s] = FAST || s < valid ? v.ai[off] : 0.0f;
            }
            a.r[h] = make_float4(xr[0], xr[1], xr[2], xr[3]);
            a.i[h] = make_float4(xi[0], xi[1], xi[2], xi[3]);
        }
    }
}

template <int TN>
constexpr int sk_plane()  // one plane of one B buffer: NC = 16 TN staged columns
{
    return kSkBK * sk_ldb<TN>();
}

// the workgroup's tile (x = row tile) of slice view v; REAL: real slice
// (only the real planes enter).  TN: the 16-column blocks staged and
// multiplied; TW >= TN: the blocks written, those past TN as zeros.  RT:
// the live blocks are tl <= TN, tested at run time (else TN are live, a
// compile-time count, so that the MFMA chains carry no branches).
template <int OPA, int TN, int TW, bool REAL, bool FAST, bool RT>
__device__ __forceinline__ void sk_tile(const CgemmArgs& p, const SliceView& v, int x, int tl, float* lds)
{
    constexpr int NC = 16 * TN;                   // B columns staged (n rounded up to the tile)
    constexpr int GB = (kSkBK * NC / 4 + 255) / 256;  // 4-column groups of a B stage per thread
    constexpr int PL = sk_plane<TN>();
    constexpr int LDB = sk_ldb<TN>();
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = lane & 15, g = lane >> 4;
    const int row = x * kSkRows + 16 * wave + r;
    const bool veca = OPA == OP_N && vec_ok(v.ar, v.ai, p.lda);
    const bool vecb = vec_ok(v.br, v.bi, p.ldb);
    const int nst = (v.K - v.K0 + kSkBK - 1) / kSkBK;
    const int nl = n_live(p);             // live columns (a multiple of 4); the rest come out zero

    floatx4 p1[TN], p2[TN], p3[TN];
#pragma unroll
    for (int t = 0; t < TN; ++t) p1[t] = p2[t] = p3[t] = floatx4{0.f, 0.f, 0.f, 0.f};

    Quad bq[GB];
    bool bok[GB];  // FAST: the group lies in the stage and in the n columns (else stored as zeros)
#pragma unroll
    for (int u = 0; u < GB; ++u) {
        const int e = tid + 256 * u;
        bok[u] = e < kSkBK * NC / 4 && 4 * (e % (NC / 4)) < nl;
    }
    // B stage at k0 into registers (zero outside k < K and columns < n)
    auto load_b = [&](int k0) {
#pragma unroll
        for (int u = 0; u < GB; ++u) {
            const int e = tid + 256 * u;
            const int kr = e / (NC / 4), col = 4 * (e % (NC / 4));
            const int k = k0 + kr;
            if (FAST) {  // clamped in-range load; the mask is applied when it is stored
                const long long off = (long long)(bok[u] ? k : k0) * p.ldb + (bok[u] ? col : 0);
                bq[u].r = *reinterpret_cast<const float4*>(v.br + off);
                bq[u].i = *reinterpret_cast<const float4*>(v.bi + off);
            } else {
                const int valid = (e < kSkBK * NC / 4 && k < v.K) ? max(0, min(4, nl - col)) : 0;
                bq[u] = load4(v.br, v.bi, (long long)k * p.ldb + col, valid, vecb, false);
            }
        }
    };
    // the staged registers into LDS buffer buf (row k, 4 columns per store)
    auto store_b = [&](int buf) {
        float* br = lds + buf * 2 * PL;
        float* bi = br + PL;
#pragma unroll
        for (int u = 0; u < GB; ++u) {
            const int e = tid + 256 * u;
            if (e < kSkBK * NC / 4) {
                const int kr = e / (NC / 4), col = 4 * (e % (NC / 4));
                if (FAST && !bok[u]) bq[u].r = bq[u].i = make_float4(0.f, 0.f, 0.f, 0.f);
                *reinterpret_cast<float4*>(br + kr * LDB + col) = bq[u].r;
                *reinterpret_cast<float4*>(bi + kr * LDB + col) = bq[u].i;
            }
        }
    };
    auto compute = [&](const AStage& a, int buf) {
        const float* br = lds + buf * 2 * PL;
        const float* bi = br + PL;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            float4 fr[TN], fi[TN];
#pragma unroll
            for (int t = 0; t < TN; ++t) {
                if (RT && t >= tl) continue;
                const int off = (16 * h + 4 * g) * LDB + 16 * t + r;
                fr[t] = make_float4(br[off], br[off + LDB], br[off + 2 * LDB], br[off + 3 * LDB]);
                fi[t] = make_float4(bi[off], bi[off + LDB], bi[off + 2 * LDB], bi[off + 3 * LDB]);
            }
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                // OP_C: ai is Im A(k, row), op(A) has -ai; p2 then holds +sum b_i ai
                const float ar = (&a.r[h].x)[s], ai = (&a.i[h].x)[s];
                const float as = OPA == OP_C ? ar - ai : ar + ai;
#pragma unroll
                for (int t = 0; t < TN; ++t) {
                    if (RT && t >= tl) continue;
                    const float b_r = (&fr[t].x)[s], b_i = (&fi[t].x)[s];
                    p1[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(b_r, ar, p1[t], 0, 0, 0);
                    if (!REAL) {
                        p2[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(b_i, ai, p2[t], 0, 0, 0);
                        p3[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(b_r + b_i, as, p3[t], 0, 0, 0);
                    }
                }
            }
        }
    };
    // stage st: publish B stage st+1 (loaded during stage st-1), prefetch B
    // stage st+2 (registers) and then A stage st+2 (into nxt2, the slot stage
    // st-1 used), multiply stage st.  Loads complete in issue order, so the
    // one wait (for B stage st+1, at the top) leaves A stage st+1 in flight;
    // the scheduling barriers keep that order.  Prefetches past the end
    // re-read the last stage (never used), so that no load sits behind a
    // branch.
    auto body = [&](int st, const AStage& cur, AStage& nxt2) {
        store_b((st + 1) & 1);
        const int nx = min(st + 2, nst - 1);
        load_b(v.K0 + kSkBK * nx);
        __builtin_amdgcn_sched_barrier(0);
        sk_load_a<OPA, FAST>(nxt2, v, p, row, v.K0 + kSkBK * nx, g, veca);
        __builtin_amdgcn_sched_barrier(0);
        compute(cur, st & 1);
        __syncthreads();
    };

    // prologue in the loop's issue order (B stage 1 before A stage 1), so
    // that the loads in flight where the loop starts are those of its
    // steady state and the first wait of each pass leaves A in flight
    AStage a0, a1, a2;
    if (nst > 0) {
        load_b(v.K0);
        __builtin_amdgcn_sched_barrier(0);
        sk_load_a<OPA, FAST>(a0, v, p, row, v.K0, g, veca);
        __builtin_amdgcn_sched_barrier(0);
        store_b(0);
        load_b(v.K0 + kSkBK * min(1, nst - 1));
        __builtin_amdgcn_sched_barrier(0);
        sk_load_a<OPA, FAST>(a1, v, p, row, v.K0 + kSkBK * min(1, nst - 1), g, veca);
        __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();
    int st = 0;
    for (; st + 3 <= nst; st += 3) {
        body(st, a0, a2);
        body(st + 1, a1, a0);
        body(st + 2, a2, a1);
    }
    if (st < nst) body(st, a0, a2);
    if (st + 1 < nst) body(st + 1, a1, a0);

    // epilogue: lane (r, g) holds row `row`, columns 16 t + 4 g .. + 3
    if (row < p.m) {
        const bool vecc = ((reinterpret_cast<unsigned long long>(v.cr) | reinterpret_cast<unsigned long long>(v.ci)) &
                           15) == 0 &&
                          (v.ldc & 3) == 0;
#pragma unroll
        for (int t = 0; t < TW; ++t) {
            const int col = 16 * t + 4 * g;
            if (col < p.n) {  // n is a multiple of 4: all four columns in range
                // 3M: Re = p1 - p2, Im = p3 - p1 - p2 (OP_C: p2 has the opposite sign)
                floatx4 cre = floatx4{0.f, 0.f, 0.f, 0.f}, cim = cre;
                if (t < TN) {
                    const floatx4 q2 = OPA == OP_C ? -p2[t] : p2[t];
                    cre = REAL ? p1[t] : p1[t] - q2;
                    cim = REAL ? floatx4{0.f, 0.f, 0.f, 0.f} : p3[t] - p1[t] - q2;
                }
                const long long off = (long long)row * v.ldc + col;
                if (vecc) {
                    *reinterpret_cast<floatx4*>(v.cr + off) = cre;
                    *reinterpret_cast<floatx4*>(v.ci + off) = cim;
                } else {
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        v.cr[off + j] = cre[j];
                        v.ci[off + j] = cim[j];
                    }
                }
            }
        }
    }
}

// The tile with the live column blocks of the launch (tl <= TNI) as a
// compile-time count: TNI, or fewer for a device-capped width.  The
// conjugated-A form keeps one body per width with a run-time count: its
// element-wise A loads leave no registers for the extra bodies.
template <int OPA, int TNI, int TW>
__device__ __forceinline__ void sk_live(const CgemmArgs& p, const SliceView& v, int x, bool fast, int tl, float* lds)
{
    constexpr bool RT = OPA == OP_C;
    if constexpr (TNI > 1 && !RT) {
        if (tl < TNI) {
            sk_live<OPA, TNI - 1, TW>(p, v, x, fast, tl, lds);
            return;
        }
    }
    if (v.real) {
        if (fast)
            sk_tile<OPA, TNI, TW, true, true, RT>(p, v, x, tl, lds);
        else
            sk_tile<OPA, TNI, TW, true, false, RT>(p, v, x, tl, lds);
    } else {
        if (fast)
            sk_tile<OPA, TNI, TW, false, true, RT>(p, v, x, tl, lds);
        else
            sk_tile<OPA, TNI, TW, false, false, RT>(p, v, x, tl, lds);
    }
}

// three wavefronts per SIMD for the 48- and 64-column tiles (they fit
// without spills; measured 6% faster than the two their default allocation
// allows)
template <int OPA, int TN>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(TN >= 3 ? 3 : 1, TN >= 3 ? 3 : 10))) void
k_skinny(CgemmArgs p)
{
    __shared__ __attribute__((aligned(16))) float lds[2 * 2 * sk_plane<TN>()];
    if (!apply_dyn(p)) return;
    int x, y, z;
    xcd_tile(x, y, z);  // x = row tile, z = kp * nslices + slice
    if (!slice_live(p, z % p.nslices) || x * kSkRows >= m_live(p)) return;
    const SliceView v = slice_view(p, z % p.nslices, z / p.nslices);
    const bool fast = (x + 1) * kSkRows <= p.m && (v.K - v.K0) % kSkBK == 0 && vec_ok(v.br, v.bi, p.ldb) &&
                      (OPA == OP_C || vec_ok(v.ar, v.ai, p.lda));
    const int tl = (n_live(p) + 15) / 16;  // live 16-column blocks (uniform, 1 .. TN)
    // a device-capped width of at most 48 columns writes the 48 columns of
    // the three-block tile (the blocks past the live ones as zeros)
    if constexpr (TN == 4) {
        if (p.dyn_n && tl <= 3) {
            sk_live<OPA, 3, 3>(p, v, x, fast, tl, lds);
            return;
        }
    }
    sk_live<OPA, TN, TN>(p, v, x, fast, tl, lds);
}

// -------------------------------------------------------------- wide FP32 --
// Products with a short inner dimension: A (m x k, k <= 64) times B (k x n),
// neither transposed (the reconstruction W = Q M1 of the randomized SVT, and
// with at most 64 output columns the products by R^-1 and the Ritz bases).
// A workgroup of four wavefronts covers 64 rows x 256 columns (x 64 columns,
// masked, for the narrow outputs).  Each wavefront keeps its 16 rows of A in registers, in the MFMA
// operand layout of k_skinny (loaded once), and walks the four 64-column
// blocks; the k x 64 block of B goes through LDS (row-major, rows padded to
// 68 floats, double-buffered: the next block's loads are in flight while
// this one is multiplied), and the results leave as 16-byte stores while the
// next block's MFMAs run.  Full tiles only (m a multiple of 64, n of 256,
// 16-byte aligned planes and rows); 3M complex form.
constexpr int kWideRows = 64, kWideCols = 256, kWideBlk = 64, kWideMaxK = 64;
constexpr int kWideLDB = kWideBlk + 4;  // 4 x 68 = 16 mod 64 banks: a lane's four fragment reads hit distinct banks

// KC: staged inner rows (the live k rounded up to 16, a compile-time count;
// zero beyond k)
// NB: 64-column blocks per workgroup (4: the unmasked full tiles; 1: a
// masked tile for narrow outputs, rows < m and columns < n, n a multiple of 4)
// TW: the 16-column groups of a block that are computed and stored (4, or
// fewer in the masked tile for a device-capped n; the rest are left alone)
template <bool REAL, int KC, int NB, int TW = 4>
__device__ __forceinline__ void wide_tile(const CgemmArgs& p, const SliceView& v, int x, int y, float* lds)
{
    constexpr bool MASK = NB == 1;
    static_assert(TW >= 1 && TW <= 4 && (MASK || TW == 4), "column groups");
    constexpr int GB = KC * (kWideBlk / 4) / 256;  // 4-column groups of a B block per thread
    constexpr int nh = KC / 16;
    constexpr int PL = KC * kWideLDB;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = lane & 15, g = lane >> 4;
    const int row = y * kWideRows + 16 * wave + r;
    const int K = v.K;
    const int n0 = x * kWideBlk * NB;

    // A: chunk h holds A(row, 16 h + 4 g + s), s = 0..3
    float fa_r[nh * 4], fa_i[nh * 4];
    const bool veca = vec_ok(v.ar, v.ai, p.lda);
    auto put_a = [&](int h, const float4& qr, const float4& qi) __attribute__((always_inline)) {
        fa_r[4 * h + 0] = qr.x;
        fa_r[4 * h + 1] = qr.y;
        fa_r[4 * h + 2] = qr.z;
        fa_r[4 * h + 3] = qr.w;
        fa_i[4 * h + 0] = qi.x;
        fa_i[4 * h + 1] = qi.y;
        fa_i[4 * h + 2] = qi.z;
        fa_i[4 * h + 3] = qi.w;
    };
    float4 bq_r[GB], bq_i[GB];
    bool bok[GB];  // MASK: the group's columns exist (else stored as zeros)
    // B block j into registers: rows beyond K read row K-1 (kept in range) and are zeroed when stored
    auto load_b = [&](int j) __attribute__((always_inline)) {
#pragma unroll
        for (int u = 0; u < GB; ++u) {
            const int e = tid + 256 * u;
            {
                const int kr = min(e / (kWideBlk / 4), K - 1);
                int col = n0 + kWideBlk * j + 4 * (e % (kWideBlk / 4));
                bok[u] = !MASK || col < p.n;
                if (MASK && !bok[u]) col = 0;  // an in-range group, zeroed when stored
                const long long off = (long long)kr * p.ldb + col;
                bq_r[u] = *reinterpret_cast<const float4*>(v.br + off);
                bq_i[u] = *reinterpret_cast<const float4*>(v.bi + off);
            }
        }
    };
    auto store_b = [&](int buf) __attribute__((always_inline)) {
        float* br = lds + buf * 2 * PL;
        float* bi = br + PL;
#pragma unroll
        for (int u = 0; u < GB; ++u) {
            const int e = tid + 256 * u;
            {
                const int kr = e / (kWideBlk / 4), c = 4 * (e % (kWideBlk / 4));
                float4 qr = bq_r[u], qi = bq_i[u];  // by value: a select of two lvalues would go through memory
                if (kr >= K || !bok[u]) qr = qi = make_float4(0.f, 0.f, 0.f, 0.f);
                *reinterpret_cast<float4*>(br + kr * kWideLDB + c) = qr;
                *reinterpret_cast<float4*>(bi + kr * kWideLDB + c) = qi;
            }
        }
    };
    const bool vecc = ((reinterpret_cast<unsigned long long>(v.cr) | reinterpret_cast<unsigned long long>(v.ci)) &
                       15) == 0 &&
                      (v.ldc & 3) == 0;

    // the one-block tile issues B block 0 first, so that the A loads (and
    // any wait the A path's selects need) queue behind it rather than ahead
    // of it (the four-block tile loads A first: B's registers live across
    // the A loads would spill it)
    if constexpr (NB == 1) load_b(0);
    if (veca && K == KC && (!MASK || (y + 1) * kWideRows <= p.m)) {
        // every chunk whole and every row present: plain 16-byte loads, all
        // in flight together (the masked form below waits between chunks)
#pragma unroll
        for (int h = 0; h < nh; ++h) {
            const long long off = (long long)row * p.lda + 16 * h + 4 * g;
            put_a(h, *reinterpret_cast<const float4*>(v.ar + off), *reinterpret_cast<const float4*>(v.ai + off));
        }
    } else {
#pragma unroll
        for (int h = 0; h < nh; ++h) {
            const int kb = 16 * h + 4 * g;
            const int valid = MASK && row >= p.m ? 0 : max(0, min(4, K - kb));
            const Quad q = load4(v.ar, v.ai, (long long)row * p.lda + kb, valid, veca, false);
            put_a(h, q.r, q.i);
        }
    }
    if constexpr (NB > 1) load_b(0);
    store_b(0);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        const bool more = j + 1 < NB;
        if (more) load_b(j + 1);
        floatx4 p1[4], p2[4], p3[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) p1[t] = p2[t] = p3[t] = floatx4{0.f, 0.f, 0.f, 0.f};
        const float* br = lds + (j & 1) * 2 * PL;
        const float* bi = br + PL;
#pragma unroll
        for (int h = 0; h < nh; ++h) {
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const float ar = fa_r[4 * h + s], ai = fa_i[4 * h + s];
                const float as = ar + ai;
                const int off = (16 * h + 4 * g + s) * kWideLDB + r;
#pragma unroll
                for (int t = 0; t < TW; ++t) {
                    const float b_r = br[off + 16 * t], b_i = bi[off + 16 * t];
                    p1[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(b_r, ar, p1[t], 0, 0, 0);
                    if (!REAL) {
                        p2[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(b_i, ai, p2[t], 0, 0, 0);
                        p3[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(b_r + b_i, as, p3[t], 0, 0, 0);
                    }
                }
            }
            // one chunk's fragments live at a time (the scheduler would hoist them all)
            __builtin_amdgcn_sched_barrier(0);
        }
        // the next B block into the other buffer before this block's stores:
        // its wait then covers only its own loads (stores count in the same
        // counter and would be waited for too)
        if (more) store_b((j + 1) & 1);
        __builtin_amdgcn_sched_barrier(0);
        // lane (r, g) holds row `row`, columns 16 t + 4 g .. + 3 of the block
#pragma unroll
        for (int t = 0; t < TW; ++t) {
            const floatx4 cre = REAL ? p1[t] : p1[t] - p2[t];
            const floatx4 cim = REAL ? floatx4{0.f, 0.f, 0.f, 0.f} : p3[t] - p1[t] - p2[t];
            const int col = n0 + kWideBlk * j + 16 * t + 4 * g;
            if (MASK && (row >= p.m || col >= p.n)) continue;  // n a multiple of 4: all four columns or none
            const long long off = (long long)row * v.ldc + col;
            if (vecc) {
                *reinterpret_cast<floatx4*>(v.cr + off) = cre;
                *reinterpret_cast<floatx4*>(v.ci + off) = cim;
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    v.cr[off + q] = cre[q];
                    v.ci[off + q] = cim[q];
                }
            }
        }
        __syncthreads();
    }
}

// the tile at the inner depth of the launch's live k (kc <= KC, a multiple
// of 16), so that no MFMA chain waits behind a branch on a device-capped k
template <int KC, int NB>
__device__ __forceinline__ void wide_live(const CgemmArgs& p, const SliceView& v, int x, int y, int kc, float* lds)
{
    if constexpr (KC > 16) {
        if (kc < KC) {
            wide_live<KC - 16, NB>(p, v, x, y, kc, lds);
            return;
        }
    }
    if constexpr (NB == 1) {
        // the 16-column groups of the device-capped n (the one block of the masked tile)
        const int tw = (n_live(p) + 15) / 16;
        if (tw <= 1)
            v.real ? wide_tile<true, KC, NB, 1>(p, v, x, y, lds) : wide_tile<false, KC, NB, 1>(p, v, x, y, lds);
        else if (tw == 2)
            v.real ? wide_tile<true, KC, NB, 2>(p, v, x, y, lds) : wide_tile<false, KC, NB, 2>(p, v, x, y, lds);
        else if (tw == 3)
            v.real ? wide_tile<true, KC, NB, 3>(p, v, x, y, lds) : wide_tile<false, KC, NB, 3>(p, v, x, y, lds);
        else
            v.real ? wide_tile<true, KC, NB, 4>(p, v, x, y, lds) : wide_tile<false, KC, NB, 4>(p, v, x, y, lds);
    } else {
        if (v.real)
            wide_tile<true, KC, NB>(p, v, x, y, lds);
        else
            wide_tile<false, KC, NB>(p, v, x, y, lds);
    }
}

// three wavefronts per SIMD for the four-block tile (no spills; measured 7%
// faster than two)
template <int KC, int NB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NB > 1 ? 3 : 1, NB > 1 ? 3 : 10))) void
k_wide(CgemmArgs p)
{
    __shared__ __attribute__((aligned(16))) float wlds[(NB > 1 ? 2 : 1) * 2 * KC * kWideLDB];
    if (!apply_dyn(p)) return;
    int x, y, z;
    xcd_tile(x, y, z);  // x = column group (64 NB), y = 64-row tile, z = slice
    if (!slice_live(p, z) || y * kWideRows >= m_live(p) || x * kWideBlk * NB >= n_live(p)) return;
    const SliceView v = slice_view(p, z, 0);
    wide_live<KC, NB>(p, v, x, y, (v.K + 15) / 16 * 16, wlds);
}

// Batched products of uneven shapes: a persistent grid walks a list of
// output tiles, each naming its product (items[unit.item]), slice, tile
// origin and operand forms.
template <class T>
__global__ __launch_bounds__(256) void k_cgemm_batch(const CgemmArgs* __restrict__ items,
                                                     const GemmUnit* __restrict__ units, int nunits)
{
    __shared__ __attribute__((aligned(16))) float smem[f32_smem_floats<T>()];
    for (int u = blockIdx.x; u < nunits; u += gridDim.x) {
        const GemmUnit w = units[u];
        const CgemmArgs p = items[w.item];
        __syncthreads();
        switch (w.op) {
            case GEMM_CN: cgemm_f32_tile<OP_C, OP_N, T>(p, w.slice, w.m0, w.n0, smem); break;
            case GEMM_NC: cgemm_f32_tile<OP_N, OP_C, T>(p, w.slice, w.m0, w.n0, smem); break;
            default: cgemm_f32_tile<OP_N, OP_N, T>(p, w.slice, w.m0, w.n0, smem); break;
        }
    }
}

// ------------------------------------------------------------- BF16 (x3) --
// Slice products on the bf16 planes of the forward transform (hi = bf16(x)
// and, when splitting, lo = bf16(x - hi) of every real and imaginary part).
// Rows of op(A) and columns of op(B) both hold the inner index contiguous,
// k-blocked by the stage depth and padded with zeros to a whole block, so
// one stage of a run of rows is one contiguous span and every operand moves
// in 16-byte groups of 8 values straight from global memory into LDS
// (global_load_lds, 1 KB per wavefront instruction, no registers, no
// conversion) and from LDS into v_mfma_f32_16x16x32_bf16.
// Per output, the products hi*hi, hi*lo, lo*hi of each real product
// accumulate in FP32 in that order.
//
// Pipeline: S LDS stages of 32 inner-dimension values; the loads of stage
// c+S-1 are in flight while stage c is multiplied, one barrier per stage.
// LDS rows are 64 bytes (four 16-byte groups); group g of row R sits in slot
// g ^ ((R >> 1) & 3).  The MFMA fragment read (lane = 16 g + r, 16 bytes of
// row R0 + r at group g) then runs at the full 256 bytes per clock without
// bank conflicts; unswizzled 64-byte rows, and rows padded to 80 bytes,
// measured one conflict cycle per clock of the read on gfx950.
//
// Workgroups: one per tile of a complex slice, then groups of rpw tiles of
// the real slices (a real tile issues a quarter of the products of a
// complex one), so that the real DC and Nyquist slices of the t-product do
// not take a round of the GPU of their own.  XCD-aware numbering: the
// hardware deals workgroup ids round-robin to the 8 XCDs; XCD x takes one
// contiguous run of tiles (neighbouring tiles of one slice share panels of
// A or B in its L2).

template <int BM_, int BN_, int WGM_, int WGN_>
struct BTile {
    static constexpr int BM = BM_, BN = BN_, WGM = WGM_, WGN = WGN_;
    static constexpr int NW = WGM * WGN, NT = 64 * NW;
    static constexpr int WM = BM / WGM, WN = BN / WGN, TM = WM / 16, TN = WN / 16;
    static_assert(TM >= 1 && TN >= 1 && WM % 16 == 0 && WN % 16 == 0, "16 x 16 MFMA tiles");
};
using B64x64 = BTile<64, 64, 2, 2>;      // wavefront tile 32 x 32
using B128x32 = BTile<128, 32, 4, 1>;    // 32 x 32
using B128x128 = BTile<128, 128, 2, 4>;  // 64 x 32, eight wavefronts

constexpr int kBK = 32;  // inner-dimension values per stage (one MFMA step), 64-byte LDS rows

// stages: as many as fit kLdsBudget bytes (at most 4, at least 2)
template <class T, bool SPLIT>
constexpr int bf16_stage_elems()
{
    return (SPLIT ? 4 : 2) * (T::BM + T::BN) * kBK;
}
template <class T, bool SPLIT>
constexpr int bf16_stages()
{
    constexpr int budget = T::NW == 8 ? 128 * 1024 : 80 * 1024;
    constexpr int n = budget / (2 * bf16_stage_elems<T, SPLIT>());
    return n > 4 ? 4 : (n < 2 ? 2 : n);
}

typedef __attribute__((address_space(3))) void* lds_ptr;

__device__ __forceinline__ int swz(int r) { return (r >> 1) & 3; }

// wait until at most n of this wavefront's global loads are outstanding
// (gfx9 s_waitcnt encoding: vmcnt in bits 3:0 and 15:14, the other counters
// left at their maxima)
template <int N>
__device__ __forceinline__ void wait_vm()
{
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// workgroup barrier without a memory fence: LDS written by the global loads
// is covered by each wavefront's own wait_vm before it; the wavefront's LDS
// reads have all returned (lgkmcnt 0) before it arrives, so no buffer is
// refilled under a read in flight
__device__ __forceinline__ void barrier_only()
{
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt((15) | (3 << 14) | (7 << 4) | (0 << 8));
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

#define TP_MFMA_BF16(a, b, c)                                                                                  \
    __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, (a)), __builtin_bit_cast(bf16x8, (b)), \
                                            (c), 0, 0, 0)

__device__ __forceinline__ shortx8 neg_bf16x8(shortx8 v)
{
    return v ^ (shortx8){(short)0x8000, (short)0x8000, (short)0x8000, (short)0x8000,
                         (short)0x8000, (short)0x8000, (short)0x8000, (short)0x8000};
}

// One BM x BN output tile of slice s at (m0, n0).  Planes used: complex
// (hi re, hi im[, lo re, lo im]); real (hi re[, lo re]).  A stage holds the
// NPU planes of the A panel (BM rows each), then those of the B panel.
template <class T, bool SPLIT, bool CPLX>
__device__ __forceinline__ void bf16_tile(const Bf16Args& p, int s, int m0, int n0, unsigned short* lds)
{
    constexpr int BM = T::BM, BN = T::BN, TM = T::TM, TN = T::TN, NW = T::NW;
    constexpr int S = bf16_stages<T, SPLIT>(), STAGE = bf16_stage_elems<T, SPLIT>();
    constexpr int NPU = (SPLIT ? 2 : 1) * (CPLX ? 2 : 1);
    constexpr int RA = NPU * BM, RB = NPU * BN;  // LDS rows of a stage used by this tile
    constexpr int NBLK = (RA + RB) / 16;          // 1 KB blocks (16 rows) per stage
    constexpr int LPW = (NBLK + NW - 1) / NW;     // loads per wavefront per stage (at most)
    constexpr int LPW_MIN = NBLK / NW;            // (at least)
    static_assert(BM % 16 == 0 && BN % 16 == 0, "16-row blocks");
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = (wave / T::WGN) * T::WM, wc = (wave % T::WGN) * T::WN;
    const int g = lane >> 4, r16 = lane & 15;
    // used plane u -> stored plane
    auto stored = [](int u) { return CPLX ? u : 2 * u; };

    // this lane's part of a block: row lane/4, LDS slot lane%4, which holds
    // the 16-byte group (lane%4) ^ swz(row) of the row
    const int brow = lane >> 2, bgrp = (lane & 3) ^ swz(lane >> 2);
    const unsigned short* A = p.a + (long long)s * p.a_slice + bgrp * 8;
    const unsigned short* B = p.b + (long long)s * p.b_slice + bgrp * 8;
    auto issue = [&](int buf, int k0) {
#pragma unroll
        for (int j = 0; j < LPW; ++j) {
            const int b = wave + j * NW;
            if (j < LPW_MIN || b < NBLK) {
                const unsigned short* src;
                if (b < RA / 16) {
                    const int u = b / (BM / 16), r = min(m0 + (b % (BM / 16)) * 16 + brow, p.m - 1);
                    src = A + stored(u) * p.a_plane + (long long)(k0 / kBK) * p.m * kBK + (long long)r * kBK;
                } else {
                    const int bb = b - RA / 16;
                    const int u = bb / (BN / 16), r = min(n0 + (bb % (BN / 16)) * 16 + brow, p.n - 1);
                    src = B + stored(u) * p.b_plane + (long long)(k0 / kBK) * p.n * kBK + (long long)r * kBK;
                }
                __builtin_amdgcn_global_load_lds((void*)src, (lds_ptr)(lds + buf * STAGE + b * 512), 16, 0, 0);
            }
        }
    };

    floatx4 accr[TM][TN], acci[TM][TN];
#pragma unroll
    for (int ti = 0; ti < TM; ++ti)
#pragma unroll
        for (int tj = 0; tj < TN; ++tj) {
            accr[ti][tj] = floatx4{0.f, 0.f, 0.f, 0.f};
            acci[ti][tj] = floatx4{0.f, 0.f, 0.f, 0.f};
        }

    // fragment of row R (a multiple of 16 plus r16): 16 bytes at slot g ^ swz(r16)
    const int foff = r16 * kBK + ((g ^ swz(r16)) * 8);
    const int nk = (p.k + kBK - 1) / kBK;
#pragma unroll
    for (int st = 0; st < S - 1; ++st)
        if (st < nk) issue(st, st * kBK);
    for (int c = 0; c < nk; ++c) {
        // stage c has landed once at most the later stages' loads are outstanding
        if (c + S - 2 < nk)
            wait_vm<LPW_MIN * (S - 2)>();
        else
            wait_vm<0>();
        barrier_only();  // stage c complete everywhere; stage c-1 no longer read
        if (c + S - 1 < nk) issue((c + S - 1) % S, (c + S - 1) * kBK);
        const unsigned short* sA = lds + (c % S) * STAGE;
        const unsigned short* sB = sA + RA * kBK;
        // 16x16x32 operands: lane (g, r16) holds k = 8g .. 8g+7 of row (column) r16.
        // Row tiles in pairs, so that four accumulators rotate between
        // dependent products.
        constexpr int TP = TM < 2 ? TM : 2;
#pragma unroll
        for (int t0 = 0; t0 < TM; t0 += TP) {
            shortx8 fa[TP][NPU];
#pragma unroll
            for (int i = 0; i < TP; ++i)
#pragma unroll
                for (int u = 0; u < NPU; ++u)
                    fa[i][u] = *reinterpret_cast<const shortx8*>(sA + (u * BM + wr + 16 * (t0 + i)) * kBK + foff);
#pragma unroll
            for (int tj = 0; tj < TN; ++tj) {
                shortx8 fb[NPU];
#pragma unroll
                for (int u = 0; u < NPU; ++u)
                    fb[u] = *reinterpret_cast<const shortx8*>(sB + (u * BN + wc + 16 * tj) * kBK + foff);
                if constexpr (CPLX) {
                    // Cr += Ar Br - Ai Bi, Ci += Ar Bi + Ai Br for each (a-part, b-part)
                    const shortx8 nb1 = neg_bf16x8(fb[1]);
#define TP_CTERM(ar, ai, br, bi, nbi)                                                                  \
    _Pragma("unroll") for (int i = 0; i < TP; ++i) accr[t0 + i][tj] = TP_MFMA_BF16(ar, br, accr[t0 + i][tj]); \
    _Pragma("unroll") for (int i = 0; i < TP; ++i) acci[t0 + i][tj] = TP_MFMA_BF16(ar, bi, acci[t0 + i][tj]); \
    _Pragma("unroll") for (int i = 0; i < TP; ++i) accr[t0 + i][tj] = TP_MFMA_BF16(ai, nbi, accr[t0 + i][tj]); \
    _Pragma("unroll") for (int i = 0; i < TP; ++i) acci[t0 + i][tj] = TP_MFMA_BF16(ai, br, acci[t0 + i][tj]);
                    TP_CTERM(fa[i][0], fa[i][1], fb[0], fb[1], nb1)  // hi * hi
                    if constexpr (SPLIT) {
                        const shortx8 nb3 = neg_bf16x8(fb[3]);
                        TP_CTERM(fa[i][0], fa[i][1], fb[2], fb[3], nb3)  // hi * lo
                        TP_CTERM(fa[i][2], fa[i][3], fb[0], fb[1], nb1)  // lo * hi
                    }
#undef TP_CTERM
                } else {
#pragma unroll
                    for (int i = 0; i < TP; ++i) accr[t0 + i][tj] = TP_MFMA_BF16(fa[i][0], fb[0], accr[t0 + i][tj]);
                    if constexpr (SPLIT) {
#pragma unroll
                        for (int i = 0; i < TP; ++i)
                            accr[t0 + i][tj] = TP_MFMA_BF16(fa[i][0], fb[1], accr[t0 + i][tj]);
#pragma unroll
                        for (int i = 0; i < TP; ++i)
                            accr[t0 + i][tj] = TP_MFMA_BF16(fa[i][1], fb[0], accr[t0 + i][tj]);
                    }
                }
            }
        }
    }
    // every wavefront is done with the last stage before LDS is reused
    __syncthreads();

    float* cr = p.cr + (long long)s * p.sc;
    float* ci = p.ci + (long long)s * p.sc;
#pragma unroll
    for (int ti = 0; ti < TM; ++ti)
#pragma unroll
        for (int tj = 0; tj < TN; ++tj)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int row = m0 + wr + 16 * ti + 4 * g + j, col = n0 + wc + 16 * tj + r16;
                if (row < p.m && col < p.n) {
                    const long long off = (long long)row * p.ldc + col;
                    cr[off] = accr[ti][tj][j];
                    ci[off] = CPLX ? acci[ti][tj][j] : 0.0f;
                }
            }
}

template <class T, bool SPLIT>
__global__ __launch_bounds__(T::NT) void k_cgemm_bf16(Bf16Args p)
{
    __shared__ __attribute__((aligned(1024))) unsigned short lds[bf16_stages<T, SPLIT>() * bf16_stage_elems<T, SPLIT>()];
    const int ntn = (p.n + T::BN - 1) / T::BN, tps = ((p.m + T::BM - 1) / T::BM) * ntn;
    const int nct = p.ncs * tps, nrt = p.nreal * tps;
    const int total = gridDim.x, w = blockIdx.x, x = w & 7;
    const int t = x * (total >> 3) + min(x, total & 7) + (w >> 3);
    if (t < nct) {
        const int rem = t % tps;
        bf16_tile<T, SPLIT, true>(p, p.cs0 + t / tps, (rem / ntn) * T::BM, (rem % ntn) * T::BN, lds);
        return;
    }
    const int r0 = (t - nct) * p.rpw, r1 = min(nrt, r0 + p.rpw);
    for (int r = r0; r < r1; ++r) {
        const int rem = r % tps;
        bf16_tile<T, SPLIT, false>(p, p.real_s[r / tps], (rem / ntn) * T::BM, (rem % ntn) * T::BN, lds);
    }
}

// The same products on v_mfma_f32_32x32x16_bf16 (32 x 32 outputs per
// instruction, 16 inner-dimension values): stages of 16 values, so that
// larger tiles (fewer operand bytes through L2 per product) still fit
// several stages in LDS.  LDS rows are 32 bytes (two 16-byte halves); half h
// of row R sits in slot h ^ ((R >> 3) & 1), which measured free of bank
// conflicts for the fragment read (lane = 32 h + r, row R0 + r).
template <int BM_, int BN_, int WGM_, int WGN_>
struct BTile32 {
    static constexpr int BM = BM_, BN = BN_, WGM = WGM_, WGN = WGN_;
    static constexpr int NW = WGM * WGN, NT = 64 * NW;
    static constexpr int WM = BM / WGM, WN = BN / WGN, TM = WM / 32, TN = WN / 32;
    static_assert(TM >= 1 && TN >= 1 && WM % 32 == 0 && WN % 32 == 0, "32 x 32 MFMA tiles");
};
using C256x128 = BTile32<256, 128, 4, 2>;  // wavefront tile 64 x 64, eight wavefronts
using C128x128 = BTile32<128, 128, 2, 2>;  // 64 x 64

constexpr int kBK32 = 16;  // inner-dimension values per stage of the 32 x 32 kernel

template <class T, bool SPLIT>
constexpr int bf16w_stage_elems()
{
    return (SPLIT ? 4 : 2) * (T::BM + T::BN) * kBK32;
}
template <class T, bool SPLIT>
constexpr int bf16w_stages()
{
    constexpr int budget = T::NW == 8 ? 144 * 1024 : 80 * 1024;
    constexpr int n = budget / (2 * bf16w_stage_elems<T, SPLIT>());
    return n > 4 ? 4 : (n < 2 ? 2 : n);
}

typedef float floatx16 __attribute__((ext_vector_type(16)));

#define TP_MFMA32_BF16(a, b, c)                                                                                \
    __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, (a)), __builtin_bit_cast(bf16x8, (b)), \
                                            (c), 0, 0, 0)

template <class T, bool SPLIT, bool CPLX>
__device__ __forceinline__ void bf16w_tile(const Bf16Args& p, int s, int m0, int n0, unsigned short* lds)
{
    constexpr int BM = T::BM, BN = T::BN, TM = T::TM, TN = T::TN, NW = T::NW;
    constexpr int S = bf16w_stages<T, SPLIT>(), STAGE = bf16w_stage_elems<T, SPLIT>();
    constexpr int NPU = (SPLIT ? 2 : 1) * (CPLX ? 2 : 1);
    constexpr int RA = NPU * BM, RB = NPU * BN;  // LDS rows of a stage used by this tile
    constexpr int NBLK = (RA + RB) / 32;          // 1 KB blocks (32 rows) per stage
    constexpr int LPW = (NBLK + NW - 1) / NW, LPW_MIN = NBLK / NW;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = (wave / T::WGN) * T::WM, wc = (wave % T::WGN) * T::WN;
    const int r32 = lane & 31, kh = lane >> 5;
    auto stored = [](int u) { return CPLX ? u : 2 * u; };

    // this lane's part of a block: row lane/2, slot lane%2 holding half (lane%2) ^ ((row >> 3) & 1)
    const int brow = lane >> 1, bhalf = (lane & 1) ^ ((brow >> 3) & 1);
    const unsigned short* A = p.a + (long long)s * p.a_slice + bhalf * 8;
    const unsigned short* B = p.b + (long long)s * p.b_slice + bhalf * 8;
    auto issue = [&](int buf, int k0) {
#pragma unroll
        for (int j = 0; j < LPW; ++j) {
            const int b = wave + j * NW;
            if (j < LPW_MIN || b < NBLK) {
                const unsigned short* src;
                if (b < RA / 32) {
                    const int u = b / (BM / 32), r = min(m0 + (b % (BM / 32)) * 32 + brow, p.m - 1);
                    src = A + stored(u) * p.a_plane + (long long)(k0 / kBK32) * p.m * kBK32 + (long long)r * kBK32;
                } else {
                    const int bb = b - RA / 32;
                    const int u = bb / (BN / 32), r = min(n0 + (bb % (BN / 32)) * 32 + brow, p.n - 1);
                    src = B + stored(u) * p.b_plane + (long long)(k0 / kBK32) * p.n * kBK32 + (long long)r * kBK32;
                }
                __builtin_amdgcn_global_load_lds((void*)src, (lds_ptr)(lds + buf * STAGE + b * 512), 16, 0, 0);
            }
        }
    };

    floatx16 accr[TM][TN], acci[TM][TN];
#pragma unroll
    for (int ti = 0; ti < TM; ++ti)
#pragma unroll
        for (int tj = 0; tj < TN; ++tj)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                accr[ti][tj][v] = 0.0f;
                acci[ti][tj][v] = 0.0f;
            }

    // fragment of row R0 + r32 (R0 a multiple of 32), values 8 kh .. 8 kh + 7
    const int foff = r32 * kBK32 + ((kh ^ ((r32 >> 3) & 1)) * 8);
    const int nk = (p.k + kBK32 - 1) / kBK32;
#pragma unroll
    for (int st = 0; st < S - 1; ++st)
        if (st < nk) issue(st, st * kBK32);
    for (int c = 0; c < nk; ++c) {
        if (c + S - 2 < nk)
            wait_vm<LPW_MIN * (S - 2)>();
        else
            wait_vm<0>();
        barrier_only();
        if (c + S - 1 < nk) issue((c + S - 1) % S, (c + S - 1) * kBK32);
        const unsigned short* sA = lds + (c % S) * STAGE;
        const unsigned short* sB = sA + RA * kBK32;
        shortx8 fa[TM][NPU], fb[TN][NPU];
#pragma unroll
        for (int u = 0; u < NPU; ++u) {
#pragma unroll
            for (int ti = 0; ti < TM; ++ti)
                fa[ti][u] = *reinterpret_cast<const shortx8*>(sA + (u * BM + wr + 32 * ti) * kBK32 + foff);
#pragma unroll
            for (int tj = 0; tj < TN; ++tj)
                fb[tj][u] = *reinterpret_cast<const shortx8*>(sB + (u * BN + wc + 32 * tj) * kBK32 + foff);
        }
        if constexpr (CPLX) {
            shortx8 nb1[TN], nb3[TN];
#pragma unroll
            for (int tj = 0; tj < TN; ++tj) {
                nb1[tj] = neg_bf16x8(fb[tj][1]);
                if constexpr (SPLIT) nb3[tj] = neg_bf16x8(fb[tj][3]);
            }
            // Cr += Ar Br - Ai Bi, Ci += Ar Bi + Ai Br for each (a-part, b-part); each
            // product over all (ti, tj) before the next, so dependent MFMAs are 2 TM TN apart
#define TP_W4(acc, a, b)                                                    \
    _Pragma("unroll") for (int ti = 0; ti < TM; ++ti)                       \
    _Pragma("unroll") for (int tj = 0; tj < TN; ++tj) acc[ti][tj] = TP_MFMA32_BF16(a, b, acc[ti][tj]);
            TP_W4(accr, fa[ti][0], fb[tj][0])
            TP_W4(acci, fa[ti][0], fb[tj][1])
            TP_W4(accr, fa[ti][1], nb1[tj])
            TP_W4(acci, fa[ti][1], fb[tj][0])
            if constexpr (SPLIT) {
                TP_W4(accr, fa[ti][0], fb[tj][2])
                TP_W4(acci, fa[ti][0], fb[tj][3])
                TP_W4(accr, fa[ti][1], nb3[tj])
                TP_W4(acci, fa[ti][1], fb[tj][2])
                TP_W4(accr, fa[ti][2], fb[tj][0])
                TP_W4(acci, fa[ti][2], fb[tj][1])
                TP_W4(accr, fa[ti][3], nb1[tj])
                TP_W4(acci, fa[ti][3], fb[tj][0])
            }
        } else {
            TP_W4(accr, fa[ti][0], fb[tj][0])
            if constexpr (SPLIT) {
                TP_W4(accr, fa[ti][0], fb[tj][1])
                TP_W4(accr, fa[ti][1], fb[tj][0])
            }
#undef TP_W4
        }
    }
    __syncthreads();

    float* cr = p.cr + (long long)s * p.sc;
    float* ci = p.ci + (long long)s * p.sc;
    // output value v of a lane: row 8 (v / 4) + 4 kh + v % 4, column r32 of the 32 x 32 block
#pragma unroll
    for (int ti = 0; ti < TM; ++ti)
#pragma unroll
        for (int tj = 0; tj < TN; ++tj)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int row = m0 + wr + 32 * ti + 8 * (v >> 2) + 4 * kh + (v & 3), col = n0 + wc + 32 * tj + r32;
                if (row < p.m && col < p.n) {
                    const long long off = (long long)row * p.ldc + col;
                    cr[off] = accr[ti][tj][v];
                    ci[off] = CPLX ? acci[ti][tj][v] : 0.0f;
                }
            }
}

template <class T, bool SPLIT>
__global__ __launch_bounds__(T::NT) void k_cgemm_bf16w(Bf16Args p)
{
    __shared__ __attribute__((aligned(1024))) unsigned short lds[bf16w_stages<T, SPLIT>() * bf16w_stage_elems<T, SPLIT>()];
    const int ntn = (p.n + T::BN - 1) / T::BN, tps = ((p.m + T::BM - 1) / T::BM) * ntn;
    const int nct = p.ncs * tps, nrt = p.nreal * tps;
    const int total = gridDim.x, w = blockIdx.x, x = w & 7;
    const int t = x * (total >> 3) + min(x, total & 7) + (w >> 3);
    if (t < nct) {
        const int rem = t % tps;
        bf16w_tile<T, SPLIT, true>(p, p.cs0 + t / tps, (rem / ntn) * T::BM, (rem % ntn) * T::BN, lds);
        return;
    }
    const int r0 = (t - nct) * p.rpw, r1 = min(nrt, r0 + p.rpw);
    for (int r = r0; r < r1; ++r) {
        const int rem = r % tps;
        bf16w_tile<T, SPLIT, false>(p, p.real_s[r / tps], (rem / ntn) * T::BM, (rem % ntn) * T::BN, lds);
    }
}

template <class T>
dim3 grid_of(const CgemmArgs& a)
{
    return dim3((a.n + T::BN - 1) / T::BN, (a.m + T::BM - 1) / T::BM, a.nslices);
}

template <int OPA, int OPB, class T>
hipError_t launch_f32(const CgemmArgs& a, hipStream_t s)
{
    // inner-dimension stage (tunable): 32 columns for long inner dimensions on
    // tiles at least 64 wide; narrow tiles keep 16, whose smaller LDS stage
    // fits twice the workgroups per CU (measured faster on the skinny
    // range-finder products)
    const int bkp = param(TP_PARAM_GEMM_BK);
    const bool bk32 = bkp == 32 || (bkp == 0 && a.k >= 256 && T::BN >= 64);
    auto kern = bk32 ? k_cgemm_f32<OPA, OPB, T, 32> : k_cgemm_f32<OPA, OPB, T, 16>;
    if (a.ksplit > 1) {
        if (!a.part) return hipErrorInvalidValue;
        dim3 g = grid_of<T>(a);
        g.z *= a.ksplit;
        kern<<<g, 256, 0, s>>>(a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        const long long total = (long long)a.nslices * a.m * a.n;
        long long blocks = (total + 255) / 256;
        if (blocks > 4096) blocks = 4096;
        k_splitk_reduce<<<(int)blocks, 256, 0, s>>>(a);
        return hipGetLastError();
    }
    kern<<<grid_of<T>(a), 256, 0, s>>>(a);
    return hipGetLastError();
}

template <int OPA, int TN>
hipError_t launch_skinny_tn(const CgemmArgs& a, hipStream_t s, bool reduce)
{
    const dim3 g((a.m + kSkRows - 1) / kSkRows, 1, a.nslices * (a.ksplit > 1 ? a.ksplit : 1));
    if (a.ksplit > 1 && !a.part) return hipErrorInvalidValue;
    k_skinny<OPA, TN><<<g, 256, 0, s>>>(a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || a.ksplit <= 1 || !reduce) return e;
    const long long total = (long long)a.nslices * a.m * a.n;
    long long blocks = (total + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    k_splitk_reduce<<<(int)blocks, 256, 0, s>>>(a);
    return hipGetLastError();
}

// reduce = false: a split product leaves its parts in a.part (summed by the caller)
template <int OPA>
hipError_t launch_skinny(const CgemmArgs& a, hipStream_t s, bool reduce = true)
{
    if (a.n <= 16) return launch_skinny_tn<OPA, 1>(a, s, reduce);
    if (a.n <= 32) return launch_skinny_tn<OPA, 2>(a, s, reduce);
    if (a.n <= 48) return launch_skinny_tn<OPA, 3>(a, s, reduce);
    return launch_skinny_tn<OPA, 4>(a, s, reduce);
}

// the wide kernel takes FP32 products A B, 1 <= k <= 64 (the same for every
// slice), whole 64 x 256 tiles, 16-byte aligned planes and rows (B and C), no
// split
// 0: no; 4: whole 64 x 256 tiles (unmasked); 1: outputs at most 64 columns
// wide, a multiple of 4 (masked rows and columns)
int wide_form(const CgemmArgs& a, int opa, int opb)
{
    const unsigned long long al = reinterpret_cast<unsigned long long>(a.br) |
                                  reinterpret_cast<unsigned long long>(a.bi) |
                                  reinterpret_cast<unsigned long long>(a.cr) | reinterpret_cast<unsigned long long>(a.ci);
    if (!(opa == OP_N && opb == OP_N && !a.kdyn && a.k >= 1 && a.k <= kWideMaxK && a.ksplit <= 1 && (al & 15) == 0 &&
          a.ldb % 4 == 0 && a.sb % 4 == 0 && a.ldc % 4 == 0 && a.sc % 4 == 0))
        return 0;
    if (a.m % kWideRows == 0 && a.n % kWideCols == 0) return 4;
    if (a.n <= kWideBlk && a.n % 4 == 0) return 1;
    return 0;
}

template <int NB>
hipError_t launch_wide_nb(const CgemmArgs& a, hipStream_t s)
{
    const dim3 g((a.n + kWideBlk * NB - 1) / (kWideBlk * NB), (a.m + kWideRows - 1) / kWideRows, a.nslices);
    if (a.k <= 16)
        k_wide<16, NB><<<g, 256, 0, s>>>(a);
    else if (a.k <= 32)
        k_wide<32, NB><<<g, 256, 0, s>>>(a);
    else if (a.k <= 48)
        k_wide<48, NB><<<g, 256, 0, s>>>(a);
    else
        k_wide<64, NB><<<g, 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_wide(const CgemmArgs& a, int form, hipStream_t s)
{
    return form == 4 ? launch_wide_nb<4>(a, s) : launch_wide_nb<1>(a, s);
}

// the skinny kernel takes FP32 products with op(B) = B, n <= 64 and a
// multiple of 4, and (by shape) an inner dimension long enough to stream
bool skinny_ok(const CgemmArgs& a, int opb, int kmin) { return opb == OP_N && a.n <= 64 && a.n % 4 == 0 && a.k >= kmin; }

template <class T, bool W = false>
hipError_t launch_bf16(Bf16Args a, hipStream_t s)
{
    const long long tps = (long long)((a.m + T::BM - 1) / T::BM) * ((a.n + T::BN - 1) / T::BN);
    const long long nwg = a.ncs * tps + (a.nreal * tps + a.rpw - 1) / a.rpw;
    if (nwg <= 0) return hipSuccess;
    if constexpr (W) {
        if (a.split)
            k_cgemm_bf16w<T, true><<<(unsigned)nwg, T::NT, 0, s>>>(a);
        else
            k_cgemm_bf16w<T, false><<<(unsigned)nwg, T::NT, 0, s>>>(a);
    } else {
        if (a.split)
            k_cgemm_bf16<T, true><<<(unsigned)nwg, T::NT, 0, s>>>(a);
        else
            k_cgemm_bf16<T, false><<<(unsigned)nwg, T::NT, 0, s>>>(a);
    }
    return hipGetLastError();
}

int cu_count()
{
    static const int n = [] {
        int d = 0, v = 0;
        if (hipGetDevice(&d) != hipSuccess || hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, d) !=
                                                   hipSuccess)
            return 256;
        return v > 0 ? v : 256;
    }();
    return n;
}

// bf16 tile: the tuned one if set (1: 64 x 64, 2: 128 x 128, 3: 128 x 32,
// 4: 256 x 128 and 5: 128 x 128 on 32 x 32 x 16 products, others 64 x 64),
// else the one with the least estimated time: workgroups per compute unit
// times the work of a tile over the fraction of peak such tiles sustain.
int pick_bf16(int m, int n, int ncs, int nreal)
{
    const int tuned = param(TP_PARAM_GEMM_VARIANT);
    if (tuned >= 1 && tuned <= 8) return tuned <= 5 ? tuned : 1;
    struct Cand {
        int id, bm, bn;
        double eff;
    };
    const Cand cands[] = {{4, 256, 128, 1.0}, {2, 128, 128, 0.9}, {1, 64, 64, 0.5}, {3, 128, 32, 0.45}};
    int best = 1;
    double best_cost = 0.0;
    for (const Cand& c : cands) {
        const long long tps = (long long)((m + c.bm - 1) / c.bm) * ((n + c.bn - 1) / c.bn);
        const long long nwg = ncs * tps + (nreal * tps + 1) / 2;
        const double cost = (double)((nwg + cu_count() - 1) / cu_count()) * c.bm * c.bn / c.eff;
        if (best_cost == 0.0 || cost < best_cost) {
            best = c.id;
            best_cost = cost;
        }
    }
    return best;
}

bool bf16_wide(int variant) { return variant == 4 || variant == 5; }
template <int OPA, int OPB>
hipError_t launch_ops(const CgemmArgs& a, int variant, hipStream_t s)
{
    switch (variant) {
        case 2: return launch_f32<OPA, OPB, T128x128>(a, s);
        case 3: return launch_f32<OPA, OPB, T128x64>(a, s);
        case 4: return launch_f32<OPA, OPB, T128x32>(a, s);
        case 5: return launch_f32<OPA, OPB, T256x16>(a, s);
        case 6: return launch_f32<OPA, OPB, T64x48>(a, s);
        default: return launch_f32<OPA, OPB, T64x64>(a, s);
    }
}

long long tiles(long long m, long long n, int bm, int bn, int ns) { return ((m + bm - 1) / bm) * ((n + bn - 1) / bn) * ns; }

// tile variant: the tuned one if set, else by shape (skinny outputs get
// narrow tiles; large products with enough tiles to fill the GPU get 128-wide)
int pick_variant(const CgemmArgs& a)
{
    const int tuned = param(TP_PARAM_GEMM_VARIANT);
    if (tuned >= 1 && tuned <= 8) return tuned;
    if (a.n <= 16) return 5;
    if (a.n <= 32) return 4;
    if (a.n <= 48) return 6;
    // short inner dimensions (rank-L reconstructions) stay on 64 x 64, whose
    // higher occupancy overlaps the output writes (measured faster)
    if (a.k < 128) return 1;
    if (a.m >= 256 && a.n >= 256 && tiles(a.m, a.n, 128, 128, a.nslices) >= 2048) return 2;
    if (a.m >= 128 && tiles(a.m, a.n, 128, 64, a.nslices) >= 2048) return 3;
    return 1;
}

}  // namespace

int batch_tile(int tile) { return tile == 1 ? 64 : 32; }

size_t splitk_bytes(int ksplit, int nslices, int m, int n)
{
    return ksplit > 1 ? align_up((size_t)2 * ksplit * nslices * m * n * sizeof(float)) : 0;
}

hipError_t launch_cgemm_batch(const CgemmArgs* items, const GemmUnit* units, int nunits, int tile, int grid,
                              double flops, double bytes, hipStream_t s)
{
    if (nunits <= 0) return hipSuccess;
    trace_work(flops, bytes);
    const int g = grid < nunits ? grid : nunits;
    if (tile == 1)
        k_cgemm_batch<T64x64><<<g, 256, 0, s>>>(items, units, nunits);
    else
        k_cgemm_batch<T32x32><<<g, 256, 0, s>>>(items, units, nunits);
    return hipGetLastError();
}

namespace {
void trace_gemm_work(const CgemmArgs& a)
{
    // a product over a device-counted set of slices has no work the host knows
    if (a.dyn_ns) return;
    const int nreal = (a.real_first ? 1 : 0) + (a.real_last && a.nslices > 1 ? 1 : 0);
    if (a.gate || a.dyn_m || a.dyn_n || a.dyn_k) {
        trace_gemm_dyn(a.gate, a.dyn_m, a.dyn_n, a.dyn_k, a.m, a.n, a.k, a.nslices, nreal);
        return;
    }
    const double mnk = (double)a.m * a.n * a.k, elems = (double)a.m * a.k + (double)a.k * a.n + (double)a.m * a.n;
    trace_work(mnk * (8.0 * (a.nslices - nreal) + 2.0 * nreal), elems * (8.0 * (a.nslices - nreal) + 4.0 * nreal));
}
}  // namespace

bool cgemm_parts_ok(const CgemmArgs& a, int opa, int opb)
{
    const int tuned = param(TP_PARAM_GEMM_VARIANT);
    return a.m > 0 && a.n > 0 && a.nslices > 0 && a.ksplit > 1 && a.part && (tuned == 0 || tuned == 7) &&
           skinny_ok(a, opb, 64) && (opa == OP_N || opa == OP_C);
}

hipError_t launch_cgemm_parts(const CgemmArgs& a, int opa, int opb, hipStream_t s)
{
    if (!cgemm_parts_ok(a, opa, opb)) return hipErrorInvalidValue;
    trace_gemm_work(a);
    return opa == OP_N ? launch_skinny<OP_N>(a, s, false) : launch_skinny<OP_C>(a, s, false);
}

hipError_t launch_cgemm(const CgemmArgs& a, int opa, int opb, int prec, hipStream_t s)
{
    if (a.m <= 0 || a.n <= 0 || a.nslices <= 0) return hipSuccess;
    trace_gemm_work(a);
    if (prec != TP_PREC_FP32) return hipErrorInvalidValue;
    const int variant = pick_variant(a);
    const int tuned = param(TP_PARAM_GEMM_VARIANT);
    // a device-capped inner dimension that fits the wide kernel stays short:
    // the wide kernel skips its dead 16-deep chunks
    if (tuned == 0 && a.dyn_k && wide_form(a, opa, opb)) return launch_wide(a, wide_form(a, opa, opb), s);
    if ((tuned == 0 || tuned == 7) && skinny_ok(a, opb, tuned == 7 ? 1 : 64) && (opa == OP_N || opa == OP_C))
        return opa == OP_N ? launch_skinny<OP_N>(a, s) : launch_skinny<OP_C>(a, s);
    if (tuned == 0 || tuned == 8) {
        const int form = wide_form(a, opa, opb);
        if (form) return launch_wide(a, form, s);
    }
    if (opa == OP_N && opb == OP_N) return launch_ops<OP_N, OP_N>(a, variant, s);
    if (opa == OP_C && opb == OP_N) return launch_ops<OP_C, OP_N>(a, variant, s);
    if (opa == OP_N && opb == OP_C) return launch_ops<OP_N, OP_C>(a, variant, s);
    return launch_ops<OP_C, OP_C>(a, variant, s);
}

int bf16_plan(int m, int n, int k, int ncs, int nreal, int* bkl)
{
    (void)k;
    const int v = pick_bf16(m, n, ncs, nreal);
    if (bkl) *bkl = bf16_wide(v) ? kBK32 : kBK;
    return v;
}

hipError_t launch_cgemm_bf16(Bf16Args a, hipStream_t s)
{
    if (a.m <= 0 || a.n <= 0 || a.ncs + a.nreal <= 0) return hipSuccess;
    const int v = a.variant;
    if (v < 1 || v > 5 || a.bkl != (bf16_wide(v) ? kBK32 : kBK) || a.ld % a.bkl || a.ld < a.k || a.nreal < 0 ||
        a.nreal > 2 || a.k <= 0)
        return hipErrorInvalidValue;
    {
        const double mnk = (double)a.m * a.n * a.k;
        const double np = a.split ? 4.0 : 2.0;  // bf16 planes per operand
        const double ns = (double)a.ncs + a.nreal;
        trace_work(mnk * (8.0 * a.ncs + 2.0 * a.nreal),
                   ns * (2.0 * np * ((double)a.m * a.k + (double)a.k * a.n) + 8.0 * (double)a.m * a.n));
    }
    a.rpw = 2;
    switch (v) {
        case 2: return launch_bf16<B128x128>(a, s);
        case 3: return launch_bf16<B128x32>(a, s);
        case 4: return launch_bf16<C256x128, true>(a, s);
        case 5: return launch_bf16<C128x128, true>(a, s);
        default: return launch_bf16<B64x64>(a, s);
    }
}

}  // namespace tp
