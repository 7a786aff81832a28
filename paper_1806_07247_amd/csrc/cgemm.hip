// Batched planar-complex slice GEMM on the gfx950 matrix cores:
//   C^(s) = op(A^(s)) op(B^(s)),  s = 0 .. nslices-1,
// the dense per-slice step of Algorithm 1 (Cbar^(i) = Abar^(i) Bbar^(i) for the
// ceil((n3+1)/2) leading slices, eq (10)), also used for the reconstruction
// products of the singular value thresholding.
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
// Tiling: 256 threads = 4 wavefronts in a 2x2 arrangement; workgroup tile
// 64x64 (complex), wavefront tile 32x32 = 2x2 MFMA tiles of 16x16.  Operand
// tiles are staged through LDS (double buffered) with the k index contiguous
// so that each lane reads its MFMA operands with 16-byte LDS loads.
#include "tp_internal.h"

namespace tp {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef short shortx8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int BM = 64, BN = 64;

struct SliceView {
    const float *ar, *ai, *br, *bi;
    float *cr, *ci;
    int K;
    bool real;
};

__device__ __forceinline__ SliceView slice_view(const CgemmArgs& p, int s)
{
    SliceView v;
    v.ar = p.ar + s * p.sa;
    v.ai = p.ai + s * p.sa;
    v.br = p.br + s * p.sb;
    v.bi = p.bi + s * p.sb;
    v.cr = p.cr + s * p.sc;
    v.ci = p.ci + s * p.sc;
    v.K = p.kdyn ? min(p.kdyn[s], p.k) : p.k;
    v.real = (p.real_first && s == 0) || (p.real_last && s == p.nslices - 1);
    return v;
}

// Loads one BKxBM (A) and BKxBN (B) panel of op(A), op(B) into registers.
// Each thread holds 4 consecutive elements of each plane.
//   A, OP_N: thread -> (row t/ (BK/4) , k group)    contiguous along k
//   A, OP_C: thread -> (k  t / 16, row group of 4)  contiguous along rows
//   B, OP_N: thread -> (k  t / 16, col group of 4)  contiguous along cols
//   B, OP_C: thread -> (col t / (BK/4), k group)    contiguous along k
template <int OPA, int OPB, int BK>
struct PanelLoader {
    static constexpr int KQ = BK / 4;            // float4 groups along k
    static constexpr int NLOAD = (BM * BK) / 256 / 4;  // float4 groups per thread
    float a_r[NLOAD][4], a_i[NLOAD][4], b_r[NLOAD][4], b_i[NLOAD][4];

    __device__ __forceinline__ void load(const SliceView& v, const CgemmArgs& p, int m0, int n0, int k0, int tid)
    {
#pragma unroll
        for (int u = 0; u < NLOAD; ++u) {
            const int t = tid + u * 256;
            if (OPA == OP_N) {
                const int r = t / KQ, kq = (t % KQ) * 4, row = m0 + r;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int kk = k0 + kq + e;
                    const bool in = row < p.m && kk < v.K;
                    const long long off = (long long)row * p.lda + kk;
                    a_r[u][e] = in ? v.ar[off] : 0.0f;
                    a_i[u][e] = in ? v.ai[off] : 0.0f;
                }
            } else {
                const int kk = k0 + t / (BM / 4), r4 = (t % (BM / 4)) * 4;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int row = m0 + r4 + e;
                    const bool in = row < p.m && kk < v.K;
                    const long long off = (long long)kk * p.lda + row;
                    a_r[u][e] = in ? v.ar[off] : 0.0f;
                    a_i[u][e] = in ? -v.ai[off] : 0.0f;
                }
            }
            if (OPB == OP_N) {
                const int kk = k0 + t / (BN / 4), c4 = (t % (BN / 4)) * 4;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int col = n0 + c4 + e;
                    const bool in = col < p.n && kk < v.K;
                    const long long off = (long long)kk * p.ldb + col;
                    b_r[u][e] = in ? v.br[off] : 0.0f;
                    b_i[u][e] = in ? v.bi[off] : 0.0f;
                }
            } else {
                const int c = t / KQ, kq = (t % KQ) * 4, col = n0 + c;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int kk = k0 + kq + e;
                    const bool in = col < p.n && kk < v.K;
                    const long long off = (long long)col * p.ldb + kk;
                    b_r[u][e] = in ? v.br[off] : 0.0f;
                    b_i[u][e] = in ? -v.bi[off] : 0.0f;
                }
            }
        }
    }

    // Writes the staged panel as sX[row][k] (row = m for A, n for B) with
    // leading dimension LDK, via a per-element conversion functor.
    template <int LDK, class Store>
    __device__ __forceinline__ void store(int tid, Store&& st) const
    {
#pragma unroll
        for (int u = 0; u < NLOAD; ++u) {
            const int t = tid + u * 256;
            if (OPA == OP_N) {
                const int r = t / KQ, kq = (t % KQ) * 4;
#pragma unroll
                for (int e = 0; e < 4; ++e) st.a(r * LDK + kq + e, a_r[u][e], a_i[u][e]);
            } else {
                const int kk = t / (BM / 4), r4 = (t % (BM / 4)) * 4;
#pragma unroll
                for (int e = 0; e < 4; ++e) st.a((r4 + e) * LDK + kk, a_r[u][e], a_i[u][e]);
            }
            if (OPB == OP_N) {
                const int kk = t / (BN / 4), c4 = (t % (BN / 4)) * 4;
#pragma unroll
                for (int e = 0; e < 4; ++e) st.b((c4 + e) * LDK + kk, b_r[u][e], b_i[u][e]);
            } else {
                const int c = t / KQ, kq = (t % KQ) * 4;
#pragma unroll
                for (int e = 0; e < 4; ++e) st.b(c * LDK + kq + e, b_r[u][e], b_i[u][e]);
            }
        }
    }
};

__device__ __forceinline__ void write_tile(const SliceView& v, const CgemmArgs& p, int m0, int n0, int wr, int wc,
                                           int lane, const floatx4 (&accr)[2][2], const floatx4 (&acci)[2][2])
{
    const int g = lane >> 4, c16 = lane & 15;
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int row = m0 + wr + 16 * ti + 4 * g + j;
                const int col = n0 + wc + 16 * tj + c16;
                if (row < p.m && col < p.n) {
                    const long long off = (long long)row * p.ldc + col;
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

template <int OPA, int OPB>
__global__ __launch_bounds__(256) void k_cgemm_f32(CgemmArgs p)
{
    constexpr int BK = 16, LDK = BK + 4;
    __shared__ __attribute__((aligned(16))) float sAr[2][BM * LDK];
    __shared__ __attribute__((aligned(16))) float sAi[2][BM * LDK];
    __shared__ __attribute__((aligned(16))) float sBr[2][BN * LDK];
    __shared__ __attribute__((aligned(16))) float sBi[2][BN * LDK];

    const SliceView v = slice_view(p, blockIdx.z);
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    const int g = lane >> 4, r16 = lane & 15;

    floatx4 accr[2][2], acci[2][2];
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj) {
            accr[ti][tj] = floatx4{0.f, 0.f, 0.f, 0.f};
            acci[ti][tj] = floatx4{0.f, 0.f, 0.f, 0.f};
        }

    PanelLoader<OPA, OPB, BK> ld;
    const int nk = (v.K + BK - 1) / BK;
    if (nk > 0) {
        ld.load(v, p, m0, n0, 0, tid);
        ld.template store<LDK>(tid, StoreF32{sAr[0], sAi[0], sBr[0], sBi[0]});
    }
    __syncthreads();
    for (int c = 0; c < nk; ++c) {
        const int cur = c & 1;
        if (c + 1 < nk) ld.load(v, p, m0, n0, (c + 1) * BK, tid);
        // lane (g, r16) of MFMA step s uses k = 4g + s: one 16-byte LDS read per operand
        float4 fa_r[2], fa_i[2], fb_r[2], fb_i[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            fa_r[t] = *reinterpret_cast<const float4*>(&sAr[cur][(wr + 16 * t + r16) * LDK + 4 * g]);
            fa_i[t] = *reinterpret_cast<const float4*>(&sAi[cur][(wr + 16 * t + r16) * LDK + 4 * g]);
            fb_r[t] = *reinterpret_cast<const float4*>(&sBr[cur][(wc + 16 * t + r16) * LDK + 4 * g]);
            fb_i[t] = *reinterpret_cast<const float4*>(&sBi[cur][(wc + 16 * t + r16) * LDK + 4 * g]);
        }
        if (v.real) {
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int ti = 0; ti < 2; ++ti)
#pragma unroll
                    for (int tj = 0; tj < 2; ++tj)
                        accr[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                            (&fa_r[ti].x)[s], (&fb_r[tj].x)[s], accr[ti][tj], 0, 0, 0);
        } else {
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int ti = 0; ti < 2; ++ti)
#pragma unroll
                    for (int tj = 0; tj < 2; ++tj) {
                        const float ar = (&fa_r[ti].x)[s], ai = (&fa_i[ti].x)[s];
                        const float br = (&fb_r[tj].x)[s], bi = (&fb_i[tj].x)[s];
                        accr[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, br, accr[ti][tj], 0, 0, 0);
                        acci[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, bi, acci[ti][tj], 0, 0, 0);
                        accr[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x4f32(-ai, bi, accr[ti][tj], 0, 0, 0);
                        acci[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai, br, acci[ti][tj], 0, 0, 0);
                    }
        }
        if (c + 1 < nk) ld.template store<LDK>(tid, StoreF32{sAr[cur ^ 1], sAi[cur ^ 1], sBr[cur ^ 1], sBi[cur ^ 1]});
        __syncthreads();
    }
    write_tile(v, p, m0, n0, wr, wc, lane, accr, acci);
}

// ------------------------------------------------------------- BF16 (x3) --
__device__ __forceinline__ unsigned short bf16_rne(float x)
{
    unsigned int u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(unsigned short h) { return __uint_as_float(((unsigned int)h) << 16); }

struct StoreBF16 {
    unsigned short *arh, *ail, *aih, *arl, *brh, *brl, *bih, *bil;
    bool split;
    __device__ __forceinline__ void a(int i, float r, float im) const
    {
        const unsigned short rh = bf16_rne(r), ih = bf16_rne(im);
        arh[i] = rh;
        aih[i] = ih;
        if (split) {
            arl[i] = bf16_rne(r - bf16_to_f32(rh));
            ail[i] = bf16_rne(im - bf16_to_f32(ih));
        }
    }
    __device__ __forceinline__ void b(int i, float r, float im) const
    {
        const unsigned short rh = bf16_rne(r), ih = bf16_rne(im);
        brh[i] = rh;
        bih[i] = ih;
        if (split) {
            brl[i] = bf16_rne(r - bf16_to_f32(rh));
            bil[i] = bf16_rne(im - bf16_to_f32(ih));
        }
    }
};

__device__ __forceinline__ shortx8 neg_bf16x8(shortx8 v)
{
    return v ^ (shortx8){(short)0x8000, (short)0x8000, (short)0x8000, (short)0x8000,
                         (short)0x8000, (short)0x8000, (short)0x8000, (short)0x8000};
}

#define TP_MFMA_BF16(a, b, c)                                                                  \
    __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, (a)), __builtin_bit_cast(bf16x8, (b)), \
                                            (c), 0, 0, 0)

template <int OPA, int OPB, bool SPLIT>
__global__ __launch_bounds__(256) void k_cgemm_bf16(CgemmArgs p)
{
    constexpr int BK = 32, LDK = BK + 8;  // 16-byte aligned rows, staggered banks
    constexpr int NP = SPLIT ? 2 : 1;
    __shared__ __attribute__((aligned(16))) unsigned short sA[2][NP][2][BM * LDK];  // [buf][hi/lo][re/im]
    __shared__ __attribute__((aligned(16))) unsigned short sB[2][NP][2][BN * LDK];

    const SliceView v = slice_view(p, blockIdx.z);
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    const int g = lane >> 4, r16 = lane & 15;

    floatx4 accr[2][2], acci[2][2];
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj) {
            accr[ti][tj] = floatx4{0.f, 0.f, 0.f, 0.f};
            acci[ti][tj] = floatx4{0.f, 0.f, 0.f, 0.f};
        }

    auto storer = [&](int b) {
        return StoreBF16{sA[b][0][0], sA[b][NP - 1][1], sA[b][0][1], sA[b][NP - 1][0],
                         sB[b][0][0], sB[b][NP - 1][0], sB[b][0][1], sB[b][NP - 1][1], SPLIT};
    };

    PanelLoader<OPA, OPB, BK> ld;
    const int nk = (v.K + BK - 1) / BK;
    if (nk > 0) {
        ld.load(v, p, m0, n0, 0, tid);
        ld.template store<LDK>(tid, storer(0));
    }
    __syncthreads();
    for (int c = 0; c < nk; ++c) {
        const int cur = c & 1;
        if (c + 1 < nk) ld.load(v, p, m0, n0, (c + 1) * BK, tid);
        // 16x16x32 operands: lane (g, r16) holds k = 8g .. 8g+7 of row (col) r16
        shortx8 fa[2][NP][2], fb[2][NP][2];
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int h = 0; h < NP; ++h)
#pragma unroll
                for (int ri = 0; ri < 2; ++ri) {
                    fa[t][h][ri] = *reinterpret_cast<const shortx8*>(&sA[cur][h][ri][(wr + 16 * t + r16) * LDK + 8 * g]);
                    fb[t][h][ri] = *reinterpret_cast<const shortx8*>(&sB[cur][h][ri][(wc + 16 * t + r16) * LDK + 8 * g]);
                }
#pragma unroll
        for (int ti = 0; ti < 2; ++ti)
#pragma unroll
            for (int tj = 0; tj < 2; ++tj) {
                // terms (a-part, b-part): hi*hi, then hi*lo and lo*hi when splitting
#pragma unroll
                for (int term = 0; term < (SPLIT ? 3 : 1); ++term) {
                    const int ha = (term == 2) ? 1 : 0, hb = (term == 1) ? 1 : 0;
                    const shortx8 ar = fa[ti][ha][0], ai = fa[ti][ha][1];
                    const shortx8 br = fb[tj][hb][0], bi = fb[tj][hb][1];
                    accr[ti][tj] = TP_MFMA_BF16(ar, br, accr[ti][tj]);
                    if (!v.real) {
                        acci[ti][tj] = TP_MFMA_BF16(ar, bi, acci[ti][tj]);
                        accr[ti][tj] = TP_MFMA_BF16(neg_bf16x8(ai), bi, accr[ti][tj]);
                        acci[ti][tj] = TP_MFMA_BF16(ai, br, acci[ti][tj]);
                    }
                }
            }
        if (c + 1 < nk) ld.template store<LDK>(tid, storer(cur ^ 1));
        __syncthreads();
    }
    write_tile(v, p, m0, n0, wr, wc, lane, accr, acci);
}

template <int OPA, int OPB>
hipError_t launch_ops(const CgemmArgs& a, int prec, hipStream_t s)
{
    dim3 grid((a.n + BN - 1) / BN, (a.m + BM - 1) / BM, a.nslices);
    if (prec == TP_PREC_FP32)
        k_cgemm_f32<OPA, OPB><<<grid, 256, 0, s>>>(a);
    else if (prec == TP_PREC_BF16X3)
        k_cgemm_bf16<OPA, OPB, true><<<grid, 256, 0, s>>>(a);
    else
        k_cgemm_bf16<OPA, OPB, false><<<grid, 256, 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_cgemm(const CgemmArgs& a, int opa, int opb, int prec, hipStream_t s)
{
    if (a.m <= 0 || a.n <= 0 || a.nslices <= 0) return hipSuccess;
    if (opa == OP_N && opb == OP_N) return launch_ops<OP_N, OP_N>(a, prec, s);
    if (opa == OP_C && opb == OP_N) return launch_ops<OP_C, OP_N>(a, prec, s);
    if (opa == OP_N && opb == OP_C) return launch_ops<OP_N, OP_C>(a, prec, s);
    return launch_ops<OP_C, OP_C>(a, prec, s);
}

}  // namespace tp
