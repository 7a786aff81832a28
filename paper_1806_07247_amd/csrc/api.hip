// C-ABI entry points of libtp.so: argument checks, workspace carving and the
// kernel sequence of each operation.  See include/tp.h for the contract.
#include <cmath>
#include <cstring>
#include <initializer_list>
#include <algorithm>
#include <utility>
#include <vector>

#include "tp_internal.h"

namespace {

constexpr int kMaxN3 = 1024;

bool bad_dim(int v) { return v <= 0; }

bool bad_slice(long long a, long long b) { return a * b >= (1LL << 31); }

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Workspace of tprod: half spectra of A, B and C (planar complex).  With
// bf16 slice products, A and B are bf16 planes instead (hi re, hi im, and for
// BF16X3 lo re, lo im): A as n1 rows of the inner index, B as l columns of
// it, k-blocked and zero-padded to ld = n2 rounded up to the block length
// the product reads (tp::SplitOut).
struct TprodLayout {
    tp::Planes a, b, c;
    unsigned short *ah, *bh;
    int ld, np, bkl, variant;
};

int bf16_planes(int prec) { return prec == TP_PREC_BF16X3 ? 4 : 2; }

// real slices of the half spectrum: 0, and n3/2 for even n3
int real_slices(int n3) { return (n3 % 2 == 0) ? 2 : 1; }

tp::Arena tprod_arena(void* ws, size_t bytes, int n1, int n2, int l, int n3, int prec, TprodLayout* L)
{
    const size_t h = (size_t)tp::half_slices(n3);
    tp::Arena ar(ws, bytes);
    TprodLayout t{};
    if (prec == TP_PREC_FP32) {
        t.a.re = ar.take<float>(h * n1 * n2);
        t.a.im = ar.take<float>(h * n1 * n2);
        t.b.re = ar.take<float>(h * n2 * l);
        t.b.im = ar.take<float>(h * n2 * l);
    } else {
        t.np = bf16_planes(prec);
        const int nreal = real_slices(n3);
        t.variant = tp::bf16_plan(n1, l, n2, (int)h - nreal, nreal, &t.bkl);
        t.ld = (n2 + t.bkl - 1) / t.bkl * t.bkl;
        t.ah = ar.take<unsigned short>((size_t)t.np * h * n1 * t.ld);
        t.bh = ar.take<unsigned short>((size_t)t.np * h * l * t.ld);
    }
    t.c.re = ar.take<float>(h * n1 * l);
    t.c.im = ar.take<float>(h * n1 * l);
    if (L) *L = t;
    return ar;
}

// Workspace of prox_tnn / tnn.
struct SvtLayout {
    tp::Planes ybar;   // half spectrum of Y; reused for the thresholded slices
    tp::Planes w;      // rotated (then scaled) columns, R x P per slice
    tp::Planes t;      // first reconstruction product, p x p per slice
    double* sigma;     // P per slice
    int* keep;         // per slice
    void* jscratch;    // Jacobi work matrices when a slice does not fit in LDS
    size_t jscratch_bytes;
    tp::Planes tmp;    // transform scratch of order-p tensors (when asked for)
};

// the layout for h Fourier slices; tmp: scratch planes of h slices for the
// transforms of order-p tensors when no reconstruction planes can serve
tp::Arena svt_arena_h(void* ws, size_t bytes, int n1, int n2, size_t h, bool recon, SvtLayout* L,
                      bool any_count = false, bool tmp = false)
{
    const size_t mn = (size_t)n1 * n2, p = (size_t)(n1 < n2 ? n1 : n2), P = p;
    tp::Arena ar(ws, bytes);
    SvtLayout t{};
    t.ybar.re = ar.take<float>(h * mn);
    t.ybar.im = ar.take<float>(h * mn);
    if (recon) {
        t.w.re = ar.take<float>(h * mn);
        t.w.im = ar.take<float>(h * mn);
        t.t.re = ar.take<float>(h * p * p);
        t.t.im = ar.take<float>(h * p * p);
        t.keep = ar.take<int>(h);
    }
    t.sigma = ar.take<double>(h * P);
    t.jscratch_bytes = tp::jacobi_scratch_bytes(n1, n2, (int)h, false);
    if (any_count) {  // any batch of up to h slices (a compact set of fallback slices)
        const size_t one = tp::jacobi_scratch_bytes(n1, n2, 1, false);
        if (one * h + 4096 > t.jscratch_bytes) t.jscratch_bytes = one * h + 4096;
    }
    t.jscratch = t.jscratch_bytes ? ar.take<char>(t.jscratch_bytes) : nullptr;
    if (tmp) {
        t.tmp.re = ar.take<float>(h * mn);
        t.tmp.im = ar.take<float>(h * mn);
    }
    if (L) *L = t;
    return ar;
}

tp::Arena svt_arena(void* ws, size_t bytes, int n1, int n2, int n3, bool recon, SvtLayout* L, bool any_count = false)
{
    return svt_arena_h(ws, bytes, n1, n2, (size_t)tp::half_slices(n3), recon, L, any_count);
}

// Matrix SVT W^(k) = U (S - tau)_+ V^* of `nslices` slices held in yb (planar
// row-major n1 x n2 per slice), written back to yb: one-sided Jacobi on each
// slice (or its conjugate transpose when wide), shrinkage of the rotated
// columns, then W = What What^* Ybar (or Ybar Bhat Bhat^*) as two products.
int run_svt(const SvtLayout& L, tp::Planes yb, int n1, int n2, int nslices, int real_first, int real_last,
            double tau, int* info, int* rank, hipStream_t s, const int* count = nullptr)
{
    const bool tr = n1 < n2;
    const int R = tr ? n2 : n1, P = tr ? n1 : n2, p = P;
    const long long mn = (long long)n1 * n2;
    const int h = nslices;
    tp::JacobiArgs j{};
    j.yr = yb.re;
    j.yi = yb.im;
    j.wr = L.w.re;
    j.wi = L.w.im;
    j.sigma = L.sigma;
    j.info = info;
    j.m = n1;
    j.n = n2;
    j.nslices = h;
    j.max_sweeps = tp::param(TP_PARAM_JACOBI_SWEEPS);
    j.transpose = tr ? 1 : 0;
    j.tol = tp::jacobi_tol(R);
    j.count = count;
    TP_LAUNCH(tp::K_JACOBI, s, tp::launch_jacobi(j, L.jscratch, L.jscratch_bytes, s));
    // shrinkage (eq (21)): scaled columns sqrt(d_j)/sigma_j w_j
    TP_LAUNCH(tp::K_SHRINK, s,
              tp::launch_shrink(L.w.re, L.w.im, L.sigma, rank ? rank : L.keep, R, P, h, tau, s, count));
    // W = U (S - tau)_+ V^* as two slice products
    tp::CgemmArgs g{};
    g.nslices = h;
    g.dyn_ns = count;
    g.real_first = real_first;
    g.real_last = real_last;
    if (!tr) {
        // T = What^* Ybar (n x n), then W = What T (m x n)
        g.ar = L.w.re; g.ai = L.w.im; g.lda = n2; g.sa = mn;
        g.br = yb.re; g.bi = yb.im; g.ldb = n2; g.sb = mn;
        g.cr = L.t.re; g.ci = L.t.im; g.ldc = p; g.sc = (long long)p * p;
        g.m = n2; g.n = n2; g.k = n1;
        TP_LAUNCH(tp::K_CGEMM, s, tp::launch_cgemm(g, tp::OP_C, tp::OP_N, TP_PREC_FP32, s));
        g.ar = L.w.re; g.ai = L.w.im; g.lda = n2; g.sa = mn;
        g.br = L.t.re; g.bi = L.t.im; g.ldb = p; g.sb = (long long)p * p;
        g.cr = yb.re; g.ci = yb.im; g.ldc = n2; g.sc = mn;
        g.m = n1; g.n = n2; g.k = n2;
        TP_LAUNCH(tp::K_CGEMM, s, tp::launch_cgemm(g, tp::OP_N, tp::OP_N, TP_PREC_FP32, s));
    } else {
        // T = Ybar Bhat (m x m), then W = T Bhat^* (m x n); Bhat is n x m
        g.ar = yb.re; g.ai = yb.im; g.lda = n2; g.sa = mn;
        g.br = L.w.re; g.bi = L.w.im; g.ldb = n1; g.sb = mn;
        g.cr = L.t.re; g.ci = L.t.im; g.ldc = p; g.sc = (long long)p * p;
        g.m = n1; g.n = n1; g.k = n2;
        TP_LAUNCH(tp::K_CGEMM, s, tp::launch_cgemm(g, tp::OP_N, tp::OP_N, TP_PREC_FP32, s));
        g.ar = L.t.re; g.ai = L.t.im; g.lda = p; g.sa = (long long)p * p;
        g.br = L.w.re; g.bi = L.w.im; g.ldb = n1; g.sb = mn;
        g.cr = yb.re; g.ci = yb.im; g.ldc = n2; g.sc = mn;
        g.m = n1; g.n = n2; g.k = n1;
        TP_LAUNCH(tp::K_CGEMM, s, tp::launch_cgemm(g, tp::OP_N, tp::OP_C, TP_PREC_FP32, s));
    }
    return TP_OK;
}


// split-K partial buffer of the learned path: up to kMaxSplit parts of an
// (max(n1, n2) x l_max) product per slice
constexpr int kMaxSplit = 4;

// Workspace of the learned-rank prox.
struct LearnedLayout {
    SvtLayout full;                 // full path, sized for any batch of up to h slices
    tp::Planes wbar;                // thresholded slices (m x n)
    tp::Planes cy;                  // compact fallback slices (m x n)
    tp::Planes om, ya, yb, za, zb;  // sketch (n x L), ranges (m x L), co-ranges (n x L)
    tp::Planes rinv, rh, T, m1;     // L x L, L x L, L x L, L x n
    double2* part;
    double2* rtot;
    float2* jcols;
    float2* jv;
    double* jsig;
    double* fpart;                  // per-band column norms of the features
    float* kpart;                   // split-K partial products
    size_t kpart_bytes;
    double* fro2;                   // ||Ybar^(k)||_F^2 per slice
    double* accpart;                // per-band partial residual sums of the accuracy check
    float* feats;
    tp::Planes vp, cp, t1, t2;      // V_r, U_r S (planar L x L), residual products (m x L)
    int *kpred, *lact, *fb, *rank, *status, *idx, *cinfo, *crank, *prefb, *bad;
    int* ctl;                       // device-side control values (widths, gates, counts; Ctl)
};

// Entries of LearnedLayout::ctl, written and read on the device only.
enum Ctl {
    C_L1 = 0,      // sketch width of the first attempt (0: no randomized slice)
    C_G1 = 1,      // gate of the first attempt
    C_RETRY = 2,   // gate of the wide retry (some count check failed below the widest sketch)
    C_L2 = 3,      // sketch width of the retry
    C_G2 = 4,      // gate of the retry
    C_NFB = 5,     // number of fallback slices
    C_ROUND = 8,   // C_ROUND + 32 a + r: round r (r >= 1) of the accuracy loop of attempt a
    C_COUNT = 72
};
constexpr int kMaxRounds = 31;

tp::Arena learned_arena(void* ws, size_t bytes, int n1, int n2, int n3, int Lw, LearnedLayout* out)
{
    const size_t h = (size_t)tp::half_slices(n3), mn = (size_t)n1 * n2, L = (size_t)Lw;
    LearnedLayout t{};
    tp::Arena ar(ws, bytes);
    SvtLayout f{};
    // the full-path buffers first (svt_arena's own layout), then the rest
    tp::Arena fa = svt_arena(ws, bytes, n1, n2, n3, true, &f, true);
    ar.used = fa.used;
    ar.ok = fa.ok;
    t.full = f;
    auto planes = [&](size_t count) {
        tp::Planes pl;
        pl.re = ar.take<float>(count);
        pl.im = ar.take<float>(count);
        return pl;
    };
    t.wbar = planes(h * mn);
    t.cy = planes(h * mn);
    t.om = planes(h * n2 * L);
    t.ya = planes(h * n1 * L);
    t.yb = planes(h * n1 * L);
    t.za = planes(h * n2 * L);
    t.zb = planes(h * n2 * L);
    t.rinv = planes(h * L * L);
    t.rh = planes(h * L * L);
    t.T = planes(h * L * L);
    t.m1 = planes(h * L * n2);
    t.vp = planes(h * L * L);
    t.cp = planes(h * L * L);
    t.t1 = planes(h * n1 * L);
    t.t2 = planes(h * n1 * L);
    const int mx = n1 > n2 ? n1 : n2;
    t.part = reinterpret_cast<double2*>(ar.take<char>(tp::cholqr_part_bytes(mx, Lw, (int)h)));
    t.rtot = ar.take<double2>(h * L * L);
    t.jcols = ar.take<float2>(h * L * L);
    t.jv = ar.take<float2>(h * L * L);
    t.jsig = ar.take<double>(h * L);
    t.fpart = reinterpret_cast<double*>(ar.take<char>(tp::features_part_bytes(n1, n2, (int)h)));
    t.kpart_bytes = tp::splitk_bytes(kMaxSplit, (int)h, mx, Lw);
    t.kpart = reinterpret_cast<float*>(ar.take<char>(t.kpart_bytes));
    t.fro2 = ar.take<double>(h);
    t.accpart = reinterpret_cast<double*>(ar.take<char>(tp::accuracy_part_bytes((int)h)));
    t.feats = ar.take<float>(h * TP_MLP_INPUTS);
    // kpred, lact and prefb adjacent: the host reads them with one copy
    t.kpred = ar.take<int>(3 * h);
    t.lact = t.kpred + h;
    t.prefb = t.kpred + 2 * h;
    t.fb = ar.take<int>(h);
    t.rank = ar.take<int>(h);
    t.status = ar.take<int>(h);
    t.idx = ar.take<int>(h);
    t.cinfo = ar.take<int>(h);
    t.crank = ar.take<int>(h);
    t.bad = ar.take<int>(h);
    t.ctl = ar.take<int>(C_COUNT);
    if (out) *out = t;
    return ar;
}

// parts of the inner dimension for a product with few output tiles (so that
// enough workgroups run), each part at least 128 long
int pick_ksplit(int m, int n, int k, int nslices, size_t part_bytes)
{
    if (!part_bytes || k < 256) return 1;
    const long long tiles = (long long)((m + 63) / 64) * ((n + 63) / 64) * nslices;
    int ks = 1;
    const int forced = tp::param(TP_PARAM_GEMM_KSPLIT);
    if (forced > 0)
        ks = std::min(forced, kMaxSplit);
    else
        while (ks < kMaxSplit && tiles * ks * 2 <= 4096 && k / (ks * 2) >= 128) ks *= 2;
    while (ks > 1 && tp::splitk_bytes(ks, nslices, m, n) > part_bytes) ks /= 2;
    return ks;
}

// slice GEMM of planar stacks: C = op(A) op(B) with op(A) m x k, op(B) k x n
// (part: optional split-K scratch of part_bytes)
tp::CgemmArgs gemm_args(tp::Planes a, long long lda, long long sa, tp::Planes b, long long ldb, long long sb,
                        tp::Planes c, long long ldc, long long sc, int m, int n, int k, int nslices, int real_last,
                        float* part, size_t part_bytes)
{
    tp::CgemmArgs g{};
    g.ksplit = pick_ksplit(m, n, k, nslices, part ? part_bytes : 0);
    g.part = part;
    g.ar = a.re; g.ai = a.im; g.lda = lda; g.sa = sa;
    g.br = b.re; g.bi = b.im; g.ldb = ldb; g.sb = sb;
    g.cr = c.re; g.ci = c.im; g.ldc = ldc; g.sc = sc;
    g.m = m; g.n = n; g.k = k;
    g.nslices = nslices;
    g.real_first = 1;
    g.real_last = real_last;
    return g;
}

// device-side values of a launch (CgemmArgs): gate and caps of m, n, k
struct Dyn {
    const int* gate = nullptr;
    const int* m = nullptr;
    const int* n = nullptr;
    const int* k = nullptr;
};

void set_dyn(tp::CgemmArgs& g, const Dyn& d)
{
    g.gate = d.gate;
    g.dyn_m = d.m;
    g.dyn_n = d.n;
    g.dyn_k = d.k;
}

int gemm(tp::Planes a, long long lda, long long sa, int opa, tp::Planes b, long long ldb, long long sb, int opb,
         tp::Planes c, long long ldc, long long sc, int m, int n, int k, int nslices, int real_last, hipStream_t s,
         float* part = nullptr, size_t part_bytes = 0, const Dyn& d = Dyn())
{
    tp::CgemmArgs g = gemm_args(a, lda, sa, b, ldb, sb, c, ldc, sc, m, n, k, nslices, real_last, part, part_bytes);
    set_dyn(g, d);
    TP_LAUNCH(tp::K_CGEMM, s, tp::launch_cgemm(g, opa, opb, TP_PREC_FP32, s));
    return TP_OK;
}

// CholeskyQR of y (rows x L per slice) with `passes` passes (2: CholeskyQR2),
// tmp of the same size; the result ends in y (with one pass the two plane
// pairs are swapped).  With want_r (two passes) the combined R of both
// passes is kept and R^* written to Lw.rh.  gram_ready: the first pass's
// Gram partials are already in Lw.part (gemm_gram).
// gate / width: the call's device gate and live sketch width (L is the
// launch width, max_rank)
int cholqr(LearnedLayout& Lw, tp::Planes& y, tp::Planes& tmp, int rows, int L, int h, int real_last, int passes,
           bool want_r, hipStream_t s, bool gram_ready = false, const int* gate = nullptr, const int* width = nullptr)
{
    if (want_r && passes != 2) return TP_ERR_ARG;
    tp::Planes src = y, dst = tmp;
    // (columns past the live width: no later product, Gram or store reads them)
    Dyn d;
    d.gate = gate;
    d.k = width;
    d.n = width;
    for (int pass = 0; pass < passes; ++pass) {
        TP_LAUNCH(tp::K_CHOLQR, s,
                  tp::launch_cholqr_pass(src.re, src.im, rows, L, Lw.lact, h, pass, Lw.part, Lw.rinv.re, Lw.rinv.im,
                                         want_r ? Lw.rtot : nullptr, want_r ? Lw.rh.re : nullptr,
                                         want_r ? Lw.rh.im : nullptr, Lw.status, s, gram_ready && pass == 0, gate));
        const int st = gemm(src, L, (long long)rows * L, tp::OP_N, Lw.rinv, L, (long long)L * L, tp::OP_N, dst, L,
                            (long long)rows * L, rows, L, L, h, real_last, s, nullptr, 0, d);
        if (st != TP_OK) return st;
        std::swap(src, dst);
    }
    if (passes % 2) std::swap(y, tmp);
    return TP_OK;
}

// CholeskyQR2 of src into dst through mid (three buffers: the result lands in
// dst, whatever held it before)
int cholqr3(LearnedLayout& Lw, tp::Planes src, tp::Planes mid, tp::Planes dst, int rows, int L, int h, int real_last,
            hipStream_t s, const int* gate, const int* width)
{
    Dyn d;
    d.gate = gate;
    d.k = width;
    d.n = width;
    const tp::Planes io[3] = {src, mid, dst};
    for (int pass = 0; pass < 2; ++pass) {
        TP_LAUNCH(tp::K_CHOLQR, s,
                  tp::launch_cholqr_pass(io[pass].re, io[pass].im, rows, L, Lw.lact, h, pass, Lw.part, Lw.rinv.re,
                                         Lw.rinv.im, nullptr, nullptr, nullptr, Lw.status, s, false, gate));
        const int st = gemm(io[pass], L, (long long)rows * L, tp::OP_N, Lw.rinv, L, (long long)L * L, tp::OP_N,
                            io[pass + 1], L, (long long)rows * L, rows, L, L, h, real_last, s, nullptr, 0, d);
        if (st != TP_OK) return st;
    }
    return TP_OK;
}

// device int ranges copied, one after the other, to dst on the host through a
// pinned buffer of the calling thread (kept for the life of the process), after the work queued
// on s before the call: the host-driven form of the learned-rank prox reads
// its device decisions with this.
struct IntRange {
    const int* src;
    int n;
};
hipError_t read_device_ints(std::initializer_list<IntRange> ranges, int* dst, hipStream_t s)
{
    thread_local int* pin = nullptr;
    thread_local int cap = 0;
    int total = 0;
    for (const IntRange& r : ranges) total += r.n;
    if (total > cap) {
        const int want = std::max(total, 1024);
        int* p = nullptr;
        const hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&p), (size_t)want * sizeof(int),
                                           hipHostMallocDefault);
        if (e != hipSuccess) return e;
        if (pin) (void)hipHostFree(pin);  // every earlier copy has completed (synchronized below)
        pin = p;
        cap = want;
    }
    hipError_t e = hipSuccess;
    int at = 0;
    for (const IntRange& r : ranges) {  // one after the other in dst
        if (e == hipSuccess && r.n > 0)
            e = hipMemcpyAsync(pin + at, r.src, (size_t)r.n * sizeof(int), hipMemcpyDeviceToHost, s);
        at += r.n;
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    std::memcpy(dst, pin, (size_t)total * sizeof(int));
    return hipSuccess;
}

// The range-finder product C = op(A) B (m x n per slice, row-major, packed)
// whose result a CholeskyQR takes next: a split narrow product leaves its
// parts, and their sum is formed together with the first pass's Gram (one
// pass over C instead of the reduction's write and the Gram's read).
// *gram_ready tells the CholeskyQR whether that happened.
int gemm_gram(LearnedLayout& Lw, tp::Planes a, long long lda, long long sa, int opa, tp::Planes b, long long ldb,
              long long sb, tp::Planes c, int m, int n, int k, int nslices, int real_last, hipStream_t s,
              bool* gram_ready, const int* gate = nullptr, const int* width = nullptr)
{
    const long long sc = (long long)m * n;
    tp::CgemmArgs g = gemm_args(a, lda, sa, b, ldb, sb, c, n, sc, m, n, k, nslices, real_last, Lw.kpart,
                                Lw.kpart_bytes);
    Dyn d;
    d.gate = gate;
    d.n = width;
    set_dyn(g, d);
    *gram_ready = false;
    if (!tp::cgemm_parts_ok(g, opa, tp::OP_N))
        return gemm(a, lda, sa, opa, b, ldb, sb, tp::OP_N, c, n, sc, m, n, k, nslices, real_last, s, Lw.kpart,
                    Lw.kpart_bytes, d);
    TP_LAUNCH(tp::K_CGEMM, s, tp::launch_cgemm_parts(g, opa, tp::OP_N, s));
    TP_LAUNCH(tp::K_CHOLQR, s,
              tp::launch_reduce_gram(Lw.kpart, g.ksplit, m, n, nslices, 1, real_last, c.re, c.im, Lw.lact, Lw.part, s,
                                     gate, width));
    *gram_ready = true;
    return TP_OK;
}

// Workspace of tsvd.
struct TsvdLayout {
    tp::Planes abar, l, q, s;
    float2* cols;
    float2* v;
    double* sigma;
    void* jscratch;
    size_t jscratch_bytes;
};

tp::Arena tsvd_arena(void* ws, size_t bytes, int n1, int n2, int n3, TsvdLayout* L)
{
    const size_t h = (size_t)tp::half_slices(n3);
    const size_t R = n1 >= n2 ? n1 : n2, P = n1 >= n2 ? n2 : n1, mn = (size_t)n1 * n2;
    tp::Arena ar(ws, bytes);
    TsvdLayout t{};
    t.abar.re = ar.take<float>(h * mn);
    t.abar.im = ar.take<float>(h * mn);
    t.cols = ar.take<float2>(h * R * P);
    t.v = ar.take<float2>(h * P * P);
    t.sigma = ar.take<double>(h * P);
    t.l.re = ar.take<float>(h * R * R);
    t.l.im = ar.take<float>(h * R * R);
    t.q.re = ar.take<float>(h * P * P);
    t.q.im = ar.take<float>(h * P * P);
    t.s.re = ar.take<float>(h * mn);
    t.s.im = ar.take<float>(h * mn);
    t.jscratch_bytes = tp::jacobi_scratch_bytes(n1, n2, (int)h, true);
    t.jscratch = t.jscratch_bytes ? ar.take<char>(t.jscratch_bytes) : nullptr;
    if (L) *L = t;
    return ar;
}

// Order-p tensors: dims[0 .. nd-1] = n3 .. np (host array).  Shape check and
// the slice counts: h = r * (floor(np/2)+1) Fourier slices, r = n3 ... n_(p-1).
constexpr int kMaxNd = 8;
constexpr long long kMaxSlicesNd = 65535;  // slice counts index a grid dimension

int check_nd(int nd, const int* dims, long long* h, long long* r)
{
    if (nd < 1 || nd > kMaxNd) return TP_ERR_SHAPE;
    if (!dims) return TP_ERR_ARG;
    long long rr = 1;
    for (int a = 0; a < nd; ++a) {
        if (dims[a] <= 0 || dims[a] > kMaxN3) return TP_ERR_SHAPE;
        if (a < nd - 1) rr *= dims[a];
        if (rr > kMaxSlicesNd) return TP_ERR_SHAPE;
    }
    const long long hh = rr * (dims[nd - 1] / 2 + 1);
    if (hh > kMaxSlicesNd) return TP_ERR_SHAPE;
    *h = hh;
    *r = rr;
    return TP_OK;
}

// Workspace of tprod_nd: the A, B, C slices and one scratch set for the transforms.
struct TprodNdLayout {
    tp::Planes a, b, c, tmp;
};

tp::Arena tprod_nd_arena(void* ws, size_t bytes, int n1, int n2, int l, size_t h, TprodNdLayout* L)
{
    tp::Arena ar(ws, bytes);
    TprodNdLayout t{};
    const size_t sa = h * n1 * n2, sb = h * n2 * l, sc = h * n1 * l;
    t.a.re = ar.take<float>(sa);
    t.a.im = ar.take<float>(sa);
    t.b.re = ar.take<float>(sb);
    t.b.im = ar.take<float>(sb);
    t.c.re = ar.take<float>(sc);
    t.c.im = ar.take<float>(sc);
    const size_t st = std::max(sa, std::max(sb, sc));
    t.tmp.re = ar.take<float>(st);
    t.tmp.im = ar.take<float>(st);
    if (L) *L = t;
    return ar;
}

}  // namespace

namespace tp {

// Argument checks of tp_tprod (Definition 2.1 sizes).
int check_tprod(const float* A, const float* B, const float* C, int n1, int n2, int l, int n3, int prec)
{
    if (!A || !B || !C) return TP_ERR_ARG;
    if (prec != TP_PREC_FP32 && prec != TP_PREC_BF16X3 && prec != TP_PREC_BF16) return TP_ERR_ARG;
    if (::bad_dim(n1) || ::bad_dim(n2) || ::bad_dim(l) || ::bad_dim(n3) || n3 > kMaxN3) return TP_ERR_SHAPE;
    if (::bad_slice(n1, n2) || ::bad_slice(n2, l) || ::bad_slice(n1, l)) return TP_ERR_SHAPE;
    return TP_OK;
}

// Algorithm 1 on checked arguments, with the half spectra in `workspace`.
int run_tprod(const float* A, const float* B, float* C, int n1, int n2, int l, int n3, int prec, void* workspace,
              size_t workspace_bytes, hipStream_t s)
{
    TprodLayout L;
    tp::Arena ar = ::tprod_arena(workspace, workspace_bytes, n1, n2, l, n3, prec, &L);
    if (!ar.ok) return TP_ERR_WORKSPACE;
    const int h = tp::half_slices(n3);
    if (prec != TP_PREC_FP32) {
        // step 1 into bf16 planes: A row-major (n1 x n2), B transposed (l x n2)
        const long long pa = (long long)h * n1 * L.ld, pb = (long long)h * l * L.ld;
        const int split = prec == TP_PREC_BF16X3 ? 1 : 0;
        const tp::SplitOut oa{L.ah, pa, (long long)n1 * L.ld, n1, n2, L.ld, L.bkl, n2, 1, split};
        const tp::SplitOut ob{L.bh, pb, (long long)l * L.ld, l, n2, L.ld, L.bkl, 1, l, split};
        TP_LAUNCH(tp::K_RFFT, s, tp::launch_rfft_split(A, oa, n3, s));
        TP_LAUNCH(tp::K_RFFT, s, tp::launch_rfft_split(B, ob, n3, s));
        // step 2: slices 0 and (even n3) h-1 are real
        tp::Bf16Args g{};
        g.a = L.ah;
        g.b = L.bh;
        g.a_plane = pa;
        g.a_slice = (long long)n1 * L.ld;
        g.b_plane = pb;
        g.b_slice = (long long)l * L.ld;
        g.ld = L.ld;
        g.bkl = L.bkl;
        g.variant = L.variant;
        g.cr = L.c.re;
        g.ci = L.c.im;
        g.ldc = l;
        g.sc = (long long)n1 * l;
        g.m = n1;
        g.n = l;
        g.k = n2;
        g.nreal = real_slices(n3);
        g.real_s[0] = 0;
        g.real_s[1] = h - 1;
        g.cs0 = 1;
        g.ncs = h - g.nreal;
        g.split = split;
        TP_LAUNCH(tp::K_CGEMM, s, tp::launch_cgemm_bf16(g, s));
        TP_LAUNCH(tp::K_IRFFT, s, tp::launch_irfft(L.c.re, L.c.im, C, (long long)n1 * l, n3, s));
        return TP_OK;
    }
    // Algorithm 1, step 1: DFT of the tubes of A and B
    TP_LAUNCH(tp::K_RFFT, s, tp::launch_rfft(A, L.a.re, L.a.im, (long long)n1 * n2, n3, s));
    TP_LAUNCH(tp::K_RFFT, s, tp::launch_rfft(B, L.b.re, L.b.im, (long long)n2 * l, n3, s));
    // step 2: Cbar^(k) = Abar^(k) Bbar^(k), k < floor(n3/2)+1
    tp::CgemmArgs g{};
    g.ar = L.a.re;
    g.ai = L.a.im;
    g.lda = n2;
    g.sa = (long long)n1 * n2;
    g.br = L.b.re;
    g.bi = L.b.im;
    g.ldb = l;
    g.sb = (long long)n2 * l;
    g.cr = L.c.re;
    g.ci = L.c.im;
    g.ldc = l;
    g.sc = (long long)n1 * l;
    g.m = n1;
    g.n = l;
    g.k = n2;
    g.nslices = h;
    g.real_first = 1;
    g.real_last = (n3 % 2 == 0) ? 1 : 0;
    g.kdyn = nullptr;
    TP_LAUNCH(tp::K_CGEMM, s, tp::launch_cgemm(g, tp::OP_N, tp::OP_N, prec, s));
    // step 3: inverse DFT (conjugate fill implicit)
    TP_LAUNCH(tp::K_IRFFT, s, tp::launch_irfft(L.c.re, L.c.im, C, (long long)n1 * l, n3, s));
    return TP_OK;
}


}  // namespace tp

extern "C" {

const char* tp_status_string(int status)
{
    switch (status) {
        case TP_OK: return "ok";
        case TP_ERR_ARG: return "invalid argument";
        case TP_ERR_SHAPE: return "invalid or unsupported shape";
        case TP_ERR_WORKSPACE: return "workspace missing or too small";
        case TP_ERR_HIP: return "HIP kernel launch failed";
        case TP_ERR_UNSUPPORTED: return "unsupported request";
        default: return "unknown status";
    }
}

int tp_version(void) { return 100; }

size_t tp_tprod_workspace_size(int n1, int n2, int l, int n3, int prec)
{
    if (bad_dim(n1) || bad_dim(n2) || bad_dim(l) || bad_dim(n3)) return 0;
    if (prec != TP_PREC_FP32 && prec != TP_PREC_BF16X3 && prec != TP_PREC_BF16) return 0;
    return tprod_arena(nullptr, 0, n1, n2, l, n3, prec, nullptr).used;
}

int tp_tprod(const float* A, const float* B, float* C, int n1, int n2, int l, int n3, int prec,
             void* workspace, size_t workspace_bytes, void* stream)
{
    const int c = tp::check_tprod(A, B, C, n1, n2, l, n3, prec);
    if (c != TP_OK) return c;
    return tp::run_tprod(A, B, C, n1, n2, l, n3, prec, workspace, workspace_bytes, as_stream(stream));
}

size_t tp_prox_tnn_workspace_size(int n1, int n2, int n3)
{
    if (bad_dim(n1) || bad_dim(n2) || bad_dim(n3)) return 0;
    return svt_arena(nullptr, 0, n1, n2, n3, true, nullptr).used;
}

int tp_prox_tnn(const float* Y, float* X, int n1, int n2, int n3, float tau, int* info, int* rank,
                void* workspace, size_t workspace_bytes, void* stream)
{
    if (!Y || !X) return TP_ERR_ARG;
    if (!(tau >= 0.0f) || std::isinf(tau)) return TP_ERR_ARG;
    if (bad_dim(n1) || bad_dim(n2) || bad_dim(n3) || n3 > kMaxN3) return TP_ERR_SHAPE;
    if (bad_slice(n1, n2) || (n1 > 2048 && n2 > 2048)) return TP_ERR_SHAPE;
    if ((n1 < n2 ? n2 : n1) > 2048) return TP_ERR_UNSUPPORTED;
    SvtLayout L;
    tp::Arena ar = svt_arena(workspace, workspace_bytes, n1, n2, n3, true, &L);
    if (!ar.ok) return TP_ERR_WORKSPACE;
    hipStream_t s = as_stream(stream);
    const int h = tp::half_slices(n3);
    const long long mn = (long long)n1 * n2;

    // Algorithm 3, step 1
    TP_LAUNCH(tp::K_RFFT, s, tp::launch_rfft(Y, L.ybar.re, L.ybar.im, mn, n3, s));
    // step 2: matrix SVT of each leading slice, in place in L.ybar
    const int st = run_svt(L, L.ybar, n1, n2, h, 1, (n3 % 2 == 0) ? 1 : 0, (double)tau, info, rank, s);
    if (st != TP_OK) return st;
    // step 3: inverse DFT (conjugate fill implicit)
    TP_LAUNCH(tp::K_IRFFT, s, tp::launch_irfft(L.ybar.re, L.ybar.im, X, mn, n3, s));
    return TP_OK;
}

size_t tp_tnn_workspace_size(int n1, int n2, int n3)
{
    if (bad_dim(n1) || bad_dim(n2) || bad_dim(n3)) return 0;
    return svt_arena(nullptr, 0, n1, n2, n3, false, nullptr).used;
}

int tp_tnn(const float* A, int n1, int n2, int n3, double* out, int* info, void* workspace,
           size_t workspace_bytes, void* stream)
{
    if (!A || !out) return TP_ERR_ARG;
    if (bad_dim(n1) || bad_dim(n2) || bad_dim(n3) || n3 > kMaxN3) return TP_ERR_SHAPE;
    if (bad_slice(n1, n2)) return TP_ERR_SHAPE;
    if ((n1 < n2 ? n2 : n1) > 2048) return TP_ERR_UNSUPPORTED;
    SvtLayout L;
    tp::Arena ar = svt_arena(workspace, workspace_bytes, n1, n2, n3, false, &L);
    if (!ar.ok) return TP_ERR_WORKSPACE;
    hipStream_t s = as_stream(stream);
    const int h = tp::half_slices(n3);
    const bool tr = n1 < n2;
    TP_LAUNCH(tp::K_RFFT, s, tp::launch_rfft(A, L.ybar.re, L.ybar.im, (long long)n1 * n2, n3, s));
    tp::JacobiArgs j{};
    j.yr = L.ybar.re;
    j.yi = L.ybar.im;
    j.sigma = L.sigma;
    j.info = info;
    j.m = n1;
    j.n = n2;
    j.nslices = h;
    j.max_sweeps = tp::param(TP_PARAM_JACOBI_SWEEPS);
    j.transpose = tr ? 1 : 0;
    j.tol = tp::jacobi_tol(tr ? n2 : n1);
    TP_LAUNCH(tp::K_JACOBI, s, tp::launch_jacobi(j, L.jscratch, L.jscratch_bytes, s));
    TP_LAUNCH(tp::K_TNN_REDUCE, s, tp::launch_tnn_reduce(L.sigma, h, tr ? n1 : n2, n3, out, s));
    return TP_OK;
}

// ------------------------------------------------------ order-p tensors --
size_t tp_tprod_nd_workspace_size(int n1, int n2, int l, int nd, const int* dims)
{
    long long h = 0, r = 0;
    if (bad_dim(n1) || bad_dim(n2) || bad_dim(l) || check_nd(nd, dims, &h, &r) != TP_OK) return 0;
    return tprod_nd_arena(nullptr, 0, n1, n2, l, (size_t)h, nullptr).used;
}

int tp_tprod_nd(const float* A, const float* B, float* C, int n1, int n2, int l, int nd, const int* dims,
                void* workspace, size_t workspace_bytes, void* stream)
{
    if (!A || !B || !C) return TP_ERR_ARG;
    long long h = 0, r = 0;
    const int c = check_nd(nd, dims, &h, &r);
    if (c != TP_OK) return c;
    if (bad_dim(n1) || bad_dim(n2) || bad_dim(l)) return TP_ERR_SHAPE;
    if (bad_slice(n1, n2) || bad_slice(n2, l) || bad_slice(n1, l)) return TP_ERR_SHAPE;
    TprodNdLayout L;
    tp::Arena ar = tprod_nd_arena(workspace, workspace_bytes, n1, n2, l, (size_t)h, &L);
    if (!ar.ok) return TP_ERR_WORKSPACE;
    hipStream_t s = as_stream(stream);
    // DFT over modes 3..p of the frontal elements of A and B
    TP_LAUNCH(tp::K_RFFT, s, tp::launch_rfft_nd(A, (long long)n1 * n2, nd, dims, L.a, L.tmp, s));
    TP_LAUNCH(tp::K_RFFT, s, tp::launch_rfft_nd(B, (long long)n2 * l, nd, dims, L.b, L.tmp, s));
    // the order-p form of eq (10): Cbar = Abar Bbar on every kept slice
    tp::CgemmArgs g{};
    g.ar = L.a.re;
    g.ai = L.a.im;
    g.lda = n2;
    g.sa = (long long)n1 * n2;
    g.br = L.b.re;
    g.bi = L.b.im;
    g.ldb = l;
    g.sb = (long long)n2 * l;
    g.cr = L.c.re;
    g.ci = L.c.im;
    g.ldc = l;
    g.sc = (long long)n1 * l;
    g.m = n1;
    g.n = l;
    g.k = n2;
    g.nslices = (int)h;
    g.real_first = 1;  // all bins 0
    g.real_last = (nd == 1 && dims[0] % 2 == 0) ? 1 : 0;
    TP_LAUNCH(tp::K_CGEMM, s, tp::launch_cgemm(g, tp::OP_N, tp::OP_N, TP_PREC_FP32, s));
    TP_LAUNCH(tp::K_IRFFT, s, tp::launch_irfft_nd(L.c, L.tmp, C, (long long)n1 * l, nd, dims, s));
    return TP_OK;
}

size_t tp_prox_tnn_nd_workspace_size(int n1, int n2, int nd, const int* dims)
{
    long long h = 0, r = 0;
    if (bad_dim(n1) || bad_dim(n2) || check_nd(nd, dims, &h, &r) != TP_OK) return 0;
    return svt_arena_h(nullptr, 0, n1, n2, (size_t)h, true, nullptr).used;
}

int tp_prox_tnn_nd(const float* Y, float* X, int n1, int n2, int nd, const int* dims, float tau, int* info,
                   int* rank, void* workspace, size_t workspace_bytes, void* stream)
{
    if (!Y || !X) return TP_ERR_ARG;
    if (!(tau >= 0.0f) || std::isinf(tau)) return TP_ERR_ARG;
    long long h = 0, r = 0;
    const int c = check_nd(nd, dims, &h, &r);
    if (c != TP_OK) return c;
    if (bad_dim(n1) || bad_dim(n2) || bad_slice(n1, n2)) return TP_ERR_SHAPE;
    if ((n1 < n2 ? n2 : n1) > 2048) return TP_ERR_UNSUPPORTED;
    SvtLayout L;
    tp::Arena ar = svt_arena_h(workspace, workspace_bytes, n1, n2, (size_t)h, true, &L);
    if (!ar.ok) return TP_ERR_WORKSPACE;
    hipStream_t s = as_stream(stream);
    const long long mn = (long long)n1 * n2;
    // the rotated-column planes are free until the SVT and after it: transform scratch
    TP_LAUNCH(tp::K_RFFT, s, tp::launch_rfft_nd(Y, mn, nd, dims, L.ybar, L.w, s));
    const int st = run_svt(L, L.ybar, n1, n2, (int)h, 1, (nd == 1 && dims[0] % 2 == 0) ? 1 : 0, (double)tau,
                           info, rank, s);
    if (st != TP_OK) return st;
    TP_LAUNCH(tp::K_IRFFT, s, tp::launch_irfft_nd(L.ybar, L.w, X, mn, nd, dims, s));
    return TP_OK;
}

size_t tp_tnn_nd_workspace_size(int n1, int n2, int nd, const int* dims)
{
    long long h = 0, r = 0;
    if (bad_dim(n1) || bad_dim(n2) || check_nd(nd, dims, &h, &r) != TP_OK) return 0;
    return svt_arena_h(nullptr, 0, n1, n2, (size_t)h, false, nullptr, false, true).used;
}

int tp_tnn_nd(const float* A, int n1, int n2, int nd, const int* dims, double* out, int* info, void* workspace,
              size_t workspace_bytes, void* stream)
{
    if (!A || !out) return TP_ERR_ARG;
    long long h = 0, r = 0;
    const int c = check_nd(nd, dims, &h, &r);
    if (c != TP_OK) return c;
    if (bad_dim(n1) || bad_dim(n2) || bad_slice(n1, n2)) return TP_ERR_SHAPE;
    if ((n1 < n2 ? n2 : n1) > 2048) return TP_ERR_UNSUPPORTED;
    SvtLayout L;
    tp::Arena ar = svt_arena_h(workspace, workspace_bytes, n1, n2, (size_t)h, false, &L, false, true);
    if (!ar.ok) return TP_ERR_WORKSPACE;
    hipStream_t s = as_stream(stream);
    const bool tr = n1 < n2;
    TP_LAUNCH(tp::K_RFFT, s, tp::launch_rfft_nd(A, (long long)n1 * n2, nd, dims, L.ybar, L.tmp, s));
    tp::JacobiArgs j{};
    j.yr = L.ybar.re;
    j.yi = L.ybar.im;
    j.sigma = L.sigma;
    j.info = info;
    j.m = n1;
    j.n = n2;
    j.nslices = (int)h;
    j.max_sweeps = tp::param(TP_PARAM_JACOBI_SWEEPS);
    j.transpose = tr ? 1 : 0;
    j.tol = tp::jacobi_tol(tr ? n2 : n1);
    TP_LAUNCH(tp::K_JACOBI, s, tp::launch_jacobi(j, L.jscratch, L.jscratch_bytes, s));
    TP_LAUNCH(tp::K_TNN_REDUCE, s,
              tp::launch_tnn_reduce(L.sigma, (int)h, tr ? n1 : n2, dims[nd - 1], out, s, (int)r));
    return TP_OK;
}

// singular values of the h leading slices into L.sigma (unsorted), for tsn and tubalrank
int slice_sigmas(const float* A, int n1, int n2, int n3, const SvtLayout& L, int* info, hipStream_t s)
{
    const int h = tp::half_slices(n3);
    const bool tr = n1 < n2;
    TP_LAUNCH(tp::K_RFFT, s, tp::launch_rfft(A, L.ybar.re, L.ybar.im, (long long)n1 * n2, n3, s));
    tp::JacobiArgs j{};
    j.yr = L.ybar.re;
    j.yi = L.ybar.im;
    j.sigma = L.sigma;
    j.info = info;
    j.m = n1;
    j.n = n2;
    j.nslices = h;
    j.max_sweeps = tp::param(TP_PARAM_JACOBI_SWEEPS);
    j.transpose = tr ? 1 : 0;
    j.tol = tp::jacobi_tol(tr ? n2 : n1);
    TP_LAUNCH(tp::K_JACOBI, s, tp::launch_jacobi(j, L.jscratch, L.jscratch_bytes, s));
    return TP_OK;
}

int check_sigma_call(const float* A, const void* out, int n1, int n2, int n3)
{
    if (!A || !out) return TP_ERR_ARG;
    if (bad_dim(n1) || bad_dim(n2) || bad_dim(n3) || n3 > kMaxN3) return TP_ERR_SHAPE;
    if (bad_slice(n1, n2)) return TP_ERR_SHAPE;
    if ((n1 < n2 ? n2 : n1) > 2048) return TP_ERR_UNSUPPORTED;
    return TP_OK;
}

size_t tp_tsn_workspace_size(int n1, int n2, int n3) { return tp_tnn_workspace_size(n1, n2, n3); }

int tp_tsn(const float* A, int n1, int n2, int n3, double* out, int* info, void* workspace, size_t workspace_bytes,
           void* stream)
{
    const int c = check_sigma_call(A, out, n1, n2, n3);
    if (c != TP_OK) return c;
    SvtLayout L;
    tp::Arena ar = svt_arena(workspace, workspace_bytes, n1, n2, n3, false, &L);
    if (!ar.ok) return TP_ERR_WORKSPACE;
    hipStream_t s = as_stream(stream);
    const int st = slice_sigmas(A, n1, n2, n3, L, info, s);
    if (st != TP_OK) return st;
    TP_LAUNCH(tp::K_TNN_REDUCE, s,
              tp::launch_tsn_reduce(L.sigma, tp::half_slices(n3), n1 < n2 ? n1 : n2, out, s));
    return TP_OK;
}

size_t tp_tubalrank_workspace_size(int n1, int n2, int n3)
{
    const size_t base = tp_tnn_workspace_size(n1, n2, n3);
    if (!base) return 0;
    return base + tp::align_up((size_t)tp::half_slices(n3) * (n1 < n2 ? n1 : n2) * sizeof(double));
}

int tp_tubalrank(const float* A, int n1, int n2, int n3, double tol, int* out, int* info, void* workspace,
                 size_t workspace_bytes, void* stream)
{
    const int c = check_sigma_call(A, out, n1, n2, n3);
    if (c != TP_OK) return c;
    if (std::isnan(tol) || std::isinf(tol)) return TP_ERR_ARG;
    SvtLayout L;
    tp::Arena ar = svt_arena(workspace, workspace_bytes, n1, n2, n3, false, &L);
    double* sorted = ar.take<double>((size_t)tp::half_slices(n3) * (n1 < n2 ? n1 : n2));
    if (!ar.ok) return TP_ERR_WORKSPACE;
    hipStream_t s = as_stream(stream);
    const int st = slice_sigmas(A, n1, n2, n3, L, info, s);
    if (st != TP_OK) return st;
    const double scale = (double)(n1 > n2 ? n1 : n2) * 0x1p-23;  // max(n1, n2) * eps of FP32
    TP_LAUNCH(tp::K_TNN_REDUCE, s,
              tp::launch_tubal_rank(L.sigma, sorted, tp::half_slices(n3), n1 < n2 ? n1 : n2, n3, tol, scale, out,
                                    s));
    return TP_OK;
}

int tp_tran(const float* A, float* out, int n1, int n2, int n3, void* stream)
{
    if (!A || !out) return TP_ERR_ARG;
    if (bad_dim(n1) || bad_dim(n2) || bad_dim(n3)) return TP_ERR_SHAPE;
    if (A == out && !(n1 == 1 && n2 == 1 && n3 == 1)) return TP_ERR_ARG;  // not in place
    hipStream_t s = as_stream(stream);
    TP_LAUNCH(tp::K_TENSOR_OP, s, tp::launch_tran(A, out, n1, n2, n3, s));
    return TP_OK;
}

int tp_teye(float* out, int n, int n3, void* stream)
{
    if (!out) return TP_ERR_ARG;
    if (bad_dim(n) || bad_dim(n3)) return TP_ERR_SHAPE;
    hipStream_t s = as_stream(stream);
    TP_LAUNCH(tp::K_TENSOR_OP, s, tp::launch_teye(out, n, n3, s));
    return TP_OK;
}

size_t tp_tsvd_workspace_size(int n1, int n2, int n3)
{
    if (bad_dim(n1) || bad_dim(n2) || bad_dim(n3)) return 0;
    return tsvd_arena(nullptr, 0, n1, n2, n3, nullptr).used;
}

int tp_tsvd(const float* A, float* U, float* S, float* V, int n1, int n2, int n3, int* info, void* workspace,
            size_t workspace_bytes, void* stream)
{
    if (!A || !U || !S || !V) return TP_ERR_ARG;
    if (bad_dim(n1) || bad_dim(n2) || bad_dim(n3) || n3 > kMaxN3) return TP_ERR_SHAPE;
    if (bad_slice(n1, n2) || bad_slice(n1, n1) || bad_slice(n2, n2)) return TP_ERR_SHAPE;
    if ((n1 < n2 ? n2 : n1) > 2048) return TP_ERR_UNSUPPORTED;
    TsvdLayout L;
    tp::Arena ar = tsvd_arena(workspace, workspace_bytes, n1, n2, n3, &L);
    if (!ar.ok) return TP_ERR_WORKSPACE;
    hipStream_t s = as_stream(stream);
    const int h = tp::half_slices(n3);
    const bool tr = n1 < n2;
    const int R = tr ? n2 : n1, P = tr ? n1 : n2;
    // Algorithm 2, step 1
    TP_LAUNCH(tp::K_RFFT, s, tp::launch_rfft(A, L.abar.re, L.abar.im, (long long)n1 * n2, n3, s));
    // step 2: SVD of each leading slice (real Jacobi on the real slices), bases sorted and completed
    tp::JacobiArgs j{};
    j.yr = L.abar.re;
    j.yi = L.abar.im;
    j.sigma = L.sigma;
    j.info = info;
    j.m = n1;
    j.n = n2;
    j.nslices = h;
    j.max_sweeps = tp::param(TP_PARAM_JACOBI_SWEEPS);
    j.transpose = tr ? 1 : 0;
    j.tol = tp::jacobi_tol(R);
    j.cols = L.cols;
    j.qout = L.v;
    TP_LAUNCH(tp::K_JACOBI, s, tp::launch_jacobi(j, L.jscratch, L.jscratch_bytes, s));
    TP_LAUNCH(tp::K_TSVD_FINISH, s,
              tp::launch_tsvd_finish(L.cols, L.sigma, L.v, L.l, L.q, L.s, R, P, n1, n2, h, s));
    // A = L S Q^* slice-wise (or Q S L^* for the transposed work matrix)
    const tp::Planes& ub = tr ? L.q : L.l;
    const tp::Planes& vb = tr ? L.l : L.q;
    // step 3: inverse DFTs (conjugate fill of the trailing slices implicit)
    TP_LAUNCH(tp::K_IRFFT, s, tp::launch_irfft(ub.re, ub.im, U, (long long)n1 * n1, n3, s));
    TP_LAUNCH(tp::K_IRFFT, s, tp::launch_irfft(L.s.re, L.s.im, S, (long long)n1 * n2, n3, s));
    TP_LAUNCH(tp::K_IRFFT, s, tp::launch_irfft(vb.re, vb.im, V, (long long)n2 * n2, n3, s));
    return TP_OK;
}

size_t tp_prox_tnn_learned_workspace_size(int n1, int n2, int n3, int max_rank)
{
    if (bad_dim(n1) || bad_dim(n2) || bad_dim(n3) || max_rank < 1 || max_rank > tp::kMaxL) return 0;
    return learned_arena(nullptr, 0, n1, n2, n3, max_rank, nullptr).used;
}

int tp_prox_tnn_learned(const float* Y, float* X, int n1, int n2, int n3, float tau, const tp_learned_opts* opts,
                        int* rank, int* fallback, int* info, float* sigma_out, void* workspace, size_t workspace_bytes,
                        void* stream)
{
    if (!Y || !X || !opts) return TP_ERR_ARG;
    if (!(tau >= 0.0f) || std::isinf(tau)) return TP_ERR_ARG;
    if (opts->max_rank < 1 || opts->max_rank > tp::kMaxL || opts->oversample < 0 || opts->power_iters < 0 ||
        opts->power_iters > 16 || opts->max_power_iters > 64 || !(opts->accuracy >= 0.0f) ||
        (!opts->mlp && opts->fixed_rank < 0) || opts->accuracy_ref < 0 || opts->accuracy_ref > 1)
        return TP_ERR_ARG;
    if (bad_dim(n1) || bad_dim(n2) || bad_dim(n3) || n3 > kMaxN3) return TP_ERR_SHAPE;
    if (bad_slice(n1, n2)) return TP_ERR_SHAPE;
    if ((n1 < n2 ? n2 : n1) > 2048) return TP_ERR_UNSUPPORTED;
    LearnedLayout W;
    tp::Arena ar = learned_arena(workspace, workspace_bytes, n1, n2, n3, opts->max_rank, &W);
    if (!ar.ok) return TP_ERR_WORKSPACE;
    hipStream_t s = as_stream(stream);
    const int h = tp::half_slices(n3), p = n1 < n2 ? n1 : n2, rl = (n3 % 2 == 0) ? 1 : 0;
    const long long mn = (long long)n1 * n2;
    int* fb = fallback ? fallback : W.fb;
    int* rk = rank ? rank : W.rank;
    const tp::Planes ybar = W.full.ybar;
    // Every launch below is sized for the widest sketch, L = max_rank; the
    // width a call actually uses, which slices take the randomized path,
    // whether an accuracy round or the wide retry runs, and which slices
    // fall back are decided on the device (W.ctl) and read by the launches
    // themselves, so the call never waits for the host and can be captured
    // in a HIP graph.
    const int L = opts->max_rank;
    int* ctl = W.ctl;
    // Host-driven form (TP_PARAM_LEARNED_HOST = 1): the host reads those
    // decisions where they are taken (after each accuracy round, after the
    // retry test) and leaves out the launches that would exit at their gate;
    // the call then waits for the device there and cannot be captured, so a
    // capturing stream keeps the device-gated form.  Both give the same bits.
    bool host = tp::param(TP_PARAM_LEARNED_HOST) == 1;
    if (host) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) host = false;
    }
    const int qmax = std::max(opts->max_power_iters, opts->power_iters);
    const int rounds = opts->accuracy > 0.0f ? std::min(qmax - opts->power_iters, kMaxRounds - 1) : 0;

    TP_LAUNCH(tp::K_RFFT, s, tp::launch_rfft(Y, ybar.re, ybar.im, mn, n3, s));
    // predicted count per slice and sketch width
    TP_LAUNCH(tp::K_FEATURES, s,
              tp::launch_features(ybar.re, ybar.im, n1, n2, n3, h, (double)tau, opts->prev_rank, opts->prev_sigma,
                                  W.feats, W.fpart, W.fro2, s));
    TP_LAUNCH(tp::K_PREDICT, s,
              tp::launch_predict(opts->mlp, W.feats, h, p, opts->fixed_rank, opts->oversample, L, W.kpred, W.lact,
                                 W.prefb, rk, s));
    TP_LAUNCH(tp::K_PREDICT, s, tp::launch_fill_int(W.status, h, 0, s));
    TP_LAUNCH(tp::K_PREDICT, s, tp::launch_fill_int(ctl, C_COUNT, 0, s));
    TP_LAUNCH(tp::K_PREDICT, s,
              tp::launch_width(W.kpred, W.lact, W.prefb, fb, h, p, opts->oversample, L, nullptr, ctl + C_L1,
                               ctl + C_G1, true, s));

    tp::WarmBasis warm{};
    if (opts->warm_basis && opts->warm_cols) {
        warm.re = opts->warm_basis;
        warm.im = opts->warm_basis + (long long)h * n2 * opts->max_rank;
        warm.ld = opts->max_rank;
        warm.cols = opts->warm_cols;
    }
    const long long sy = (long long)n1 * L, sz = (long long)n2 * L, sl = (long long)L * L;

    // Host-driven form: when the first attempt's accuracy rounds end after a
    // host read, the same read takes the inputs of the wide-retry test (the
    // fallback flags, counts and widths are final there), and the host
    // applies the test of k_retry to them; with no retry the fallback count
    // is known as well, so the steady state waits for the device once.
    struct {
        bool valid = false, retry = false;
        int nfb = 0;
    } early;
    std::vector<int> hv;
    auto count_fb = [&](const int* v) {
        int c = 0;
        for (int q = 0; q < h; ++q) c += v[q] ? 1 : 0;
        return c;
    };

    // One attempt of the randomized SVT, run when *gate != 0 at sketch width *width.
    // (the retry attempt, at the widest sketch, has TP_PARAM_RETRY_ROUNDS
    // accuracy rounds, at most as many as the first)
    auto attempt = [&](int a, const int* gate, const int* width) -> int {
        int st = TP_OK;
        const int nround = a == 0 ? rounds : std::min(rounds, tp::param(TP_PARAM_RETRY_ROUNDS));
        // range finder: Y = Ybar Om, re-orthonormalised; power iterations
        TP_LAUNCH(tp::K_SKETCH, s,
                  tp::launch_sketch(W.om.re, W.om.im, n2, L, W.lact, h, n3, opts->seed, warm, s, gate));
        bool gr = false;
        st = gemm_gram(W, ybar, n2, mn, tp::OP_N, W.om, L, sz, W.ya, n1, L, n2, h, rl, s, &gr, gate, width);
        // a basis that only feeds the next power-iteration product takes one
        // (shifted, FP64 Gram) CholeskyQR pass: it needs to be well
        // conditioned, not orthonormal to working precision; the Y that the
        // projection Ybar^* Q uses (the last one) takes CholeskyQR2
        if (st == TP_OK)
            st = cholqr(W, W.ya, W.yb, n1, L, h, rl, opts->power_iters > 0 ? 1 : 2, false, s, gr, gate, width);
        for (int it = 0; st == TP_OK && it < opts->power_iters; ++it) {
            bool g1 = false, g2 = false;
            st = gemm_gram(W, ybar, n2, mn, tp::OP_C, W.ya, L, sy, W.za, n2, L, n1, h, rl, s, &g1, gate, width);
            if (st == TP_OK) st = cholqr(W, W.za, W.zb, n2, L, h, rl, 1, false, s, g1, gate, width);
            if (st == TP_OK)
                st = gemm_gram(W, ybar, n2, mn, tp::OP_N, W.za, L, sz, W.ya, n1, L, n2, h, rl, s, &g2, gate, width);
            if (st == TP_OK)
                st = cholqr(W, W.ya, W.yb, n1, L, h, rl, it + 1 == opts->power_iters ? 2 : 1, false, s, g2, gate,
                            width);
        }
        if (st != TP_OK) return st;
        Dyn dk;  // products over the sketch columns
        dk.gate = gate;
        dk.k = width;
        for (int r = 0; r <= nround; ++r) {
            // round r runs when the previous round's a posteriori check found
            // an inaccurate slice (round 0: when the attempt runs)
            const int* run = r == 0 ? gate : ctl + C_ROUND + 32 * a + r;
            // Bh = Ybar^* Q = Q2 R2
            bool gz = false;
            st = gemm_gram(W, ybar, n2, mn, tp::OP_C, W.ya, L, sy, W.za, n2, L, n1, h, rl, s, &gz, run, width);
            if (st == TP_OK) st = cholqr(W, W.za, W.zb, n2, L, h, rl, 2, true, s, gz, run, width);
            if (st != TP_OK) return st;
            // SVD of R2^* (one workgroup per slice, LDS), count check, core T
            tp::JacobiArgs j{};
            j.yr = W.rh.re;
            j.yi = W.rh.im;
            j.sigma = W.jsig;
            j.m = L;
            j.n = L;
            j.nslices = h;
            j.max_sweeps = tp::param(TP_PARAM_JACOBI_SWEEPS);
            j.tol = tp::jacobi_tol(L);
            j.cols = W.jcols;
            j.qout = W.jv;
            j.whole = 1;
            j.gate = run;
            j.pdyn = width;
            TP_LAUNCH(tp::K_JACOBI, s, tp::launch_jacobi(j, nullptr, 0, s));
            // (with the a posteriori check, V_r and C_r also go to the planar
            // operands of its products in the same launch)
            const bool acc = opts->accuracy > 0.0f;
            TP_LAUNCH(tp::K_RSVD_CHECK, s,
                      tp::launch_rsvd_check(W.jcols, W.jsig, W.jv, W.kpred, W.lact, W.prefb, W.status, L,
                                            (double)tau, W.T, fb, rk, h, s, run, acc ? W.vp : tp::Planes{},
                                            acc ? W.cp : tp::Planes{}));
            if (!acc) break;
            // a posteriori check: residuals Ybar v_j - sigma_j u_j of the kept Ritz triplets
            Dyn dr;
            dr.gate = run;
            dr.k = width;
            Dyn dn;
            dn.gate = run;
            dn.n = width;
            st = gemm(ybar, n2, mn, tp::OP_N, W.za, L, sz, tp::OP_N, W.yb, L, sy, n1, L, n2, h, rl, s, W.kpart,
                      W.kpart_bytes, dn);  // Ybar Q2
            if (st == TP_OK)
                st = gemm(W.yb, L, sy, tp::OP_N, W.vp, L, sl, tp::OP_N, W.t1, L, sy, n1, L, L, h, rl, s, nullptr, 0, dr);
            if (st == TP_OK)
                st = gemm(W.ya, L, sy, tp::OP_N, W.cp, L, sl, tp::OP_N, W.t2, L, sy, n1, L, L, h, rl, s, nullptr, 0, dr);
            if (st != TP_OK) return st;
            const bool last = r == nround;
            int* next = last ? nullptr : ctl + C_ROUND + 32 * a + r + 1;
            TP_LAUNCH(tp::K_ACCURACY, s,
                      tp::launch_accuracy_round(W.t1, W.t2, W.jsig, W.lact,
                                                opts->accuracy_ref == 0 ? W.fro2 : nullptr, n1, L, (double)tau,
                                                (double)opts->accuracy, W.bad, h, W.accpart, fb, run, next, last, s));
            if (last) break;
            if (host) {  // the later rounds run only when this one found an inaccurate slice
                const bool pre = a == 0 && opts->retry_wide;
                hv.resize(2 + 4 * h);
                const hipError_t e =
                    pre ? read_device_ints({{next, 1}, {ctl + C_G1, 1}, {fb, h}, {W.kpred, 3 * h}}, hv.data(), s)
                        : read_device_ints({{next, 1}}, hv.data(), s);
                if (e != hipSuccess) return TP_ERR_HIP;
                if (!hv[0] && pre) {  // the wide-retry test (k_retry) on the final flags of this attempt
                    const int* f = hv.data() + 2;
                    const int *kp = f + h, *la = kp + h, *pf = la + h;
                    const int kwide = std::min(std::max(L - opts->oversample, 0), p);
                    const int lwide = std::min(kwide + opts->oversample, p);
                    bool any = false;
                    for (int q = 0; q < h; ++q)
                        any = any || (hv[1] != 0 && f[q] && !pf[q] && la[q] < lwide && kp[q] < kwide);
                    early.valid = true;
                    early.retry = any;
                    early.nfb = count_fb(f);
                }
                if (!hv[0]) break;
            }
            // the next subspace iteration needs no new product: Ybar^* Y is
            // the projection just formed (its orthonormal basis Q2 is in W.za),
            // and Ybar Q2, whose span is that of the iteration's Ybar Z, is the
            // residual check's product in W.yb; Y = orth(Ybar Q2), its two
            // CholeskyQR passes going W.yb -> W.t1 -> W.ya
            st = cholqr3(W, W.yb, W.t1, W.ya, n1, L, h, rl, s, next, width);
            if (st != TP_OK) return st;
        }
        if (opts->basis_out && opts->basis_cols_out) {
            // the right Ritz vectors Q2 V for the next call's warm start: its
            // sketch then starts from the singular basis, so its R2^* comes out
            // nearly diagonal and the small Jacobi SVD needs few sweeps
            TP_LAUNCH(tp::K_ACCURACY, s, tp::launch_cm_to_planar(W.jv, W.vp, L, h, s, gate));
            st = gemm(W.za, L, sz, tp::OP_N, W.vp, L, sl, tp::OP_N, W.zb, L, sz, n2, L, L, h, rl, s, nullptr, 0, dk);
            if (st != TP_OK) return st;
            // (valid columns 0 for fallback slices, so a closed attempt stores zeros)
            TP_LAUNCH(tp::K_SKETCH, s,
                      tp::launch_store_basis(W.zb.re, W.zb.im, n2, L, W.lact, fb, h, opts->basis_out,
                                             opts->basis_out + (long long)h * n2 * opts->max_rank, opts->max_rank,
                                             opts->basis_cols_out, s));
        }
        if (sigma_out)  // singular values of the slices kept on the randomized path
            TP_LAUNCH(tp::K_RSVD_CHECK, s, tp::launch_sigma_top(W.jsig, L, W.lact, nullptr, fb, h, sigma_out, s));
        // W = Q (T Q2^*)
        Dyn dmk;
        dmk.gate = gate;
        dmk.m = width;
        dmk.k = width;
        st = gemm(W.T, L, sl, tp::OP_N, W.za, L, sz, tp::OP_C, W.m1, n2, (long long)L * n2, L, n2, L, h, rl, s,
                  nullptr, 0, dmk);
        if (st == TP_OK)
            st = gemm(W.ya, L, sy, tp::OP_N, W.m1, n2, (long long)L * n2, tp::OP_N, W.wbar, n2, mn, n1, n2, L, h, rl,
                      s, nullptr, 0, dk);
        return st;
    };

    int st = attempt(0, ctl + C_G1, ctl + C_L1);
    if (st != TP_OK) return st;
    // host-driven form: the number of fallback slices once the host knows it
    // (-1: not read); the fallback flags are final when no retry runs
    int host_nfb = -1;
    if (opts->retry_wide) {
        // slices whose count check failed below the widest sketch: one retry
        // with kpred = max_rank - oversample (the whole call is recomputed
        // at the retry's width)
        // (host-driven, with the test already taken on the host and no retry:
        // both would only write the zero gates the call started with)
        if (!(host && early.valid && !early.retry)) {
            TP_LAUNCH(tp::K_PREDICT, s,
                      tp::launch_retry(fb, W.prefb, W.kpred, W.lact, h, p, opts->oversample, L, ctl + C_G1,
                                       ctl + C_RETRY, s));
            TP_LAUNCH(tp::K_PREDICT, s,
                      tp::launch_width(W.kpred, W.lact, W.prefb, fb, h, p, opts->oversample, L, ctl + C_RETRY,
                                       ctl + C_L2, ctl + C_G2, false, s));
        }
        bool retry = true;
        if (host) {
            // a closed retry changes nothing: its gated launches exit, and the
            // basis and singular values it stores are the first attempt's,
            // stored again (its gate is the retry test's result: a retried
            // slice has a nonzero width)
            if (early.valid) {
                retry = early.retry;
                if (!retry) host_nfb = early.nfb;
            } else {
                hv.resize(1 + h);
                if (read_device_ints({{ctl + C_G2, 1}, {fb, h}}, hv.data(), s) != hipSuccess) return TP_ERR_HIP;
                retry = hv[0] != 0;
                if (!retry) host_nfb = count_fb(hv.data() + 1);
            }
        }
        if (retry) {
            st = attempt(1, ctl + C_G2, ctl + C_L2);
            if (st != TP_OK) return st;
        }
    }
    if (host && host_nfb < 0) {
        hv.resize(h);
        if (read_device_ints({{fb, h}}, hv.data(), s) != hipSuccess) return TP_ERR_HIP;
        host_nfb = count_fb(hv.data());
    }
    // fallback slices: the full SVD on a compact batch whose size is known
    // on the device only (every launch reads it; nothing runs for none)
    const int* nfb = ctl + C_NFB;
    if (host_nfb != 0) {  // (none: the count stays 0 and every launch below would exit)
        TP_LAUNCH(tp::K_GATHER, s, tp::launch_compact(fb, h, W.idx, ctl + C_NFB, s));
        TP_LAUNCH(tp::K_GATHER, s,
                  tp::launch_gather(ybar.re, ybar.im, W.cy.re, W.cy.im, W.idx, h, mn, false, s, nfb));
        SvtLayout F = W.full;
        st = run_svt(F, W.cy, n1, n2, h, 0, 0, (double)tau, W.cinfo, W.crank, s, nfb);
        if (st != TP_OK) return st;
        TP_LAUNCH(tp::K_GATHER, s,
                  tp::launch_gather(W.cy.re, W.cy.im, W.wbar.re, W.wbar.im, W.idx, h, mn, true, s, nfb));
        if (sigma_out)
            TP_LAUNCH(tp::K_GATHER, s,
                      tp::launch_sigma_top(F.sigma, p, nullptr, W.idx, nullptr, h, sigma_out, s, nfb));
    }
    TP_LAUNCH(tp::K_GATHER, s, tp::launch_fb_results(W.idx, nfb, W.crank, W.cinfo, fb, rk, info, h, s));
    TP_LAUNCH(tp::K_IRFFT, s, tp::launch_irfft(W.wbar.re, W.wbar.im, X, mn, n3, s));
    return TP_OK;
}

size_t tp_slice_features_workspace_size(int n1, int n2, int n3)
{
    if (bad_dim(n1) || bad_dim(n2) || bad_dim(n3)) return 0;
    const size_t h = (size_t)tp::half_slices(n3);
    return 2 * tp::align_up(h * n1 * n2 * sizeof(float)) + tp::features_part_bytes(n1, n2, (int)h);
}

int tp_slice_features(const float* Y, int n1, int n2, int n3, float tau, const int* prev_rank, const float* prev_sigma,
                      float* feats, void* workspace, size_t workspace_bytes, void* stream)
{
    if (!Y || !feats) return TP_ERR_ARG;
    if (!(tau >= 0.0f) || std::isinf(tau)) return TP_ERR_ARG;
    if (bad_dim(n1) || bad_dim(n2) || bad_dim(n3) || n3 > kMaxN3 || bad_slice(n1, n2)) return TP_ERR_SHAPE;
    const size_t h = (size_t)tp::half_slices(n3);
    tp::Arena ar(workspace, workspace_bytes);
    float* re = ar.take<float>(h * n1 * n2);
    float* im = ar.take<float>(h * n1 * n2);
    double* part = reinterpret_cast<double*>(ar.take<char>(tp::features_part_bytes(n1, n2, (int)h)));
    if (!ar.ok) return TP_ERR_WORKSPACE;
    hipStream_t s = as_stream(stream);
    TP_LAUNCH(tp::K_RFFT, s, tp::launch_rfft(Y, re, im, (long long)n1 * n2, n3, s));
    TP_LAUNCH(tp::K_FEATURES, s,
              tp::launch_features(re, im, n1, n2, n3, (int)h, (double)tau, prev_rank, prev_sigma, feats, part, nullptr,
                                  s));
    return TP_OK;
}

int tp_mlp_param_count(void) { return tp::mlp_param_count(); }

int tp_mlp_forward(const float* params, const float* x, float* y, int batch, void* stream)
{
    if (!params || !x || !y || batch < 0) return TP_ERR_ARG;
    if (batch == 0) return TP_OK;
    hipStream_t s = as_stream(stream);
    TP_LAUNCH(tp::K_MLP, s, tp::launch_mlp_forward(params, x, y, batch, s));
    return TP_OK;
}

size_t tp_mlp_train_workspace_size(int batch) { return batch > 0 ? tp::mlp_train_bytes(batch) : 0; }

int tp_mlp_loss_grad(const float* params, const float* x, const float* t, int batch, float under, float* grad,
                     float* loss, void* workspace, size_t workspace_bytes, void* stream)
{
    if (!params || !x || !t || !grad || !loss || batch <= 0 || !(under > 0.0f)) return TP_ERR_ARG;
    if (!workspace || workspace_bytes < tp::mlp_train_bytes(batch)) return TP_ERR_WORKSPACE;
    hipStream_t s = as_stream(stream);
    TP_LAUNCH(tp::K_MLP, s, tp::launch_mlp_loss_grad(params, x, t, batch, under, grad, loss, workspace, s));
    return TP_OK;
}

int tp_mlp_adam(float* params, const float* grad, float* m, float* v, int step, float lr, float beta1, float beta2,
                float eps, void* stream)
{
    if (!params || !grad || !m || !v || step < 1 || !(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) ||
        !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
        return TP_ERR_ARG;
    hipStream_t s = as_stream(stream);
    TP_LAUNCH(tp::K_MLP, s, tp::launch_adam(params, grad, m, v, tp::mlp_param_count(), step, lr, beta1, beta2, eps, s));
    return TP_OK;
}

}  // extern "C"
