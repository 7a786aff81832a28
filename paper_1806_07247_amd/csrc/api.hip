// C-ABI entry points of libtp.so: argument checks, workspace carving and the
// kernel sequence of each operation.  See include/tp.h for the contract.
#include <cmath>

#include "tp_internal.h"

namespace {

constexpr int kMaxN3 = 1024;

bool bad_dim(int v) { return v <= 0; }

bool bad_slice(long long a, long long b) { return a * b >= (1LL << 31); }

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Workspace of tprod: half spectra of A, B and C (planar complex).
struct TprodLayout {
    tp::Planes a, b, c;
};

tp::Arena tprod_arena(void* ws, size_t bytes, int n1, int n2, int l, int n3, TprodLayout* L)
{
    const size_t h = (size_t)tp::half_slices(n3);
    tp::Arena ar(ws, bytes);
    TprodLayout t;
    t.a.re = ar.take<float>(h * n1 * n2);
    t.a.im = ar.take<float>(h * n1 * n2);
    t.b.re = ar.take<float>(h * n2 * l);
    t.b.im = ar.take<float>(h * n2 * l);
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
};

tp::Arena svt_arena(void* ws, size_t bytes, int n1, int n2, int n3, bool recon, SvtLayout* L)
{
    const size_t h = (size_t)tp::half_slices(n3);
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
    t.jscratch = t.jscratch_bytes ? ar.take<char>(t.jscratch_bytes) : nullptr;
    if (L) *L = t;
    return ar;
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

}  // namespace

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
    (void)prec;
    if (bad_dim(n1) || bad_dim(n2) || bad_dim(l) || bad_dim(n3)) return 0;
    return tprod_arena(nullptr, 0, n1, n2, l, n3, nullptr).used;
}

int tp_tprod(const float* A, const float* B, float* C, int n1, int n2, int l, int n3, int prec,
             void* workspace, size_t workspace_bytes, void* stream)
{
    if (!A || !B || !C) return TP_ERR_ARG;
    if (prec != TP_PREC_FP32 && prec != TP_PREC_BF16X3 && prec != TP_PREC_BF16) return TP_ERR_ARG;
    if (bad_dim(n1) || bad_dim(n2) || bad_dim(l) || bad_dim(n3) || n3 > kMaxN3) return TP_ERR_SHAPE;
    if (bad_slice(n1, n2) || bad_slice(n2, l) || bad_slice(n1, l)) return TP_ERR_SHAPE;
    TprodLayout L;
    tp::Arena ar = tprod_arena(workspace, workspace_bytes, n1, n2, l, n3, &L);
    if (!ar.ok) return TP_ERR_WORKSPACE;
    hipStream_t s = as_stream(stream);
    const int h = tp::half_slices(n3);

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
    const bool tr = n1 < n2;           // work on Ybar^* when the slices are wide
    const int R = tr ? n2 : n1, P = tr ? n1 : n2, p = P;
    const long long mn = (long long)n1 * n2;

    // Algorithm 3, step 1
    TP_LAUNCH(tp::K_RFFT, s, tp::launch_rfft(Y, L.ybar.re, L.ybar.im, mn, n3, s));
    // step 2: SVD of each leading slice ...
    tp::JacobiArgs j{};
    j.yr = L.ybar.re;
    j.yi = L.ybar.im;
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
    TP_LAUNCH(tp::K_JACOBI, s, tp::launch_jacobi(j, L.jscratch, L.jscratch_bytes, s));
    // ... shrinkage (eq (21)): scaled columns sqrt(d_j)/sigma_j w_j
    TP_LAUNCH(tp::K_SHRINK, s, tp::launch_shrink(L.w.re, L.w.im, L.sigma, rank ? rank : L.keep, R, P, h, (double)tau, s));
    // ... and W = U (S - tau)_+ V^* as two slice products
    tp::CgemmArgs g{};
    g.nslices = h;
    g.real_first = 1;
    g.real_last = (n3 % 2 == 0) ? 1 : 0;
    if (!tr) {
        // T = What^* Ybar (n x n), then W = What T (m x n)
        g.ar = L.w.re; g.ai = L.w.im; g.lda = n2; g.sa = mn;
        g.br = L.ybar.re; g.bi = L.ybar.im; g.ldb = n2; g.sb = mn;
        g.cr = L.t.re; g.ci = L.t.im; g.ldc = p; g.sc = (long long)p * p;
        g.m = n2; g.n = n2; g.k = n1;
        TP_LAUNCH(tp::K_CGEMM, s, tp::launch_cgemm(g, tp::OP_C, tp::OP_N, TP_PREC_FP32, s));
        g.ar = L.w.re; g.ai = L.w.im; g.lda = n2; g.sa = mn;
        g.br = L.t.re; g.bi = L.t.im; g.ldb = p; g.sb = (long long)p * p;
        g.cr = L.ybar.re; g.ci = L.ybar.im; g.ldc = n2; g.sc = mn;
        g.m = n1; g.n = n2; g.k = n2;
        TP_LAUNCH(tp::K_CGEMM, s, tp::launch_cgemm(g, tp::OP_N, tp::OP_N, TP_PREC_FP32, s));
    } else {
        // T = Ybar Bhat (m x m), then W = T Bhat^* (m x n); Bhat is n x m
        g.ar = L.ybar.re; g.ai = L.ybar.im; g.lda = n2; g.sa = mn;
        g.br = L.w.re; g.bi = L.w.im; g.ldb = n1; g.sb = mn;
        g.cr = L.t.re; g.ci = L.t.im; g.ldc = p; g.sc = (long long)p * p;
        g.m = n1; g.n = n1; g.k = n2;
        TP_LAUNCH(tp::K_CGEMM, s, tp::launch_cgemm(g, tp::OP_N, tp::OP_N, TP_PREC_FP32, s));
        g.ar = L.t.re; g.ai = L.t.im; g.lda = p; g.sa = (long long)p * p;
        g.br = L.w.re; g.bi = L.w.im; g.ldb = n1; g.sb = mn;
        g.cr = L.ybar.re; g.ci = L.ybar.im; g.ldc = n2; g.sc = mn;
        g.m = n1; g.n = n2; g.k = n1;
        TP_LAUNCH(tp::K_CGEMM, s, tp::launch_cgemm(g, tp::OP_N, tp::OP_C, TP_PREC_FP32, s));
    }
    // step 3: inverse DFT (conjugate fill implicit)
    TP_LAUNCH(tp::K_IRFFT, s, tp::launch_irfft(L.ybar.re, L.ybar.im, X, mn, n3, s));
    (void)R;
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

}  // extern "C"
