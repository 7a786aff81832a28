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
    TP_TRY(tp::launch_rfft(A, L.a.re, L.a.im, (long long)n1 * n2, n3, s));
    TP_TRY(tp::launch_rfft(B, L.b.re, L.b.im, (long long)n2 * l, n3, s));
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
    TP_TRY(tp::launch_cgemm(g, tp::OP_N, tp::OP_N, prec, s));
    // step 3: inverse DFT (conjugate fill implicit)
    TP_TRY(tp::launch_irfft(L.c.re, L.c.im, C, (long long)n1 * l, n3, s));
    return TP_OK;
}

}  // extern "C"
