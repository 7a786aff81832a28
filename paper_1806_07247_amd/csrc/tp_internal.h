// Internal declarations of the gfx950 t-product library (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "tp.h"

namespace tp {

constexpr size_t kAlign = 256;

__host__ __device__ inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// number of Fourier slices that get a dense operation: ceil((n3+1)/2) = floor(n3/2)+1
inline int half_slices(int n3) { return n3 / 2 + 1; }

// Linear carve-out of the caller's workspace.
struct Arena {
    char* base;
    size_t cap;
    size_t used = 0;
    bool ok = true;
    Arena(void* p, size_t n) : base(static_cast<char*>(p)), cap(n) {}
    template <class T>
    T* take(size_t count) {
        size_t bytes = align_up(count * sizeof(T));
        if (used + bytes > cap || (base == nullptr && bytes)) {
            ok = false;
            used += bytes;
            return nullptr;
        }
        T* p = reinterpret_cast<T*>(base + used);
        used += bytes;
        return p;
    }
};

// Planar complex slice stack: re and im planes, each nslices x rows x cols.
struct Planes {
    float* re;
    float* im;
};

// ---------------------------------------------------------------- FFT ----
// Forward real DFT of every tube of the tube-major tensor x (ntubes x n3) into
// the first floor(n3/2)+1 slices of planar (re, im), slice-major: element k of
// tube q lands at re[k*ntubes + q].
// Batched transforms: 64 tubes of one tensor per unit (kBatchMaxN3 >= n3).
// Forward: src (tube-major) -> re/im (slice-major planes of that tensor);
// inverse: re/im -> dst.
constexpr int kBatchMaxN3 = 128;
struct FftUnit {
    const float* src;
    float* re;
    float* im;
    float* dst;
    long long ntubes;  // tubes of the tensor (n1 * n2)
    long long base;    // first tube of the unit
    int n3;
    int nt;            // tubes in the unit (<= 64)
};
// max_n3: the largest n3 among the units (sizes the LDS tile)
hipError_t launch_fft_batch(const FftUnit* units, int nunits, int inverse, int max_n3, int grid, hipStream_t s);
hipError_t launch_rfft(const float* x, float* re, float* im, long long ntubes, int n3, hipStream_t s);
// Inverse of the above: x = (1/n3) sum over the full conjugate-symmetric
// spectrum; the imaginary parts of slice 0 (and n3/2 for even n3) are ignored.
hipError_t launch_irfft(const float* re, const float* im, float* x, long long ntubes, int n3, hipStream_t s);

// Order-p tensors (p = 2 + nd; dims[0 .. nd-1] = n3 .. np, host array): the
// DFT over modes 3..p of every frontal element.  x is C-ordered
// (mrow = n1*n2 frontal elements, then modes 3..p, np fastest).  The output
// dst holds h = n3 ... n_(p-1) * (floor(np/2)+1) slices of mrow elements,
// slice s = kp * (n3 ... n_(p-1)) + (k3, ..., k_(p-1)) (row-major), kp the
// bin of the last mode (the others' conjugates implicit, as for p = 3).
// tmp is scratch planes of the same size.  nd = 1 is launch_rfft.
hipError_t launch_rfft_nd(const float* x, long long mrow, int nd, const int* dims, Planes dst, Planes tmp,
                          hipStream_t s);
// Inverse of launch_rfft_nd; src and tmp are both overwritten.
hipError_t launch_irfft_nd(Planes src, Planes tmp, float* x, long long mrow, int nd, const int* dims, hipStream_t s);

// Forward transform written as bf16 planes for the bf16 slice products.
// Per bin k the planes hold an outer x ld matrix (element (o, i) is bin k of
// tube q = o*q_outer + i*q_inner of x for i < inner, and 0 for
// inner <= i < ld), stored k-blocked: blocks of bkl consecutive i, each
// block an outer x bkl row-major panel, at k*slice + (i / bkl)*outer*bkl +
// o*bkl + i % bkl (ld a multiple of bkl).  A run of rows of one block is
// then contiguous.  Planes, plane elements apart: hi re, hi im, and with
// split lo re, lo im, where hi = bf16(v) and lo = bf16(v - hi) (round to
// nearest even).
struct SplitOut {
    unsigned short* p;
    long long plane, slice;
    int outer, inner, ld, bkl;
    long long q_outer, q_inner;
    int split;
};
hipError_t launch_rfft_split(const float* x, const SplitOut& o, int n3, hipStream_t s);

// ---------------------------------------------------------- slice GEMM ----
enum Op { OP_N = 0, OP_C = 1 };  // op(X) = X or X^* (conjugate transpose)

struct CgemmArgs {
    const float* ar;
    const float* ai;
    long long lda, sa;  // row stride, slice stride (elements)
    const float* br;
    const float* bi;
    long long ldb, sb;
    float* cr;
    float* ci;
    long long ldc, sc;
    int m, n, k;         // op(A) is m x k, op(B) is k x n
    int nslices;
    int real_first;      // slice 0 is real (imaginary planes are zero)
    int real_last;       // slice nslices-1 is real
    const int* kdyn;     // optional per-slice inner dimension (<= k), device
    int ksplit;          // > 1: the inner dimension is cut in ksplit parts (FP32 only) whose
    float* part;         // products go to part (re: [ksplit][nslices][m][n], then im) and are summed
    // Device-side values for launches sized on the host for their largest
    // shape (all optional): gate 0 makes the launch do nothing; dyn_k caps k;
    // dyn_m, dyn_n are the rows and columns computed (m and n keep the layout
    // of the output and split parts; outputs past them are undefined: left
    // alone or written with zeros); dyn_ns is the count of live slices (the
    // others are left alone).
    const int* gate;
    const int* dyn_m;
    const int* dyn_n;
    const int* dyn_k;
    const int* dyn_ns;
};
// bytes of the split-K partial buffer of a product
size_t splitk_bytes(int ksplit, int nslices, int m, int n);

// Batched slice products of uneven shapes (FP32): one unit per output tile.
enum { GEMM_NN = 0, GEMM_CN = 1, GEMM_NC = 2 };
struct GemmUnit {
    int item;   // index into the CgemmArgs table
    int slice;
    int m0, n0; // tile origin
    int op;     // GEMM_NN, GEMM_CN (op(A) = A^*), GEMM_NC (op(B) = B^*)
};
// tile: 0 = 32 x 32, 1 = 64 x 64 outputs per workgroup; batch_tile gives the edge
int batch_tile(int tile);
hipError_t launch_cgemm_batch(const CgemmArgs* items, const GemmUnit* units, int nunits, int tile, int grid,
                              double flops, double bytes, hipStream_t s);
// FP32 slice products (prec must be TP_PREC_FP32; the bf16 products take
// their operands as bf16 planes, launch_cgemm_bf16)
hipError_t launch_cgemm(const CgemmArgs& a, int opa, int opb, int prec, hipStream_t s);

// C^(s) = A^(s) B^(s) on bf16 planes (see SplitOut): A as m rows of the
// inner index (outer = m), B as n columns of it (outer = n), both k-blocked
// with the block length bf16_plan gives for the product, zero past k.
// Planes hi re, hi im, then (split) lo re, lo im; strides in elements.
// Slices cs0 .. cs0+ncs-1 are complex; real_s[0 .. nreal-1] are real
// (imaginary planes ignored, Ci written as 0).  Output planar FP32 as
// CgemmArgs.
struct Bf16Args {
    const unsigned short* a;
    const unsigned short* b;
    long long a_plane, a_slice, b_plane, b_slice;
    int ld;       // k rounded up to the block length
    int bkl;      // block length of the planes (from bf16_plan)
    int variant;  // tile (from bf16_plan)
    float* cr;
    float* ci;
    long long ldc, sc;
    int m, n, k;
    int cs0, ncs;
    int nreal;
    int real_s[2];
    int split;  // 1: hi*hi + hi*lo + lo*hi, 0: hi*hi
    int rpw;    // real-slice tiles per workgroup (set by the launcher)
};
// tile variant of a bf16 product and the plane block length it reads
int bf16_plan(int m, int n, int k, int ncs, int nreal, int* bkl);
hipError_t launch_cgemm_bf16(Bf16Args a, hipStream_t s);
// FP32 narrow-output products split along k (ksplit > 1, part given): the
// parts only, left in a.part ([ksplit][nslices][m][n], re then im) for the
// caller to sum (launch_reduce_gram); cgemm_parts_ok says whether a product
// qualifies
bool cgemm_parts_ok(const CgemmArgs& a, int opa, int opb);
hipError_t launch_cgemm_parts(const CgemmArgs& a, int opa, int opb, hipStream_t s);

// -------------------------------------------------------------- Jacobi ----
struct JacobiArgs {
    const float* yr;  // input slices (planar, row-major m x n per slice)
    const float* yi;
    float* wr;        // output: rotated columns, row-major rows x p per slice
    float* wi;
    double* sigma;    // p per slice (unsorted norms of the rotated columns)
    int* info;        // per slice: sweeps used, negated when the cap was hit (may be null)
    int m, n;         // slice shape
    int nslices;
    int max_sweeps;
    int transpose;    // work on Y^* (used when m < n)
    double tol;       // rotate a pair when |x^* y| > tol ||x|| ||y||
    float2* cols;     // optional: rotated columns, column-major R x P per slice
    float2* qout;     // optional: accumulated rotations V, column-major P x P per slice
    int whole;        // 1: one workgroup per slice whenever the slice fits in LDS
    const int* count; // optional device count of live slices (<= nslices); the rest are skipped
    const int* gate;  // optional device flag: 0 makes the call do nothing
    const int* pdyn;  // optional device cap on the columns swept (one workgroup per slice only; the
                      // layout keeps n, the columns beyond are left as they are).  The rows from
                      // *pdyn on must be zero: the rotations touch the first *pdyn rows only
};
// Batched per-slice SVDs (whole slice in LDS, R = max(m, n) <= 128) and
// shrinkage over (item, slice) units.
struct SliceUnit {
    int item;
    int slice;
};
struct ShrinkItem {
    const double* sigma;  // h x P
    float* wr;            // h x R x P rotated columns (planar)
    float* wi;
    int R, P, h;
    int rel;              // 1: tau = tau_rel * max sigma of the item
    double tau;           // absolute tau, or tau_rel
    int* keep;            // optional: #{sigma_j > tau} per slice
    float* tau_out;       // optional: the tau used
};
size_t jacobi_batch_lds(int max_r, int max_p);
hipError_t launch_jacobi_batch(const JacobiArgs* items, const SliceUnit* units, int nunits, int max_r, int max_p,
                               int grid, hipStream_t st);
hipError_t launch_shrink_batch(const ShrinkItem* items, const SliceUnit* units, int nunits, int grid, hipStream_t st);
// Definition 2.2 (conjugate transpose of a real tensor) and 2.3 (identity)
hipError_t launch_tran(const float* a, float* out, int n1, int n2, int n3, hipStream_t s);
hipError_t launch_teye(float* out, int n, int n3, hipStream_t s);
// tsn (Definition 2.8): the largest singular value over the slices
hipError_t launch_tsn_reduce(const double* sigma, int nslices, int P, double* out, hipStream_t st);
// tubal rank (Definition 2.7) from the unsorted singular values of the h
// leading slices: sorted (h x P scratch) then counted against tol
hipError_t launch_tubal_rank(const double* sigma, double* sorted, int nslices, int P, int n3, double tol,
                             double tol_scale, int* out, hipStream_t st);
hipError_t launch_jacobi(const JacobiArgs& a, void* scratch, size_t scratch_bytes, hipStream_t s);
size_t jacobi_scratch_bytes(int m, int n, int nslices, bool withv);
// Jacobi convergence threshold for an R-row work matrix of FP32 data
inline double jacobi_tol(int rows) { return __builtin_sqrt((double)(rows > 4 ? rows : 4)) * 0x1p-23; }

// t-SVD outputs from the Jacobi results: sorted bases L (R x R, completed), Q (P x P), diagonal S (m x n)
hipError_t launch_tsvd_finish(const float2* cols, const double* sigma, const float2* q, Planes L, Planes Q, Planes S,
                              int R, int P, int m, int n, int nslices, hipStream_t s);

// columns w_j of each slice scaled by sqrt((1 - tau/sigma_j)_+) / sigma_j; keep = #{sigma_j > tau}
hipError_t launch_shrink(float* wr, float* wi, const double* sigma, int* keep, int R, int P, int nslices, double tau,
                         hipStream_t s, const int* count = nullptr);
// (1/n3) sum over all n3 slices of the singular values, from the half spectrum
// (1/(n3*period)) sum of sigma over the slices, weighted 1 for self-conjugate
// last-mode bins (slice / period = 0 or n3/2) and 2 for the others
hipError_t launch_tnn_reduce(const double* sigma, int nslices, int P, int n3, double* out, hipStream_t s,
                             int period = 1);

// ------------------------------------------------------------- learned ----
constexpr int kMaxL = 64;  // widest randomized sketch (l_max)
int mlp_param_count();
// A previous call's range basis (planar n x ld per slice, cols[s] valid columns)
struct WarmBasis {
    const float* re;  // null: no warm start
    const float* im;
    int ld;
    const int* cols;
};
// Sketch Om (n x L per slice): the warm columns where given, else Gaussian
hipError_t launch_sketch(float* omr, float* omi, int n, int L, const int* lact, int nslices, int n3,
                         unsigned long long seed, WarmBasis warm, hipStream_t s, const int* gate = nullptr);
hipError_t launch_store_basis(const float* zr, const float* zi, int n, int L, const int* lact, const int* fb,
                              int nslices, float* outr, float* outi, int ld, int* cols, hipStream_t st,
                              const int* gate = nullptr);
size_t cholqr_part_bytes(int m, int L, int nslices);
// one CholeskyQR pass on Y (m x L per slice): Gram in FP64, Cholesky, Rinv (FP32 planar);
// rtot/rhr/rhi optional (accumulated R and, after pass 1, R^* restricted to the active block)
// gram_ready: the Gram partials of Y are already in part (launch_reduce_gram)
hipError_t launch_cholqr_pass(const float* yr, const float* yi, int m, int L, const int* lact, int nslices, int pass,
                              double2* part, float* rir, float* rii, double2* rtot, float* rhr, float* rhi,
                              int* status, hipStream_t s, bool gram_ready = false, const int* gate = nullptr);
// the split parts of a narrow product summed in the fixed order kp = 0, 1, ...
// into Y = (yr, yi) (m x L per slice, row-major, slice stride m L; imaginary
// plane zero on the real slices), and the FP64 Gram partials of Y that
// launch_cholqr_pass would form, in its layout (part)
hipError_t launch_reduce_gram(const float* parts, int ksplit, int m, int L, int nslices, int real_first, int real_last,
                              float* yr, float* yi, const int* lact, double2* part, hipStream_t s,
                              const int* gate = nullptr, const int* width = nullptr);
// status: per-slice CholeskyQR breakdown flags (or null), OR-ed into fallback;
// vp / cp (optional): V_r and C_r also written planar row-major
hipError_t launch_rsvd_check(const float2* cols, const double* sigma, const float2* vr, const int* kpred,
                             const int* lact, const int* prefb, const int* status, int L, double tau, Planes T,
                             int* fallback, int* rank, int nslices, hipStream_t s, const int* gate = nullptr,
                             Planes vp = Planes{}, Planes cp = Planes{});
hipError_t launch_cm_to_planar(const float2* src, Planes dst, int L, int nslices, hipStream_t s,
                               const int* gate = nullptr, const float2* src2 = nullptr, Planes dst2 = Planes{});
// part: accuracy_part_bytes(nslices) of workspace for the per-band partial sums
size_t accuracy_part_bytes(int nslices);
hipError_t launch_accuracy(Planes t1, Planes t2, const double* sigma, const int* lact, const double* fro2, int m,
                           int L, double tau, double delta, int* bad, int nslices, double* part, hipStream_t st,
                           const int* gate = nullptr);
// per-slice features; part: features_part_bytes(m, n, nslices) of scratch
size_t features_part_bytes(int m, int n, int nslices);
hipError_t launch_features(const float* yr, const float* yi, int m, int n, int n3, int nslices, double tau,
                           const int* prev, const float* prev_sigma, float* feats, double* part, double* fro2,
                           hipStream_t st);
hipError_t launch_sigma_top(const double* sig, int P, const int* lact, const int* map, const int* skip, int rows,
                            float* out, hipStream_t s, const int* count = nullptr);
hipError_t launch_predict(const float* params, const float* feats, int nslices, int p, int fixed_rank, int oversample,
                          int L, int* kpred, int* lact, int* fallback, int* rank, hipStream_t s);
hipError_t launch_mlp_forward(const float* params, const float* x, float* y, int batch, hipStream_t s);
size_t mlp_train_bytes(int batch);
hipError_t launch_mlp_loss_grad(const float* params, const float* x, const float* t, int batch, float under,
                                float* grad, float* loss, void* ws, hipStream_t s);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int count, int step, float lr, float b1, float b2,
                       float eps, hipStream_t s);
hipError_t launch_gather(const float* sr, const float* si, float* dr, float* di, const int* idx, int cnt, long long per,
                         bool scatter, hipStream_t s, const int* count = nullptr);
// device-side control of the learned prox (single-workgroup kernels; see learned.hip)
hipError_t launch_width(int* kpred, int* lact, const int* prefb, int* fb, int nslices, int p, int oversample,
                        int max_rank, const int* gate_in, int* ctl_L, int* ctl_gate, bool set_fb, hipStream_t s);
hipError_t launch_retry(const int* fb, const int* prefb, int* kpred, int* lact, int nslices, int p, int oversample,
                        int max_rank, const int* gate_in, int* ctl_retry, hipStream_t s);
hipError_t launch_round(int* bad, int* fb, int nslices, const int* cur, int* next, bool last, hipStream_t s);
// the a posteriori check of a round (when *cur) and the round's end (k_round) in two launches
hipError_t launch_accuracy_round(Planes t1, Planes t2, const double* sigma, const int* lact, const double* fro2, int m,
                                 int L, double tau, double delta, int* bad, int nslices, double* part, int* fb,
                                 const int* cur, int* next, bool last, hipStream_t s);
hipError_t launch_compact(const int* fb, int nslices, int* idx, int* count, hipStream_t s);
hipError_t launch_fb_results(const int* idx, const int* count, const int* crank, const int* cinfo, const int* fb,
                             int* rank, int* info, int nslices, hipStream_t s);
hipError_t launch_copy_planes(const float* sr, const float* si, float* dr, float* di, long long n, const int* gate,
                              hipStream_t s);
hipError_t launch_fill_int(int* p, long long n, int v, hipStream_t s);

// tp_tprod after its argument checks (check_tprod), on a caller-given workspace
int check_tprod(const float* A, const float* B, const float* C, int n1, int n2, int l, int n3, int prec);
int run_tprod(const float* A, const float* B, float* C, int n1, int n2, int l, int n3, int prec, void* workspace,
              size_t workspace_bytes, hipStream_t s);

// ------------------------------------------------------------ tunables ----
// current value of a TP_PARAM_* setting (tp_set_param), default if unset
int param(int key);

// per-slice inverse (Gauss-Jordan) and QR (Householder) of the tensor
// inverse and T-QR: one workgroup per slice, planar complex slices
hipError_t launch_slice_inv(const float* ar, const float* ai, float* wr, float* wi, float* br, float* bi, int n,
                            int nslices, int* info, hipStream_t st);
hipError_t launch_slice_qr(const float* ar, const float* ai, float* wr, float* wi, float* vr, float* vi,
                           double* beta, float* qr, float* qi, float* rr, float* ri, int m, int n, int nslices,
                           hipStream_t st);

// ------------------------------------------------------------- tracing ----
enum KernelId {
    K_RFFT = 0, K_IRFFT = 1, K_CGEMM = 2, K_JACOBI = 3, K_SHRINK = 4, K_TNN_REDUCE = 5, K_TSVD_FINISH = 6,
    K_FEATURES = 7, K_PREDICT = 8, K_SKETCH = 9, K_CHOLQR = 10, K_RSVD_CHECK = 11, K_GATHER = 12, K_MLP = 13,
    K_ACCURACY = 14, K_TENSOR_OP = 15, K_TRPCA = 16
};

// Records HIP events around the launches in its scope while tracing is on,
// with the algorithmic work the launchers in the scope report.
class TraceScope {
   public:
    TraceScope(hipStream_t s, int id);
    ~TraceScope();

   private:
    hipStream_t stream_;
    int id_;
    void* start_;
};

// Called by a launcher: adds the algorithmic flops and HBM bytes of the
// kernel it enqueues to the enclosing TraceScope (ignored when not tracing).
void trace_work(double flops, double bytes);
// A slice product whose gate or live sizes are device values: its work is
// evaluated when the trace is collected, from the values then in device
// memory (collect after each call for exact figures).
void trace_gemm_dyn(const int* gate, const int* m, const int* n, const int* k, int hm, int hn, int hk, int nslices,
                    int nreal);

}  // namespace tp

// enqueue one stage: trace it, and turn a launch failure into TP_ERR_HIP
#define TP_LAUNCH(id, stream, expr)                   \
    do {                                              \
        hipError_t _e;                                \
        {                                             \
            tp::TraceScope _ts((stream), (id));       \
            _e = (expr);                              \
        }                                             \
        if (_e != hipSuccess) return TP_ERR_HIP;      \
    } while (0)

#define TP_TRY(expr)                                  \
    do {                                              \
        hipError_t _e = (expr);                       \
        if (_e != hipSuccess) return TP_ERR_HIP;      \
    } while (0)
