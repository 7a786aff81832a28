/*
 * tp.h -- C ABI of the gfx950 (MI355X) t-product library libtp.so.
 *
 * The library computes the Fourier-domain slice pipeline of the t-product
 * toolbox (C. Lu, "Tensor-Tensor Product Toolbox", 2018): a real DFT along
 * every mode-3 tube, one dense operation on each of the ceil((n3+1)/2)
 * leading Fourier slices, and the inverse DFT.
 *
 * Conventions shared by every entry point
 *   Tensors   An n1 x n2 x n3 real tensor is FP32, row-major with the tube
 *             index last: A(i,j,t) is A[(i*n2 + j)*n3 + t] (0-based; the paper
 *             indexes from 1).  This is the layout of a contiguous
 *             (n1, n2, n3) array.
 *   Memory    Every tensor, output and workspace pointer is device memory of
 *             the current HIP device, owned by the caller; inputs are not
 *             modified.  Inputs and outputs must not overlap.
 *   Workspace Scratch memory is passed in by the caller: its size comes from
 *             the matching *_workspace_size query and must be at least that
 *             large.  The library allocates no device memory and does not
 *             synchronise; every call only enqueues kernels on `stream`
 *             (a hipStream_t, NULL for the default stream).  Exceptions:
 *             tp_trpca (its stopping test), and tp_prox_tnn_learned when
 *             TP_PARAM_LEARNED_HOST is set (see there).
 *   Errors    Arguments are checked on the host before anything is enqueued;
 *             a negative tp_status is returned and nothing runs.  TP_ERR_HIP
 *             reports a failed kernel launch (hipGetLastError).  Outcomes that
 *             are only known on the device go to an optional per-slice int
 *             array `info` (device memory, floor(n3/2)+1 entries).
 *   Sizes     1 <= n3 <= 1024; n1, n2, l >= 1; element counts < 2^31 per slice.
 */
#ifndef TP_H
#define TP_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum tp_status {
    TP_OK = 0,
    TP_ERR_ARG = -1,         /* null pointer, negative or NaN scalar, bad enum */
    TP_ERR_SHAPE = -2,       /* non-positive or unsupported size */
    TP_ERR_WORKSPACE = -3,   /* workspace missing or smaller than the query */
    TP_ERR_HIP = -4,         /* a kernel launch failed */
    TP_ERR_UNSUPPORTED = -5  /* valid request the library does not handle */
} tp_status;

/* Arithmetic of the slice products (tp_tprod).  All accumulate in FP32.
 *   TP_PREC_FP32    FP32 matrix-core products.
 *   TP_PREC_BF16X3  each FP32 operand split into bf16 hi + lo (both rounded to
 *                   nearest even); hi*hi + hi*lo + lo*hi on bf16 matrix cores.
 *   TP_PREC_BF16    hi*hi only (operands rounded to bf16). */
typedef enum tp_prec { TP_PREC_FP32 = 0, TP_PREC_BF16X3 = 1, TP_PREC_BF16 = 2 } tp_prec;

/* Human-readable name of a tp_status value. */
const char* tp_status_string(int status);

/* Library ABI version (major*100 + minor). */
int tp_version(void);

/*
 * t-product C = A * B (Definition 2.1, eq (9)), computed by Algorithm 1:
 * DFT of every tube of A and B, Cbar^(k) = Abar^(k) Bbar^(k) for the
 * floor(n3/2)+1 leading slices (eq (10)), inverse DFT (the remaining slices
 * are the conjugates, implicit in the real inverse transform).
 *   A  n1 x n2 x n3 (input)       B  n2 x l x n3 (input)
 *   C  n1 x l x n3 (output)       prec  a tp_prec value
 */
size_t tp_tprod_workspace_size(int n1, int n2, int l, int n3, int prec);
int tp_tprod(const float* A, const float* B, float* C, int n1, int n2, int l, int n3, int prec,
             void* workspace, size_t workspace_bytes, void* stream);

/*
 * tp_tprod without a caller-given workspace, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  The same computation and kernels as
 * tp_tprod (bitwise equal results); the half spectra live in a device array
 * of the library, tp_tprod_noalloc_max_bytes() bytes per GPU, allocated when
 * the library is loaded on a device and held until the process ends.  The
 * call allocates nothing and does not synchronise.
 * Errors as tp_tprod, plus TP_ERR_WORKSPACE (before anything is enqueued)
 * when tp_tprod_workspace_size(n1, n2, l, n3, prec) exceeds that size.
 * Every call on one GPU uses that GPU's one array: calls that overlap on a
 * GPU (concurrent streams, threads) race and must be serialised by the
 * caller; a call fully overwrites what it uses, so no state carries over.
 */
int tp_tprod_noalloc(const float* A, const float* B, float* C, int n1, int n2, int l, int n3, int prec,
                     void* stream);
size_t tp_tprod_noalloc_max_bytes(void);

/*
 * t-SVD A = U * S * V^* (Theorem 2.2), computed by Algorithm 2: DFT of the
 * tubes of A; for each of the floor(n3/2)+1 leading Fourier slices a full
 * SVD by one-sided Jacobi (real rotations on the real DC and, for even n3,
 * middle slices, so that U, S, V come out real), singular values sorted in
 * decreasing order (so eq (13) holds), left/right bases completed to square
 * unitary matrices; inverse DFTs of Ubar, Sbar, Vbar (the trailing slices are
 * the conjugates, implicit in the real inverse transform).
 *   A  n1 x n2 x n3 (input)
 *   U  n1 x n1 x n3, S n1 x n2 x n3 (f-diagonal), V n2 x n2 x n3 (outputs)
 *   info  as for tp_prox_tnn
 * U and V are unique only up to the usual SVD freedoms (phases, rotations
 * inside repeated singular values, the completed bases); S is unique.
 */
size_t tp_tsvd_workspace_size(int n1, int n2, int n3);
int tp_tsvd(const float* A, float* U, float* S, float* V, int n1, int n2, int n3, int* info,
            void* workspace, size_t workspace_bytes, void* stream);

/*
 * Proximal operator of the tensor nuclear norm, X = Prox_tau(Y) (eq (19)),
 * computed by Algorithm 3 (t-SVT, Theorem 2.3): DFT of the tubes of Y; for
 * each of the floor(n3/2)+1 leading Fourier slices a full SVD by one-sided
 * Jacobi and W^(k) = U (S - tau)_+ V^* (formed as U_J D U_J^* Y^(k) with
 * D = diag((1 - tau/sigma_j)_+), which needs no V); inverse DFT.
 *   Y, X   n1 x n2 x n3 (input, output)
 *   tau    >= 0 (tau = 0 returns Y up to rounding); NaN or < 0: TP_ERR_ARG
 *   info   optional device int[floor(n3/2)+1]: the number of Jacobi sweeps
 *          used by each slice (> 0), negated when the sweep cap (30 unless
 *          changed with TP_PARAM_JACOBI_SWEEPS) was
 *          reached without convergence (the result is still written)
 *   rank   optional device int[floor(n3/2)+1]: #{sigma_j > tau} per slice
 */
size_t tp_prox_tnn_workspace_size(int n1, int n2, int n3);
int tp_prox_tnn(const float* Y, float* X, int n1, int n2, int n3, float tau, int* info, int* rank,
                void* workspace, size_t workspace_bytes, void* stream);

/*
 * Tensor spectral norm (Definition 2.8): ||A|| = ||bcirc(A)|| = the largest
 * singular value over the Fourier slices, written as one device double.
 * Workspace and info as tp_tnn.
 */
size_t tp_tsn_workspace_size(int n1, int n2, int n3);
int tp_tsn(const float* A, int n1, int n2, int n3, double* out, int* info, void* workspace, size_t workspace_bytes,
           void* stream);

/*
 * Tensor tubal rank (Definition 2.7): the number of nonzero singular tubes
 * S(i,i,:) of the t-SVD, written as one device int.  In floating point a tube
 * counts when S(i,i,1) > tol, with S(i,i,1) = (1/n3) sum_k sigma_i(Abar^(k))
 * (the first frontal slice of S is the mean of the Fourier-domain S; each
 * slice's singular values taken in decreasing order); tol < 0 selects
 * max(n1, n2) * 2^-23 * S(1,1,1) (FP32 working precision).
 */
size_t tp_tubalrank_workspace_size(int n1, int n2, int n3);
int tp_tubalrank(const float* A, int n1, int n2, int n3, double tol, int* out, int* info, void* workspace,
                 size_t workspace_bytes, void* stream);

/*
 * Conjugate tensor transpose (Definition 2.2) of a real n1 x n2 x n3 tensor:
 * out (n2 x n1 x n3, tube-major, not overlapping A) has frontal slice t equal
 * to the transpose of A's slice (n3 - t) mod n3.  Identity tensor (Definition
 * 2.3): out (n x n x n3) gets I_n in its first frontal slice and zeros
 * elsewhere.  Neither needs a workspace.
 */
int tp_tran(const float* A, float* out, int n1, int n2, int n3, void* stream);
int tp_teye(float* out, int n, int n3, void* stream);

/*
 * Learned-rank prox_tnn: the same operator as tp_prox_tnn (Theorem 2.3), with
 * each leading Fourier slice's SVT computed on a randomized range whose width
 * is predicted per slice.  Per slice k: features of the slice (below) go
 * through the MLP (or fixed_rank is used) to give kpred, the predicted number
 * of singular values above tau; l = min(kpred + oversample, min(n1, n2)).
 * The call's sketch width L is the largest l, rounded up to a multiple of 8
 * (at most max_rank); every slice uses l = min(L, min(n1, n2)) columns and
 * kpred = max(kpred, l - oversample).
 * Y = Ybar^(k) Om with the Gaussian sketch Om (Philox4x32-10 on counter
 * {row, column, slice, 0}, key = seed; Box-Muller; real on the real slices);
 * power_iters times {Z = Ybar^* Q, Y = Ybar Z}, every product re-orthonormalised
 * by CholeskyQR (Gram, Cholesky and inverse in FP64; two passes on every Y,
 * one on the bases that only feed the next product); Bh = Ybar^* Q =
 * Q2 R2 (CholeskyQR2); one-sided Jacobi SVD of R2^* = U_r S V_r^*; and
 * W^(k) = Q U_r (S - tau)_+ V_r^* Q2^*.  A slice falls back to the full SVD
 * path of tp_prox_tnn when l > max_rank, or when the check sigma_(kpred+1) <
 * tau fails on the singular values of R2^* (with retry_wide, a slice failing
 * the check below the widest sketch is first redone once with kpred =
 * max_rank - oversample, and falls back if it fails there).  With accuracy > 0, the kept
 * Ritz triplets (u_j, sigma_j, v_j), sigma_j > tau, are checked a posteriori:
 * when sum_j ||Ybar v_j - sigma_j u_j||^2 > accuracy^2 D on some slice, with
 * D = max(sum_j (sigma_j - tau)^2, ||Ybar^(k)||_F^2) (accuracy_ref = 0: the
 * error relative to the larger of the result and the input, the scale at
 * which FP32 data can resolve a result much smaller than its input) or
 * D = sum_j (sigma_j - tau)^2 (accuracy_ref = 1: relative to the result),
 * all slices get one more power iteration, up to
 * max_power_iters in total (at most 30 beyond power_iters; in a wide retry
 * at most one beyond), and slices still failing then fall back (the extra iteration reuses the projection's basis
 * Q2 as its Z and the check's product Ybar Q2 as its Y, so it forms no new
 * product with Ybar).
 * With l = min(n1,n2) or an exact rank <= l the result equals tp_prox_tnn's
 * up to rounding.
 *   opts       required (see tp_learned_opts); rank, fallback, info optional
 *              device int[floor(n3/2)+1]: the number of singular values
 *              above tau used, 1 for a fallback slice, and the Jacobi sweeps of
 *              the fallback slices (0 for the others).
 * Every decision above that depends on the data (the width L, which slices
 * take the randomized path, whether each accuracy round and the wide retry
 * run, which slices fall back) is taken on the device: the call enqueues a
 * fixed sequence of launches for its arguments, sized for L = max_rank,
 * whose kernels read the width, gates and fallback count from the workspace
 * (a launch whose gate is closed does nothing).  Like the other entry points
 * it allocates nothing and does not synchronise, so a HIP graph may capture
 * it; each possible accuracy round adds about twenty such launches, so
 * max_power_iters - power_iters is best kept small.  With
 * TP_PARAM_LEARNED_HOST = 1 the host instead reads those decisions where
 * they are taken and enqueues only the launches that run (same results; the
 * call then synchronises `stream`, allocates a small pinned host buffer per
 * calling thread on first use, and keeps the device-gated form on a
 * capturing stream).
 * Features (TP_MLP_INPUTS = 12, FP32, per slice; p = min(n1,n2)):
 *   0 log(tau / rms sigma), rms sigma = ||Ybar^(k)||_F / sqrt(p)
 *   1 log(max column norm / tau)
 *   2 prev_rank / p and 3 one when prev_rank is given (else 0, 0)
 *   4 k/(n3/2)    5 one for a real slice    6 log(p)/8    7 log(max(n1,n2)/p)
 *   with prev_sigma (the previous call's leading singular values s_1 >= s_2
 *   >= ... of the slice, TP_SIGMA_KEEP per slice, zero-padded; c of them
 *   nonzero), else zeros:
 *   8 #{s_j > tau}/p   9 #{s_j > tau/1.25}/p   10 log(s_1/tau)
 *   11 one when c > 0 and s_c > tau (the previous sketch saw no value below tau)
 * the logarithms clamped to [-30, 30] (their clamped limits where a norm or tau
 * is 0: feature 0 is 30 for a zero slice).  The MLP maps them to y and
 * kpred = round(expm1(y * log1p(p))) clipped to [0, p].
 * Warm start (optional): basis_out receives this call's right Ritz vectors
 * Q2 V of every slice (the right range basis rotated by the small SVD, so
 * the next sketch starts from the singular basis and its small SVD needs few
 * sweeps), planar complex float[2][floor(n3/2)+1][n2][max_rank]
 * (re plane, then im plane; columns beyond basis_cols_out[k] zero;
 * basis_cols_out[k] = 0 for a fallback slice).  Passed back as warm_basis /
 * warm_cols of the next call (same n1, n2, n3, max_rank), its first
 * warm_cols[k] columns replace the Gaussian columns of slice k's sketch, so a
 * sequence of calls on slowly changing inputs (the prox calls of an ADMM
 * run) continues one subspace iteration instead of restarting it.  The
 * result is checked as without warm start.
 * sigma_out (optional, device float[(floor(n3/2)+1) * TP_SIGMA_KEEP]) receives
 * this call's leading singular values per slice in that layout (from the
 * randomized SVD, or from the full SVD for fallback slices), to be passed as
 * prev_sigma of the next call.
 */
#define TP_MLP_INPUTS 12
#define TP_SIGMA_KEEP 64
#define TP_MLP_HIDDEN 64
typedef struct tp_learned_opts {
    const float* mlp;          /* device MLP parameters (tp_mlp_param_count floats) or NULL */
    int fixed_rank;            /* kpred of every slice when mlp is NULL */
    const int* prev_rank;      /* device int[floor(n3/2)+1] or NULL (a feature) */
    const float* prev_sigma;   /* device float[(floor(n3/2)+1) * TP_SIGMA_KEEP] or NULL */
    int oversample;            /* extra sketch columns (the paper setting: 10) */
    int power_iters;           /* subspace iterations (2) */
    int max_rank;              /* l_max <= 64: wider slices use the full SVD */
    unsigned long long seed;   /* sketch seed */
    float accuracy;            /* a posteriori residual tolerance, 0 = no check */
    int max_power_iters;       /* cap on power iterations with the check */
    int retry_wide;            /* 1: retry count-check failures once at the widest sketch */
    int accuracy_ref;          /* 0: check relative to max(result, input), 1: to the result */
    const float* warm_basis;   /* device, optional: a previous call's basis_out */
    const int* warm_cols;      /* device int[floor(n3/2)+1]: its basis_cols_out */
    float* basis_out;          /* device, optional: this call's range basis Q2 */
    int* basis_cols_out;       /* device int[floor(n3/2)+1]: valid columns per slice */
} tp_learned_opts;
size_t tp_prox_tnn_learned_workspace_size(int n1, int n2, int n3, int max_rank);
int tp_prox_tnn_learned(const float* Y, float* X, int n1, int n2, int n3, float tau,
                        const tp_learned_opts* opts, int* rank, int* fallback, int* info,
                        float* sigma_out, void* workspace, size_t workspace_bytes, void* stream);
/* the per-slice features above, feats is device float[(floor(n3/2)+1) * TP_MLP_INPUTS] */
size_t tp_slice_features_workspace_size(int n1, int n2, int n3);
int tp_slice_features(const float* Y, int n1, int n2, int n3, float tau, const int* prev_rank,
                      const float* prev_sigma, float* feats, void* workspace, size_t workspace_bytes,
                      void* stream);

/*
 * Rank-predicting MLP: TP_MLP_INPUTS -> 64 -> 64 -> 64 -> 1, ReLU hidden
 * layers.  Parameters (device float, tp_mlp_param_count() of them) are packed
 * W1 (64 x TP_MLP_INPUTS, row-major), b1 (64), W2 (64 x 64), b2, W3 (64 x 64),
 * b3, w4 (64), b4 (1).  x is batch x TP_MLP_INPUTS row-major, y and t are
 * batch floats.
 * tp_mlp_loss_grad: loss = mean_s c(e_s) e_s^2 with e_s = y_s - t_s and
 * c(e) = 1 for e >= 0, `under` for e < 0 (under-prediction costs a fallback);
 * grad receives d loss / d params and loss (device float) its value; the sums
 * over the batch run in index order (bitwise reproducible).
 * tp_mlp_adam: Adam step number `step` (>= 1) on params with moments m, v.
 */
int tp_mlp_param_count(void);
int tp_mlp_forward(const float* params, const float* x, float* y, int batch, void* stream);
size_t tp_mlp_train_workspace_size(int batch);
int tp_mlp_loss_grad(const float* params, const float* x, const float* t, int batch, float under,
                     float* grad, float* loss, void* workspace, size_t workspace_bytes, void* stream);
int tp_mlp_adam(float* params, const float* grad, float* m, float* v, int step, float lr, float beta1,
                float beta2, float eps, void* stream);

/*
 * Tensor inverse (Definition 2.4): B with A * B = B * A = I for a square
 * n x n x n3 tensor A.  The Fourier slices of I are identities, so B's
 * slices are the inverses of A's: real DFT, Gauss-Jordan with partial
 * pivoting (largest modulus, first row on ties; FP32 data, FP64 moduli) on
 * each of the floor(n3/2)+1 leading slices, inverse DFT.  n <= 1024.
 *   A, B   device n x n x n3
 *   info   device int[floor(n3/2)+1] or NULL: 0, or j+1 when slice k's pivot
 *          of step j is zero (a singular slice; B is then undefined)
 */
size_t tp_tinv_workspace_size(int n, int n3);
int tp_tinv(const float* A, float* B, int n, int n3, int* info, void* workspace, size_t workspace_bytes,
            void* stream);

/*
 * T-QR (Theorem 2.4): A = Q * R with Q (n1 x n1 x n3) orthogonal
 * (Definition 2.5) and R (n1 x n2 x n3) f-upper triangular.  Per Fourier
 * slice a Householder QR (FP32 data, FP64 norms and dot products), with row i
 * of R and column i of Q rephased so that the Fourier slices of R have real,
 * non-negative diagonals: R is then unique for full-rank slices, and so are
 * Q's first min(n1, n2) columns (the rest complete the basis).  The theorem
 * names the orthogonal factor U; it is Q.
 *   A      device n1 x n2 x n3;  Q  device n1 x n1 x n3;  R  device n1 x n2 x n3
 */
size_t tp_tqr_workspace_size(int n1, int n2, int n3);
int tp_tqr(const float* A, float* Q, float* R, int n1, int n2, int n3, void* workspace, size_t workspace_bytes,
           void* stream);

/*
 * Tensor robust PCA, the recovery problem the paper names as the use of the
 * TNN and its prox (Section 1; eq (19) and Theorem 2.3):
 *   min ||L||_* + lambda ||S||_1   s.t.   L + S = X
 * (||.||_* the TNN of Definition 2.9).  The paper gives no algorithm for it;
 * this is the inexact augmented Lagrangian method, one prox per iteration:
 *   L' = prox_tnn(X - S - Lam/mu, 1/mu)       (tp_prox_tnn, or the learned-rank
 *                                               prox with `learned`)
 *   S' = sign(r) max(|r| - lambda/mu, 0),  r = X - L' - Lam/mu
 *   Lam <- Lam + mu (L' + S' - X);  mu <- min(rho mu, mu_max)
 * until max(max|L' - L|, max|S' - S|, max|L' + S' - X|) <= tol max(1, max|X|)
 * (a relative tolerance: FP32 data cannot reach the absolute 1e-8 customary
 * in double precision) or max_iter iterations.  Everything but the prox is
 * one fused pass over the entries per iteration.
 *   X          device, n1 x n2 x n3 (read only)
 *   L, S       device, n1 x n2 x n3 (outputs; overwritten from zero)
 *   Lam        device n1 x n2 x n3 or NULL: the final multiplier (the
 *              workspace holds it when NULL)
 *   iters, converged   host ints or NULL: iterations run; 1 if the
 *              stopping test was met
 *   opts       required.  lambda <= 0 selects 1/sqrt(max(n1, n2) n3).
 *              learned NULL: the full-SVD prox (Algorithm 3).  Otherwise the
 *              learned-rank prox with those settings; the driver chains its
 *              calls itself (the previous call's counts and singular values
 *              as features, its range basis as warm start, seed + i for call
 *              i), so learned->prev_rank, prev_sigma, warm_basis, warm_cols,
 *              basis_out and basis_cols_out are ignored.
 *              record: NULL, or where to keep what each prox call saw and
 *              did (tp_trpca_record), for training the rank predictor and
 *              for replaying the calls.
 * Errors: TP_ERR_ARG (null pointers, mu <= 0, rho < 1, mu_max < mu or
 * infinite, tol < 0, max_iter < 1, a learned max_rank outside 1..64, a NaN
 * in X, a record with max_calls < 0), TP_ERR_SHAPE, TP_ERR_WORKSPACE, or the
 * prox's error.  The call waits for the stream once per iteration (the
 * stopping test is read on the host).
 */
/* Per-call record of tp_trpca: call i (0-based, i < max_calls; later calls
 * are not kept) has tau_i = 1/mu_i, mu_0 = mu, mu_(i+1) = min(rho mu_i,
 * mu_max) in double precision, and the learned prox's seed + i.  Every
 * buffer is optional (NULL) device memory with max_calls rows; h =
 * floor(n3/2)+1.
 *   inputs       float[max_calls][n1*n2*n3]: the prox input Y_i
 *   features     float[max_calls][h][TP_MLP_INPUTS]: tp_slice_features of
 *                Y_i (with call i-1's counts and singular values for the
 *                learned prox, none for the full one)
 *   counts       int[max_calls][h]: the learned prox's count per slice
 *   sigmas       float[max_calls][h][TP_SIGMA_KEEP]: its sigma_out
 *   bases        float[max_calls][2][h][n2][max_rank]: its basis_out
 *   basis_cols   int[max_calls][h]: its basis_cols_out
 * (counts, sigmas, bases and basis_cols need the learned prox.) */
typedef struct tp_trpca_record {
    int max_calls;
    float* inputs;
    float* features;
    int* counts;
    float* sigmas;
    float* bases;
    int* basis_cols;
} tp_trpca_record;
typedef struct tp_trpca_opts {
    float lambda;                   /* <= 0: 1/sqrt(max(n1, n2) n3) */
    float mu;                       /* initial penalty (1e-3) */
    float rho;                      /* penalty growth per iteration (1.1) */
    float mu_max;                   /* penalty cap (1e10) */
    float tol;                      /* relative stopping tolerance (1e-5) */
    int max_iter;                   /* iteration cap (500) */
    const tp_learned_opts* learned; /* NULL: full-SVD prox; else learned-rank prox settings */
    const tp_trpca_record* record;  /* NULL, or per-call records */
} tp_trpca_opts;
size_t tp_trpca_workspace_size(int n1, int n2, int n3, const tp_trpca_opts* opts);
int tp_trpca(const float* X, float* L, float* S, int n1, int n2, int n3, const tp_trpca_opts* opts, float* Lam,
             int* iters, int* converged, void* workspace, size_t workspace_bytes, void* stream);

/*
 * Tensor nuclear norm (Definition 2.9 with eq (14)):
 *   ||A||_* = sum_i S(i,i,1) = (1/n3) sum_k sum_i sigma_i(Abar^(k)),
 * summed over all n3 slices through the conjugate symmetry of eq (8) (the
 * DC and, for even n3, middle slices once, the others twice), in FP64.
 *   out    device double (output)
 *   info   as for tp_prox_tnn
 */
size_t tp_tnn_workspace_size(int n1, int n2, int n3);
int tp_tnn(const float* A, int n1, int n2, int n3, double* out, int* info, void* workspace,
           size_t workspace_bytes, void* stream);

/*
 * Order-p tensors, p = 2 + nd (the p-way extension the introduction of the
 * paper defers to its reference [6]).  A tensor n1 x n2 x n3 x ... x np is
 * C-ordered with np fastest (for nd = 1 exactly the 3-way layout above);
 * dims[0 .. nd-1] = n3 .. np is a HOST int array, 1 <= nd <= 8, every
 * dims[a] in 1..1024, and the number of Fourier slices
 * h = n3 ... n_(p-1) * (floor(np/2)+1) at most 65535 (TP_ERR_SHAPE
 * otherwise).  The t-product is defined recursively on the last mode (a
 * block circulant of order-(p-1) tensors, Definition 2.1 at p = 3), which a
 * DFT along each of modes 3..p diagonalises: the library transforms modes
 * 3..p (a real DFT along mode p, keeping floor(np/2)+1 bins as in eq (8),
 * complex DFTs along modes 3..p-1), works on the h kept Fourier slices as
 * Algorithms 1 and 3 do, and transforms back.  FP32 arithmetic only.
 *
 * tp_tprod_nd: C = A * B, A n1 x n2 x dims, B n2 x l x dims, C n1 x l x dims.
 * tp_prox_tnn_nd: X = Prox_tau(Y) for ||X||_* = (1/rho) sum over all
 *   rho = n3 ... np Fourier slices of the matrix nuclear norms (eq (14) over
 *   modes 3..p): the matrix SVT with threshold tau on every slice (Theorem
 *   2.3; Parseval over modes 3..p carries its proof over).  info and rank as
 *   for tp_prox_tnn, device int[h] each, slice s = kp * (n3 ... n_(p-1)) +
 *   (k3, ..., k_(p-1)) in row-major order, kp the mode-p bin.
 * tp_tnn_nd: that nuclear norm into the device double out (the slices with
 *   mode-p bin 0 or, for even np, np/2 once, the others twice), FP64 sums.
 * Errors as the 3-way calls.  nd = 1 computes exactly what tp_tprod (FP32),
 * tp_prox_tnn and tp_tnn compute.
 */
size_t tp_tprod_nd_workspace_size(int n1, int n2, int l, int nd, const int* dims);
int tp_tprod_nd(const float* A, const float* B, float* C, int n1, int n2, int l, int nd, const int* dims,
                void* workspace, size_t workspace_bytes, void* stream);
size_t tp_prox_tnn_nd_workspace_size(int n1, int n2, int nd, const int* dims);
int tp_prox_tnn_nd(const float* Y, float* X, int n1, int n2, int nd, const int* dims, float tau, int* info,
                   int* rank, void* workspace, size_t workspace_bytes, void* stream);
size_t tp_tnn_nd_workspace_size(int n1, int n2, int nd, const int* dims);
int tp_tnn_nd(const float* A, int n1, int n2, int nd, const int* dims, double* out, int* info, void* workspace,
              size_t workspace_bytes, void* stream);

/*
 * Batched tprod and prox_tnn over many tensors of uneven sizes (the slice
 * pipeline of Algorithms 1 and 3 applied to each tensor).  A plan lists the
 * work of every tensor; each stage of the pipeline is then one launch of a
 * persistent kernel over all tensors (transforms, slice products, Jacobi
 * SVDs, shrinkage), so the cost of a batch does not grow with launches per
 * tensor.
 *   tp_batch_create  validates the items and sizes the plan (host only; the
 *                    item array is copied; the tensors must stay allocated
 *                    while the plan is used).  op is TP_BATCH_TPROD
 *                    (C_i = A_i * B_i, n1 x l x n3) or TP_BATCH_PROX
 *                    (C_i = prox of tau_i ||.||_* at A_i, n1 x n2 x n3; n1, n2
 *                    <= 128).  With TP_BATCH_TAU_REL (prox only) tau_i =
 *                    item.tau * tsn(A_i), tsn = max_k sigma_1(Abar^(k))
 *                    (Definition 2.8), computed on the device between the SVD
 *                    and the shrinkage.  n3 <= 128.  opts may be NULL (all
 *                    zero = automatic): tile 1 = 32x32, 2 = 64x64 output tiles
 *                    of the slice products; grid_* persistent workgroups per
 *                    stage; max_sweeps the Jacobi cap.
 *   tp_batch_workspace_size  device bytes for the tables and all planes.
 *   tp_batch_bind    writes the plan's descriptor tables into the workspace
 *                    (device memory, caller-owned, at least the size above) on
 *                    `stream` and waits for the copy.
 *   tp_batch_run     enqueues the stages on `stream`; no allocation, copy or
 *                    synchronisation, so a HIP graph may capture it and
 *                    replay it while the workspace and the tensors live.
 *   tp_batch_stats   unit counts and the chosen launch shapes.
 * Optional per-item outputs (device, prox only): rank int[floor(n3/2)+1]
 * (#{sigma_j > tau_i} per slice) and tau_used float[1].
 */
#define TP_BATCH_TPROD 0
#define TP_BATCH_PROX 1
#define TP_BATCH_TAU_REL 1
typedef struct tp_batch_item {
    int n1, n2, l, n3;
    const float* A;
    const float* B;      /* tprod only */
    float* C;
    float tau;           /* prox: tau, or its factor of tsn(A) with TP_BATCH_TAU_REL */
    int* rank;           /* optional, prox */
    float* tau_used;     /* optional, prox */
} tp_batch_item;
typedef struct tp_batch_opts {
    int tile;            /* 0 auto, 1 = 32x32, 2 = 64x64 */
    int grid_fft, grid_gemm, grid_jacobi;  /* 0 auto */
    int max_sweeps;      /* 0 = TP_PARAM_JACOBI_SWEEPS */
} tp_batch_opts;
typedef struct tp_batch_stats_t {
    int fft_units, gemm_units, slice_units, tile, grid_fft, grid_gemm, grid_jacobi;
    double gemm_flops, fft_bytes;
} tp_batch_stats_t;
typedef struct tp_batch tp_batch;
int tp_batch_create(tp_batch** plan, int op, const tp_batch_item* items, int count, int flags,
                    const tp_batch_opts* opts);
size_t tp_batch_workspace_size(const tp_batch* plan);
int tp_batch_bind(tp_batch* plan, void* workspace, size_t workspace_bytes, void* stream);
int tp_batch_run(const tp_batch* plan, void* stream);
int tp_batch_stats(const tp_batch* plan, tp_batch_stats_t* stats);
int tp_batch_destroy(tp_batch* plan);

/*
 * Tunable launch parameters (process-wide, host side).  They select among
 * equivalent kernel schedules: results stay within the documented
 * tolerances for every setting, but workspace sizes may change, so query them
 * after setting.  tp_set_param returns TP_ERR_ARG for an unknown key or a
 * negative value; 0 restores the default of a key.  tp_get_param returns the
 * value in effect (the default when unset), or -1 for an unknown key.
 *   TP_PARAM_JACOBI_BLOCK         block width of the multi-workgroup Jacobi
 *                                 (0 = chosen from the slice height)
 *   TP_PARAM_JACOBI_MODE          0 auto, 1 one workgroup per slice when the
 *                                 slice fits in LDS, 2 always multi-workgroup
 *   TP_PARAM_JACOBI_BLOCKED_BELOW auto mode: slices that fit in LDS go
 *                                 multi-workgroup when fewer than this many
 *                                 slices are processed (default 128)
 *   TP_PARAM_JACOBI_SWEEPS        sweep cap (default 30)
 *   TP_PARAM_GEMM_VARIANT         slice GEMM tile variant: 0 = by shape, 1 = 64x64,
 *                                 2 = 128x128, 3 = 128x64, 4 = 128x32, 5 = 256x16,
 *                                 6 = 64x48 (output rows x columns per workgroup),
 *                                 7 = narrow-output kernel (FP32, op(B) = B, at most
 *                                 64 output columns and a multiple of 4, inner
 *                                 dimension >= 64; by shape it takes every such
 *                                 product, variants 1 .. 6 keep them on the tiles),
 *                                 8 = wide-output kernel (FP32, A B, inner dimension
 *                                 1 .. 64, m a multiple of 64 and n of 256, 16-byte
 *                                 aligned B and C; by shape it takes every such
 *                                 product that the narrow kernel does not)
 *   TP_PARAM_FFT_GRID             persistent workgroups per compute unit of the
 *                                 tube transforms (0 = default 8)
 *   TP_PARAM_GEMM_BK              FP32 slice GEMM inner-dimension stage: 16 or 32
 *                                 columns (0 = 32 when the inner dimension is >= 256
 *                                 and the tile is at least 64 columns wide)
 *   TP_PARAM_GEMM_KSPLIT          learned-rank prox: parts of the inner dimension of
 *                                 its long products (0 = by shape, else 1 .. 4)
 *   TP_PARAM_FFT_DIRECT           loads of the power-of-two forward transform: 1 =
 *                                 each lane reads its own tube with 16-byte loads
 *                                 (default), 2 = staged through LDS (the inverse
 *                                 always stores through LDS, coalesced)
 *   TP_PARAM_JACOBI_STEPWISE      form of the multi-workgroup Jacobi without V:
 *                                 1 = one launch per block step, the blocks
 *                                 staged in LDS; 2 = one launch per sweep, the
 *                                 column pairs in registers; 0 = by slice height
 *                                 (per sweep above 256 rows)
 *   TP_PARAM_RETRY_ROUNDS         learned-rank prox: accuracy rounds of the wide
 *                                 retry attempt (0 = default 2; at most the
 *                                 first attempt's max_power_iters - power_iters)
 *   TP_PARAM_JACOBI_GRAM          multi-workgroup Jacobi without V: block pairs
 *                                 through their Gram matrices (MFMA products,
 *                                 FP64 rotations of the Gram matrix, one MFMA
 *                                 update of the columns per block pair): 0 = on,
 *                                 16-column block pairs up to 256 rows and 32
 *                                 above; 1 = off (the column-rotation forms);
 *                                 2 = 16 columns; 3 = 32 columns
 *   TP_PARAM_LEARNED_HOST         learned-rank prox: 1 = the host reads the
 *                                 device's decisions (after each accuracy round,
 *                                 after the retry test, the fallback count) and
 *                                 enqueues only the work that runs; the call then
 *                                 synchronizes its stream at those points and
 *                                 cannot be captured (on a capturing stream it
 *                                 keeps the default).  0 (default): every launch
 *                                 is enqueued and gated on the device, so the
 *                                 call never waits for the device and can be
 *                                 captured.  Both give the same bits.
 * The bf16 slice products (TP_PREC_BF16X3, TP_PREC_BF16) read
 * TP_PARAM_GEMM_VARIANT as: 1 = 64x64, 2 = 128x128, 3 = 128x32 tiles on
 * 16x16x32 products, 4 = 256x128 and 5 = 128x128 on 32x32x16 products,
 * 6 .. 8 = 64x64 (0 = by shape); the workspace size depends on the choice.
 */
enum {
    TP_PARAM_JACOBI_BLOCK = 0,
    TP_PARAM_JACOBI_MODE = 1,
    TP_PARAM_JACOBI_BLOCKED_BELOW = 2,
    TP_PARAM_JACOBI_SWEEPS = 3,
    TP_PARAM_GEMM_VARIANT = 4,
    TP_PARAM_FFT_GRID = 5,
    TP_PARAM_FFT_DIRECT = 6,
    TP_PARAM_GEMM_BK = 7,
    TP_PARAM_GEMM_KSPLIT = 8,
    TP_PARAM_JACOBI_STEPWISE = 9,
    TP_PARAM_RETRY_ROUNDS = 10,
    TP_PARAM_JACOBI_GRAM = 11,
    TP_PARAM_LEARNED_HOST = 12,
    TP_PARAM_COUNT = 13
};
int tp_set_param(int key, int value);
int tp_get_param(int key);

/*
 * Stage timing (a profiling aid; not for use under stream capture).  While
 * enabled, every entry point records a HIP event on its stream before and
 * after each kernel it enqueues.  tp_trace_collect waits for those events and
 * writes, in launch order, the kernel id and its elapsed time in ms for up to
 * `capacity` launches; it returns the number of launches recorded since the
 * last collect (or a negative tp_status) and forgets them.
 * Kernel ids: 0 rfft, 1 irfft, 2 cgemm, 3 jacobi, 4 shrink, 5 tnn_reduce,
 * 6 tsvd_finish, 7 features, 8 predict, 9 sketch, 10 cholqr, 11 rsvd_check,
 * 12 gather, 13 mlp, 14 accuracy, 15 tensor_op, 16 trpca.
 * tp_trace_collect_work also writes, per launch, the algorithmic work the
 * library assigns to it (host arrays, either may be NULL): for the slice
 * products 8 m n k flops per complex slice and 2 m n k per real one, and the
 * FP32 bytes of both operands and the result (8 per complex element, 4 per
 * real one); for the transforms 4 n1 n2 n3 bytes on the tensor side plus
 * 8 h n1 n2 on the slice side; 0 for the other kernels.  A product whose
 * gate or sizes are decided on the device (the learned-rank prox) gets the
 * work of the sizes it ran at, 0 when its gate was closed, evaluated at
 * collection time from the values then in device memory: collect after each
 * such call for exact figures.  Products over a device-counted set of
 * slices (the learned prox's full-SVD fallback) are given no work.
 */
int tp_trace_enable(int enable);
int tp_trace_collect(int* kernel_ids, float* ms, int capacity);
int tp_trace_collect_work(int* kernel_ids, float* ms, double* flops, double* bytes, int capacity);
const char* tp_kernel_name(int id);

#ifdef __cplusplus
}
#endif
#endif /* TP_H */
