/*
 * tp_oracle.h -- FP64 CPU oracle for the t-product toolbox (Lu, 2018).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may include, link or
 * call this library: only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code with the GPU library.
 *
 * Conventions (all buffers are host memory owned by the caller):
 *   - a real tensor A of size n1 x n2 x n3 is row-major with the tube index
 *     last: A(i,j,t) = A[(i*n2 + j)*n3 + t], 0-based (the paper is 1-based);
 *   - a complex tensor uses the same index order with C99 double complex
 *     elements (interleaved re, im);
 *   - a matrix is row-major: M(i,j) = M[i*ncols + j].
 *
 * Every routine computes in double precision.  Functions that return int
 * return 0 on success, a positive sweep-cap code when a Jacobi iteration did
 * not converge, or a negative value on a bad argument.
 */
#ifndef TP_ORACLE_H
#define TP_ORACLE_H

#include <complex.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef double _Complex or_cplx;

/* threads used by the OpenMP loops (0 = library default) */
void or_set_threads(int nthreads);
int or_get_threads(void);

/* Section 2.2, eq (2) and eq (1): DFT along every mode-3 tube, or its inverse
 * F^* / n3 when inverse != 0.  X and Y may not alias. */
void or_dft3(const or_cplx* X, int n1, int n2, int n3, int inverse, or_cplx* Y);

/* Section 2.2, eq (6): bcirc(A), an (n1*n3) x (n2*n3) real matrix. */
void or_bcirc(const double* A, int n1, int n2, int n3, double* M);
/* Section 2.3: unfold(A) is (n1*n3) x n2; fold is its inverse. */
void or_unfold(const double* A, int n1, int n2, int n3, double* M);
void or_fold(const double* M, int n1, int n2, int n3, double* A);

/* Definition 2.1, eq (9), evaluated block row by block row:
 * C^(r) = sum_c A^((r-c) mod n3) B^(c). */
void or_tprod_def(const double* A, const double* B, int n1, int n2, int l, int n3, double* C);
/* the same definition at selected flat indices of C (idx[e] = (i*l + j)*n3 + t) */
void or_tprod_def_entries(const double* A, const double* B, int n1, int n2, int l, int n3,
                          const long long* idx, long long nidx, double* out);
/* Algorithm 1: DFT, products of the ceil((n3+1)/2) leading Fourier slices,
 * conjugate fill of the rest, inverse DFT (real part returned). */
void or_tprod_fft(const double* A, const double* B, int n1, int n2, int l, int n3, double* C);

/* Definition 2.2 (conjugate transpose of a real tensor) and Definition 2.3. */
void or_tran(const double* A, int n1, int n2, int n3, double* At);
void or_teye(int n, int n3, double* Ieye);

/* SVD of an m x n complex matrix by one-sided Jacobi.  sigma[min(m,n)] is
 * sorted in decreasing order.  full != 0: U is m x m and V is n x n (bases
 * completed); full == 0: U is m x p and V is n x p, p = min(m,n).  U or V may
 * be NULL.  Returns the number of sweeps (>= 0) or -1 if the sweep cap hit. */
int or_svd(const or_cplx* M, int m, int n, int full, double* sigma, or_cplx* U, or_cplx* V);

/* Theorem 2.2 / Algorithm 2.  U is n1 x n1 x n3, S is n1 x n2 x n3, V is
 * n2 x n2 x n3.  maximag (may be NULL) receives the largest imaginary part
 * left by the inverse DFTs (it should be rounding noise). */
int or_tsvd(const double* A, int n1, int n2, int n3, double* U, double* S, double* V,
            double* maximag);
/* singular values of every Fourier slice: sig is n3 x min(n1,n2), row k for
 * slice k (all n3 slices, no symmetry used). */
int or_slice_sigma(const double* A, int n1, int n2, int n3, double* sig);
/* Definition 2.9 with eq (14): sum_i S(i,i,1) = (1/n3) sum_k ||Abar^(k)||_* . */
double or_tnn(const double* A, int n1, int n2, int n3);
/* Definition 2.8 with eq (17): ||bcirc(A)|| = max_k sigma_1(Abar^(k)). */
double or_tsn(const double* A, int n1, int n2, int n3);

/* Definition 2.7: the number of nonzero singular tubes S(i,i,:) of the
 * t-SVD.  In floating point a tube counts when S(i,i,1) > tol, where
 * S(i,i,1) = (1/n3) sum_k sigma_i(Abar^(k)) (the first frontal slice of S is
 * the mean of the Fourier-domain S, eq (2) inverted at t = 0) with each
 * slice's singular values in decreasing order; tol < 0 selects
 * max(n1, n2) * eps * S(1,1,1). */
int or_tubalrank(const double* A, int n1, int n2, int n3, double tol, double eps);
/* Theorem 2.3 / Algorithm 3: Prox of the TNN at tau. */
int or_prox_tnn(const double* Y, int n1, int n2, int n3, double tau, double* X);
/* Theorem 2.4 (T-QR): A = Q * R, Q n1 x n1 x n3 orthogonal, R n1 x n2 x n3
 * f-upper triangular; per Fourier slice a Householder QR with diag(R) real
 * and >= 0.  Returns 0 (< 0 on a bad argument). */
int or_tqr(const double* A, int n1, int n2, int n3, double* Q, double* R);
/* Definition 2.4: the inverse B of the n x n x n3 tensor A (Gauss-Jordan with
 * partial pivoting per Fourier slice).  Returns 0, or 1 + the first singular
 * Fourier slice (< 0 on a bad argument). */
int or_tinv(const double* A, int n, int n3, double* B);
/* Tensor robust PCA, min ||L||_* + lam ||S||_1 s.t. L + S = X, by the inexact
 * augmented Lagrangian method around or_prox_tnn (the paper names the problem
 * but gives no algorithm; the steps are listed in tp_oracle.c).  L, S, Lam
 * are outputs (n1*n2*n3 each); returns 1 if converged, 0 if not, < 0 on a bad
 * argument; *iters = iterations run. */
int or_trpca(const double* X, int n1, int n2, int n3, double lam, double mu, double rho, double mu_max,
             double tol, int max_iter, double* L, double* S, double* Lam, int* iters);
/* matrix singular value thresholding U (S - tau)_+ V^* of a real m x n matrix */
int or_svt_real(const double* M, int m, int n, double tau, double* out);

#ifdef __cplusplus
}
#endif
#endif

#ifndef TP_ORACLE_LEARNED_H
#define TP_ORACLE_LEARNED_H
#ifdef __cplusplus
extern "C" {
#endif

/* Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11):
 * ten rounds of the 4x32 Philox S-box on counter ctr[4] with key key[2]. */
void or_philox4x32_10(const unsigned int ctr[4], const unsigned int key[2], unsigned int out[4]);

/* The Gaussian test matrix of the randomized range finder for slice `slice`:
 * entry (i, j) (i < n rows, j < l columns) comes from Philox on counter
 * {i, j, slice, 0} with key {seed low, seed high}; the first two outputs x0, x1
 * give u = (x + 0.5) 2^-32 and by Box-Muller z0 = sqrt(-2 ln u0) cos(2 pi u1),
 * z1 = sqrt(-2 ln u0) sin(2 pi u1).  Complex slices: (z0 + i z1)/sqrt(2);
 * real slices: z0.  Values are rounded to float, then widened.  Om is n x l
 * row-major complex. */
void or_sketch_matrix(int n, int l, int slice, int real, unsigned long long seed, or_cplx* Om);

/* CholeskyQR2 of the m x l complex matrix Y (row-major, in place -> Q), with
 * R (l x l upper triangular, row-major) the product of both factors.  Columns
 * j >= lact are zero on input and output (R = identity there).  A shift
 * 1e-13 * trace(G)/lact is added to the Gram diagonal before the first
 * Cholesky (the second Gram is close to the identity and is not shifted). */
int or_cholqr2(or_cplx* Y, int m, int l, int lact, or_cplx* R);

/* Prox of the TNN (Theorem 2.3) with each leading Fourier slice's SVT done
 * on a randomized range (Halko, Martinsson, Tropp 2011): for slice k with
 * predicted count kpred[k], l = min(kpred[k] + oversample, min(n1, n2));
 * Y = Abar Om; `power` times {Z = Abar^* Q, Y = Abar Z}, every product
 * re-orthonormalised by CholeskyQR2; Bh = Abar^* Q; (Q2, R2) = CholeskyQR2(Bh);
 * SVD of R2^*; W = Q T Q2^* with T = U_r (S - tau)_+ V_r^*.  The slice falls
 * back to the full SVD (Algorithm 3) when l >= lfull or when the (kpred+1)-th
 * singular value of R2^* is not below tau.  fallback[k] (may be NULL)
 * receives 1 for a fallback, rank[k] (may be NULL) the number of singular
 * values above tau that were used. */
int or_prox_tnn_rsvd(const double* Y, int n1, int n2, int n3, double tau, const int* kpred, int oversample,
                     int power, int lfull, unsigned long long seed, double* X, int* fallback, int* rank);

/* Per-slice features of the rank predictor, for the floor(n3/2)+1 leading
 * Fourier slices (row k of feats, 12 values): log(tau / (||Ybar^(k)||_F /
 * sqrt(p))), log(max column norm / tau), prev[k]/p and 1 (0, 0 without prev),
 * k/(n3/2), 1 for a real slice, log(p)/8, log(max(n1,n2)/p); from the
 * previous leading singular values s (psig, 64 per slice, decreasing,
 * zero-padded; zeros without psig): #{s > tau}/p, #{s > tau/1.25}/p,
 * log(s_1/tau), [s_c > tau] with c the number of nonzero s; p = min(n1,n2);
 * logarithms clamped to [-30, 30]. */
void or_slice_features(const double* Y, int n1, int n2, int n3, double tau, const int* prev, const double* psig,
                       double* feats);

/* MLP with ReLU hidden layers: sizes d -> h -> h -> h -> 1.  Parameters packed
 * as W1 (h x d, row-major), b1 (h), W2 (h x h), b2, W3 (h x h), b3, w4 (h), b4.
 * or_mlp_forward: y[s] for the N rows of X (N x d).
 * or_mlp_loss_grad: loss = mean_s c(e_s) e_s^2 with e_s = y_s - t_s and
 * c(e) = 1 for e >= 0, `under` for e < 0; grad receives d loss / d params. */
int or_mlp_param_count(int d, int h);
void or_mlp_forward(const double* params, int d, int h, const double* X, int N, double* y);
double or_mlp_loss_grad(const double* params, int d, int h, const double* X, const double* t, int N,
                        double under, double* grad);

#ifdef __cplusplus
}
#endif
#endif
