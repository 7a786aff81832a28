/*
 * tp_oracle.c -- plain FP64 CPU oracle for the t-product toolbox (Lu, 2018).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
 * baseline of the benchmark, never by the product path.  It shares no code
 * with the GPU library.  The code favours being checkable against the paper
 * over speed: every routine follows a definition or an algorithm of the paper
 * step by step, in double precision, with no FFT, no BLAS and no LAPACK.
 * OpenMP only spreads independent slices, tubes or rows over host threads.
 *
 * Readings of the paper taken here (the paper is 1-based, this file 0-based):
 *   - the number of Fourier slices that get a dense operation in Algorithms
 *     1-3, ceil((n3+1)/2), equals floor(n3/2)+1;
 *   - for even n3 the slice k = n3/2 is self-conjugate and hence real, like
 *     the slice k = 0 (Lemma 2.1 / eq (8) only state it for the first);
 *   - the tensor nuclear norm carries the 1/n3 factor of Definition 2.9 with
 *     eq (14); eq (18) omits it;
 *   - "SVD" is computed by one-sided (Hestenes) Jacobi; the DFT twiddles
 *     omega^e are reduced exactly modulo n and the quarter-turn values are
 *     exact, so the real slices come out with exactly zero imaginary parts.
 */
#include "tp_oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAX_SWEEPS 100

typedef long long i64;

static int g_threads = 0;

void or_set_threads(int nthreads)
{
    g_threads = nthreads;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
}

int or_get_threads(void)
{
#ifdef _OPENMP
    return g_threads > 0 ? g_threads : omp_get_max_threads();
#else
    return 1;
#endif
}

static void* xmalloc(size_t bytes)
{
    void* p = malloc(bytes ? bytes : 1);
    if (!p) abort();
    return p;
}

static inline i64 idx3(i64 i, i64 j, i64 t, int n2, int n3) { return (i * n2 + j) * n3 + t; }
static inline int mod(i64 a, int n) { i64 r = a % n; return (int)(r < 0 ? r + n : r); }
static inline double abs2(or_cplx z) { return creal(z) * creal(z) + cimag(z) * cimag(z); }

/* ------------------------------------------------------------------------ */
/* Section 2.2: omega = exp(-2 pi i / n) (definition of F_n) raised to e.     */
/* ------------------------------------------------------------------------ */
static or_cplx omega_pow(i64 e, int n)
{
    i64 m = mod(e, n);
    if (m == 0) return 1.0;
    if (2 * m == n) return -1.0;
    if (4 * m == n) return -I;
    if (4 * m == 3 * (i64)n) return I;
    double ang = -2.0 * M_PI * (double)m / (double)n;
    return cos(ang) + I * sin(ang);
}

/* eq (2): Y(i,j,k) = sum_t omega^(k t) X(i,j,t); inverse: F^{-1} = F^* / n (eq (1)) */
void or_dft3(const or_cplx* X, int n1, int n2, int n3, int inverse, or_cplx* Y)
{
    or_cplx* w = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)n3 * n3);
    for (int k = 0; k < n3; ++k)
        for (int t = 0; t < n3; ++t) {
            or_cplx f = omega_pow((i64)k * t, n3);
            w[k * n3 + t] = inverse ? conj(f) / (double)n3 : f;
        }
    const i64 ntubes = (i64)n1 * n2;
#pragma omp parallel for schedule(static)
    for (i64 tube = 0; tube < ntubes; ++tube) {
        const or_cplx* x = X + tube * n3;
        or_cplx* y = Y + tube * n3;
        for (int k = 0; k < n3; ++k) {
            or_cplx s = 0.0;
            for (int t = 0; t < n3; ++t) s += w[k * n3 + t] * x[t];
            y[k] = s;
        }
    }
    free(w);
}

/* ------------------------------------------------------------------------ */
/* Section 2.2 eq (6) and Section 2.3 (unfold / fold).                        */
/* ------------------------------------------------------------------------ */
void or_bcirc(const double* A, int n1, int n2, int n3, double* M)
{
    const i64 ncol = (i64)n2 * n3;
    for (int r = 0; r < n3; ++r)          /* block row    */
        for (int c = 0; c < n3; ++c) {    /* block column */
            int s = mod((i64)r - c, n3);  /* block (r,c) = A^((r-c) mod n3) */
            for (int i = 0; i < n1; ++i)
                for (int j = 0; j < n2; ++j)
                    M[((i64)r * n1 + i) * ncol + (i64)c * n2 + j] = A[idx3(i, j, s, n2, n3)];
        }
}

void or_unfold(const double* A, int n1, int n2, int n3, double* M)
{
    for (int t = 0; t < n3; ++t)
        for (int i = 0; i < n1; ++i)
            for (int j = 0; j < n2; ++j) M[((i64)t * n1 + i) * n2 + j] = A[idx3(i, j, t, n2, n3)];
}

void or_fold(const double* M, int n1, int n2, int n3, double* A)
{
    for (int t = 0; t < n3; ++t)
        for (int i = 0; i < n1; ++i)
            for (int j = 0; j < n2; ++j) A[idx3(i, j, t, n2, n3)] = M[((i64)t * n1 + i) * n2 + j];
}

/* ------------------------------------------------------------------------ */
/* Definition 2.1, eq (9).  Block row r of bcirc(A) times unfold(B):         */
/*   C^(r) = sum_c A^((r-c) mod n3) B^(c).                                   */
/* ------------------------------------------------------------------------ */
void or_tprod_def(const double* A, const double* B, int n1, int n2, int l, int n3, double* C)
{
    /* frontal slices of B, B^(c)(p,j), stored slice by slice for locality */
    double* Bs = (double*)xmalloc(sizeof(double) * (size_t)n3 * n2 * l);
    for (int c = 0; c < n3; ++c)
        for (int p = 0; p < n2; ++p)
            for (int j = 0; j < l; ++j) Bs[((i64)c * n2 + p) * l + j] = B[idx3(p, j, c, l, n3)];
#pragma omp parallel
    {
        double* row = (double*)xmalloc(sizeof(double) * (size_t)l);
#pragma omp for schedule(dynamic)
        for (int i = 0; i < n1; ++i)
            for (int r = 0; r < n3; ++r) {
                for (int j = 0; j < l; ++j) row[j] = 0.0;
                for (int c = 0; c < n3; ++c) {
                    int s = mod((i64)r - c, n3);
                    for (int p = 0; p < n2; ++p) {
                        double a = A[idx3(i, p, s, n2, n3)];
                        const double* b = Bs + ((i64)c * n2 + p) * l;
                        for (int j = 0; j < l; ++j) row[j] += a * b[j];
                    }
                }
                for (int j = 0; j < l; ++j) C[idx3(i, j, r, l, n3)] = row[j];
            }
        free(row);
    }
    free(Bs);
}

void or_tprod_def_entries(const double* A, const double* B, int n1, int n2, int l, int n3,
                          const long long* idx, long long nidx, double* out)
{
    (void)n1;
#pragma omp parallel for schedule(static)
    for (i64 e = 0; e < nidx; ++e) {
        i64 f = idx[e];
        int t = (int)(f % n3);
        int j = (int)((f / n3) % l);
        int i = (int)(f / ((i64)n3 * l));
        double s = 0.0;
        for (int c = 0; c < n3; ++c) {
            int sl = mod((i64)t - c, n3);
            for (int p = 0; p < n2; ++p) s += A[idx3(i, p, sl, n2, n3)] * B[idx3(p, j, c, l, n3)];
        }
        out[e] = s;
    }
}

static or_cplx* real_to_complex(const double* A, i64 n)
{
    or_cplx* z = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)n);
    for (i64 e = 0; e < n; ++e) z[e] = A[e];
    return z;
}

/* frontal slice k of a complex tensor as a row-major n1 x n2 matrix */
static void get_slice(const or_cplx* X, int n1, int n2, int n3, int k, or_cplx* M)
{
    for (int i = 0; i < n1; ++i)
        for (int j = 0; j < n2; ++j) M[(i64)i * n2 + j] = X[idx3(i, j, k, n2, n3)];
}

static void put_slice(or_cplx* X, int n1, int n2, int n3, int k, const or_cplx* M)
{
    for (int i = 0; i < n1; ++i)
        for (int j = 0; j < n2; ++j) X[idx3(i, j, k, n2, n3)] = M[(i64)i * n2 + j];
}

/* Algorithm 1, step 2 second branch (and the same step of Algorithms 2, 3):
 * slice k >= floor(n3/2)+1 is the conjugate of slice n3-k. */
static void conj_fill(or_cplx* X, int n1, int n2, int n3)
{
    const int h = n3 / 2 + 1;
    for (int k = h; k < n3; ++k)
        for (int i = 0; i < n1; ++i)
            for (int j = 0; j < n2; ++j) X[idx3(i, j, k, n2, n3)] = conj(X[idx3(i, j, n3 - k, n2, n3)]);
}

/* real part of the inverse DFT; returns max |imag| */
static double idft_real(const or_cplx* Xbar, int n1, int n2, int n3, double* X)
{
    const i64 n = (i64)n1 * n2 * n3;
    or_cplx* x = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)n);
    or_dft3(Xbar, n1, n2, n3, 1, x);
    double mi = 0.0;
    for (i64 e = 0; e < n; ++e) {
        X[e] = creal(x[e]);
        if (fabs(cimag(x[e])) > mi) mi = fabs(cimag(x[e]));
    }
    free(x);
    return mi;
}

void or_tprod_fft(const double* A, const double* B, int n1, int n2, int l, int n3, double* C)
{
    const int h = n3 / 2 + 1;
    or_cplx* za = real_to_complex(A, (i64)n1 * n2 * n3);
    or_cplx* zb = real_to_complex(B, (i64)n2 * l * n3);
    or_cplx* Ab = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)n1 * n2 * n3);
    or_cplx* Bb = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)n2 * l * n3);
    or_cplx* Cb = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)n1 * l * n3);
    or_dft3(za, n1, n2, n3, 0, Ab); /* step 1 */
    or_dft3(zb, n2, l, n3, 0, Bb);
    free(za);
    free(zb);
#pragma omp parallel for schedule(dynamic)
    for (int k = 0; k < h; ++k) { /* step 2, first branch: Cbar^(k) = Abar^(k) Bbar^(k) */
        or_cplx* a = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)n1 * n2);
        or_cplx* b = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)n2 * l);
        or_cplx* c = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)n1 * l);
        get_slice(Ab, n1, n2, n3, k, a);
        get_slice(Bb, n2, l, n3, k, b);
        for (i64 e = 0; e < (i64)n1 * l; ++e) c[e] = 0.0;
        for (int i = 0; i < n1; ++i)
            for (int p = 0; p < n2; ++p) {
                or_cplx av = a[(i64)i * n2 + p];
                for (int j = 0; j < l; ++j) c[(i64)i * l + j] += av * b[(i64)p * l + j];
            }
        put_slice(Cb, n1, l, n3, k, c);
        free(a);
        free(b);
        free(c);
    }
    conj_fill(Cb, n1, l, n3);    /* step 2, second branch */
    idft_real(Cb, n1, l, n3, C); /* step 3 */
    free(Ab);
    free(Bb);
    free(Cb);
}

/* Definition 2.2: transpose every frontal slice, then reverse slices 2..n3. */
void or_tran(const double* A, int n1, int n2, int n3, double* At)
{
    for (int i = 0; i < n1; ++i)
        for (int j = 0; j < n2; ++j)
            for (int t = 0; t < n3; ++t) At[idx3(j, i, t, n1, n3)] = A[idx3(i, j, mod((i64)n3 - t, n3), n2, n3)];
}

/* Definition 2.3: first frontal slice I_n, the others zero. */
void or_teye(int n, int n3, double* Ieye)
{
    memset(Ieye, 0, sizeof(double) * (size_t)n * n * n3);
    for (int i = 0; i < n; ++i) Ieye[idx3(i, i, 0, n, n3)] = 1.0;
}

/* ------------------------------------------------------------------------ */
/* SVD by one-sided (Hestenes) Jacobi.                                        */
/* ------------------------------------------------------------------------ */

/* Orthogonalise the n columns (length m) of the column-major array a by plane
 * rotations until every pair satisfies |a_p^* a_q| <= m eps ||a_p|| ||a_q||.
 * The rotations are accumulated into v (n x n column-major) when v != NULL.
 * Returns the number of sweeps, or -1 when the sweep cap is reached. */
static int jacobi_columns(or_cplx* a, int m, int n, or_cplx* v)
{
    const double tol = (double)m * DBL_EPSILON;
    for (int sweep = 1; sweep <= OR_MAX_SWEEPS; ++sweep) {
        int rotated = 0;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                or_cplx* x = a + (i64)p * m;
                or_cplx* y = a + (i64)q * m;
                double alpha = 0.0, beta = 0.0;
                or_cplx gamma = 0.0;
                for (int i = 0; i < m; ++i) {
                    alpha += abs2(x[i]);
                    beta += abs2(y[i]);
                    gamma += conj(x[i]) * y[i];
                }
                double g = cabs(gamma);
                if (g == 0.0 || g <= tol * sqrt(alpha) * sqrt(beta)) continue;
                rotated = 1;
                /* with y~ = conj(e) y, e = gamma/|gamma|, the pair (x, y~) has a
                 * real inner product |gamma|; the real rotation
                 *   x' = c x - s y~,  y~' = s x + c y~
                 * zeroes it when t = s/c solves t^2 + 2 zeta t - 1 = 0,
                 * zeta = (beta - alpha) / (2 |gamma|) (smaller root). */
                or_cplx e = gamma / g;
                double zeta = (beta - alpha) / (2.0 * g);
                double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + hypot(1.0, zeta));
                double c = 1.0 / hypot(1.0, t);
                double s = c * t;
                or_cplx sce = s * conj(e), se = s * e;
                for (int i = 0; i < m; ++i) {
                    or_cplx xi = x[i], yi = y[i];
                    x[i] = c * xi - sce * yi;
                    y[i] = se * xi + c * yi;
                }
                if (v) {
                    or_cplx* vx = v + (i64)p * n;
                    or_cplx* vy = v + (i64)q * n;
                    for (int i = 0; i < n; ++i) {
                        or_cplx xi = vx[i], yi = vy[i];
                        vx[i] = c * xi - sce * yi;
                        vy[i] = se * xi + c * yi;
                    }
                }
            }
        if (!rotated) return sweep;
    }
    return -1;
}

/* Fill columns r..ncol-1 of the row-major m x ncol matrix U, whose columns
 * 0..r-1 are orthonormal, with further orthonormal columns: each time the unit
 * vector e_c with the largest component outside the current span is taken and
 * orthogonalised twice (classical Gram-Schmidt). */
static void complete_basis(or_cplx* U, int m, int ncol, int r)
{
    or_cplx* w = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)m);
    for (int j = r; j < ncol; ++j) {
        int best = 0;
        double bestres = -1.0;
        for (int c = 0; c < m; ++c) { /* ||P_perp e_c||^2 = 1 - sum_q |U(c,q)|^2 */
            double in = 0.0;
            for (int q = 0; q < j; ++q) in += abs2(U[(i64)c * ncol + q]);
            if (1.0 - in > bestres) {
                bestres = 1.0 - in;
                best = c;
            }
        }
        for (int i = 0; i < m; ++i) w[i] = (i == best) ? 1.0 : 0.0;
        for (int pass = 0; pass < 2; ++pass)
            for (int q = 0; q < j; ++q) {
                or_cplx coef = 0.0;
                for (int i = 0; i < m; ++i) coef += conj(U[(i64)i * ncol + q]) * w[i];
                for (int i = 0; i < m; ++i) w[i] -= coef * U[(i64)i * ncol + q];
            }
        double nrm = 0.0;
        for (int i = 0; i < m; ++i) nrm += abs2(w[i]);
        nrm = sqrt(nrm);
        for (int i = 0; i < m; ++i) U[(i64)i * ncol + j] = w[i] / nrm;
    }
    free(w);
}

int or_svd(const or_cplx* M, int m, int n, int full, double* sigma, or_cplx* U, or_cplx* V)
{
    if (m <= 0 || n <= 0) return -2;
    if (m < n) {
        /* M^* = U' S V'^*  gives  M = V' S U'^* */
        or_cplx* Mh = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)m * n);
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < n; ++j) Mh[(i64)j * m + i] = conj(M[(i64)i * n + j]);
        int rc = or_svd(Mh, n, m, full, sigma, V, U);
        free(Mh);
        return rc;
    }
    const int p = n; /* m >= n */
    or_cplx* a = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)m * n); /* column-major */
    or_cplx* v = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)n * n);
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < n; ++j) a[(i64)j * m + i] = M[(i64)i * n + j];
    for (int i = 0; i < n * n; ++i) v[i] = 0.0;
    for (int i = 0; i < n; ++i) v[(i64)i * n + i] = 1.0;
    int sweeps = jacobi_columns(a, m, n, v);

    double* s = (double*)xmalloc(sizeof(double) * (size_t)n);
    int* order = (int*)xmalloc(sizeof(int) * (size_t)n);
    for (int j = 0; j < n; ++j) {
        double acc = 0.0;
        for (int i = 0; i < m; ++i) acc += abs2(a[(i64)j * m + i]);
        s[j] = sqrt(acc);
        order[j] = j;
    }
    for (int j = 1; j < n; ++j) { /* stable insertion sort, decreasing */
        int o = order[j], q = j;
        while (q > 0 && s[order[q - 1]] < s[o]) {
            order[q] = order[q - 1];
            --q;
        }
        order[q] = o;
    }
    for (int r = 0; r < p; ++r) sigma[r] = s[order[r]];

    if (V) {
        const int ncv = full ? n : p; /* == n */
        for (int i = 0; i < n; ++i)
            for (int r = 0; r < ncv; ++r) V[(i64)i * ncv + r] = v[(i64)order[r] * n + i];
    }
    if (U) {
        const int ncu = full ? m : p;
        int rank = 0;
        for (int r = 0; r < p; ++r)
            if (sigma[r] > 0.0) rank = r + 1;
        for (int r = 0; r < rank; ++r)
            for (int i = 0; i < m; ++i) U[(i64)i * ncu + r] = a[(i64)order[r] * m + i] / sigma[r];
        complete_basis(U, m, ncu, rank);
    }
    free(s);
    free(order);
    free(a);
    free(v);
    return sweeps < 0 ? -1 : sweeps;
}

/* ------------------------------------------------------------------------ */
/* Theorem 2.2 / Algorithm 2: t-SVD.                                          */
/* ------------------------------------------------------------------------ */
int or_tsvd(const double* A, int n1, int n2, int n3, double* U, double* S, double* V,
            double* maximag)
{
    const int h = n3 / 2 + 1, p = n1 < n2 ? n1 : n2;
    or_cplx* za = real_to_complex(A, (i64)n1 * n2 * n3);
    or_cplx* Ab = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)n1 * n2 * n3);
    or_dft3(za, n1, n2, n3, 0, Ab); /* step 1 */
    free(za);
    or_cplx* Ub = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)n1 * n1 * n3);
    or_cplx* Sb = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)n1 * n2 * n3);
    or_cplx* Vb = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)n2 * n2 * n3);
    for (i64 e = 0; e < (i64)n1 * n2 * n3; ++e) Sb[e] = 0.0;
    int status = 0;
#pragma omp parallel for schedule(dynamic)
    for (int k = 0; k < h; ++k) { /* step 2, first loop */
        or_cplx* a = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)n1 * n2);
        or_cplx* u = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)n1 * n1);
        or_cplx* v = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)n2 * n2);
        double* sg = (double*)xmalloc(sizeof(double) * (size_t)p);
        get_slice(Ab, n1, n2, n3, k, a);
        int rc = or_svd(a, n1, n2, 1, sg, u, v);
        if (rc < 0) {
#pragma omp atomic write
            status = 1;
        }
        put_slice(Ub, n1, n1, n3, k, u);
        put_slice(Vb, n2, n2, n3, k, v);
        for (int i = 0; i < p; ++i) Sb[idx3(i, i, k, n2, n3)] = sg[i];
        free(a);
        free(u);
        free(v);
        free(sg);
    }
    conj_fill(Ub, n1, n1, n3); /* step 2, second loop (S is real: conj is a copy) */
    conj_fill(Sb, n1, n2, n3);
    conj_fill(Vb, n2, n2, n3);
    double m1 = idft_real(Ub, n1, n1, n3, U); /* step 3 */
    double m2 = idft_real(Sb, n1, n2, n3, S);
    double m3 = idft_real(Vb, n2, n2, n3, V);
    if (maximag) *maximag = fmax(m1, fmax(m2, m3));
    free(Ab);
    free(Ub);
    free(Sb);
    free(Vb);
    return status;
}

int or_slice_sigma(const double* A, int n1, int n2, int n3, double* sig)
{
    const int p = n1 < n2 ? n1 : n2;
    or_cplx* za = real_to_complex(A, (i64)n1 * n2 * n3);
    or_cplx* Ab = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)n1 * n2 * n3);
    or_dft3(za, n1, n2, n3, 0, Ab);
    free(za);
    int status = 0;
#pragma omp parallel for schedule(dynamic)
    for (int k = 0; k < n3; ++k) {
        or_cplx* a = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)n1 * n2);
        get_slice(Ab, n1, n2, n3, k, a);
        if (or_svd(a, n1, n2, 0, sig + (i64)k * p, NULL, NULL) < 0) {
#pragma omp atomic write
            status = 1;
        }
        free(a);
    }
    free(Ab);
    return status;
}

/* Definition 2.9 with eq (14): sum_i S(i,i,1) = (1/n3) sum_k sum_i sigma_i(Abar^(k)) */
double or_tnn(const double* A, int n1, int n2, int n3)
{
    const int p = n1 < n2 ? n1 : n2;
    double* sig = (double*)xmalloc(sizeof(double) * (size_t)n3 * p);
    or_slice_sigma(A, n1, n2, n3, sig);
    double acc = 0.0;
    for (int k = 0; k < n3; ++k)
        for (int i = 0; i < p; ++i) acc += sig[(i64)k * p + i];
    free(sig);
    return acc / (double)n3;
}

/* Definition 2.8 with eq (17) */
double or_tsn(const double* A, int n1, int n2, int n3)
{
    const int p = n1 < n2 ? n1 : n2;
    double* sig = (double*)xmalloc(sizeof(double) * (size_t)n3 * p);
    or_slice_sigma(A, n1, n2, n3, sig);
    double mx = 0.0;
    for (int k = 0; k < n3; ++k) mx = fmax(mx, sig[(i64)k * p]);
    free(sig);
    return mx;
}

int or_tubalrank(const double* A, int n1, int n2, int n3, double tol, double eps)
{
    const int p = n1 < n2 ? n1 : n2;
    double* sig = (double*)xmalloc(sizeof(double) * (size_t)n3 * p);
    or_slice_sigma(A, n1, n2, n3, sig); /* each slice's values, decreasing */
    double s0 = 0.0;
    for (int k = 0; k < n3; ++k) s0 += sig[(i64)k * p];
    s0 /= n3;
    if (tol < 0.0) tol = (double)(n1 > n2 ? n1 : n2) * eps * s0;
    int rank = 0;
    for (int i = 0; i < p; ++i) {
        double si = 0.0;
        for (int k = 0; k < n3; ++k) si += sig[(i64)k * p + i];
        if (si / n3 > tol) ++rank;
    }
    free(sig);
    return rank;
}

/* U (S - tau)_+ V^* of a complex m x n matrix, written to out */
static int svt_complex(const or_cplx* a, int m, int n, double tau, or_cplx* out)
{
    const int p = m < n ? m : n;
    or_cplx* u = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)m * p);
    or_cplx* v = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)n * p);
    double* sg = (double*)xmalloc(sizeof(double) * (size_t)p);
    int rc = or_svd(a, m, n, 0, sg, u, v);
    for (i64 e = 0; e < (i64)m * n; ++e) out[e] = 0.0;
    for (int r = 0; r < p; ++r) {
        double d = sg[r] - tau;
        if (d <= 0.0) continue; /* t_+ = max(t, 0) */
        for (int i = 0; i < m; ++i) {
            or_cplx ui = d * u[(i64)i * p + r];
            for (int j = 0; j < n; ++j) out[(i64)i * n + j] += ui * conj(v[(i64)j * p + r]);
        }
    }
    free(u);
    free(v);
    free(sg);
    return rc < 0 ? 1 : 0;
}

/* Theorem 2.3 / Algorithm 3 (t-SVT) */
int or_prox_tnn(const double* Y, int n1, int n2, int n3, double tau, double* X)
{
    if (!(tau >= 0.0)) return -1;
    const int h = n3 / 2 + 1;
    or_cplx* zy = real_to_complex(Y, (i64)n1 * n2 * n3);
    or_cplx* Yb = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)n1 * n2 * n3);
    or_cplx* Wb = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)n1 * n2 * n3);
    or_dft3(zy, n1, n2, n3, 0, Yb); /* step 1 */
    free(zy);
    int status = 0;
#pragma omp parallel for schedule(dynamic)
    for (int k = 0; k < h; ++k) { /* step 2, first loop: matrix SVT of slice k */
        or_cplx* a = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)n1 * n2);
        or_cplx* w = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)n1 * n2);
        get_slice(Yb, n1, n2, n3, k, a);
        if (svt_complex(a, n1, n2, tau, w)) {
#pragma omp atomic write
            status = 1;
        }
        put_slice(Wb, n1, n2, n3, k, w);
        free(a);
        free(w);
    }
    conj_fill(Wb, n1, n2, n3);      /* step 2, second loop */
    idft_real(Wb, n1, n2, n3, X);   /* step 3 */
    free(Yb);
    free(Wb);
    return status;
}

int or_svt_real(const double* M, int m, int n, double tau, double* out)
{
    or_cplx* a = real_to_complex(M, (i64)m * n);
    or_cplx* w = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)m * n);
    int rc = svt_complex(a, m, n, tau, w);
    for (i64 e = 0; e < (i64)m * n; ++e) out[e] = creal(w[e]);
    free(a);
    free(w);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Tensor robust PCA by the inexact augmented Lagrangian method             */
/* ------------------------------------------------------------------------ */
/*
 * The problem the paper names as the use of the prox of Theorem 2.3:
 *   min ||L||_* + lam ||S||_1  s.t.  L + S = X   (||.||_* the TNN, Def 2.9).
 * The paper states no algorithm for it; this is the standard inexact ALM
 * (alternating minimisation of the augmented Lagrangian
 * ||L||_* + lam ||S||_1 + <Lam, L + S - X> + mu/2 ||L + S - X||_F^2, then a
 * multiplier step), with the stopping test and the relative tolerance the
 * GPU driver uses:
 *   L' = prox_tnn(X - S - Lam/mu, 1/mu)           (eq (19), Theorem 2.3)
 *   S' = soft(X - L' - Lam/mu, lam/mu)            (entrywise shrinkage)
 *   R  = L' + S' - X;  Lam <- Lam + mu R;  mu <- min(rho mu, mu_max)
 *   stop when max(max|L' - L|, max|S' - S|, max|R|) <= tol max(1, max|X|).
 * Returns 1 when the test was met within max_iter iterations, 0 otherwise,
 * negative on a bad argument; *iters receives the iterations run.
 */
int or_trpca(const double* X, int n1, int n2, int n3, double lam, double mu, double rho, double mu_max,
             double tol, int max_iter, double* L, double* S, double* Lam, int* iters)
{
    if (n1 < 1 || n2 < 1 || n3 < 1 || !(lam > 0.0) || !(mu > 0.0) || !(rho >= 1.0) || max_iter < 1) return -1;
    const i64 n = (i64)n1 * n2 * n3;
    double* Y = (double*)xmalloc((size_t)n * sizeof(double));
    double* Ln = (double*)xmalloc((size_t)n * sizeof(double));
    double scale = 1.0;
    for (i64 e = 0; e < n; ++e) {
        L[e] = S[e] = Lam[e] = 0.0;
        if (fabs(X[e]) > scale) scale = fabs(X[e]);
    }
    int converged = 0, it = 0;
    while (it < max_iter && !converged) {
        ++it;
        for (i64 e = 0; e < n; ++e) Y[e] = X[e] - S[e] - Lam[e] / mu;
        or_prox_tnn(Y, n1, n2, n3, 1.0 / mu, Ln);
        double dl = 0.0, ds = 0.0, dr = 0.0;
        const double thr = lam / mu;
        for (i64 e = 0; e < n; ++e) {
            const double r = X[e] - Ln[e] - Lam[e] / mu;
            const double sn = r > thr ? r - thr : (r < -thr ? r + thr : 0.0);
            const double res = Ln[e] + sn - X[e];
            dl = fmax(dl, fabs(Ln[e] - L[e]));
            ds = fmax(ds, fabs(sn - S[e]));
            dr = fmax(dr, fabs(res));
            Lam[e] += mu * res;
            L[e] = Ln[e];
            S[e] = sn;
        }
        mu = fmin(rho * mu, mu_max);
        converged = fmax(dl, fmax(ds, dr)) <= tol * scale;
    }
    free(Y);
    free(Ln);
    if (iters) *iters = it;
    return converged;
}

/* ------------------------------------------------------------------------ */
/* Tensor QR (Theorem 2.4) and tensor inverse (Definition 2.4)              */
/* ------------------------------------------------------------------------ */
/*
 * Householder QR of the m x n complex matrix a (FP64): a = q r with q m x m
 * unitary and r m x n upper trapezoidal.  Reflector j makes column j zero
 * below row j: H = I - 2 v v^* / (v^* v) with v = x + phi |x| e_1, x the part
 * of column j from row j down and phi the phase of x_0 (so no cancellation),
 * giving H x = -phi |x| e_1.  q = H_0 H_1 ... H_{k-1} is formed by applying
 * the reflectors to the identity in reverse order.  Finally row i of r and
 * column i of q are rephased so that r(i,i) is real and >= 0, which makes the
 * factorisation unique for full-rank matrices (up to the complement columns
 * of q when m > n).  On real data every step stays real.
 */
static void qr_householder(const or_cplx* a, int m, int n, or_cplx* q, or_cplx* r)
{
    const int k = m < n ? m : n;
    or_cplx* w = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)m * n);
    or_cplx* v = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)m * (k > 0 ? k : 1));
    double* beta = (double*)xmalloc(sizeof(double) * (size_t)(k > 0 ? k : 1));
    memcpy(w, a, sizeof(or_cplx) * (size_t)m * n);
    for (int j = 0; j < k; ++j) {
        double s2 = 0.0;
        for (int i = j; i < m; ++i) s2 += abs2(w[(i64)i * n + j]);
        for (int i = 0; i < m; ++i) v[(i64)i * k + j] = 0.0;
        if (s2 == 0.0) {
            beta[j] = 0.0;
            continue;
        }
        const double s = sqrt(s2);
        const or_cplx alpha = w[(i64)j * n + j];
        const double aa = cabs(alpha);
        const or_cplx phi = aa > 0.0 ? alpha / aa : 1.0;
        double vv = 0.0;
        for (int i = j; i < m; ++i) {
            const or_cplx vi = (i == j) ? alpha + phi * s : w[(i64)i * n + j];
            v[(i64)i * k + j] = vi;
            vv += abs2(vi);
        }
        beta[j] = 2.0 / vv;
        for (int c = j; c < n; ++c) { /* column c <- H column c */
            or_cplx t = 0.0;
            for (int i = j; i < m; ++i) t += conj(v[(i64)i * k + j]) * w[(i64)i * n + c];
            t *= beta[j];
            for (int i = j; i < m; ++i) w[(i64)i * n + c] -= v[(i64)i * k + j] * t;
        }
    }
    for (int i = 0; i < m; ++i)
        for (int c = 0; c < m; ++c) q[(i64)i * m + c] = (i == c) ? 1.0 : 0.0;
    for (int j = k - 1; j >= 0; --j) {
        if (beta[j] == 0.0) continue;
        for (int c = j; c < m; ++c) {
            or_cplx t = 0.0;
            for (int i = j; i < m; ++i) t += conj(v[(i64)i * k + j]) * q[(i64)i * m + c];
            t *= beta[j];
            for (int i = j; i < m; ++i) q[(i64)i * m + c] -= v[(i64)i * k + j] * t;
        }
    }
    for (int i = 0; i < m; ++i)
        for (int c = 0; c < n; ++c) r[(i64)i * n + c] = (c >= i) ? w[(i64)i * n + c] : 0.0;
    for (int i = 0; i < k; ++i) { /* r(i,i) real >= 0 */
        const or_cplx d = r[(i64)i * n + i];
        const double ad = cabs(d);
        if (ad == 0.0) continue;
        const or_cplx ph = conj(d) / ad;
        for (int c = i; c < n; ++c) r[(i64)i * n + c] *= ph;
        r[(i64)i * n + i] = ad;
        for (int row = 0; row < m; ++row) q[(i64)row * m + i] *= conj(ph);
    }
    free(w);
    free(v);
    free(beta);
}

/* Theorem 2.4: A = Q * R with Q (n1 x n1 x n3) orthogonal and R (n1 x n2 x n3)
 * f-upper triangular, by the pipeline of Algorithm 2 with a QR per Fourier
 * slice (k < h; the rest by conjugate symmetry). */
int or_tqr(const double* A, int n1, int n2, int n3, double* Q, double* R)
{
    if (n1 < 1 || n2 < 1 || n3 < 1) return -1;
    const int h = n3 / 2 + 1;
    or_cplx* za = real_to_complex(A, (i64)n1 * n2 * n3);
    or_cplx* Ab = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)n1 * n2 * n3);
    or_dft3(za, n1, n2, n3, 0, Ab);
    free(za);
    or_cplx* Qb = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)n1 * n1 * n3);
    or_cplx* Rb = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)n1 * n2 * n3);
#pragma omp parallel for schedule(dynamic)
    for (int k = 0; k < h; ++k) {
        or_cplx* a = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)n1 * n2);
        or_cplx* q = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)n1 * n1);
        or_cplx* r = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)n1 * n2);
        get_slice(Ab, n1, n2, n3, k, a);
        qr_householder(a, n1, n2, q, r);
        put_slice(Qb, n1, n1, n3, k, q);
        put_slice(Rb, n1, n2, n3, k, r);
        free(a);
        free(q);
        free(r);
    }
    conj_fill(Qb, n1, n1, n3);
    conj_fill(Rb, n1, n2, n3);
    idft_real(Qb, n1, n1, n3, Q);
    idft_real(Rb, n1, n2, n3, R);
    free(Ab);
    free(Qb);
    free(Rb);
    return 0;
}

/* Inverse of the n x n complex matrix a by Gauss-Jordan elimination with
 * partial pivoting (largest modulus, first on ties) on [a | I].  Returns 0,
 * or j + 1 when the pivot of step j is zero (singular). */
static int inv_gauss_jordan(const or_cplx* a, int n, or_cplx* out)
{
    const int w2 = 2 * n;
    or_cplx* w = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)n * w2);
    for (int i = 0; i < n; ++i)
        for (int c = 0; c < w2; ++c) w[(i64)i * w2 + c] = c < n ? a[(i64)i * n + c] : (c - n == i ? 1.0 : 0.0);
    int rc = 0;
    for (int j = 0; j < n && !rc; ++j) {
        int p = j;
        double best = cabs(w[(i64)j * w2 + j]);
        for (int i = j + 1; i < n; ++i) {
            const double t = cabs(w[(i64)i * w2 + j]);
            if (t > best) {
                best = t;
                p = i;
            }
        }
        if (best == 0.0) {
            rc = j + 1;
            break;
        }
        if (p != j)
            for (int c = 0; c < w2; ++c) {
                const or_cplx t = w[(i64)j * w2 + c];
                w[(i64)j * w2 + c] = w[(i64)p * w2 + c];
                w[(i64)p * w2 + c] = t;
            }
        const or_cplx piv = w[(i64)j * w2 + j];
        for (int c = 0; c < w2; ++c) w[(i64)j * w2 + c] /= piv;
        for (int i = 0; i < n; ++i) {
            if (i == j) continue;
            const or_cplx f = w[(i64)i * w2 + j];
            if (f == 0.0) continue;
            for (int c = 0; c < w2; ++c) w[(i64)i * w2 + c] -= f * w[(i64)j * w2 + c];
        }
    }
    for (int i = 0; i < n; ++i)
        for (int c = 0; c < n; ++c) out[(i64)i * n + c] = w[(i64)i * w2 + n + c];
    free(w);
    return rc;
}

/* Definition 2.4: B with A * B = B * A = I, slice by slice in the Fourier
 * domain (the Fourier slices of I are identities).  Returns 0, or 1 + the
 * first Fourier slice (k < h) that is singular (B then undefined). */
int or_tinv(const double* A, int n, int n3, double* B)
{
    if (n < 1 || n3 < 1) return -1;
    const int h = n3 / 2 + 1;
    or_cplx* za = real_to_complex(A, (i64)n * n * n3);
    or_cplx* Ab = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)n * n * n3);
    or_dft3(za, n, n, n3, 0, Ab);
    free(za);
    or_cplx* Bb = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)n * n * n3);
    int bad = 0;
    for (int k = 0; k < h; ++k) {
        or_cplx* a = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)n * n);
        or_cplx* b = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)n * n);
        get_slice(Ab, n, n, n3, k, a);
        if (inv_gauss_jordan(a, n, b) && !bad) bad = k + 1;
        put_slice(Bb, n, n, n3, k, b);
        free(a);
        free(b);
    }
    conj_fill(Bb, n, n, n3);
    idft_real(Bb, n, n, n3, B);
    free(Ab);
    free(Bb);
    return bad;
}
