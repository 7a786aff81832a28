/*
 * tp_oracle_learned.c -- FP64 CPU oracle of the learned-rank prox: the
 * counter-based sketch, CholeskyQR2, the randomized SVT of each Fourier slice
 * with its check and fallback, and the rank-predicting MLP with its gradient.
 *
 * TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU baseline of the
 * benchmark); it shares no code with the GPU library.
 *
 * The randomized range finder follows Halko, Martinsson and Tropp (2011,
 * "Finding structure with randomness", Algorithms 4.3/4.4 with
 * re-orthonormalisation after every product); CholeskyQR2 follows
 * Fukaya et al. (2014); Philox4x32-10 follows Salmon et al. (SC'11).  The
 * exact prox it approximates is Theorem 2.3 / Algorithm 3 of the paper.
 */
#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "tp_oracle.h"

typedef long long i64;

static void* xmalloc(size_t bytes)
{
    void* p = malloc(bytes ? bytes : 1);
    if (!p) abort();
    return p;
}

/* ------------------------------------------------------------- Philox -- */
void or_philox4x32_10(const unsigned int ctr[4], const unsigned int key[2], unsigned int out[4])
{
    const unsigned int M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    unsigned int c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3], k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += W0;
            k1 += W1;
        }
        const unsigned long long p0 = (unsigned long long)M0 * c0;
        const unsigned long long p1 = (unsigned long long)M1 * c2;
        const unsigned int hi0 = (unsigned int)(p0 >> 32), lo0 = (unsigned int)p0;
        const unsigned int hi1 = (unsigned int)(p1 >> 32), lo1 = (unsigned int)p1;
        const unsigned int n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

void or_sketch_matrix(int n, int l, int slice, int real, unsigned long long seed, or_cplx* Om)
{
    const unsigned int key[2] = {(unsigned int)seed, (unsigned int)(seed >> 32)};
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < l; ++j) {
            const unsigned int ctr[4] = {(unsigned int)i, (unsigned int)j, (unsigned int)slice, 0u};
            unsigned int x[4];
            or_philox4x32_10(ctr, key, x);
            const double u0 = ((double)x[0] + 0.5) * 0x1p-32, u1 = ((double)x[1] + 0.5) * 0x1p-32;
            const double rad = sqrt(-2.0 * log(u0));
            const double z0 = rad * cos(2.0 * M_PI * u1), z1 = rad * sin(2.0 * M_PI * u1);
            if (real)
                Om[(i64)i * l + j] = (double)(float)z0;
            else
                Om[(i64)i * l + j] = (double)(float)(z0 * M_SQRT1_2) + I * (double)(float)(z1 * M_SQRT1_2);
        }
}

/* -------------------------------------------------------- CholeskyQR2 -- */
int or_cholqr2(or_cplx* Y, int m, int l, int lact, or_cplx* R)
{
    or_cplx* G = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)l * l);
    or_cplx* R1 = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)l * l);
    or_cplx* T = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)l * l);
    for (int i = 0; i < l * l; ++i) R[i] = (i / l == i % l) ? 1.0 : 0.0;
    int status = 0;
    for (int pass = 0; pass < 2 && lact > 0; ++pass) {
        /* G = Y^* Y on the active columns; the first pass adds a small
         * diagonal shift (the second Gram is close to the identity) */
        double tr = 0.0;
        for (int a = 0; a < lact; ++a)
            for (int b = 0; b < lact; ++b) {
                or_cplx s = 0.0;
                for (int i = 0; i < m; ++i) s += conj(Y[(i64)i * l + a]) * Y[(i64)i * l + b];
                G[a * l + b] = s;
            }
        for (int a = 0; a < lact; ++a) tr += creal(G[a * l + a]);
        const double shift = pass == 0 ? 1e-13 * tr / lact : 0.0;
        for (int a = 0; a < lact; ++a) G[a * l + a] += shift;
        /* G = R1^* R1, R1 upper triangular with a positive diagonal */
        for (int i = 0; i < l * l; ++i) R1[i] = (i / l == i % l) ? 1.0 : 0.0;
        for (int j = 0; j < lact; ++j) {
            double d = creal(G[j * l + j]);
            for (int k = 0; k < j; ++k) d -= creal(R1[k * l + j]) * creal(R1[k * l + j]) + cimag(R1[k * l + j]) * cimag(R1[k * l + j]);
            if (!(d > 0.0)) {
                status = -1;
                d = DBL_MIN;
            }
            const double rjj = sqrt(d);
            R1[j * l + j] = rjj;
            for (int c = j + 1; c < lact; ++c) {
                or_cplx s = G[j * l + c];
                for (int k = 0; k < j; ++k) s -= conj(R1[k * l + j]) * R1[k * l + c];
                R1[j * l + c] = s / rjj;
            }
        }
        /* Y <- Y R1^{-1}: each row solves x R1 = y */
        for (int i = 0; i < m; ++i) {
            or_cplx* y = Y + (i64)i * l;
            for (int j = 0; j < lact; ++j) {
                or_cplx s = y[j];
                for (int k = 0; k < j; ++k) s -= y[k] * R1[k * l + j];
                y[j] = s / R1[j * l + j];
            }
        }
        /* R <- R1 R */
        for (int a = 0; a < l; ++a)
            for (int b = 0; b < l; ++b) {
                or_cplx s = 0.0;
                for (int k = 0; k < l; ++k) s += R1[a * l + k] * R[k * l + b];
                T[a * l + b] = s;
            }
        memcpy(R, T, sizeof(or_cplx) * (size_t)l * l);
    }
    free(G);
    free(R1);
    free(T);
    return status;
}

/* ------------------------------------------------ randomized slice SVT -- */
static void get_slice(const or_cplx* X, int n1, int n2, int n3, int k, or_cplx* M)
{
    for (int i = 0; i < n1; ++i)
        for (int j = 0; j < n2; ++j) M[(i64)i * n2 + j] = X[((i64)i * n2 + j) * n3 + k];
}

static void put_slice(or_cplx* X, int n1, int n2, int n3, int k, const or_cplx* M)
{
    for (int i = 0; i < n1; ++i)
        for (int j = 0; j < n2; ++j) X[((i64)i * n2 + j) * n3 + k] = M[(i64)i * n2 + j];
}

/* C (m x p) = op(A) op(B); opa/opb: 0 plain, 1 conjugate transpose; A is
 * stored with `lda` columns, B with `ldb` columns (row-major). */
static void cmatmul(const or_cplx* A, int lda, int opa, const or_cplx* B, int ldb, int opb, int m, int k, int p,
                    or_cplx* C)
{
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < p; ++j) {
            or_cplx s = 0.0;
            for (int t = 0; t < k; ++t) {
                const or_cplx a = opa ? conj(A[(i64)t * lda + i]) : A[(i64)i * lda + t];
                const or_cplx b = opb ? conj(B[(i64)j * ldb + t]) : B[(i64)t * ldb + j];
                s += a * b;
            }
            C[(i64)i * p + j] = s;
        }
}

/* exact matrix SVT U (S - tau)_+ V^* of slice a (m x n) */
static int svt_full(const or_cplx* a, int m, int n, double tau, or_cplx* w, int* rank)
{
    const int p = m < n ? m : n;
    or_cplx* u = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)m * p);
    or_cplx* v = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)n * p);
    double* sg = (double*)xmalloc(sizeof(double) * (size_t)p);
    int rc = or_svd(a, m, n, 0, sg, u, v);
    int kk = 0;
    for (i64 e = 0; e < (i64)m * n; ++e) w[e] = 0.0;
    for (int r = 0; r < p; ++r) {
        const double d = sg[r] - tau;
        if (d <= 0.0) continue;
        ++kk;
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < n; ++j) w[(i64)i * n + j] += d * u[(i64)i * p + r] * conj(v[(i64)j * p + r]);
    }
    if (rank) *rank = kk;
    free(u);
    free(v);
    free(sg);
    return rc < 0 ? 1 : 0;
}

int or_prox_tnn_rsvd(const double* Y, int n1, int n2, int n3, double tau, const int* kpred, int oversample,
                     int power, int lfull, unsigned long long seed, double* X, int* fallback, int* rank)
{
    if (!(tau >= 0.0)) return -1;
    const int h = n3 / 2 + 1, m = n1, n = n2, p = n1 < n2 ? n1 : n2;
    const i64 tot = (i64)n1 * n2 * n3;
    or_cplx* zy = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)tot);
    or_cplx* Yb = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)tot);
    or_cplx* Wb = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)tot);
    for (i64 e = 0; e < tot; ++e) zy[e] = Y[e];
    or_dft3(zy, n1, n2, n3, 0, Yb);
    int status = 0;
#pragma omp parallel for schedule(dynamic)
    for (int k = 0; k < h; ++k) {
        const int real = (k == 0) || (n3 % 2 == 0 && k == n3 / 2);
        or_cplx* a = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)m * n);
        or_cplx* w = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)m * n);
        get_slice(Yb, n1, n2, n3, k, a);
        int l = kpred[k] + oversample;
        if (l > p) l = p;
        int fb = (l >= lfull) ? 1 : 0, kk = 0;
        for (i64 e = 0; e < (i64)m * n; ++e) w[e] = 0.0;
        if (!fb && l > 0) {
            or_cplx* Om = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)n * l);
            or_cplx* Qm = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)m * l);
            or_cplx* Zn = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)n * l);
            or_cplx* Rt = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)l * l);
            or_cplx* Mr = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)l * l);
            or_cplx* Ur = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)l * l);
            or_cplx* Vr = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)l * l);
            or_cplx* T = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)l * l);
            or_cplx* TQ = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)l * n);
            double* s = (double*)xmalloc(sizeof(double) * (size_t)l);
            or_sketch_matrix(n, l, k, real, seed, Om);
            cmatmul(a, n, 0, Om, l, 0, m, n, l, Qm); /* Y = Abar Om */
            or_cholqr2(Qm, m, l, l, Rt);
            for (int it = 0; it < power; ++it) {
                cmatmul(a, n, 1, Qm, l, 0, n, m, l, Zn); /* Z = Abar^* Q */
                or_cholqr2(Zn, n, l, l, Rt);
                cmatmul(a, n, 0, Zn, l, 0, m, n, l, Qm); /* Y = Abar Z */
                or_cholqr2(Qm, m, l, l, Rt);
            }
            cmatmul(a, n, 1, Qm, l, 0, n, m, l, Zn); /* Bh = Abar^* Q = B^* */
            or_cholqr2(Zn, n, l, l, Rt);              /* Bh = Q2 R2 */
            for (int i = 0; i < l; ++i)               /* M = R2^* */
                for (int j = 0; j < l; ++j) Mr[i * l + j] = conj(Rt[j * l + i]);
            or_svd(Mr, l, l, 0, s, Ur, Vr);
            const int kp = kpred[k];
            if (kp < l && s[kp] >= tau) fb = 1; /* check sigma_(k+1) < tau */
            if (!fb) {
                for (int i = 0; i < l; ++i)
                    for (int j = 0; j < l; ++j) {
                        or_cplx t = 0.0;
                        for (int r = 0; r < l; ++r) {
                            const double d = s[r] - tau;
                            if (d > 0.0) t += Ur[i * l + r] * d * conj(Vr[j * l + r]);
                        }
                        T[i * l + j] = t;
                    }
                for (int r = 0; r < l; ++r) kk += s[r] > tau ? 1 : 0;
                cmatmul(T, l, 0, Zn, l, 1, l, l, n, TQ); /* T Q2^* */
                cmatmul(Qm, l, 0, TQ, n, 0, m, l, n, w); /* W = Q T Q2^* */
            }
            free(Om);
            free(Qm);
            free(Zn);
            free(Rt);
            free(Mr);
            free(Ur);
            free(Vr);
            free(T);
            free(TQ);
            free(s);
        }
        if (fb) {
            if (svt_full(a, m, n, tau, w, &kk)) {
#pragma omp atomic write
                status = 1;
            }
        }
        if (fallback) fallback[k] = fb;
        if (rank) rank[k] = kk;
        put_slice(Wb, n1, n2, n3, k, w);
        free(a);
        free(w);
    }
    for (int k = h; k < n3; ++k) /* conjugate fill */
        for (int i = 0; i < n1; ++i)
            for (int j = 0; j < n2; ++j) Wb[((i64)i * n2 + j) * n3 + k] = conj(Wb[((i64)i * n2 + j) * n3 + (n3 - k)]);
    or_dft3(Wb, n1, n2, n3, 1, zy);
    for (i64 e = 0; e < tot; ++e) X[e] = creal(zy[e]);
    free(zy);
    free(Yb);
    free(Wb);
    return status;
}

/* ---------------------------------------------------------------- MLP -- */
int or_mlp_param_count(int d, int h) { return h * d + h + 2 * (h * h + h) + h + 1; }

typedef struct {
    const double *W1, *b1, *W2, *b2, *W3, *b3, *w4, *b4;
} mlp_view;

static mlp_view mlp_unpack(const double* p, int d, int h)
{
    mlp_view v;
    v.W1 = p;
    v.b1 = v.W1 + h * d;
    v.W2 = v.b1 + h;
    v.b2 = v.W2 + h * h;
    v.W3 = v.b2 + h;
    v.b3 = v.W3 + h * h;
    v.w4 = v.b3 + h;
    v.b4 = v.w4 + h;
    return v;
}

/* one sample: activations z1..z3 (pre-ReLU) and the output */
static double mlp_sample(const mlp_view* v, int d, int h, const double* x, double* z1, double* z2, double* z3)
{
    for (int i = 0; i < h; ++i) {
        double s = v->b1[i];
        for (int j = 0; j < d; ++j) s += v->W1[i * d + j] * x[j];
        z1[i] = s;
    }
    for (int i = 0; i < h; ++i) {
        double s = v->b2[i];
        for (int j = 0; j < h; ++j) s += v->W2[i * h + j] * fmax(z1[j], 0.0);
        z2[i] = s;
    }
    for (int i = 0; i < h; ++i) {
        double s = v->b3[i];
        for (int j = 0; j < h; ++j) s += v->W3[i * h + j] * fmax(z2[j], 0.0);
        z3[i] = s;
    }
    double y = v->b4[0];
    for (int j = 0; j < h; ++j) y += v->w4[j] * fmax(z3[j], 0.0);
    return y;
}

void or_mlp_forward(const double* params, int d, int h, const double* X, int N, double* y)
{
    mlp_view v = mlp_unpack(params, d, h);
    double* z = (double*)xmalloc(sizeof(double) * 3 * (size_t)h);
    for (int s = 0; s < N; ++s) y[s] = mlp_sample(&v, d, h, X + (i64)s * d, z, z + h, z + 2 * h);
    free(z);
}

double or_mlp_loss_grad(const double* params, int d, int h, const double* X, const double* t, int N,
                        double under, double* grad)
{
    const int np = or_mlp_param_count(d, h);
    mlp_view v = mlp_unpack(params, d, h);
    /* gradient pointers in the same packing */
    double* gW1 = grad;
    double* gb1 = gW1 + h * d;
    double* gW2 = gb1 + h;
    double* gb2 = gW2 + h * h;
    double* gW3 = gb2 + h;
    double* gb3 = gW3 + h * h;
    double* gw4 = gb3 + h;
    double* gb4 = gw4 + h;
    for (int i = 0; i < np; ++i) grad[i] = 0.0;
    double* z = (double*)xmalloc(sizeof(double) * 6 * (size_t)h);
    double *z1 = z, *z2 = z + h, *z3 = z + 2 * h, *d1 = z + 3 * h, *d2 = z + 4 * h, *d3 = z + 5 * h;
    double loss = 0.0;
    for (int s = 0; s < N; ++s) {
        const double* x = X + (i64)s * d;
        const double y = mlp_sample(&v, d, h, x, z1, z2, z3);
        const double e = y - t[s];
        const double c = e >= 0.0 ? 1.0 : under;
        loss += c * e * e;
        const double dy = 2.0 * c * e / N;
        gb4[0] += dy;
        for (int j = 0; j < h; ++j) {
            gw4[j] += dy * fmax(z3[j], 0.0);
            d3[j] = z3[j] > 0.0 ? dy * v.w4[j] : 0.0;
        }
        for (int i = 0; i < h; ++i) {
            gb3[i] += d3[i];
            for (int j = 0; j < h; ++j) gW3[i * h + j] += d3[i] * fmax(z2[j], 0.0);
        }
        for (int j = 0; j < h; ++j) {
            double s2 = 0.0;
            for (int i = 0; i < h; ++i) s2 += v.W3[i * h + j] * d3[i];
            d2[j] = z2[j] > 0.0 ? s2 : 0.0;
        }
        for (int i = 0; i < h; ++i) {
            gb2[i] += d2[i];
            for (int j = 0; j < h; ++j) gW2[i * h + j] += d2[i] * fmax(z1[j], 0.0);
        }
        for (int j = 0; j < h; ++j) {
            double s1 = 0.0;
            for (int i = 0; i < h; ++i) s1 += v.W2[i * h + j] * d2[i];
            d1[j] = z1[j] > 0.0 ? s1 : 0.0;
        }
        for (int i = 0; i < h; ++i) {
            gb1[i] += d1[i];
            for (int j = 0; j < d; ++j) gW1[i * d + j] += d1[i] * x[j];
        }
    }
    free(z);
    return loss / N;
}

/* ---------------------------------------------------------- features -- */
void or_slice_features(const double* Y, int n1, int n2, int n3, double tau, const int* prev, const double* psig,
                       double* feats)
{
    const int h = n3 / 2 + 1, p = n1 < n2 ? n1 : n2;
    const i64 tot = (i64)n1 * n2 * n3;
    or_cplx* zy = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)tot);
    or_cplx* Yb = (or_cplx*)xmalloc(sizeof(or_cplx) * (size_t)tot);
    for (i64 e = 0; e < tot; ++e) zy[e] = Y[e];
    or_dft3(zy, n1, n2, n3, 0, Yb);
    for (int k = 0; k < h; ++k) {
        double nrm2 = 0.0, cmax = 0.0;
        for (int j = 0; j < n2; ++j) {
            double c = 0.0;
            for (int i = 0; i < n1; ++i) {
                const or_cplx v = Yb[((i64)i * n2 + j) * n3 + k];
                c += creal(v) * creal(v) + cimag(v) * cimag(v);
            }
            nrm2 += c;
            cmax = fmax(cmax, c);
        }
        const double t2 = tau * tau;
        double* f = feats + (i64)k * 12;
        /* log(tau / rms sigma): +30 for a zero slice, -30 for tau = 0 (the clamped limits) */
        f[0] = nrm2 > 0.0 ? (t2 > 0.0 ? fmin(30.0, fmax(-30.0, 0.5 * log(t2 * p / nrm2))) : -30.0) : 30.0;
        f[1] = (cmax > 0.0 && t2 > 0.0) ? fmin(30.0, fmax(-30.0, 0.5 * log(cmax / t2))) : (cmax > 0.0 ? 30.0 : -30.0);
        f[2] = prev ? (double)prev[k] / p : 0.0;
        f[3] = prev ? 1.0 : 0.0;
        f[4] = n3 > 1 ? (double)k / (double)(n3 / 2 > 0 ? n3 / 2 : 1) : 0.0;
        f[5] = (k == 0 || (n3 % 2 == 0 && k == n3 / 2)) ? 1.0 : 0.0;
        f[6] = log((double)p) / 8.0;
        f[7] = log((double)(n1 > n2 ? n1 : n2) / (double)p);
        f[8] = f[9] = f[10] = f[11] = 0.0;
        if (psig) { /* previous leading singular values, 64 per slice, decreasing, zero-padded */
            const double* sv = psig + (i64)k * 64;
            int a = 0, b = 0, c = 0;
            for (int j = 0; j < 64; ++j) {
                c += sv[j] > 0.0 ? 1 : 0;
                a += sv[j] > tau ? 1 : 0;
                b += sv[j] > tau / 1.25 ? 1 : 0;
            }
            f[8] = (double)a / p;
            f[9] = (double)b / p;
            f[10] = (sv[0] > 0.0 && tau > 0.0) ? fmin(30.0, fmax(-30.0, log(sv[0] / tau))) : (sv[0] > 0.0 ? 30.0 : -30.0);
            f[11] = (c > 0 && sv[c - 1] > tau) ? 1.0 : 0.0;
        }
    }
    free(zy);
    free(Yb);
}
