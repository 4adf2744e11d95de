/*
 * Direct nonuniform discrete Fourier transforms in FP64 -- the oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may include,
 * link or call this file; it shares no code with the GPU path.  It is
 * compiled with gcc into a host shared library and driven from tests/,
 * from the smoke check and from the CPU baseline leg of the benchmark.
 *
 * Every routine here is the plain O(N*M) definition of a transform from
 * Ruiz-Antolin & Townsend, "A nonuniform fast Fourier transform based on low
 * rank approximation":
 *   type II   f_j = sum_k c_k exp(-2 pi i x_j k)           (Sec. 1, eq. (2))
 *   type I    f_k = sum_j c_j exp(-2 pi i x_j k)           (Sec. 3.1, transpose of II)
 *   adjoint   f_k = sum_j c_j exp(+2 pi i x_j k)           (conjugate transpose of II)
 *   type III  f_j = sum_k c_k exp(-2 pi i x_j w_k)          (Sec. 3.2)
 *   2-D II    f_j = sum_{k1,k2} C_{k1 k2} exp(-2 pi i (k1 x_j + k2 y_j))  (Sec. 4, first display)
 *   3-D II, I and adjoint: the same with a third axis (k3, z_j)
 * and the nearest-grid assignment of Sec. 2.2 (s = round(N x), t = s mod N).
 *
 * Two things keep the sums accurate to a few units in the last place:
 *  1. The phase a*b is split exactly as p + e with p = fl(a*b) and
 *     e = fma(a, b, -p) (TwoProduct, Dekker 1971), and reduced modulo 1 as
 *     (p - floor(p)) + e, whose first part is exact.  A plain fl(x*k) at
 *     k ~ 2^20 carries ~1e-10 of absolute phase error, far above eps=1e-12.
 *  2. exp(2 pi i phi) is evaluated after an exact quarter-turn reduction, so
 *     phases that are multiples of 1/4 give exactly 0 and +-1, and the
 *     complex products are accumulated with the compensated dot product Dot2
 *     (Ogita, Rump & Oishi 2005: TwoProduct + TwoSum per term).
 * Rows are independent and each row is summed in index order, so results are
 * deterministic regardless of the OpenMP thread count.
 *
 * Complex arrays are interleaved (re, im) doubles.  Build with
 *   gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC
 * (contraction must stay off: TwoSum/TwoProduct rely on each operation
 * being rounded on its own).
 */
#include <math.h>
#include <stdint.h>
#include <omp.h>

#define TWO_PI 6.283185307179586476925286766559

/* ---- error-free transformations ---------------------------------------- */

static inline void two_sum(double a, double b, double *s, double *e)
{
    double x = a + b;
    double z = x - a;
    *e = (a - (x - z)) + (b - z);
    *s = x;
}

static inline void two_prod(double a, double b, double *p, double *e)
{
    double x = a * b;
    *e = fma(a, b, -x);
    *p = x;
}

/* Dot2 accumulator: value = s + t. */
typedef struct { double s, t; } acc2;

static inline void acc2_add_prod(acc2 *a, double x, double y)
{
    double h, r, q;
    two_prod(x, y, &h, &r);
    two_sum(a->s, h, &a->s, &q);
    a->t += q + r;
}

/* Exact reduction of a*b modulo 1 into [-1/2, 1/2] (one final rounding). */
static inline double phase_mod1(double a, double b)
{
    double p, e;
    two_prod(a, b, &p, &e);
    double fr = p - floor(p);          /* exact */
    double phi = fr + e;               /* one rounding, |phi| < 2 */
    return phi - nearbyint(phi);       /* exact */
}

/* (cos, sin) of 2*pi*phi for |phi| <= 1: quarter turns are taken out
 * exactly, the remainder |rho| <= 1/8 goes to libm. */
static inline void cis2pi(double phi, double *co, double *si)
{
    double q = nearbyint(4.0 * phi);   /* 4*phi exact */
    double rho = phi - 0.25 * q;       /* exact */
    double c0, s0;
    if (rho == 0.0) { c0 = 1.0; s0 = 0.0; }
    else { double th = TWO_PI * rho; c0 = cos(th); s0 = sin(th); }
    int iq = ((int)q) & 3;
    switch (iq) {
    case 0: *co = c0;  *si = s0;  break;
    case 1: *co = -s0; *si = c0;  break;   /* times i  */
    case 2: *co = -c0; *si = -s0; break;   /* times -1 */
    default: *co = s0; *si = -c0; break;   /* times -i */
    }
}

/* out = sum_i c_i * exp(sign * 2 pi i * phi_i), phi_i = a * b_i (mod 1). */
static void phase_sum(double a, int64_t n, const double *b, const double *c,
                      int sign, double *out)
{
    acc2 re = {0.0, 0.0}, im = {0.0, 0.0};
    for (int64_t i = 0; i < n; ++i) {
        double co, si;
        cis2pi(phase_mod1(a, b[i]), &co, &si);
        if (sign < 0) si = -si;
        double cr = c[2 * i], ci = c[2 * i + 1];
        acc2_add_prod(&re, cr, co);
        acc2_add_prod(&re, -ci, si);
        acc2_add_prod(&im, cr, si);
        acc2_add_prod(&im, ci, co);
    }
    out[0] = re.s + re.t;
    out[1] = im.s + im.t;
}

/* ---- exported transforms ------------------------------------------------ */

void oracle_set_threads(int n) { if (n > 0) omp_set_num_threads(n); }
int oracle_max_threads(void) { return omp_get_max_threads(); }

/* Type II (Sec. 1, eq. (2)): f_j = sum_{k<N} c_k exp(-2 pi i x_j k), j < M. */
int oracle_nudft2(int64_t N, const double *c, int64_t M, const double *x, double *f)
{
    if (N < 0 || M < 0) return -1;
    /* k is an integer below 2^53, so (double)k is exact */
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j < M; ++j) {
        acc2 re = {0.0, 0.0}, im = {0.0, 0.0};
        for (int64_t k = 0; k < N; ++k) {
            double co, si;
            cis2pi(phase_mod1(x[j], (double)k), &co, &si);
            si = -si;
            double cr = c[2 * k], ci = c[2 * k + 1];
            acc2_add_prod(&re, cr, co);
            acc2_add_prod(&re, -ci, si);
            acc2_add_prod(&im, cr, si);
            acc2_add_prod(&im, ci, co);
        }
        f[2 * j] = re.s + re.t;
        f[2 * j + 1] = im.s + im.t;
    }
    return 0;
}

/* Type I (Sec. 3.1) and the adjoint of type II:
 *   f_k = sum_{j<M} c_j exp(sign * 2 pi i x_j k) for each requested k.
 * sign = -1 is the paper's type I (the transpose of type II),
 * sign = +1 is the conjugate transpose (adjoint) of type II. */
int oracle_nudft1(int64_t M, const double *x, const double *c, int64_t nk,
                  const int64_t *k, int sign, double *f)
{
    if (M < 0 || nk < 0 || (sign != 1 && sign != -1)) return -1;
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < nk; ++q)
        phase_sum((double)k[q], M, x, c, sign, f + 2 * q);
    return 0;
}

/* Type III (Sec. 3.2): f_j = sum_{k<N} c_k exp(-2 pi i x_j w_k). */
int oracle_nudft3(int64_t N, const double *w, const double *c, int64_t M,
                  const double *x, double *f)
{
    if (N < 0 || M < 0) return -1;
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j < M; ++j)
        phase_sum(x[j], N, w, c, -1, f + 2 * j);
    return 0;
}

/* 2-D type II (Sec. 4): f_j = sum_{k1<N1, k2<N2} C[k1*N2+k2] exp(-2 pi i (k1 x_j + k2 y_j)).
 * The two phases are reduced modulo 1 separately (each exactly) and added. */
int oracle_nudft2d(int64_t N1, int64_t N2, const double *C, int64_t M,
                   const double *x, const double *y, double *f)
{
    if (N1 < 0 || N2 < 0 || M < 0) return -1;
    #pragma omp parallel for schedule(dynamic, 4)
    for (int64_t j = 0; j < M; ++j) {
        acc2 re = {0.0, 0.0}, im = {0.0, 0.0};
        for (int64_t k1 = 0; k1 < N1; ++k1) {
            double p1 = phase_mod1(x[j], (double)k1);
            for (int64_t k2 = 0; k2 < N2; ++k2) {
                double phi = p1 + phase_mod1(y[j], (double)k2);
                double co, si;
                cis2pi(phi - nearbyint(phi), &co, &si);
                si = -si;
                const double *cc = C + 2 * (k1 * N2 + k2);
                acc2_add_prod(&re, cc[0], co);
                acc2_add_prod(&re, -cc[1], si);
                acc2_add_prod(&im, cc[0], si);
                acc2_add_prod(&im, cc[1], co);
            }
        }
        f[2 * j] = re.s + re.t;
        f[2 * j + 1] = im.s + im.t;
    }
    return 0;
}

/* Adjoint (sign = +1) or 2-D type I (sign = -1, the transpose) of the 2-D
 * type II, evaluated at the requested coefficient indices:
 *   out_q = sum_{j<M} g_j exp(sign 2 pi i (k1_q x_j + k2_q y_j)). */
int oracle_nudft2d_adj(int64_t M, const double *x, const double *y, const double *g,
                       int64_t nq, const int64_t *k1, const int64_t *k2, int sign, double *out)
{
    if (M < 0 || nq < 0 || (sign != 1 && sign != -1)) return -1;
    #pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < nq; ++q) {
        acc2 re = {0.0, 0.0}, im = {0.0, 0.0};
        for (int64_t j = 0; j < M; ++j) {
            double phi = phase_mod1(x[j], (double)k1[q]) + phase_mod1(y[j], (double)k2[q]);
            double co, si;
            cis2pi(phi - nearbyint(phi), &co, &si);
            si *= (double)sign;
            double gr = g[2 * j], gi = g[2 * j + 1];
            acc2_add_prod(&re, gr, co);
            acc2_add_prod(&re, -gi, si);
            acc2_add_prod(&im, gr, si);
            acc2_add_prod(&im, gi, co);
        }
        out[2 * q] = re.s + re.t;
        out[2 * q + 1] = im.s + im.t;
    }
    return 0;
}

/* 3-D type II: f_j = sum_{k1<N1, k2<N2, k3<N3} C[(k1*N2+k2)*N3+k3]
 *   exp(-2 pi i (k1 x_j + k2 y_j + k3 z_j)); the three phases reduced modulo 1 separately. */
int oracle_nudft3d(int64_t N1, int64_t N2, int64_t N3, const double *C, int64_t M,
                   const double *x, const double *y, const double *z, double *f)
{
    if (N1 < 0 || N2 < 0 || N3 < 0 || M < 0) return -1;
    #pragma omp parallel for schedule(dynamic, 4)
    for (int64_t j = 0; j < M; ++j) {
        acc2 re = {0.0, 0.0}, im = {0.0, 0.0};
        for (int64_t k1 = 0; k1 < N1; ++k1) {
            double p1 = phase_mod1(x[j], (double)k1);
            for (int64_t k2 = 0; k2 < N2; ++k2) {
                double p12 = p1 + phase_mod1(y[j], (double)k2);
                for (int64_t k3 = 0; k3 < N3; ++k3) {
                    double phi = p12 + phase_mod1(z[j], (double)k3);
                    double co, si;
                    cis2pi(phi - nearbyint(phi), &co, &si);
                    si = -si;
                    const double *cc = C + 2 * ((k1 * N2 + k2) * N3 + k3);
                    acc2_add_prod(&re, cc[0], co);
                    acc2_add_prod(&re, -cc[1], si);
                    acc2_add_prod(&im, cc[0], si);
                    acc2_add_prod(&im, cc[1], co);
                }
            }
        }
        f[2 * j] = re.s + re.t;
        f[2 * j + 1] = im.s + im.t;
    }
    return 0;
}

/* Adjoint (sign = +1) or type I (sign = -1, the transpose) of the 3-D type II at the
 * requested coefficient indices:
 *   out_q = sum_{j<M} g_j exp(sign 2 pi i (k1_q x_j + k2_q y_j + k3_q z_j)). */
int oracle_nudft3d_adj(int64_t M, const double *x, const double *y, const double *z, const double *g,
                       int64_t nq, const int64_t *k1, const int64_t *k2, const int64_t *k3, int sign,
                       double *out)
{
    if (M < 0 || nq < 0 || (sign != 1 && sign != -1)) return -1;
    #pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < nq; ++q) {
        acc2 re = {0.0, 0.0}, im = {0.0, 0.0};
        for (int64_t j = 0; j < M; ++j) {
            double phi = phase_mod1(x[j], (double)k1[q]) + phase_mod1(y[j], (double)k2[q])
                         + phase_mod1(z[j], (double)k3[q]);
            double co, si;
            cis2pi(phi - nearbyint(phi), &co, &si);
            si *= (double)sign;
            double gr = g[2 * j], gi = g[2 * j + 1];
            acc2_add_prod(&re, gr, co);
            acc2_add_prod(&re, -gi, si);
            acc2_add_prod(&im, gr, si);
            acc2_add_prod(&im, gi, co);
        }
        out[2 * q] = re.s + re.t;
        out[2 * q + 1] = im.s + im.t;
    }
    return 0;
}

/* 2-D type III: f_j = sum_{k<Q} c_k exp(-2 pi i (x_j w1_k + y_j w2_k)).  Both products
 * are non-integer; each is reduced modulo 1 exactly and the two are added. */
int oracle_nudft3_2d(int64_t Q, const double *w1, const double *w2, const double *c, int64_t M,
                     const double *x, const double *y, double *f)
{
    if (Q < 0 || M < 0) return -1;
    #pragma omp parallel for schedule(dynamic, 4)
    for (int64_t j = 0; j < M; ++j) {
        acc2 re = {0.0, 0.0}, im = {0.0, 0.0};
        for (int64_t k = 0; k < Q; ++k) {
            double phi = phase_mod1(x[j], w1[k]) + phase_mod1(y[j], w2[k]);
            double co, si;
            cis2pi(phi - nearbyint(phi), &co, &si);
            si = -si;
            double cr = c[2 * k], ci = c[2 * k + 1];
            acc2_add_prod(&re, cr, co);
            acc2_add_prod(&re, -ci, si);
            acc2_add_prod(&im, cr, si);
            acc2_add_prod(&im, ci, co);
        }
        f[2 * j] = re.s + re.t;
        f[2 * j + 1] = im.s + im.t;
    }
    return 0;
}

/* Nearest-grid assignment on a grid of n points (Sec. 2.2):
 *   s_j = round(n x_j)  (round-to-nearest-even of the rounded product),
 *   t_j = s_j mod n     (Euclidean, so negative x wraps too),
 *   d_j = n x_j - s_j   (single rounding through fma).
 * Returns -1 if any x is not finite or n < 1, else 0. */
int oracle_grid_assign(int64_t n, int64_t M, const double *x, int64_t *s,
                       int64_t *t, double *d)
{
    if (n < 1 || M < 0) return -1;
    for (int64_t j = 0; j < M; ++j)
        if (!isfinite(x[j])) return -1;
    for (int64_t j = 0; j < M; ++j) {
        double nx = (double)n * x[j];
        double sj = nearbyint(nx);
        int64_t si = (int64_t)sj;
        int64_t ti = si % n;
        if (ti < 0) ti += n;
        s[j] = si;
        t[j] = ti;
        d[j] = fma((double)n, x[j], -sj);
    }
    return 0;
}
