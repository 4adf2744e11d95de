// Type III (Sec. 3.2): f_j = sum_k c_k exp(-2 pi i x_j w_k), x_j in [0, 1), w_k in [0, N).
// With s_j = round(N x_j), t_j = s_j mod N and d_j = N x_j - s_j,
//   exp(-2 pi i x_j w_k) = exp(-2 pi i d_j w_k / N) * B_jk * exp(-2 pi i t_j w_k / N),
//   B_jk = 1 if s_j < N, exp(-2 pi i w_k) if s_j = N,
// the first factor is the rank-K expansion u_r(d_j) v_r(w_k / N) of Sec. 2.1.2
// (X = d_j, Y = 2 pi w_k / N), and the last is row t_j of the type-I matrix on
// the samples w/N.  So f = sum_r u_r o [ F1(v_r o c) or F1(v_r o e^{-2 pi i w} o c) ](t),
// each F1 a type-I transform (nufft1) with N modes.
#include "kernels.h"

namespace nufft {

// t_j, d_j, wrap flag, max |d_j| (bits of a non-negative double), and any-wrap flag.
__global__ void __launch_bounds__(256)
k_t3_assign(const double *__restrict__ x, int64_t M, int64_t N, int32_t *__restrict__ t, double *__restrict__ d,
            int32_t *__restrict__ wrap, unsigned long long *gbits, int *flags)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    const double xj = x[j];
    if (!isfinite(xj) || xj < 0.0 || xj >= 1.0) {
        atomicOr(flags, 1);
        t[j] = 0;
        d[j] = 0.0;
        wrap[j] = 0;
        return;
    }
    const double Nd = (double)N;
    const double s = rint(Nd * xj);
    const double dj = fma(Nd, xj, -s);
    const int w = s >= Nd ? 1 : 0;
    t[j] = w ? 0 : (int32_t)s;
    d[j] = dj;
    wrap[j] = w;
    if (w) atomicOr(flags, 2);
    atomicMax(gbits, (unsigned long long)__double_as_longlong(fabs(dj)));
}

// x'_k = w_k / N (the samples of the inner type-I transform); flags bad frequencies.
__global__ void __launch_bounds__(256)
k_t3_freq(const double *__restrict__ w, int64_t N, double *__restrict__ xs, int *flags)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const double wk = w[k];
    if (!isfinite(wk) || wk < 0.0 || wk >= (double)N) atomicOr(flags, 4);
    xs[k] = wk / (double)N;
}

// c'_k = v_r(w_k / N) c_k, and (if with_wrap) c''_k = c'_k exp(-2 pi i w_k).
template <typename R>
__global__ void __launch_bounds__(256)
k_t3_scale(const cx_t<R> *__restrict__ c, const double *__restrict__ w, int64_t N, int r, int with_wrap,
           cx_t<R> *__restrict__ c1, cx_t<R> *__restrict__ c2)
{
    using C = cx_t<R>;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const double wk = w[k];
    const double z = 2.0 * wk / (double)N - 1.0;
    double v;
    if (r == 0) v = 0.5;
    else {
        double a = 1.0, b = z;
        for (int q = 1; q < r; ++q) {
            const double cn = 2.0 * z * b - a;
            a = b;
            b = cn;
        }
        v = b;
    }
    const C ck = c[k];
    const C s1 = cmake<C>((R)(v * (double)ck.x), (R)(v * (double)ck.y));
    c1[k] = s1;
    if (with_wrap) {
        // exp(-2 pi i w) with w reduced exactly modulo 1
        const double fr = wk - floor(wk);
        double sn, cs;
        sincospi(2.0 * fr, &sn, &cs);
        c2[k] = cmake<C>((R)(cs * (double)s1.x + sn * (double)s1.y), (R)(cs * (double)s1.y - sn * (double)s1.x));
    }
}

// f_j (+)= u_r(d_j) * y[t_j] (or y2[t_j] for wrapped samples), u_r from the monomial form.
template <typename R>
__global__ void __launch_bounds__(256)
k_t3_accum(const double *__restrict__ d, const int32_t *__restrict__ t, const int32_t *__restrict__ wrap,
           int64_t M, Factors<double> fac, int r, const cx_t<R> *__restrict__ y, const cx_t<R> *__restrict__ y2,
           cx_t<R> *__restrict__ f)
{
    using C = cx_t<R>;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    const double dj = d[j];
    double sn, cs;
    sincospi(dj, &sn, &cs);
    const double p = upoly(fac, r, dj * fac.inv_gamma);
    // u_r = i^r exp(-i pi d) p
    double ur = cs * p, ui = -sn * p;
    for (int q = 0; q < (r & 3); ++q) {
        const double tmp = ur;
        ur = -ui;
        ui = tmp;
    }
    const C yy = (wrap[j] && y2) ? y2[t[j]] : y[t[j]];
    C acc = r == 0 ? cmake<C>(0, 0) : f[j];
    acc.x += (R)(ur * (double)yy.x - ui * (double)yy.y);
    acc.y += (R)(ur * (double)yy.y + ui * (double)yy.x);
    f[j] = acc;
}

// ---- 2-D type III: f_j = sum_k c_k exp(-2 pi i (x_j w1_k + y_j w2_k)) ------------------------
// Each axis factors as in the 1-D case, with s^x_j = round(n1 x_j) in [0, n1]
// and d^x_j = n1 x_j - s^x_j (likewise y with n2).  The row s^x, s^y of the
// 2-D type-I matrix on the samples (w1/n1, w2/n2) is read from an inner 2-D
// type I with n1 + 1 by n2 + 1 modes, so s = n needs no wrap factor:
//   f = sum_{r1,r2} u^x_r1(d^x) u^y_r2(d^y) o F1_2D(v^x_r1(w1/n1) v^y_r2(w2/n2) o c)[s^x][s^y].

// s, d per axis; max |d| per axis (bits of non-negative doubles); flags bad samples.
__global__ void __launch_bounds__(256)
k_t3d_assign(const double *__restrict__ x, const double *__restrict__ y, int64_t M, int64_t n1, int64_t n2,
             int32_t *__restrict__ sx, int32_t *__restrict__ sy, double *__restrict__ dx, double *__restrict__ dy,
             unsigned long long *gbits, int *flags)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    const double xj = x[j], yj = y[j];
    if (!isfinite(xj) || !isfinite(yj) || xj < 0.0 || xj >= 1.0 || yj < 0.0 || yj >= 1.0) {
        atomicOr(flags, 1);
        sx[j] = sy[j] = 0;
        dx[j] = dy[j] = 0.0;
        return;
    }
    const double a = rint((double)n1 * xj), b = rint((double)n2 * yj);
    const double da = fma((double)n1, xj, -a), db = fma((double)n2, yj, -b);
    sx[j] = (int32_t)a;
    sy[j] = (int32_t)b;
    dx[j] = da;
    dy[j] = db;
    atomicMax(gbits, (unsigned long long)__double_as_longlong(fabs(da)));
    atomicMax(gbits + 1, (unsigned long long)__double_as_longlong(fabs(db)));
}

// samples of the inner 2-D type I: (w1_k / n1, w2_k / n2); flags frequencies outside [0, n).
__global__ void __launch_bounds__(256)
k_t3d_freq(const double *__restrict__ w1, const double *__restrict__ w2, int64_t Q, int64_t n1, int64_t n2,
           double *__restrict__ xs, double *__restrict__ ys, int *flags)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= Q) return;
    const double a = w1[k], b = w2[k];
    if (!isfinite(a) || !isfinite(b) || a < 0.0 || a >= (double)n1 || b < 0.0 || b >= (double)n2) atomicOr(flags, 4);
    xs[k] = a / (double)n1;
    ys[k] = b / (double)n2;
}

__device__ __forceinline__ double t3_cheb(int r, double z)
{
    if (r == 0) return 0.5;
    double a = 1.0, b = z;
    for (int q = 1; q < r; ++q) {
        const double cn = 2.0 * z * b - a;
        a = b;
        b = cn;
    }
    return b;
}

// c'_k = v_r1(w1_k / n1) v_r2(w2_k / n2) c_k
template <typename R>
__global__ void __launch_bounds__(256)
k_t3d_scale(const cx_t<R> *__restrict__ c, const double *__restrict__ w1, const double *__restrict__ w2, int64_t Q,
            int64_t n1, int64_t n2, int r1, int r2, cx_t<R> *__restrict__ c1)
{
    using C = cx_t<R>;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= Q) return;
    const double v = t3_cheb(r1, 2.0 * w1[k] / (double)n1 - 1.0) * t3_cheb(r2, 2.0 * w2[k] / (double)n2 - 1.0);
    const C ck = c[k];
    c1[k] = cmake<C>((R)(v * (double)ck.x), (R)(v * (double)ck.y));
}

// u_r(d) = i^r exp(-i pi d) P_r(d / gamma) in FP64
__device__ __forceinline__ void t3_u(const Factors<double> &fac, int r, double d, double *ur, double *ui)
{
    double sn, cs;
    sincospi(d, &sn, &cs);
    const double p = upoly(fac, r, d * fac.inv_gamma);
    double a = cs * p, b = -sn * p;
    for (int q = 0; q < (r & 3); ++q) {
        const double t = a;
        a = -b;
        b = t;
    }
    *ur = a;
    *ui = b;
}

// f_j (+)= u^x_r1(d^x_j) u^y_r2(d^y_j) F[s^x_j][s^y_j]  (F row-major with ld = n2 + 1)
template <typename R>
__global__ void __launch_bounds__(256)
k_t3d_accum(const double *__restrict__ dx, const double *__restrict__ dy, const int32_t *__restrict__ sx,
            const int32_t *__restrict__ sy, int64_t M, Factors<double> fx, Factors<double> fy, int r1, int r2,
            const cx_t<R> *__restrict__ F, int64_t ld, int first, cx_t<R> *__restrict__ f)
{
    using C = cx_t<R>;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    double ar, ai, br, bi;
    t3_u(fx, r1, dx[j], &ar, &ai);
    t3_u(fy, r2, dy[j], &br, &bi);
    const double ur = ar * br - ai * bi, ui = ar * bi + ai * br;
    const C yy = F[(int64_t)sx[j] * ld + sy[j]];
    C acc = first ? cmake<C>(0, 0) : f[j];
    acc.x += (R)(ur * (double)yy.x - ui * (double)yy.y);
    acc.y += (R)(ur * (double)yy.y + ui * (double)yy.x);
    f[j] = acc;
}

hipError_t t3d_assign(const double *x, const double *y, int64_t M, int64_t n1, int64_t n2, int32_t *sx, int32_t *sy,
                      double *dx, double *dy, unsigned long long *gbits, int *flags, hipStream_t s)
{
    hipLaunchKernelGGL(k_t3d_assign, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, x, y, M, n1, n2, sx, sy, dx,
                       dy, gbits, flags);
    return hipGetLastError();
}

hipError_t t3d_freq(const double *w1, const double *w2, int64_t Q, int64_t n1, int64_t n2, double *xs, double *ys,
                    int *flags, hipStream_t s)
{
    hipLaunchKernelGGL(k_t3d_freq, dim3((unsigned)((Q + 255) / 256)), dim3(256), 0, s, w1, w2, Q, n1, n2, xs, ys,
                       flags);
    return hipGetLastError();
}

template <typename R>
hipError_t t3d_scale(const cx_t<R> *c, const double *w1, const double *w2, int64_t Q, int64_t n1, int64_t n2, int r1,
                     int r2, cx_t<R> *c1, hipStream_t s)
{
    hipLaunchKernelGGL(k_t3d_scale<R>, dim3((unsigned)((Q + 255) / 256)), dim3(256), 0, s, c, w1, w2, Q, n1, n2, r1,
                       r2, c1);
    return hipGetLastError();
}

template <typename R>
hipError_t t3d_accum(const double *dx, const double *dy, const int32_t *sx, const int32_t *sy, int64_t M,
                     const Factors<double> &fx, const Factors<double> &fy, int r1, int r2, const cx_t<R> *F,
                     int64_t ld, int first, cx_t<R> *f, hipStream_t s)
{
    hipLaunchKernelGGL(k_t3d_accum<R>, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, dx, dy, sx, sy, M, fx, fy,
                       r1, r2, F, ld, first, f);
    return hipGetLastError();
}

template hipError_t t3d_scale<float>(const float2 *, const double *, const double *, int64_t, int64_t, int64_t, int,
                                     int, float2 *, hipStream_t);
template hipError_t t3d_scale<double>(const double2 *, const double *, const double *, int64_t, int64_t, int64_t,
                                      int, int, double2 *, hipStream_t);
template hipError_t t3d_accum<float>(const double *, const double *, const int32_t *, const int32_t *, int64_t,
                                     const Factors<double> &, const Factors<double> &, int, int, const float2 *,
                                     int64_t, int, float2 *, hipStream_t);
template hipError_t t3d_accum<double>(const double *, const double *, const int32_t *, const int32_t *, int64_t,
                                      const Factors<double> &, const Factors<double> &, int, int, const double2 *,
                                      int64_t, int, double2 *, hipStream_t);

hipError_t t3_assign(const double *x, int64_t M, int64_t N, int32_t *t, double *d, int32_t *wrap,
                     unsigned long long *gbits, int *flags, hipStream_t s)
{
    hipLaunchKernelGGL(k_t3_assign, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, x, M, N, t, d, wrap, gbits,
                       flags);
    return hipGetLastError();
}

hipError_t t3_freq(const double *w, int64_t N, double *xs, int *flags, hipStream_t s)
{
    hipLaunchKernelGGL(k_t3_freq, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, w, N, xs, flags);
    return hipGetLastError();
}

template <typename R>
hipError_t t3_scale(const cx_t<R> *c, const double *w, int64_t N, int r, int with_wrap, cx_t<R> *c1, cx_t<R> *c2,
                    hipStream_t s)
{
    hipLaunchKernelGGL(k_t3_scale<R>, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, c, w, N, r, with_wrap, c1,
                       c2);
    return hipGetLastError();
}

template <typename R>
hipError_t t3_accum(const double *d, const int32_t *t, const int32_t *wrap, int64_t M, const Factors<double> &fac,
                    int r, const cx_t<R> *y, const cx_t<R> *y2, cx_t<R> *f, hipStream_t s)
{
    hipLaunchKernelGGL(k_t3_accum<R>, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, d, t, wrap, M, fac, r, y,
                       y2, f);
    return hipGetLastError();
}

template hipError_t t3_scale<float>(const float2 *, const double *, int64_t, int, int, float2 *, float2 *,
                                    hipStream_t);
template hipError_t t3_scale<double>(const double2 *, const double *, int64_t, int, int, double2 *, double2 *,
                                     hipStream_t);
template hipError_t t3_accum<float>(const double *, const int32_t *, const int32_t *, int64_t,
                                    const Factors<double> &, int, const float2 *, const float2 *, float2 *,
                                    hipStream_t);
template hipError_t t3_accum<double>(const double *, const int32_t *, const int32_t *, int64_t,
                                     const Factors<double> &, int, const double2 *, const double2 *, double2 *,
                                     hipStream_t);

}  // namespace nufft
