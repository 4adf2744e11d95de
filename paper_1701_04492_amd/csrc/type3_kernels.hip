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
