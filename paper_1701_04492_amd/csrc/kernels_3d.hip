// 3-D transforms by the construction of Sec. 4 with a third axis; the type II:
//
//   f_j = sum_{k1,k2,k3} C[k1][k2][k3] exp(-2 pi i (k1 x_j + k2 y_j + k3 z_j)).
//
// The z axis gets the rank-K3 expansion of Sec. 2.1-2.2 on a grid of Gz
// points: exp(-2 pi i k3 z_j) ~ sum_r u^z_r(j) v^z_r(k3) exp(-2 pi i k3 t^z_j / Gz).
// So, with D_r[m][k1][k2] = sum_k3 v^z_r(k3) C[k1][k2][k3] exp(-2 pi i k3 m / Gz)
// (one length-Gz FFT per (k1, k2), here `k_3d_zfft`),
//
//   f_j = sum_r u^z_r(j) * [2-D type II of D_r[t^z_j] at (x_j, y_j)],
//
// and the samples of one z slice m form problem m of one stacked 2-D plan
// (its keys carry the slice, so one pass-B launch serves every slice).
// `k_3d_accum` adds u^z_r times the 2-D results into f.
//
// The 3-D type I (sign -1, the transpose) and adjoint (sign +1) run the same
// factoring backwards: with w_r(j) = u^z_r(j) (type I) or its conjugate
// (adjoint), `k_3d_weight` forms w_r(j) c_j, each slice m gets a 2-D type I
// of those weights, E_r[m][k1][k2], and `k_3d_zfft_t`
// finishes C[k1][k2][k3] += v^z_r(k3) sum_m E_r[m][k1][k2] exp(sign 2 pi i k3 m / Gz).
#include "fused_common.h"
#include "kernels_3d.h"

namespace nufft {

// s = rint(Gz z), t = s mod Gz (Euclidean), X = (Gz z - s) n3 / Gz; max |X|; bad samples flagged.
template <typename R>
__global__ void __launch_bounds__(256)
k_3d_assign(const double *__restrict__ z, int64_t M, int64_t n3, int64_t Gz, int32_t *__restrict__ t,
            R *__restrict__ X, unsigned long long *gbits, int *flags)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    const double zj = z[j];
    if (!isfinite(zj)) {
        atomicOr(flags, 1);
        t[j] = 0;
        X[j] = 0;
        return;
    }
    const double s = rint((double)Gz * zj);
    const double d = fma((double)Gz, zj, -s) * ((double)n3 / (double)Gz);
    int64_t tt = (int64_t)s % Gz;
    if (tt < 0) tt += Gz;
    t[j] = (int32_t)tt;
    X[j] = (R)d;
    atomicMax(gbits, (unsigned long long)__double_as_longlong(fabs(d)));
}

// D_r[m][row] = FFT_m( v^z_r(k3) C[row][k3] ), rows = n1 * n2, RC rows per workgroup
// (256 threads), written slice-major so that slice m is one contiguous n1 x n2 array.
template <typename R, int GZ>
__global__ void __launch_bounds__(256)
k_3d_zfft(const cx_t<R> *__restrict__ Cin, int64_t rows, int64_t n3, int r, const cx_t<R> *__restrict__ tw_g,
          cx_t<R> *__restrict__ D)
{
    using C = cx_t<R>;
    constexpr int TPF = GZ / 16;
    constexpr int RC = 256 / TPF;
    constexpr int P = fft_pitch(GZ);
    __shared__ C buf[RC * P];
    __shared__ C tw[GZ];
    load_tw_s<C, GZ, -1, 256>(tw, tw_g);
    const int tid = threadIdx.x;
    const int g = tid / TPF, lt = tid % TPF;
    const int64_t row0 = (int64_t)blockIdx.x * RC;
    const int64_t row = row0 + g;
    const ZMap zm = zmap(n3);
    C v[16];
    R zq[16], wq[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int64_t k3 = lt + q * TPF;
        const bool in = row < rows && k3 < n3;
        const C c = Cin[min(row, rows - 1) * n3 + min(k3, n3 - 1)];   // clamped: the loads issue together
        v[q] = in ? c : cmake<C>(0, 0);
        zq[q] = zcoord<R>(k3, zm);
    }
    cheb_v_many<R, 16>(r, zq, wq);
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] = cscale(v[q], wq[q]);
    __syncthreads();   // the twiddle table is in LDS
    block_fft_regs<C, GZ, -1, fft_wave_sync<GZ>>(buf + g * P, tw, lt, v);
    __syncthreads();   // the transposed store reads other transforms
    // slice-major store: consecutive threads write consecutive rows of one slice
    constexpr int E = (RC * GZ) / 256;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = tid + e * 256;
        const int gg = i % RC, m = i / RC;
        if (row0 + gg < rows) D[(int64_t)m * rows + row0 + gg] = buf[gg * P + lds_pad(m)];
    }
}

// f[j] (+)= u^z_r(X_j) fs[j]; u_r = i^r exp(-i pi X) P_r(X / gamma).
template <typename R>
__global__ void __launch_bounds__(256)
k_3d_accum(const cx_t<R> *__restrict__ fs, const R *__restrict__ Xz, int64_t M, Factors<R> fac, int r,
           cx_t<R> *__restrict__ f)
{
    using C = cx_t<R>;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    const R X = Xz[j];
    R sn, cs;
    sincospi_r(X, &sn, &cs);
    const RankPoly<R> up = rank_poly(fac, r);
    const C u = crot(cscale(cmake<C>(cs, -sn), rank_eval(up, X * fac.inv_gamma)), r);
    const C add = cmul(u, fs[j]);
    f[j] = r == 0 ? add : cadd(f[j], add);
}

// cw[j] = w_r(j) c[j], w_r = u^z_r (DIR -1) or its conjugate (DIR +1).
template <typename R, int DIR>
__global__ void __launch_bounds__(256)
k_3d_weight(const cx_t<R> *__restrict__ c, const R *__restrict__ Xz, int64_t M, Factors<R> fac, int r,
            cx_t<R> *__restrict__ cw)
{
    using C = cx_t<R>;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    const R X = Xz[j];
    R sn, cs;
    sincospi_r(X, &sn, &cs);
    const RankPoly<R> up = rank_poly(fac, r);
    C u = crot(cscale(cmake<C>(cs, -sn), rank_eval(up, X * fac.inv_gamma)), r);
    if (DIR > 0) u = cconj(u);
    cw[j] = cmul(u, c[j]);
}

// C[row][k3] (r == 0 ? = : +=) v^z_r(k3) sum_m E[m][row] exp(DIR 2 pi i k3 m / GZ), k3 < n3:
// RC rows per workgroup (256 threads), E read slice-major (consecutive threads read
// consecutive rows of one slice), C written row-major with k3 fastest.
template <typename R, int GZ, int DIR>
__global__ void __launch_bounds__(256)
k_3d_zfft_t(const cx_t<R> *__restrict__ E, int64_t rows, int64_t n3, int r, const cx_t<R> *__restrict__ tw_g,
            cx_t<R> *__restrict__ Cout)
{
    using C = cx_t<R>;
    constexpr int TPF = GZ / 16;
    constexpr int RC = 256 / TPF;
    constexpr int P = fft_pitch(GZ);
    constexpr int NE = (RC * GZ) / 256;
    __shared__ C buf[RC * P];
    __shared__ C tw[GZ];
    load_tw_s<C, GZ, DIR, 256>(tw, tw_g);
    const int tid = threadIdx.x;
    const int64_t row0 = (int64_t)blockIdx.x * RC;
    C v[NE];
#pragma unroll
    for (int e = 0; e < NE; ++e) {
        const int i = tid + e * 256;
        const int gg = i % RC, m = i / RC;
        const bool in = row0 + gg < rows;
        const C x = E[(int64_t)m * rows + min(row0 + gg, rows - 1)];   // clamped: the loads issue together
        v[e] = in ? x : cmake<C>(0, 0);
    }
#pragma unroll
    for (int e = 0; e < NE; ++e) {
        const int i = tid + e * 256;
        buf[(i % RC) * P + lds_pad(i / RC)] = v[e];
    }
    __syncthreads();   // the rows and the twiddle table are in LDS
    block_fft_lds<C, GZ, DIR, fft_wave_sync<GZ>>(buf + (tid / TPF) * P, tw, tid % TPF);
    __syncthreads();   // the row-major store reads other transforms
    const ZMap zm = zmap(n3);
    R zq[NE], wq[NE];
#pragma unroll
    for (int e = 0; e < NE; ++e) zq[e] = zcoord<R>((tid + e * 256) % GZ, zm);
    cheb_v_many<R, NE>(r, zq, wq);
#pragma unroll
    for (int e = 0; e < NE; ++e) {
        const int i = tid + e * 256;
        const int gg = i / GZ, k3 = i % GZ;
        if (k3 < n3 && row0 + gg < rows) {
            C *o = Cout + (row0 + gg) * n3 + k3;
            const C add = cscale(buf[gg * P + lds_pad(k3)], wq[e]);
            *o = r == 0 ? add : cadd(*o, add);
        }
    }
}

template <typename R>
hipError_t launch_3d_assign(const double *z, int64_t M, int64_t n3, int64_t Gz, int32_t *t, R *X,
                            unsigned long long *gbits, int *flags, hipStream_t s)
{
    hipLaunchKernelGGL(k_3d_assign<R>, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, z, M, n3, Gz, t, X, gbits,
                       flags);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_3d_zfft(const cx_t<R> *Cin, int64_t rows, int64_t n3, int64_t Gz, int r, const cx_t<R> *tw,
                          cx_t<R> *D, hipStream_t s)
{
    switch (Gz) {
#define ZF(GG)                                                                                               \
    case GG: {                                                                                               \
        constexpr int RC = 256 / (GG / 16);                                                                  \
        hipLaunchKernelGGL((k_3d_zfft<R, GG>), dim3((unsigned)((rows + RC - 1) / RC)), dim3(256), 0, s, Cin, \
                           rows, n3, r, tw, D);                                                              \
        break;                                                                                               \
    }
        ZF(16) ZF(32) ZF(64) ZF(128) ZF(256) ZF(512) ZF(1024)
#undef ZF
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename R>
hipError_t launch_3d_accum(const cx_t<R> *fs, const R *Xz, int64_t M, const Factors<R> &fac, int r, cx_t<R> *f,
                           hipStream_t s)
{
    hipLaunchKernelGGL(k_3d_accum<R>, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, fs, Xz, M, fac, r, f);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_3d_weight(const cx_t<R> *c, const R *Xz, int64_t M, const Factors<R> &fac, int r, int sign,
                            cx_t<R> *cw, hipStream_t s)
{
    const dim3 g((unsigned)((M + 255) / 256));
    if (sign < 0)
        hipLaunchKernelGGL((k_3d_weight<R, -1>), g, dim3(256), 0, s, c, Xz, M, fac, r, cw);
    else
        hipLaunchKernelGGL((k_3d_weight<R, 1>), g, dim3(256), 0, s, c, Xz, M, fac, r, cw);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_3d_zfft_t(const cx_t<R> *E, int64_t rows, int64_t n3, int64_t Gz, int r, int sign,
                            const cx_t<R> *tw, cx_t<R> *Cout, hipStream_t s)
{
    switch (Gz) {
#define ZT(GG)                                                                                                   \
    case GG: {                                                                                                   \
        constexpr int RC = 256 / (GG / 16);                                                                      \
        const dim3 g((unsigned)((rows + RC - 1) / RC));                                                          \
        if (sign < 0)                                                                                            \
            hipLaunchKernelGGL((k_3d_zfft_t<R, GG, -1>), g, dim3(256), 0, s, E, rows, n3, r, tw, Cout);         \
        else                                                                                                     \
            hipLaunchKernelGGL((k_3d_zfft_t<R, GG, 1>), g, dim3(256), 0, s, E, rows, n3, r, tw, Cout);          \
        break;                                                                                                   \
    }
        ZT(16) ZT(32) ZT(64) ZT(128) ZT(256) ZT(512) ZT(1024)
#undef ZT
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template hipError_t launch_3d_assign<float>(const double *, int64_t, int64_t, int64_t, int32_t *, float *,
                                            unsigned long long *, int *, hipStream_t);
template hipError_t launch_3d_assign<double>(const double *, int64_t, int64_t, int64_t, int32_t *, double *,
                                             unsigned long long *, int *, hipStream_t);
template hipError_t launch_3d_zfft<float>(const float2 *, int64_t, int64_t, int64_t, int, const float2 *, float2 *,
                                          hipStream_t);
template hipError_t launch_3d_zfft<double>(const double2 *, int64_t, int64_t, int64_t, int, const double2 *,
                                           double2 *, hipStream_t);
template hipError_t launch_3d_accum<float>(const float2 *, const float *, int64_t, const Factors<float> &, int,
                                           float2 *, hipStream_t);
template hipError_t launch_3d_accum<double>(const double2 *, const double *, int64_t, const Factors<double> &, int,
                                            double2 *, hipStream_t);

template hipError_t launch_3d_weight<float>(const float2 *, const float *, int64_t, const Factors<float> &, int, int,
                                            float2 *, hipStream_t);
template hipError_t launch_3d_weight<double>(const double2 *, const double *, int64_t, const Factors<double> &, int,
                                             int, double2 *, hipStream_t);
template hipError_t launch_3d_zfft_t<float>(const float2 *, int64_t, int64_t, int64_t, int, int, const float2 *,
                                            float2 *, hipStream_t);
template hipError_t launch_3d_zfft_t<double>(const double2 *, int64_t, int64_t, int64_t, int, int,
                                             const double2 *, double2 *, hipStream_t);

}  // namespace nufft
