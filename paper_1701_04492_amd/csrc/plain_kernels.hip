// Plain (unfused) online stage of the type-II NUFFT, Sec. 2.3 two-step form
// (and of its transpose and adjoint, Sec. 3.1, further down):
//   W_r = D_{v_r} c (K x L buffer in HBM)      -> k_scale
//   X_r = F_L W_r (stand-alone FFT passes)      -> k_fft_rows / k_fft_cols
//   f_j = sum_r U[j][r] X_r[t_j]                -> k_gather (U stored by the plan)
// Every intermediate goes through HBM; this is the reference point the fused
// kernels are measured against.
#include "fft.h"
#include "kernels.h"

namespace nufft {

// v_r(k) = T_r(2k/N - 1) (v_0 halved), W[r][k] = v_r(k) c_k for k < N, 0 for N <= k < L.
// mode 1 multiplies c_k by -2 pi i k (derivative in x, calculus on eq. (2)).
template <typename R>
__global__ void __launch_bounds__(256)
k_scale(const cx_t<R> *__restrict__ c, int64_t N, int64_t L, int K, int mode,
        cx_t<R> *__restrict__ W)
{
    using C = cx_t<R>;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= L) return;
    C ck = cmake<C>(0, 0);
    R z = 0;
    if (k < N) {
        ck = c[k];
        if (mode == 1) {
            const R w = (R)(-2.0 * M_PI * (double)k);
            ck = cmake<C>(-w * ck.y, w * ck.x);
        }
        z = (R)(2.0 * (double)k / (double)N - 1.0);
    }
    R tm2 = 1, tm1 = z;
    for (int r = 0; r < K; ++r) {
        R v;
        if (r == 0) v = (R)0.5;
        else if (r == 1) v = z;
        else { v = 2 * z * tm1 - tm2; tm2 = tm1; tm1 = v; }
        W[(int64_t)r * L + k] = cscale(ck, v);
    }
}

// Loads the forward table e^{-2 pi i m / L}, conjugated for DIR = +1, into LDS.
template <typename C, int L, int DIR>
__device__ __forceinline__ void load_tw(C *tw_s, const C *__restrict__ tw_g)
{
    for (int m = threadIdx.x; m < L; m += blockDim.x) {
        C w = tw_g[m];
        tw_s[m] = DIR < 0 ? w : cconj(w);
    }
}

// exp(DIR 2 pi i m / L) from the two-level tables hi[m >> 12] * lo[m & 4095].
template <typename C, int DIR>
__device__ __forceinline__ C twiddle_big(const C *__restrict__ hi, const C *__restrict__ lo, int64_t m)
{
    C w = cmul(hi[m >> 12], lo[m & 4095]);
    return DIR < 0 ? w : cconj(w);
}

// G rows of length L per workgroup, FFT along the row.  Rows of batch b are
// in[b*rows*L + row*L + k].  TRANSPOSE = 0 writes out[b][row][n]; TRANSPOSE = 1
// writes out[b][n*rows + row] (the output order of the second four-step pass).
template <typename R, int L, int G, int DIR, int TRANSPOSE>
__global__ void __launch_bounds__(G * L / 16)
k_fft_rows(const cx_t<R> *__restrict__ in, cx_t<R> *__restrict__ out, int64_t rows,
           const cx_t<R> *__restrict__ tw_g)
{
    using C = cx_t<R>;
    constexpr int NT = G * L / 16;
    constexpr int P = fft_pitch(L);
    __shared__ C buf[G * P];
    __shared__ C tw[L];
    const int64_t b = blockIdx.y;
    const int64_t row0 = (int64_t)blockIdx.x * G;
    const C *src = in + (b * rows + row0) * L;
    load_tw<C, L, DIR>(tw, tw_g);
    for (int i = threadIdx.x; i < G * L; i += NT) {
        const int g = i / L, k = i % L;
        buf[g * P + lds_pad(k)] = src[(int64_t)g * L + k];
    }
    __syncthreads();
    const int g = threadIdx.x / (L / 16), lt = threadIdx.x % (L / 16);
    block_fft_lds<C, L, DIR>(buf + g * P, tw, lt);
    if (TRANSPOSE == 0) {
        C *dst = out + (b * rows + row0) * L;
        for (int i = threadIdx.x; i < G * L; i += NT) {
            const int gg = i / L, n = i % L;
            dst[(int64_t)gg * L + n] = buf[gg * P + lds_pad(n)];
        }
    } else {
        C *dst = out + b * rows * L;
        for (int i = threadIdx.x; i < G * L; i += NT) {
            const int gg = i % G, n = i / G;
            dst[(int64_t)n * rows + row0 + gg] = buf[gg * P + lds_pad(n)];
        }
    }
}

// First four-step pass, in place: data[b][k2][k1] (L2 rows of L1 columns);
// each workgroup takes G adjacent columns, transforms along k2 and multiplies
// by exp(DIR 2 pi i k1 n2 / (L1 L2)).
template <typename R, int L2, int G, int DIR>
__global__ void __launch_bounds__(G * L2 / 16)
k_fft_cols(cx_t<R> *__restrict__ data, int64_t L1, const cx_t<R> *__restrict__ tw_g,
           const cx_t<R> *__restrict__ hi, const cx_t<R> *__restrict__ lo)
{
    using C = cx_t<R>;
    constexpr int NT = G * L2 / 16;
    constexpr int P = fft_pitch_g(L2, G);
    __shared__ C buf[G * P];
    __shared__ C tw[L2];
    const int64_t b = blockIdx.y;
    const int64_t col0 = (int64_t)blockIdx.x * G;
    C *base = data + b * L1 * L2 + col0;
    load_tw<C, L2, DIR>(tw, tw_g);
    for (int i = threadIdx.x; i < G * L2; i += NT) {
        const int g = i % G, k2 = i / G;
        buf[g * P + lds_pad(k2)] = base[(int64_t)k2 * L1 + g];
    }
    __syncthreads();
    const int g = threadIdx.x / (L2 / 16), lt = threadIdx.x % (L2 / 16);
    block_fft_lds<C, L2, DIR>(buf + g * P, tw, lt);
    for (int i = threadIdx.x; i < G * L2; i += NT) {
        const int gg = i % G, n2 = i / G;
        const C w = twiddle_big<C, DIR>(hi, lo, (col0 + gg) * (int64_t)n2);
        base[(int64_t)n2 * L1 + gg] = cmul(buf[gg * P + lds_pad(n2)], w);
    }
}

// U[j][r] = u_r(X_j) = i^r exp(-i pi X_j) P_r(X_j / gamma) (Sec. 2.1.2), stored by the plan.
template <typename R>
__global__ void __launch_bounds__(256)
k_build_U(const R *__restrict__ X, int64_t M, Factors<R> fac, cx_t<R> *__restrict__ U)
{
    using C = cx_t<R>;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    const R Xj = X[j];
    R sn, cs;
    sincospi_r(Xj, &sn, &cs);
    const C E = cmake<C>(cs, -sn);
    const R z = Xj * fac.inv_gamma;
    for (int r = 0; r < fac.K; ++r) {
        const R p = upoly(fac, r, z);
        U[j * fac.K + r] = crot(cscale(E, p), r);
    }
}

// f_j = sum_r U[j][r] X_r[t_j]   (the gather I(t,:) and the row sum of Sec. 2.3).
// mode 1 writes gx_j = Re(conj(g_j) f_j) instead (derivative pass).
template <typename R>
__global__ void __launch_bounds__(256)
k_gather(const cx_t<R> *__restrict__ U, const cx_t<R> *__restrict__ Xr, const int32_t *__restrict__ t,
         int64_t M, int K, int64_t L, cx_t<R> *__restrict__ f, int mode, const cx_t<R> *__restrict__ g,
         double *__restrict__ gx)
{
    using C = cx_t<R>;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    const int64_t tj = t[j];
    C acc = cmake<C>(0, 0);
    for (int r = 0; r < K; ++r) acc = cadd(acc, cmul(U[j * K + r], Xr[(int64_t)r * L + tj]));
    if (mode == 0) f[j] = acc;
    else {
        const C gj = g[j];
        gx[j] = (double)(gj.x * acc.x + gj.y * acc.y);
    }
}

// ---- type I / adjoint (Sec. 3.1, the transpose of the two-step form) ---------
//   W_r[n] = sum_{j: t_j = n} u_r(j) c_j       (DIR = -1, type I)
//   W_r[n] = sum_{j: t_j = n} conj(u_r(j)) c_j (DIR = +1, adjoint)   -> k_spread
//   X_r = F_L W_r (DIR -1) or F_L^H W_r (DIR +1)  -> k_fft_cols / k_fft_rows
//   f_k = sum_r v_r(k) X_r[k], k < N             -> k_vsum
// One thread per grid point n sums the samples of its segment of the plan's
// sorted order (key (n mod L2) L1 + n / L2, CSR offsets off[]) in that order:
// a deterministic sum with no atomics; every W_r[n], n < L, is written.
template <typename R, int DIR>
__global__ void __launch_bounds__(256)
k_spread(const cx_t<R> *__restrict__ c, const int32_t *__restrict__ perm, const int32_t *__restrict__ off,
         const cx_t<R> *__restrict__ U, int K, int64_t L, int L1, int L2, cx_t<R> *__restrict__ W)
{
    using C = cx_t<R>;
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= L) return;
    const int64_t key = (n % L2) * L1 + n / L2;
    const int i0 = off[key], i1 = off[key + 1];
    C acc[NUFFT_KMAX];
#pragma unroll
    for (int r = 0; r < NUFFT_KMAX; ++r) acc[r] = cmake<C>(0, 0);
    for (int i = i0; i < i1; ++i) {
        const int64_t j = perm[i];
        const C cj = c[j];
#pragma unroll
        for (int r = 0; r < NUFFT_KMAX; ++r) {
            if (r < K) {
                const C u = U[j * K + r];
                acc[r] = cadd(acc[r], cmul(DIR < 0 ? u : cconj(u), cj));
            }
        }
    }
#pragma unroll
    for (int r = 0; r < NUFFT_KMAX; ++r)
        if (r < K) W[(int64_t)r * L + n] = acc[r];
}

// f_k = sum_r v_r(k) X[r][k], v_r(k) = T_r(2k/N - 1) (v_0 halved), k < N.
template <typename R>
__global__ void __launch_bounds__(256)
k_vsum(const cx_t<R> *__restrict__ X, int64_t N, int64_t L, int K, cx_t<R> *__restrict__ f)
{
    using C = cx_t<R>;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const R z = (R)(2.0 * (double)k / (double)N - 1.0);
    C acc = cmake<C>(0, 0);
    R tm2 = 1, tm1 = z;
    for (int r = 0; r < K; ++r) {
        R v;
        if (r == 0) v = (R)0.5;
        else if (r == 1) v = z;
        else { v = 2 * z * tm1 - tm2; tm2 = tm1; tm1 = v; }
        acc = cadd(acc, cscale(X[(int64_t)r * L + k], v));
    }
    f[k] = acc;
}

// ---- launchers --------------------------------------------------------------

template <typename R>
hipError_t plain_build_U(const R *X, int64_t M, const Factors<R> &fac, cx_t<R> *U, hipStream_t s)
{
    if (M == 0) return hipSuccess;
    hipLaunchKernelGGL(k_build_U<R>, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, X, M, fac, U);
    return hipGetLastError();
}

template <typename R, int L, int G, int DIR, int TR>
static void launch_rows(const cx_t<R> *in, cx_t<R> *out, int64_t rows, int64_t batch, const cx_t<R> *tw,
                        hipStream_t s)
{
    hipLaunchKernelGGL((k_fft_rows<R, L, G, DIR, TR>), dim3((unsigned)(rows / G), (unsigned)batch),
                       dim3(G * L / 16), 0, s, in, out, rows, tw);
}

template <typename R, int DIR, int TR>
static bool dispatch_rows(int L, const cx_t<R> *in, cx_t<R> *out, int64_t rows, int64_t batch,
                          const cx_t<R> *tw, hipStream_t s)
{
    // TR = 0 (one-pass transforms): one row per workgroup.  TR = 1 (second
    // four-step pass): G adjacent rows per workgroup so that the transposed
    // store writes G-element runs; G shrinks as rows grow (LDS budget).
    constexpr bool F = sizeof(R) == 4;
#define ROWS_CASE(LL, GF, GD)                                                                        \
    case LL: {                                                                                       \
        constexpr int G = TR == 0 ? 1 : (F ? GF : GD);                                               \
        if (rows % G) return false;                                                                  \
        launch_rows<R, LL, G, DIR, TR>(in, out, rows, batch, tw, s);                                 \
        return true;                                                                                 \
    }
    switch (L) {
        ROWS_CASE(16, 8, 4)
        ROWS_CASE(32, 8, 4)
        ROWS_CASE(64, 8, 4)
        ROWS_CASE(128, 8, 4)
        ROWS_CASE(256, 8, 4)
        ROWS_CASE(512, 8, 4)
        ROWS_CASE(1024, 8, 4)
        ROWS_CASE(2048, 4, 2)
        ROWS_CASE(4096, 2, 1)
    default: return false;
    }
#undef ROWS_CASE
}

template <typename R, int DIR>
static bool dispatch_cols(int L2, cx_t<R> *data, int64_t L1, int64_t batch, const cx_t<R> *tw,
                          const cx_t<R> *hi, const cx_t<R> *lo, hipStream_t s)
{
    constexpr bool F = sizeof(R) == 4;
#define COLS_CASE(LL, GF, GD)                                                                        \
    case LL: {                                                                                       \
        constexpr int G = F ? GF : GD;                                                               \
        hipLaunchKernelGGL((k_fft_cols<R, LL, G, DIR>), dim3((unsigned)(L1 / G), (unsigned)batch),   \
                           dim3(G * LL / 16), 0, s, data, L1, tw, hi, lo);                           \
        return true;                                                                                 \
    }
    switch (L2) {
        COLS_CASE(64, 8, 4)
        COLS_CASE(128, 8, 4)
        COLS_CASE(256, 8, 4)
        COLS_CASE(512, 8, 4)
        COLS_CASE(1024, 8, 4)
        COLS_CASE(2048, 8, 2)
    default: return false;
    }
#undef COLS_CASE
}

template <typename R>
hipError_t plain_exec(const PlainArgs<R> &a, hipStream_t s)
{
    using C = cx_t<R>;
    const int64_t L = a.L;
    prof_begin(a.prof, "plain_scale", s);
    hipLaunchKernelGGL(k_scale<R>, dim3((unsigned)((L + 255) / 256)), dim3(256), 0, s, a.c, a.N, L, a.K,
                       a.mode, a.W);
    prof_end(a.prof, s);
    bool ok;
    const C *spec;
    if (a.L2 == 1) {   // one-pass FFT of each row, in place
        prof_begin(a.prof, "plain_fft", s);
        ok = dispatch_rows<R, -1, 0>((int)L, a.W, a.W, 1, a.K, a.tw1, s);
        prof_end(a.prof, s);
        spec = a.W;
    } else {
        prof_begin(a.prof, "plain_fft_cols", s);
        ok = dispatch_cols<R, -1>(a.L2, a.W, a.L1, a.K, a.tw2, a.hi, a.lo, s);
        prof_end(a.prof, s);
        prof_begin(a.prof, "plain_fft_rows", s);
        ok = ok && dispatch_rows<R, -1, 1>(a.L1, a.W, a.W2, a.L2, a.K, a.tw1, s);
        prof_end(a.prof, s);
        spec = a.W2;
    }
    if (!ok) return hipErrorInvalidValue;
    if (a.M > 0) {
        prof_begin(a.prof, "plain_gather", s);
        hipLaunchKernelGGL(k_gather<R>, dim3((unsigned)((a.M + 255) / 256)), dim3(256), 0, s, a.U, spec,
                           a.t, a.M, a.K, L, a.f, a.mode, a.g, a.gx);
        prof_end(a.prof, s);
    }
    return hipGetLastError();
}

template <typename R, int DIR>
static hipError_t plain_type1_dir(const PlainT1Args<R> &a, hipStream_t s)
{
    using C = cx_t<R>;
    const int64_t L = a.L;
    prof_begin(a.prof, DIR > 0 ? "plain_adj_spread" : "plain_type1_spread", s);
    hipLaunchKernelGGL((k_spread<R, DIR>), dim3((unsigned)((L + 255) / 256)), dim3(256), 0, s, a.c, a.perm, a.off,
                       a.U, a.K, L, a.L1, a.L2, a.W);
    prof_end(a.prof, s);
    bool ok;
    const C *spec;
    // tables of the forward sign; the kernels conjugate them for DIR = +1
    if (a.L2 == 1) {
        prof_begin(a.prof, DIR > 0 ? "plain_adj_fft" : "plain_type1_fft", s);
        ok = dispatch_rows<R, DIR, 0>((int)L, a.W, a.W, 1, a.K, a.tw1, s);
        prof_end(a.prof, s);
        spec = a.W;
    } else {
        prof_begin(a.prof, DIR > 0 ? "plain_adj_fft_cols" : "plain_type1_fft_cols", s);
        ok = dispatch_cols<R, DIR>(a.L2, a.W, a.L1, a.K, a.tw2, a.hi, a.lo, s);
        prof_end(a.prof, s);
        prof_begin(a.prof, DIR > 0 ? "plain_adj_fft_rows" : "plain_type1_fft_rows", s);
        ok = ok && dispatch_rows<R, DIR, 1>(a.L1, a.W, a.W2, a.L2, a.K, a.tw1, s);
        prof_end(a.prof, s);
        spec = a.W2;
    }
    if (!ok) return hipErrorInvalidValue;
    prof_begin(a.prof, DIR > 0 ? "plain_adj_vsum" : "plain_type1_vsum", s);
    hipLaunchKernelGGL(k_vsum<R>, dim3((unsigned)((a.N + 255) / 256)), dim3(256), 0, s, spec, a.N, L, a.K, a.f);
    prof_end(a.prof, s);
    return hipGetLastError();
}

template <typename R>
hipError_t plain_type1(const PlainT1Args<R> &a, int sign, hipStream_t s)
{
    return sign < 0 ? plain_type1_dir<R, -1>(a, s) : plain_type1_dir<R, 1>(a, s);
}

template <typename R>
hipError_t plain_fft(int64_t L, int L1, int L2, cx_t<R> *data, cx_t<R> *out, const cx_t<R> *tw1,
                     const cx_t<R> *tw2, const cx_t<R> *hi, const cx_t<R> *lo, cx_t<R> **result, hipStream_t s)
{
    bool ok;
    if (L2 == 1) {
        ok = dispatch_rows<R, -1, 0>((int)L, data, data, 1, 1, tw1, s);
        *result = data;
    } else {
        ok = dispatch_cols<R, -1>(L2, data, L1, 1, tw2, hi, lo, s);
        ok = ok && dispatch_rows<R, -1, 1>(L1, data, out, L2, 1, tw1, s);
        *result = out;
    }
    if (!ok) return hipErrorInvalidValue;
    return hipGetLastError();
}

template hipError_t plain_fft<float>(int64_t, int, int, float2 *, float2 *, const float2 *, const float2 *,
                                     const float2 *, const float2 *, float2 **, hipStream_t);
template hipError_t plain_fft<double>(int64_t, int, int, double2 *, double2 *, const double2 *, const double2 *,
                                      const double2 *, const double2 *, double2 **, hipStream_t);
template hipError_t plain_build_U<float>(const float *, int64_t, const Factors<float> &, float2 *, hipStream_t);
template hipError_t plain_build_U<double>(const double *, int64_t, const Factors<double> &, double2 *,
                                          hipStream_t);
template hipError_t plain_exec<float>(const PlainArgs<float> &, hipStream_t);
template hipError_t plain_type1<float>(const PlainT1Args<float> &, int, hipStream_t);
template hipError_t plain_type1<double>(const PlainT1Args<double> &, int, hipStream_t);
template hipError_t plain_exec<double>(const PlainArgs<double> &, hipStream_t);

}  // namespace nufft
