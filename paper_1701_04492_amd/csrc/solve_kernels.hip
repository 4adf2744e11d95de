// Device pieces of the inverse type-II transform (Sec. 3.3): conjugate
// gradients on the normal equations F2^* F2 c = F2^* f, whose matrix is
// Hermitian Toeplitz with first column tau_m = sum_p exp(2 pi i x_p m).  The
// product with it goes through the circulant matrix of size Lc >= 2N whose
// first column is [tau_0 .. tau_{N-1}, 0 .., conj(tau_{N-1}) .. conj(tau_1)]:
// T c = first N entries of IDFT(DFT(col) o DFT([c, 0])), with the inverse DFT
// written as a forward one between two conjugations.
#include "solve.h"

namespace nufft {

template <typename R>
__global__ void __launch_bounds__(256) k_fill(cx_t<R> *__restrict__ v, int64_t n, R re, R im)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = cmake<cx_t<R>>(re, im);
}

template <typename R>
__global__ void __launch_bounds__(256)
k_circulant_column(const cx_t<R> *__restrict__ tau, int64_t N, int64_t Lc, cx_t<R> *__restrict__ col)
{
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= Lc) return;
    cx_t<R> v = cmake<cx_t<R>>(0, 0);
    if (m < N) v = tau[m];
    else if (Lc - m < N) v = cconj(tau[Lc - m]);
    col[m] = v;
}

template <typename R>
__global__ void __launch_bounds__(256)
k_pad(const cx_t<R> *__restrict__ p, int64_t N, int64_t Lc, cx_t<R> *__restrict__ out)
{
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m < Lc) out[m] = m < N ? p[m] : cmake<cx_t<R>>(0, 0);
}

// q <- conj(lam o q) / Lc (the middle of IDFT(lam o DFT(.)) as a forward DFT)
template <typename R>
__global__ void __launch_bounds__(256)
k_circulant_scale(cx_t<R> *__restrict__ q, const cx_t<R> *__restrict__ lam, int64_t Lc)
{
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= Lc) return;
    const R s = (R)(1.0 / (double)Lc);
    const cx_t<R> v = cmul(lam[m], q[m]);
    q[m] = cmake<cx_t<R>>(v.x * s, -v.y * s);
}

template <typename R>
__global__ void __launch_bounds__(256)
k_take_conj(const cx_t<R> *__restrict__ q, int64_t N, cx_t<R> *__restrict__ out)
{
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m < N) out[m] = cconj(q[m]);
}

// partial sums of conj(a) b (FP64), one per workgroup, then their sum in block 0
// of a second launch: a fixed reduction order.
template <typename R>
__global__ void __launch_bounds__(256)
k_dot_partial(const cx_t<R> *__restrict__ a, const cx_t<R> *__restrict__ b, int64_t n, double2 *__restrict__ part)
{
    __shared__ double sr[256], si[256];
    double re = 0, im = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double ax = a[i].x, ay = a[i].y, bx = b[i].x, by = b[i].y;
        re += ax * bx + ay * by;
        im += ax * by - ay * bx;
    }
    sr[threadIdx.x] = re;
    si[threadIdx.x] = im;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sr[threadIdx.x] += sr[threadIdx.x + w];
            si[threadIdx.x] += si[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = make_double2(sr[0], si[0]);
}

__global__ void __launch_bounds__(256) k_dot_final(const double2 *__restrict__ part, int n, double2 *__restrict__ out)
{
    __shared__ double sr[256], si[256];
    double re = 0, im = 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        re += part[i].x;
        im += part[i].y;
    }
    sr[threadIdx.x] = re;
    si[threadIdx.x] = im;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sr[threadIdx.x] += sr[threadIdx.x + w];
            si[threadIdx.x] += si[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = make_double2(sr[0], si[0]);
}

// x += alpha p, r -= alpha Ap
template <typename R>
__global__ void __launch_bounds__(256)
k_cg_step(cx_t<R> *__restrict__ x, cx_t<R> *__restrict__ r, const cx_t<R> *__restrict__ p,
          const cx_t<R> *__restrict__ ap, double alpha, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const R a = (R)alpha;
    x[i] = cmake<cx_t<R>>(x[i].x + a * p[i].x, x[i].y + a * p[i].y);
    r[i] = cmake<cx_t<R>>(r[i].x - a * ap[i].x, r[i].y - a * ap[i].y);
}

// p = r + beta p
template <typename R>
__global__ void __launch_bounds__(256)
k_cg_direction(cx_t<R> *__restrict__ p, const cx_t<R> *__restrict__ r, double beta, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const R b = (R)beta;
    p[i] = cmake<cx_t<R>>(r[i].x + b * p[i].x, r[i].y + b * p[i].y);
}

static inline dim3 blocks_for(int64_t n) { return dim3((unsigned)((n + 255) / 256)); }

template <typename R>
hipError_t solve_fill(cx_t<R> *v, int64_t n, double re, double im, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill<R>, blocks_for(n), dim3(256), 0, s, v, n, (R)re, (R)im);
    return hipGetLastError();
}

template <typename R>
hipError_t solve_circulant_column(const cx_t<R> *tau, int64_t N, int64_t Lc, cx_t<R> *col, hipStream_t s)
{
    hipLaunchKernelGGL(k_circulant_column<R>, blocks_for(Lc), dim3(256), 0, s, tau, N, Lc, col);
    return hipGetLastError();
}

template <typename R>
hipError_t solve_pad(const cx_t<R> *p, int64_t N, int64_t Lc, cx_t<R> *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_pad<R>, blocks_for(Lc), dim3(256), 0, s, p, N, Lc, out);
    return hipGetLastError();
}

template <typename R>
hipError_t solve_circulant_scale(cx_t<R> *q, const cx_t<R> *lam, int64_t Lc, hipStream_t s)
{
    hipLaunchKernelGGL(k_circulant_scale<R>, blocks_for(Lc), dim3(256), 0, s, q, lam, Lc);
    return hipGetLastError();
}

template <typename R>
hipError_t solve_take_conj(const cx_t<R> *q, int64_t N, cx_t<R> *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_take_conj<R>, blocks_for(N), dim3(256), 0, s, q, N, out);
    return hipGetLastError();
}

template <typename R>
hipError_t solve_dot(const cx_t<R> *a, const cx_t<R> *b, int64_t n, double2 *part, double2 *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_dot_partial<R>, dim3(SOLVE_DOT_BLOCKS), dim3(256), 0, s, a, b, n, part);
    hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(256), 0, s, (const double2 *)part, SOLVE_DOT_BLOCKS, out);
    return hipGetLastError();
}

template <typename R>
hipError_t solve_step(cx_t<R> *x, cx_t<R> *r, const cx_t<R> *p, const cx_t<R> *ap, double alpha, int64_t n,
                      hipStream_t s)
{
    hipLaunchKernelGGL(k_cg_step<R>, blocks_for(n), dim3(256), 0, s, x, r, p, ap, alpha, n);
    return hipGetLastError();
}

template <typename R>
hipError_t solve_direction(cx_t<R> *p, const cx_t<R> *r, double beta, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_cg_direction<R>, blocks_for(n), dim3(256), 0, s, p, r, beta, n);
    return hipGetLastError();
}

#define SOLVE_INST(R)                                                                                         \
    template hipError_t solve_fill<R>(cx_t<R> *, int64_t, double, double, hipStream_t);                       \
    template hipError_t solve_circulant_column<R>(const cx_t<R> *, int64_t, int64_t, cx_t<R> *, hipStream_t); \
    template hipError_t solve_pad<R>(const cx_t<R> *, int64_t, int64_t, cx_t<R> *, hipStream_t);              \
    template hipError_t solve_circulant_scale<R>(cx_t<R> *, const cx_t<R> *, int64_t, hipStream_t);           \
    template hipError_t solve_take_conj<R>(const cx_t<R> *, int64_t, cx_t<R> *, hipStream_t);                 \
    template hipError_t solve_dot<R>(const cx_t<R> *, const cx_t<R> *, int64_t, double2 *, double2 *,         \
                                     hipStream_t);                                                            \
    template hipError_t solve_step<R>(cx_t<R> *, cx_t<R> *, const cx_t<R> *, const cx_t<R> *, double,         \
                                      int64_t, hipStream_t);                                                  \
    template hipError_t solve_direction<R>(cx_t<R> *, const cx_t<R> *, double, int64_t, hipStream_t);
SOLVE_INST(float)
SOLVE_INST(double)
#undef SOLVE_INST

}  // namespace nufft
