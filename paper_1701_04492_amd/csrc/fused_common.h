// Device helpers shared by the fused kernels (1-D, 2-D, batched).
#pragma once

#include "fft.h"
#include "kernels.h"

namespace nufft {

template <typename C, int L, int DIR>
__device__ __forceinline__ void load_tw_s(C *tw_s, const C *__restrict__ tw_g)
{
    for (int m = threadIdx.x; m < L; m += blockDim.x) {
        C w = tw_g[m];
        tw_s[m] = DIR < 0 ? w : cconj(w);
    }
}

template <typename C, int DIR>
__device__ __forceinline__ C tw_big(const C *__restrict__ hi, const C *__restrict__ lo, int64_t m)
{
    C w = cmul(hi[m >> 12], lo[m & 4095]);
    return DIR < 0 ? w : cconj(w);
}

// T_r(z) (v_0 = 1/2 is the halved T_0) by the three-term recurrence.
template <typename R>
__device__ __forceinline__ R cheb_v(int r, R z)
{
    if (r == 0) return (R)0.5;
    R a = 1, b = z;
    for (int q = 1; q < r; ++q) {
        const R c = 2 * z * b - a;
        a = b;
        b = c;
    }
    return b;
}

// c_k, or -2 pi i k c_k for the derivative pass.
template <typename R>
__device__ __forceinline__ cx_t<R> load_coef(const cx_t<R> *__restrict__ c, int64_t k, int64_t N, int mode)
{
    using C = cx_t<R>;
    if (k >= N) return cmake<C>(0, 0);
    C ck = c[k];
    if (mode == 1) {
        const R w = (R)(-2.0 * M_PI * (double)k);
        ck = cmake<C>(-w * ck.y, w * ck.x);
    }
    return ck;
}

template <typename R>
__device__ __forceinline__ R zcoord(int64_t k, int64_t N)
{
    return (R)(2.0 * (double)k / (double)N - 1.0);
}

// Workgroups are dispatched to the eight XCDs round robin (block b runs on
// XCD b mod 8).  Renumbering the tasks so that consecutive tasks share an
// XCD lets neighbouring tasks hit the same L2 (the column block of c read by
// every rank chunk of pass A; the halves of a cache line written by
// neighbouring tiles).  The grid is 8 * ceil(T / 8); surplus blocks return.
__device__ __forceinline__ int xcd_task(int T)
{
    const int per = (T + 7) >> 3;
    const int b = blockIdx.x;
    const int task = (b & 7) * per + (b >> 3);
    return task < T ? task : -1;
}

static inline unsigned xcd_grid(int T) { return (unsigned)(8 * ((T + 7) / 8)); }

}  // namespace nufft
