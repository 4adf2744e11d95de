// Shared types and helpers of the MI355X low-rank NUFFT library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nufft_mi355x.h"

// Complex element type per real type: interleaved (re, im).
template <typename R> struct cx;
template <> struct cx<float> { using T = float2; };
template <> struct cx<double> { using T = double2; };
template <typename R> using cx_t = typename cx<R>::T;

template <typename C>
__host__ __device__ __forceinline__ C cmake(decltype(C{}.x) a, decltype(C{}.x) b) { C r; r.x = a; r.y = b; return r; }

template <typename C>
__device__ __forceinline__ C cadd(C a, C b) { return cmake<C>(a.x + b.x, a.y + b.y); }
template <typename C>
__device__ __forceinline__ C csub(C a, C b) { return cmake<C>(a.x - b.x, a.y - b.y); }
template <typename C>
__device__ __forceinline__ C cmul(C a, C b) { return cmake<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
template <typename C>
__device__ __forceinline__ C cconj(C a) { return cmake<C>(a.x, -a.y); }
template <typename C, typename R>
__device__ __forceinline__ C cscale(C a, R s) { return cmake<C>(a.x * s, a.y * s); }

// a * i^q for a compile-time or uniform quarter-turn count q (mod 4).
template <typename C>
__device__ __forceinline__ C crot(C a, int q)
{
    switch (q & 3) {
    case 0: return a;
    case 1: return cmake<C>(-a.y, a.x);
    case 2: return cmake<C>(-a.x, -a.y);
    default: return cmake<C>(a.y, -a.x);
    }
}

// Largest rank the kernels support (K <= 20 covers eps down to ~1e-16 at gamma = 1/2).
#define NUFFT_KMAX 20
// Per-rank coefficient row length in the u-polynomial table: the polynomial
// sum'_p b_pr T_p(z) keeps only powers of the parity of r, written in w = z^2.
#define NUFFT_UCOEF_STRIDE 12

// Factors of the rank-K approximation, uploaded by the plan (device copy).
//   u_r(X) = i^r exp(-i pi X) sum_m ucoef[r][m] z^(2m + (r&1)),  z = X / gamma
//   v_r(k) = T_r(2k/N - 1), v_0 halved
template <typename R>
struct Factors {
    R ucoef[NUFFT_KMAX * NUFFT_UCOEF_STRIDE];
    int nterm[NUFFT_KMAX];   // number of w-coefficients of rank r
    int K;
    R inv_gamma;             // 1/gamma, or 0 when gamma == 0
};

// Optional per-kernel timing: when enabled on a plan, a pair of HIP events is
// recorded on the launch stream around every kernel of an exec call.
struct Profiler;
void prof_begin(Profiler *p, const char *name, hipStream_t s);
void prof_end(Profiler *p, hipStream_t s);

#define NUFFT_HIP_CHECK(expr)                                   \
    do {                                                        \
        hipError_t _e = (expr);                                 \
        if (_e != hipSuccess) return NUFFT_ERR_HIP;             \
    } while (0)
