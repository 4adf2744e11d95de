// Inverse type-II transform (Sec. 3.3): device helpers of the CG solver.
#pragma once

#include "kernels.h"

#define SOLVE_DOT_BLOCKS 512

namespace nufft {

template <typename R> hipError_t solve_fill(cx_t<R> *v, int64_t n, double re, double im, hipStream_t s);
template <typename R>
hipError_t solve_circulant_column(const cx_t<R> *tau, int64_t N, int64_t Lc, cx_t<R> *col, hipStream_t s);
template <typename R> hipError_t solve_pad(const cx_t<R> *p, int64_t N, int64_t Lc, cx_t<R> *out, hipStream_t s);
template <typename R> hipError_t solve_circulant_scale(cx_t<R> *q, const cx_t<R> *lam, int64_t Lc, hipStream_t s);
template <typename R> hipError_t solve_take_conj(const cx_t<R> *q, int64_t N, cx_t<R> *out, hipStream_t s);
// *out = sum_i conj(a_i) b_i in FP64 (part: SOLVE_DOT_BLOCKS partial sums)
template <typename R>
hipError_t solve_dot(const cx_t<R> *a, const cx_t<R> *b, int64_t n, double2 *part, double2 *out, hipStream_t s);
template <typename R>
hipError_t solve_step(cx_t<R> *x, cx_t<R> *r, const cx_t<R> *p, const cx_t<R> *ap, double alpha, int64_t n,
                      hipStream_t s);
template <typename R> hipError_t solve_direction(cx_t<R> *p, const cx_t<R> *r, double beta, int64_t n, hipStream_t s);

}  // namespace nufft
