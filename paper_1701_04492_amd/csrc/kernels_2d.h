// 2-D type II (Sec. 4): arguments and launchers.
#pragma once

#include "kernels.h"

namespace nufft {

template <typename R>
struct Args2D {
    int64_t N1, N2, M;        // coefficient rows (x, k1), columns (y, k2), samples
    int Gx, Gy;               // FFT grids of the two axes (powers of two >= 16)
    int S;                    // problems stacked in the plan (1: a plain 2-D plan); coefficient
                              // arrays S x N1 x N2 back to back, sample j in problem slice[j]
    Factors<R> fx, fy;        // rank factors of the two axes
    const uint32_t *keys;     // M sorted keys (slice * Gy + ty) * Gx + tx
    const int32_t *perm;      // M sample index per sorted position
    const R *Xxs, *Xys;       // M sorted perturbations of the two axes
    const int32_t *off;       // S * Gx * Gy + 1 first sorted position per key
    const int4 *tasks;        // forward pass-B tasks (column slice * Gy + n2, first, end)
    int ntasks;
    const int4 *atasks;       // adjoint pass-B' tasks (column, first, end, partial slot or -1)
    int natasks;
    const int4 *rtasks;       // split columns (column, first slot, slots)
    int nrtasks;
    cx_t<R> *Zp;              // partial rows of split columns: slots x Ky x Gx
    cx_t<R> *H;               // Ky x (S Gy) x Gx intermediate [r2][slice * Gy + n2][k1]
    const cx_t<R> *twx, *twxi, *twy, *twyi;   // FFT tables, both signs
    Profiler *prof;
};

template <typename R>
hipError_t fused_2d(const Args2D<R> &a, const cx_t<R> *Cin, cx_t<R> *f, hipStream_t s);
// sign = +1: the adjoint, C = sum_j g_j exp(+2 pi i (k1 x_j + k2 y_j));
// sign = -1: the 2-D type I, C = sum_j g_j exp(-2 pi i (k1 x_j + k2 y_j)).
template <typename R>
hipError_t fused_2d_adj(const Args2D<R> &a, const cx_t<R> *gin, cx_t<R> *Cout, int sign, hipStream_t s);
int pass_b2d_cap(int GX, bool fp32);
int pass_b2d_adj_cap(int GX, bool fp32);
template <typename R>
hipError_t launch_assign2d(const double *x, const double *y, const int32_t *slice, int64_t M, int64_t GX,
                           int64_t GY, double sx, double sy, R *Xx, R *Xy, uint32_t *key, int32_t *hist,
                           unsigned long long *gbits, int *bad, hipStream_t s);

}  // namespace nufft
