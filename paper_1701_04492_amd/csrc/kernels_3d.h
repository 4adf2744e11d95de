// 3-D type II, type I and adjoint (Sec. 4's construction with a third axis): device launchers.
#pragma once

#include "kernels.h"

namespace nufft {

// t = round(Gz z) mod Gz and X = (Gz z - round(Gz z)) n3 / Gz per sample; max |X| into gbits
// (bits of a non-negative double); flags |= 1 for a non-finite z.
template <typename R>
hipError_t launch_3d_assign(const double *z, int64_t M, int64_t n3, int64_t Gz, int32_t *t, R *X,
                            unsigned long long *gbits, int *flags, hipStream_t s);
// D[m * rows + row] = sum_{k3 < n3} v_r(k3) Cin[row * n3 + k3] exp(-2 pi i k3 m / Gz), m < Gz (16..1024);
// tw: the stage-major length-Gz twiddle table
template <typename R>
hipError_t launch_3d_zfft(const cx_t<R> *Cin, int64_t rows, int64_t n3, int64_t Gz, int r, const cx_t<R> *tw,
                          cx_t<R> *D, hipStream_t s);
// f[j] = (r == 0 ? 0 : f[j]) + u_r(Xz[j]) fs[j]
template <typename R>
hipError_t launch_3d_accum(const cx_t<R> *fs, const R *Xz, int64_t M, const Factors<R> &fac, int r, cx_t<R> *f,
                           hipStream_t s);
// cw[j] = w_r(j) c[j], w_r = u^z_r (sign -1) or its conjugate (sign +1), j < M
template <typename R>
hipError_t launch_3d_weight(const cx_t<R> *c, const R *Xz, int64_t M, const Factors<R> &fac, int r, int sign,
                            cx_t<R> *cw, hipStream_t s);
// Cout[row * n3 + k3] (r == 0 ? = : +=) v_r(k3) sum_{m < Gz} E[m * rows + row] exp(sign 2 pi i k3 m / Gz),
// k3 < n3; tw: the stage-major length-Gz table of the -1 direction
template <typename R>
hipError_t launch_3d_zfft_t(const cx_t<R> *E, int64_t rows, int64_t n3, int64_t Gz, int r, int sign,
                            const cx_t<R> *tw, cx_t<R> *Cout, hipStream_t s);

}  // namespace nufft
