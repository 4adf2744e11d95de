// Host FP64 factor generator (Sec. 2.1.2, Table 1, Lemma A.1).
#pragma once

#include <stdint.h>

#include "common.h"

namespace nufft {

// J_n(z), integer n, |z| <= pi/4 (the range -gamma pi/2 covers).
double bessel_jn(int n, double z);

// b[p*size + r] = a_pr / i^r (real): 4 J_{(p+r)/2}(-gamma pi/2) J_{(r-p)/2}(-gamma pi/2), p = r mod 2.
void bessel_b(double gamma, int size, double *b);

// Smallest K whose truncation tail sum_{max(p,r)>=K} w_p w_r |a_pr| is <= eps
// (w_0 = 1/2); 1 when gamma = 0; -1 if no K <= NUFFT_KMAX suffices.
int choose_rank(double eps, double gamma);

// mono[r*K + m]: coefficient of z^m in P_r(z) = sum'_{p<K} b_pr T_p(z).
void u_monomials(double gamma, int K, double *mono);

// (cos, sin)(2 pi m / L), octant-reduced.
void cis_2pi_frac(int64_t m, int64_t L, double *c, double *s);

// out[2i], out[2i+1] = exp(dir 2 pi i (i*step) / L) for i < count.
void twiddles(int64_t L, int64_t count, int64_t step, int dir, double *out);
// FFT stage twiddles of a length-L transform (L a power of two, 16..4096), in
// the stage-major order the LDS FFT reads for first radix r0 (16 or 8); L entries.
void fft_twiddles(int64_t L, int dir, double *out, int r0 = 16);

}  // namespace nufft
