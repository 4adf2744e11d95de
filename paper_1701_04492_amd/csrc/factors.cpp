// Host FP64 factor generator: Bessel coefficients, the rank K(eps, gamma),
// the u-polynomials in monomial form, and FFT twiddle tables.
//
// Sec. 2.1.2 / Lemma A.1: on [-gamma, gamma] x [0, 2 pi]
//   exp(-i X Y) = sum'_p sum'_r a_pr exp(-i pi X) T_p(X/gamma) T_r(Y/pi - 1),
//   a_pr = 4 i^r J_{(p+r)/2}(-gamma pi/2) J_{(r-p)/2}(-gamma pi/2) for p = r (mod 2), else 0,
// primes halving the first term.  With X = N(x_j - s_j/L) and Y = 2 pi k / N
// this gives the rank-K factors u_r(X) v_r(k) of A_jk (Sec. 2.2).
#include "factors.h"

#include <cmath>
#include <cstring>

namespace nufft {

// J_n(z) for integer n and |z| <= pi/4 by its power series
// J_n(z) = sum_m (-1)^m (z/2)^(2m+n) / (m! (m+n)!): for such z the terms
// decrease from the first one on, so the sum has no cancellation.
double bessel_jn(int n, double z)
{
    if (n < 0) return (n & 1) ? -bessel_jn(-n, z) : bessel_jn(-n, z);
    const double h = 0.5 * z;
    double lead = 1.0;                      // (z/2)^n / n!
    for (int i = 1; i <= n; ++i) lead *= h / i;
    if (lead == 0.0) return 0.0;
    double term = lead, sum = lead;
    const double h2 = h * h;
    for (int m = 1; m < 60; ++m) {
        term *= -h2 / ((double)m * (double)(m + n));
        sum += term;
        if (std::fabs(term) <= 1e-18 * std::fabs(sum)) break;
    }
    return sum;
}

void bessel_b(double gamma, int size, double *b)
{
    const double z = -gamma * M_PI / 2.0;
    for (int p = 0; p < size; ++p)
        for (int r = 0; r < size; ++r) {
            double v = 0.0;
            if (((p + r) & 1) == 0) v = 4.0 * bessel_jn((p + r) / 2, z) * bessel_jn((r - p) / 2, z);
            b[p * size + r] = v;
        }
}

static const int kTail = 64;

int choose_rank(double eps, double gamma)
{
    if (gamma == 0.0) return 1;
    static thread_local double wa[kTail * kTail];
    bessel_b(gamma, kTail, wa);
    double total = 0.0;
    for (int p = 0; p < kTail; ++p)
        for (int r = 0; r < kTail; ++r) {
            double w = (p == 0 ? 0.5 : 1.0) * (r == 0 ? 0.5 : 1.0);
            wa[p * kTail + r] = w * std::fabs(wa[p * kTail + r]);
            total += wa[p * kTail + r];
        }
    // tail(K) = total - sum_{p,r<K}: grow the leading block one row+column at a time
    double head = 0.0;
    for (int K = 1; K <= NUFFT_KMAX; ++K) {
        const int k = K - 1;
        for (int i = 0; i < k; ++i) head += wa[i * kTail + k] + wa[k * kTail + i];
        head += wa[k * kTail + k];
        if (total - head <= eps) return K;
    }
    return -1;
}

void u_monomials(double gamma, int K, double *mono /*[K][K]*/)
{
    // P_r(z) = sum'_p b_pr T_p(z) in powers of z; T_p coefficients by T_{p+1} = 2 z T_p - T_{p-1}.
    double b[NUFFT_KMAX * NUFFT_KMAX];
    bessel_b(gamma, K, b);
    double T[NUFFT_KMAX][NUFFT_KMAX];
    std::memset(T, 0, sizeof(T));
    T[0][0] = 1.0;
    if (K > 1) T[1][1] = 1.0;
    for (int p = 2; p < K; ++p)
        for (int m = 0; m < K; ++m)
            T[p][m] = (m > 0 ? 2.0 * T[p - 1][m - 1] : 0.0) - T[p - 2][m];
    for (int r = 0; r < K; ++r)
        for (int m = 0; m < K; ++m) {
            double s = 0.0;
            for (int p = 0; p < K; ++p) s += (p == 0 ? 0.5 : 1.0) * b[p * K + r] * T[p][m];
            mono[r * K + m] = s;
        }
}

// cos/sin of 2 pi m / L: whole quarter turns are taken out exactly, the
// remaining angle (below pi/2) goes to libm.
void cis_2pi_frac(int64_t m, int64_t L, double *c, double *s)
{
    m %= L;
    if (m < 0) m += L;
    const int64_t q = (4 * m) / L;                           // quarter turns
    const double f = (double)(4 * m - q * L) / (double)L;    // in [0, 1), exact for L <= 2^50
    double cf = 1.0, sf = 0.0;
    if (f != 0.0) { cf = std::cos(f * (M_PI / 2.0)); sf = std::sin(f * (M_PI / 2.0)); }
    switch (q & 3) {
    case 0: *c = cf;  *s = sf;  break;
    case 1: *c = -sf; *s = cf;  break;
    case 2: *c = -cf; *s = -sf; break;
    default: *c = sf; *s = -cf; break;
    }
}

void fft_twiddles(int64_t L, int dir, double *out, int r0)
{
    const int64_t P = L % 3 == 0 ? 3 : (L % 5 == 0 ? 5 : 1);
    if (P > 1) {
        // mixed length P Q: the Q-point table, then the radix-P stage's
        // exp(dir 2 pi i s m / L) at Q + (s - 1) Q + m, 1 <= s < P, m < Q
        const int64_t Q = L / P;
        fft_twiddles(Q, dir, out, r0);
        for (int64_t sj = 1; sj < P; ++sj)
            for (int64_t m = 0; m < Q; ++m) {
                double c, s;
                cis_2pi_frac(sj * m, L, &c, &s);
                out[2 * (Q + (sj - 1) * Q + m)] = c;
                out[2 * (Q + (sj - 1) * Q + m) + 1] = dir * s;
            }
        return;
    }
    // Stage-major layout read by the LDS FFT: the stage that combines NS-point
    // transforms with radix R keeps exp(dir 2 pi i q k / (NS R)), 0 <= k < NS,
    // 1 <= q < R, at NS - 1 + k (R - 1) + q - 1 (the stages tile [0, L - 1)).
    // Consecutive k are R - 1 elements apart: an odd stride, so the lanes of a
    // wave read different LDS banks.
    out[2 * (L - 1)] = 1.0;   // entry L - 1 is unused
    out[2 * (L - 1) + 1] = 0.0;
    for (int64_t NS = 1; NS < L;) {
        // the stage radices of the LDS FFT: r0 first, then 16 while possible, then the remainder
        const int64_t R = NS == 1 ? (r0 < L ? r0 : L) : (L / NS >= 16) ? 16 : L / NS;
        for (int64_t k = 0; k < NS; ++k)
            for (int64_t q = 1; q < R; ++q) {
                double c, s;
                cis_2pi_frac(q * k, NS * R, &c, &s);
                const int64_t m = NS - 1 + k * (R - 1) + q - 1;
                out[2 * m] = c;
                out[2 * m + 1] = dir * s;
            }
        NS *= R;
    }
}

void twiddles(int64_t L, int64_t count, int64_t step, int dir, double *out)
{
    for (int64_t m = 0; m < count; ++m) {
        double c, s;
        cis_2pi_frac(m * step, L, &c, &s);
        out[2 * m] = c;
        out[2 * m + 1] = dir * s;
    }
}

}  // namespace nufft
