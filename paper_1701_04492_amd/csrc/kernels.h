// Internal declarations shared by the kernel translation units and the C ABI.
#pragma once

#include "common.h"

namespace nufft {

__device__ __forceinline__ void sincospi_r(float x, float *s, float *c) { sincospif(x, s, c); }
__device__ __forceinline__ void sincospi_r(double x, double *s, double *c) { sincospi(x, s, c); }

// P_r(z) = sum'_p b_pr T_p(z), evaluated from its monomial form: only powers
// of the parity of r occur, so P_r(z) = z^(r&1) * Q_r(z^2) with Q_r by Horner.
template <typename R>
__device__ __forceinline__ R upoly(const Factors<R> &fac, int r, R z)
{
    const R w = z * z;
    const R *cf = fac.ucoef + r * NUFFT_UCOEF_STRIDE;
    const int n = fac.nterm[r];
    R acc = cf[n - 1];
    for (int m = n - 2; m >= 0; --m) acc = acc * w + cf[m];
    return (r & 1) ? acc * z : acc;
}

// The same polynomial for one rank r that is uniform across the workgroup,
// with its coefficients loaded once into registers and reused for every
// sample (a per-term load inside the evaluation would wait for each term).
// A rank of K has at most ceil(K / 2) terms and the table is zero past
// nterm[r]: a fixed-length Horner chain over the first rank_terms<R>
// coefficients gives the same value with no branch or select.  FP32 plans
// have K <= NUFFT_KMAX_F32 (eps >= 1e-7, or 5e-8 per axis in 2-D, gives
// K <= 12 at gamma = 1/2; the plan builders reject more), so 6 terms; FP64
// plans use the full NUFFT_KMAX / 2.
#define NUFFT_KMAX_F32 12
template <typename R>
inline constexpr int rank_terms = sizeof(R) == 4 ? NUFFT_KMAX_F32 / 2 : NUFFT_KMAX / 2;
template <typename R>
struct RankPoly {
    R c[rank_terms<R>];
    int odd;
};
template <typename R>
__device__ __forceinline__ RankPoly<R> rank_poly(const Factors<R> &fac, int r)
{
    RankPoly<R> p;
#pragma unroll
    for (int m = 0; m < rank_terms<R>; ++m) p.c[m] = fac.ucoef[r * NUFFT_UCOEF_STRIDE + m];
    p.odd = r & 1;
    return p;
}
template <typename R>
__device__ __forceinline__ R rank_eval(const RankPoly<R> &p, R z)
{
    const R w = z * z;
    R acc = p.c[rank_terms<R> - 1];
#pragma unroll
    for (int m = rank_terms<R> - 2; m >= 0; --m) acc = acc * w + p.c[m];
    return p.odd ? acc * z : acc;
}

// rank_eval with the rank's parity given by the caller (a compile-time
// constant where the caller's rank index is, as for the ranks of an unrolled
// chunk that starts at an even rank)
template <typename R>
__device__ __forceinline__ R rank_eval_par(const RankPoly<R> &p, R z, bool odd)
{
    const R w = z * z;
    R acc = p.c[rank_terms<R> - 1];
#pragma unroll
    for (int m = rank_terms<R> - 2; m >= 0; --m) acc = acc * w + p.c[m];
    return odd ? acc * z : acc;
}

// Same polynomial from a coefficient table staged in LDS: for kernels where the
// rank differs between the lanes of a wave (a per-lane index into the
// kernel-argument table would turn every coefficient into a vector load).
template <typename R>
__device__ __forceinline__ R upoly_lds(const R *ucoef_s, const int *nterm_s, int r, R z)
{
    const R w = z * z;
    const R *cf = ucoef_s + r * NUFFT_UCOEF_STRIDE;
    const int n = nterm_s[r];
    R acc = cf[n - 1];
    for (int m = n - 2; m >= 0; --m) acc = acc * w + cf[m];
    return (r & 1) ? acc * z : acc;
}

template <typename R>
__device__ __forceinline__ void stage_factors(const Factors<R> &fac, R *ucoef_s, int *nterm_s)
{
    for (int i = threadIdx.x; i < NUFFT_KMAX * NUFFT_UCOEF_STRIDE; i += blockDim.x) ucoef_s[i] = fac.ucoef[i];
    for (int i = threadIdx.x; i < NUFFT_KMAX; i += blockDim.x) nterm_s[i] = fac.nterm[i];
}

// ---- plan kernels ----------------------------------------------------------
template <typename R>
hipError_t launch_assign(const double *x, int64_t M, int64_t L, double n_over_L, int L1, int L2,
                         int32_t *t, R *X, uint32_t *key, int32_t *hist, unsigned long long *gbits,
                         int *bad, hipStream_t s);
template <typename R>
hipError_t launch_gather_sorted(const int32_t *perm, const R *X, int64_t n, R *Xs, hipStream_t s);
hipError_t launch_iota(int32_t *v, int64_t n, hipStream_t s);
// out[i] = in[i * stride], i < n
hipError_t launch_strided_i32(const int32_t *in, int64_t stride, int64_t n, int32_t *out, hipStream_t s);
hipError_t launch_invert_perm(const int32_t *perm, int64_t n, int32_t *sinv, hipStream_t s);
// The destination-bucketed layout of the sample permutation (blocks of 2^shift
// samples): bdst[i] is sorted position i's place in the layout ordered by
// (bucket perm[i] >> shift, i), lidx[p] = perm[i] mod 2^shift of the sample at
// place p.  keys, vals, keys_alt, vals_alt (n each) and tmp (radix_tmp_elems(n)) are scratch.
hipError_t launch_bucket_maps(const int32_t *perm, int64_t n, int shift, uint32_t *keys, int32_t *vals,
                              uint32_t *keys_alt, int32_t *vals_alt, int32_t *tmp, int32_t *bdst, uint16_t *lidx,
                              hipStream_t s);
hipError_t exclusive_scan(const int32_t *in, int32_t *out, int64_t n, int32_t *tmp, hipStream_t s);
int64_t scan_tmp_elems(int64_t n);
int64_t radix_tmp_elems(int64_t n);
hipError_t radix_sort_pairs(uint32_t *keys, int32_t *vals, uint32_t *keys_alt, int32_t *vals_alt,
                            int64_t n, int key_bits, int32_t *tmp, hipStream_t s,
                            uint32_t **keys_sorted, int32_t **vals_sorted);

// ---- plain (unfused) online stage -------------------------------------------
template <typename R>
struct PlainArgs {
    const cx_t<R> *c;      // N coefficients
    int64_t N, L, M;
    int L1, L2;            // L = L1 * L2; L2 == 1 means one-pass FFTs of length L
    int K, mode;           // mode 0: f = F2 c; mode 1: gx = Re(conj(g) F2(-2 pi i k c))
    cx_t<R> *W, *W2;       // K x L work buffers
    const cx_t<R> *tw1, *tw2, *hi, *lo;   // twiddle tables (forward sign)
    const cx_t<R> *U;      // M x K stored factors
    const int32_t *t;      // M grid indices
    cx_t<R> *f;            // M outputs (mode 0)
    const cx_t<R> *g;      // M upstream gradients (mode 1)
    double *gx;            // M outputs (mode 1)
    Profiler *prof;
};

// Plain type I / adjoint (Sec. 3.1): spread into W (K x L), stand-alone FFT
// passes (W2: second four-step buffer), weighted sum over r into f (N).
template <typename R>
struct PlainT1Args {
    const cx_t<R> *c;      // M inputs
    int64_t N, L, M;
    int L1, L2, K;
    const int32_t *perm, *off;   // the plan's sorted order and its CSR offsets per key
    const cx_t<R> *U;      // M x K stored factors
    cx_t<R> *W, *W2;
    const cx_t<R> *tw1, *tw2, *hi, *lo;   // forward-sign tables
    cx_t<R> *f;            // N outputs
    Profiler *prof;
};
template <typename R>
hipError_t plain_type1(const PlainT1Args<R> &a, int sign, hipStream_t s);

template <typename R>
hipError_t plain_build_U(const R *X, int64_t M, const Factors<R> &fac, cx_t<R> *U, hipStream_t s);
template <typename R>
hipError_t plain_exec(const PlainArgs<R> &a, hipStream_t s);
// Forward DFT of one vector of length L = L1 * L2 (the split and tables of a
// plan with that grid).  L2 == 1: in place in `data`; otherwise `data` is
// overwritten and the result is written to `out`.  *result: where it is.
template <typename R>
hipError_t plain_fft(int64_t L, int L1, int L2, cx_t<R> *data, cx_t<R> *out, const cx_t<R> *tw1,
                     const cx_t<R> *tw2, const cx_t<R> *hi, const cx_t<R> *lo, cx_t<R> **result, hipStream_t s);

// ---- fused online stage -------------------------------------------------------
template <typename R>
struct FusedArgs {
    int64_t N, L, M;
    int L1, L2;              // L = L1 * L2 (L2 == 1: the whole transform in one workgroup)
    Factors<R> fac;
    const uint32_t *keys;    // M sorted keys: (t mod L2) * L1 + t / L2
    const int32_t *perm;     // M: sample index at each sorted position
    const R *Xs;             // M sorted perturbations X = N (x - s/L)
    const int32_t *off;      // L + 1: first sorted position of each key
    const int32_t *sinv;     // M: sorted position of each sample (two-pass plans)
    cx_t<R> *gsort;          // M: a sample-ordered input put in sorted order (two-pass plans)
    int presorted;           // 1: gsort already holds the sorted input of this call
    const int32_t *t;        // M grid indices, sample order
    const R *X;              // M perturbations, sample order
    cx_t<R> *Y;              // K x L intermediate of the two-pass split
    cx_t<R> *Zp;             // partial rows of the dense-tile adjoint pass B' (else null)
    int half;                // FP32 only: Y in fp16 pairs with block exponents E (half-precision exchange)
    int8_t *E;               // K x max(L1, L2) block exponents of the half-precision exchange
    const cx_t<R> *tw1, *tw2, *hi, *lo;
    const cx_t<R> *tw1i, *tw2i;   // inverse-sign twiddles of lengths L1, L2
    // tuning schedule of the two-pass kernels (0: default; 1: first FFT radix 8,
    // with these stage-major tables of that radix order; 2: alternative tile shapes)
    int sched;
    const cx_t<R> *tw1r8, *tw1ir8, *tw2r8, *tw2ir8;
    // destination-bucketed permutation (null bdst: sample-order outputs are
    // written at perm[i] directly, and inputs are put in sorted order by sinv)
    int bshift;
    const int32_t *bdst;     // M: place of sorted position i in the bucketed layout
    const uint16_t *lidx;    // M: sample index within its bucket, per place
    void *bbuf;              // M values (complex or double): the bucketed layout
    cx_t<R> *part;           // scratch for partial sums of the one-workgroup adjoint
    int64_t part_cap;        // complex elements available in part
    Profiler *prof;
};

// f = F2 c (mode 0), or gx = Re(conj(g) F2(-2 pi i k c)) (mode 1)
template <typename R>
hipError_t fused_type2(const FusedArgs<R> &a, const cx_t<R> *c, cx_t<R> *f, int mode,
                       const cx_t<R> *g, double *gx, hipStream_t s);
// sign -1: f = F2^T c (type I); sign +1: f = F2^H c (adjoint)
template <typename R>
hipError_t fused_type1(const FusedArgs<R> &a, const cx_t<R> *c, cx_t<R> *f, int sign, hipStream_t s);
// slices per tile of the dense-tile adjoint pass B' (0: not used; tiles of about M / L2 samples)
int pass_b_adj_splits(int64_t M, int L2, int L1, bool fp32);
// a sample-ordered M-vector into a.gsort (two-pass plans); `name` labels it for the profiler
template <typename R>
hipError_t fused_sort_input(const FusedArgs<R> &a, const cx_t<R> *in, const char *name, hipStream_t s);

}  // namespace nufft
