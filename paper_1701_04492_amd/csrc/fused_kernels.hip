// Fused online stage of the low-rank NUFFT (Sec. 2.2-2.3 and Sec. 3.1).
//
// Type II, f_j = sum_r u_r(j) X_r[t_j] with X_r = F_L (v_r o c):
//  * L <= 4096: one kernel.  Each workgroup rebuilds all K spectra in LDS
//    (scale, FFT) and serves a slice of the samples straight from LDS.
//  * L = L1 * L2: two kernels around one K-wide exchange through HBM.
//    Pass A (per group of G columns k1): c is held in registers; for each r
//    it is scaled by v_r, transformed along k2 and multiplied by the
//    inter-pass twiddle, giving Y_r[n2][k1].
//    Pass B (per output tile n2): for each r the row Y_r[n2][:] is
//    transformed along k1 into X_r[n2 + L2 n1] in LDS; the samples whose
//    t_j falls in the tile (sorted there by the plan) accumulate
//    u_r(j) X_r[t_j] in registers and are written once.
// The factors are evaluated on the fly: v_r(k) = T_r(2k/N - 1) by its
// three-term recurrence and u_r(X) = i^r exp(-i pi X) P_r(X/gamma) with P_r
// from its monomial form (Sec. 2.1.2), so no N x K table is read.
//
// Type I / adjoint run the same two passes in reverse (Sec. 3.1): the
// samples of a tile are summed per grid point (the sorted order makes each
// point's samples one contiguous segment: a deterministic sum, no atomics),
// transformed along n1, and pass A' transforms along n2, scales by v_r and
// sums over r in registers.
#include <algorithm>
#include <atomic>

#include "fused_common.h"

namespace nufft {

// ============================================================================
// L <= 4096: whole transform per workgroup
// ============================================================================

#define SMALL_NT 256
#define SMALL_SLOTS 8

template <typename R, int L>
__global__ void __launch_bounds__(SMALL_NT)
k_small_fwd(const cx_t<R> *__restrict__ c, int64_t N, int64_t M, const int32_t *__restrict__ t,
            const R *__restrict__ X, Factors<R> fac, const cx_t<R> *__restrict__ tw_g,
            cx_t<R> *__restrict__ f, int mode, const cx_t<R> *__restrict__ gup, double *__restrict__ gx)
{
    using C = cx_t<R>;
    constexpr int TPF = L / 16;
    constexpr int RC = SMALL_NT / TPF;          // transforms computed side by side
    constexpr int P = fft_pitch(L);
    __shared__ C buf[RC * P];
    __shared__ C tw[L];
    load_tw_s<C, L, -1, SMALL_NT>(tw, tw_g);

    const int tid = threadIdx.x;
    const int64_t j0 = (int64_t)blockIdx.x * (SMALL_NT * SMALL_SLOTS);
    // sample data: all loads issued together (clamped indices), one wait
    int pos[SMALL_SLOTS];
    R xs[SMALL_SLOTS];
    C acc[SMALL_SLOTS];
#pragma unroll
    for (int s = 0; s < SMALL_SLOTS; ++s) {
        const int64_t j = min(j0 + s * SMALL_NT + tid, M - 1);
        pos[s] = t[j];
        xs[s] = X[j];
        acc[s] = cmake<C>(0, 0);
    }
    const int g = tid / TPF, lt = tid % TPF;
    const ZMap zm = zmap(N);
    for (int r0 = 0; r0 < fac.K; r0 += RC) {
        const int r = r0 + g;
        C v[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) v[q] = load_coef<R>(c, lt + q * TPF, N, mode);
        R zq[16], wq[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) zq[q] = zcoord<R>(lt + q * TPF, zm);
        cheb_v_many<R, 16>(r < fac.K ? r : 0, zq, wq);
#pragma unroll
        for (int q = 0; q < 16; ++q) v[q] = r < fac.K ? cscale(v[q], wq[q]) : cmake<C>(0, 0);
        __syncthreads();   // previous gather finished with buf
        block_fft_regs<C, L, -1, fft_wave_sync<L>>(buf + g * P, tw, lt, v, r < fac.K);   // idle rank slots skip
        fft_publish<L>();
        const int nr = min(RC, fac.K - r0);
        // rank outer (coefficients loaded once), samples inner
        for (int gg = 0; gg < nr; ++gg) {
            const int rr = r0 + gg;
            const RankPoly<R> up = rank_poly(fac, rr);
#pragma unroll
            for (int s = 0; s < SMALL_SLOTS; ++s) {
                if (j0 + s * SMALL_NT < M) {   // else no lane has a sample in this slot
                    const C xv = buf[gg * P + lds_pad(pos[s])];
                    acc[s] = cadd(acc[s], crot(cscale(xv, rank_eval(up, xs[s] * fac.inv_gamma)), rr));
                }
            }
        }
    }
    C gj[SMALL_SLOTS];
    if (mode != 0) {
#pragma unroll
        for (int s = 0; s < SMALL_SLOTS; ++s) gj[s] = gup[min(j0 + s * SMALL_NT + tid, M - 1)];
    }
#pragma unroll
    for (int s = 0; s < SMALL_SLOTS; ++s) {
        const int64_t j = j0 + s * SMALL_NT + tid;
        if (j < M) {
            R sn, cs;
            sincospi_r(xs[s], &sn, &cs);
            const C out = cmul(cmake<C>(cs, -sn), acc[s]);
            if (mode == 0) f[j] = out;
            else gx[j] = (double)(gj[s].x * out.x + gj[s].y * out.y);
        }
    }
}

// Type I (DIR = -1) / adjoint (DIR = +1) for L <= 4096.  Workgroup b spreads
// the sorted samples [b*span, (b+1)*span) and writes its N outputs to
// out + b*N (partial sums, added in order by k_sum_parts when there are
// several workgroups).
template <typename R, int L, int DIR>
__global__ void __launch_bounds__(SMALL_NT)
k_small_adj(const cx_t<R> *__restrict__ c, int64_t N, int64_t M, int64_t span,
            const int32_t *__restrict__ perm, const R *__restrict__ Xs, const int32_t *__restrict__ off,
            Factors<R> fac, const cx_t<R> *__restrict__ tw_g, cx_t<R> *__restrict__ out)
{
    using C = cx_t<R>;
    constexpr int TPF = L / 16;
    constexpr int RC = SMALL_NT / TPF;
    constexpr int P = fft_pitch(L);
    constexpr int OPT = (L + SMALL_NT - 1) / SMALL_NT;   // outputs per thread
    __shared__ C buf[RC * P];
    __shared__ C tw[L];
    __shared__ R ucoef_s[NUFFT_KMAX * NUFFT_UCOEF_STRIDE];
    __shared__ int nterm_s[NUFFT_KMAX];
    load_tw_s<C, L, DIR, SMALL_NT>(tw, tw_g);
    stage_factors(fac, ucoef_s, nterm_s);
    __syncthreads();

    const int tid = threadIdx.x;
    const int64_t lo = (int64_t)blockIdx.x * span, hi = min(M, lo + span);
    const int g = tid / TPF, lt = tid % TPF;
    C oacc[OPT];
#pragma unroll
    for (int m = 0; m < OPT; ++m) oacc[m] = cmake<C>(0, 0);
    const ZMap zm = zmap(N);

    for (int r0 = 0; r0 < fac.K; r0 += RC) {
        const int r = r0 + g;
        C v[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int n = lt + q * TPF;
            C a = cmake<C>(0, 0);
            if (r < fac.K) {
                const int64_t b0 = max((int64_t)off[n], lo), b1 = min((int64_t)off[n + 1], hi);
                for (int64_t i = b0; i < b1; ++i) {
                    const R Xi = Xs[i];
                    R sn, cs;
                    sincospi_r(Xi, &sn, &cs);
                    const C e = cmake<C>(cs, DIR * sn);          // exp(DIR i pi X)
                    const C val = cmul(e, c[perm[i]]);
                    a = cadd(a, cscale(val, upoly_lds(ucoef_s, nterm_s, r, Xi * fac.inv_gamma)));
                }
                a = crot(a, -DIR * r);                            // i^r (type I) or i^-r (adjoint)
            }
            v[q] = a;
        }
        __syncthreads();
        block_fft_regs<C, L, DIR, fft_wave_sync<L>>(buf + g * P, tw, lt, v, r < fac.K);   // idle rank slots skip
        fft_publish<L>();
        const int nr = min(RC, fac.K - r0);
        // T_{r0 + gg} for the consecutive ranks of the chunk by the recurrence
        R zq[OPT], t0[OPT], t1[OPT];
#pragma unroll
        for (int m = 0; m < OPT; ++m) zq[m] = zcoord<R>(tid + m * SMALL_NT, zm);
        cheb_pair_many<R, OPT>(r0, zq, t0, t1);
        for (int gg = 0; gg < nr; ++gg) {
#pragma unroll
            for (int m = 0; m < OPT; ++m) {
                const int k = tid + m * SMALL_NT;
                const R w = (r0 + gg == 0) ? (R)0.5 : t0[m];
                if (k < N && k < L) oacc[m] = cadd(oacc[m], cscale(buf[gg * P + lds_pad(k)], w));
                const R c = 2 * zq[m] * t1[m] - t0[m];
                t0[m] = t1[m];
                t1[m] = c;
            }
        }
    }
#pragma unroll
    for (int m = 0; m < OPT; ++m) {
        const int k = tid + m * SMALL_NT;
        if (k < N && k < L) out[(int64_t)blockIdx.x * N + k] = oacc[m];
    }
}

template <typename R>
__global__ void __launch_bounds__(256)
k_sum_parts(const cx_t<R> *__restrict__ part, int nparts, int64_t N, cx_t<R> *__restrict__ f)
{
    using C = cx_t<R>;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    C a = part[k];
    for (int b = 1; b < nparts; ++b) a = cadd(a, part[(int64_t)b * N + k]);
    f[k] = a;
}

// out[sinv[j]] = in[j]: a sample-ordered vector put in the plan's sorted order.
// Reads are coalesced and the writes scattered; a gather in sorted order would
// instead fetch a whole cache line per 8- or 16-byte element.
template <typename R>
__global__ void __launch_bounds__(256)
k_scatter_sorted(const cx_t<R> *__restrict__ in, const int32_t *__restrict__ sinv, int64_t M,
                 cx_t<R> *__restrict__ out)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < M) out[sinv[j]] = in[j];
}

// ---- the permutation through the destination-bucketed layout ------------------
// (large plans; see bucketed_store).  Bucket q holds the samples
// j in [q BS, (q+1) BS) (BS = 2^bshift); place p of its range holds sample
// q BS + lidx[p], the places ordered by sorted position.  One workgroup per
// bucket moves it through LDS in both directions with coalesced reads and
// writes.

// out[q BS + lidx[p]] = in[p] for p in bucket q: the bucketed layout to sample order.
template <typename T, int BS>
__global__ void __launch_bounds__(1024)
k_bucket_to_samples(const T *__restrict__ in, const uint16_t *__restrict__ lidx, int64_t M, T *__restrict__ out)
{
    __shared__ T v[BS];
    const int64_t base = (int64_t)blockIdx.x * BS;
    const int n = (int)min((int64_t)BS, M - base);
    constexpr int E = BS / 1024;
    T w[E];
    int li[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int p = min((int)threadIdx.x + e * 1024, n - 1);
        w[e] = in[base + p];
        li[e] = lidx[base + p];
    }
#pragma unroll
    for (int e = 0; e < E; ++e)
        if ((int)threadIdx.x + e * 1024 < n) v[li[e]] = w[e];
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int t = threadIdx.x + e * 1024;
        if (t < n) out[base + t] = v[t];
    }
}

// out[p] = in[q BS + lidx[p]] for p in bucket q: sample order to the bucketed layout.
template <typename T, int BS>
__global__ void __launch_bounds__(1024)
k_samples_to_bucket(const T *__restrict__ in, const uint16_t *__restrict__ lidx, int64_t M, T *__restrict__ out)
{
    __shared__ T v[BS];
    const int64_t base = (int64_t)blockIdx.x * BS;
    const int n = (int)min((int64_t)BS, M - base);
    constexpr int E = BS / 1024;
    T w[E];
#pragma unroll
    for (int e = 0; e < E; ++e) w[e] = in[base + min((int)threadIdx.x + e * 1024, n - 1)];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int t = threadIdx.x + e * 1024;
        if (t < n) v[t] = w[e];
    }
    __syncthreads();
    int li[E];
#pragma unroll
    for (int e = 0; e < E; ++e) li[e] = lidx[base + min((int)threadIdx.x + e * 1024, n - 1)];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int p = threadIdx.x + e * 1024;
        if (p < n) out[base + p] = v[li[e]];
    }
}

// out[i] = in[bdst[i]] for a range of RNG sorted positions per workgroup: the
// range's places are ordered by bucket in LDS, so that the reads of one bucket
// (consecutive places) coalesce, and the values are written back in sorted order.
template <typename T, int RNG, int NT>
__global__ void __launch_bounds__(NT)
k_bucket_to_sorted(const T *__restrict__ in, const int32_t *__restrict__ bdst, int64_t M, int shift, int nbk,
                   T *__restrict__ out)
{
    constexpr int E = RNG / NT;
    __shared__ int hist[1026], wsum[NT / 64 + 1];
    __shared__ int dsts[RNG];
    __shared__ unsigned short locs[RNG];
    __shared__ T v[RNG];
    const int tid = threadIdx.x;
    const int64_t i0 = (int64_t)blockIdx.x * RNG;
    const int n = (int)min((int64_t)RNG, M - i0);
    int d[E];
#pragma unroll
    for (int e = 0; e < E; ++e) d[e] = bdst[i0 + min(tid + e * NT, n - 1)];
    for (int b = tid; b < nbk; b += NT) hist[b] = 0;
    __syncthreads();
    int rank[E];
#pragma unroll
    for (int e = 0; e < E; ++e) rank[e] = tid + e * NT < n ? atomicAdd(&hist[d[e] >> shift], 1) : 0;
    __syncthreads();
    block_exclusive_scan<NT>(hist, nbk, wsum);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        if (tid + e * NT < n) {
            const int slot = hist[d[e] >> shift] + rank[e];
            dsts[slot] = d[e];
            locs[slot] = (unsigned short)(tid + e * NT);
        }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int t = tid + e * NT;
        if (t < n) v[locs[t]] = in[dsts[t]];
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int t = tid + e * NT;
        if (t < n) out[i0 + t] = v[t];
    }
}

// Launches KERNEL<T, BS> over the plan's blocks for its block size BS = 2^bshift
// (2^12 to 2^14 samples; 2^12 and 2^13 for 16-byte values, whose LDS copy of
// a block would not fit at 2^14).
#define BUCKET_LAUNCH(KERNEL, T, a, s, ...)                                                              \
    do {                                                                                                 \
        const unsigned nbk_ = (unsigned)(((a).M + (int64_t(1) << (a).bshift) - 1) >> (a).bshift);      \
        if ((a).bshift == 12)                                                                            \
            hipLaunchKernelGGL((KERNEL<T, 4096>), dim3(nbk_), dim3(1024), 0, s, __VA_ARGS__);           \
        else if ((a).bshift == 13)                                                                       \
            hipLaunchKernelGGL((KERNEL<T, 8192>), dim3(nbk_), dim3(1024), 0, s, __VA_ARGS__);           \
        else if constexpr (sizeof(T) <= 8) {                                                             \
            if ((a).bshift == 14)                                                                        \
                hipLaunchKernelGGL((KERNEL<T, 16384>), dim3(nbk_), dim3(1024), 0, s, __VA_ARGS__);      \
            else                                                                                         \
                return hipErrorInvalidValue;                                                             \
        } else                                                                                           \
            return hipErrorInvalidValue;                                                                 \
    } while (0)

// Bucketed outputs (values of type T at the places of the plan's layout) to sample order.
template <typename T, typename R>
static hipError_t bucket_to_samples(const FusedArgs<R> &a, const T *in, T *out, hipStream_t s)
{
    BUCKET_LAUNCH(k_bucket_to_samples, T, a, s, in, a.lidx, a.M, out);
    return hipGetLastError();
}

template <typename R>
hipError_t fused_sort_input(const FusedArgs<R> &a, const cx_t<R> *in, const char *name, hipStream_t s)
{
    using C = cx_t<R>;
    prof_begin(a.prof, name, s);
    if (a.bdst) {
        // sample order -> bucketed layout (coalesced through LDS) -> sorted order (coalesced runs)
        const int nbk = (int)((a.M + (int64_t(1) << a.bshift) - 1) >> a.bshift);
        BUCKET_LAUNCH(k_samples_to_bucket, C, a, s, in, a.lidx, a.M, (C *)a.bbuf);
        constexpr int RNG = sizeof(R) == 4 ? 4096 : 2048;
        hipLaunchKernelGGL((k_bucket_to_sorted<C, RNG, 512>), dim3((unsigned)((a.M + RNG - 1) / RNG)), dim3(512), 0, s,
                           (const C *)a.bbuf, a.bdst, a.M, a.bshift, nbk, a.gsort);
    } else {
        hipLaunchKernelGGL(k_scatter_sorted<R>, dim3((unsigned)((a.M + 255) / 256)), dim3(256), 0, s, in, a.sinv, a.M,
                           a.gsort);
    }
    prof_end(a.prof, s);
    return hipGetLastError();
}

// ============================================================================
// L = L1 * L2: pass A (columns) and pass B (rows + samples)
// ============================================================================

// Pass A of type II.  Task = (G adjacent columns k1, a chunk of RCA ranks);
// k = k1 + L1 k2.  Each column is one length-L2 transform done by L2/16
// threads.  The G x L2 block of c is read with coalesced G-wide rows and
// transposed through LDS into the operand order of the first radix-16 stage
// (k2 = lt + q L2/16); for each rank of the chunk it is scaled by v_r,
// transformed, multiplied by exp(-2 pi i k1 n2 / L) and stored as
// Y_r[n2][k1] (G-element runs).
// H (FP32 only): Y in fp16 pairs with one scale exponent per (rank, column),
// E[r * L1 + k1] (the half-precision exchange).
template <typename R, int L2, int G, bool TWG, bool H, int FR = 16>
__global__ void __launch_bounds__(G * L2 / 16)
k_passA(const cx_t<R> *__restrict__ c, int64_t N, int64_t L1, int K, int RCA, int mode,
        const cx_t<R> *__restrict__ tw_g, const cx_t<R> *__restrict__ hi, const cx_t<R> *__restrict__ lo,
        cx_t<R> *__restrict__ Y, int8_t *__restrict__ E)
{
    using C = cx_t<R>;
    constexpr int TPF = L2 / 16;
    constexpr int NT = G * TPF;
    constexpr int P = fft_pitch_g(L2, G);
    static_assert(!H || sizeof(R) == 4, "the half-precision exchange is an FP32 path");
    __shared__ C buf[G * P];
    __shared__ C tw_s[TWG ? 1 : L2];
    __shared__ unsigned smax[H ? 2 * G : 1];   // per-column block maxima (float bits), two parities
    const C *tw = TWG ? tw_g : tw_s;
    const int nrc = (K + RCA - 1) / RCA;
    const int task = xcd_task((int)(L1 / G) * nrc);
    if (task < 0) return;
    const int cg = task / nrc, rc = task % nrc;
    const int r_lo = rc * RCA, r_hi = min(K, r_lo + RCA);
    if (!TWG) load_tw_s<C, L2, -1, NT>(tw_s, tw_g);
    const int tid = threadIdx.x;
    const int g = tid / TPF, lt = tid % TPF;
    const int64_t k1_0 = (int64_t)cg * G;
    const int64_t L = L1 * L2;
    if (H && tid < 2 * G) smax[tid] = 0;
    {
        C cl[16];   // all 16 loads in flight before the first LDS store
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int i = tid + e * NT;
            cl[e] = load_coef<R>(c, k1_0 + i % G + L1 * (int64_t)(i / G), N, mode);
        }
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int i = tid + e * NT;
            buf[(i % G) * P + lds_pad(i / G)] = cl[e];
        }
    }
    __syncthreads();
    C cv[16];
    R zk[16];
    const ZMap zm = zmap(N);
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        cv[q] = buf[g * P + lds_pad(lt + q * TPF)];
        zk[q] = zcoord<R>((k1_0 + g) + L1 * (int64_t)(lt + q * TPF), zm);
    }
    // inter-pass twiddles of this thread's 16 output positions: the same for every rank
    C wt[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int i = tid + e * NT;
        wt[e] = tw_big<C, -1>(hi, lo, (k1_0 + i % G) * (int64_t)(i / G));
    }
    for (int r = r_lo; r < r_hi; ++r) {
        C v[16];
        {
            R wq[16];
            cheb_v_many<R, 16>(r, zk, wq);
#pragma unroll
            for (int q = 0; q < 16; ++q) v[q] = cscale(cv[q], wq[q]);
        }
        __syncthreads();   // earlier readers of buf are done
        if constexpr (fft_radix_p(L2) == 1) {
            block_fft_regs<C, L2, -1, fft_wave_sync<L2>, FR>(buf + g * P, tw, lt, v);
            fft_publish<L2>();
        } else {   // mixed length: its radix-3/5 stage reads across the transform's waves
#pragma unroll
            for (int q = 0; q < 16; ++q) buf[g * P + lds_pad(lt + q * TPF)] = v[q];
            __syncthreads();
            block_fft_any_lds<C, L2, -1, FR>(buf + g * P, tw, lt);
        }
        if constexpr (H) {
            // this thread's 16 outputs all lie in column gg = tid % G (NT is a multiple of G)
            C o[16];
            float m = 0.0f;
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int i = tid + e * NT;
                o[e] = cmul(buf[(i % G) * P + fft_out_pos<L2>(i / G)], wt[e]);
                m = fmaxf(m, cmaxabs(o[e]));
            }
            m = wave_max_mod(m, G);
            unsigned *sm = smax + (r & 1) * G;
            if ((tid & 63) < G) atomicMax(&sm[tid & 63], __float_as_uint(m));
            __syncthreads();
            const int gg = tid % G;
            const int ex = hx_exponent(__uint_as_float(sm[gg]));
            if (tid < G) {
                E[(int64_t)r * L1 + k1_0 + tid] = (int8_t)ex;
                smax[((r + 1) & 1) * G + tid] = 0;   // its last readers finished before this rank's first barrier
            }
            __half2 *Yr = reinterpret_cast<__half2 *>(Y) + (int64_t)r * L + k1_0;
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int n2 = (tid + e * NT) / G;
                Yr[(int64_t)n2 * L1 + gg] = hx_pack(o[e], ex);
            }
        } else {
            C *Yr = Y + (int64_t)r * L + k1_0;
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int i = tid + e * NT;
                const int gg = i % G, n2 = i / G;
                Yr[(int64_t)n2 * L1 + gg] = cmul(buf[gg * P + fft_out_pos<L2>(n2)], wt[e]);
            }
        }
    }
}

// Pass A with wide column blocks (FP32; launched at L2 = 2048, see WIDE_A): G
// columns per workgroup with each thread transforming two of them (columns g
// and g + G/2), so that the exchange is written in G*8-byte runs (64 bytes at
// G = 8; G*4 = 32 bytes for the half-precision exchange) at the register budget
// of G/2 columns.  Narrow runs waste most of each DRAM burst: measured on this
// store pattern alone, 32-byte runs reach 3.3 TB/s and 64-byte runs 5.7 TB/s.
// The inter-pass twiddle of output (k1, n2) is Bv[jb] * Av[ja] with
// n2 = n2_0 + (NT/G)(8 jb + ja): twelve table values per thread instead of 32.
// H: Y in fp16 pairs scaled per (rank, column) by 2^E[r * L1 + k1]; a thread's
// 32 outputs all lie in its column, so it forms them twice (for the column's
// block maximum, then to pack them) instead of holding 64 more registers.
template <typename R, int L2, int G, bool H = false, int FR = 16>
__global__ void __launch_bounds__(G / 2 * L2 / 16)
k_passA_wide(const cx_t<R> *__restrict__ c, int64_t N, int64_t L1, int K, int RCA, int mode,
             const cx_t<R> *__restrict__ tw_g, const cx_t<R> *__restrict__ hi, const cx_t<R> *__restrict__ lo,
             cx_t<R> *__restrict__ Y, int8_t *__restrict__ E = nullptr)
{
    using C = cx_t<R>;
    constexpr int TPF = L2 / 16;
    constexpr int GH = G / 2;            // columns per half
    constexpr int NT = GH * TPF;
    constexpr int P = fft_pitch_g(L2, G);
    constexpr int ST = NT / G;           // rows between a thread's consecutive outputs
    static_assert(fft_radix_p(L2) == 1 && NT % G == 0 && G * L2 == 32 * NT, "two halves of 16 elements");
    static_assert(!H || sizeof(R) == 4, "the half-precision exchange is an FP32 path");
    __shared__ C buf[G * P];
    __shared__ C tw_s[L2];
    __shared__ unsigned smax[H ? 2 * G : 1];   // per-column block maxima (float bits), two parities
    const int nrc = (K + RCA - 1) / RCA;
    const int task = xcd_task((int)(L1 / G) * nrc);
    if (task < 0) return;
    const int cg = task / nrc, rc = task % nrc;
    const int r_lo = rc * RCA, r_hi = min(K, r_lo + RCA);
    load_tw_s<C, L2, -1, NT>(tw_s, tw_g);
    const int tid = threadIdx.x;
    if (H && tid < 2 * G) smax[tid] = 0;
    const int g = tid / TPF, lt = tid % TPF;
    const int64_t k1_0 = (int64_t)cg * G;
    const int64_t L = L1 * L2;
    // the G x L2 block of c: G-wide rows, two rounds of 16 loads in flight
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        C cl[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int i = tid + (h * 16 + e) * NT;
            cl[e] = load_coef<R>(c, k1_0 + i % G + L1 * (int64_t)(i / G), N, mode);
        }
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int i = tid + (h * 16 + e) * NT;
            buf[(i % G) * P + lds_pad(i / G)] = cl[e];
        }
    }
    __syncthreads();
    C cv[2][16];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int q = 0; q < 16; ++q) cv[h][q] = buf[(g + h * GH) * P + lds_pad(lt + q * TPF)];
    // twiddle factors of this thread's outputs: column gg = tid % G, rows n2_0 + ST e
    const int gg = tid % G, n2_0 = tid / G;
    const int64_t k1 = k1_0 + gg;
    C Av[8], Bv[4];
#pragma unroll
    for (int j = 0; j < 8; ++j) Av[j] = tw_big<C, -1>(hi, lo, (k1 * ST * j) % L);
#pragma unroll
    for (int j = 0; j < 4; ++j) Bv[j] = tw_big<C, -1>(hi, lo, k1 * (n2_0 + 8 * ST * j));
    const ZMap zm = zmap(N);
    // L1 is a power of two: row offsets are shifts (a runtime multiply is a quarter-rate
    // integer instruction, and these are formed anew for every rank)
    const int l1s = __builtin_ctzll((unsigned long long)L1);
    for (int r = r_lo; r < r_hi; ++r) {
        __syncthreads();   // earlier readers of buf are done
        // the sample coordinates are recomputed per rank: an empty asm makes the row
        // index opaque, so the compiler keeps them out of registers across ranks
        int lr = lt;
        asm volatile("" : "+v"(lr));
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            C v[16];
            R wq[16], zk[16];
            const int kc = (int)k1_0 + g + h * GH;   // mode indices are below 2^23
#pragma unroll
            for (int q = 0; q < 16; ++q) zk[q] = zcoord<R>((int64_t)(kc + ((lr + q * TPF) << l1s)), zm);
            cheb_v_many<R, 16>(r, zk, wq);
#pragma unroll
            for (int q = 0; q < 16; ++q) v[q] = cscale(cv[h][q], wq[q]);
            block_fft_regs<C, L2, -1, fft_wave_sync<L2>, FR>(buf + (g + h * GH) * P, tw_s, lt, v);
        }
        __syncthreads();   // both halves' transforms are visible
        // (opaque copies again: the 32 output addresses are formed here, not kept across ranks)
        int n2o = n2_0, go = gg;
        asm volatile("" : "+v"(n2o), "+v"(go));
        if constexpr (H) {
            float m = 0.0f;
#pragma unroll
            for (int jb = 0; jb < 4; ++jb) {
                C o[8];
#pragma unroll
                for (int ja = 0; ja < 8; ++ja) o[ja] = buf[go * P + lds_pad(n2o + ST * (8 * jb + ja))];
#pragma unroll
                for (int ja = 0; ja < 8; ++ja) m = fmaxf(m, cmaxabs(cmul(cmul(o[ja], Bv[jb]), Av[ja])));
            }
            // lanes agreeing mod G share the column; lane l < G then holds column l's wave maximum
            m = wave_max_mod(m, G);
            unsigned *sm = smax + (r & 1) * G;
            if ((tid & 63) < G) atomicMax(&sm[tid & 63], __float_as_uint(m));
            __syncthreads();
            const int ex = hx_exponent(__uint_as_float(sm[go]));
            if (tid < G) {
                E[(int64_t)r * L1 + k1_0 + tid] = (int8_t)ex;
                smax[((r + 1) & 1) * G + tid] = 0;   // its last readers finished before this rank's first barrier
            }
            __half2 *Yh = reinterpret_cast<__half2 *>(Y) + (int64_t)r * L + k1_0 + go;
#pragma unroll
            for (int jb = 0; jb < 4; ++jb) {
                C o[8];
#pragma unroll
                for (int ja = 0; ja < 8; ++ja) o[ja] = buf[go * P + lds_pad(n2o + ST * (8 * jb + ja))];
#pragma unroll
                for (int ja = 0; ja < 8; ++ja)
                    Yh[(int64_t)(n2o + ST * (8 * jb + ja)) << l1s] = hx_pack(cmul(cmul(o[ja], Bv[jb]), Av[ja]), ex);
            }
        } else {
            C *Yr = Y + (int64_t)r * L + k1_0 + go;
#pragma unroll
            for (int jb = 0; jb < 4; ++jb) {
                C o[8];
#pragma unroll
                for (int ja = 0; ja < 8; ++ja) o[ja] = buf[go * P + lds_pad(n2o + ST * (8 * jb + ja))];
#pragma unroll
                for (int ja = 0; ja < 8; ++ja)
                    Yr[(int64_t)(n2o + ST * (8 * jb + ja)) << l1s] = cmul(cmul(o[ja], Bv[jb]), Av[ja]);
            }
        }
    }
}

// LDS bytes of the bucketed store of pass B's outputs (bucketed_store): bin
// counts of up to 1024 buckets, wave sums, then NT*S values and their places.
__host__ __device__ constexpr int bucket_scratch_bytes(int NT, int S, int vbytes)
{
    return 4352 + NT * S * (vbytes + 4);
}
// Whether pass B with these shapes can order its outputs by bucket inside its
// FFT buffer (values of complex size, or double for the derivative pass).
__host__ __device__ constexpr bool pass_b_buckets(int L1, int RC, int S, int cbytes)
{
    return bucket_scratch_bytes(RC * L1 / 16, S, cbytes > 8 ? cbytes : 8) <= cbytes * RC * fft_pitch(L1);
}

// Pass B of type II.  Task = one output tile n2 (or a share of it, below); a
// workgroup takes its XCD's tasks in turn (xcd_tasks), as many workgroups as the
// device holds at once.  RC ranks are transformed side by side (L1/16 threads
// each); the next chunk's rows, or at a task's last chunk the next task's first
// rows, are loaded into registers while the current chunk is transformed and
// gathered.  Every
// sample of the tile (up to NT*S per round) gathers its RC spectrum values
// from LDS and accumulates u_r(j) X_r[t_j] in registers.  When K <= RC the
// transforms are done once per task and serve every round of its samples;
// otherwise each round repeats them (rounds are rare then: S is sized so
// that one round holds about 1.25 L1 samples, the mean tile when M = N).
// With many more samples than grid points, `splits` tasks share a tile, each
// transforming its rows and taking an equal slice of the tile's samples.
// H: Y holds fp16 pairs scaled per (rank, column) by 2^E[r * L1 + k1].
// MODE: the output mode fixed at compile time (0 type II, 1 derivative), or -1 to
// take the argument.  The two-rank, nine-slot shape at 2048 points asks for two
// workgroups per CU in its launch bounds (the registers of two waves per SIMD).
template <typename R, int L1, int RC, int S, bool TWG, bool H, int FR = 16, int MODE = -1>
__global__ void __launch_bounds__(RC * L1 / 16, (L1 == 2048 && RC == 2 && S == 9) ? 2 : 1)
k_passB(const cx_t<R> *__restrict__ Y, int64_t L2, int64_t M, const uint32_t *__restrict__ keys,
        const int32_t *__restrict__ perm, const R *__restrict__ Xs, const int32_t *__restrict__ off,
        Factors<R> fac, const cx_t<R> *__restrict__ tw_g, cx_t<R> *__restrict__ f, int mode_arg,
        const cx_t<R> *__restrict__ gup, double *__restrict__ gx, const int8_t *__restrict__ E, int splits,
        const int32_t *__restrict__ bdst, int bshift, int nbk, void *__restrict__ bout)
{
    using C = cx_t<R>;
    const int mode = MODE >= 0 ? MODE : mode_arg;
    constexpr int TPF = L1 / 16;
    constexpr int NT = RC * TPF;
    constexpr int P = fft_pitch(L1);
    constexpr int CAP = NT * S;
    static_assert(bucket_scratch_bytes(NT, S, sizeof(C)) <= (int)sizeof(C) * RC * P || !pass_b_buckets(L1, RC, S, sizeof(C)),
                  "bucketed store scratch exceeds the FFT buffer");
    __shared__ C buf[RC * P];
    __shared__ C tw_s[TWG ? 1 : L1];
    const C *tw = TWG ? tw_g : tw_s;
    const int T = (int)L2 * splits;
    int task, tend, tstep;
    xcd_tasks(T, &task, &tend, &tstep);
    if (task >= tend) return;
    if (!TWG) load_tw_s<C, L1, -1, NT>(tw_s, tw_g);
    const int tid = threadIdx.x;
    const int g = tid / TPF, lt = tid % TPF;
    const int64_t L = (int64_t)L1 * L2;
    int64_t tile_lo = 0, tile_hi = 0;   // the current task's samples [tile_lo, tile_hi)
    // Rank row rr of tile n2f, the lanes' 16 elements (zero for rr >= K), in
    // two steps so that a prefetch stays in flight: fetch issues the loads
    // into raw registers (fp16 pairs and exponents for H), take decodes them.
    using Raw = typename std::conditional<H, __half2, C>::type;
    // (a rank beyond K loads nothing: its lanes are zero and its transform is discarded)
    auto fetch = [&](int64_t n2f, int rr, Raw (&w)[16], int8_t (&ev)[16]) __attribute__((always_inline)) {
        const bool in = rr < fac.K;
        const C *Yrow = Y + n2f * L1 + lt;
        const __half2 *Yhrow = reinterpret_cast<const __half2 *>(Y) + n2f * L1 + lt;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            if constexpr (H) {
                w[q] = in ? Yhrow[(int64_t)rr * L + q * TPF] : __half2{};
                ev[q] = in ? E[(int64_t)rr * L1 + lt + q * TPF] : (int8_t)0;
            } else {
                w[q] = in ? Yrow[(int64_t)rr * L + q * TPF] : cmake<C>(0, 0);
            }
        }
    };
    auto take = [&](const Raw (&w)[16], const int8_t (&ev)[16], C (&v)[16]) __attribute__((always_inline)) {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            if constexpr (H) v[q] = hx_unpack(w[q], ev[q]);
            else v[q] = w[q];
        }
    };

    // gather of ranks r0 .. r0 + nr - 1 from the spectra in buf into the sample sums
    auto gather = [&](int r0, int nr, int64_t c0, const uint32_t (&kv)[S], const R (&xs)[S], C (&acc)[S]) __attribute__((always_inline)) {
        // rank outer (its coefficients loaded once), samples inner
#pragma unroll
        for (int gg = 0; gg < RC; ++gg) {
            if (gg < nr) {
                const int rr = r0 + gg;
                const RankPoly<R> up = rank_poly(fac, rr);
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    if (c0 + s * NT < tile_hi) {   // else no lane has a sample in this slot
                        const C xv = buf[gg * P + lds_pad((int)(kv[s] & (uint32_t)(L1 - 1)))];
                        acc[s] = cadd(acc[s], crot(cscale(xv, rank_eval(up, xs[s] * fac.inv_gamma)), rr));
                    }
                }
            }
        }
    };
    // K <= RC: every rank is transformed in the first round, and the spectra
    // stay in LDS for all later rounds of the tile (many samples per tile: M >> N)
    const bool once = fac.K <= RC;

    // the workgroup's tasks in turn; the first rank chunk of the next task is
    // fetched while the last one of the current task is transformed
    Raw vn[16];
    int8_t en[16];
    bool have = false;   // vn holds the first chunk of this task
    for (; task < tend; task += tstep) {
    const int64_t n2 = task / splits;
    const int part = task % splits;
    // this task's share of the tile's samples (the whole tile unless splits > 1)
    const int64_t t_lo = off[n2 * L1], t_cnt = off[(n2 + 1) * L1] - t_lo;
    tile_lo = t_lo + t_cnt * part / splits;
    tile_hi = t_lo + t_cnt * (part + 1) / splits;
    const int nxt = task + tstep;
    if (tile_lo >= tile_hi) have = false;   // no sample: nothing is transformed
    for (int64_t c0 = tile_lo; c0 < tile_hi; c0 += CAP) {
        // the round's sample data: every load issued before any is used
        // (indices clamped into the tile), then one wait
        uint32_t kv[S];
        R xs[S];
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int64_t i = min(c0 + s * NT + tid, tile_hi - 1);
            kv[s] = keys[i];
            xs[s] = Xs[i];
        }
        C acc[S];
#pragma unroll
        for (int s = 0; s < S; ++s) acc[s] = cmake<C>(0, 0);
        const bool transform = !once || c0 == tile_lo;
        // last round: fetch the next task's rows (not where the registers run short:
        // the 4096-point rows spill, the 128-point kernel would lose a wave per SIMD)
        constexpr bool XPF = L1 >= 256 && L1 <= 2048;
        const bool ahead = XPF && !once && c0 + CAP >= tile_hi && nxt < tend;
        if (transform && !have) fetch(n2, g, vn, en);
        have = false;
        for (int r0 = 0; r0 < fac.K; r0 += RC) {
            if (transform) {
                C v[16];
                take(vn, en, v);
                if (r0 + RC < fac.K) {
                    fetch(n2, r0 + RC + g, vn, en);
                } else if (ahead) {
                    fetch(nxt / splits, g, vn, en);
                    have = true;
                }
                __syncthreads();
                // a rank slot beyond K (the last chunk of ranks) skips its transform
                block_fft_regs<C, L1, -1, fft_wave_sync<L1>, FR>(buf + g * P, tw, lt, v, r0 + g < fac.K);
                fft_publish<L1>();
            }
            gather(r0, min(RC, fac.K - r0), c0, kv, xs, acc);
        }
        // output places: the samples' indices, or (bdst) their places in the
        // destination-bucketed layout; loaded together once the sums are done
        int32_t jv[S];
        C gj[S];         // derivative pass: g in sorted order (contiguous)
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int64_t i = min(c0 + s * NT + tid, tile_hi - 1);
            jv[s] = bdst ? bdst[i] : perm[i];
            if (mode != 0) gj[s] = gup[i];
        }
        C out[S];
        bool valid[S];
#pragma unroll
        for (int s = 0; s < S; ++s) {
            valid[s] = c0 + s * NT + tid < tile_hi;
            R sn, cs;
            sincospi_r(xs[s], &sn, &cs);
            out[s] = cmul(cmake<C>(cs, -sn), acc[s]);
        }
        bool bucketed = false;
        if constexpr (pass_b_buckets(L1, RC, S, sizeof(C))) {
            if (bdst) {
                // the spectra in buf are not read again (K > RC): its space holds the
                // bucketed ordering of this round's outputs
                int *hist = reinterpret_cast<int *>(buf);
                int *wsum = hist + 1026;
                char *vbase = reinterpret_cast<char *>(buf) + 4352;
                if (mode == 0) {
                    bucketed_store<C, NT, S>(out, jv, valid, bshift, nbk, reinterpret_cast<C *>(bout), hist, wsum,
                                             reinterpret_cast<C *>(vbase), reinterpret_cast<int *>(vbase + CAP * sizeof(C)));
                } else {
                    double d[S];
#pragma unroll
                    for (int s = 0; s < S; ++s) d[s] = (double)(gj[s].x * out[s].x + gj[s].y * out[s].y);
                    bucketed_store<double, NT, S>(d, jv, valid, bshift, nbk, reinterpret_cast<double *>(bout), hist,
                                                  wsum, reinterpret_cast<double *>(vbase),
                                                  reinterpret_cast<int *>(vbase + CAP * sizeof(double)));
                }
                bucketed = true;
            }
        }
        if (!bucketed) {
#pragma unroll
            for (int s = 0; s < S; ++s) {
                if (valid[s]) {
                    if (mode == 0) f[jv[s]] = out[s];
                    else gx[jv[s]] = (double)(gj[s].x * out[s].x + gj[s].y * out[s].y);
                }
            }
        }
        if (!once) __syncthreads();   // the next round's transforms overwrite buf
    }
    }
}

// Pass B' of type I / adjoint.  Task = tile n2.  The tile's samples are
// staged once in LDS as exp(DIR i pi X_j) c_j, z_j = X_j / gamma and their
// grid point n1 (up to SCAP of them; any further ones are read from global
// memory).  Thread t walks one contiguous run of the sorted order: the
// samples from t*cnt/NT to (t+1)*cnt/NT, both ends moved forward to the next
// grid-point boundary, so that every grid point's samples belong to one run
// and the runs are about equally long whatever the points' occupancy.  For
// each chunk of RC ranks the walk sums P_r(z_j) exp(DIR i pi X_j) c_j for
// every rank of the chunk in sample order and stores each grid value when
// the grid point changes; the factor i^r (type I) or i^-r (adjoint) is
// taken into the sum, as a sign on the polynomial and, for odd powers, a
// swap of the components (exact, so the stored value is the rotated sum).
// Grid points without samples stay zero: the grids are cleared once, and
// each output read clears the value it has read.  The RC grids are then
// transformed along n1 and multiplied by exp(DIR 2 pi i n2 k1 / L):
// Z_r[n2][k1].
// TWG: read the FFT twiddles (already of sign DIR) from global memory instead
// of an LDS copy, for the sizes where LDS would otherwise cap occupancy.
// H (FP32 only): Z in fp16 pairs with one scale exponent per (rank, row),
// E[r * L2 + n2] (the half-precision exchange).
template <typename R, int L1, int RC, int SCAP, int dir, bool TWG, bool H, int FR = 16>
__global__ void __launch_bounds__(RC * L1 / 16)
k_passB_adj(const cx_t<R> *__restrict__ csort, int64_t L2, const R *__restrict__ Xs,
            const uint32_t *__restrict__ keys, const int32_t *__restrict__ off,
            Factors<R> fac, const cx_t<R> *__restrict__ tw_g, const cx_t<R> *__restrict__ hi,
            const cx_t<R> *__restrict__ lo, cx_t<R> *__restrict__ Z, int8_t *__restrict__ E)
{
    using C = cx_t<R>;
    constexpr int TPF = L1 / 16;
    constexpr int NT = RC * TPF;
    constexpr int P = fft_pitch(L1);
    __shared__ C buf[RC * P];
    __shared__ C tw_s[TWG ? 1 : L1];
    const C *tw = TWG ? tw_g : tw_s;
    // staged samples: in FP32 one 16-byte record (value, z, grid point) each,
    // which the walk reads in one access; in FP64 three arrays
    constexpr bool REC = sizeof(R) == 4;
    __shared__ float4 srec[REC ? SCAP : 1];
    __shared__ C sval[REC ? 1 : SCAP];
    __shared__ R sz[REC ? 1 : SCAP];
    __shared__ unsigned short spos[REC ? 1 : SCAP];
    __shared__ int soff[L1 + 1];
    __shared__ unsigned smax[H ? 2 * RC : 1];   // per-row block maxima (float bits), two parities
    static_assert(!H || sizeof(R) == 4, "the half-precision exchange is an FP32 path");
    auto put_s = [&](int i, const C &v, R z, int n1) __attribute__((always_inline)) {
        if constexpr (REC) {
            srec[i] = make_float4(v.x, v.y, z, __int_as_float(n1));
        } else {
            sval[i] = v;
            sz[i] = z;
            spos[i] = (unsigned short)n1;
        }
    };
    auto get_s = [&](int i, C &v, R &z, int &n1) __attribute__((always_inline)) {
        if constexpr (REC) {
            const float4 t = srec[i];
            v = cmake<C>(t.x, t.y);
            z = t.z;
            n1 = __float_as_int(t.w);
        } else {
            v = sval[i];
            z = sz[i];
            n1 = spos[i];
        }
    };
    const int task = xcd_task((int)L2);
    if (task < 0) return;
    const int tid = threadIdx.x;
    if (H && tid < 2 * RC) smax[tid] = 0;
    if (!TWG) load_tw_s<C, L1, -1, NT>(tw_s, tw_g);   // tw_g already has the sign DIR
    const int g = tid / TPF, lt = tid % TPF;
    const int64_t n2 = task;
    const int64_t L = (int64_t)L1 * L2;
    const int tile_lo = off[n2 * L1];
    {
        constexpr int E = (L1 + 1 + NT - 1) / NT;
        int o[E];
#pragma unroll
        for (int e = 0; e < E; ++e) o[e] = off[n2 * L1 + min(tid + e * NT, L1)];
#pragma unroll
        for (int e = 0; e < E; ++e)
            if (tid + e * NT <= L1) soff[tid + e * NT] = o[e] - tile_lo;
    }
    const int cnt = off[(n2 + 1) * L1] - tile_lo;
    const int nst = min(cnt, SCAP);
    if (nst > 0) {
        // stage the tile's samples: all index/value loads of a thread in flight
        // together (clamped indices), then the dependent loads of c, one wait each
        constexpr int SU = (SCAP + NT - 1) / NT;   // staging rounds per thread
        constexpr int SB = SU < 8 ? SU : 8;          // rounds whose loads are in flight together
        for (int u0 = 0; u0 < SU; u0 += SB) {
            if (u0 * NT >= nst) break;
            R xv[SB];
            uint32_t kv[SB];
            C cj[SB];
#pragma unroll
            for (int u = 0; u < SB; ++u) {
                const int i = tile_lo + min(tid + (u0 + u) * NT, nst - 1);
                xv[u] = Xs[i];
                kv[u] = keys[i];
                cj[u] = csort[i];
            }
#pragma unroll
            for (int u = 0; u < SB; ++u) {
                const int i = tid + (u0 + u) * NT;
                if (i < nst) {
                    R sn, cs;
                    sincospi_r(xv[u], &sn, &cs);
                    put_s(i, cmul(cmake<C>(cs, dir * sn), cj[u]), xv[u] * fac.inv_gamma,
                          (int)(kv[u] & (uint32_t)(L1 - 1)));
                }
            }
        }
    }
    for (int i = tid; i < RC * P; i += NT) buf[i] = cmake<C>(0, 0);
    // inter-pass twiddles of this thread's 16 grid points k1 (the same for every rank)
    C wt[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const C w = tw_big<C, -1>(hi, lo, n2 * (int64_t)(lt + q * TPF));
        wt[q] = dir > 0 ? cconj(w) : w;
    }
    __syncthreads();
    // this thread's run [i0, i1): the balanced split points moved to the next
    // grid-point boundary (soff[n + 1] is the first sample after point n)
    auto snap = [&](int b) __attribute__((always_inline)) {
        if (b <= 0 || b >= cnt) return b;
        int n1;
        if (b - 1 < SCAP) {
            C v;
            R z;
            get_s(b - 1, v, z, n1);
        } else {
            n1 = (int)(keys[tile_lo + b - 1] & (uint32_t)(L1 - 1));
        }
        return soff[n1 + 1];
    };
    const int i0 = snap((int)((int64_t)tid * cnt / NT)), i1 = snap((int)((int64_t)(tid + 1) * cnt / NT));
    for (int r0 = 0; r0 < fac.K; r0 += RC) {
        const int nr = min(RC, fac.K - r0);
        C a[RC];
#pragma unroll
        for (int gg = 0; gg < RC; ++gg) a[gg] = cmake<C>(0, 0);
        // rank r0 + gg with the factor i^q, q = -dir (r0 + gg), split as
        // (-1)^(q >> 1) on the coefficients and i^(q & 1), q & 1 = the rank's parity
        // (known at compile time when RC is even: r0 is then even)
        RankPoly<R> up[RC];
        bool odd[RC];
#pragma unroll
        for (int gg = 0; gg < RC; ++gg) {
            const int r = min(r0 + gg, fac.K - 1);
            up[gg] = rank_poly(fac, r);
            odd[gg] = RC % 2 == 0 ? (gg & 1) != 0 : (r & 1) != 0;
            if (((-dir * r) >> 1) & 1) {
#pragma unroll
                for (int m = 0; m < rank_terms<R>; ++m) up[gg].c[m] = -up[gg].c[m];
            }
        }
        int ncur = -1;
        // one sample of the walk: store the finished grid value when the grid
        // point changes, then add this sample's terms
        auto step = [&](const C &val, R z, int n1) __attribute__((always_inline)) {
            if (n1 != ncur) {
                if (ncur >= 0) {
#pragma unroll
                    for (int gg = 0; gg < RC; ++gg)
                        if (gg < nr) buf[gg * P + lds_pad(ncur)] = a[gg];
                }
#pragma unroll
                for (int gg = 0; gg < RC; ++gg) a[gg] = cmake<C>(0, 0);
                ncur = n1;
            }
            const R w = z * z;
#pragma unroll
            for (int gg = 0; gg < RC; ++gg) {
                if (gg < nr) {
                    R p = up[gg].c[rank_terms<R> - 1];
#pragma unroll
                    for (int m = rank_terms<R> - 2; m >= 0; --m) p = p * w + up[gg].c[m];
                    if (odd[gg]) {
                        p = p * z;
                        a[gg] = cmake<C>(a[gg].x - val.y * p, a[gg].y + val.x * p);
                    } else {
                        a[gg] = cmake<C>(a[gg].x + val.x * p, a[gg].y + val.y * p);
                    }
                }
            }
        };
        if (i1 <= SCAP) {
            // the whole slice is staged: its LDS reads go out four samples at a time
            for (int i = i0; i < i1; i += 4) {
                C vv[4];
                R zz[4];
                int nn[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) get_s(min(i + u, i1 - 1), vv[u], zz[u], nn[u]);
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (i + u < i1) step(vv[u], zz[u], nn[u]);
            }
        } else {
            for (int i = i0; i < i1; ++i) {
                if (i < SCAP) {
                    C v;
                    R z;
                    int n1;
                    get_s(i, v, z, n1);
                    step(v, z, n1);
                } else {
                    const R Xi = Xs[tile_lo + i];
                    R sn, cs;
                    sincospi_r(Xi, &sn, &cs);
                    step(cmul(cmake<C>(cs, dir * sn), csort[tile_lo + i]), Xi * fac.inv_gamma,
                         (int)(keys[tile_lo + i] & (uint32_t)(L1 - 1)));
                }
            }
        }
        if (ncur >= 0) {
#pragma unroll
            for (int gg = 0; gg < RC; ++gg)
                if (gg < nr) buf[gg * P + lds_pad(ncur)] = a[gg];
        }
        __syncthreads();
        block_fft_lds<C, L1, dir, fft_wave_sync<L1>, FR>(buf + g * P, tw, lt);   // each thread then reads only its own transform
        const int r = r0 + g;
        const bool more = r0 + RC < fac.K;   // a later chunk spreads into buf: clear what is read
        if constexpr (H) {
            // row g's block maximum over its TPF threads (whole waves when TPF >= 64)
            C o[16];
            float m = 0.0f;
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                C &b = buf[g * P + lds_pad(lt + q * TPF)];
                o[q] = cmul(b, wt[q]);
                if (more) b = cmake<C>(0, 0);
                m = fmaxf(m, cmaxabs(o[q]));
            }
            m = wave_max_group(m, TPF);
            const int par = (r0 / RC) & 1;
            if ((lt & 63) == 0) atomicMax(&smax[par * RC + g], __float_as_uint(m));
            __syncthreads();
            const int ex = hx_exponent(__uint_as_float(smax[par * RC + g]));
            if (tid < RC) smax[(par ^ 1) * RC + tid] = 0;   // its last readers finished at the previous chunk's end
            if (r < fac.K) {
                __half2 *Zr = reinterpret_cast<__half2 *>(Z) + (int64_t)r * L + n2 * L1;
#pragma unroll
                for (int q = 0; q < 16; ++q) Zr[lt + q * TPF] = hx_pack(o[q], ex);
                if (lt == 0) E[(int64_t)r * L2 + n2] = (int8_t)ex;
            }
        } else {
            C *Zr = Z + (int64_t)r * L + n2 * L1;
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int k1 = lt + q * TPF;
                C &b = buf[g * P + lds_pad(k1)];
                const C v = b;
                if (more) b = cmake<C>(0, 0);
                if (r < fac.K) Zr[k1] = cmul(v, wt[q]);
            }
        }
        __syncthreads();   // the next chunk overwrites buf
    }
}

// Adjoint / type-I pass B' for tiles with many more samples than grid points
// (M >> N): task = (tile n2, slice `part` of its sorted samples), splits slices
// per tile.  The slice's samples (up to SCAPD staged in LDS, the rest read from
// global memory) are spread with the balanced segmented sum, so a grid point
// holding hundreds of samples is shared by many threads; each slice's RC
// grids are transformed and written as partial rows to Zp, which
// k_sum_split_rows adds in slice order.
template <typename R, int L1, int RC, int SCAPD, int dir, bool TWG>
__global__ void __launch_bounds__(RC * L1 / 16)
k_passB_adj_dense(const cx_t<R> *__restrict__ csort, int64_t L2, const R *__restrict__ Xs,
                  const uint32_t *__restrict__ keys, const int32_t *__restrict__ off, Factors<R> fac,
                  const cx_t<R> *__restrict__ tw_g, const cx_t<R> *__restrict__ hi, const cx_t<R> *__restrict__ lo,
                  int splits, cx_t<R> *__restrict__ Zp)
{
    using C = cx_t<R>;
    constexpr int TPF = L1 / 16;
    constexpr int NT = RC * TPF;
    constexpr int P = fft_pitch(L1);
    __shared__ C buf[RC * P];
    __shared__ C tw_s[TWG ? 1 : L1];
    const C *tw = TWG ? tw_g : tw_s;
    __shared__ C sval[SCAPD];
    __shared__ R sz[SCAPD];
    __shared__ unsigned short spos[SCAPD];
    __shared__ C hv[RC * NT], tv[RC * NT];
    __shared__ int hix[NT], tix[NT], nxa[NT], nxb[NT];
    const int task = xcd_task((int)L2 * splits);
    if (task < 0) return;
    const int tid = threadIdx.x;
    if (!TWG) load_tw_s<C, L1, -1, NT>(tw_s, tw_g);   // tw_g already has the sign DIR
    const int g = tid / TPF, lt = tid % TPF;
    const int64_t n2 = task / splits;
    const int part = task % splits;
    const int t_lo = off[n2 * L1], t_cnt = off[(n2 + 1) * L1] - t_lo;
    const int base = t_lo + (int)((int64_t)t_cnt * part / splits);
    const int cnt = t_lo + (int)((int64_t)t_cnt * (part + 1) / splits) - base;
    const int nst = min(cnt, SCAPD);
    for (int i = tid; i < nst; i += NT) {
        const R xv = Xs[base + i];
        R sn, cs;
        sincospi_r(xv, &sn, &cs);
        sval[i] = cmul(cmake<C>(cs, dir * sn), csort[base + i]);
        sz[i] = xv * fac.inv_gamma;
        spos[i] = (unsigned short)(keys[base + i] & (uint32_t)(L1 - 1));
    }
    C wt[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const C w = tw_big<C, -1>(hi, lo, n2 * (int64_t)(lt + q * TPF));
        wt[q] = dir > 0 ? cconj(w) : w;
    }
    __syncthreads();
    struct Sample {
        int n;
        C val;
        R z;
    };
    auto load = [&](int i) -> Sample {
        if (i < SCAPD) return Sample{(int)spos[i], sval[i], sz[i]};
        const R xv = Xs[base + i];
        R sn, cs;
        sincospi_r(xv, &sn, &cs);
        return Sample{(int)(keys[base + i] & (uint32_t)(L1 - 1)), cmul(cmake<C>(cs, dir * sn), csort[base + i]),
                      xv * fac.inv_gamma};
    };
    auto pos = [&](int i) -> int { return load(i).n; };
    for (int r0 = 0; r0 < fac.K; r0 += RC) {
        const int nr = min(RC, fac.K - r0);
        for (int m = tid; m < RC * P; m += NT) buf[m] = cmake<C>(0, 0);
        __syncthreads();
        RankPoly<R> up[RC];
#pragma unroll
        for (int gg = 0; gg < RC; ++gg) up[gg] = rank_poly(fac, min(r0 + gg, fac.K - 1));
        // i^r for the type I, i^-r for the adjoint: a constant factor, applied after the transform
        auto contrib = [&](const Sample &sm, int gg) -> C { return cscale(sm.val, rank_eval(up[gg], sm.z)); };
        seg_spread<C, RC, NT>(cnt, nr, pos, load, contrib, buf, P, hv, tv, hix, tix, nxa, nxb);
        __syncthreads();
        block_fft_lds<C, L1, dir, fft_wave_sync<L1>>(buf + g * P, tw, lt);   // each thread then reads only its own transform
        const int r = r0 + g;
        if (r < fac.K) {
            C *Zr = Zp + (((int64_t)n2 * splits + part) * fac.K + r) * L1;
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int k1 = lt + q * TPF;
                Zr[k1] = crot(cmul(buf[g * P + lds_pad(k1)], wt[q]), -dir * r);
            }
        }
        __syncthreads();   // the next chunk overwrites buf
    }
}

// Rows of the adjoint pass B' whose tile was split over `splits` tasks: the
// partial rows are added in slice order (a fixed order: deterministic) into
// Z_r[n2][:]; with the half-precision exchange the row gets its block
// exponent here.  Block = (n2, r), L1 <= 4096 = 256 x 16.
template <typename R, bool H>
__global__ void __launch_bounds__(256)
k_sum_split_rows(const cx_t<R> *__restrict__ Zp, int splits, int K, int L1, int64_t L2, cx_t<R> *__restrict__ Z,
                 int8_t *__restrict__ E)
{
    using C = cx_t<R>;
    const int64_t n2 = blockIdx.x;
    const int r = blockIdx.y;
    const int64_t L = (int64_t)L1 * L2;
    C acc[16];
    float m = 0.0f;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int k1 = threadIdx.x + e * 256;
        acc[e] = cmake<C>(0, 0);
        if (k1 < L1) {
            for (int q = 0; q < splits; ++q) acc[e] = cadd(acc[e], Zp[((n2 * splits + q) * K + r) * L1 + k1]);
            if constexpr (H) m = fmaxf(m, cmaxabs(acc[e]));
        }
    }
    if constexpr (H) {
        __shared__ unsigned smax;
        if (threadIdx.x == 0) smax = 0;
        __syncthreads();
        m = wave_max_group(m, 64);
        if ((threadIdx.x & 63) == 0) atomicMax(&smax, __float_as_uint(m));
        __syncthreads();
        const int ex = hx_exponent(__uint_as_float(smax));
        __half2 *Zr = reinterpret_cast<__half2 *>(Z) + (int64_t)r * L + n2 * L1;
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int k1 = threadIdx.x + e * 256;
            if (k1 < L1) Zr[k1] = hx_pack(acc[e], ex);
        }
        if (threadIdx.x == 0) E[(int64_t)r * L2 + n2] = (int8_t)ex;
    } else {
        C *Zr = Z + (int64_t)r * L + n2 * L1;
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int k1 = threadIdx.x + e * 256;
            if (k1 < L1) Zr[k1] = acc[e];
        }
    }
}

// Where the wide column blocks run (FP32 plans with the full-precision exchange
// and the default schedule): columns of 2048 points (at 1024 points the narrow
// pass A measured faster, 35 against 40 us at 2^20); pass A' also needs
// L1/G >= 256 column groups, since it cannot split its ranks over workgroups
// (at 2^20, 64 wide workgroups took 101 us against 47 us for the narrow kernel).
// (L1 is a power of two on every plan; the wide kernels form row offsets by shifts)
#define WIDE_A(L1, L2) ((L2) == 2048 && ((L1) & ((L1) - 1)) == 0)
#define WIDE_A_ADJ(L1, L2) ((L2) == 2048 && (L1) / 8 >= 256 && ((L1) & ((L1) - 1)) == 0)
// Pass A' with wide column blocks (FP32; launched at L2 = 2048 with at least
// 256 column groups, see WIDE_A_ADJ): G columns per workgroup, each thread
// transforming two of them, so that the intermediate is read in G*8-byte runs
// (64 bytes at G = 8, G*4 = 32 bytes for the half-precision exchange; a
// 16-byte-run read of the same block measured 2.3 TB/s against 4.1 TB/s at
// 64 bytes).  The rank's block goes to LDS in two rounds of sixteen loads per
// thread (no register prefetch: the accumulators of 32 outputs hold the
// registers); outputs (k1, n2) with k1 = tid mod G accumulate in registers.
// H: Z in fp16 pairs scaled per (rank, row) by 2^E[r * L2 + n2]; the rank's L2
// row exponents are staged in LDS first (one 4-byte word per thread).
template <typename R, int L2, int G, int DIR, bool H = false, int FR = 16>
__global__ void __launch_bounds__(G / 2 * L2 / 16)
k_passA_adj_wide(const cx_t<R> *__restrict__ Z, int64_t N, int64_t L1, int K, const cx_t<R> *__restrict__ tw_g,
                 cx_t<R> *__restrict__ out, const int8_t *__restrict__ E = nullptr)
{
    using C = cx_t<R>;
    constexpr int TPF = L2 / 16;
    constexpr int GH = G / 2;
    constexpr int NT = GH * TPF;
    constexpr int P = fft_pitch_g(L2, G);
    constexpr int ST = NT / G;
    static_assert(fft_radix_p(L2) == 1 && NT % G == 0 && G * L2 == 32 * NT, "two halves of 16 elements");
    static_assert(!H || (sizeof(R) == 4 && L2 == 4 * NT), "the half exchange: FP32, one exponent word per thread");
    __shared__ C buf[G * P];
    __shared__ C tw_s[L2];
    __shared__ uint32_t sexp[H ? L2 / 4 : 1];   // the rank's row exponents (int8), four per word
    const int task = xcd_task((int)(L1 / G));
    if (task < 0) return;
    load_tw_s<C, L2, -1, NT>(tw_s, tw_g);   // tw_g already has the sign DIR
    const int tid = threadIdx.x;
    const int g = tid / TPF, lt = tid % TPF;
    const int64_t k1_0 = (int64_t)task * G;
    const int64_t L = L1 * L2;
    const ZMap zm = zmap(N);
    const int gg = tid % G, n2_0 = tid / G;
    const int l1s = __builtin_ctzll((unsigned long long)L1);   // L1 is a power of two: offsets are shifts
    C acc[32];
#pragma unroll
    for (int e = 0; e < 32; ++e) acc[e] = cmake<C>(0, 0);
    for (int r = 0; r < K; ++r) {
        __syncthreads();   // the previous rank's readers of buf are done
        // (an opaque copy of the thread index: the 32 load and LDS addresses are
        // formed per rank instead of being kept in registers across ranks)
        int ti = tid;
        asm volatile("" : "+v"(ti));
        const int64_t zo = (int64_t)r * L + k1_0 + ti % G + ((int64_t)(ti / G) << l1s);
        if constexpr (H) sexp[tid] = reinterpret_cast<const uint32_t *>(E + (int64_t)r * L2)[tid];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            using Raw = typename std::conditional<H, __half2, C>::type;
            Raw cl[16];
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int64_t at = zo + ((int64_t)((h * 16 + e) * ST) << l1s);
                if constexpr (H) cl[e] = reinterpret_cast<const __half2 *>(Z)[at];
                else cl[e] = Z[at];
            }
            if (H && h == 0) __syncthreads();   // the exponents are visible (the first round's loads in flight)
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int n = ti / G + (h * 16 + e) * ST;
                C v;
                if constexpr (H) v = hx_unpack(cl[e], reinterpret_cast<const int8_t *>(sexp)[n]);
                else v = cl[e];
                buf[(ti % G) * P + lds_pad(n)] = v;
            }
        }
        __syncthreads();
#pragma unroll
        for (int h = 0; h < 2; ++h) block_fft_lds<C, L2, DIR, fft_wave_sync<L2>, FR>(buf + (g + h * GH) * P, tw_s, lt);
        __syncthreads();   // every transform is visible
        const int n2o = ti / G, go = ti % G;
#pragma unroll
        for (int h = 0; h < 32; h += 8) {
            R zq[8], wq[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) zq[e] = zcoord<R>((int64_t)((int)k1_0 + go + ((n2o + ST * (h + e)) << l1s)), zm);
            cheb_v_many<R, 8>(r, zq, wq);
#pragma unroll
            for (int e = 0; e < 8; ++e)
                acc[h + e] = cadd(acc[h + e], cscale(buf[go * P + lds_pad(n2o + ST * (h + e))], wq[e]));
        }
    }
#pragma unroll
    for (int e = 0; e < 32; ++e) {
        const int64_t k = k1_0 + gg + L1 * (int64_t)(n2_0 + ST * e);
        if (k < N) out[k] = acc[e];
    }
}

// Pass A' of type I / adjoint.  Task = G adjacent columns k1.  For each r the
// columns Z_r[:][k1] (the next rank's block is loaded into registers while
// this one is transformed) are transformed along n2 -> k2 and accumulated
// with weight v_r(k1 + L1 k2) in registers; the sum over r is written once.
// H: Z holds fp16 pairs scaled per (rank, row) by 2^E[r * L2 + n2].
template <typename R, int L2, int G, int DIR, bool TWG, bool H, int FR = 16>
__global__ void __launch_bounds__(G * L2 / 16)
k_passA_adj(const cx_t<R> *__restrict__ Z, int64_t N, int64_t L1, int K, const cx_t<R> *__restrict__ tw_g,
            cx_t<R> *__restrict__ out, const int8_t *__restrict__ E)
{
    using C = cx_t<R>;
    constexpr int TPF = L2 / 16;
    constexpr int NT = G * TPF;
    constexpr int P = fft_pitch_g(L2, G);
    __shared__ C buf[G * P];
    __shared__ C tw_s[TWG ? 1 : L2];
    const C *tw = TWG ? tw_g : tw_s;   // tw_g already has sign DIR
    const int task = xcd_task((int)(L1 / G));
    if (task < 0) return;
    if (!TWG) load_tw_s<C, L2, -1, NT>(tw_s, tw_g);
    const int tid = threadIdx.x;
    const int g = tid / TPF, lt = tid % TPF;
    const int64_t k1_0 = (int64_t)task * G;
    const int64_t L = L1 * L2;
    const ZMap zm = zmap(N);
    C acc[16];
    // rank r's block of G columns in raw registers (fp16 pairs for H); for H the
    // rank's L2 row exponents go through LDS (L2 / NT = 16 / G bytes per thread,
    // one load), which keeps 16 exponent registers out of this register-bound kernel
    using Raw = typename std::conditional<H, __half2, C>::type;
    constexpr int EB = 16 / G;   // exponent bytes per thread
    using EWord = typename std::conditional<EB == 8, uint2, typename std::conditional<EB == 4, uint32_t,
                                            uint16_t>::type>::type;
    static_assert(!H || (EB == 2 || EB == 4 || EB == 8), "G must be 2, 4 or 8 for the half exchange");
    __shared__ EWord sexp[H ? 2 * NT : 1];
    Raw zn[16];
    auto fetch = [&](int r) {
        if constexpr (H) {   // the exponent word first, so that its wait leaves the values in flight
            const EWord ew = reinterpret_cast<const EWord *>(E + (int64_t)r * L2)[tid];
            sexp[(r & 1) * NT + tid] = ew;
        }
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int i = tid + e * NT;
            const int64_t at = (int64_t)r * L + k1_0 + (i % G) + (int64_t)(i / G) * L1;
            if constexpr (H) zn[e] = reinterpret_cast<const __half2 *>(Z)[at];
            else zn[e] = Z[at];
        }
    };
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[e] = cmake<C>(0, 0);
    fetch(0);
    for (int r = 0; r < K; ++r) {
        __syncthreads();   // previous readers of buf are done; rank r's exponents are visible
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int i = tid + e * NT;
            C v;
            if constexpr (H) {
                const int8_t *ex = reinterpret_cast<const int8_t *>(sexp + (r & 1) * NT);
                v = hx_unpack(zn[e], ex[i / G]);
            } else {
                v = zn[e];
            }
            buf[(i % G) * P + lds_pad(i / G)] = v;
        }
        if (r + 1 < K) fetch(r + 1);   // its exponents go to the other parity, last read at rank r - 1
        __syncthreads();
        block_fft_any_lds<C, L2, DIR, FR>(buf + g * P, tw, lt);
#pragma unroll
        for (int h = 0; h < 16; h += 8) {   // two halves of 8: bounded transient registers
            R zq[8], wq[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int i = tid + (h + e) * NT;
                zq[e] = zcoord<R>(k1_0 + (i % G) + L1 * (int64_t)(i / G), zm);
            }
            cheb_v_many<R, 8>(r, zq, wq);
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int i = tid + (h + e) * NT;
                acc[h + e] = cadd(acc[h + e], cscale(buf[(i % G) * P + fft_out_pos<L2>(i / G)], wq[e]));
            }
        }
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int i = tid + e * NT;
        const int64_t k = k1_0 + (i % G) + L1 * (int64_t)(i / G);
        if (k < N) out[k] = acc[e];
    }
}

// ============================================================================
// dispatch
// ============================================================================

static inline int ilog2(int64_t v) { int l = 0; while ((int64_t(1) << l) < v) ++l; return l; }

// Tasks per tile of pass B: 1 while a tile holds about one round of samples
// (M ~ N); with many more samples than grid points the tiles are split so that
// each task keeps about max(CAP, L1) samples (the row transforms it repeats
// are then a small part of its work), at most 64 ways.
static int pass_b_splits(int64_t M, int L2, int L1, int cap)
{
    const int64_t per = std::max<int64_t>(cap, L1);
    const int64_t want = (M + (int64_t)L2 * per - 1) / ((int64_t)L2 * per);
    return (int)std::min<int64_t>(64, std::max<int64_t>(1, want));
}

// Samples staged in LDS by one adjoint pass-B' workgroup (SCAP of the
// instantiations below), per row length L1 and precision.
static constexpr int pba_cap(int L1, bool fp32)
{
    return L1 <= 128 ? 256 : L1 == 256 ? 384 : L1 == 512 ? 768 : L1 == 1024 ? 1280 : L1 == 2048 ? 2304
                                                                                                 : (fp32 ? 5120 : 2560);
}
// Samples staged per task of the dense-tile adjoint pass B' (measured: the
// smaller staging lets two workgroups share a CU at L1 = 128).
static constexpr int pba_dense_cap(int L1, bool fp32) { return (L1 <= 128 ? 1024 : 2048) / (fp32 ? 1 : 2); }

// Dense-tile adjoint pass B': 0 (not used) while the tiles hold at most twice
// the staging capacity of the per-grid-point walk on average; else the number
// of slices per tile, about one dense staging load each, at most 64.  The
// plan sizes Zp (slices x K x L partial rows) by the same rule.
int pass_b_adj_splits(int64_t M, int L2, int L1, bool fp32)
{
    if (L2 <= 1) return 0;
    const int64_t avg = M / L2;
    if (avg <= 2 * (int64_t)pba_cap(L1, fp32)) return 0;
    const int64_t cap = pba_dense_cap(L1, fp32);
    return (int)std::min<int64_t>(64, std::max<int64_t>(1, (avg + cap - 1) / cap));
}

// Launches CALL with the compile-time flag HX = a.half (FP32 plans with the
// half-precision exchange), HX = false otherwise.
#define HX_DISPATCH(CALL)                                                                                  \
    do {                                                                                                   \
        auto go_ = [&](auto hc_) {                                                                         \
            constexpr bool HX = decltype(hc_)::value;                                                      \
            CALL;                                                                                          \
        };                                                                                                 \
        bool done_ = false;                                                                                \
        if constexpr (sizeof(R) == 4) {                                                                    \
            if (a.half) {                                                                                  \
                go_(std::true_type{});                                                                     \
                done_ = true;                                                                              \
            }                                                                                              \
        }                                                                                                  \
        if (!done_) go_(std::false_type{});                                                                \
    } while (0)

template <typename R, int L>
static void run_small_fwd(const FusedArgs<R> &a, const cx_t<R> *c, cx_t<R> *f, int mode,
                          const cx_t<R> *g, double *gx, hipStream_t s)
{
    const int64_t per = SMALL_NT * SMALL_SLOTS;
    const unsigned nb = (unsigned)((a.M + per - 1) / per);
    if (nb == 0) return;
    prof_begin(a.prof, mode ? "gradx_small" : "fwd_small", s);
    hipLaunchKernelGGL((k_small_fwd<R, L>), dim3(nb), dim3(SMALL_NT), 0, s, c, a.N, a.M, a.t, a.X, a.fac,
                       a.tw1, f, mode, g, gx);
    prof_end(a.prof, s);
}

template <typename R, int L, int DIR>
static hipError_t run_small_adj(const FusedArgs<R> &a, const cx_t<R> *c, cx_t<R> *f, hipStream_t s)
{
    const int64_t span_min = 65536;
    int64_t nparts = (a.M + span_min - 1) / span_min;
    if (nparts < 1) nparts = 1;
    if (nparts > 1 && nparts * a.N > a.part_cap) nparts = a.part_cap / a.N;
    if (nparts < 1) nparts = 1;
    const int64_t span = (a.M + nparts - 1) / nparts;
    const char *nm = DIR > 0 ? "adj_small" : "type1_small";
    if (nparts == 1) {
        prof_begin(a.prof, nm, s);
        hipLaunchKernelGGL((k_small_adj<R, L, DIR>), dim3(1), dim3(SMALL_NT), 0, s, c, a.N, a.M,
                           (int64_t)(a.M > 0 ? a.M : 1), a.perm, a.Xs, a.off, a.fac, a.tw1, f);
        prof_end(a.prof, s);
    } else {
        prof_begin(a.prof, nm, s);
        hipLaunchKernelGGL((k_small_adj<R, L, DIR>), dim3((unsigned)nparts), dim3(SMALL_NT), 0, s, c, a.N,
                           a.M, span, a.perm, a.Xs, a.off, a.fac, a.tw1, a.part);
        prof_end(a.prof, s);
        prof_begin(a.prof, "sum_parts", s);
        hipLaunchKernelGGL(k_sum_parts<R>, dim3((unsigned)((a.N + 255) / 256)), dim3(256), 0, s,
                           (const cx_t<R> *)a.part, (int)nparts, a.N, f);
        prof_end(a.prof, s);
    }
    return hipGetLastError();
}

// Column lengths L2 = 3 * 2^k and 5 * 2^k of the oversampled grids between
// powers of two (radix-3/5 stage, then power-of-two transforms of 64 to 512
// points), with the columns per pass-A / pass-A' workgroup in FP32 and FP64
// (half as many in FP64, whose transforms hold twice the registers).
#define MIXED_L2_SWITCH(MACRO) \
    MACRO(192, 16, 8)          \
    MACRO(384, 16, 8)          \
    MACRO(768, 8, 4)           \
    MACRO(1536, 4, 2)          \
    MACRO(320, 16, 8)          \
    MACRO(640, 8, 4)           \
    MACRO(1280, 4, 2)

#define SMALL_SWITCH(MACRO) \
    switch (a.L) {          \
        MACRO(16)           \
        MACRO(32)           \
        MACRO(64)           \
        MACRO(128)          \
        MACRO(256)          \
        MACRO(512)          \
        MACRO(1024)         \
        MACRO(2048)         \
        MACRO(4096)         \
    default: return hipErrorInvalidValue; \
    }

// Launch shapes of the two-pass kernels at the large tile sizes (FP32).  The
// defaults can be overridden at compile time to compare shapes.
#ifndef NUFFT_F32_GA1024
#define NUFFT_F32_GA1024 8      // pass A: adjacent columns per workgroup at L2 = 1024
#endif
#ifndef NUFFT_F32_GA2048
#define NUFFT_F32_GA2048 4
#endif
#ifndef NUFFT_F32_GAA1024
#define NUFFT_F32_GAA1024 4     // pass A'
#endif
#ifndef NUFFT_F32_GAA2048
#define NUFFT_F32_GAA2048 2
#endif
#ifndef NUFFT_F32_PB2048_RC
#define NUFFT_F32_PB2048_RC 4   // pass B at L1 = 2048: ranks side by side, sample slots
#endif
#ifndef NUFFT_F32_PB2048_S
#define NUFFT_F32_PB2048_S 5
#endif
#ifndef NUFFT_F32_PBA2048_RC
#define NUFFT_F32_PBA2048_RC 2  // adjoint pass B' at L1 = 2048: ranks side by side
#endif
#ifndef NUFFT_F32_PB1024_RC
#define NUFFT_F32_PB1024_RC 4
#endif
#ifndef NUFFT_F32_PB1024_S
#define NUFFT_F32_PB1024_S 5
#endif

// Column groups per pass-A workgroup: G adjacent columns (G x 8-byte runs in
// FP32) while the LDS budget allows.
template <typename R> struct Cfg;
template <> struct Cfg<float> {
    static constexpr int G1024 = NUFFT_F32_GA1024, G2048 = NUFFT_F32_GA2048;
    static constexpr int GA1024 = NUFFT_F32_GAA1024, GA2048 = NUFFT_F32_GAA2048;
};
template <> struct Cfg<double> {
    static constexpr int G1024 = 4, G2048 = 2;
    static constexpr int GA1024 = 4, GA2048 = 2;
};

// Ranks per pass-A task.  Every task pays a fixed set-up (twiddle table and
// the column block of c), so ranks are split only until there are about one
// task per CU.
static inline int pass_a_ranks(int K, int ncg)
{
    const int want = 256;
    int nrc = (want + ncg - 1) / ncg;           // rank chunks per column group
    if (nrc < 1) nrc = 1;
    if (nrc > K) nrc = K;
    return (K + nrc - 1) / nrc;
}

// ---- launches of the two-pass kernels, and the tuning schedules ----------------
// A plan's schedule (FusedArgs::sched, chosen by timing at plan time) selects,
// for FP32 two-pass plans with L1, L2 in {1024, 2048}:
//   0  the default shapes, FFT stages 16 x 16 x ... (first radix 16);
//   1  the default shapes with first radix 8 (8 x 16 x 16 for 2048 points,
//      8 x 16 x 8 for 1024), which reads the plan's radix-8 twiddle tables;
//   2  the alternative tile shapes: half the columns per pass-A workgroup,
//      pass B with half the ranks side by side and twice the sample slots,
//      pass B' with half the ranks, twice the columns per pass-A' workgroup.
// Other plans always run schedule 0.
static inline bool sched_sizes(int L1, int64_t L2)
{
    return (L1 == 1024 || L1 == 2048) && (L2 == 1024 || L2 == 2048);
}

template <typename R, int LL, int G, bool HX, int FR>
static void launch_pass_a(const FusedArgs<R> &a, const cx_t<R> *c, int mode, hipStream_t s)
{
    const int ncg = a.L1 / G, rca = pass_a_ranks(a.fac.K, ncg);
    const int T = ncg * ((a.fac.K + rca - 1) / rca);
    hipLaunchKernelGGL((k_passA<R, LL, G, false, HX, FR>), dim3(xcd_grid(T)), dim3(G * LL / 16), 0, s, c, a.N,
                       (int64_t)a.L1, a.fac.K, rca, mode, FR == 8 ? a.tw2r8 : a.tw2, a.hi, a.lo, a.Y, a.E);
}

// Grid for a kernel whose workgroups take their tasks in turn (xcd_tasks): the
// workgroups the device holds at once (per-CU occupancy x CUs, rounded down to a
// multiple of 8), at most xcd_grid(T).  cap caches the answer per device and
// belongs to one kernel (kernels of one signature share the pointer type F, so
// the caller keeps it: 0 not queried yet, -1 no answer, one block per task).
constexpr int RESIDENT_MAXDEV = 64;
template <typename F>
static unsigned resident_grid(F kernel, int threads, int T, std::atomic<int> (&cap)[RESIDENT_MAXDEV])
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= RESIDENT_MAXDEV) return xcd_grid(T);
    int c = cap[dev].load(std::memory_order_relaxed);
    if (c == 0) {   // concurrent first calls may both query; they store the same answer
        int per_cu = 0, ncu = 0;
        const bool ok = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) == hipSuccess &&
                        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess;
        c = ok && per_cu * ncu >= 8 ? (per_cu * ncu) / 8 * 8 : -1;
        cap[dev].store(c, std::memory_order_relaxed);
    }
    const unsigned full = xcd_grid(T);
    return c > 0 && (unsigned)c < full ? (unsigned)c : full;
}

// Pass B writes its outputs through the destination-bucketed layout (a.bbuf,
// then bucket_to_samples) when the plan has one and the shapes allow it; returns whether it did.
template <typename R, int LL, int RR, int SS, bool HX, int FR, int MODE = -1>
static bool launch_pass_b(const FusedArgs<R> &a, cx_t<R> *f, int mode, const cx_t<R> *g, double *gx, hipStream_t s)
{
    const int sp = pass_b_splits(a.M, a.L2, LL, RR * (LL / 16) * SS);
    const int nbk = (int)((a.M + (int64_t(1) << a.bshift) - 1) >> a.bshift);
    // the bucket counts are scanned by the workgroup's threads, two each
    const bool buck = a.bdst && a.fac.K > RR && nbk <= 2 * RR * (LL / 16) &&
                      pass_b_buckets(LL, RR, SS, (int)sizeof(cx_t<R>));
    const auto kern = k_passB<R, LL, RR, SS, false, HX, FR, MODE>;
    static std::atomic<int> cap[RESIDENT_MAXDEV];   // this instantiation's resident workgroups per device
    hipLaunchKernelGGL(kern, dim3(resident_grid(kern, RR * LL / 16, (int)a.L2 * sp, cap)), dim3(RR * LL / 16), 0, s,
                       (const cx_t<R> *)a.Y, (int64_t)a.L2, a.M, a.keys, a.perm, a.Xs, a.off, a.fac,
                       FR == 8 ? a.tw1r8 : a.tw1, f, mode, g, gx, a.E, sp, buck ? a.bdst : nullptr, a.bshift, nbk,
                       a.bbuf);
    return buck;
}

template <typename R, int LL, int RR, int SC, int DIR, bool TG, bool HX, int FR>
static void launch_pass_b_adj(const FusedArgs<R> &a, hipStream_t s)
{
    const cx_t<R> *tw = FR == 8 ? (DIR < 0 ? a.tw1r8 : a.tw1ir8) : (DIR < 0 ? a.tw1 : a.tw1i);
    hipLaunchKernelGGL((k_passB_adj<R, LL, RR, SC, DIR, TG, HX, FR>), dim3(xcd_grid(a.L2)), dim3(RR * LL / 16), 0, s,
                       a.gsort, (int64_t)a.L2, a.Xs, a.keys, a.off, a.fac, tw, a.hi, a.lo, a.Y, a.E);
}

template <typename R, int LL, int G, int DIR, bool HX, int FR>
static void launch_pass_a_adj(const FusedArgs<R> &a, cx_t<R> *f, hipStream_t s)
{
    const cx_t<R> *tw = FR == 8 ? (DIR < 0 ? a.tw2r8 : a.tw2ir8) : (DIR < 0 ? a.tw2 : a.tw2i);
    hipLaunchKernelGGL((k_passA_adj<R, LL, G, DIR, false, HX, FR>), dim3(xcd_grid(a.L1 / G)), dim3(G * LL / 16), 0, s,
                       (const cx_t<R> *)a.Y, a.N, (int64_t)a.L1, a.fac.K, tw, f, a.E);
}

// Schedules 1 and 2 of an FP32 plan (false: not this plan's sizes, run the default).
// GD: columns per workgroup relative to the default (1, or 2 for half as many);
// FR: first radix.
template <typename R, int GD, int FR>
static bool tuned_pass_a(const FusedArgs<R> &a, const cx_t<R> *c, int mode, hipStream_t s)
{
    if (a.half || !sched_sizes(a.L1, a.L2)) return false;
    if (a.L2 == 1024) launch_pass_a<R, 1024, Cfg<R>::G1024 / GD, false, FR>(a, c, mode, s);
    else launch_pass_a<R, 2048, Cfg<R>::G2048 / GD, false, FR>(a, c, mode, s);
    return true;
}
template <typename R, int RD, int FR>
static bool tuned_pass_b(const FusedArgs<R> &a, cx_t<R> *f, int mode, const cx_t<R> *g, double *gx, hipStream_t s,
                         bool *buck)
{
    if (a.half || !sched_sizes(a.L1, a.L2)) return false;
    if (a.L1 == 1024)
        *buck = launch_pass_b<R, 1024, NUFFT_F32_PB1024_RC / RD, NUFFT_F32_PB1024_S * RD, false, FR>(a, f, mode, g, gx, s);
    else
        *buck = launch_pass_b<R, 2048, NUFFT_F32_PB2048_RC / RD, NUFFT_F32_PB2048_S * RD, false, FR>(a, f, mode, g, gx, s);
    return true;
}
template <typename R, int DIR, int RD, int FR>
static bool tuned_pass_b_adj(const FusedArgs<R> &a, hipStream_t s)
{
    if (a.half || !sched_sizes(a.L1, a.L2)) return false;
    if (a.L1 == 1024) launch_pass_b_adj<R, 1024, 4 / RD, pba_cap(1024, true), DIR, false, false, FR>(a, s);
    else launch_pass_b_adj<R, 2048, NUFFT_F32_PBA2048_RC / RD, pba_cap(2048, true), DIR, true, false, FR>(a, s);
    return true;
}
template <typename R, int DIR, int GM, int FR>
static bool tuned_pass_a_adj(const FusedArgs<R> &a, cx_t<R> *f, hipStream_t s)
{
    if (a.half || !sched_sizes(a.L1, a.L2)) return false;
    if (a.L2 == 1024) launch_pass_a_adj<R, 1024, Cfg<R>::GA1024 * GM, DIR, false, FR>(a, f, s);
    else launch_pass_a_adj<R, 2048, Cfg<R>::GA2048 * GM, DIR, false, FR>(a, f, s);
    return true;
}

template <typename R>
hipError_t fused_type2(const FusedArgs<R> &a, const cx_t<R> *c, cx_t<R> *f, int mode, const cx_t<R> *g,
                       double *gx, hipStream_t s)
{
    if (a.L2 == 1) {
#define SF(LL) case LL: run_small_fwd<R, LL>(a, c, f, mode, g, gx, s); break;
        SMALL_SWITCH(SF)
#undef SF
        return hipGetLastError();
    }
    if (mode != 0) {   // the derivative pass reads g in sorted order
        if (!a.presorted) {
            const hipError_t e = fused_sort_input<R>(a, g, "gradx_sort", s);
            if (e != hipSuccess) return e;
        }
        g = a.gsort;
    }
    // pass A
    prof_begin(a.prof, mode ? "gradx_passA" : "fwd_passA", s);
    bool ok = false;
    if constexpr (sizeof(R) == 4) {
        if (a.sched == 1) ok = tuned_pass_a<R, 1, 8>(a, c, mode, s);          // 8 x 16 x ... column FFTs
        else if (a.sched == 2) ok = tuned_pass_a<R, 2, 16>(a, c, mode, s);    // half the columns per workgroup
    }
    if constexpr (sizeof(R) == 4) {
        if (!ok && WIDE_A(a.L1, a.L2)) {   // L2 = 2048: eight columns per workgroup
            const int ncg = a.L1 / 8, rca = pass_a_ranks(a.fac.K, ncg);
            const int T = ncg * ((a.fac.K + rca - 1) / rca);
            HX_DISPATCH(hipLaunchKernelGGL((k_passA_wide<R, 2048, 8, HX>), dim3(xcd_grid(T)), dim3(4 * 128), 0, s, c,
                                           a.N, (int64_t)a.L1, a.fac.K, rca, mode, a.tw2, a.hi, a.lo, a.Y, a.E));
            ok = true;
        }
    }
    if (!ok) {
        switch (a.L2) {
#define PA(LL, GG)                                                                                         \
    case LL: {                                                                                             \
        constexpr int G = GG;                                                                              \
        HX_DISPATCH((launch_pass_a<R, LL, G, HX, 16>(a, c, mode, s)));                                      \
        break;                                                                                             \
    }
            PA(64, 8)
            PA(128, 8)
            PA(256, 8)
            PA(512, 8)
            PA(1024, Cfg<R>::G1024)
            PA(2048, Cfg<R>::G2048)
#undef PA
#define PAM(LL, GF, GD)                                                                                    \
    case LL:                                                                                               \
        if (a.half) return hipErrorInvalidValue;                                                           \
        launch_pass_a<R, LL, sizeof(R) == 4 ? GF : GD, false, 16>(a, c, mode, s);                          \
        break;
            MIXED_L2_SWITCH(PAM)
#undef PAM
        default: return hipErrorInvalidValue;
        }
    }
    prof_end(a.prof, s);
    // pass B: RC ranks side by side, S sample slots per thread (about 1.25 x the
    // mean tile population L1 when M = N)
    prof_begin(a.prof, mode ? "gradx_passB" : "fwd_passB", s);
    ok = false;
    bool buck = false;   // pass B wrote the outputs in the destination-bucketed layout
    if constexpr (sizeof(R) == 4) {
        if (a.sched == 1) ok = tuned_pass_b<R, 1, 8>(a, f, mode, g, gx, s, &buck);
        else if (a.sched == 2) ok = tuned_pass_b<R, 2, 16>(a, f, mode, g, gx, s, &buck);
    }
    if constexpr (sizeof(R) == 4) {
        // 2048-point rows: two ranks side by side and nine sample slots, the registers held
        // to two 4-wave workgroups per CU (some spill), one kernel per mode so that each has
        // its own register allocation (31 spills each, against 66 for one kernel serving
        // both).  Measured at 2^22: forward 155 against 164 us, derivative 156 against 171.
        if (!ok && !a.half && a.L1 == 2048) {
            buck = mode == 0 ? launch_pass_b<R, 2048, 2, 9, false, 16, 0>(a, f, mode, g, gx, s)
                             : launch_pass_b<R, 2048, 2, 9, false, 16, 1>(a, f, mode, g, gx, s);
            ok = true;
        }
    }
    if (!ok) {
        switch (a.L1) {
#define PB(LL, RF, SF, RD, SD)                                                                             \
    case LL: {                                                                                             \
        constexpr bool F = sizeof(R) == 4;                                                                 \
        constexpr int RR = F ? RF : RD, SS = F ? SF : SD;                                                  \
        HX_DISPATCH((buck = launch_pass_b<R, LL, RR, SS, HX, 16>(a, f, mode, g, gx, s)));                   \
        break;                                                                                             \
    }
            PB(128, 16, 1, 8, 2)
            PB(256, 16, 2, 8, 3)
            PB(512, 8, 3, 4, 5)
            PB(1024, NUFFT_F32_PB1024_RC, NUFFT_F32_PB1024_S, 4, 5)
            PB(2048, NUFFT_F32_PB2048_RC, NUFFT_F32_PB2048_S, 2, 5)
            PB(4096, 2, 10, 1, 5)
#undef PB
        default: return hipErrorInvalidValue;
        }
    }
    prof_end(a.prof, s);
    if (buck) {   // the bucketed outputs to sample order
        prof_begin(a.prof, mode ? "gradx_unsort" : "fwd_unsort", s);
        const hipError_t e = mode ? bucket_to_samples<double>(a, (const double *)a.bbuf, gx, s)
                                  : bucket_to_samples<cx_t<R>>(a, (const cx_t<R> *)a.bbuf, f, s);
        prof_end(a.prof, s);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

template <typename R, int DIR>
static hipError_t fused_type1_dir(const FusedArgs<R> &a, const cx_t<R> *c, cx_t<R> *f, hipStream_t s)
{
    if (a.L2 == 1) {
#define SA(LL) case LL: return run_small_adj<R, LL, DIR>(a, c, f, s);
        SMALL_SWITCH(SA)
#undef SA
    }
    if (!a.presorted) {
        const hipError_t e = fused_sort_input<R>(a, c, DIR > 0 ? "adj_sort" : "type1_sort", s);
        if (e != hipSuccess) return e;
    }
    const int sp = pass_b_adj_splits(a.M, a.L2, a.L1, sizeof(R) == 4);
    if (sp > 0 && !a.Zp) return hipErrorInvalidValue;   // the plan sizes Zp by the same rule
    prof_begin(a.prof, DIR > 0 ? "adj_passB" : "type1_passB", s);
    bool ok = false;
    if constexpr (sizeof(R) == 4) {
        if (sp == 0 && a.sched == 1) ok = tuned_pass_b_adj<R, DIR, 1, 8>(a, s);
        else if (sp == 0 && a.sched == 2) ok = tuned_pass_b_adj<R, DIR, 2, 16>(a, s);
    }
    if (!ok) {
        switch (a.L1) {
#define PBA(LL, RF, RD, TG)                                                                                \
    case LL: {                                                                                             \
        constexpr bool F = sizeof(R) == 4;                                                                 \
        constexpr int RR = F ? RF : RD, SC = pba_cap(LL, F);                                               \
        if (sp > 0) {                                                                                      \
            hipLaunchKernelGGL((k_passB_adj_dense<R, LL, RR, pba_dense_cap(LL, F), DIR, TG>),              \
                               dim3(xcd_grid(a.L2 * sp)), dim3(RR * LL / 16), 0, s, a.gsort, (int64_t)a.L2,  \
                               a.Xs, a.keys, a.off, a.fac, DIR < 0 ? a.tw1 : a.tw1i, a.hi, a.lo, sp, a.Zp);  \
        } else {                                                                                           \
            HX_DISPATCH((launch_pass_b_adj<R, LL, RR, SC, DIR, TG, HX, 16>(a, s)));                         \
        }                                                                                                  \
        break;                                                                                             \
    }
            PBA(128, 16, 8, false)
            PBA(256, 16, 8, false)
            PBA(512, 8, 4, false)
            PBA(1024, 4, 4, false)
            PBA(2048, NUFFT_F32_PBA2048_RC, 2, true)
            PBA(4096, 1, 1, true)
#undef PBA
        default: return hipErrorInvalidValue;
        }
    }
    prof_end(a.prof, s);
    if (sp > 0) {
        prof_begin(a.prof, DIR > 0 ? "adj_sum" : "type1_sum", s);
        HX_DISPATCH(hipLaunchKernelGGL((k_sum_split_rows<R, HX>), dim3(a.L2, a.fac.K), dim3(256), 0, s,
                                       (const cx_t<R> *)a.Zp, sp, a.fac.K, a.L1, (int64_t)a.L2, a.Y, a.E));
        prof_end(a.prof, s);
    }
    prof_begin(a.prof, DIR > 0 ? "adj_passA" : "type1_passA", s);
    ok = false;
    if constexpr (sizeof(R) == 4) {
        if (a.sched == 1) ok = tuned_pass_a_adj<R, DIR, 1, 8>(a, f, s);
        else if (a.sched == 2) ok = tuned_pass_a_adj<R, DIR, 2, 16>(a, f, s);
    }
    if constexpr (sizeof(R) == 4) {
        if (!ok && WIDE_A_ADJ(a.L1, a.L2)) {   // L2 = 2048: eight columns per workgroup
            const cx_t<R> *tw = DIR < 0 ? a.tw2 : a.tw2i;
            HX_DISPATCH(hipLaunchKernelGGL((k_passA_adj_wide<R, 2048, 8, DIR, HX>), dim3(xcd_grid(a.L1 / 8)),
                                           dim3(4 * 128), 0, s, (const cx_t<R> *)a.Y, a.N, (int64_t)a.L1, a.fac.K,
                                           tw, f, a.E));
            ok = true;
        }
    }
    if (!ok) {
        switch (a.L2) {
#define PAA(LL, GG)                                                                                        \
    case LL: {                                                                                             \
        constexpr int G = GG;                                                                              \
        HX_DISPATCH((launch_pass_a_adj<R, LL, G, DIR, HX, 16>(a, f, s)));                                   \
        break;                                                                                             \
    }
            PAA(64, 8)
            PAA(128, 8)
            PAA(256, 8)
            PAA(512, 8)
            PAA(1024, Cfg<R>::GA1024)
            PAA(2048, Cfg<R>::GA2048)
#undef PAA
#define PAAM(LL, GF, GD)                                                                                   \
    case LL:                                                                                               \
        if (a.half) return hipErrorInvalidValue;                                                           \
        launch_pass_a_adj<R, LL, sizeof(R) == 4 ? GF : GD, DIR, false, 16>(a, f, s);                       \
        break;
            MIXED_L2_SWITCH(PAAM)
#undef PAAM
        default: return hipErrorInvalidValue;
        }
    }
    prof_end(a.prof, s);
    return hipGetLastError();
}

template <typename R>
hipError_t fused_type1(const FusedArgs<R> &a, const cx_t<R> *c, cx_t<R> *f, int sign, hipStream_t s)
{
    return sign < 0 ? fused_type1_dir<R, -1>(a, c, f, s) : fused_type1_dir<R, 1>(a, c, f, s);
}

template hipError_t fused_type2<float>(const FusedArgs<float> &, const float2 *, float2 *, int, const float2 *,
                                       double *, hipStream_t);
template hipError_t fused_type2<double>(const FusedArgs<double> &, const double2 *, double2 *, int,
                                        const double2 *, double *, hipStream_t);
template hipError_t fused_sort_input<float>(const FusedArgs<float> &, const float2 *, const char *, hipStream_t);
template hipError_t fused_sort_input<double>(const FusedArgs<double> &, const double2 *, const char *,
                                             hipStream_t);
template hipError_t fused_type1<float>(const FusedArgs<float> &, const float2 *, float2 *, int, hipStream_t);
template hipError_t fused_type1<double>(const FusedArgs<double> &, const double2 *, double2 *, int,
                                        hipStream_t);

}  // namespace nufft
