// Device helpers shared by the fused kernels (1-D, 2-D, batched).
#pragma once

#include <hip/hip_fp16.h>

#include <type_traits>

#include "fft.h"
#include "kernels.h"

namespace nufft {

// ---- half-precision exchange (FP32 plans with NUFFT_FLAG_HALF_EXCHANGE) ----
// The K x L intermediate of the two-pass split is stored as two fp16 per
// complex value (4 bytes instead of 8) with one power-of-two scale 2^s per
// block of values that one pass writes together: a column of pass A, a row of
// pass B'.  s maps the block's largest |re|, |im| into [2^14, 2^15), below the
// fp16 maximum 65504; every value above 2^-28 of the block maximum keeps the
// relative rounding 2^-11 of fp16, smaller ones an absolute error below 2^-39
// of the maximum.  The scaling itself is exact (ldexp).
__device__ __forceinline__ int hx_exponent(float m)
{
    if (!(m > 0.0f) || !(m <= 3.4e38f)) return 0;   // all-zero block, or inf / NaN: stored unscaled
    const int s = 14 - ilogbf(m);
    return s > 127 ? 127 : s;                        // fits int8 (s >= -113)
}
__device__ __forceinline__ __half2 hx_pack(float2 v, int s)
{
    return __floats2half2_rn(ldexpf(v.x, s), ldexpf(v.y, s));
}
__device__ __forceinline__ float2 hx_unpack(__half2 h, int s)
{
    const float2 f = __half22float2(h);
    return make_float2(ldexpf(f.x, -s), ldexpf(f.y, -s));
}
__device__ __forceinline__ float cmaxabs(float2 v) { return fmaxf(fabsf(v.x), fabsf(v.y)); }
// max over the lanes of a wave whose lane index agrees modulo S (S a power of two)
__device__ __forceinline__ float wave_max_mod(float m, int S)
{
    for (int o = S; o < 64; o <<= 1) m = fmaxf(m, __shfl_xor(m, o));
    return m;
}
// max over each aligned group of S consecutive lanes (S a power of two)
__device__ __forceinline__ float wave_max_group(float m, int S)
{
    for (int o = 1; o < S && o < 64; o <<= 1) m = fmaxf(m, __shfl_xor(m, o));
    return m;
}

// Copies the length-L FFT twiddle table (conjugated for DIR = +1) into LDS
// with the workgroup's NT threads.  Every load is issued before the first
// store (clamped addresses, no branch around a load), so the copy costs one
// memory latency instead of one per iteration.
template <typename C, int L, int DIR, int NT>
__device__ __forceinline__ void load_tw_s(C *tw_s, const C *__restrict__ tw_g)
{
    constexpr int E = (L + NT - 1) / NT;
    C w[E];
#pragma unroll
    for (int e = 0; e < E; ++e) w[e] = tw_g[min((int)threadIdx.x + e * NT, L - 1)];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int m = threadIdx.x + e * NT;
        if (m < L) tw_s[m] = DIR < 0 ? w[e] : cconj(w[e]);
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

// Unhalved Chebyshev pairs (T_r(z_e), T_{r+1}(z_e)) for E values by the
// three-term recurrence.  One loop advances all E chains per step, so their
// dependent steps interleave (E separate calls of cheb_v would run E serial
// loops of r - 1 dependent steps each).
template <typename R, int E>
__device__ __forceinline__ void cheb_pair_many(int r, const R (&z)[E], R (&t0)[E], R (&t1)[E])
{
#pragma unroll
    for (int e = 0; e < E; ++e) {
        t0[e] = 1;
        t1[e] = z[e];
    }
    for (int q = 0; q < r; ++q) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const R c = 2 * z[e] * t1[e] - t0[e];
            t0[e] = t1[e];
            t1[e] = c;
        }
    }
}

// v_r(z_e) = T_r(z_e) (halved for r = 0) for E values at once.
template <typename R, int E>
__device__ __forceinline__ void cheb_v_many(int r, const R (&z)[E], R (&out)[E])
{
    R t1[E];
    cheb_pair_many<R, E>(r, z, out, t1);
    if (r == 0) {
#pragma unroll
        for (int e = 0; e < E; ++e) out[e] = (R)0.5;
    }
}

// c_k, or -2 pi i k c_k for the derivative pass; zero for k >= N.  The load
// itself is unconditional (from a clamped index), so that a run of such
// loads is issued back to back and waited for once.
template <typename R>
__device__ __forceinline__ cx_t<R> load_coef(const cx_t<R> *__restrict__ c, int64_t k, int64_t N, int mode)
{
    using C = cx_t<R>;
    const bool in = k < N;
    C ck = c[in ? k : N - 1];
    if (mode == 1) {
        const R w = (R)(-2.0 * M_PI * (double)k);
        ck = cmake<C>(-w * ck.y, w * ck.x);
    }
    return in ? ck : cmake<C>(0, 0);
}

// Chebyshev coordinate 2k/N - 1 of mode k: zmap(N) holds 2/N (one FP64
// division per thread), zcoord is one FP64 fma rounded once to R.  Mode
// indices are below 2^31 (N <= 2^23).
struct ZMap {
    double s;
};
__device__ __forceinline__ ZMap zmap(int64_t N) { return ZMap{2.0 / (double)N}; }
template <typename R>
__device__ __forceinline__ R zcoord(int64_t k, ZMap z)
{
    return (R)__builtin_fma((double)(int32_t)k, z.s, -1.0);
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

// The same mapping for a grid of fewer blocks than tasks (a multiple of 8,
// W = gridDim.x / 8 per XCD): block b takes the tasks first, first + step, ...
// below end of its XCD's share, first = (b & 7) * ceil(T / 8) + (b >> 3),
// step = W.  With the grid xcd_grid(T) every block takes the task xcd_task gives.
__device__ __forceinline__ void xcd_tasks(int T, int *first, int *end, int *step)
{
    const int per = (T + 7) >> 3;
    const int b = blockIdx.x;
    const int base = (b & 7) * per;
    *first = base + (b >> 3);
    *end = min(T, base + per);
    *step = (int)(gridDim.x >> 3);
}


// ---- destination-bucketed permutation writes ---------------------------------
// Scattering values to random positions costs one DRAM transaction per value;
// grouping them so that the lanes of one store instruction write neighbouring
// places makes the stores coalesce.  The plan orders the places of a large
// permutation by destination bucket (blocks of 2^shift samples): the values of
// one workgroup that fall into the same bucket have consecutive places.

// Exclusive prefix sum of cnt[0..n) in LDS, in place, by the NT threads of the
// workgroup (n <= 2 NT); returns the total.  Ends with a barrier.
template <int NT>
__device__ __forceinline__ int block_exclusive_scan(int *cnt, int n, int *wsum)
{
    const int tid = threadIdx.x;
    const int a = 2 * tid < n ? cnt[2 * tid] : 0, b = 2 * tid + 1 < n ? cnt[2 * tid + 1] : 0;
    int v = a + b;
    const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(v, o);
        if (lane >= o) v += u;
    }
    if (lane == 63) wsum[wave] = v;
    __syncthreads();
    if (tid == 0) {
        int run = 0;
        for (int w = 0; w < NT / 64; ++w) {
            const int t = wsum[w];
            wsum[w] = run;
            run += t;
        }
        wsum[NT / 64] = run;
    }
    __syncthreads();
    const int excl = v - (a + b) + wsum[wave];
    if (2 * tid < n) cnt[2 * tid] = excl;
    if (2 * tid + 1 < n) cnt[2 * tid + 1] = excl + a;
    __syncthreads();
    return wsum[NT / 64];
}

// The S values per thread of a workgroup (slot s of thread t valid when
// valid[s]) written to out[dst[s]], dst being places of the bucketed layout:
// the values are ordered by bucket (dst >> shift) in LDS, then thread t writes
// the t-th, so that the values of one bucket, which have consecutive places,
// go out in coalesced runs.  nbk <= 2 NT buckets.  LDS scratch (may alias
// other buffers no longer read): hist (nbk + 1 ints), wsum (NT/64 + 1 ints),
// vals (NT*S values), dsts (NT*S ints).  Begins and ends with a barrier.
template <typename T, int NT, int S>
__device__ __forceinline__ void bucketed_store(const T (&val)[S], const int (&dst)[S], const bool (&valid)[S],
                                               int shift, int nbk, T *__restrict__ out, int *hist, int *wsum,
                                               T *vals, int *dsts)
{
    const int tid = threadIdx.x;
    __syncthreads();   // the caller's readers of the scratch are done
    for (int b = tid; b < nbk; b += NT) hist[b] = 0;
    __syncthreads();
    int rank[S];
#pragma unroll
    for (int s = 0; s < S; ++s) rank[s] = valid[s] ? atomicAdd(&hist[dst[s] >> shift], 1) : 0;
    __syncthreads();
    const int n = block_exclusive_scan<NT>(hist, nbk, wsum);
#pragma unroll
    for (int s = 0; s < S; ++s) {
        if (valid[s]) {
            const int slot = hist[dst[s] >> shift] + rank[s];
            vals[slot] = val[s];
            dsts[slot] = dst[s];
        }
    }
    __syncthreads();
    for (int t = tid; t < n; t += NT) out[dsts[t]] = vals[t];
    __syncthreads();
}

// Deterministic segmented sum of per-sample contributions into RC grids in LDS.
// The cnt samples of a tile are sorted by grid point; thread t takes a
// balanced slice of them (empty slices, when cnt < NT, only at the end), sums
// contrib(i, gg) over runs of equal grid point and stores every run that
// starts and ends inside its slice straight into grid gg.  A run that crosses
// slice boundaries leaves one partial per thread in head/tail slots; the
// thread in whose slice the run starts adds the partials of the following
// slices.  With few crossing runs it walks them in thread order; when many
// slices are wholly inside one run (a heavily populated grid point) the sums
// over the following slices come from a segmented suffix sum by pointer
// jumping (log2 NT barrier steps) instead of a walk over hundreds of slices.
// Either way the order of the additions is fixed: the result does not depend
// on timing.
// load(i) returns sample i (a struct whose member n is its grid point); the
// loads of four samples are issued together.  contrib(sample, gg) is its term
// for grid gg; pos(i) is sample i's grid point alone.
// Grids must be zero on entry where no sample falls; the caller synchronises
// before reading them.  Scratch: hv, tv (RC*NT values), hix, tix, nxa, nxb (NT ints).
template <typename C, int RC, int NT, typename PosF, typename LoadF, typename ContribF>
__device__ __forceinline__ void seg_spread(int cnt, int nr, PosF pos, LoadF load, ContribF contrib, C *grid,
                                           int pitch, C *hv, C *tv, int *hix, int *tix, int *nxa, int *nxb)
{
    const int tid = threadIdx.x;
    const int per = cnt / NT, rem = cnt % NT;
    const int i0 = tid * per + min(tid, rem), i1 = i0 + per + (tid < rem ? 1 : 0);
    C a[RC];
#pragma unroll
    for (int gg = 0; gg < RC; ++gg) a[gg] = cmake<C>(0, 0);
    int ncur = -1, nfirst = -1;
    using Sample = decltype(load(0));
    for (int i = i0; i < i1; i += 4) {
        Sample sm[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) sm[u] = load(min(i + u, i1 - 1));
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (i + u < i1) {
                const int n = sm[u].n;
                if (n != ncur) {
                    if (ncur >= 0) {
                        if (ncur == nfirst) {
#pragma unroll
                            for (int gg = 0; gg < RC; ++gg) hv[gg * NT + tid] = a[gg];
                        } else {
#pragma unroll
                            for (int gg = 0; gg < RC; ++gg)
                                if (gg < nr) grid[gg * pitch + lds_pad(ncur)] = a[gg];
                        }
                    } else {
                        nfirst = n;
                    }
#pragma unroll
                    for (int gg = 0; gg < RC; ++gg) a[gg] = cmake<C>(0, 0);
                    ncur = n;
                }
#pragma unroll
                for (int gg = 0; gg < RC; ++gg)
                    if (gg < nr) a[gg] = cadd(a[gg], contrib(sm[u], gg));
            }
        }
    }
    // the last run of the slice (possibly also its first); a keeps its sum
    if (ncur >= 0) {
        if (ncur == nfirst) {
#pragma unroll
            for (int gg = 0; gg < RC; ++gg) hv[gg * NT + tid] = a[gg];
        }
#pragma unroll
        for (int gg = 0; gg < RC; ++gg) tv[gg * NT + tid] = a[gg];
    }
    hix[tid] = nfirst;   // -1 for an empty slice
    tix[tid] = ncur;
    __syncthreads();
    // link: this slice lies wholly inside one run that continues into the next slice
    const bool link = nfirst >= 0 && nfirst == ncur && tid + 1 < NT && hix[tid + 1] == ncur;
    const bool jump = __syncthreads_count(link) >= 16;
    bool head_starts_here = false, last_starts_here = false;
    if (nfirst >= 0) {
        head_starts_here = (i0 == 0) || pos(i0 - 1) != nfirst;
        // the first run: complete here unless it is also the last run (then handled below)
        if (head_starts_here && nfirst != ncur) {
#pragma unroll
            for (int gg = 0; gg < RC; ++gg)
                if (gg < nr) grid[gg * pitch + lds_pad(nfirst)] = hv[gg * NT + tid];
        }
        last_starts_here = (nfirst != ncur) || head_starts_here;
    }
    const bool cont = nfirst >= 0 && tid + 1 < NT && hix[tid + 1] == ncur;   // the last run goes on
    if (jump) {
        // S_u = H_u + (link_u ? S_{u+1} : 0) by pointer jumping; tv becomes the
        // second buffer (this thread's tail sum stays in a)
        C *X = hv, *Y = tv;
        int *nx = nxa, *ny = nxb;
        nx[tid] = link ? tid + 1 : -1;
        __syncthreads();
        for (int d = 1; d < NT; d <<= 1) {
            const int n = nx[tid];
            C v[RC];
#pragma unroll
            for (int gg = 0; gg < RC; ++gg) v[gg] = X[gg * NT + tid];
            if (n >= 0) {
#pragma unroll
                for (int gg = 0; gg < RC; ++gg) v[gg] = cadd(v[gg], X[gg * NT + n]);
            }
#pragma unroll
            for (int gg = 0; gg < RC; ++gg) Y[gg * NT + tid] = v[gg];
            ny[tid] = n >= 0 ? nx[n] : -1;
            __syncthreads();
            C *t = X;
            X = Y;
            Y = t;
            int *tn = nx;
            nx = ny;
            ny = tn;
        }
        if (last_starts_here) {
#pragma unroll
            for (int gg = 0; gg < RC; ++gg) {
                const C sum = cont ? cadd(a[gg], X[gg * NT + tid + 1]) : a[gg];
                if (gg < nr) grid[gg * pitch + lds_pad(ncur)] = sum;
            }
        }
    } else if (last_starts_here) {
        C sum[RC];
#pragma unroll
        for (int gg = 0; gg < RC; ++gg) sum[gg] = a[gg];
        for (int u = tid + 1; u < NT; ++u) {
            if (hix[u] != ncur) break;                   // (empty slices only follow the last sample)
#pragma unroll
            for (int gg = 0; gg < RC; ++gg) sum[gg] = cadd(sum[gg], hv[gg * NT + u]);
            if (tix[u] != ncur) break;                   // the run ends inside slice u
        }
#pragma unroll
        for (int gg = 0; gg < RC; ++gg)
            if (gg < nr) grid[gg * pitch + lds_pad(ncur)] = sum[gg];
    }
}
}  // namespace nufft
