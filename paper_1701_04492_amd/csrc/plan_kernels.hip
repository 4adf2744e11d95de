// Planning-stage kernels (Sec. 2.2 and Sec. 2.3, "Planning the transform"):
// nearest-grid assignment, gamma, and a stable sort of the samples by the
// FFT output tile they read from.
#include "kernels.h"

namespace nufft {

__device__ __forceinline__ double wave_max(double v)
{
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// s_j = round(L x_j) (ties to even, on the rounded product), t_j = s_j mod L
// (Euclidean), d_j = L x_j - s_j through one fma, X_j = d_j N / L (Sec. 2.2,
// eq. (s_vec), (t_vec); oversampled grid of Sec. 2.3).  Also: the sort key
// of the sample (its FFT output tile, then its position in the tile), a
// histogram of keys, max |X_j| (as the bit pattern of a non-negative double),
// and a flag for non-finite samples.
template <typename R>
__global__ void __launch_bounds__(256)
k_assign(const double *__restrict__ x, int64_t M, int64_t L, double n_over_L, int L1,
         int L2, int32_t *__restrict__ t_out, R *__restrict__ X_out,
         uint32_t *__restrict__ key_out, int32_t *__restrict__ hist,
         unsigned long long *gamma_bits, int *bad)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double amax = 0.0;
    if (j < M) {
        const double xj = x[j];
        int t = 0;
        double X = 0.0;
        if (!isfinite(xj)) {
            atomicOr(bad, 1);
        } else {
            const double Ld = (double)L;
            const double s = rint(Ld * xj);
            const double d = fma(Ld, xj, -s);
            double tt = fmod(s, Ld);
            if (tt < 0.0) tt += Ld;
            t = (int)tt;
            X = d * n_over_L;
            amax = fabs(X);
        }
        const uint32_t key = ((uint32_t)t % (uint32_t)L2) * (uint32_t)L1 + (uint32_t)t / (uint32_t)L2;
        t_out[j] = t;
        X_out[j] = (R)X;
        key_out[j] = key;
        atomicAdd(&hist[key], 1);
    }
    __shared__ double red[4];
    amax = wave_max(amax);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = amax;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
        atomicMax(gamma_bits, (unsigned long long)__double_as_longlong(m));
    }
}

// ---- exclusive scan of int32 (three kernels) ------------------------------

#define SCAN_BLOCK 1024   // elements per workgroup (256 threads x 4)

__device__ __forceinline__ int wave_incl_scan(int v)
{
    const int lane = threadIdx.x & 63;
    for (int off = 1; off < 64; off <<= 1) {
        int u = __shfl_up(v, off, 64);
        if (lane >= off) v += u;
    }
    return v;
}

// Exclusive scan of 256 per-thread values within the workgroup; returns the
// thread's exclusive prefix and stores the block total in *total.
__device__ __forceinline__ int block_excl_scan(int v, int *total)
{
    __shared__ int wsum[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int incl = wave_incl_scan(v);
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    int base = 0;
    for (int w = 0; w < wave; ++w) base += wsum[w];
    *total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();
    return base + incl - v;
}

__global__ void __launch_bounds__(256)
k_scan_local(const int32_t *__restrict__ in, int64_t n, int32_t *__restrict__ out,
             int32_t *__restrict__ block_sums)
{
    const int64_t base = (int64_t)blockIdx.x * SCAN_BLOCK + threadIdx.x * 4;
    int v[4], s = 0;
    for (int i = 0; i < 4; ++i) {
        v[i] = (base + i < n) ? in[base + i] : 0;
        s += v[i];
    }
    int total;
    int run = block_excl_scan(s, &total);
    for (int i = 0; i < 4; ++i) {
        if (base + i < n) out[base + i] = run;
        run += v[i];
    }
    if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

// One workgroup scans the block sums in chunks of 1024 (exclusive, in place).
__global__ void __launch_bounds__(256)
k_scan_sums(int32_t *__restrict__ sums, int64_t nb)
{
    __shared__ int carry_s;
    if (threadIdx.x == 0) carry_s = 0;
    __syncthreads();
    for (int64_t c0 = 0; c0 < nb; c0 += SCAN_BLOCK) {
        const int64_t base = c0 + threadIdx.x * 4;
        int v[4], s = 0;
        for (int i = 0; i < 4; ++i) {
            v[i] = (base + i < nb) ? sums[base + i] : 0;
            s += v[i];
        }
        int total;
        int run = block_excl_scan(s, &total) + carry_s;
        for (int i = 0; i < 4; ++i) {
            if (base + i < nb) sums[base + i] = run;
            run += v[i];
        }
        __syncthreads();
        if (threadIdx.x == 0) carry_s += total;
        __syncthreads();
    }
}

__global__ void __launch_bounds__(256)
k_scan_add(int32_t *__restrict__ out, int64_t n, const int32_t *__restrict__ block_sums)
{
    const int64_t base = (int64_t)blockIdx.x * SCAN_BLOCK + threadIdx.x * 4;
    const int add = block_sums[blockIdx.x];
    for (int i = 0; i < 4; ++i)
        if (base + i < n) out[base + i] += add;
}

hipError_t exclusive_scan(const int32_t *in, int32_t *out, int64_t n, int32_t *tmp, hipStream_t s)
{
    const int64_t nb = (n + SCAN_BLOCK - 1) / SCAN_BLOCK;
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scan_local, dim3((unsigned)nb), dim3(256), 0, s, in, n, out, tmp);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(256), 0, s, tmp, nb);
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(256), 0, s, out, n, (const int32_t *)tmp);
    return hipGetLastError();
}

int64_t scan_tmp_elems(int64_t n) { return (n + SCAN_BLOCK - 1) / SCAN_BLOCK + 1; }

// ---- stable LSD radix sort of (key, value) pairs, 8-bit digits -----------

#define RS_BLOCK 1024   // elements per workgroup (256 threads x 4 rounds)

__global__ void __launch_bounds__(256)
k_digit_hist(const uint32_t *__restrict__ keys, int64_t n, int shift, int32_t *__restrict__ hist,
             int64_t nblocks)
{
    __shared__ int cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_BLOCK;
    for (int i = threadIdx.x; i < RS_BLOCK; i += 256) {
        const int64_t g = base + i;
        if (g < n) atomicAdd(&cnt[(keys[g] >> shift) & 255u], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

// Scatter of one digit pass.  Elements keep their input order within a digit:
// within a wave the rank among equal digits comes from ballots, across the
// four waves and the four rounds from a running per-digit cursor updated in
// wave order.
__global__ void __launch_bounds__(256)
k_digit_scatter(const uint32_t *__restrict__ kin, const int32_t *__restrict__ vin, int64_t n,
                int shift, const int32_t *__restrict__ offs, int64_t nblocks,
                uint32_t *__restrict__ kout, int32_t *__restrict__ vout)
{
    __shared__ int cursor[256];
    cursor[threadIdx.x] = offs[(int64_t)threadIdx.x * nblocks + blockIdx.x];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const unsigned long long lt_mask = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    for (int round = 0; round < 4; ++round) {
        const int64_t g = (int64_t)blockIdx.x * RS_BLOCK + round * 256 + threadIdx.x;
        const bool valid = g < n;
        uint32_t key = 0;
        int32_t val = 0;
        int d = 0;
        if (valid) {
            key = kin[g];
            val = vin[g];
            d = (key >> shift) & 255u;
        }
        unsigned long long same = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1;
            const unsigned long long bb = __ballot(bit);
            same &= bit ? bb : ~bb;
        }
        const int rank = __popcll(same & lt_mask);
        const int cnt = __popcll(same);
        const bool leader = valid && rank == 0;
        for (int w = 0; w < 4; ++w) {
            int pos = 0;
            if (wave == w && valid) pos = cursor[d] + rank;
            __syncthreads();
            if (wave == w && leader) cursor[d] += cnt;
            __syncthreads();
            if (wave == w && valid) {
                kout[pos] = key;
                vout[pos] = val;
            }
        }
    }
}

__global__ void k_iota(int32_t *v, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = (int32_t)i;
}

// out[i] = in[i * stride], i < n (every stride-th entry, e.g. the first offset of each column).
__global__ void k_strided_i32(const int32_t *__restrict__ in, int64_t stride, int64_t n, int32_t *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = in[i * stride];
}

// sinv[perm[i]] = i: the sorted position of every sample.
__global__ void k_invert_perm(const int32_t *__restrict__ perm, int64_t n, int32_t *__restrict__ sinv)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) sinv[perm[i]] = (int32_t)i;
}

// Destination buckets of the sample permutation (blocks of 2^shift sample
// indices): key[i] = perm[i] >> shift for every sorted position i.
__global__ void k_bucket_keys(const int32_t *__restrict__ perm, int64_t n, int shift, uint32_t *__restrict__ key)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) key[i] = (uint32_t)perm[i] >> shift;
}

// order[p]: the sorted position at bucketed position p (stable by bucket);
// bdst[i] = p, lidx[p] = perm[i] mod 2^shift.
__global__ void k_bucket_maps(const int32_t *__restrict__ order, const int32_t *__restrict__ perm, int64_t n,
                              int shift, int32_t *__restrict__ bdst, uint16_t *__restrict__ lidx)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) {
        const int32_t i = order[p];
        bdst[i] = (int32_t)p;
        lidx[p] = (uint16_t)(perm[i] & ((1 << shift) - 1));
    }
}

hipError_t launch_bucket_maps(const int32_t *perm, int64_t n, int shift, uint32_t *keys, int32_t *vals,
                              uint32_t *keys_alt, int32_t *vals_alt, int32_t *tmp, int32_t *bdst, uint16_t *lidx,
                              hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const unsigned nb = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_bucket_keys, dim3(nb), dim3(256), 0, s, perm, n, shift, keys);
    hipLaunchKernelGGL(k_iota, dim3(nb), dim3(256), 0, s, vals, n);
    int bits = 0;
    while ((int64_t(1) << bits) < ((n + (int64_t(1) << shift) - 1) >> shift)) ++bits;
    uint32_t *ks = keys;
    int32_t *order = vals;
    if (bits > 0) {
        const hipError_t e = radix_sort_pairs(keys, vals, keys_alt, vals_alt, n, bits, tmp, s, &ks, &order);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_bucket_maps, dim3(nb), dim3(256), 0, s, (const int32_t *)order, perm, n, shift, bdst, lidx);
    return hipGetLastError();
}

int64_t radix_tmp_elems(int64_t n)
{
    const int64_t nb = (n + RS_BLOCK - 1) / RS_BLOCK;
    return 256 * nb + scan_tmp_elems(256 * nb);
}

hipError_t radix_sort_pairs(uint32_t *keys, int32_t *vals, uint32_t *keys_alt, int32_t *vals_alt,
                            int64_t n, int key_bits, int32_t *tmp, hipStream_t s,
                            uint32_t **keys_sorted, int32_t **vals_sorted)
{
    const int64_t nb = (n + RS_BLOCK - 1) / RS_BLOCK;
    int32_t *hist = tmp;
    int32_t *scan_tmp = tmp + 256 * nb;
    uint32_t *ki = keys, *ko = keys_alt;
    int32_t *vi = vals, *vo = vals_alt;
    for (int shift = 0; shift < key_bits; shift += 8) {
        hipLaunchKernelGGL(k_digit_hist, dim3((unsigned)nb), dim3(256), 0, s, ki, n, shift, hist, nb);
        hipError_t e = exclusive_scan(hist, hist, 256 * nb, scan_tmp, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_digit_scatter, dim3((unsigned)nb), dim3(256), 0, s, ki, vi, n, shift,
                           (const int32_t *)hist, nb, ko, vo);
        uint32_t *kt = ki; ki = ko; ko = kt;
        int32_t *vt = vi; vi = vo; vo = vt;
    }
    *keys_sorted = ki;
    *vals_sorted = vi;
    return hipGetLastError();
}

template <typename R>
__global__ void k_gather_sorted(const int32_t *__restrict__ perm, const R *__restrict__ X, int64_t n,
                                R *__restrict__ Xs)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) Xs[i] = X[perm[i]];
}

template <typename R>
hipError_t launch_assign(const double *x, int64_t M, int64_t L, double n_over_L, int L1, int L2,
                         int32_t *t, R *X, uint32_t *key, int32_t *hist, unsigned long long *gbits,
                         int *bad, hipStream_t s)
{
    if (M == 0) return hipSuccess;
    const unsigned nb = (unsigned)((M + 255) / 256);
    hipLaunchKernelGGL(k_assign<R>, dim3(nb), dim3(256), 0, s, x, M, L, n_over_L, L1, L2, t, X,
                       key, hist, gbits, bad);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_gather_sorted(const int32_t *perm, const R *X, int64_t n, R *Xs, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_sorted<R>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, perm, X,
                       n, Xs);
    return hipGetLastError();
}

hipError_t launch_iota(int32_t *v, int64_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_iota, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, v, n);
    return hipGetLastError();
}

hipError_t launch_strided_i32(const int32_t *in, int64_t stride, int64_t n, int32_t *out, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_strided_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in, stride, n, out);
    return hipGetLastError();
}

hipError_t launch_invert_perm(const int32_t *perm, int64_t n, int32_t *sinv, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_invert_perm, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, perm, n, sinv);
    return hipGetLastError();
}

template hipError_t launch_assign<float>(const double *, int64_t, int64_t, double, int, int, int32_t *,
                                         float *, uint32_t *, int32_t *, unsigned long long *, int *,
                                         hipStream_t);
template hipError_t launch_assign<double>(const double *, int64_t, int64_t, double, int, int, int32_t *,
                                          double *, uint32_t *, int32_t *, unsigned long long *, int *,
                                          hipStream_t);
template hipError_t launch_gather_sorted<float>(const int32_t *, const float *, int64_t, float *,
                                                hipStream_t);
template hipError_t launch_gather_sorted<double>(const int32_t *, const double *, int64_t, double *,
                                                 hipStream_t);

}  // namespace nufft
