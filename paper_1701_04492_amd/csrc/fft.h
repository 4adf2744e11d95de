// Workgroup-level FFT building blocks for gfx950.
//
// A length-L transform (L a power of two, 16 <= L <= 4096) is held in LDS and
// computed by L/16 threads with 16 complex values per thread per stage
// (Stockham auto-sort).  The stage radices are R0, then 16 while at least 16
// points per sub-transform remain, then the remainder: R0 = 16 gives radix-16
// stages and one radix-2/4/8 stage last; R0 = 8 starts with a radix-8 stage
// (two butterflies per thread), e.g. 8 x 16 x 16 instead of 16 x 16 x 8 for
// L = 2048.  The order is a tuning choice (the arithmetic per point is the
// same).  Several transforms share a workgroup; every thread of the workgroup
// runs the same stage sequence, so __syncthreads() separates the read and
// write phases of each stage.
//
// LDS layout: element i of a transform lives at lds_pad(i) = i + i/16 (one
// spare slot per 16 breaks the power-of-two strides of the radix-16 write
// phase), and consecutive transforms are fft_pitch(L) elements apart (odd,
// so that the same element of neighbouring transforms falls in different
// banks).
//
// Direction DIR = -1 computes X_n = sum_k x_k exp(-2 pi i n k / L) (the DFT of
// Sec. 1); DIR = +1 the unnormalised inverse.  Twiddles come from an L-entry
// table computed in FP64 on the host, stage-major: the stage that combines
// NS-point transforms with radix R reads exp(DIR 2 pi i q k / (NS R)) at
// NS - 1 + k (R - 1) + q - 1 (an odd stride between consecutive k, so the
// lanes of a wave hit different LDS banks).
#pragma once

#include "common.h"

__host__ __device__ constexpr int lds_pad(int i) { return i + (i >> 4); }
__host__ __device__ constexpr int fft_pitch(int L) { return L + L / 16 + 1; }

// Pitch for G transforms that are also accessed across transforms (lane order:
// transform index fastest, then element).  With P = 32/G (mod 32) float2
// slots, the G transforms x 32/G consecutive elements touched by 32 lanes
// fall into 32 distinct bank pairs.
__host__ __device__ constexpr int fft_pitch_g(int L, int G)
{
    const int target = G >= 32 ? 1 : 32 / G;
    int p = L + L / 16;
    while (p % 32 != target % 32) ++p;
    return p;
}

namespace fftk {

// Radix of the stage that combines NS-point sub-transforms (first radix R0).
template <int L, int NS, int R0>
__host__ __device__ constexpr int stage_radix()
{
    return NS == 1 ? (R0 < L ? R0 : L) : (L / NS >= 16 ? 16 : L / NS);
}

// Ordering between the read and write phases of a stage.  WS (wave sync): the
// transform's threads all belong to one wavefront and no other wave touches
// its buffer, so LDS ordering inside the wave suffices (no workgroup barrier).
template <bool WS>
__device__ __forceinline__ void stage_sync()
{
    if constexpr (WS) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

template <typename C, int DIR>
__device__ __forceinline__ C mul_w4(C a)   // a * exp(DIR 2 pi i / 4) = a * (DIR i)
{
    return DIR < 0 ? cmake<C>(a.y, -a.x) : cmake<C>(-a.y, a.x);
}

template <typename C, int DIR>
__device__ __forceinline__ void dft2(C &a, C &b)
{
    C t = a;
    a = cadd(t, b);
    b = csub(t, b);
}

template <typename C, int DIR>
__device__ __forceinline__ void dft4(C &a0, C &a1, C &a2, C &a3)
{
    C t0 = cadd(a0, a2), t1 = csub(a0, a2);
    C t2 = cadd(a1, a3), t3 = mul_w4<C, DIR>(csub(a1, a3));
    a0 = cadd(t0, t2);
    a2 = csub(t0, t2);
    a1 = cadd(t1, t3);
    a3 = csub(t1, t3);
}

// exp(DIR 2 pi i m / 16) for the radix-8/16 internal twiddles.
template <typename C, int DIR>
__device__ __forceinline__ C w16(int m)
{
    using R = decltype(C{}.x);
    const R c1 = (R)0.92387953251128675613, s1 = (R)0.38268343236508977173, h = (R)0.70710678118654752440;
    R c, s;
    switch (m) {
    case 0: c = 1; s = 0; break;
    case 1: c = c1; s = s1; break;
    case 2: c = h; s = h; break;
    case 3: c = s1; s = c1; break;
    case 4: c = 0; s = 1; break;
    case 6: c = -h; s = h; break;
    default: c = -c1; s = -s1; break;    // m = 9
    }
    return cmake<C>(c, DIR * s);
}

template <typename C, int DIR>
__device__ __forceinline__ void dft8(C *v)
{
    C e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    C o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4<C, DIR>(e0, e1, e2, e3);
    dft4<C, DIR>(o0, o1, o2, o3);
    o1 = cmul(o1, w16<C, DIR>(2));
    o2 = mul_w4<C, DIR>(o2);
    o3 = cmul(o3, w16<C, DIR>(6));
    v[0] = cadd(e0, o0); v[4] = csub(e0, o0);
    v[1] = cadd(e1, o1); v[5] = csub(e1, o1);
    v[2] = cadd(e2, o2); v[6] = csub(e2, o2);
    v[3] = cadd(e3, o3); v[7] = csub(e3, o3);
}

// 16-point DFT as 4 x 4: inner DFT4 over stride-4 groups, twiddle W16^(l k1), outer DFT4.
template <typename C, int DIR>
__device__ __forceinline__ void dft16(C *v)
{
    C a[4][4];
#pragma unroll
    for (int l = 0; l < 4; ++l) {
        C a0 = v[l], a1 = v[4 + l], a2 = v[8 + l], a3 = v[12 + l];
        dft4<C, DIR>(a0, a1, a2, a3);
        a[l][0] = a0; a[l][1] = a1; a[l][2] = a2; a[l][3] = a3;
    }
#pragma unroll
    for (int l = 1; l < 4; ++l)
#pragma unroll
        for (int k1 = 1; k1 < 4; ++k1) {
            const int m = l * k1;
            if (m == 4) a[l][k1] = mul_w4<C, DIR>(a[l][k1]);
            else a[l][k1] = cmul(a[l][k1], w16<C, DIR>(m));
        }
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        C b0 = a[0][k1], b1 = a[1][k1], b2 = a[2][k1], b3 = a[3][k1];
        dft4<C, DIR>(b0, b1, b2, b3);
        v[k1] = b0; v[k1 + 4] = b1; v[k1 + 8] = b2; v[k1 + 12] = b3;
    }
}

template <int R, typename C, int DIR>
__device__ __forceinline__ void dft(C *v)
{
    if constexpr (R == 2) dft2<C, DIR>(v[0], v[1]);
    else if constexpr (R == 4) dft4<C, DIR>(v[0], v[1], v[2], v[3]);
    else if constexpr (R == 8) dft8<C, DIR>(v);
    else dft16<C, DIR>(v);
}

// One Stockham stage on a transform already in registers: v holds, for each
// of the 16/R butterflies b = lt + i*(L/16) this thread owns, the R inputs
// x[b + q*L/R].  Applies the stage twiddles, the radix-R DFT, and writes the
// outputs to LDS in auto-sorted order.
// `active` false: the thread's transform is not needed (its threads form whole
// waves); it skips the arithmetic and the LDS traffic but still takes part in
// every barrier of the stage sequence.
template <typename C, int L, int DIR, int NS, int R, bool WS>
__device__ __forceinline__ void stage_compute_store(C *buf, const C *tw, int lt, C *v, bool active)
{
    constexpr int BPT = 16 / R;
    if (active) {
#pragma unroll
        for (int i = 0; i < BPT; ++i) {
            const int b = lt + i * (L / 16);
            if constexpr (NS > 1) {
                const int k = b % NS;
#pragma unroll
                for (int q = 1; q < R; ++q)
                    v[i * R + q] = cmul(v[i * R + q], tw[(NS - 1) + k * (R - 1) + (q - 1)]);
            }
            dft<R, C, DIR>(v + i * R);
        }
    }
    stage_sync<WS>();   // every thread has read its inputs of this stage
    if (active) {
#pragma unroll
        for (int i = 0; i < BPT; ++i) {
            const int b = lt + i * (L / 16);
            const int base = (b / NS) * NS * R + (b % NS);
#pragma unroll
            for (int q = 0; q < R; ++q) buf[lds_pad(base + q * NS)] = v[i * R + q];
        }
    }
    stage_sync<WS>();
}

template <typename C, int L, int DIR, int NS, bool WS, int R0 = 16>
__device__ __forceinline__ void stages_from(C *buf, const C *tw, int lt, bool active)
{
    if constexpr (NS < L) {
        constexpr int R = stage_radix<L, NS, R0>();
        constexpr int BPT = 16 / R;
        C v[16];
        if (active) {
#pragma unroll
            for (int i = 0; i < BPT; ++i) {
                const int b = lt + i * (L / 16);
#pragma unroll
                for (int q = 0; q < R; ++q) v[i * R + q] = buf[lds_pad(b + q * (L / R))];
            }
        }
        stage_compute_store<C, L, DIR, NS, R, WS>(buf, tw, lt, v, active);
        stages_from<C, L, DIR, NS * R, WS, R0>(buf, tw, lt, active);
    }
}

}  // namespace fftk

// Transforms of at most 1024 points are held by at most 64 threads, i.e. each
// lies inside one wavefront (transforms start at multiples of L/16 threads,
// which divides 64).  Their stages then need only wave-level ordering, and
// the waves of a workgroup do not wait for each other inside the FFT.  A
// caller that reads transforms of other waves afterwards calls fft_publish<L>()
// (a workgroup barrier when the stages were wave-synchronous).
template <int L>
inline constexpr bool fft_wave_sync = (L <= 1024);
template <int L>
__device__ __forceinline__ void fft_publish()
{
    if constexpr (fft_wave_sync<L>) __syncthreads();
}

// Full transform whose input is already in LDS (natural order, padded).
// Result: natural order in the same buffer.  Called by all threads of the
// workgroup; lt in [0, L/16) is this thread's lane within the transform.
template <typename C, int L, int DIR, bool WS = false, int R0 = 16>
__device__ __forceinline__ void block_fft_lds(C *buf, const C *tw, int lt, bool active = true)
{
    static_assert(L >= 16 && L <= 4096 && (L & (L - 1)) == 0, "unsupported FFT length");
    static_assert(!WS || L <= 1024, "a wave-synchronous transform must fit one wavefront");
    static_assert(R0 == 16 || R0 == 8, "first radix 16 or 8");
    fftk::stages_from<C, L, DIR, 1, WS, R0>(buf, tw, lt, active);
}

// ---- mixed radix: L = P Q points, P = 3 or 5, Q a power of two --------------
// One radix-P decimation-in-frequency stage splits the transform into P
// transforms of Q points on interleaved outputs.  With W_n = exp(DIR 2 pi i / n):
//   X[P k + s] = sum_{m<Q} W_Q^{m k} y_s[m],
//   y_s[m]     = W_L^{s m} sum_{p<P} x[m + p Q] W_P^{s p}.
// The padded natural layout puts x[m + p Q] at lds_pad(m) + p (Q + Q/16), so
// y_s overwrites the inputs of its butterflies in place and sub-transform s
// runs on the padded buffer at s (Q + Q/16); X[n] ends at fft_out_pos<L>(n).
// Twiddle table of a mixed length L (L entries, sign DIR): the stage-major
// table of the Q-point transform in entries [0, Q), then W_L^{s m} at
// Q + (s - 1) Q + m for 1 <= s < P, m < Q.

__host__ __device__ constexpr int fft_radix_p(int L) { return L % 3 == 0 ? 3 : (L % 5 == 0 ? 5 : 1); }

// Padded LDS position of output n of a length-L transform (natural order for
// powers of two; the sub-transform layout above for mixed lengths).
template <int L>
__host__ __device__ constexpr int fft_out_pos(int n)
{
    constexpr int P = fft_radix_p(L), Q = L / P;
    if constexpr (P == 1) return lds_pad(n);
    else return (n % P) * (Q + Q / 16) + lds_pad(n / P);
}

namespace fftk {

// In-place P-point DFT (P = 3 or 5): x[s] <- sum_p x[p] exp(DIR 2 pi i s p / P).
template <typename C, int P, int DIR>
__device__ __forceinline__ void dftp(C *x)
{
    using R = decltype(C{}.x);
    if constexpr (P == 3) {
        const R c1 = (R)-0.5, s1 = (R)0.86602540378443864676;   // cos, sin of 2 pi / 3
        const C t = cadd(x[1], x[2]);
        const C u = cmake<C>(x[0].x + c1 * t.x, x[0].y + c1 * t.y);
        const C d = csub(x[1], x[2]);
        const C v = mul_w4<C, DIR>(cmake<C>(s1 * d.x, s1 * d.y));   // DIR i s1 (x1 - x2)
        x[0] = cadd(x[0], t);
        x[1] = cadd(u, v);
        x[2] = csub(u, v);
    } else {
        static_assert(P == 5, "radix 3 or 5");
        // cos and sin of 2 pi / 5 and 4 pi / 5
        const R c1 = (R)0.30901699437494742410, s1 = (R)0.95105651629515357212;
        const R c2 = (R)-0.80901699437494742410, s2 = (R)0.58778525229247312917;
        const C a1 = cadd(x[1], x[4]), b1 = csub(x[1], x[4]);
        const C a2 = cadd(x[2], x[3]), b2 = csub(x[2], x[3]);
        const C u1 = cmake<C>(x[0].x + c1 * a1.x + c2 * a2.x, x[0].y + c1 * a1.y + c2 * a2.y);
        const C u2 = cmake<C>(x[0].x + c2 * a1.x + c1 * a2.x, x[0].y + c2 * a1.y + c1 * a2.y);
        const C v1 = mul_w4<C, DIR>(cmake<C>(s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y));
        const C v2 = mul_w4<C, DIR>(cmake<C>(s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y));
        x[0] = cadd(x[0], cadd(a1, a2));
        x[1] = cadd(u1, v1);
        x[4] = csub(u1, v1);
        x[2] = cadd(u2, v2);
        x[3] = csub(u2, v2);
    }
}

}  // namespace fftk

// Full transform of any supported length L (a power of two up to 4096, or P Q
// with P = 3, 5 and Q a power of two, 64 <= Q <= 1024) whose input is in LDS
// (natural padded order), by the L/16 threads of the transform (lane lt).
// Called by all threads of the workgroup; the caller has made the input
// visible (a barrier).  Ends with the results readable by every thread of
// the workgroup at fft_out_pos<L>(n).
template <typename C, int L, int DIR, int R0 = 16>
__device__ __forceinline__ void block_fft_any_lds(C *buf, const C *tw, int lt)
{
    constexpr int P = fft_radix_p(L);
    if constexpr (P == 1) {
        block_fft_lds<C, L, DIR, fft_wave_sync<L>, R0>(buf, tw, lt);
        fft_publish<L>();
    } else {
        constexpr int Q = L / P, QP = Q + Q / 16, TPF = L / 16;
        static_assert(Q * P == L && (Q & (Q - 1)) == 0 && Q >= 64 && Q <= 1024, "unsupported mixed length");
        const C *twp = tw + Q;
        for (int m = lt; m < Q; m += TPF) {   // the Q radix-P butterflies
            C x[P];
#pragma unroll
            for (int p = 0; p < P; ++p) x[p] = buf[lds_pad(m) + p * QP];
            fftk::dftp<C, P, DIR>(x);
            buf[lds_pad(m)] = x[0];
#pragma unroll
            for (int q = 1; q < P; ++q) buf[lds_pad(m) + q * QP] = cmul(x[q], twp[(q - 1) * Q + m]);
        }
        __syncthreads();
        // sub-transform s: threads s Q/16 .. (s + 1) Q/16 - 1 of the transform (one wavefront)
        block_fft_lds<C, Q, DIR, fft_wave_sync<Q>, R0>(buf + (lt / (Q / 16)) * QP, tw, lt % (Q / 16));
        __syncthreads();
    }
}

// Full transform whose input is in registers: v[q] = x[lt + q*L/16], q < 16
// (exactly the operands of the first radix-16 stage, so that stage skips the
// LDS round trip).  The caller must have finished every earlier read of buf
// (a __syncthreads() since the last use).  Result: natural order in buf.
// `active` false (uniform over whole waves): the transform is skipped, the
// barriers are still taken, and its part of buf is left as it was.
template <typename C, int L, int DIR, bool WS = false, int R0 = 16>
__device__ __forceinline__ void block_fft_regs(C *buf, const C *tw, int lt, C *v, bool active = true)
{
    static_assert(L >= 16 && L <= 4096 && (L & (L - 1)) == 0, "unsupported FFT length");
    static_assert(!WS || L <= 1024, "a wave-synchronous transform must fit one wavefront");
    static_assert(R0 == 16 || R0 == 8, "first radix 16 or 8");
    if constexpr (R0 == 16) {
        // first stage: NS = 1, R = 16, one butterfly per thread, no twiddles
        if (active) {
            fftk::dft<16, C, DIR>(v);
            const int base = lt * 16;
#pragma unroll
            for (int q = 0; q < 16; ++q) buf[lds_pad(base + q)] = v[q];
        }
        fftk::stage_sync<WS>();
        fftk::stages_from<C, L, DIR, 16, WS>(buf, tw, lt, active);
    } else {
        // first stage: NS = 1, R = 8, two butterflies per thread: butterfly i
        // (b = lt + i L/16) takes x[b + q L/8] = v[i + 2q]
        C w[16];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int q = 0; q < 8; ++q) w[i * 8 + q] = v[i + 2 * q];
        fftk::stage_compute_store<C, L, DIR, 1, 8, WS>(buf, tw, lt, w, active);
        fftk::stages_from<C, L, DIR, 8, WS, 8>(buf, tw, lt, active);
    }
}
