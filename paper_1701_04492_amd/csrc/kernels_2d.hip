// 2-D type II and its adjoint (Sec. 4).
//
//   f_j = sum_{k1<N1, k2<N2} C[k1][k2] exp(-2 pi i (k1 x_j + k2 y_j))
//       ~ sum_{r1<Kx, r2<Ky} u^x_r1(j) u^y_r2(j) G_{r1 r2}[tx_j][ty_j],
//   G_{r1 r2} = F_{Gx} (v^x_r1 o C o v^y_r2) F_{Gy}^T  (eq. (NUFFTII_2D)),
// x pairing with k1 on a grid of Gx points and y with k2 on Gy points.  The
// transform along k2 does not depend on r1 and is done once per r2 (the
// saving noted at the end of Sec. 4):
//   pass A (per group of G rows k1, chunk of ranks r2):
//     H_r2[n2][k1] = sum_k2 C[k1][k2] v^y_r2(k2) exp(-2 pi i k2 n2 / Gy)
//   pass B (per column n2 and sample range): for every r2, r1:
//     X = F_{Gx}(v^x_r1 o H_r2[n2][:]) and f_j += u^x_r1 u^y_r2 X[tx_j] for
//     the samples with ty_j = n2 (sorted there by the plan).
// The adjoint runs the two passes in reverse with the conjugate factors; the
// 2-D type I (Sec. 3.1 applied per axis, the transpose of the type II) runs
// the same two passes with the factors unconjugated and forward-sign FFTs.
// Both are instantiated from one template on the sign DIR of the exponent.
#include "fused_common.h"
#include "kernels_2d.h"

namespace nufft {

// ---- pass A: rows of C, FFT along k2, transposed store ---------------------
template <typename R, int GY, int G>
__global__ void __launch_bounds__(G * GY / 16)
k_2d_passA(const cx_t<R> *__restrict__ Cin, int64_t N1, int64_t N2, int64_t GX, Factors<R> fy, int RCA,
           const cx_t<R> *__restrict__ tw_g, cx_t<R> *__restrict__ H, int64_t rstride)
{
    // stacked problems: blockIdx.y is the problem; H_r2 rows are rstride apart
    Cin += (int64_t)blockIdx.y * N1 * N2;
    H += (int64_t)blockIdx.y * GY * GX;
    using C = cx_t<R>;
    constexpr int TPF = GY / 16;
    constexpr int NT = G * TPF;
    constexpr int P = fft_pitch_g(GY, G);
    __shared__ C buf[G * P];
    __shared__ C tw[GY];
    const int K = fy.K;
    const int nrc = (K + RCA - 1) / RCA;
    const int ncg = (int)((N1 + G - 1) / G);
    const int task = xcd_task(ncg * nrc);
    if (task < 0) return;
    const int cg = task / nrc, rc = task % nrc;
    const int r_lo = rc * RCA, r_hi = min(K, r_lo + RCA);
    load_tw_s<C, GY, -1, NT>(tw, tw_g);
    const int tid = threadIdx.x;
    const int g = tid / TPF, lt = tid % TPF;
    const int64_t k1_0 = (int64_t)cg * G;
    const int64_t k1 = k1_0 + g;
    const ZMap zm = zmap(N2);
    C cv[16];
    R zk[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {   // clamped address, no branch: the 16 loads issue together
        const int64_t k2 = lt + q * TPF;
        const bool in = k1 < N1 && k2 < N2;
        const C v = Cin[min(k1, N1 - 1) * N2 + min(k2, N2 - 1)];
        cv[q] = in ? v : cmake<C>(0, 0);
        zk[q] = zcoord<R>(k2, zm);
    }
    for (int r = r_lo; r < r_hi; ++r) {
        C v[16];
        {
            R wq[16];
            cheb_v_many<R, 16>(r, zk, wq);
#pragma unroll
            for (int q = 0; q < 16; ++q) v[q] = cscale(cv[q], wq[q]);
        }
        __syncthreads();
        block_fft_regs<C, GY, -1, fft_wave_sync<GY>>(buf + g * P, tw, lt, v);
        fft_publish<GY>();
        C *Hr = H + (int64_t)r * rstride + k1_0;
#pragma unroll 4
        for (int e = 0; e < 16; ++e) {
            const int i = tid + e * NT;
            const int gg = i % G, n2 = i / G;
            if (k1_0 + gg < N1) Hr[(int64_t)n2 * GX + gg] = buf[gg * P + lds_pad(n2)];
        }
    }
}

// ---- pass B: one column n2, a range of its samples ---------------------------
template <typename R, int GX, int RC, int S>
__global__ void __launch_bounds__(RC * GX / 16)
k_2d_passB(const cx_t<R> *__restrict__ H, int64_t N1, int64_t GY, const int4 *__restrict__ tasks, int ntasks,
           const uint32_t *__restrict__ keys, const int32_t *__restrict__ perm, const R *__restrict__ Xxs,
           const R *__restrict__ Xys, Factors<R> fx, Factors<R> fy, const cx_t<R> *__restrict__ tw_g,
           cx_t<R> *__restrict__ f)
{
    using C = cx_t<R>;
    constexpr int TPF = GX / 16;
    constexpr int NT = RC * TPF;
    constexpr int P = fft_pitch(GX);
    __shared__ C buf[RC * P];
    __shared__ C tw[GX];
    __shared__ C hrow[GX];
    const int task = xcd_task(ntasks);
    if (task < 0) return;
    const int4 tk = tasks[task];
    const int64_t n2 = tk.x, i_lo = tk.y, i_hi = tk.z;
    load_tw_s<C, GX, -1, NT>(tw, tw_g);
    const int tid = threadIdx.x;
    const int g = tid / TPF, lt = tid % TPF;
    // sample data of the task: loads issued together (clamped indices), one wait
    uint32_t kv[S];
    R xx[S], xy[S], py[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int64_t i = min(i_lo + s * NT + tid, i_hi - 1);
        kv[s] = keys[i];
        xx[s] = Xxs[i];
        xy[s] = Xys[i];
    }
    C acc[S];
#pragma unroll
    for (int s = 0; s < S; ++s) acc[s] = cmake<C>(0, 0);
    const ZMap zm = zmap(N1);
    // The RC transforms of a round all start from the same row H_r2[n2][:]: it
    // is staged once per r2 in LDS (GX/NT elements per thread), and the next
    // row is loaded into registers while the current one is in use.  Rows
    // k1 >= N1 of H are never written: they read as zero.
    constexpr int HE = GX / NT;
    C hn[HE];
    auto load_row = [&](int r2) {
        const C *Hrow = H + ((int64_t)r2 * GY + n2) * GX;
#pragma unroll
        for (int e = 0; e < HE; ++e) {
            const int k1 = tid + e * NT;
            const C v = Hrow[min(k1, (int)N1 - 1)];
            hn[e] = k1 < N1 ? v : cmake<C>(0, 0);
        }
    };
    load_row(0);
    for (int r2 = 0; r2 < fy.K; ++r2) {
        __syncthreads();   // every reader of the previous row is done
#pragma unroll
        for (int e = 0; e < HE; ++e) hrow[tid + e * NT] = hn[e];
        if (r2 + 1 < fy.K) load_row(r2 + 1);
        {
            const RankPoly<R> uy = rank_poly(fy, r2);
#pragma unroll
            for (int s = 0; s < S; ++s)
                if (i_lo + s * NT < i_hi) py[s] = rank_eval(uy, xy[s] * fy.inv_gamma);
        }
        for (int r0 = 0; r0 < fx.K; r0 += RC) {
            const int r1 = r0 + g;
            __syncthreads();   // the row is staged; the previous gather is finished with buf
            C v[16];
            {
                R zq[16], wq[16];
#pragma unroll
                for (int q = 0; q < 16; ++q) zq[q] = zcoord<R>(lt + q * TPF, zm);
                cheb_v_many<R, 16>(r1 < fx.K ? r1 : 0, zq, wq);
#pragma unroll
                for (int q = 0; q < 16; ++q) v[q] = r1 < fx.K ? cscale(hrow[lt + q * TPF], wq[q]) : cmake<C>(0, 0);
            }
            block_fft_regs<C, GX, -1, fft_wave_sync<GX>>(buf + g * P, tw, lt, v, r1 < fx.K);
            fft_publish<GX>();
            const int nr = min(RC, fx.K - r0);
            for (int gg = 0; gg < nr; ++gg) {   // rank outer (coefficients loaded once), samples inner
                const int rr = r0 + gg;
                const RankPoly<R> ux = rank_poly(fx, rr);
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    if (i_lo + s * NT < i_hi) {
                        const int pos = (int)(kv[s] & (uint32_t)(GX - 1));
                        const C xv = buf[gg * P + lds_pad(pos)];
                        acc[s] = cadd(acc[s], crot(cscale(xv, rank_eval(ux, xx[s] * fx.inv_gamma) * py[s]), rr + r2));
                    }
                }
            }
        }
    }
    int32_t jv[S];   // output positions, loaded together at the end
#pragma unroll
    for (int s = 0; s < S; ++s) jv[s] = perm[min(i_lo + s * NT + tid, i_hi - 1)];
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int64_t i = i_lo + s * NT + tid;
        if (i < i_hi) {
            R sn, cs;
            sincospi_r(xx[s] + xy[s], &sn, &cs);
            f[jv[s]] = cmul(cmake<C>(cs, -sn), acc[s]);
        }
    }
}

// ---- adjoint / type-I pass B': one column n2 (or a slice of its samples) -> Z_r2[n2][k1] ----
// Task = (n2, first, end, slot): the sorted samples [first, end) of column n2,
// at most SCAP of them, staged once in LDS (exp(DIR i pi (Xx + Xy)) g_j, zx,
// zy, tx).  For each r2 and chunk of RC ranks r1 they are summed per grid point
// (balanced segmented sum, deterministic), transformed along n1 (sign DIR),
// weighted by v^x_r1(k1) and summed over r1 in registers; the row for
// r2 is written once: to Z_r2[n2][:] when the task holds the whole column
// (slot < 0), else to partial row `slot` of Zp, which k_2d_sum_parts adds up.
// Sparse tasks (no thread's grid points hold more than about twice the
// average) take a second route: thread (g, lt) owns the 16 grid points
// lt + q GX/16 of rank slot g, which are exactly the operands of its first
// FFT stage.  Per r2 the samples' w_j = exp(DIR i pi (Xx + Xy)) g_j P^y_r2(zy_j)
// are formed once; per rank the thread sums each owned point's run of
// samples in registers and starts the transform from registers: no grid
// clearing, no cross-thread stitching, no grid stores.
template <typename R, int GX, int RC, int SCAP, bool TWG, int DIR>
__global__ void __launch_bounds__(RC * GX / 16)
k_2d_passB_adj(const cx_t<R> *__restrict__ gin, int64_t N1, int64_t GY, const int4 *__restrict__ tasks, int ntasks,
               const int32_t *__restrict__ perm, const uint32_t *__restrict__ keys, const R *__restrict__ Xxs,
               const R *__restrict__ Xys, Factors<R> fx, Factors<R> fy, const cx_t<R> *__restrict__ twd_g,
               cx_t<R> *__restrict__ Z, cx_t<R> *__restrict__ Zp)
{
    using C = cx_t<R>;
    constexpr int TPF = GX / 16;
    constexpr int NT = RC * TPF;
    constexpr int ZA = GX / NT;           // output positions per thread
    constexpr int P = fft_pitch(GX);
    __shared__ __align__(16) C buf[RC * P];   // 16-byte aligned: cleared with 16-byte stores
    __shared__ C tw_s[TWG ? 1 : GX];
    // one 16-byte (FP32) record per staged sample: exp(DIR i pi (Xx + Xy)) g_j, zx, zy
    struct alignas(4 * sizeof(R)) Staged {
        R re, im, zx, zy;
    };
    __shared__ Staged sst[SCAP];
    __shared__ unsigned short spos[SCAP];
    // the segmented spread's scratch; the owner route's per-r2 sample records reuse it
    struct alignas(4 * sizeof(R)) Weighted {
        R re, im, zx, pad;
    };
    constexpr int SEGS = 2 * RC * NT * (int)sizeof(C) + 4 * NT * (int)sizeof(int);
    constexpr int SEGW = SCAP * (int)sizeof(Weighted);
    constexpr int SEGB = SEGS > SEGW ? SEGS : SEGW;
    __shared__ __align__(16) char segs[SEGB];
    C *hv = reinterpret_cast<C *>(segs), *tv = hv + RC * NT;
    int *hix = reinterpret_cast<int *>(tv + RC * NT), *tix = hix + NT, *nxa = tix + NT, *nxb = nxa + NT;
    Weighted *sw = reinterpret_cast<Weighted *>(segs);
    const C *tw = TWG ? twd_g : tw_s;
    const int task = xcd_task(ntasks);
    if (task < 0) return;
    const int4 tk = tasks[task];
    const int tid = threadIdx.x;
    if (!TWG) load_tw_s<C, GX, -1, NT>(tw_s, twd_g);   // twd_g already has the sign DIR
    const int g = tid / TPF, lt = tid % TPF;
    const int64_t n2 = tk.x;
    const int tile_lo = tk.y;
    const int cnt = min(tk.z - tk.y, SCAP);   // the plan never makes a task larger than SCAP
    if (cnt > 0) {
        // stage the samples: index/value loads of a thread issued together
        // (clamped indices), then the dependent loads of g
        constexpr int SU = (SCAP + NT - 1) / NT;
        constexpr int SB = SU < 8 ? SU : 8;
        for (int u0 = 0; u0 < SU; u0 += SB) {
            if (u0 * NT >= cnt) break;
            R ax[SB], ay[SB];
            int32_t jv[SB];
            uint32_t kv[SB];
#pragma unroll
            for (int u = 0; u < SB; ++u) {
                const int i = tile_lo + min(tid + (u0 + u) * NT, cnt - 1);
                ax[u] = Xxs[i];
                ay[u] = Xys[i];
                jv[u] = perm[i];
                kv[u] = keys[i];
            }
            C gv[SB];
#pragma unroll
            for (int u = 0; u < SB; ++u) gv[u] = gin[jv[u]];
#pragma unroll
            for (int u = 0; u < SB; ++u) {
                const int i = tid + (u0 + u) * NT;
                if (i < cnt) {
                    R sn, cs;
                    sincospi_r(ax[u] + ay[u], &sn, &cs);
                    const C v = cmul(cmake<C>(cs, DIR * sn), gv[u]);   // exp(DIR i pi (Xx + Xy))
                    sst[i] = Staged{v.x, v.y, ax[u] * fx.inv_gamma, ay[u] * fy.inv_gamma};
                    spos[i] = (unsigned short)(kv[u] & (uint32_t)(GX - 1));
                }
            }
        }
    }
    const ZMap zm = zmap(N1);
    // runs of the owned grid points: start | count << 16 (counts <= SCAP < 2^16),
    // from the first sample at or after each point (binary search in spos),
    // built in buf before its first transform
    __syncthreads();   // staging done
    int *soff = reinterpret_cast<int *>(buf);   // GX + 1 ints
    static_assert((GX + 1) * (int)sizeof(int) <= RC * P * (int)sizeof(C), "offsets exceed the grid buffer");
    for (int p = tid; p <= GX; p += NT) {
        int lo = 0, hi = cnt;   // first i with spos[i] >= p
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if ((int)spos[mid] < p) lo = mid + 1;
            else hi = mid;
        }
        soff[p] = lo;
    }
    __syncthreads();
    int pk[16];
    int work = 0;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int p = lt + q * TPF;
        const int a = soff[p], n = soff[p + 1] - a;
        pk[q] = a | (n << 16);
        work += n;
    }
    // the owner route when no thread's points hold more than twice the average plus 16
    const bool own = !__syncthreads_or(work > 2 * (cnt * 16 / GX) + 16);
    if (own) {
        for (int r2 = 0; r2 < fy.K; ++r2) {
            __syncthreads();   // the previous r2's readers of sw and buf are done
            const RankPoly<R> uy = rank_poly(fy, r2);
            for (int i = tid; i < cnt; i += NT) {
                const Staged t = sst[i];
                const R wy = rank_eval(uy, t.zy);
                sw[i] = Weighted{t.re * wy, t.im * wy, t.zx, (R)0};
            }
            C za[ZA];
#pragma unroll
            for (int m = 0; m < ZA; ++m) za[m] = cmake<C>(0, 0);
            for (int r0 = 0; r0 < fx.K; r0 += RC) {
                const int nr = min(RC, fx.K - r0);
                const int r1 = r0 + g;
                const RankPoly<R> ux = rank_poly(fx, min(r1, fx.K - 1));
                __syncthreads();   // sw complete; the previous chunk's readers of buf are done
                C v[16];
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    C acc = cmake<C>(0, 0);
                    const int a = pk[q] & 0xffff, e = a + (pk[q] >> 16);
                    for (int i = a; i < e; ++i) {
                        const Weighted w = sw[i];
                        acc = cadd(acc, cscale(cmake<C>(w.re, w.im), rank_eval(ux, w.zx)));
                    }
                    // i^(r1 + r2) for the type I, i^-(r1 + r2) for the adjoint
                    v[q] = crot(acc, -DIR * (r1 + r2));
                }
                block_fft_regs<C, GX, DIR, fft_wave_sync<GX>>(buf + g * P, tw, lt, v, r1 < fx.K);
                fft_publish<GX>();
                R zq[ZA], t0[ZA], t1[ZA];
#pragma unroll
                for (int m = 0; m < ZA; ++m) zq[m] = zcoord<R>(tid + m * NT, zm);
                cheb_pair_many<R, ZA>(r0, zq, t0, t1);
                for (int gg = 0; gg < nr; ++gg) {
#pragma unroll
                    for (int m = 0; m < ZA; ++m) {
                        const int k1 = tid + m * NT;
                        const R w = (r0 + gg == 0) ? (R)0.5 : t0[m];
                        za[m] = cadd(za[m], cscale(buf[gg * P + lds_pad(k1)], w));
                        const R c = 2 * zq[m] * t1[m] - t0[m];
                        t0[m] = t1[m];
                        t1[m] = c;
                    }
                }
            }
            C *Zrow = tk.w < 0 ? Z + ((int64_t)r2 * GY + n2) * GX : Zp + ((int64_t)tk.w * fy.K + r2) * GX;
#pragma unroll
            for (int m = 0; m < ZA; ++m) Zrow[tid + m * NT] = za[m];
        }
        return;
    }
    for (int r2 = 0; r2 < fy.K; ++r2) {
        __syncthreads();   // staging done
        const RankPoly<R> uy = rank_poly(fy, r2);   // P^y_r2 is evaluated per sample in the spread
        C za[ZA];
#pragma unroll
        for (int m = 0; m < ZA; ++m) za[m] = cmake<C>(0, 0);
        for (int r0 = 0; r0 < fx.K; r0 += RC) {
            const int nr = min(RC, fx.K - r0);
            if constexpr (sizeof(R) == 4) {   // 16-byte stores: two grid values each
                float4 *b4 = reinterpret_cast<float4 *>(buf);
                for (int m = tid; m < (RC * P) / 2; m += NT) b4[m] = make_float4(0.f, 0.f, 0.f, 0.f);
                if ((RC * P) % 2 && tid == 0) buf[RC * P - 1] = cmake<C>(0, 0);
            } else {
                for (int m = tid; m < RC * P; m += NT) buf[m] = cmake<C>(0, 0);
            }
            __syncthreads();
            auto pos = [&](int i) -> int { return (int)spos[i]; };
            RankPoly<R> ux[RC];
#pragma unroll
            for (int gg = 0; gg < RC; ++gg) ux[gg] = rank_poly(fx, min(r0 + gg, fx.K - 1));
            struct Sample {
                int n;
                C w;   // exp(DIR i pi (Xx + Xy)) g_j P^y_r2(zy_j)
                R zx;
            };
            // the factor i^(r1 + r2) (type I) or i^-(r1 + r2) (adjoint), r1 = r0 + gg:
            // the part of r0 + r2 is applied once per sample, that of gg (a
            // compile-time index in the unrolled chunk) per rank
            auto load = [&](int i) -> Sample {
                const Staged t = sst[i];
                return Sample{(int)spos[i], crot(cscale(cmake<C>(t.re, t.im), rank_eval(uy, t.zy)), -DIR * (r0 + r2)),
                              t.zx};
            };
            auto contrib = [&](const Sample &sm, int gg) -> C {
                const bool odd = RC % 2 == 0 ? (gg & 1) != 0 : ((r0 + gg) & 1) != 0;
                return crot(cscale(sm.w, rank_eval_par(ux[gg], sm.zx, odd)), -DIR * gg);
            };
            seg_spread<C, RC, NT>(cnt, nr, pos, load, contrib, buf, P, hv, tv, hix, tix, nxa, nxb);
            __syncthreads();
            block_fft_lds<C, GX, DIR, fft_wave_sync<GX>>(buf + g * P, tw, lt);
            fft_publish<GX>();
            // T_{r0 + gg} for the consecutive ranks of the chunk by the recurrence
            R zq[ZA], t0[ZA], t1[ZA];
#pragma unroll
            for (int m = 0; m < ZA; ++m) zq[m] = zcoord<R>(tid + m * NT, zm);
            cheb_pair_many<R, ZA>(r0, zq, t0, t1);
            for (int gg = 0; gg < nr; ++gg) {
#pragma unroll
                for (int m = 0; m < ZA; ++m) {
                    const int k1 = tid + m * NT;
                    const R w = (r0 + gg == 0) ? (R)0.5 : t0[m];
                    za[m] = cadd(za[m], cscale(buf[gg * P + lds_pad(k1)], w));
                    const R c = 2 * zq[m] * t1[m] - t0[m];
                    t0[m] = t1[m];
                    t1[m] = c;
                }
            }
            __syncthreads();
        }
        C *Zrow = tk.w < 0 ? Z + ((int64_t)r2 * GY + n2) * GX : Zp + ((int64_t)tk.w * fy.K + r2) * GX;
#pragma unroll
        for (int m = 0; m < ZA; ++m) Zrow[tid + m * NT] = za[m];
    }
}

// Columns whose samples were split over several pass-B' tasks: task t = (n2,
// first slot, number of slots) adds the partial rows in slot order (a fixed
// order: the result does not depend on timing).  Block = (t, r2).
template <typename R>
__global__ void __launch_bounds__(256)
k_2d_sum_parts(const int4 *__restrict__ rtasks, const cx_t<R> *__restrict__ Zp, int64_t GX, int64_t GY, int Ky,
               cx_t<R> *__restrict__ Z)
{
    using C = cx_t<R>;
    const int4 rt = rtasks[blockIdx.x];
    const int r2 = blockIdx.y;
    for (int64_t k1 = threadIdx.x; k1 < GX; k1 += blockDim.x) {
        C a = Zp[((int64_t)rt.y * Ky + r2) * GX + k1];
        for (int q = 1; q < rt.z; ++q) a = cadd(a, Zp[((int64_t)(rt.y + q) * Ky + r2) * GX + k1]);
        Z[((int64_t)r2 * GY + rt.x) * GX + k1] = a;
    }
}

// ---- adjoint / type-I pass A': G rows k1, FFT along n2 -> k2 (sign DIR), weighted sum over r2 ----
template <typename R, int GY, int G, int DIR>
__global__ void __launch_bounds__(G * GY / 16)
k_2d_passA_adj(const cx_t<R> *__restrict__ Z, int64_t N1, int64_t N2, int64_t GX, int Ky,
               const cx_t<R> *__restrict__ twd_g, cx_t<R> *__restrict__ Cout, int64_t rstride)
{
    // stacked problems: blockIdx.y is the problem; Z_r2 rows are rstride apart
    Z += (int64_t)blockIdx.y * GY * GX;
    Cout += (int64_t)blockIdx.y * N1 * N2;
    using C = cx_t<R>;
    constexpr int TPF = GY / 16;
    constexpr int NT = G * TPF;
    constexpr int P = fft_pitch_g(GY, G);
    __shared__ C buf[G * P];
    __shared__ C tw[GY];
    const int ncg = (int)((N1 + G - 1) / G);
    const int task = xcd_task(ncg);
    if (task < 0) return;
    const int tid = threadIdx.x;
    load_tw_s<C, GY, -1, NT>(tw, twd_g);   // twd_g already has the sign DIR
    const int g = tid / TPF, lt = tid % TPF;
    const int64_t k1_0 = (int64_t)task * G;
    const ZMap zm = zmap(N2);
    C acc[16], zn[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int i = tid + e * NT;
        acc[e] = cmake<C>(0, 0);
        const C v = Z[(int64_t)(i / G) * GX + min(k1_0 + (i % G), N1 - 1)];   // clamped: no branch
        zn[e] = (k1_0 + (i % G) < N1) ? v : cmake<C>(0, 0);
    }
    for (int r = 0; r < Ky; ++r) {
        __syncthreads();
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int i = tid + e * NT;
            buf[(i % G) * P + lds_pad(i / G)] = zn[e];
        }
        if (r + 1 < Ky) {
            const C *Zr = Z + (int64_t)(r + 1) * rstride + k1_0;
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int i = tid + e * NT;
                const C v = Zr[(int64_t)(i / G) * GX + min((int64_t)(i % G), N1 - 1 - k1_0)];
                zn[e] = (k1_0 + (i % G) < N1) ? v : cmake<C>(0, 0);
            }
        }
        __syncthreads();
        block_fft_lds<C, GY, DIR, fft_wave_sync<GY>>(buf + g * P, tw, lt);
        fft_publish<GY>();
#pragma unroll
        for (int h = 0; h < 16; h += 8) {   // two halves of 8: bounded transient registers
            R zq[8], wq[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) zq[e] = zcoord<R>((tid + (h + e) * NT) / G, zm);
            cheb_v_many<R, 8>(r, zq, wq);
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int i = tid + (h + e) * NT;
                acc[h + e] = cadd(acc[h + e], cscale(buf[(i % G) * P + lds_pad(i / G)], wq[e]));
            }
        }
    }
    // transpose through LDS so that rows of C are written contiguously
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int i = tid + e * NT;
        buf[(i % G) * P + lds_pad(i / G)] = acc[e];
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int i = tid + e * NT;
        const int gg = i / GY, k2 = i % GY;
        if (k1_0 + gg < N1 && k2 < N2) Cout[(k1_0 + gg) * N2 + k2] = buf[gg * P + lds_pad(k2)];
    }
}

// ---- dispatch -----------------------------------------------------------------

template <typename R>
hipError_t fused_2d(const Args2D<R> &a, const cx_t<R> *Cin, cx_t<R> *f, hipStream_t s)
{
    constexpr bool F = sizeof(R) == 4;
    const int64_t cols = (int64_t)a.S * a.Gy;   // pass-B columns over the stacked problems
    const int64_t rstride = cols * a.Gx;         // distance between the intermediate's ranks
    prof_begin(a.prof, "fwd2d_passA", s);
    switch (a.Gy) {
#define A2(GG, GF, GD)                                                                                      \
    case GG: {                                                                                              \
        constexpr int G = F ? GF : GD;                                                                      \
        const int ncg = (int)((a.N1 + G - 1) / G);                                                          \
        int nrc = (256 + ncg - 1) / ncg;                                                                    \
        nrc = nrc < 1 ? 1 : (nrc > a.fy.K ? a.fy.K : nrc);                                                  \
        const int rca = (a.fy.K + nrc - 1) / nrc;                                                           \
        const int T = ncg * ((a.fy.K + rca - 1) / rca);                                                     \
        hipLaunchKernelGGL((k_2d_passA<R, GG, G>), dim3(xcd_grid(T), a.S), dim3(G * GG / 16), 0, s, Cin, a.N1,  \
                           a.N2, (int64_t)a.Gx, a.fy, rca, a.twy, a.H, rstride);                            \
        break;                                                                                              \
    }
        A2(16, 8, 8)
        A2(32, 8, 8)
        A2(64, 8, 8)
        A2(128, 8, 8)
        A2(256, 8, 8)
        A2(512, 8, 4)
        A2(1024, 8, 4)
        A2(2048, 4, 2)
#undef A2
    default: return hipErrorInvalidValue;
    }
    prof_end(a.prof, s);
    prof_begin(a.prof, "fwd2d_passB", s);
    switch (a.Gx) {
#define B2(GG, RF, SF, RD, SD)                                                                              \
    case GG: {                                                                                              \
        constexpr int RR = F ? RF : RD, SS = F ? SF : SD;                                                   \
        hipLaunchKernelGGL((k_2d_passB<R, GG, RR, SS>), dim3(xcd_grid(a.ntasks)), dim3(RR * GG / 16), 0, s,   \
                           (const cx_t<R> *)a.H, a.N1, cols, a.tasks, a.ntasks, a.keys, a.perm,              \
                           a.Xxs, a.Xys, a.fx, a.fy, a.twx, f);                                             \
        break;                                                                                              \
    }
        B2(16, 16, 4, 16, 4)
        B2(32, 16, 4, 16, 4)
        B2(64, 16, 4, 16, 4)
        B2(128, 16, 4, 8, 4)
        B2(256, 16, 4, 8, 4)
        B2(512, 8, 8, 4, 4)
        B2(1024, 4, 8, 4, 4)
        B2(2048, 2, 8, 2, 4)
#undef B2
    default: return hipErrorInvalidValue;
    }
    prof_end(a.prof, s);
    return hipGetLastError();
}

template <typename R, int DIR>
static hipError_t fused_2d_t1_dir(const Args2D<R> &a, const cx_t<R> *gin, cx_t<R> *Cout, hipStream_t s)
{
    constexpr bool F = sizeof(R) == 4;
    const cx_t<R> *twx = DIR < 0 ? a.twx : a.twxi, *twy = DIR < 0 ? a.twy : a.twyi;
    const int64_t cols = (int64_t)a.S * a.Gy;   // pass-B' columns over the stacked problems
    const int64_t rstride = cols * a.Gx;
    prof_begin(a.prof, DIR > 0 ? "adj2d_passB" : "type1_2d_passB", s);
    switch (a.Gx) {
#define BA2(GG, RF, SCF, RD, SCD, TG)                                                                        \
    case GG: {                                                                                              \
        constexpr int RR = F ? RF : RD, SC = F ? SCF : SCD;                                                 \
        hipLaunchKernelGGL((k_2d_passB_adj<R, GG, RR, SC, TG, DIR>), dim3(xcd_grid(a.natasks)),             \
                           dim3(RR * GG / 16), 0, s, gin, a.N1, cols, a.atasks, a.natasks, a.perm,            \
                           a.keys, a.Xxs, a.Xys, a.fx, a.fy, twx, a.H, a.Zp);                               \
        break;                                                                                              \
    }
        BA2(16, 16, 256, 16, 256, false)
        BA2(32, 16, 256, 16, 256, false)
        BA2(64, 16, 256, 16, 256, false)
        BA2(128, 16, 512, 8, 512, false)
        BA2(256, 16, 512, 8, 512, false)
        BA2(512, 8, 1024, 4, 768, false)
        BA2(1024, 4, 1280, 4, 768, true)
        BA2(2048, 2, 2304, 2, 1280, true)
#undef BA2
    default: return hipErrorInvalidValue;
    }
    prof_end(a.prof, s);
    if (a.nrtasks > 0) {
        prof_begin(a.prof, DIR > 0 ? "adj2d_sum" : "type1_2d_sum", s);
        hipLaunchKernelGGL(k_2d_sum_parts<R>, dim3(a.nrtasks, a.fy.K), dim3(256), 0, s, a.rtasks,
                           (const cx_t<R> *)a.Zp, (int64_t)a.Gx, cols, a.fy.K, a.H);
        prof_end(a.prof, s);
    }
    prof_begin(a.prof, DIR > 0 ? "adj2d_passA" : "type1_2d_passA", s);
    switch (a.Gy) {
#define AA2(GG, GF, GD)                                                                                     \
    case GG: {                                                                                              \
        constexpr int G = F ? GF : GD;                                                                      \
        const int ncg = (int)((a.N1 + G - 1) / G);                                                          \
        hipLaunchKernelGGL((k_2d_passA_adj<R, GG, G, DIR>), dim3(xcd_grid(ncg), a.S), dim3(G * GG / 16), 0, s, \
                           (const cx_t<R> *)a.H, a.N1, a.N2, (int64_t)a.Gx, a.fy.K, twy, Cout, rstride);    \
        break;                                                                                              \
    }
        AA2(16, 8, 8)
        AA2(32, 8, 8)
        AA2(64, 8, 8)
        AA2(128, 8, 8)
        AA2(256, 8, 8)
        AA2(512, 8, 4)
        AA2(1024, 8, 4)
        AA2(2048, 4, 2)
#undef AA2
    default: return hipErrorInvalidValue;
    }
    prof_end(a.prof, s);
    return hipGetLastError();
}

template <typename R>
hipError_t fused_2d_adj(const Args2D<R> &a, const cx_t<R> *gin, cx_t<R> *Cout, int sign, hipStream_t s)
{
    return sign < 0 ? fused_2d_t1_dir<R, -1>(a, gin, Cout, s) : fused_2d_t1_dir<R, 1>(a, gin, Cout, s);
}

// Samples per adjoint pass-B' task (the LDS staging capacity of the instantiation above).
int pass_b2d_adj_cap(int GX, bool fp32)
{
    switch (GX) {
    case 16: case 32: case 64: return 256;
    case 128: case 256: return 512;
    case 512: return fp32 ? 1024 : 768;
    case 1024: return fp32 ? 1280 : 768;
    case 2048: return fp32 ? 2304 : 1280;
    default: return 0;
    }
}

// Samples per forward pass-B task (threads x slots of the instantiation above).
int pass_b2d_cap(int GX, bool fp32)
{
    switch (GX) {
    case 16: case 32: case 64: return (16 * GX / 16) * 4;
    case 128: case 256: return fp32 ? (16 * GX / 16) * 4 : (8 * GX / 16) * 4;
    case 512: return fp32 ? (8 * 512 / 16) * 8 : (4 * 512 / 16) * 4;
    case 1024: return fp32 ? (4 * 1024 / 16) * 8 : (4 * 1024 / 16) * 4;
    case 2048: return fp32 ? (2 * 2048 / 16) * 8 : (2 * 2048 / 16) * 4;
    default: return 0;
    }
}

// ---- plan kernel: both axes at once ----------------------------------------------
template <typename R>
__global__ void __launch_bounds__(256)
k_assign2d(const double *__restrict__ x, const double *__restrict__ y, const int32_t *__restrict__ slice, int64_t M,
           int64_t GX, int64_t GY, double sx, double sy, R *__restrict__ Xx, R *__restrict__ Xy,
           uint32_t *__restrict__ key, int32_t *__restrict__ hist, unsigned long long *gbits, int *bad)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double ax = 0.0, ay = 0.0;
    if (j < M) {
        const double xj = x[j], yj = y[j];
        int tx = 0, ty = 0;
        double dx = 0.0, dy = 0.0;
        if (!isfinite(xj) || !isfinite(yj)) {
            atomicOr(bad, 1);
        } else {
            const double gx = (double)GX, gy = (double)GY;
            const double s1 = rint(gx * xj), s2 = rint(gy * yj);
            dx = fma(gx, xj, -s1) * sx;
            dy = fma(gy, yj, -s2) * sy;
            double t1 = fmod(s1, gx), t2 = fmod(s2, gy);
            if (t1 < 0.0) t1 += gx;
            if (t2 < 0.0) t2 += gy;
            tx = (int)t1;
            ty = (int)t2;
            ax = fabs(dx);
            ay = fabs(dy);
        }
        const uint32_t sl = slice ? (uint32_t)slice[j] : 0u;   // the plan bounds S * GX * GY below 2^32
        const uint32_t k = (sl * (uint32_t)GY + (uint32_t)ty) * (uint32_t)GX + (uint32_t)tx;
        Xx[j] = (R)dx;
        Xy[j] = (R)dy;
        key[j] = k;
        atomicAdd(&hist[k], 1);
    }
    // wave maxima, then one atomic per wave and axis
    for (int o = 32; o > 0; o >>= 1) {
        ax = fmax(ax, __shfl_xor(ax, o, 64));
        ay = fmax(ay, __shfl_xor(ay, o, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMax(gbits, (unsigned long long)__double_as_longlong(ax));
        atomicMax(gbits + 1, (unsigned long long)__double_as_longlong(ay));
    }
}

template <typename R>
hipError_t launch_assign2d(const double *x, const double *y, const int32_t *slice, int64_t M, int64_t GX,
                           int64_t GY, double sx, double sy, R *Xx, R *Xy, uint32_t *key, int32_t *hist,
                           unsigned long long *gbits, int *bad, hipStream_t s)
{
    hipLaunchKernelGGL(k_assign2d<R>, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, x, y, slice, M, GX, GY,
                       sx, sy, Xx, Xy, key, hist, gbits, bad);
    return hipGetLastError();
}

template hipError_t fused_2d<float>(const Args2D<float> &, const float2 *, float2 *, hipStream_t);
template hipError_t fused_2d<double>(const Args2D<double> &, const double2 *, double2 *, hipStream_t);
template hipError_t fused_2d_adj<float>(const Args2D<float> &, const float2 *, float2 *, int, hipStream_t);
template hipError_t fused_2d_adj<double>(const Args2D<double> &, const double2 *, double2 *, int, hipStream_t);
template hipError_t launch_assign2d<float>(const double *, const double *, const int32_t *, int64_t, int64_t,
                                           int64_t, double, double, float *, float *, uint32_t *, int32_t *,
                                           unsigned long long *, int *, hipStream_t);
template hipError_t launch_assign2d<double>(const double *, const double *, const int32_t *, int64_t, int64_t,
                                            int64_t, double, double, double *, double *, uint32_t *, int32_t *,
                                            unsigned long long *, int *, hipStream_t);

}  // namespace nufft
