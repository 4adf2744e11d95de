// Batches of independent type-II transforms of uneven sizes in one persistent
// launch (oversampled grids L_b >= N_b as in Sec. 2.3).
//
// A task table, built by the plan, lists for every transform b either
//   SMALL tasks (L_b <= 4096: scale, all K FFTs in LDS and a slice of the
//   samples, as the one-workgroup kernel does), or
//   PASS_A tasks (a group of columns of the two-pass split) followed, after
//   every phase-1 task of the batch, by PASS_B tasks (a run of consecutive
//   output tiles, about 2048 grid points, so that the per-task set-up is
//   amortised over many small tiles).
// Workgroups claim tasks in table order from an atomic counter, one task
// ahead of the one they run.  A PASS_B task waits until every PASS_A task of
// its transform has finished (counter per transform, device-scope
// release/acquire).  Because all phase-1 tasks precede all PASS_B tasks in the
// table and a phase-1 task never waits, every wait ends: each unfinished
// PASS_A task the waiter depends on is held, as its current or next task, by
// a running workgroup whose current task does not wait.  The last workgroup
// to leave resets the counters, so the launch can be replayed (HIP graph)
// without any memset.
#include "batch.h"
#include "fused_common.h"

namespace nufft {

#define BNT 256              // threads per workgroup of the persistent kernel
#ifndef BSLOTS
#define BSLOTS 8             // sample slots per thread in SMALL tasks
#endif
#ifndef NUFFT_BATCH_WAVES
#define NUFFT_BATCH_WAVES 2  // waves per SIMD the register allocation targets
#endif

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// ---- SMALL: whole transform in LDS, samples [chunk * BNT * BSLOTS, ...) -----------------
template <typename R, int L>
__device__ __forceinline__ void b_small_body(const BatchDesc<R> &d, const cx_t<R> *__restrict__ c, cx_t<R> *__restrict__ f, int chunk,
                        char *lds)
{
    using C = cx_t<R>;
    constexpr int TPF = L / 16;
    constexpr int RC = BNT / TPF;
    constexpr int P = fft_pitch(L);
    C *buf = (C *)lds;
    C *tw = buf + RC * P;
    load_tw_s<C, L, -1, BNT>(tw, d.tw1);
    const int tid = threadIdx.x;
    const int64_t j0 = (int64_t)chunk * (BNT * BSLOTS);
    const Factors<R> &fac = *d.fac;
    const int K = fac.K;
    int pos[BSLOTS];
    R xs[BSLOTS];
    C acc[BSLOTS];
#pragma unroll
    for (int s = 0; s < BSLOTS; ++s) {
        const int64_t j = min(j0 + s * BNT + tid, d.M - 1);   // clamped: loads issued together
        pos[s] = d.t[j];
        xs[s] = d.X[j];
        acc[s] = cmake<C>(0, 0);
    }
    const int g = tid / TPF, lt = tid % TPF;
    const ZMap zm = zmap(d.N);
    for (int r0 = 0; r0 < K; r0 += RC) {
        const int r = r0 + g;
        C v[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) v[q] = load_coef<R>(c, lt + q * TPF, d.N, 0);
#pragma unroll
        for (int q = 0; q < 16; ++q)
            v[q] = r < K ? cscale(v[q], cheb_v<R>(r, zcoord<R>(lt + q * TPF, zm))) : cmake<C>(0, 0);
        __syncthreads();
        block_fft_regs<C, L, -1, fft_wave_sync<L>>(buf + g * P, tw, lt, v, r < K);   // idle rank slots skip
        fft_publish<L>();
        const int nr = min(RC, K - r0);
        for (int gg = 0; gg < nr; ++gg) {   // rank outer (coefficients loaded once), samples inner
            const int rr = r0 + gg;
            const RankPoly<R> up = rank_poly(fac, rr);
#pragma unroll
            for (int s = 0; s < BSLOTS; ++s) {
                if (j0 + s * BNT < d.M)
                    acc[s] = cadd(acc[s], crot(cscale(buf[gg * P + lds_pad(pos[s])],
                                                      rank_eval(up, xs[s] * fac.inv_gamma)), rr));
            }
        }
    }
#pragma unroll
    for (int s = 0; s < BSLOTS; ++s) {
        const int64_t j = j0 + s * BNT + tid;
        if (j < d.M) {
            R sn, cs;
            sincospi_r(xs[s], &sn, &cs);
            f[j] = cmul(cmake<C>(cs, -sn), acc[s]);
        }
    }
}

// ---- PASS_A: G = 4096 / L2 adjacent columns, all K ranks -------------------------------
template <typename R, int L2>
__device__ __forceinline__ void b_passA_body(const BatchDesc<R> &d, const cx_t<R> *__restrict__ c, int cg, char *lds)
{
    using C = cx_t<R>;
    constexpr int TPF = L2 / 16;
    constexpr int G = BNT / TPF;
    constexpr int P = fft_pitch_g(L2, G);
    C *buf = (C *)lds;
    C *tw = buf + G * P;
    load_tw_s<C, L2, -1, BNT>(tw, d.tw2);
    const int tid = threadIdx.x;
    const int g = tid / TPF, lt = tid % TPF;
    const int64_t L1 = d.L1;
    const int64_t k1_0 = (int64_t)cg * G;
    const int64_t L = d.L;
    const int K = d.fac->K;
    {
        C cl[16];   // all loads in flight before the first LDS store
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int i = tid + e * BNT;
            cl[e] = load_coef<R>(c, k1_0 + i % G + L1 * (int64_t)(i / G), d.N, 0);
        }
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int i = tid + e * BNT;
            buf[(i % G) * P + lds_pad(i / G)] = cl[e];
        }
    }
    __syncthreads();
    C cv[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) cv[q] = buf[g * P + lds_pad(lt + q * TPF)];
    const ZMap zm = zmap(d.N);
    C wt[16];   // inter-pass twiddles of this thread's output positions, the same for every rank
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int i = tid + e * BNT;
        wt[e] = tw_big<C, -1>(d.hi, d.lo, (k1_0 + i % G) * (int64_t)(i / G));
    }
    for (int r = 0; r < K; ++r) {
        C v[16];
#pragma unroll
        for (int q = 0; q < 16; ++q)
            v[q] = cscale(cv[q], cheb_v<R>(r, zcoord<R>((k1_0 + g) + L1 * (int64_t)(lt + q * TPF), zm)));
        __syncthreads();
        block_fft_regs<C, L2, -1, fft_wave_sync<L2>>(buf + g * P, tw, lt, v);
        fft_publish<L2>();
        C *Yr = d.Y + (int64_t)r * L + k1_0;
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int i = tid + e * BNT;
            const int gg = i % G, n2 = i / G;
            Yr[(int64_t)n2 * L1 + gg] = cmul(buf[gg * P + lds_pad(n2)], wt[e]);
        }
    }
    __syncthreads();   // LDS is reused by the next task
}

// ---- PASS_B: one tile n2, RC = 4096 / L1 ranks side by side ------------------------------
template <typename R, int L1, int S>
__device__ __forceinline__ void b_passB_body(const BatchDesc<R> &d, cx_t<R> *__restrict__ f, int n2_first, int n2_count, char *lds)
{
    using C = cx_t<R>;
    constexpr int TPF = L1 / 16;
    constexpr int RC = BNT / TPF;
    constexpr int P = fft_pitch(L1);
    constexpr int CAP = BNT * S;
    C *buf = (C *)lds;
    C *tw = buf + RC * P;
    load_tw_s<C, L1, -1, BNT>(tw, d.tw1);
    const int tid = threadIdx.x;
    const int g = tid / TPF, lt = tid % TPF;
    const int64_t L = d.L;
    const Factors<R> &fac = *d.fac;
    const int K = fac.K;
    for (int n2 = n2_first; n2 < n2_first + n2_count; ++n2) {
    const int64_t tile_lo = d.off[(int64_t)n2 * L1], tile_hi = d.off[(int64_t)(n2 + 1) * L1];
    const C *Yrow = d.Y + (int64_t)n2 * L1 + lt;
    for (int64_t c0 = tile_lo; c0 < tile_hi; c0 += CAP) {
        uint32_t kv[S];
        R xs[S];
        int32_t jv[S];
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int64_t i = min(c0 + s * BNT + tid, tile_hi - 1);   // clamped: loads issued together
            kv[s] = d.keys[i];
            xs[s] = d.Xs[i];
            jv[s] = d.perm[i];
        }
        C vn[16];   // rows of the next rank chunk, loaded while this one is used
#pragma unroll
        for (int q = 0; q < 16; ++q) vn[q] = g < K ? Yrow[(int64_t)g * L + q * TPF] : cmake<C>(0, 0);
        C acc[S];
#pragma unroll
        for (int s = 0; s < S; ++s) acc[s] = cmake<C>(0, 0);
        for (int r0 = 0; r0 < K; r0 += RC) {
            C v[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) v[q] = vn[q];
            const int rn = r0 + RC + g;
            if (r0 + RC < K) {
#pragma unroll
                for (int q = 0; q < 16; ++q) vn[q] = rn < K ? Yrow[(int64_t)rn * L + q * TPF] : cmake<C>(0, 0);
            }
            __syncthreads();
            block_fft_regs<C, L1, -1, fft_wave_sync<L1>>(buf + g * P, tw, lt, v, r0 + g < K);   // idle slots skip
            fft_publish<L1>();
            const int nr = min(RC, K - r0);
            for (int gg = 0; gg < nr; ++gg) {   // rank outer (coefficients loaded once), samples inner
                const int rr = r0 + gg;
                const RankPoly<R> up = rank_poly(fac, rr);
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    if (c0 + s * BNT < tile_hi) {
                        const int pos = (int)(kv[s] & (uint32_t)(L1 - 1));
                        acc[s] = cadd(acc[s], crot(cscale(buf[gg * P + lds_pad(pos)],
                                                          rank_eval(up, xs[s] * fac.inv_gamma)), rr));
                    }
                }
            }
        }
#pragma unroll
        for (int s = 0; s < S; ++s) {
            if (c0 + s * BNT + tid < tile_hi) {
                R sn, cs;
                sincospi_r(xs[s], &sn, &cs);
                f[jv[s]] = cmul(cmake<C>(cs, -sn), acc[s]);
            }
        }
        __syncthreads();
    }
    }
}

// The persistent kernel calls the task bodies as functions (inlining all of
// them into one kernel spills); the phased kernels inline the one they run.
template <typename R, int L>
__device__ __noinline__ void b_small(const BatchDesc<R> &d, const cx_t<R> *__restrict__ c, cx_t<R> *__restrict__ f,
                                     int chunk, char *lds)
{
    b_small_body<R, L>(d, c, f, chunk, lds);
}
template <typename R, int L2>
__device__ __noinline__ void b_passA(const BatchDesc<R> &d, const cx_t<R> *__restrict__ c, int cg, char *lds)
{
    b_passA_body<R, L2>(d, c, cg, lds);
}
template <typename R, int L1, int S>
__device__ __noinline__ void b_passB(const BatchDesc<R> &d, cx_t<R> *__restrict__ f, int n2_first, int n2_count,
                                     char *lds)
{
    b_passB_body<R, L1, S>(d, f, n2_first, n2_count, lds);
}

template <typename R>
__global__ void __launch_bounds__(BNT) __attribute__((amdgpu_waves_per_eu(NUFFT_BATCH_WAVES)))
k_batch(const BatchDesc<R> *__restrict__ descs, const int4 *__restrict__ tasks, int ntasks, BatchCtl *ctl,
        const cx_t<R> *const *__restrict__ cs, cx_t<R> *const *__restrict__ fs, int64_t spin_limit,
        int unreachable)
{
    extern __shared__ __align__(16) char lds[];
    __shared__ int s_task;
    const int tid = threadIdx.x;
    // Claim-ahead: the next task is claimed while the current one runs.  A
    // PASS_B task held as "next" never blocks a PASS_A task it depends on:
    // every PASS_A task precedes every PASS_B task in the table, so a
    // workgroup whose current task waits holds only PASS_B tasks.
    if (tid == 0) s_task = atomicAdd(&ctl->next, 1);
    __syncthreads();
    int t = uniform(s_task);
    for (;;) {
        __syncthreads();   // s_task is rewritten only after everyone has read it
        if (t >= ntasks) break;
        if (tid == 0) s_task = atomicAdd(&ctl->next, 1);
        const int4 tk = tasks[t];
        const int type = uniform(tk.x), b = uniform(tk.y), par = uniform(tk.z), par2 = uniform(tk.w);
        const BatchDesc<R> &d = descs[b];
        if (type == BATCH_PASS_B) {
            if (tid == 0) {
                const int target = unreachable ? 0x7fffffff : d.n_pass_a;
                int64_t it = 0;
                while (__hip_atomic_load(&ctl->done_a[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
                    if (it++ >= spin_limit) {   // cannot happen by construction; never hang
                        atomicAdd(&ctl->timeouts, 1);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(2);
                }
            }
            __syncthreads();
            __threadfence();   // acquire: see the pass-A results of other workgroups
        }
        switch (type) {
        case BATCH_SMALL:
            switch (d.L) {
#define BS(LL) case LL: b_small<R, LL>(d, cs[b], fs[b], par, lds); break;
                BS(16) BS(32) BS(64) BS(128) BS(256) BS(512) BS(1024) BS(2048) BS(4096)
#undef BS
            default: break;
            }
            break;
        case BATCH_PASS_A:
            switch (d.L2) {
#define BA(LL) case LL: b_passA<R, LL>(d, cs[b], par, lds); break;
                BA(64) BA(128) BA(256) BA(512) BA(1024)
#undef BA
            default: break;
            }
            __threadfence();   // release the pass-A results
            __syncthreads();
            if (tid == 0) atomicAdd(&ctl->done_a[b], 1);
            break;
        default:
            switch (d.L1) {
#define BB(LL, SS) case LL: b_passB<R, LL, SS>(d, fs[b], par, par2, lds); break;
                BB(128, 1) BB(256, 2) BB(512, 3) BB(1024, 5)
#undef BB
            default: break;
            }
            break;
        }
        __syncthreads();   // the task is done; s_task holds the next claim
        t = uniform(s_task);
    }
    // the last workgroup out resets the queue for the next launch
    if (tid == 0) {
        __threadfence();
        const int e = atomicAdd(&ctl->exited, 1);
        if (e == (int)gridDim.x - 1) {
            for (int i = 0; i < ctl->ntransforms; ++i) atomicExch(&ctl->done_a[i], 0);
            atomicExch(&ctl->next, 0);
            __threadfence();
            atomicExch(&ctl->exited, 0);
        }
    }
}

// Phased execution of the same task table: one plain launch per task type
// (SMALL, PASS_A, PASS_B), one workgroup per task, in stream order.  The
// PASS_B launch starts after every PASS_A task has finished, so no task waits
// and there is no queue state; each kernel is compiled for its own task type
// only (fewer registers than the persistent kernel, which holds all three).
template <typename R, int TYPE>
__global__ void __launch_bounds__(BNT) __attribute__((amdgpu_waves_per_eu(NUFFT_BATCH_WAVES)))
k_batch_phase(const BatchDesc<R> *__restrict__ descs, const int4 *__restrict__ tasks, int ntasks,
              const cx_t<R> *const *__restrict__ cs, cx_t<R> *const *__restrict__ fs)
{
    extern __shared__ __align__(16) char lds[];
    const int t = (int)blockIdx.x;
    if (t >= ntasks) return;
    const int4 tk = tasks[t];
    const int b = uniform(tk.y), par = uniform(tk.z), par2 = uniform(tk.w);
    const BatchDesc<R> &d = descs[b];
    if constexpr (TYPE == BATCH_SMALL) {
        switch (d.L) {
#define BS(LL) case LL: b_small_body<R, LL>(d, cs[b], fs[b], par, lds); break;
            BS(16) BS(32) BS(64) BS(128) BS(256) BS(512) BS(1024) BS(2048) BS(4096)
#undef BS
        default: break;
        }
    } else if constexpr (TYPE == BATCH_PASS_A) {
        switch (d.L2) {
#define BA(LL) case LL: b_passA_body<R, LL>(d, cs[b], par, lds); break;
            BA(64) BA(128) BA(256) BA(512) BA(1024)
#undef BA
        default: break;
        }
    } else {
        switch (d.L1) {
#define BB(LL, SS) case LL: b_passB_body<R, LL, SS>(d, fs[b], par, par2, lds); break;
            BB(128, 1) BB(256, 2) BB(512, 3) BB(1024, 5)
#undef BB
        default: break;
        }
    }
}

size_t batch_lds_bytes(int L, int L1, int L2, bool fp32)
{
    const size_t es = fp32 ? 8 : 16;
    if (L2 == 1) {
        const int tpf = L / 16, rc = BNT / tpf;
        return es * ((size_t)rc * fft_pitch(L) + L);
    }
    const size_t a = es * ((size_t)(BNT / (L2 / 16)) * fft_pitch_g(L2, BNT / (L2 / 16)) + L2);
    const size_t b = es * ((size_t)(BNT / (L1 / 16)) * fft_pitch(L1) + L1);
    return a > b ? a : b;
}

int batch_threads() { return BNT; }
int batch_small_chunk() { return BNT * BSLOTS; }
int batch_pass_a_cols(int L2) { return BNT / (L2 / 16); }
int batch_pass_b_points() { return 2048; }

template <typename R>
hipError_t batch_launch(const BatchDesc<R> *descs, const int4 *tasks, int ntasks, BatchCtl *ctl,
                        const cx_t<R> *const *cs, cx_t<R> *const *fs, int grid, size_t lds, int64_t spin_limit,
                        int unreachable, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch<R>, dim3(grid), dim3(BNT), lds, s, descs, tasks, ntasks, ctl, cs, fs, spin_limit,
                       unreachable);
    return hipGetLastError();
}

template <typename R>
hipError_t batch_launch_phased(const BatchDesc<R> *descs, const int4 *tasks, const int *counts,
                               const cx_t<R> *const *cs, cx_t<R> *const *fs, size_t lds, hipStream_t s)
{
    const int4 *t = tasks;
    if (counts[0] > 0)
        hipLaunchKernelGGL((k_batch_phase<R, BATCH_SMALL>), dim3(counts[0]), dim3(BNT), lds, s, descs, t, counts[0],
                           cs, fs);
    t += counts[0];
    if (counts[1] > 0)
        hipLaunchKernelGGL((k_batch_phase<R, BATCH_PASS_A>), dim3(counts[1]), dim3(BNT), lds, s, descs, t,
                           counts[1], cs, fs);
    t += counts[1];
    if (counts[2] > 0)
        hipLaunchKernelGGL((k_batch_phase<R, BATCH_PASS_B>), dim3(counts[2]), dim3(BNT), lds, s, descs, t,
                           counts[2], cs, fs);
    return hipGetLastError();
}

template <typename R>
hipError_t batch_set_lds_limit(size_t lds)
{
    const void *fns[] = {(const void *)k_batch<R>, (const void *)k_batch_phase<R, BATCH_SMALL>,
                         (const void *)k_batch_phase<R, BATCH_PASS_A>, (const void *)k_batch_phase<R, BATCH_PASS_B>};
    for (const void *fn : fns) {
        const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template hipError_t batch_launch<float>(const BatchDesc<float> *, const int4 *, int, BatchCtl *,
                                        const float2 *const *, float2 *const *, int, size_t, int64_t, int,
                                        hipStream_t);
template hipError_t batch_launch<double>(const BatchDesc<double> *, const int4 *, int, BatchCtl *,
                                         const double2 *const *, double2 *const *, int, size_t, int64_t, int,
                                         hipStream_t);
template hipError_t batch_launch_phased<float>(const BatchDesc<float> *, const int4 *, const int *,
                                               const float2 *const *, float2 *const *, size_t, hipStream_t);
template hipError_t batch_launch_phased<double>(const BatchDesc<double> *, const int4 *, const int *,
                                                const double2 *const *, double2 *const *, size_t, hipStream_t);
template hipError_t batch_set_lds_limit<float>(size_t);
template hipError_t batch_set_lds_limit<double>(size_t);

}  // namespace nufft
