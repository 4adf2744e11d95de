// Plan object behind the opaque nufft_plan_t handle.
#pragma once

#include <vector>

#include "kernels.h"

enum PlanKind { PLAN_1D = 1, PLAN_2D = 2, PLAN_BATCH = 3, PLAN_3D = 4 };

struct Profiler {
    struct Rec {
        const char *name;
        hipEvent_t a, b;
    };
    bool on = false;
    std::vector<Rec> pool;   // event pairs, reused across enable/reset
    size_t used = 0;
    ~Profiler();
};

// Bump allocation from a caller-provided device block (the fixed scratch of the
// allocation-free entry point): blocks are 256-byte aligned and never freed one
// by one; the block is reused from the start by the next call.
struct Arena {
    char *base = nullptr;
    size_t cap = 0, used = 0;
};

struct nufft_plan_s {
    int kind = 0;
    Arena *arena = nullptr;         // non-null: alloc() carves from it instead of hipMalloc
    nufft_dtype dtype = NUFFT_C64;
    uint32_t flags = 0;
    int64_t N = 0, M = 0, L = 0;    // modes, samples, FFT grid
    int L1 = 0, L2 = 1;             // L = L1 * L2 (L2 == 1: one-pass)
    double eps = 0, gamma = 0;
    int K = 0;
    Factors<float> facf;
    Factors<double> facd;

    // device buffers (owned)
    int32_t *t = nullptr;           // M grid indices, sample order
    void *X = nullptr;              // M perturbations N(x - s/L), sample order
    void *Xs = nullptr;             // M perturbations, sorted order
    uint32_t *keys = nullptr;       // M sorted keys (t mod L2) * L1 + t / L2
    int32_t *perm = nullptr;        // M sample index per sorted position
    int32_t *off = nullptr;         // L + 1 CSR offsets per key
    int32_t *sinv = nullptr;        // M sorted position per sample (two-pass)
    // destination-bucketed layout of the permutation (large two-pass plans, else null):
    // buckets of 2^bshift samples; bdst[i] place of sorted position i, lidx[p] its
    // sample index within the bucket; bbuf: M values of max(complex, double) size
    int bshift = 0;
    int buckets_off = 0;   // tests: scatter and gather directly
    int32_t *bdst = nullptr;
    uint16_t *lidx = nullptr;
    void *bbuf = nullptr;
    void *gsort = nullptr;          // M complex: sample-ordered input in sorted order (two-pass)
    void *U = nullptr, *W = nullptr, *W2 = nullptr;   // plain path
    void *Y = nullptr;              // K x L two-pass intermediate (fp16 pairs with NUFFT_FLAG_HALF_EXCHANGE)
    int8_t *E = nullptr;            // K x max(L1, L2) block exponents of the half-precision exchange
    void *tw1 = nullptr, *tw2 = nullptr, *hi = nullptr, *lo = nullptr;
    void *tw1i = nullptr, *tw2i = nullptr;   // inverse-sign tables
    // tuning schedule of the two-pass kernels and the twiddle tables of its
    // radix-8-first FFT stage order (FP32 plans with L1, L2 in {1024, 2048})
    int sched = 0;
    void *tw1r8 = nullptr, *tw1ir8 = nullptr, *tw2r8 = nullptr, *tw2ir8 = nullptr;
    void *part = nullptr;           // partial sums of the one-workgroup adjoint
    int64_t part_cap = 0;

    // 2-D plans (Sec. 4): x pairs with k1 < N1 on Gx points, y with k2 < N2 on Gy points
    int64_t N1 = 0, N2 = 0;
    int Gx = 0, Gy = 0, Kx = 0, Ky = 0;
    // S independent 2-D problems of the same shape stacked in one plan (the z
    // slices of a 3-D transform): sample j belongs to problem slice[j] (read at
    // build time only; null: S = 1); inputs and outputs are S arrays back to back
    int S = 1;
    const int32_t *slice = nullptr;
    // 3-D plans: the z axis (n3 modes on Gz points, rank K3, factors, perturbation
    // per sample), the stacked 2-D plan of the z slices (a child), and the
    // Gz x N1 x N2 intermediate, twiddle table and M-sample scratch
    int64_t N3 = 0, Gz = 0;
    int K3 = 0;
    Factors<float> ffz;
    Factors<double> fdz;
    void *Xz = nullptr, *Dz = nullptr, *twz = nullptr, *fsz = nullptr;
    nufft_plan_s *stack = nullptr;
    double gammax = 0, gammay = 0;
    Factors<float> ffx, ffy;
    Factors<double> fdx, fdy;
    void *Xxs = nullptr, *Xys = nullptr;
    int4 *tasks = nullptr;
    int ntasks = 0;
    int4 *atasks = nullptr, *rtasks = nullptr;   // adjoint pass-B' tasks, split columns
    int natasks = 0, nrtasks = 0;
    void *Zp = nullptr;                          // partial rows: split 2-D columns, or dense 1-D adjoint tiles
    void *twx = nullptr, *twxi = nullptr, *twy = nullptr, *twyi = nullptr;

    // batch plans: member plans are the children
    void *bdesc = nullptr, *bfac = nullptr, *btasks = nullptr, *bctl = nullptr;
    void **bcs = nullptr, **bfs = nullptr;          // device arrays of member pointers
    std::vector<const void *> hcs;                   // last uploaded pointers
    std::vector<void *> hfs;
    int bntasks = 0, bgrid = 0;
    int bmode = 0;                  // 0: one persistent launch; 1: three phased launches
    void *btasks3 = nullptr;        // the tasks ordered SMALL, PASS_A, PASS_B (phased mode)
    int bcnt[3] = {0, 0, 0};        // their counts
    size_t blds = 0;

    Profiler prof;
    hipStream_t last = nullptr;     // stream of the latest call on the plan (waited for by nufft_destroy)
    // persistent batch launch: bound of a pass-B wait, and (tests) an unreachable wait target
    int64_t spin_limit = int64_t(1) << 28;
    int wait_unreachable = 0;

    std::vector<void *> blocks;
    std::vector<nufft_plan_s *> children;   // sub-plans (2-D axes, batch members)

    void *alloc(size_t bytes);
    const void *factors() const { return dtype == NUFFT_C64 ? (const void *)&facf : (const void *)&facd; }
    ~nufft_plan_s();
};

namespace nufft {
using Plan = nufft_plan_s;
bool choose_grid(int64_t N, int64_t *L, int *L1, int *L2);
bool grid_split(int64_t L, int *L1, int *L2);
template <typename R> nufft_status build_1d(Plan *p, const double *x, hipStream_t s);
template <typename R> FusedArgs<R> fused_args(const Plan *p);
template <typename R> nufft_status upload_twiddles(Plan *p, hipStream_t s);
}  // namespace nufft
