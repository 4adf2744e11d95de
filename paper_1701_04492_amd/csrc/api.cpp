// C ABI of the MI355X low-rank NUFFT: plans, dispatch, error handling.
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <new>
#include <algorithm>
#include <vector>

#include "factors.h"
#include "kernels.h"
#include "plan.h"
#include "kernels_2d.h"
#include "kernels_3d.h"
#include "solve.h"
#include "batch.h"
#include "noalloc.h"

using namespace nufft;

// Failure injection for tests: >= 0 counts the device allocations left before
// one is refused (then the countdown disarms itself); < 0: none is refused.
static std::atomic<long long> alloc_countdown{-1};

void *nufft_plan_s::alloc(size_t bytes)
{
    long long v = alloc_countdown.load(std::memory_order_relaxed);
    while (v >= 0 && !alloc_countdown.compare_exchange_weak(v, v - 1, std::memory_order_relaxed)) {
    }
    if (v == 0) return nullptr;   // the injected failure
    if (bytes == 0) bytes = 16;
    if (arena) {
        const size_t at = (arena->used + 255) & ~(size_t)255;
        if (at + bytes > arena->cap) return nullptr;
        arena->used = at + bytes;
        return arena->base + at;
    }
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    blocks.push_back(p);
    return p;
}

nufft_plan_s::~nufft_plan_s()
{
    for (void *p : blocks) (void)hipFree(p);
    for (nufft_plan_s *c : children) delete c;
}

Profiler::~Profiler()
{
    for (Rec &r : pool) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
}

void prof_begin(Profiler *p, const char *name, hipStream_t s)
{
    if (!p || !p->on) return;
    if (p->used == p->pool.size()) {
        Profiler::Rec r;
        if (hipEventCreate(&r.a) != hipSuccess) return;
        if (hipEventCreate(&r.b) != hipSuccess) { (void)hipEventDestroy(r.a); return; }
        p->pool.push_back(r);
    }
    p->pool[p->used].name = name;
    (void)hipEventRecord(p->pool[p->used].a, s);
}

void prof_end(Profiler *p, hipStream_t s)
{
    if (!p || !p->on || p->used == p->pool.size()) return;
    (void)hipEventRecord(p->pool[p->used].b, s);
    ++p->used;
}

// ---- autotuning decisions -------------------------------------------------------
// A choice made by timing is remembered per problem class for the life of the
// process (and, when the environment variable NUFFT_MI355X_WISDOM names a file,
// read from and appended to that JSON object), so that later plans of the
// class are not timed again and get the same configuration.
static std::mutex tune_mu;
static std::map<std::string, long long> tune_table;
static bool tune_loaded = false;

static const char *wisdom_path()
{
    const char *p = std::getenv("NUFFT_MI355X_WISDOM");
    return (p && *p) ? p : nullptr;
}

// The file is one JSON object of "key": integer members, as written below.
static void tune_load_locked()
{
    tune_loaded = true;
    const char *path = wisdom_path();
    if (!path) return;
    FILE *fp = std::fopen(path, "r");
    if (!fp) return;
    std::string txt;
    char buf[4096];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof(buf), fp)) > 0) txt.append(buf, n);
    std::fclose(fp);
    size_t i = 0;
    while ((i = txt.find('"', i)) != std::string::npos) {
        const size_t j = txt.find('"', i + 1);
        if (j == std::string::npos) break;
        const std::string key = txt.substr(i + 1, j - i - 1);
        size_t k = txt.find(':', j);
        if (k == std::string::npos) break;
        char *end = nullptr;
        const long long v = std::strtoll(txt.c_str() + k + 1, &end, 10);
        if (end == txt.c_str() + k + 1) break;
        tune_table[key] = v;
        i = (size_t)(end - txt.c_str());
    }
}

static void tune_save_locked()
{
    const char *path = wisdom_path();
    if (!path) return;
    const std::string tmp = std::string(path) + ".tmp";
    FILE *fp = std::fopen(tmp.c_str(), "w");
    if (!fp) return;
    std::fprintf(fp, "{\n");
    size_t i = 0;
    for (const auto &kv : tune_table)
        std::fprintf(fp, "  \"%s\": %lld%s\n", kv.first.c_str(), kv.second, ++i < tune_table.size() ? "," : "");
    std::fprintf(fp, "}\n");
    std::fclose(fp);
    std::rename(tmp.c_str(), path);
}

static bool tune_lookup(const std::string &key, long long *v)
{
    std::lock_guard<std::mutex> g(tune_mu);
    if (!tune_loaded) tune_load_locked();
    auto it = tune_table.find(key);
    if (it == tune_table.end()) return false;
    *v = it->second;
    return true;
}

static void tune_store(const std::string &key, long long v)
{
    std::lock_guard<std::mutex> g(tune_mu);
    if (!tune_loaded) tune_load_locked();
    tune_table[key] = v;
    tune_save_locked();
}

namespace nufft {

// Split of an FFT grid of L points into L1 x L2 (pass B transforms rows of
// L1 points, pass A columns of L2; L = L1 when L2 = 1, the one-pass path).
// A power of two up to 4096 is one pass; a larger one splits near the square
// root (L2 <= 2048, L1 <= 4096).  L = P 2^k (P = 3 or 5, the oversampled grids
// between powers of two) puts P into the columns: L2 = P Q with Q a power of
// two in [64, 512] (P = 3) or [64, 256] (P = 5), L1 a power of two in
// [128, 4096], the most balanced such split.  False: L is not supported.
bool grid_split(int64_t L, int *L1, int *L2)
{
    if (L < 16 || L > (int64_t(1) << 23)) return false;
    const int P = L % 3 == 0 ? 3 : (L % 5 == 0 ? 5 : 1);
    const int64_t r = L / P;
    if (r & (r - 1)) return false;
    if (P == 1) {
        if (L <= 4096) {
            *L1 = (int)L;
            *L2 = 1;
            return true;
        }
        int lg = 0;
        while ((int64_t(1) << lg) < L) ++lg;
        int l2 = 1 << (lg / 2);
        if (l2 > 2048) l2 = 2048;
        *L2 = l2;
        *L1 = (int)(L / l2);
        return *L1 <= 4096;
    }
    int best_q = 0;
    double best = 0.0;
    for (int64_t q = 64; q <= (P == 3 ? 512 : 256); q <<= 1) {
        const int64_t l1 = r / q;
        if (l1 < 128 || l1 > 4096) continue;
        const double imbalance = std::fabs(std::log2((double)l1 / (double)(P * q)));
        if (!best_q || imbalance < best) {
            best_q = (int)q;
            best = imbalance;
        }
    }
    if (!best_q) return false;
    *L2 = P * best_q;
    *L1 = (int)(r / best_q);
    return true;
}

// The default grid (Sec. 2.3, oversampling with N <= L < 2N): the smallest
// power of two >= N and >= 16, and its split.
bool choose_grid(int64_t N, int64_t *L, int *L1, int *L2)
{
    int64_t l = 16;
    while (l < N) l <<= 1;
    *L = l;
    return grid_split(l, L1, L2);
}

template <typename R>
static void fill_factors(Factors<R> &fac, double gamma, int K)
{
    std::memset(&fac, 0, sizeof(fac));
    double mono[NUFFT_KMAX * NUFFT_KMAX];
    u_monomials(gamma, K, mono);
    for (int r = 0; r < K; ++r) {
        const int par = r & 1;
        int n = 0;
        for (int m = par; m < K; m += 2) fac.ucoef[r * NUFFT_UCOEF_STRIDE + n++] = (R)mono[r * K + m];
        fac.nterm[r] = n;
    }
    fac.K = K;
    fac.inv_gamma = gamma > 0 ? (R)(1.0 / gamma) : (R)0;
}

template <typename R>
static nufft_status upload_table(Plan *p, const std::vector<double> &d, void **out, hipStream_t s)
{
    const size_t n = d.size() / 2;
    std::vector<R> h(2 * n);
    for (size_t i = 0; i < 2 * n; ++i) h[i] = (R)d[i];
    void *dev = p->alloc(h.size() * sizeof(R));
    if (!dev) return NUFFT_ERR_ALLOC;
    NUFFT_HIP_CHECK(hipMemcpyAsync(dev, h.data(), h.size() * sizeof(R), hipMemcpyHostToDevice, s));
    NUFFT_HIP_CHECK(hipStreamSynchronize(s));   // host staging buffer goes out of scope
    *out = dev;
    return NUFFT_OK;
}

template <typename R>
nufft_status upload_twiddles(Plan *p, hipStream_t s)
{
    std::vector<double> t1(2 * (size_t)p->L1), t1i(2 * (size_t)p->L1);
    fft_twiddles(p->L1, -1, t1.data());
    fft_twiddles(p->L1, 1, t1i.data());
    nufft_status st = upload_table<R>(p, t1, &p->tw1, s);
    if (st) return st;
    if ((st = upload_table<R>(p, t1i, &p->tw1i, s))) return st;
    if (p->L2 > 1) {
        std::vector<double> t2(2 * (size_t)p->L2), lo(2 * 4096), hi(2 * (size_t)((p->L + 4095) / 4096));
        std::vector<double> t2i(2 * (size_t)p->L2);
        fft_twiddles(p->L2, -1, t2.data());
        fft_twiddles(p->L2, 1, t2i.data());
        if ((st = upload_table<R>(p, t2i, &p->tw2i, s))) return st;
        twiddles(p->L, 4096, 1, -1, lo.data());
        twiddles(p->L, (p->L + 4095) / 4096, 4096, -1, hi.data());
        if ((st = upload_table<R>(p, t2, &p->tw2, s))) return st;
        if ((st = upload_table<R>(p, lo, &p->lo, s))) return st;
        if ((st = upload_table<R>(p, hi, &p->hi, s))) return st;
        if (sizeof(R) == 4 && (p->L1 == 1024 || p->L1 == 2048) && (p->L2 == 1024 || p->L2 == 2048)) {
            // the radix-8-first stage order of the tuning schedule 1
            fft_twiddles(p->L1, -1, t1.data(), 8);
            fft_twiddles(p->L1, 1, t1i.data(), 8);
            fft_twiddles(p->L2, -1, t2.data(), 8);
            fft_twiddles(p->L2, 1, t2i.data(), 8);
            if ((st = upload_table<R>(p, t1, &p->tw1r8, s))) return st;
            if ((st = upload_table<R>(p, t1i, &p->tw1ir8, s))) return st;
            if ((st = upload_table<R>(p, t2, &p->tw2r8, s))) return st;
            if ((st = upload_table<R>(p, t2i, &p->tw2ir8, s))) return st;
        }
    }
    return NUFFT_OK;
}

template nufft_status upload_twiddles<float>(Plan *, hipStream_t);
template nufft_status upload_twiddles<double>(Plan *, hipStream_t);

// Nearest-grid assignment, gamma, K, factors and the sorted sample order for
// one 1-D transform (Sec. 2.2, Sec. 2.3 "Planning the transform").
template <typename R>
nufft_status build_1d(Plan *p, const double *x, hipStream_t s)
{
    const int64_t M = p->M, L = p->L;
    p->t = (int32_t *)p->alloc(M * sizeof(int32_t));
    p->X = p->alloc(M * sizeof(R));
    p->Xs = p->alloc(M * sizeof(R));
    p->keys = (uint32_t *)p->alloc(M * sizeof(uint32_t));
    p->perm = (int32_t *)p->alloc(M * sizeof(int32_t));
    p->off = (int32_t *)p->alloc((L + 1) * sizeof(int32_t));
    uint32_t *keys_u = (uint32_t *)p->alloc(M * sizeof(uint32_t));
    int32_t *iota = (int32_t *)p->alloc(M * sizeof(int32_t));
    int32_t *hist = (int32_t *)p->alloc((L + 1) * sizeof(int32_t));
    const int64_t tmp_n = std::max(radix_tmp_elems(M), scan_tmp_elems(L + 1)) + 16;
    int32_t *tmp = (int32_t *)p->alloc(tmp_n * sizeof(int32_t));
    unsigned long long *dflags = (unsigned long long *)p->alloc(2 * sizeof(unsigned long long));
    if (!p->t || !p->X || !p->Xs || !p->keys || !p->perm || !p->off || !keys_u || !iota || !hist || !tmp ||
        !dflags)
        return NUFFT_ERR_ALLOC;
    NUFFT_HIP_CHECK(hipMemsetAsync(hist, 0, (L + 1) * sizeof(int32_t), s));
    NUFFT_HIP_CHECK(hipMemsetAsync(dflags, 0, 2 * sizeof(unsigned long long), s));
    NUFFT_HIP_CHECK(launch_assign<R>(x, M, L, (double)p->N / (double)L, p->L1, p->L2, p->t, (R *)p->X,
                                     keys_u, hist, dflags, (int *)(dflags + 1), s));
    NUFFT_HIP_CHECK(exclusive_scan(hist, p->off, L + 1, tmp, s));
    NUFFT_HIP_CHECK(launch_iota(iota, M, s));
    int key_bits = 0;
    while ((int64_t(1) << key_bits) < L) ++key_bits;
    uint32_t *ks;
    int32_t *vs;
    NUFFT_HIP_CHECK(radix_sort_pairs(keys_u, iota, p->keys, p->perm, M, key_bits, tmp, s, &ks, &vs));
    if (ks != p->keys) {   // odd number of digit passes: result is in the scratch pair
        NUFFT_HIP_CHECK(hipMemcpyAsync(p->keys, ks, M * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
        NUFFT_HIP_CHECK(hipMemcpyAsync(p->perm, vs, M * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    }
    NUFFT_HIP_CHECK(launch_gather_sorted<R>(p->perm, (const R *)p->X, M, (R *)p->Xs, s));
    unsigned long long hflags[2];
    NUFFT_HIP_CHECK(hipMemcpyAsync(hflags, dflags, sizeof(hflags), hipMemcpyDeviceToHost, s));
    NUFFT_HIP_CHECK(hipStreamSynchronize(s));
    if ((int)hflags[1] != 0) return NUFFT_ERR_NONFINITE;
    double gmax;
    std::memcpy(&gmax, &hflags[0], sizeof(double));
    p->gamma = (p->flags & NUFFT_FLAG_FIX_GAMMA_HALF) ? (double)p->N / (2.0 * (double)L) : gmax;
    if (p->gamma > 0.5) p->gamma = 0.5;
    p->K = choose_rank(p->eps, p->gamma);
    if (p->K < 0) return NUFFT_ERR_UNSUPPORTED;
    if (p->dtype == NUFFT_C64 && p->K > NUFFT_KMAX_F32) return NUFFT_ERR_UNSUPPORTED;   // FP32 rank polynomials
    if (p->dtype == NUFFT_C64) fill_factors(p->facf, p->gamma, p->K);
    else fill_factors(p->facd, p->gamma, p->K);
    nufft_status st = upload_twiddles<R>(p, s);
    if (st) return st;
    const size_t cs = 2 * sizeof(R);
    if (p->flags & NUFFT_FLAG_PLAIN_UNFUSED) {
        p->U = p->alloc((size_t)M * p->K * cs);
        p->W = p->alloc((size_t)p->K * L * cs);
        if (p->L2 > 1) p->W2 = p->alloc((size_t)p->K * L * cs);
        if (!p->U || !p->W || (p->L2 > 1 && !p->W2)) return NUFFT_ERR_ALLOC;
        const Factors<R> &fac = *(const Factors<R> *)p->factors();
        NUFFT_HIP_CHECK(plain_build_U<R>((const R *)p->X, M, fac, (cx_t<R> *)p->U, s));
    }
    if (p->L2 > 1) {
        const bool half = (p->flags & NUFFT_FLAG_HALF_EXCHANGE) != 0;
        p->Y = p->alloc((size_t)p->K * L * (half ? 4 : cs));
        if (half) {
            p->E = (int8_t *)p->alloc((size_t)p->K * std::max(p->L1, p->L2));
            if (!p->E) return NUFFT_ERR_ALLOC;
        }
        const int sp = pass_b_adj_splits(M, p->L2, p->L1, sizeof(R) == 4);
        if (sp > 0) {   // partial rows of the dense-tile adjoint pass B'
            p->Zp = p->alloc((size_t)sp * p->K * L * cs);
            if (!p->Zp) return NUFFT_ERR_ALLOC;
        }
        p->sinv = (int32_t *)p->alloc((size_t)M * sizeof(int32_t));
        p->gsort = p->alloc((size_t)M * cs);
        if (!p->Y || !p->sinv || !p->gsort) return NUFFT_ERR_ALLOC;
        NUFFT_HIP_CHECK(launch_invert_perm(p->perm, M, p->sinv, s));
        // Destination buckets for the permutations between sample order and sorted
        // order (large plans): about 256 blocks (one per CU for the layout passes)
        // of 2^12 to 2^14 samples (at most 2^13 in FP64), 16 to 1024 of them.
        int bshift = 12;
        while (bshift < (sizeof(R) == 4 ? 14 : 13) && (M >> bshift) > 256) ++bshift;
        const int64_t nbk = (M + (int64_t(1) << bshift) - 1) >> bshift;
        if (nbk >= 16 && nbk <= 1024) {
            p->bshift = bshift;
            p->bdst = (int32_t *)p->alloc((size_t)M * sizeof(int32_t));
            p->lidx = (uint16_t *)p->alloc((size_t)M * sizeof(uint16_t));
            p->bbuf = p->alloc((size_t)M * std::max<size_t>(cs, sizeof(double)));
            if (!p->bdst || !p->lidx || !p->bbuf) return NUFFT_ERR_ALLOC;
            // scratch: keys_u and iota, with the bucket buffer as the alternate pair
            uint32_t *kalt = (uint32_t *)p->bbuf;
            int32_t *valt = (int32_t *)p->bbuf + M;
            NUFFT_HIP_CHECK(launch_bucket_maps(p->perm, M, bshift, keys_u, iota, kalt, valt, tmp, p->bdst, p->lidx, s));
        }
    } else {
        int64_t nparts = (M + 65535) / 65536;
        if (nparts > 64) nparts = 64;
        if (nparts > 1) {
            p->part_cap = nparts * p->N;
            p->part = p->alloc((size_t)p->part_cap * cs);
            if (!p->part) return NUFFT_ERR_ALLOC;
        }
    }
    NUFFT_HIP_CHECK(hipStreamSynchronize(s));
    return NUFFT_OK;
}

template nufft_status build_1d<float>(Plan *, const double *, hipStream_t);
template nufft_status build_1d<double>(Plan *, const double *, hipStream_t);

template <typename R>
FusedArgs<R> fused_args(const Plan *p)
{
    FusedArgs<R> a;
    a.N = p->N;
    a.L = p->L;
    a.M = p->M;
    a.L1 = p->L1;
    a.L2 = p->L2;
    a.fac = *(const Factors<R> *)p->factors();
    a.keys = p->keys;
    a.perm = p->perm;
    a.Xs = (const R *)p->Xs;
    a.off = p->off;
    a.sinv = p->sinv;
    a.gsort = (cx_t<R> *)p->gsort;
    a.presorted = 0;
    a.t = p->t;
    a.X = (const R *)p->X;
    a.Y = (cx_t<R> *)p->Y;
    a.Zp = (cx_t<R> *)p->Zp;
    a.half = sizeof(R) == 4 && (p->flags & NUFFT_FLAG_HALF_EXCHANGE) && p->L2 > 1;
    a.E = p->E;
    a.tw1 = (const cx_t<R> *)p->tw1;
    a.tw1i = (const cx_t<R> *)p->tw1i;
    a.tw2i = (const cx_t<R> *)p->tw2i;
    a.tw2 = (const cx_t<R> *)p->tw2;
    a.hi = (const cx_t<R> *)p->hi;
    a.lo = (const cx_t<R> *)p->lo;
    a.part = (cx_t<R> *)p->part;
    a.part_cap = p->part_cap;
    a.bshift = p->bshift;
    a.bdst = p->buckets_off ? nullptr : p->bdst;
    a.lidx = p->lidx;
    a.bbuf = p->bbuf;
    a.sched = p->tw1r8 ? p->sched : 0;
    a.tw1r8 = (const cx_t<R> *)p->tw1r8;
    a.tw1ir8 = (const cx_t<R> *)p->tw1ir8;
    a.tw2r8 = (const cx_t<R> *)p->tw2r8;
    a.tw2ir8 = (const cx_t<R> *)p->tw2ir8;
    a.prof = const_cast<Profiler *>(&p->prof);
    return a;
}

template FusedArgs<float> fused_args<float>(const Plan *);
template FusedArgs<double> fused_args<double>(const Plan *);

template <typename R>
static hipError_t exec_type2(const Plan *p, const void *c, void *f, int mode, const void *g, double *gx,
                             hipStream_t s)
{
    using C = cx_t<R>;
    if (p->flags & NUFFT_FLAG_PLAIN_UNFUSED) {
        PlainArgs<R> a;
        a.c = (const C *)c;
        a.N = p->N;
        a.L = p->L;
        a.M = p->M;
        a.L1 = p->L1;
        a.L2 = p->L2;
        a.K = p->K;
        a.mode = mode;
        a.W = (C *)p->W;
        a.W2 = (C *)p->W2;
        a.tw1 = (const C *)p->tw1;
        a.tw2 = (const C *)p->tw2;
        a.hi = (const C *)p->hi;
        a.lo = (const C *)p->lo;
        a.U = (const C *)p->U;
        a.t = p->t;
        a.f = (C *)f;
        a.g = (const C *)g;
        a.gx = gx;
        a.prof = const_cast<Profiler *>(&p->prof);
        return plain_exec<R>(a, s);
    }
    return fused_type2<R>(fused_args<R>(p), (const C *)c, (C *)f, mode, (const C *)g, gx, s);
}

// Type I (sign -1) / adjoint (sign +1) on a 1-D plan: the plain unfused kernels
// on a NUFFT_FLAG_PLAIN_UNFUSED plan, the fused ones otherwise.
template <typename R>
static hipError_t exec_type1(const Plan *p, const void *c, void *f, int sign, hipStream_t s)
{
    using C = cx_t<R>;
    if (p->flags & NUFFT_FLAG_PLAIN_UNFUSED) {
        PlainT1Args<R> a;
        a.c = (const C *)c;
        a.N = p->N;
        a.L = p->L;
        a.M = p->M;
        a.L1 = p->L1;
        a.L2 = p->L2;
        a.K = p->K;
        a.perm = p->perm;
        a.off = p->off;
        a.U = (const C *)p->U;
        a.W = (C *)p->W;
        a.W2 = (C *)p->W2;
        a.tw1 = (const C *)p->tw1;
        a.tw2 = (const C *)p->tw2;
        a.hi = (const C *)p->hi;
        a.lo = (const C *)p->lo;
        a.f = (C *)f;
        a.prof = const_cast<Profiler *>(&p->prof);
        return plain_type1<R>(a, sign, s);
    }
    return fused_type1<R>(fused_args<R>(p), (const C *)c, (C *)f, sign, s);
}

template <typename R>
static nufft_status exec_backward(const Plan *p, const void *c, const void *g, void *gc, double *gx, hipStream_t s)
{
    using C = cx_t<R>;
    FusedArgs<R> a = fused_args<R>(p);
    const bool share = !(p->flags & NUFFT_FLAG_PLAIN_UNFUSED) && p->L2 > 1 && gc && gx;
    if (share) {
        NUFFT_HIP_CHECK(fused_sort_input<R>(a, (const C *)g, "bwd_sort", s));
        a.presorted = 1;
    }
    if (gc) {
        if (share) NUFFT_HIP_CHECK(fused_type1<R>(a, (const C *)g, (C *)gc, +1, s));
        else NUFFT_HIP_CHECK(exec_type1<R>(p, g, gc, +1, s));
    }
    if (gx) {
        if (share) NUFFT_HIP_CHECK(fused_type2<R>(a, (const C *)c, nullptr, 1, (const C *)g, gx, s));
        else NUFFT_HIP_CHECK(exec_type2<R>(p, c, nullptr, 1, g, gx, s));
    }
    return NUFFT_OK;
}


// ---- type III (Sec. 3.2) ---------------------------------------------------

hipError_t t3_assign(const double *x, int64_t M, int64_t N, int32_t *t, double *d, int32_t *wrap,
                     unsigned long long *gbits, int *flags, hipStream_t s);
hipError_t t3_freq(const double *w, int64_t N, double *xs, int *flags, hipStream_t s);
template <typename R>
hipError_t t3_scale(const cx_t<R> *c, const double *w, int64_t N, int r, int with_wrap, cx_t<R> *c1, cx_t<R> *c2,
                    hipStream_t s);
template <typename R>
hipError_t t3_accum(const double *d, const int32_t *t, const int32_t *wrap, int64_t M, const Factors<double> &fac,
                    int r, const cx_t<R> *y, const cx_t<R> *y2, cx_t<R> *f, hipStream_t s);
hipError_t t3d_assign(const double *x, const double *y, int64_t M, int64_t n1, int64_t n2, int32_t *sx, int32_t *sy,
                      double *dx, double *dy, unsigned long long *gbits, int *flags, hipStream_t s);
hipError_t t3d_freq(const double *w1, const double *w2, int64_t Q, int64_t n1, int64_t n2, double *xs, double *ys,
                    int *flags, hipStream_t s);
template <typename R>
hipError_t t3d_scale(const cx_t<R> *c, const double *w1, const double *w2, int64_t Q, int64_t n1, int64_t n2, int r1,
                     int r2, cx_t<R> *c1, hipStream_t s);
template <typename R>
hipError_t t3d_accum(const double *dx, const double *dy, const int32_t *sx, const int32_t *sy, int64_t M,
                     const Factors<double> &fx, const Factors<double> &fy, int r1, int r2, const cx_t<R> *F,
                     int64_t ld, int first, cx_t<R> *f, hipStream_t s);

// FP64 factors u_r of the type-III expansion (monomial form of Sec. 2.1.2) and
// sum_{p,r} w_p |b_pr|, the bound on sum_r |u_r| that weighs the inner errors.
static void t3_factors(double gamma, int K, Factors<double> &fac, double *su_out)
{
    std::memset(&fac, 0, sizeof(fac));
    double mono[NUFFT_KMAX * NUFFT_KMAX];
    u_monomials(gamma, K, mono);
    for (int r = 0; r < K; ++r) {
        int n = 0;
        for (int m = (r & 1); m < K; m += 2) fac.ucoef[r * NUFFT_UCOEF_STRIDE + n++] = mono[r * K + m];
        fac.nterm[r] = n;
    }
    fac.K = K;
    fac.inv_gamma = gamma > 0 ? 1.0 / gamma : 0.0;
    double b[NUFFT_KMAX * NUFFT_KMAX], su = 0.0;
    bessel_b(gamma, K, b);
    for (int p = 0; p < K; ++p)
        for (int r = 0; r < K; ++r) su += (p == 0 ? 0.5 : 1.0) * std::fabs(b[p * K + r]);
    *su_out = su;
}

// arena non-null: every temporary (and the inner plan's buffers) comes from it.
template <typename R>
static nufft_status type3(int64_t M, const double *x, int64_t N, const double *w, const void *c, void *f,
                          double eps, nufft_dtype dt, hipStream_t s, Arena *arena = nullptr)
{
    using C = cx_t<R>;
    Plan tmp;   // owns the temporaries
    tmp.arena = arena;
    Plan inner_plan;   // the inner type-I plan (its buffers are released with it)
    inner_plan.arena = arena;
    struct SyncGuard {   // destroyed before tmp: no temporary is freed under a running kernel
        hipStream_t s;
        ~SyncGuard() { (void)hipStreamSynchronize(s); }
    } guard{s};
    int32_t *t = (int32_t *)tmp.alloc(M * sizeof(int32_t));
    int32_t *wrap = (int32_t *)tmp.alloc(M * sizeof(int32_t));
    double *d = (double *)tmp.alloc(M * sizeof(double));
    double *xs = (double *)tmp.alloc(N * sizeof(double));
    unsigned long long *flags = (unsigned long long *)tmp.alloc(2 * sizeof(unsigned long long));
    C *c1 = (C *)tmp.alloc(N * sizeof(C));
    C *c2 = (C *)tmp.alloc(N * sizeof(C));
    C *y = (C *)tmp.alloc(N * sizeof(C));
    C *y2 = (C *)tmp.alloc(N * sizeof(C));
    if (!t || !wrap || !d || !xs || !flags || !c1 || !c2 || !y || !y2) return NUFFT_ERR_ALLOC;
    NUFFT_HIP_CHECK(hipMemsetAsync(flags, 0, 2 * sizeof(unsigned long long), s));
    NUFFT_HIP_CHECK(t3_assign(x, M, N, t, d, wrap, flags, (int *)(flags + 1), s));
    NUFFT_HIP_CHECK(t3_freq(w, N, xs, (int *)(flags + 1), s));
    unsigned long long h[2];
    NUFFT_HIP_CHECK(hipMemcpyAsync(h, flags, sizeof(h), hipMemcpyDeviceToHost, s));
    NUFFT_HIP_CHECK(hipStreamSynchronize(s));
    const int bad = (int)h[1];
    if (bad & 5) return NUFFT_ERR_INVALID_ARG;   // x outside [0,1) / w outside [0,N) or not finite
    const int any_wrap = (bad & 2) ? 1 : 0;
    double gamma;
    std::memcpy(&gamma, &h[0], sizeof(double));
    if (gamma > 0.5) gamma = 0.5;
    // half of eps for the factorisation of A, half for the inner type-I transforms,
    // whose errors are weighted by sum_r |u_r| <= sum_r sum'_p |b_pr|
    const int K = choose_rank(eps / 2.0, gamma);
    if (K < 0) return NUFFT_ERR_UNSUPPORTED;
    Factors<double> fac;
    double su;
    t3_factors(gamma, K, fac, &su);
    // the inner transforms work at eps_i >= the precision floor; the composed
    // bound eps/2 + su eps_i must stay within 4 eps
    const double floor_eps = dt == NUFFT_C64 ? 1e-7 : 1e-15;
    const double sw = su > 1.0 ? su : 1.0;
    double eps_i = eps / (2.0 * sw);
    if (eps_i < floor_eps) eps_i = floor_eps;
    if (eps / 2.0 + sw * eps_i > 4.0 * eps) return NUFFT_ERR_UNSUPPORTED;
    // inner type-I plan on the samples w/N with N modes
    Plan *inner = &inner_plan;
    inner->kind = PLAN_1D;
    inner->dtype = dt;
    inner->N = N;
    inner->M = N;
    inner->eps = eps_i;
    if (!choose_grid(N, &inner->L, &inner->L1, &inner->L2)) return NUFFT_ERR_UNSUPPORTED;
    nufft_status st = build_1d<R>(inner, xs, s);
    if (st) return st;
    const FusedArgs<R> ia = fused_args<R>(inner);
    for (int r = 0; r < K; ++r) {
        NUFFT_HIP_CHECK(t3_scale<R>((const C *)c, w, N, r, any_wrap, c1, c2, s));
        NUFFT_HIP_CHECK(fused_type1<R>(ia, c1, y, -1, s));
        if (any_wrap) NUFFT_HIP_CHECK(fused_type1<R>(ia, c2, y2, -1, s));
        NUFFT_HIP_CHECK(t3_accum<R>(d, t, wrap, M, fac, r, y, any_wrap ? y2 : nullptr, (C *)f, s));
    }
    return NUFFT_OK;
}

// ---- inverse type II and type I (Sec. 3.3) -----------------------------------------

// Type II (T1 = false): conjugate gradients on F2^* F2 c = F2^* f.  F2^* F2 is
// Hermitian Toeplitz with first column tau = F2^* 1; its product with a vector
// is a circulant product of size Lc >= 2N (two DFTs and a pointwise product
// with the circulant's eigenvalues lam = DFT(column)).
// Type I (T1 = true), F1 = F2^T: c = F1^* y with F1 F1^* y = f.  F1 F1^* =
// conj(F2^* F2) is Hermitian Toeplitz with first column conj(tau); CG runs on
// it with the same circulant product, and c = conj(F2 conj(y)) is one type-II
// transform.  The loop runs on the host: two FP64 dot products are read back
// per iteration.
template <typename R, bool T1>
static nufft_status solve_impl(Plan *p, const void *f, void *c, double tol, int max_iter, int *iters_out,
                               double *resid_out, hipStream_t s)
{
    using C = cx_t<R>;
    const int64_t N = p->N, M = p->M;
    int64_t Lc = 16;
    while (Lc < 2 * N) Lc <<= 1;
    Plan tmp;   // owns the temporaries
    struct SyncGuard {   // destroyed before tmp: no temporary is freed under a running kernel
        hipStream_t s;
        ~SyncGuard() { (void)hipStreamSynchronize(s); }
    } guard{s};
    Plan *circ = new (std::nothrow) Plan();
    if (!circ) return NUFFT_ERR_ALLOC;
    tmp.children.push_back(circ);
    circ->dtype = p->dtype;
    circ->N = Lc;
    if (!choose_grid(Lc, &circ->L, &circ->L1, &circ->L2)) return NUFFT_ERR_UNSUPPORTED;
    nufft_status st = upload_twiddles<R>(circ, s);
    if (st) return st;
    C *ones = (C *)tmp.alloc(M * sizeof(C));
    C *tau = (C *)tmp.alloc(N * sizeof(C));
    C *b = (C *)tmp.alloc(N * sizeof(C));
    C *r = (C *)tmp.alloc(N * sizeof(C));
    C *pv = (C *)tmp.alloc(N * sizeof(C));
    C *ap = (C *)tmp.alloc(N * sizeof(C));
    C *lam1 = (C *)tmp.alloc(Lc * sizeof(C));
    C *lam2 = (C *)tmp.alloc(Lc * sizeof(C));
    C *q1 = (C *)tmp.alloc(Lc * sizeof(C));
    C *q2 = (C *)tmp.alloc(Lc * sizeof(C));
    double2 *part = (double2 *)tmp.alloc(SOLVE_DOT_BLOCKS * sizeof(double2));
    double2 *dd = (double2 *)tmp.alloc(sizeof(double2));
    if (!ones || !tau || !b || !r || !pv || !ap || !lam1 || !lam2 || !q1 || !q2 || !part || !dd)
        return NUFFT_ERR_ALLOC;
    const C *tw1 = (const C *)circ->tw1, *tw2 = (const C *)circ->tw2;
    const C *hi = (const C *)circ->hi, *lo = (const C *)circ->lo;
    auto dot = [&](const C *u, const C *v, double *re) -> nufft_status {
        NUFFT_HIP_CHECK(solve_dot<R>(u, v, N, part, dd, s));
        double2 h;
        NUFFT_HIP_CHECK(hipMemcpyAsync(&h, dd, sizeof(h), hipMemcpyDeviceToHost, s));
        NUFFT_HIP_CHECK(hipStreamSynchronize(s));
        *re = h.x;
        return NUFFT_OK;
    };
    // eigenvalues of the circulant embedding
    NUFFT_HIP_CHECK(solve_fill<R>(ones, M, 1.0, 0.0, s));
    NUFFT_HIP_CHECK(exec_type1<R>(p, ones, tau, +1, s));
    if (T1) {   // first column of conj(F2^* F2)
        NUFFT_HIP_CHECK(solve_take_conj<R>(tau, N, ap, s));
        NUFFT_HIP_CHECK(solve_circulant_column<R>(ap, N, Lc, lam1, s));
    } else {
        NUFFT_HIP_CHECK(solve_circulant_column<R>(tau, N, Lc, lam1, s));
    }
    C *lam;
    NUFFT_HIP_CHECK(plain_fft<R>(Lc, circ->L1, circ->L2, lam1, lam2, tw1, tw2, hi, lo, &lam, s));
    // right-hand side (F2^* f, or f itself for the type I) and the CG
    // iteration from zero; x is c itself for the type II, y (in b) for the type I
    const C *rhs = (const C *)f;
    if (!T1) {
        NUFFT_HIP_CHECK(exec_type1<R>(p, f, b, +1, s));
        rhs = b;
    }
    C *x = T1 ? b : (C *)c;
    NUFFT_HIP_CHECK(solve_fill<R>(x, N, 0.0, 0.0, s));
    NUFFT_HIP_CHECK(hipMemcpyAsync(r, rhs, N * sizeof(C), hipMemcpyDeviceToDevice, s));
    NUFFT_HIP_CHECK(hipMemcpyAsync(pv, rhs, N * sizeof(C), hipMemcpyDeviceToDevice, s));
    double rs;
    if ((st = dot(r, r, &rs))) return st;
    const double bn = std::sqrt(rs);
    int it = 0;
    while (bn > 0.0 && it < max_iter && std::sqrt(rs) > tol * bn) {
        // ap = (F2^* F2) pv = first N of conj(DFT(conj(lam o DFT([pv, 0])) / Lc))
        C *res1, *res2;
        NUFFT_HIP_CHECK(solve_pad<R>(pv, N, Lc, q1, s));
        NUFFT_HIP_CHECK(plain_fft<R>(Lc, circ->L1, circ->L2, q1, q2, tw1, tw2, hi, lo, &res1, s));
        NUFFT_HIP_CHECK(solve_circulant_scale<R>(res1, lam, Lc, s));
        NUFFT_HIP_CHECK(plain_fft<R>(Lc, circ->L1, circ->L2, res1, res1 == q1 ? q2 : q1, tw1, tw2, hi, lo,
                                     &res2, s));
        NUFFT_HIP_CHECK(solve_take_conj<R>(res2, N, ap, s));
        double pap;
        if ((st = dot(pv, ap, &pap))) return st;
        if (!(pap > 0.0)) break;   // breakdown: the normal matrix is singular on this direction
        const double alpha = rs / pap;
        NUFFT_HIP_CHECK(solve_step<R>(x, r, pv, ap, alpha, N, s));
        double rs_new;
        if ((st = dot(r, r, &rs_new))) return st;
        NUFFT_HIP_CHECK(solve_direction<R>(pv, r, rs_new / rs, N, s));
        rs = rs_new;
        ++it;
    }
    if (T1) {   // c = F1^* y = conj(F2 conj(y)); r and ones are free here
        NUFFT_HIP_CHECK(solve_take_conj<R>(x, N, r, s));
        NUFFT_HIP_CHECK(exec_type2<R>(p, r, ones, 0, nullptr, nullptr, s));
        NUFFT_HIP_CHECK(solve_take_conj<R>(ones, M, (C *)c, s));
    }
    if (iters_out) *iters_out = it;
    if (resid_out) *resid_out = bn > 0.0 ? std::sqrt(rs) / bn : 0.0;
    return NUFFT_OK;
}

// ---- 2-D type II (Sec. 4) -------------------------------------------------------

template <typename R>
static void fill_factors_2d(Factors<R> &fac, double gamma, int K) { fill_factors(fac, gamma, K); }

template <typename R>
nufft_status build_2d(Plan *p, const double *x, const double *y, hipStream_t s)
{
    const int64_t M = p->M;
    const int64_t cols = (int64_t)p->S * p->Gy;   // pass-B columns over the stacked problems
    const int64_t G2 = cols * p->Gx;              // grid points, the key range
    if (G2 > (int64_t(1) << 28)) return NUFFT_ERR_UNSUPPORTED;
    R *Xx = (R *)p->alloc(M * sizeof(R));
    R *Xy = (R *)p->alloc(M * sizeof(R));
    p->Xxs = p->alloc(M * sizeof(R));
    p->Xys = p->alloc(M * sizeof(R));
    uint32_t *keys_u = (uint32_t *)p->alloc(M * sizeof(uint32_t));
    int32_t *iota = (int32_t *)p->alloc(M * sizeof(int32_t));
    p->keys = (uint32_t *)p->alloc(M * sizeof(uint32_t));
    p->perm = (int32_t *)p->alloc(M * sizeof(int32_t));
    int32_t *hist = (int32_t *)p->alloc((G2 + 1) * sizeof(int32_t));
    p->off = (int32_t *)p->alloc((G2 + 1) * sizeof(int32_t));
    const int64_t tmp_n = std::max(radix_tmp_elems(M), scan_tmp_elems(G2 + 1)) + 16;
    int32_t *tmp = (int32_t *)p->alloc(tmp_n * sizeof(int32_t));
    unsigned long long *dflags = (unsigned long long *)p->alloc(3 * sizeof(unsigned long long));
    if (!Xx || !Xy || !p->Xxs || !p->Xys || !keys_u || !iota || !p->keys || !p->perm || !hist || !p->off || !tmp ||
        !dflags)
        return NUFFT_ERR_ALLOC;
    NUFFT_HIP_CHECK(hipMemsetAsync(hist, 0, (G2 + 1) * sizeof(int32_t), s));
    NUFFT_HIP_CHECK(hipMemsetAsync(dflags, 0, 3 * sizeof(unsigned long long), s));
    NUFFT_HIP_CHECK(launch_assign2d<R>(x, y, p->slice, M, p->Gx, p->Gy, (double)p->N1 / p->Gx,
                                       (double)p->N2 / p->Gy, Xx, Xy, keys_u, hist, dflags, (int *)(dflags + 2), s));
    NUFFT_HIP_CHECK(exclusive_scan(hist, p->off, G2 + 1, tmp, s));
    NUFFT_HIP_CHECK(launch_iota(iota, M, s));
    int key_bits = 0;
    while ((int64_t(1) << key_bits) < G2) ++key_bits;
    uint32_t *ks;
    int32_t *vs;
    NUFFT_HIP_CHECK(radix_sort_pairs(keys_u, iota, p->keys, p->perm, M, key_bits, tmp, s, &ks, &vs));
    if (ks != p->keys) {
        NUFFT_HIP_CHECK(hipMemcpyAsync(p->keys, ks, M * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
        NUFFT_HIP_CHECK(hipMemcpyAsync(p->perm, vs, M * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    }
    NUFFT_HIP_CHECK(launch_gather_sorted<R>(p->perm, Xx, M, (R *)p->Xxs, s));
    NUFFT_HIP_CHECK(launch_gather_sorted<R>(p->perm, Xy, M, (R *)p->Xys, s));
    unsigned long long h[3];
    std::vector<int32_t> toff((size_t)cols + 1);
    NUFFT_HIP_CHECK(hipMemcpyAsync(h, dflags, sizeof(h), hipMemcpyDeviceToHost, s));
    // column starts off[n2 * Gx], n2 <= cols: gathered on the device, one copy
    // (into hist: G2 + 1 >= cols + 1 entries, unused after the scan)
    NUFFT_HIP_CHECK(launch_strided_i32(p->off, p->Gx, cols + 1, hist, s));
    NUFFT_HIP_CHECK(hipMemcpyAsync(toff.data(), hist, ((size_t)cols + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    NUFFT_HIP_CHECK(hipStreamSynchronize(s));
    if ((int)h[2] != 0) return NUFFT_ERR_NONFINITE;
    double gx, gy;
    std::memcpy(&gx, &h[0], sizeof(double));
    std::memcpy(&gy, &h[1], sizeof(double));
    if (p->flags & NUFFT_FLAG_FIX_GAMMA_HALF) {
        gx = (double)p->N1 / (2.0 * p->Gx);
        gy = (double)p->N2 / (2.0 * p->Gy);
    }
    p->gammax = gx > 0.5 ? 0.5 : gx;
    p->gammay = gy > 0.5 ? 0.5 : gy;
    // |A^x A^y - A^x_K A^y_K| <= eps_x + eps_y + eps_x eps_y: half of eps per axis
    p->Kx = choose_rank(p->eps / 2.0, p->gammax);
    p->Ky = choose_rank(p->eps / 2.0, p->gammay);
    if (p->Kx < 0 || p->Ky < 0) return NUFFT_ERR_UNSUPPORTED;
    if (p->dtype == NUFFT_C64 && (p->Kx > NUFFT_KMAX_F32 || p->Ky > NUFFT_KMAX_F32)) return NUFFT_ERR_UNSUPPORTED;
    p->K = p->Kx;
    p->gamma = p->gammax;
    if (p->dtype == NUFFT_C64) {
        fill_factors(p->ffx, p->gammax, p->Kx);
        fill_factors(p->ffy, p->gammay, p->Ky);
    } else {
        fill_factors(p->fdx, p->gammax, p->Kx);
        fill_factors(p->fdy, p->gammay, p->Ky);
    }
    std::vector<double> t(2 * (size_t)std::max(p->Gx, p->Gy));
    nufft_status st;
    fft_twiddles(p->Gx, -1, t.data());
    if ((st = upload_table<R>(p, std::vector<double>(t.begin(), t.begin() + 2 * p->Gx), &p->twx, s))) return st;
    fft_twiddles(p->Gx, 1, t.data());
    if ((st = upload_table<R>(p, std::vector<double>(t.begin(), t.begin() + 2 * p->Gx), &p->twxi, s))) return st;
    fft_twiddles(p->Gy, -1, t.data());
    if ((st = upload_table<R>(p, std::vector<double>(t.begin(), t.begin() + 2 * p->Gy), &p->twy, s))) return st;
    fft_twiddles(p->Gy, 1, t.data());
    if ((st = upload_table<R>(p, std::vector<double>(t.begin(), t.begin() + 2 * p->Gy), &p->twyi, s))) return st;
    // forward pass-B tasks: each column n2 split into sample ranges of at most cap
    const int cap = pass_b2d_cap(p->Gx, p->dtype == NUFFT_C64);
    if (cap <= 0) return NUFFT_ERR_UNSUPPORTED;
    std::vector<int4> tk;
    for (int n2 = 0; n2 < cols; ++n2)
        for (int a = toff[n2]; a < toff[n2 + 1]; a += cap) {
            int4 v;
            v.x = n2;
            v.y = a;
            v.z = std::min(a + cap, toff[n2 + 1]);
            v.w = 0;
            tk.push_back(v);
        }
    p->ntasks = (int)tk.size();
    p->tasks = (int4 *)p->alloc(std::max<size_t>(1, tk.size()) * sizeof(int4));
    if (!p->tasks) return NUFFT_ERR_ALLOC;
    if (!tk.empty()) {
        NUFFT_HIP_CHECK(hipMemcpyAsync(p->tasks, tk.data(), tk.size() * sizeof(int4), hipMemcpyHostToDevice, s));
        NUFFT_HIP_CHECK(hipStreamSynchronize(s));
    }
    // adjoint pass-B' tasks: a column whose samples exceed the LDS staging of one
    // workgroup is split into slices that write partial rows (summed in order)
    const int acap = pass_b2d_adj_cap(p->Gx, p->dtype == NUFFT_C64);
    if (acap <= 0) return NUFFT_ERR_UNSUPPORTED;
    std::vector<int4> at, rt;
    int nslots = 0;
    for (int n2 = 0; n2 < cols; ++n2) {
        const int a0 = toff[n2], a1 = toff[n2 + 1];
        if (a1 - a0 <= acap) {
            at.push_back(make_int4(n2, a0, a1, -1));   // also empty columns: their rows are zero
            continue;
        }
        const int parts = (a1 - a0 + acap - 1) / acap;
        rt.push_back(make_int4(n2, nslots, parts, 0));
        for (int q = 0; q < parts; ++q) {
            const int b0 = a0 + (int)((int64_t)(a1 - a0) * q / parts);
            const int b1 = a0 + (int)((int64_t)(a1 - a0) * (q + 1) / parts);
            at.push_back(make_int4(n2, b0, b1, nslots++));
        }
    }
    p->natasks = (int)at.size();
    p->nrtasks = (int)rt.size();
    p->atasks = (int4 *)p->alloc(at.size() * sizeof(int4));
    p->rtasks = (int4 *)p->alloc(std::max<size_t>(1, rt.size()) * sizeof(int4));
    if (!p->atasks || !p->rtasks) return NUFFT_ERR_ALLOC;
    if (nslots > 0) {
        p->Zp = p->alloc((size_t)nslots * p->Ky * p->Gx * 2 * sizeof(R));
        if (!p->Zp) return NUFFT_ERR_ALLOC;
    }
    NUFFT_HIP_CHECK(hipMemcpyAsync(p->atasks, at.data(), at.size() * sizeof(int4), hipMemcpyHostToDevice, s));
    if (!rt.empty())
        NUFFT_HIP_CHECK(hipMemcpyAsync(p->rtasks, rt.data(), rt.size() * sizeof(int4), hipMemcpyHostToDevice, s));
    NUFFT_HIP_CHECK(hipStreamSynchronize(s));   // the host task tables go out of scope
    p->Y = p->alloc((size_t)p->Ky * G2 * 2 * sizeof(R));
    if (!p->Y) return NUFFT_ERR_ALLOC;
    return NUFFT_OK;
}

template <typename R>
static Args2D<R> args_2d(const Plan *p)
{
    Args2D<R> a;
    a.N1 = p->N1;
    a.N2 = p->N2;
    a.M = p->M;
    a.Gx = p->Gx;
    a.Gy = p->Gy;
    a.S = p->S;
    if constexpr (sizeof(R) == 4) {
        a.fx = p->ffx;
        a.fy = p->ffy;
    } else {
        a.fx = p->fdx;
        a.fy = p->fdy;
    }
    a.keys = p->keys;
    a.perm = p->perm;
    a.Xxs = (const R *)p->Xxs;
    a.Xys = (const R *)p->Xys;
    a.off = p->off;
    a.tasks = p->tasks;
    a.ntasks = p->ntasks;
    a.atasks = p->atasks;
    a.natasks = p->natasks;
    a.rtasks = p->rtasks;
    a.nrtasks = p->nrtasks;
    a.Zp = (cx_t<R> *)p->Zp;
    a.H = (cx_t<R> *)p->Y;
    a.twx = (const cx_t<R> *)p->twx;
    a.twxi = (const cx_t<R> *)p->twxi;
    a.twy = (const cx_t<R> *)p->twy;
    a.twyi = (const cx_t<R> *)p->twyi;
    a.prof = const_cast<Profiler *>(&p->prof);
    return a;
}

// ---- batches in one persistent launch ------------------------------------------

template <typename R>
static nufft_status batch_upload_ptrs(Plan *p, const void *const *cs, void *const *fs, hipStream_t s)
{
    const size_t B = p->children.size();
    bool same = p->hcs.size() == B;
    for (size_t b = 0; same && b < B; ++b) same = p->hcs[b] == cs[b] && p->hfs[b] == fs[b];
    if (same) return NUFFT_OK;
    p->hcs.assign(cs, cs + B);
    p->hfs.assign(fs, fs + B);
    NUFFT_HIP_CHECK(hipMemcpyAsync(p->bcs, p->hcs.data(), B * sizeof(void *), hipMemcpyHostToDevice, s));
    NUFFT_HIP_CHECK(hipMemcpyAsync(p->bfs, p->hfs.data(), B * sizeof(void *), hipMemcpyHostToDevice, s));
    NUFFT_HIP_CHECK(hipStreamSynchronize(s));
    return NUFFT_OK;
}

template <typename R>
static hipError_t batch_run(const Plan *p, int mode, int grid, hipStream_t s)
{
    if (mode == 1)
        return batch_launch_phased<R>((const BatchDesc<R> *)p->bdesc, (const int4 *)p->btasks3, p->bcnt,
                                      (const cx_t<R> *const *)p->bcs, (cx_t<R> *const *)p->bfs, p->blds, s);
    return batch_launch<R>((const BatchDesc<R> *)p->bdesc, (const int4 *)p->btasks, p->bntasks, (BatchCtl *)p->bctl,
                           (const cx_t<R> *const *)p->bcs, (cx_t<R> *const *)p->bfs, grid, p->blds, p->spin_limit,
                           p->wait_unreachable, s);
}

template <typename R>
static nufft_status build_batch(Plan *p, int B, const int64_t *Ns, const int64_t *Ms, const double *const *xs,
                                hipStream_t s)
{
    std::vector<BatchDesc<R>> desc(B);
    std::vector<Factors<R>> facs(B);
    size_t lds = 0;
    int kmax = 0;
    double gmax = 0;
    for (int b = 0; b < B; ++b) {
        Plan *c = new (std::nothrow) Plan();
        if (!c) return NUFFT_ERR_ALLOC;
        p->children.push_back(c);
        c->kind = PLAN_1D;
        c->dtype = p->dtype;
        c->flags = p->flags & NUFFT_FLAG_FIX_GAMMA_HALF;
        c->N = Ns[b];
        c->M = Ms[b];
        c->eps = p->eps;
        if (!choose_grid(c->N, &c->L, &c->L1, &c->L2) || c->L > (int64_t(1) << 20)) return NUFFT_ERR_UNSUPPORTED;
        nufft_status st = build_1d<R>(c, xs[b], s);
        if (st) return st;
        facs[b] = *(const Factors<R> *)c->factors();
        BatchDesc<R> &d = desc[b];
        d.N = c->N;
        d.M = c->M;
        d.L = c->L;
        d.L1 = c->L1;
        d.L2 = c->L2;
        d.n_pass_a = c->L2 > 1 ? c->L1 / batch_pass_a_cols(c->L2) : 0;
        d.t = c->t;
        d.X = (const R *)c->X;
        d.keys = c->keys;
        d.perm = c->perm;
        d.Xs = (const R *)c->Xs;
        d.off = c->off;
        d.Y = (cx_t<R> *)c->Y;
        d.tw1 = (const cx_t<R> *)c->tw1;
        d.tw2 = (const cx_t<R> *)c->tw2;
        d.hi = (const cx_t<R> *)c->hi;
        d.lo = (const cx_t<R> *)c->lo;
        lds = std::max(lds, batch_lds_bytes((int)c->L, c->L1, c->L2, p->dtype == NUFFT_C64));
        kmax = std::max(kmax, c->K);
        gmax = std::max(gmax, c->gamma);
    }
    p->K = kmax;
    p->gamma = gmax;
    p->blds = lds;
    // task table: phase 1 (whole small transforms, pass-A column groups), then pass-B tiles;
    // members in decreasing order of grid size so that the long tasks start first
    std::vector<int> order(B);
    for (int b = 0; b < B; ++b) order[b] = b;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return desc[a].L > desc[b].L; });
    std::vector<int4> tk;
    const int chunk = batch_small_chunk();
    for (int b : order) {
        if (desc[b].L2 == 1) {
            for (int64_t j = 0; j < desc[b].M; j += chunk) tk.push_back(make_int4(BATCH_SMALL, b, (int)(j / chunk), 0));
        } else {
            for (int cg = 0; cg < desc[b].n_pass_a; ++cg) tk.push_back(make_int4(BATCH_PASS_A, b, cg, 0));
        }
    }
    // PASS_B tasks: runs of consecutive tiles holding about batch_pass_b_points() grid
    // points, so that the per-task set-up (claim, descriptor, twiddle table) is amortised
    for (int b : order)
        if (desc[b].L2 > 1) {
            const int run = (int)std::max<int64_t>(1, std::min<int64_t>(desc[b].L2, batch_pass_b_points() / desc[b].L1));
            for (int n2 = 0; n2 < desc[b].L2; n2 += run)
                tk.push_back(make_int4(BATCH_PASS_B, b, n2, (int)std::min<int64_t>(run, desc[b].L2 - n2)));
        }
    p->bntasks = (int)tk.size();
    // the same tasks grouped by type for the phased mode (each group keeps the order above)
    std::vector<int4> tk3;
    for (int type : {BATCH_SMALL, BATCH_PASS_A, BATCH_PASS_B}) {
        for (const int4 &t : tk)
            if (t.x == type) tk3.push_back(t);
        p->bcnt[type] = (int)tk3.size() - (type > 0 ? p->bcnt[0] + (type > 1 ? p->bcnt[1] : 0) : 0);
    }
    Factors<R> *dfac = (Factors<R> *)p->alloc(B * sizeof(Factors<R>));
    p->bdesc = p->alloc(B * sizeof(BatchDesc<R>));
    p->btasks = p->alloc(tk.size() * sizeof(int4));
    p->btasks3 = p->alloc(tk3.size() * sizeof(int4));
    if (!p->btasks3) return NUFFT_ERR_ALLOC;
    const size_t ctl_bytes = sizeof(BatchCtl) + (size_t)B * sizeof(int);
    p->bctl = p->alloc(ctl_bytes);
    p->bcs = (void **)p->alloc(B * sizeof(void *));
    p->bfs = (void **)p->alloc(B * sizeof(void *));
    if (!dfac || !p->bdesc || !p->btasks || !p->bctl || !p->bcs || !p->bfs) return NUFFT_ERR_ALLOC;
    for (int b = 0; b < B; ++b) desc[b].fac = dfac + b;
    std::vector<char> ctl(ctl_bytes, 0);
    ((BatchCtl *)ctl.data())->ntransforms = B;
    NUFFT_HIP_CHECK(hipMemcpyAsync(dfac, facs.data(), B * sizeof(Factors<R>), hipMemcpyHostToDevice, s));
    NUFFT_HIP_CHECK(hipMemcpyAsync(p->bdesc, desc.data(), B * sizeof(BatchDesc<R>), hipMemcpyHostToDevice, s));
    NUFFT_HIP_CHECK(hipMemcpyAsync(p->btasks, tk.data(), tk.size() * sizeof(int4), hipMemcpyHostToDevice, s));
    NUFFT_HIP_CHECK(hipMemcpyAsync(p->btasks3, tk3.data(), tk3.size() * sizeof(int4), hipMemcpyHostToDevice, s));
    NUFFT_HIP_CHECK(hipMemcpyAsync(p->bctl, ctl.data(), ctl_bytes, hipMemcpyHostToDevice, s));
    NUFFT_HIP_CHECK(hipStreamSynchronize(s));
    NUFFT_HIP_CHECK(batch_set_lds_limit<R>(lds));
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    // default: the three phased launches; NUFFT_FLAG_BATCH_PERSISTENT: one persistent launch
    const bool persistent = (p->flags & NUFFT_FLAG_BATCH_PERSISTENT) != 0;
    p->bmode = persistent ? 0 : 1;
    p->bgrid = persistent ? 2 * cus : p->bntasks;
    // the problem class: member sizes (hashed), dtype, eps, flags
    unsigned long long h = 1469598103934665603ull;
    auto mix = [&](unsigned long long v) {
        for (int i = 0; i < 8; ++i) {
            h ^= (v >> (8 * i)) & 0xff;
            h *= 1099511628211ull;
        }
    };
    for (int b = 0; b < B; ++b) {
        mix((unsigned long long)Ns[b]);
        mix((unsigned long long)Ms[b]);
    }
    char kb[192];
    std::snprintf(kb, sizeof(kb), "batch B=%d dt=%d eps=%.17g flags=%u cus=%d sizes=%016llx", B, (int)p->dtype,
                  p->eps, (unsigned)p->flags, cus, h);
    const std::string key(kb);
    long long known = 0;
    if (!(p->flags & NUFFT_FLAG_NO_AUTOTUNE) && tune_lookup(key, &known)) {
        p->bmode = (int)(known >> 32);
        p->bgrid = (int)(known & 0xffffffff);
    } else if (!(p->flags & NUFFT_FLAG_NO_AUTOTUNE)) {
        // time the launch at 1..4 workgroups per CU on scratch inputs, keep the fastest
        int64_t nc = 0, nf = 0;
        for (int b = 0; b < B; ++b) {
            nc += desc[b].N;
            nf += desc[b].M;
        }
        Plan scratch;
        cx_t<R> *cbuf = (cx_t<R> *)scratch.alloc(nc * sizeof(cx_t<R>));
        cx_t<R> *fbuf = (cx_t<R> *)scratch.alloc(nf * sizeof(cx_t<R>));
        if (!cbuf || !fbuf) return NUFFT_ERR_ALLOC;
        NUFFT_HIP_CHECK(hipMemsetAsync(cbuf, 0, nc * sizeof(cx_t<R>), s));
        std::vector<const void *> cp(B);
        std::vector<void *> fp(B);
        for (int b = 0, oc = 0, of = 0; b < B; ++b) {
            cp[b] = cbuf + oc;
            fp[b] = fbuf + of;
            oc += (int)desc[b].N;
            of += (int)desc[b].M;
        }
        nufft_status st = batch_upload_ptrs<R>(p, cp.data(), fp.data(), s);
        if (st) return st;
        hipEvent_t e0, e1;
        NUFFT_HIP_CHECK(hipEventCreate(&e0));
        NUFFT_HIP_CHECK(hipEventCreate(&e1));
        float best = 1e30f;
        // candidates: the persistent launch at 1..4 workgroups per CU, and the phased launches
        // (with NUFFT_FLAG_BATCH_PERSISTENT only the persistent grid sizes)
        for (int cand = 1; cand <= (persistent ? 4 : 5); ++cand) {
            const int mode = cand == 5 ? 1 : 0, grid = cand == 5 ? p->bntasks : cand * cus;
            NUFFT_HIP_CHECK(batch_run<R>(p, mode, grid, s));   // warm-up
            NUFFT_HIP_CHECK(hipEventRecord(e0, s));
            for (int rep = 0; rep < 3; ++rep) NUFFT_HIP_CHECK(batch_run<R>(p, mode, grid, s));
            NUFFT_HIP_CHECK(hipEventRecord(e1, s));
            NUFFT_HIP_CHECK(hipEventSynchronize(e1));
            float ms = 0;
            NUFFT_HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
            if (ms < best) {
                best = ms;
                p->bgrid = grid;
                p->bmode = mode;
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        p->hcs.clear();   // scratch pointers: force the next exec to upload its own
        p->hfs.clear();
        tune_store(key, ((long long)p->bmode << 32) | (long long)p->bgrid);
    }
    return NUFFT_OK;
}
// 3-D transforms: the z axis factored as in Sec. 2.1-2.2 (rank K3 on a grid of
// Gz points), one length-Gz FFT per (k1, k2) and rank, and for each z slice of
// the samples one 2-D transform (Sec. 4) of that slice; the compositions are
// stated with the kernels.  The Gz slice transforms are the problems of one
// stacked 2-D plan (every slice's columns in one pass-B launch).  Half of eps
// goes to the z factorisation, half to the 2-D transforms, whose errors are
// weighted by sum_r |u^z_r| w_r <= sum_{p,r} w_p w_r |b_pr| (the same bound
// serves type I, whose inner inputs are u^z_r c or its conjugate).
// p: a PLAN_3D plan with dtype, N1, N2, N3, M and eps set; it owns everything built.
template <typename R>
static nufft_status build_3d(Plan *p, const double *x, const double *y, const double *z, hipStream_t s)
{
    using C = cx_t<R>;
    const int64_t M = p->M, n1 = p->N1, n2 = p->N2, n3 = p->N3;
    int64_t Gz = 16;
    while (Gz < n3) Gz <<= 1;
    int gx = 16, gy = 16;
    while (gx < n1) gx <<= 1;
    while (gy < n2) gy <<= 1;
    if (Gz > 1024 || gx > 2048 || gy > 2048 || Gz * gx * gy > (int64_t(1) << 28)) return NUFFT_ERR_UNSUPPORTED;
    p->Gz = Gz;
    const int64_t rows = n1 * n2;
    int32_t *tz = (int32_t *)p->alloc(M * sizeof(int32_t));
    p->Xz = p->alloc(M * sizeof(R));
    unsigned long long *flags = (unsigned long long *)p->alloc(2 * sizeof(unsigned long long));
    p->Dz = p->alloc(Gz * rows * sizeof(C));
    p->fsz = p->alloc(M * sizeof(C));
    if (!tz || !p->Xz || !flags || !p->Dz || !p->fsz) return NUFFT_ERR_ALLOC;
    // z slice and perturbation per sample, and gamma_z
    NUFFT_HIP_CHECK(hipMemsetAsync(flags, 0, 2 * sizeof(unsigned long long), s));
    NUFFT_HIP_CHECK(launch_3d_assign<R>(z, M, n3, Gz, tz, (R *)p->Xz, flags, (int *)(flags + 1), s));
    unsigned long long h[2];
    NUFFT_HIP_CHECK(hipMemcpyAsync(h, flags, sizeof(h), hipMemcpyDeviceToHost, s));
    NUFFT_HIP_CHECK(hipStreamSynchronize(s));
    if ((int)h[1] != 0) return NUFFT_ERR_NONFINITE;
    double gz;
    std::memcpy(&gz, &h[0], sizeof(double));
    gz = std::min(gz, 0.5);
    p->K3 = choose_rank(p->eps / 2.0, gz);
    if (p->K3 < 0 || (sizeof(R) == 4 && p->K3 > NUFFT_KMAX_F32)) return NUFFT_ERR_UNSUPPORTED;
    if constexpr (sizeof(R) == 4) fill_factors(p->ffz, gz, p->K3);
    else fill_factors(p->fdz, gz, p->K3);
    double b[NUFFT_KMAX * NUFFT_KMAX], S = 0.0;
    bessel_b(gz, p->K3, b);
    for (int q = 0; q < p->K3; ++q)
        for (int r = 0; r < p->K3; ++r)
            S += (q == 0 ? 0.5 : 1.0) * (r == 0 ? 0.5 : 1.0) * std::fabs(b[q * p->K3 + r]);
    const double floor_eps = p->dtype == NUFFT_C64 ? 1e-7 : 1e-15;
    const double eps2 = std::max(floor_eps, p->eps / (2.0 * std::max(S, 1.0)));
    // the composed bound eps/2 + S eps2 stays within 4 eps, or the precision floor cannot serve eps
    if (p->eps / 2.0 + std::max(S, 1.0) * eps2 > 4.0 * p->eps) return NUFFT_ERR_UNSUPPORTED;
    // one stacked 2-D plan: problem m holds the samples of z slice m
    Plan *q = new (std::nothrow) Plan();
    if (!q) return NUFFT_ERR_ALLOC;
    p->children.push_back(q);
    q->kind = PLAN_2D;
    q->dtype = p->dtype;
    q->N1 = n1;
    q->N2 = n2;
    q->N = rows;
    q->M = M;
    q->eps = eps2;
    q->Gx = gx;
    q->Gy = gy;
    q->L = (int64_t)gx * gy;
    q->S = (int)Gz;
    q->slice = tz;
    const nufft_status st = build_2d<R>(q, x, y, s);
    q->slice = nullptr;   // read at build time only
    if (st) return st;
    p->stack = q;
    p->K = p->K3;
    p->gamma = gz;
    p->L = Gz * gx * gy;
    std::vector<double> t(2 * (size_t)Gz);
    fft_twiddles(Gz, -1, t.data());
    return upload_table<R>(p, t, &p->twz, s);
}

template <typename R>
static const Factors<R> &z_factors(const Plan *p)
{
    if constexpr (sizeof(R) == 4) return p->ffz;
    else return p->fdz;
}

// 3-D type II: f = sum_r u^z_r * [2-D type II of slice t^z_j of D_r]
template <typename R>
static hipError_t run_type2_3d(const Plan *p, const void *Cin, void *f, hipStream_t s)
{
    using C = cx_t<R>;
    const Args2D<R> a = args_2d<R>(p->stack);
    const int64_t rows = p->N1 * p->N2;
    C *D = (C *)p->Dz, *fs = (C *)p->fsz;
    for (int r = 0; r < p->K3; ++r) {
        hipError_t e = launch_3d_zfft<R>((const C *)Cin, rows, p->N3, p->Gz, r, (const C *)p->twz, D, s);
        if (e == hipSuccess) e = fused_2d<R>(a, D, fs, s);
        if (e == hipSuccess) e = launch_3d_accum<R>(fs, (const R *)p->Xz, p->M, z_factors<R>(p), r, (C *)f, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// 3-D type I (sign -1) / adjoint (sign +1): C = sum_r v^z_r * z-DFT over the slices
// of [2-D type I of slice m, weighted by w_r c]
template <typename R>
static hipError_t run_type1_3d(const Plan *p, const void *c, void *Cout, int sign, hipStream_t s)
{
    using C = cx_t<R>;
    const Args2D<R> a = args_2d<R>(p->stack);
    const int64_t rows = p->N1 * p->N2;
    C *D = (C *)p->Dz, *cw = (C *)p->fsz;
    for (int r = 0; r < p->K3; ++r) {
        hipError_t e = launch_3d_weight<R>((const C *)c, (const R *)p->Xz, p->M, z_factors<R>(p), r, sign, cw, s);
        if (e == hipSuccess) e = fused_2d_adj<R>(a, cw, D, sign, s);   // empty slices come out zero
        if (e == hipSuccess)
            e = launch_3d_zfft_t<R>(D, rows, p->N3, p->Gz, r, sign, (const C *)p->twz, (C *)Cout, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// 2-D type III (Sec. 3.2 applied per axis; the composition is stated with the
// kernels): Kx * Ky inner 2-D type-I transforms on the frequencies.
template <typename R>
static nufft_status type3_2d(int64_t M, const double *x, const double *y, int64_t Q, const double *w1,
                             const double *w2, int64_t n1, int64_t n2, const void *c, void *f, double eps,
                             nufft_dtype dt, hipStream_t s)
{
    using C = cx_t<R>;
    Plan tmp;   // owns the temporaries
    struct SyncGuard {   // destroyed before tmp: no temporary is freed under a running kernel
        hipStream_t s;
        ~SyncGuard() { (void)hipStreamSynchronize(s); }
    } guard{s};
    const int64_t ld = n2 + 1;
    int32_t *sx = (int32_t *)tmp.alloc(M * sizeof(int32_t));
    int32_t *sy = (int32_t *)tmp.alloc(M * sizeof(int32_t));
    double *dx = (double *)tmp.alloc(M * sizeof(double));
    double *dy = (double *)tmp.alloc(M * sizeof(double));
    double *xs = (double *)tmp.alloc(Q * sizeof(double));
    double *ys = (double *)tmp.alloc(Q * sizeof(double));
    unsigned long long *flags = (unsigned long long *)tmp.alloc(3 * sizeof(unsigned long long));
    C *c1 = (C *)tmp.alloc(Q * sizeof(C));
    C *F = (C *)tmp.alloc((n1 + 1) * ld * sizeof(C));
    if (!sx || !sy || !dx || !dy || !xs || !ys || !flags || !c1 || !F) return NUFFT_ERR_ALLOC;
    NUFFT_HIP_CHECK(hipMemsetAsync(flags, 0, 3 * sizeof(unsigned long long), s));
    NUFFT_HIP_CHECK(t3d_assign(x, y, M, n1, n2, sx, sy, dx, dy, flags, (int *)(flags + 2), s));
    NUFFT_HIP_CHECK(t3d_freq(w1, w2, Q, n1, n2, xs, ys, (int *)(flags + 2), s));
    unsigned long long h[3];
    NUFFT_HIP_CHECK(hipMemcpyAsync(h, flags, sizeof(h), hipMemcpyDeviceToHost, s));
    NUFFT_HIP_CHECK(hipStreamSynchronize(s));
    if ((int)h[2] & 5) return NUFFT_ERR_INVALID_ARG;   // samples outside [0,1)^2 / frequencies outside [0,n)
    double gx, gy;
    std::memcpy(&gx, &h[0], sizeof(double));
    std::memcpy(&gy, &h[1], sizeof(double));
    gx = std::min(gx, 0.5);
    gy = std::min(gy, 0.5);
    // half of eps for the factorisation, shared by the two axes
    // (|A^x A^y - A^x_K A^y_K| <= eps_x + eps_y + eps_x eps_y), half for the inner
    // transforms, whose errors are weighted by sum |u^x_r1| |u^y_r2| <= su_x su_y
    const int Kx = choose_rank(eps / 4.0, gx), Ky = choose_rank(eps / 4.0, gy);
    if (Kx < 0 || Ky < 0) return NUFFT_ERR_UNSUPPORTED;
    Factors<double> fx, fy;
    double sux, suy;
    t3_factors(gx, Kx, fx, &sux);
    t3_factors(gy, Ky, fy, &suy);
    const double floor_eps = dt == NUFFT_C64 ? 1e-7 : 1e-15;
    const double sw = std::max(sux, 1.0) * std::max(suy, 1.0);
    double eps_i = eps / (2.0 * sw);
    if (eps_i < floor_eps) eps_i = floor_eps;
    if (eps / 2.0 + sw * eps_i > 4.0 * eps) return NUFFT_ERR_UNSUPPORTED;   // as in the 1-D type III
    // inner 2-D type-I plan on the samples (w1/n1, w2/n2) with n1+1 by n2+1 modes
    Plan *inner = new (std::nothrow) Plan();
    if (!inner) return NUFFT_ERR_ALLOC;
    tmp.children.push_back(inner);
    inner->kind = PLAN_2D;
    inner->dtype = dt;
    inner->N1 = n1 + 1;
    inner->N2 = n2 + 1;
    inner->N = (n1 + 1) * (n2 + 1);
    inner->M = Q;
    inner->eps = eps_i;
    int gxs = 16, gys = 16;
    while (gxs < n1 + 1) gxs <<= 1;
    while (gys < n2 + 1) gys <<= 1;
    if (gxs > 2048 || gys > 2048) return NUFFT_ERR_UNSUPPORTED;
    inner->Gx = gxs;
    inner->Gy = gys;
    inner->L = (int64_t)gxs * gys;
    nufft_status st = build_2d<R>(inner, xs, ys, s);
    if (st) return st;
    const Args2D<R> ia = args_2d<R>(inner);
    for (int r1 = 0; r1 < Kx; ++r1)
        for (int r2 = 0; r2 < Ky; ++r2) {
            NUFFT_HIP_CHECK(t3d_scale<R>((const C *)c, w1, w2, Q, n1, n2, r1, r2, c1, s));
            NUFFT_HIP_CHECK(fused_2d_adj<R>(ia, c1, F, -1, s));
            NUFFT_HIP_CHECK(t3d_accum<R>(dx, dy, sx, sy, M, fx, fy, r1, r2, F, ld, r1 == 0 && r2 == 0, (C *)f, s));
        }
    return NUFFT_OK;
}

}  // namespace nufft

// ============================================================================
// exported entry points
// ============================================================================

static nufft_status from_hip(hipError_t e) { return e == hipSuccess ? NUFFT_OK : NUFFT_ERR_HIP; }

// Oversampling choice.  Sec. 2.3 leaves the grid free as long as it has at least
// N points; a larger grid lowers gamma_eff = max|X| <= N / (2L) and with it K,
// at the price of longer FFTs.  Unless NUFFT_FLAG_NO_AUTOTUNE is given, the plan
// is built on the smallest power-of-two grid L0 >= N and on 2 L0 (gamma_eff <=
// 1/4), one type-II transform of each is timed on a scratch input, and the
// faster plan is kept.  The larger grid wins when the per-sample work K M
// outweighs the FFT work K L log L, e.g. for many more samples than modes.
template <typename R>
static nufft_status time_type2(Plan *p, hipStream_t s, float *ms_out)
{
    Plan scratch;
    void *c = scratch.alloc((size_t)p->N * 2 * sizeof(R));
    void *f = scratch.alloc((size_t)p->M * 2 * sizeof(R));
    if (!c || !f) return NUFFT_ERR_ALLOC;
    NUFFT_HIP_CHECK(hipMemsetAsync(c, 0, (size_t)p->N * 2 * sizeof(R), s));
    hipEvent_t e0, e1;
    NUFFT_HIP_CHECK(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return NUFFT_ERR_HIP;
    }
    hipError_t e = exec_type2<R>(p, c, f, 0, nullptr, nullptr, s);   // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) e = exec_type2<R>(p, c, f, 0, nullptr, nullptr, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms_out, e0, e1);
    (void)hipStreamSynchronize(s);   // nothing may still use the scratch buffers freed on return
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return from_hip(e);
}

// Oversampling (Sec. 2.3): every grid L with N <= L <= 2 L0 (L0 the power of
// two the plan starts from) that the kernels support is a candidate: powers
// of two and, unless the plan uses the half-precision exchange, 3 * 2^k and
// 5 * 2^k.  A larger L lowers gamma and with it K (less work per sample) at
// the cost of a larger FFT.  Each candidate is planned on the same samples and
// its type-II transform timed (two interleaved rounds, the best of each); the
// fastest plan replaces *pp and its grid is remembered per (N, M, dtype, eps,
// flags).
template <typename R>
static nufft_status autotune_grid(Plan **pp, const double *x, hipStream_t s)
{
    Plan *p = *pp;
    const int64_t L0 = p->L;
    const bool mixed_ok = !(p->flags & NUFFT_FLAG_HALF_EXCHANGE);
    std::vector<int64_t> cand;   // besides L0, ascending
    for (int64_t b = 16; b <= 2 * L0; b <<= 1)
        for (int P : {1, 3, 5}) {
            const int64_t L = P * b;
            int l1, l2;
            if (L == L0 || L < p->N || L > 2 * L0 || (P > 1 && !mixed_ok) || !grid_split(L, &l1, &l2)) continue;
            cand.push_back(L);
        }
    std::sort(cand.begin(), cand.end());
    cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
    if (cand.empty()) return NUFFT_OK;
    char kb[192];
    std::snprintf(kb, sizeof(kb), "1d-grid N=%lld M=%lld dt=%d eps=%.17g flags=%u", (long long)p->N,
                  (long long)p->M, (int)p->dtype, p->eps, (unsigned)p->flags);
    const std::string key(kb);
    long long known = 0;
    if (tune_lookup(key, &known)) {
        if (known == L0 || std::find(cand.begin(), cand.end(), (int64_t)known) == cand.end()) return NUFFT_OK;
        cand.assign(1, (int64_t)known);
    }
    // the candidate plans (owned by `keep` until one of them replaces *pp)
    std::vector<Plan *> plans;
    struct Owner {
        std::vector<Plan *> *v;
        hipStream_t s;
        ~Owner()
        {
            if (!v->empty()) (void)hipStreamSynchronize(s);
            for (Plan *q : *v) delete q;
        }
    } keep{&plans, s};
    for (int64_t L : cand) {
        Plan *q = new (std::nothrow) Plan();
        if (!q) return NUFFT_ERR_ALLOC;
        q->kind = PLAN_1D;
        q->dtype = p->dtype;
        q->flags = p->flags;
        q->N = p->N;
        q->M = p->M;
        q->eps = p->eps;
        q->L = L;
        grid_split(L, &q->L1, &q->L2);
        const nufft_status st = build_1d<R>(q, x, s);
        if (st == NUFFT_ERR_UNSUPPORTED) {   // e.g. K beyond the FP32 rank limit on a smaller grid
            (void)hipStreamSynchronize(s);
            delete q;
            continue;
        }
        plans.push_back(q);
        if (st) return st;
    }
    if (plans.empty()) return NUFFT_OK;
    int pick = -1;   // -1: the plan on L0
    if (known) {
        pick = 0;
    } else {
        std::vector<float> best(plans.size() + 1, 1e30f);
        for (int round = 0; round < 2; ++round)
            for (size_t i = 0; i <= plans.size(); ++i) {
                float t = 0;
                const nufft_status st = time_type2<R>(i == 0 ? p : plans[i - 1], s, &t);
                if (st) return st;
                best[i] = std::min(best[i], t);
            }
        size_t bi = 0;
        for (size_t i = 1; i < best.size(); ++i)
            if (best[i] < best[bi]) bi = i;
        pick = (int)bi - 1;
        tune_store(key, pick < 0 ? (long long)L0 : (long long)plans[pick]->L);
    }
    if (pick < 0) return NUFFT_OK;
    (void)hipStreamSynchronize(s);
    Plan *q = plans[pick];
    plans.erase(plans.begin() + pick);
    delete p;
    *pp = q;
    return NUFFT_OK;
}

// Tuning schedule of the two-pass kernels (first FFT radix, tile shapes; the
// kernels list the schedules).  Unless NUFFT_FLAG_NO_AUTOTUNE is given, an
// FP32 plan offering them times one type-II transform and one adjoint under
// each schedule on scratch inputs and keeps the fastest; the choice is
// remembered per (L1, L2, K, tile population class, flags).
template <typename R>
static nufft_status autotune_schedule(Plan *p, hipStream_t s)
{
    if (!p->tw1r8) return NUFFT_OK;   // the plan offers only the default
    int mc = 0;   // tile population class: log2 of samples per grid point, rounded down, in [-8, 8]
    for (int64_t v = p->M; v >= 2 * p->L && mc < 8; v >>= 1) ++mc;
    for (int64_t v = p->M; 2 * v <= p->L && mc > -8; v <<= 1) --mc;
    char kb[192];
    std::snprintf(kb, sizeof(kb), "sched L1=%d L2=%d dt=%d K=%d mc=%d flags=%u", p->L1, p->L2, (int)p->dtype, p->K,
                  mc, (unsigned)p->flags);
    const std::string key(kb);
    long long known = 0;
    if (tune_lookup(key, &known)) {
        p->sched = (int)known;
        return NUFFT_OK;
    }
    Plan scratch;
    void *c = scratch.alloc((size_t)p->N * 2 * sizeof(R));
    void *g = scratch.alloc((size_t)p->M * 2 * sizeof(R));
    void *f = scratch.alloc((size_t)std::max(p->N, p->M) * 2 * sizeof(R));
    if (!c || !g || !f) return NUFFT_ERR_ALLOC;
    NUFFT_HIP_CHECK(hipMemsetAsync(c, 0, (size_t)p->N * 2 * sizeof(R), s));
    NUFFT_HIP_CHECK(hipMemsetAsync(g, 0, (size_t)p->M * 2 * sizeof(R), s));
    hipEvent_t e0, e1;
    NUFFT_HIP_CHECK(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return NUFFT_ERR_HIP;
    }
    // the schedules are timed in interleaved rounds and each keeps its best round,
    // so that a slow moment of the device does not decide the choice
    constexpr int NS = 3, ROUNDS = 3, REPS = 3;
    float best_of[NS];
    for (int sc = 0; sc < NS; ++sc) best_of[sc] = 1e30f;
    hipError_t e = hipSuccess;
    for (int round = 0; round < ROUNDS && e == hipSuccess; ++round)
        for (int sc = 0; sc < NS && e == hipSuccess; ++sc) {
            p->sched = sc;
            const FusedArgs<R> a = fused_args<R>(p);
            auto once = [&]() {
                hipError_t r = fused_type2<R>(a, (const cx_t<R> *)c, (cx_t<R> *)f, 0, nullptr, nullptr, s);
                if (r == hipSuccess) r = fused_type1<R>(a, (const cx_t<R> *)g, (cx_t<R> *)f, +1, s);
                return r;
            };
            e = once();   // warm-up
            if (e == hipSuccess) e = hipEventRecord(e0, s);
            for (int rep = 0; rep < REPS && e == hipSuccess; ++rep) e = once();
            if (e == hipSuccess) e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e == hipSuccess) best_of[sc] = std::min(best_of[sc], ms);
        }
    int pick = 0;
    for (int sc = 1; sc < NS; ++sc)
        if (best_of[sc] < best_of[pick]) pick = sc;
    (void)hipStreamSynchronize(s);   // nothing may still use the scratch buffers freed on return
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    p->sched = pick;
    if (e != hipSuccess) return NUFFT_ERR_HIP;
    tune_store(key, pick);
    return NUFFT_OK;
}

static bool eps_ok(double eps, nufft_dtype dt, nufft_status *st)
{
    if (!(eps > 0.0 && eps < 1.0)) { *st = NUFFT_ERR_INVALID_ARG; return false; }
    const double floor_eps = dt == NUFFT_C64 ? 1e-7 : 1e-15;
    if (eps < floor_eps) { *st = NUFFT_ERR_UNSUPPORTED; return false; }
    return true;
}

extern "C" {

// grid 0: the grid is chosen (and autotuned); else the plan uses that grid.
static nufft_status plan_1d(nufft_plan_t *out, int64_t n_modes, int64_t n_pts, const double *x_dev, double eps,
                            nufft_dtype dtype, uint32_t flags, int64_t grid, void *stream)
{
    if (!out) return NUFFT_ERR_INVALID_ARG;
    *out = nullptr;
    if (n_modes < 1 || n_pts < 1 || !x_dev) return NUFFT_ERR_INVALID_ARG;
    if (dtype != NUFFT_C64 && dtype != NUFFT_C128) return NUFFT_ERR_INVALID_ARG;
    if (flags & ~(uint32_t)(NUFFT_FLAG_FIX_GAMMA_HALF | NUFFT_FLAG_PLAIN_UNFUSED | NUFFT_FLAG_HALF_EXCHANGE |
                            NUFFT_FLAG_NO_AUTOTUNE))
        return NUFFT_ERR_INVALID_ARG;
    if ((flags & NUFFT_FLAG_HALF_EXCHANGE) && (flags & NUFFT_FLAG_PLAIN_UNFUSED)) return NUFFT_ERR_INVALID_ARG;
    if (n_pts > (int64_t(1) << 30)) return NUFFT_ERR_UNSUPPORTED;
    nufft_status st;
    if (!eps_ok(eps, dtype, &st)) return st;
    // fp16 storage rounding (2^-11 relative) must fit the error budget
    if ((flags & NUFFT_FLAG_HALF_EXCHANGE) && (dtype != NUFFT_C64 || eps < 0x1p-10)) return NUFFT_ERR_UNSUPPORTED;
    Plan *p = new (std::nothrow) Plan();
    if (!p) return NUFFT_ERR_ALLOC;
    p->kind = PLAN_1D;
    p->dtype = dtype;
    p->flags = flags;
    p->N = n_modes;
    p->M = n_pts;
    p->eps = eps;
    if (grid == 0) {
        if (!choose_grid(n_modes, &p->L, &p->L1, &p->L2)) {
            delete p;
            return NUFFT_ERR_UNSUPPORTED;
        }
    } else {
        p->L = grid;
        const bool pow2 = (grid & (grid - 1)) == 0;
        if (grid < n_modes || !grid_split(grid, &p->L1, &p->L2) ||
            (!pow2 && (flags & (NUFFT_FLAG_PLAIN_UNFUSED | NUFFT_FLAG_HALF_EXCHANGE)))) {
            delete p;
            return NUFFT_ERR_UNSUPPORTED;
        }
    }
    hipStream_t s = (hipStream_t)stream;
    st = dtype == NUFFT_C64 ? build_1d<float>(p, x_dev, s) : build_1d<double>(p, x_dev, s);
    if (st == NUFFT_OK && grid == 0 && !(flags & (NUFFT_FLAG_NO_AUTOTUNE | NUFFT_FLAG_PLAIN_UNFUSED)))
        st = dtype == NUFFT_C64 ? autotune_grid<float>(&p, x_dev, s) : autotune_grid<double>(&p, x_dev, s);
    if (st == NUFFT_OK && !(flags & (NUFFT_FLAG_NO_AUTOTUNE | NUFFT_FLAG_PLAIN_UNFUSED)))
        st = dtype == NUFFT_C64 ? autotune_schedule<float>(p, s) : autotune_schedule<double>(p, s);
    if (st != NUFFT_OK) {
        (void)hipStreamSynchronize(s);
        delete p;
        return st;
    }
    p->last = s;
    *out = p;
    return NUFFT_OK;
}

nufft_status nufft2_plan(nufft_plan_t *out, int64_t n_modes, int64_t n_pts, const double *x_dev, double eps,
                         nufft_dtype dtype, uint32_t flags, void *stream)
{
    return plan_1d(out, n_modes, n_pts, x_dev, eps, dtype, flags, 0, stream);
}

nufft_status nufft2_plan_grid(nufft_plan_t *out, int64_t n_modes, int64_t n_pts, const double *x_dev, double eps,
                              nufft_dtype dtype, uint32_t flags, int64_t grid, void *stream)
{
    if (out) *out = nullptr;
    if (grid < 1) return NUFFT_ERR_INVALID_ARG;
    return plan_1d(out, n_modes, n_pts, x_dev, eps, dtype, flags, grid, stream);
}

nufft_status nufft2_exec(nufft_plan_t plan, const void *c, void *f, void *stream)
{
    if (!plan || plan->kind != PLAN_1D || !c || !f) return NUFFT_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    plan->last = s;
    return from_hip(plan->dtype == NUFFT_C64 ? exec_type2<float>(plan, c, f, 0, nullptr, nullptr, s)
                                             : exec_type2<double>(plan, c, f, 0, nullptr, nullptr, s));
}

nufft_status nufft2_grad_x(nufft_plan_t plan, const void *c, const void *g, double *gx, void *stream)
{
    if (!plan || plan->kind != PLAN_1D || !c || !g || !gx) return NUFFT_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    plan->last = s;
    return from_hip(plan->dtype == NUFFT_C64 ? exec_type2<float>(plan, c, nullptr, 1, g, gx, s)
                                             : exec_type2<double>(plan, c, nullptr, 1, g, gx, s));
}

nufft_status nufft2_solve(nufft_plan_t plan, const void *f, void *c, double tol, int max_iter, int *iters,
                          double *resid, void *stream)
{
    if (!plan || plan->kind != PLAN_1D || !f || !c || !(tol > 0.0) || max_iter < 0) return NUFFT_ERR_INVALID_ARG;
    if (plan->N > (int64_t(1) << 22)) return NUFFT_ERR_UNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    plan->last = s;
    return plan->dtype == NUFFT_C64 ? solve_impl<float, false>(plan, f, c, tol, max_iter, iters, resid, s)
                                    : solve_impl<double, false>(plan, f, c, tol, max_iter, iters, resid, s);
}

nufft_status nufft1_solve(nufft_plan_t plan, const void *f, void *c, double tol, int max_iter, int *iters,
                          double *resid, void *stream)
{
    if (!plan || plan->kind != PLAN_1D || !f || !c || !(tol > 0.0) || max_iter < 0) return NUFFT_ERR_INVALID_ARG;
    if (plan->N > (int64_t(1) << 22)) return NUFFT_ERR_UNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    plan->last = s;
    return plan->dtype == NUFFT_C64 ? solve_impl<float, true>(plan, f, c, tol, max_iter, iters, resid, s)
                                    : solve_impl<double, true>(plan, f, c, tol, max_iter, iters, resid, s);
}

nufft_status nufft2_backward(nufft_plan_t plan, const void *c, const void *g, void *gc, double *gx, void *stream)
{
    if (!plan || plan->kind != PLAN_1D || !g || (!gc && !gx) || (gx && !c)) return NUFFT_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    plan->last = s;
    return plan->dtype == NUFFT_C64 ? exec_backward<float>(plan, c, g, gc, gx, s)
                                    : exec_backward<double>(plan, c, g, gc, gx, s);
}

nufft_status nufft1_exec(nufft_plan_t plan, const void *c, void *f, int sign, void *stream)
{
    if (!plan || plan->kind != PLAN_1D || !c || !f || (sign != 1 && sign != -1)) return NUFFT_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    plan->last = s;
    return from_hip(plan->dtype == NUFFT_C64 ? exec_type1<float>(plan, c, f, sign, s)
                                             : exec_type1<double>(plan, c, f, sign, s));
}

nufft_status nufft3_exec(int64_t n_pts, const double *x, int64_t n_freq, const double *w, const void *c, void *f,
                         double eps, nufft_dtype dtype, void *stream)
{
    if (n_pts < 1 || n_freq < 1 || !x || !w || !c || !f) return NUFFT_ERR_INVALID_ARG;
    if (dtype != NUFFT_C64 && dtype != NUFFT_C128) return NUFFT_ERR_INVALID_ARG;
    if (n_pts > (int64_t(1) << 30)) return NUFFT_ERR_UNSUPPORTED;
    nufft_status st;
    if (!eps_ok(eps, dtype, &st)) return st;
    hipStream_t s = (hipStream_t)stream;
    st = dtype == NUFFT_C64 ? type3<float>(n_pts, x, n_freq, w, c, f, eps, dtype, s)
                            : type3<double>(n_pts, x, n_freq, w, c, f, eps, dtype, s);
    if (st != NUFFT_OK) (void)hipStreamSynchronize(s);
    return st;
}

// The same transform with every temporary in the device's fixed scratch array
// (no device allocation).  Calls of one process are serialised: each one ends
// with its stream synchronised, so the next finds the array free.
static std::mutex noalloc_mu;

nufft_status nufft3_exec_noalloc(int64_t n_pts, const double *x, int64_t n_freq, const double *w, const void *c,
                                 void *f, double eps, nufft_dtype dtype, void *stream)
{
    if (n_pts < 1 || n_freq < 1 || !x || !w || !c || !f) return NUFFT_ERR_INVALID_ARG;
    if (dtype != NUFFT_C64 && dtype != NUFFT_C128) return NUFFT_ERR_INVALID_ARG;
    if (n_pts > NUFFT_NOALLOC_MAX_M || n_freq > NUFFT_NOALLOC_MAX_N) return NUFFT_ERR_UNSUPPORTED;
    nufft_status st;
    if (!eps_ok(eps, dtype, &st)) return st;
    std::lock_guard<std::mutex> g(noalloc_mu);
    void *base = nullptr;
    size_t cap = 0;
    NUFFT_HIP_CHECK(noalloc_scratch(&base, &cap));
    Arena arena;
    arena.base = (char *)base;
    arena.cap = cap;
    hipStream_t s = (hipStream_t)stream;
    st = dtype == NUFFT_C64 ? type3<float>(n_pts, x, n_freq, w, c, f, eps, dtype, s, &arena)
                            : type3<double>(n_pts, x, n_freq, w, c, f, eps, dtype, s, &arena);
    (void)hipStreamSynchronize(s);   // the array is free again when the call returns
    if (st == NUFFT_ERR_ALLOC) st = NUFFT_ERR_UNSUPPORTED;   // beyond the array (not expected within the limits)
    return st;
}

// A 3-D plan on the stream, or an error with everything it built released.
static nufft_status make_3d_plan(Plan **out, int64_t n1, int64_t n2, int64_t n3, int64_t n_pts, const double *x,
                                 const double *y, const double *z, double eps, nufft_dtype dtype, hipStream_t s)
{
    *out = nullptr;
    if (n_pts < 1 || n1 < 1 || n2 < 1 || n3 < 1 || !x || !y || !z) return NUFFT_ERR_INVALID_ARG;
    if (dtype != NUFFT_C64 && dtype != NUFFT_C128) return NUFFT_ERR_INVALID_ARG;
    if (n_pts > (int64_t(1) << 30)) return NUFFT_ERR_UNSUPPORTED;
    nufft_status st;
    if (!eps_ok(eps, dtype, &st)) return st;
    Plan *p = new (std::nothrow) Plan();
    if (!p) return NUFFT_ERR_ALLOC;
    p->kind = PLAN_3D;
    p->dtype = dtype;
    p->N1 = n1;
    p->N2 = n2;
    p->N3 = n3;
    p->N = n1 * n2 * n3;
    p->M = n_pts;
    p->eps = eps;
    st = dtype == NUFFT_C64 ? build_3d<float>(p, x, y, z, s) : build_3d<double>(p, x, y, z, s);
    if (st != NUFFT_OK) {
        (void)hipStreamSynchronize(s);
        delete p;
        return st;
    }
    p->last = s;
    *out = p;
    return NUFFT_OK;
}

static hipError_t exec_3d(const Plan *p, const void *in, void *out, int type1, int sign, hipStream_t s)
{
    if (type1)
        return p->dtype == NUFFT_C64 ? run_type1_3d<float>(p, in, out, sign, s)
                                     : run_type1_3d<double>(p, in, out, sign, s);
    return p->dtype == NUFFT_C64 ? run_type2_3d<float>(p, in, out, s) : run_type2_3d<double>(p, in, out, s);
}

// The plan-free calls: a temporary plan, released once the stream has finished with it.
static nufft_status oneshot_3d(int64_t n_pts, const double *x, const double *y, const double *z, int64_t n1,
                               int64_t n2, int64_t n3, const void *in, void *out, int type1, int sign, double eps,
                               nufft_dtype dtype, hipStream_t s)
{
    Plan *p = nullptr;
    nufft_status st = make_3d_plan(&p, n1, n2, n3, n_pts, x, y, z, eps, dtype, s);
    if (st) return st;
    st = from_hip(exec_3d(p, in, out, type1, sign, s));
    (void)hipStreamSynchronize(s);
    delete p;
    return st;
}

nufft_status nufft3d_exec(int64_t n_pts, const double *x_dev, const double *y_dev, const double *z_dev, int64_t n1,
                          int64_t n2, int64_t n3, const void *C, void *f, double eps, nufft_dtype dtype, void *stream)
{
    if (!C || !f) return NUFFT_ERR_INVALID_ARG;
    return oneshot_3d(n_pts, x_dev, y_dev, z_dev, n1, n2, n3, C, f, 0, -1, eps, dtype, (hipStream_t)stream);
}

nufft_status nufft3d_type1_exec(int64_t n_pts, const double *x_dev, const double *y_dev, const double *z_dev,
                                int64_t n1, int64_t n2, int64_t n3, const void *c, void *C, int sign, double eps,
                                nufft_dtype dtype, void *stream)
{
    if (!c || !C || (sign != 1 && sign != -1)) return NUFFT_ERR_INVALID_ARG;
    return oneshot_3d(n_pts, x_dev, y_dev, z_dev, n1, n2, n3, c, C, 1, sign, eps, dtype, (hipStream_t)stream);
}

nufft_status nufft3d_plan(nufft_plan_t *out, int64_t n1, int64_t n2, int64_t n3, int64_t n_pts, const double *x_dev,
                          const double *y_dev, const double *z_dev, double eps, nufft_dtype dtype, void *stream)
{
    if (!out) return NUFFT_ERR_INVALID_ARG;
    return make_3d_plan(out, n1, n2, n3, n_pts, x_dev, y_dev, z_dev, eps, dtype, (hipStream_t)stream);
}

nufft_status nufft3d_plan_exec(nufft_plan_t plan, const void *C, void *f, void *stream)
{
    if (!plan || plan->kind != PLAN_3D || !C || !f) return NUFFT_ERR_INVALID_ARG;
    plan->last = (hipStream_t)stream;
    return from_hip(exec_3d(plan, C, f, 0, -1, (hipStream_t)stream));
}

nufft_status nufft3d_plan_type1(nufft_plan_t plan, const void *c, void *C, int sign, void *stream)
{
    if (!plan || plan->kind != PLAN_3D || !c || !C || (sign != 1 && sign != -1)) return NUFFT_ERR_INVALID_ARG;
    plan->last = (hipStream_t)stream;
    return from_hip(exec_3d(plan, c, C, 1, sign, (hipStream_t)stream));
}

nufft_status nufft2d3_exec(int64_t n_pts, const double *x_dev, const double *y_dev, int64_t n_freq,
                           const double *w1_dev, const double *w2_dev, int64_t n1, int64_t n2, const void *c,
                           void *f, double eps, nufft_dtype dtype, void *stream)
{
    if (n_pts < 1 || n_freq < 1 || n1 < 1 || n2 < 1 || !x_dev || !y_dev || !w1_dev || !w2_dev || !c || !f)
        return NUFFT_ERR_INVALID_ARG;
    if (dtype != NUFFT_C64 && dtype != NUFFT_C128) return NUFFT_ERR_INVALID_ARG;
    if (n_pts > (int64_t(1) << 30) || n_freq > (int64_t(1) << 30)) return NUFFT_ERR_UNSUPPORTED;
    nufft_status st;
    if (!eps_ok(eps, dtype, &st)) return st;
    hipStream_t s = (hipStream_t)stream;
    st = dtype == NUFFT_C64 ? type3_2d<float>(n_pts, x_dev, y_dev, n_freq, w1_dev, w2_dev, n1, n2, c, f, eps, dtype, s)
                            : type3_2d<double>(n_pts, x_dev, y_dev, n_freq, w1_dev, w2_dev, n1, n2, c, f, eps, dtype,
                                               s);
    if (st != NUFFT_OK) (void)hipStreamSynchronize(s);
    return st;
}

nufft_status nufft2d_plan(nufft_plan_t *out, int64_t n1, int64_t n2, int64_t n_pts, const double *x_dev,
                          const double *y_dev, double eps, nufft_dtype dtype, uint32_t flags, void *stream)
{
    if (!out) return NUFFT_ERR_INVALID_ARG;
    *out = nullptr;
    if (n1 < 1 || n2 < 1 || n_pts < 1 || !x_dev || !y_dev) return NUFFT_ERR_INVALID_ARG;
    if (dtype != NUFFT_C64 && dtype != NUFFT_C128) return NUFFT_ERR_INVALID_ARG;
    if (flags & ~(uint32_t)(NUFFT_FLAG_FIX_GAMMA_HALF | NUFFT_FLAG_NO_AUTOTUNE)) return NUFFT_ERR_INVALID_ARG;
    if (n_pts > (int64_t(1) << 30)) return NUFFT_ERR_UNSUPPORTED;
    nufft_status st;
    if (!eps_ok(eps, dtype, &st)) return st;
    int gx = 16, gy = 16;
    while (gx < n1) gx <<= 1;
    while (gy < n2) gy <<= 1;
    if (gx > 2048 || gy > 2048) return NUFFT_ERR_UNSUPPORTED;
    Plan *p = new (std::nothrow) Plan();
    if (!p) return NUFFT_ERR_ALLOC;
    p->kind = PLAN_2D;
    p->dtype = dtype;
    p->flags = flags;
    p->N1 = n1;
    p->N2 = n2;
    p->N = n1 * n2;
    p->M = n_pts;
    p->eps = eps;
    p->Gx = gx;
    p->Gy = gy;
    p->L = (int64_t)gx * gy;
    hipStream_t s = (hipStream_t)stream;
    st = dtype == NUFFT_C64 ? build_2d<float>(p, x_dev, y_dev, s) : build_2d<double>(p, x_dev, y_dev, s);
    if (st != NUFFT_OK) {
        (void)hipStreamSynchronize(s);
        delete p;
        return st;
    }
    p->last = s;
    *out = p;
    return NUFFT_OK;
}

nufft_status nufft2d_exec(nufft_plan_t plan, void *C, void *f, int adjoint, void *stream)
{
    if (!plan || plan->kind != PLAN_2D || !C || !f || (adjoint != 0 && adjoint != 1)) return NUFFT_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    plan->last = s;
    hipError_t e;
    if (plan->dtype == NUFFT_C64) {
        const Args2D<float> a = args_2d<float>(plan);
        e = adjoint ? fused_2d_adj<float>(a, (const float2 *)f, (float2 *)C, 1, s)
                    : fused_2d<float>(a, (const float2 *)C, (float2 *)f, s);
    } else {
        const Args2D<double> a = args_2d<double>(plan);
        e = adjoint ? fused_2d_adj<double>(a, (const double2 *)f, (double2 *)C, 1, s)
                    : fused_2d<double>(a, (const double2 *)C, (double2 *)f, s);
    }
    return from_hip(e);
}

nufft_status nufft2d_type1_exec(nufft_plan_t plan, const void *c, void *F, int sign, void *stream)
{
    if (!plan || plan->kind != PLAN_2D || !c || !F || (sign != 1 && sign != -1)) return NUFFT_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    plan->last = s;
    if (plan->dtype == NUFFT_C64)
        return from_hip(fused_2d_adj<float>(args_2d<float>(plan), (const float2 *)c, (float2 *)F, sign, s));
    return from_hip(fused_2d_adj<double>(args_2d<double>(plan), (const double2 *)c, (double2 *)F, sign, s));
}

nufft_status nufft_batch_plan(nufft_plan_t *out, int batch, const int64_t *n_modes, const int64_t *n_pts,
                              const double *const *x_dev, double eps, nufft_dtype dtype, uint32_t flags,
                              void *stream)
{
    if (!out) return NUFFT_ERR_INVALID_ARG;
    *out = nullptr;
    if (batch < 1 || !n_modes || !n_pts || !x_dev) return NUFFT_ERR_INVALID_ARG;
    if (dtype != NUFFT_C64 && dtype != NUFFT_C128) return NUFFT_ERR_INVALID_ARG;
    if (flags & ~(uint32_t)(NUFFT_FLAG_FIX_GAMMA_HALF | NUFFT_FLAG_NO_AUTOTUNE | NUFFT_FLAG_BATCH_PERSISTENT))
        return NUFFT_ERR_INVALID_ARG;
    for (int b = 0; b < batch; ++b) {
        if (n_modes[b] < 1 || n_pts[b] < 1 || !x_dev[b]) return NUFFT_ERR_INVALID_ARG;
        if (n_modes[b] > (int64_t(1) << 20) || n_pts[b] > (int64_t(1) << 30)) return NUFFT_ERR_UNSUPPORTED;
    }
    nufft_status st;
    if (!eps_ok(eps, dtype, &st)) return st;
    Plan *p = new (std::nothrow) Plan();
    if (!p) return NUFFT_ERR_ALLOC;
    p->kind = PLAN_BATCH;
    p->dtype = dtype;
    p->flags = flags;
    p->eps = eps;
    hipStream_t s = (hipStream_t)stream;
    st = dtype == NUFFT_C64 ? build_batch<float>(p, batch, n_modes, n_pts, x_dev, s)
                            : build_batch<double>(p, batch, n_modes, n_pts, x_dev, s);
    if (st != NUFFT_OK) {
        (void)hipStreamSynchronize(s);
        delete p;
        return st;
    }
    p->L = p->bgrid;
    p->last = s;
    *out = p;
    return NUFFT_OK;
}

nufft_status nufft_batch_exec(nufft_plan_t plan, const void *const *c, void *const *f, void *stream)
{
    if (!plan || plan->kind != PLAN_BATCH || !c || !f) return NUFFT_ERR_INVALID_ARG;
    for (size_t b = 0; b < plan->children.size(); ++b)
        if (!c[b] || !f[b]) return NUFFT_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    plan->last = s;
    nufft_status st = plan->dtype == NUFFT_C64 ? batch_upload_ptrs<float>(plan, c, f, s)
                                               : batch_upload_ptrs<double>(plan, c, f, s);
    if (st) return st;
    return from_hip(plan->dtype == NUFFT_C64 ? batch_run<float>(plan, plan->bmode, plan->bgrid, s)
                                             : batch_run<double>(plan, plan->bmode, plan->bgrid, s));
}

nufft_status nufft_plan_info(nufft_plan_t plan, int *K, double *gamma, int64_t *grid)
{
    if (!plan) return NUFFT_ERR_INVALID_ARG;
    if (K) *K = plan->K;
    if (gamma) *gamma = plan->gamma;
    if (grid) *grid = plan->L;
    return NUFFT_OK;
}

nufft_status nufft_plan_tuning(nufft_plan_t plan, int *schedule, int *n_schedules)
{
    if (!plan) return NUFFT_ERR_INVALID_ARG;
    if (schedule) *schedule = plan->sched;
    if (n_schedules) *n_schedules = (plan->kind == PLAN_1D && plan->tw1r8) ? 3 : 1;
    return NUFFT_OK;
}

nufft_status nufft_debug_set_schedule(nufft_plan_t plan, int schedule)
{
    int n = 0;
    if (!plan || nufft_plan_tuning(plan, nullptr, &n) != NUFFT_OK || schedule < 0 || schedule >= n)
        return NUFFT_ERR_INVALID_ARG;
    plan->sched = schedule;
    return NUFFT_OK;
}

nufft_status nufft_debug_set_buckets(nufft_plan_t plan, int enable, int *has)
{
    if (!plan || plan->kind != PLAN_1D) return NUFFT_ERR_INVALID_ARG;
    plan->buckets_off = enable ? 0 : 1;
    if (has) *has = plan->bdst ? 1 : 0;
    return NUFFT_OK;
}

nufft_status nufft_plan_perm(nufft_plan_t plan, int32_t *perm_host)
{
    if (!plan || plan->kind != PLAN_1D || !perm_host) return NUFFT_ERR_INVALID_ARG;
    if (hipMemcpy(perm_host, plan->perm, plan->M * sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess)
        return NUFFT_ERR_HIP;
    return NUFFT_OK;
}

nufft_status nufft_batch_status(nufft_plan_t plan, int64_t *timeouts, void *stream)
{
    if (!plan || plan->kind != PLAN_BATCH || !timeouts) return NUFFT_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    BatchCtl *ctl = (BatchCtl *)plan->bctl;
    int h = 0;
    NUFFT_HIP_CHECK(hipMemcpyAsync(&h, &ctl->timeouts, sizeof(int), hipMemcpyDeviceToHost, s));
    NUFFT_HIP_CHECK(hipStreamSynchronize(s));
    if (h != 0) NUFFT_HIP_CHECK(hipMemsetAsync(&ctl->timeouts, 0, sizeof(int), s));
    NUFFT_HIP_CHECK(hipStreamSynchronize(s));
    *timeouts = h;
    return NUFFT_OK;
}

nufft_status nufft_debug_batch_wait(nufft_plan_t plan, int64_t spin_limit, int unreachable)
{
    if (!plan || plan->kind != PLAN_BATCH || spin_limit < 0) return NUFFT_ERR_INVALID_ARG;
    plan->spin_limit = spin_limit;
    plan->wait_unreachable = unreachable != 0;
    return NUFFT_OK;
}

// Waits for the plan's own stream only (unless it is capturing), then frees.
// The calls run in relaxed capture mode: another stream of this thread or
// process may be capturing a graph meanwhile, and waiting for or freeing
// memory that the capture does not use must not disturb it.
nufft_status nufft_destroy(nufft_plan_t plan)
{
    if (!plan) return NUFFT_OK;
    hipStreamCaptureMode mode = hipStreamCaptureModeRelaxed;
    const bool swapped = hipThreadExchangeStreamCaptureMode(&mode) == hipSuccess;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(plan->last, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone)
        (void)hipStreamSynchronize(plan->last);
    (void)hipGetLastError();
    delete plan;
    if (swapped) (void)hipThreadExchangeStreamCaptureMode(&mode);
    return NUFFT_OK;
}

nufft_status nufft_plan_profile(nufft_plan_t plan, int enable, int reserve)
{
    if (!plan || reserve < 0) return NUFFT_ERR_INVALID_ARG;
    plan->prof.on = enable != 0;
    plan->prof.used = 0;
    while ((int)plan->prof.pool.size() < reserve) {
        Profiler::Rec r;
        if (hipEventCreate(&r.a) != hipSuccess) return NUFFT_ERR_HIP;
        if (hipEventCreate(&r.b) != hipSuccess) { (void)hipEventDestroy(r.a); return NUFFT_ERR_HIP; }
        r.name = "";
        plan->prof.pool.push_back(r);
    }
    return NUFFT_OK;
}

nufft_status nufft_plan_profile_read(nufft_plan_t plan, int index, char *name, int name_len, int *calls,
                                     double *total_ms)
{
    if (!plan || index < 0 || !name || name_len < 1 || !calls || !total_ms) return NUFFT_ERR_INVALID_ARG;
    Profiler &pr = plan->prof;
    // distinct names in order of first appearance
    std::vector<const char *> names;
    for (size_t i = 0; i < pr.used; ++i) {
        bool seen = false;
        for (const char *n : names) seen = seen || std::strcmp(n, pr.pool[i].name) == 0;
        if (!seen) names.push_back(pr.pool[i].name);
    }
    if (index >= (int)names.size()) return NUFFT_ERR_INVALID_ARG;
    const char *want = names[index];
    int cnt = 0;
    double tot = 0.0;
    for (size_t i = 0; i < pr.used; ++i) {
        if (std::strcmp(pr.pool[i].name, want) != 0) continue;
        if (hipEventSynchronize(pr.pool[i].b) != hipSuccess) return NUFFT_ERR_HIP;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, pr.pool[i].a, pr.pool[i].b) != hipSuccess) return NUFFT_ERR_HIP;
        tot += ms;
        ++cnt;
    }
    std::strncpy(name, want, (size_t)name_len - 1);
    name[name_len - 1] = 0;
    *calls = cnt;
    *total_ms = tot;
    return NUFFT_OK;
}

const char *nufft_status_string(nufft_status status)
{
    switch (status) {
    case NUFFT_OK: return "ok";
    case NUFFT_ERR_INVALID_ARG: return "invalid argument";
    case NUFFT_ERR_UNSUPPORTED: return "unsupported request";
    case NUFFT_ERR_ALLOC: return "allocation failed";
    case NUFFT_ERR_NONFINITE: return "non-finite sample coordinate";
    case NUFFT_ERR_HIP: return "HIP runtime error";
    default: return "unknown status";
    }
}

nufft_status nufft_debug_fail_alloc(int64_t n)
{
    alloc_countdown.store(n < 0 ? -1 : (long long)n, std::memory_order_relaxed);
    return NUFFT_OK;
}

nufft_status nufft_choose_rank(double eps, double gamma, int *K)
{
    if (!K || !(eps > 0.0 && eps < 1.0) || !(gamma >= 0.0 && gamma <= 0.5)) return NUFFT_ERR_INVALID_ARG;
    const int k = choose_rank(eps, gamma);
    if (k < 0) return NUFFT_ERR_UNSUPPORTED;
    *K = k;
    return NUFFT_OK;
}

nufft_status nufft_bessel_coefficients(double gamma, int K, double *b_host)
{
    if (!b_host || K < 1 || K > 64 || !(gamma >= 0.0 && gamma <= 0.5)) return NUFFT_ERR_INVALID_ARG;
    bessel_b(gamma, K, b_host);
    return NUFFT_OK;
}

}  // extern "C"

// ---- entry points still to be implemented --------------------------------
extern "C" {







}  // extern "C"
