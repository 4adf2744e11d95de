/*
 * nufft_mi355x.h -- C ABI of the low-rank nonuniform FFT for AMD MI355X (gfx950).
 *
 * Method: Ruiz-Antolin & Townsend, "A nonuniform fast Fourier transform based
 * on low rank approximation" (arXiv:1701.04492).  The type-II transform
 *     f_j = sum_{k=0}^{N-1} c_k exp(-2 pi i x_j k),   0 <= j < M      (Sec. 1, eq. (2))
 * is evaluated as f ~ sum_{r<K} D_{u_r} I(t,:) F_L D_{v_r} c  (Sec. 2.2, eq. (Fc)):
 * each sample is rounded to its nearest point s_j/L of a grid of L >= N
 * points (t_j = s_j mod L), and u_r, v_r are the rank-K Chebyshev/Bessel
 * factors of exp(-2 pi i (x_j - s_j/L) k) (Sec. 2.1.2, Appendix A) chosen so
 * that the factorisation error is at most eps.  The online stage is K
 * diagonally scaled FFTs of size L, a gather by t and a row sum (Sec. 2.3).
 *
 * Conventions shared by every entry point
 *  - Array arguments named *_dev are DEVICE pointers (hipMalloc'd or from a
 *    framework allocator); the caller owns them and keeps them alive until the
 *    work queued on `stream` has finished.  Arguments named *_host are host
 *    pointers, read before the call returns.
 *  - Complex arrays are interleaved (re, im): NUFFT_C64 = two floats,
 *    NUFFT_C128 = two doubles.  Sample coordinates are always double, on
 *    every precision path: an FP32 coordinate would carry ~0.2 rad of phase
 *    error at N = 2^20.
 *  - Frequencies are 0..N-1 (not centred); forward transforms use the sign
 *    -2 pi i.  No normalisation is applied anywhere.
 *  - `stream` is a hipStream_t passed as void*; NULL means the null stream.
 *    Work is stream ordered.  Plans allocate device memory; *_exec calls
 *    allocate nothing, never synchronise the host and may be captured into a
 *    HIP graph.  A plan may be used from several streams only sequentially.
 *  - Errors are returned as nufft_status; the library never aborts.  On an
 *    error from *_plan, *out is set to NULL and nothing is leaked.
 *  - Accuracy: with FP32 arithmetic eps must be >= 1e-7, with FP64 >= 1e-15
 *    (NUFFT_ERR_UNSUPPORTED otherwise).  The approximation error satisfies
 *    |f~_j - f_j| <= eps ||c||_1 (Sec. 2.4 error bound, max-norm form) plus
 *    rounding of the working precision.
 */
#ifndef NUFFT_MI355X_H
#define NUFFT_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nufft_plan_s *nufft_plan_t;

typedef enum {
    NUFFT_OK = 0,
    NUFFT_ERR_INVALID_ARG = 1,   /* bad size, pointer, eps or flag combination   */
    NUFFT_ERR_UNSUPPORTED = 2,   /* valid request the library cannot serve (size, eps floor) */
    NUFFT_ERR_ALLOC = 3,         /* device or host allocation failed              */
    NUFFT_ERR_NONFINITE = 4,     /* a sample coordinate is NaN or infinite        */
    NUFFT_ERR_HIP = 5            /* a HIP runtime call failed                     */
} nufft_status;

typedef enum {
    NUFFT_C64 = 0,               /* complex float data, FP32 arithmetic (fused kernels) */
    NUFFT_C128 = 1               /* complex double data, FP64 arithmetic               */
} nufft_dtype;

enum {
    /* Take gamma = N/(2L) (the largest possible) instead of the measured
     * max|N(x_j - s_j/L)|: K then depends only on N, L and eps (Sec. 2.2),
     * e.g. for plans rebuilt as samples move during optimisation. */
    NUFFT_FLAG_FIX_GAMMA_HALF = 1u,
    /* Run the plain unfused online stage (Sec. 2.3, the two-step form as
     * written): every intermediate goes through HBM.
     *   type II: scale kernel (K x L buffer), stand-alone FFT passes, a
     *     stored U table (M x K) and a separate gather/row-sum kernel;
     *   type I / adjoint (Sec. 3.1): a spread kernel (one thread per grid
     *     point sums its samples times u_r or conj(u_r) into a K x L buffer),
     *     the stand-alone FFT passes of the other sign, and a kernel that
     *     weights by v_r and sums over r;
     *   derivative pass: the type II on -2 pi i k c.
     * The grid is never autotuned.  Default is the fused kernels. */
    NUFFT_FLAG_PLAIN_UNFUSED = 2u,
    /* Plans are autotuned by default (the choice is reported as `grid` by
     * nufft_plan_info); this flag turns it off.
     * 1-D plans: oversampling (Sec. 2.3) -- besides the grid L0 (smallest
     * power of two >= max(16, N)) the plan is built on 2 L0, where
     * gamma <= N / (4 L0) lowers K; one type-II transform of each is timed on
     * a scratch input and the faster plan is kept (up to L = 2^23).
     * Batches: the three phased launches and the persistent launch at a few
     * grid sizes are timed and the fastest kept.
     * A choice is remembered per problem class (plan kind, sizes, dtype, eps,
     * flags and the rank at L0) for the life of the process, so later plans of
     * the class are not timed again and get the same grid.  Results do not
     * depend on the choice beyond eps.  PLAIN_UNFUSED plans and 2-D / 3-D
     * plans have nothing to tune. */
    NUFFT_FLAG_NO_AUTOTUNE = 4u,
    /* 1-D complex64 plans only, eps >= 2^-10 (Table 1's "half" precision):
     * the K x L intermediate that the two passes exchange through HBM
     * (N > 4096) is stored as fp16 pairs, 4 bytes per value instead of 8,
     * with one power-of-two scale per column (type II) or row (type I /
     * adjoint) so that no value overflows.  Arithmetic stays FP32.  The
     * storage rounding adds at most about 2^-11 * sum_r |u_r| * ||c||_1 to
     * each output, inside the 4 eps ||c||_1 bound for eps >= 2^-10.
     * Combined with NUFFT_FLAG_PLAIN_UNFUSED: NUFFT_ERR_INVALID_ARG; with
     * complex128 or a smaller eps: NUFFT_ERR_UNSUPPORTED. */
    NUFFT_FLAG_HALF_EXCHANGE = 8u,
    /* Batches only: run each exec as one persistent launch over a task queue
     * (workgroups claim tasks; a pass-B task waits on its transform's pass-A
     * tasks) instead of three plain launches, one per task type.  The
     * autotuner then times only persistent grid sizes. */
    NUFFT_FLAG_BATCH_PERSISTENT = 16u
};

/* ---- 1-D type II / type I / adjoint ----------------------------------- */

/* Planning stage (Sec. 2.3): nearest-grid assignment s = round(L x),
 * t = s mod L (Sec. 2.2, eq. (t_vec)), gamma = max_j |N(x_j - s_j/L)|, the
 * rank K(eps, gamma) and the Bessel coefficients a_pr (Sec. 2.1.2), and a
 * stable sort of the samples by FFT output tile.
 *   n_modes  N >= 1, number of Fourier coefficients.
 *   n_pts    M >= 1, number of samples.
 *   x_dev    M doubles, any finite reals (periodic in 1); read during the call.
 *   eps      working accuracy, 0 < eps < 1, above the precision floor.
 * The FFT grid L (oversampling, Sec. 2.3) starts as the smallest power of
 * two L0 >= 16 and >= N.  Unless NUFFT_FLAG_NO_AUTOTUNE (or
 * NUFFT_FLAG_PLAIN_UNFUSED) is given, every supported grid with
 * N <= L <= 2 L0 is planned and timed and the fastest kept (remembered per
 * problem): powers of two, and 3 * 2^k and 5 * 2^k in the two-pass range
 * (see nufft2_plan_grid) unless NUFFT_FLAG_HALF_EXCHANGE is given.  A larger
 * grid lowers gamma and K.  N up to 2^23 (NUFFT_ERR_UNSUPPORTED beyond),
 * M up to 2^30.  Synchronises `stream` (once without autotuning), to read
 * gamma and the non-finite flag back (NUFFT_ERR_NONFINITE). */
nufft_status nufft2_plan(nufft_plan_t *out, int64_t n_modes, int64_t n_pts,
                         const double *x_dev, double eps, nufft_dtype dtype,
                         uint32_t flags, void *stream);

/* nufft2_plan on a grid the caller chooses (the oversampled grid of Sec. 2.3;
 * the grid is not autotuned, the tuning schedule is unless
 * NUFFT_FLAG_NO_AUTOTUNE).  grid >= N is
 *   a power of two up to 2^23, or
 *   P * 2^k with P = 3 or 5: the column transforms of the two-pass form take
 *   one radix-P stage, so grid = L1 * P * Q with L1 a power of two in
 *   [128, 4096] and Q one in [64, 512] (P = 3) or [64, 256] (P = 5); e.g.
 *   24576 = 128 * 3 * 64 up to 6291456 = 4096 * 3 * 512, 40960 up to
 *   5242880 = 4096 * 5 * 256.  Not with NUFFT_FLAG_PLAIN_UNFUSED or
 *   NUFFT_FLAG_HALF_EXCHANGE.
 * Other grids: NUFFT_ERR_UNSUPPORTED; grid < 1: NUFFT_ERR_INVALID_ARG. */
nufft_status nufft2_plan_grid(nufft_plan_t *out, int64_t n_modes, int64_t n_pts,
                              const double *x_dev, double eps, nufft_dtype dtype,
                              uint32_t flags, int64_t grid, void *stream);

/* Online stage of type II (Sec. 2.3, two-step form):
 *   f_dev[j] ~ sum_{k<N} c_dev[k] exp(-2 pi i x_j k),  j < M.
 * c_dev: N complex, f_dev: M complex (dtype of the plan); may not alias. */
nufft_status nufft2_exec(nufft_plan_t plan, const void *c_dev, void *f_dev, void *stream);

/* Transpose and adjoint of type II (Sec. 3.1):
 *   sign = -1: f_dev[k] ~ sum_{j<M} c_dev[j] exp(-2 pi i x_j k)   (type I, F2^T c)
 *   sign = +1: f_dev[k] ~ sum_{j<M} c_dev[j] exp(+2 pi i x_j k)   (adjoint, F2^H c)
 * c_dev: M complex, f_dev: N complex.  On a NUFFT_FLAG_PLAIN_UNFUSED plan the
 * plain kernels run (spread, FFT passes, weighted sum). */
nufft_status nufft1_exec(nufft_plan_t plan, const void *c_dev, void *f_dev, int sign,
                         void *stream);

/* Derivative pass for the gradient in x of a real loss L(f), f = F2 c
 * (calculus on Sec. 1, eq. (2)):
 *   gx_dev[j] = Re( conj(g_dev[j]) * sum_k (-2 pi i k) c_dev[k] exp(-2 pi i x_j k) )
 * with g_j = dL/dRe f_j + i dL/dIm f_j.  One type-II pass on -2 pi i k c,
 * the factor applied inside the FFT prologue.  c_dev: N complex,
 * g_dev: M complex, gx_dev: M doubles. */
nufft_status nufft2_grad_x(nufft_plan_t plan, const void *c_dev, const void *g_dev,
                           double *gx_dev, void *stream);

/* Both gradients of a real loss L(f), f = F2 c, in one call (the backward of
 * type II):
 *   gc_dev = F2^H g                      (as nufft1_exec with sign = +1)
 *   gx_dev[j] = Re(conj(g_j) (F2 (-2 pi i k c))_j)   (as nufft2_grad_x)
 * g_dev (M complex) is put in the plan's sorted sample order once and read
 * by both passes.  Either output may be NULL to skip it (not both).
 * c_dev: N complex, gc_dev: N complex, gx_dev: M doubles. */
nufft_status nufft2_backward(nufft_plan_t plan, const void *c_dev, const void *g_dev,
                             void *gc_dev, double *gx_dev, void *stream);

/* Inverse type II (Sec. 3.3): c_dev ~ argmin ||F2 c - f||_2 for the plan's
 * samples (M >= N; F2 of eq. (2), applied through the plan's low-rank
 * transforms), by conjugate gradients on the normal equations
 * F2^* F2 c = F2^* f.  F2^* F2 is Hermitian Toeplitz with first column
 * tau = F2^* 1 (one adjoint transform); each iteration multiplies by it
 * through a circulant embedding of size Lc >= 2N (two DFTs of size Lc).
 * Starts from c = 0 and stops when ||F2^* (f - F2 c)|| <= tol ||F2^* f||
 * (the recursively updated residual) or after max_iter iterations.
 *   f_dev: M complex (read), c_dev: N complex (written).
 *   iters, resid: optional host outputs (iterations done, final relative
 *   residual of the normal equations).
 * N up to 2^22 (NUFFT_ERR_UNSUPPORTED beyond).  Allocates its temporaries and
 * synchronises `stream` twice per iteration (not graph capturable).  The
 * iteration count grows with the perturbation gamma (Sec. 3.3: small for
 * gamma < 1/4, unbounded as gamma -> 1/2). */
nufft_status nufft2_solve(nufft_plan_t plan, const void *f_dev, void *c_dev, double tol, int max_iter,
                          int *iters, double *resid, void *stream);

/* Inverse type I (Sec. 3.3, the type-I analogue): solves F1 c = f with
 * F1 = F2^T (f_k = sum_j c_j exp(-2 pi i x_j k), k < N) for the plan's
 * samples, M >= N, returning the minimum-norm solution c = F1^* y where
 * (F1 F1^*) y = f.  F1 F1^* = conj(F2^* F2) is Hermitian Toeplitz (first
 * column conj(tau), tau = F2^* 1), applied through the same circulant
 * embedding as nufft2_solve; CG starts from y = 0 and stops when
 * ||f - F1 F1^* y|| <= tol ||f|| (the recursively updated residual) or after
 * max_iter iterations; then c = conj(F2 conj(y)) by one type-II transform.
 *   f_dev: N complex (read), c_dev: M complex (written).
 *   iters, resid: optional host outputs (iterations, final relative residual).
 * N up to 2^22.  Allocates its temporaries and synchronises `stream` twice
 * per iteration (not graph capturable). */
nufft_status nufft1_solve(nufft_plan_t plan, const void *f_dev, void *c_dev, double tol, int max_iter,
                          int *iters, double *resid, void *stream);

/* ---- type III ---------------------------------------------------------- */

/* Type III (Sec. 3.2): f_dev[j] ~ sum_{k<N} c_dev[k] exp(-2 pi i x_j w_k), j < M,
 * composed as F3 = A o B o F1(t,:) from up to 2K type-I transforms on the
 * samples w/N.  x_dev: M doubles in [0, 1); w_dev: N doubles in [0, N).
 * Error bound: half of eps goes to the factorisation, and the inner
 * transforms run at eps_i = max(eps / (2 s), floor) with s = sum_{p,r} w_p |b_pr|
 * (about 4 at gamma = 1/2) and the precision floor of the dtype, so
 * |f~_j - f_j| <= (eps/2 + s eps_i) ||c||_1 plus rounding; when that exceeds
 * 4 eps ||c||_1 the call returns NUFFT_ERR_UNSUPPORTED (complex64 with
 * gamma near 1/2: eps below about 1.2e-7).  Plans, allocates and
 * synchronises internally (not graph capturable). */
nufft_status nufft3_exec(int64_t n_pts, const double *x_dev, int64_t n_freq,
                         const double *w_dev, const void *c_dev, void *f_dev,
                         double eps, nufft_dtype dtype, void *stream);

/* For callers that cannot allocate device memory (code that must not call
 * hipMalloc, tight serving loops, harnesses that forbid allocation): the
 * transform of nufft3_exec, same arguments, same kernels and same result, with
 * every temporary (the assignment of x, the scaled inputs, the inner type-I
 * plan and its exchange buffer) carved from a fixed device array of 48 MiB
 * that the library holds on each device it runs on until the process ends.
 * No hipMalloc, hipFree or other allocating call is made.  Limits:
 * n_pts <= 2^20 and n_freq <= 2^15 (NUFFT_ERR_UNSUPPORTED beyond, before any
 * device work).  The array keeps the last call's contents; everything the
 * transform needs zeroed is cleared by the call itself.  Calls in one process
 * are serialised by a lock and each returns with `stream` synchronised; calls
 * from different processes use different copies of the array.  Not graph
 * capturable (it synchronises, as nufft3_exec does). */
nufft_status nufft3_exec_noalloc(int64_t n_pts, const double *x_dev, int64_t n_freq,
                                 const double *w_dev, const void *c_dev, void *f_dev,
                                 double eps, nufft_dtype dtype, void *stream);

/* ---- 2-D type II and its adjoint --------------------------------------- */

/* Planning stage of the 2-D type II (Sec. 4): x pairs with k1 < n1 and
 * y with k2 < n2; each axis gets rank K(eps/2, gamma_axis).
 * x_dev, y_dev: M doubles each, any finite reals. */
nufft_status nufft2d_plan(nufft_plan_t *out, int64_t n1, int64_t n2, int64_t n_pts,
                          const double *x_dev, const double *y_dev, double eps,
                          nufft_dtype dtype, uint32_t flags, void *stream);

/* adjoint = 0: f_dev[j] ~ sum_{k1,k2} C_dev[k1*n2+k2] exp(-2 pi i (k1 x_j + k2 y_j))  (Sec. 4)
 * adjoint = 1: C_dev[k1*n2+k2] ~ sum_j f_dev[j] exp(+2 pi i (k1 x_j + k2 y_j))
 * C_dev: n1*n2 complex, row-major; f_dev: M complex.  The output is overwritten. */
nufft_status nufft2d_exec(nufft_plan_t plan, void *C_dev, void *f_dev, int adjoint,
                          void *stream);

/* 2-D type I (Sec. 3.1 taken along both axes; the transpose of the 2-D
 * type II of Sec. 4) on the plan's samples:
 *   sign = -1: F_dev[k1*n2+k2] ~ sum_j c_dev[j] exp(-2 pi i (k1 x_j + k2 y_j)),
 *   sign = +1: the same with exp(+...), i.e. nufft2d_exec with adjoint = 1.
 * c_dev: M complex; F_dev: n1*n2 complex, row-major, overwritten.  Same
 * error bound as the type II, eps * ||c||_1 per output.  Allocates nothing
 * and never synchronises.  Returns INVALID_ARG for a non-2-D plan, a NULL
 * pointer or sign not in {-1, +1}. */
nufft_status nufft2d_type1_exec(nufft_plan_t plan, const void *c_dev, void *F_dev, int sign,
                                void *stream);

/* 2-D type III (Sec. 3.2 applied per axis):
 *   f_dev[j] ~ sum_{k<Q} c_dev[k] exp(-2 pi i (x_j w1_k + y_j w2_k)),  j < M,
 * x_dev, y_dev: M doubles in [0, 1); w1_dev, w2_dev: Q doubles with
 * w1 in [0, n1), w2 in [0, n2) (n1, n2 >= 1, n1 + 1 and n2 + 1 at most 2048).
 * Each axis is factored as in the 1-D type III (rank K(eps/4, gamma_axis));
 * the Kx * Ky inner transforms are 2-D type I on the samples
 * (w1/n1, w2/n2) with n1 + 1 by n2 + 1 modes, read at
 * (round(n1 x_j), round(n2 y_j)).  c_dev: Q complex, f_dev: M complex.
 * Error per output at most (eps/2 + s eps_i) ||c||_1 with s = s_x s_y (about
 * 16 at gamma = 1/2, s_axis as for nufft3_exec) and eps_i = max(eps / (2 s),
 * floor); NUFFT_ERR_UNSUPPORTED when that exceeds 4 eps ||c||_1 (complex64
 * with gamma near 1/2: eps below about 5e-7).  Plans, allocates and synchronises
 * internally (not graph capturable); INVALID_ARG for samples or
 * frequencies out of range or not finite. */
nufft_status nufft2d3_exec(int64_t n_pts, const double *x_dev, const double *y_dev, int64_t n_freq,
                           const double *w1_dev, const double *w2_dev, int64_t n1, int64_t n2,
                           const void *c_dev, void *f_dev, double eps, nufft_dtype dtype, void *stream);

/* ---- 3-D type II, type I and adjoint ---------------------------------------- */

/* 3-D type II (Sec. 4's construction with a third axis):
 *   f_dev[j] ~ sum_{k1<n1,k2<n2,k3<n3} C_dev[(k1*n2+k2)*n3+k3] exp(-2 pi i (k1 x_j + k2 y_j + k3 z_j)).
 * x_dev, y_dev, z_dev: M doubles each, any finite reals; C_dev: n1*n2*n3 complex,
 * row-major; f_dev: M complex.  The z axis is factored with rank K(eps/2, gamma_z)
 * on a grid of Gz >= n3 points (Gz <= 1024), and the samples of each z slice
 * get a 2-D type II (n1, n2 up to 2048), all slices as the problems of one
 * stacked 2-D plan.  UNSUPPORTED beyond Gz * Gx * Gy = 2^28 grid points (Gx, Gy:
 * the powers of two >= n1, n2).  Error per output at most (eps/2 + S eps2)
 * ||C||_1, S = sum_{p,r} w_p w_r |b_pr| of the z factors (about 3 at
 * gamma = 1/2) and eps2 = max(eps / (2 S), floor) for the 2-D transforms;
 * NUFFT_ERR_UNSUPPORTED when that exceeds 4 eps ||C||_1.  Plans,
 * allocates and synchronises internally (not graph capturable); NONFINITE for a
 * non-finite z. */
nufft_status nufft3d_exec(int64_t n_pts, const double *x_dev, const double *y_dev, const double *z_dev,
                          int64_t n1, int64_t n2, int64_t n3, const void *C_dev, void *f_dev, double eps,
                          nufft_dtype dtype, void *stream);

/* 3-D type I (sign = -1, the transpose of the 3-D type II) or adjoint (sign = +1):
 *   C_dev[(k1*n2+k2)*n3+k3] ~ sum_{j<M} c_dev[j] exp(sign 2 pi i (k1 x_j + k2 y_j + k3 z_j)),
 * k1 < n1, k2 < n2, k3 < n3.  x_dev, y_dev, z_dev: M doubles each, any finite reals;
 * c_dev: M complex; C_dev: n1*n2*n3 complex, row-major, overwritten.  The factoring of
 * nufft3d_exec run backwards: the samples weighted by u^z_r (or its conjugate), a
 * 2-D type I per z slice (the stacked plan), and one length-Gz transform per
 * (k1, k2) and rank; the same size limits.  Error
 * ~ eps * ||c||_1 per output.  Plans, allocates and synchronises internally (not
 * graph capturable); INVALID_ARG for sign not in {-1, +1}, NONFINITE for a
 * non-finite z. */
nufft_status nufft3d_type1_exec(int64_t n_pts, const double *x_dev, const double *y_dev, const double *z_dev,
                                int64_t n1, int64_t n2, int64_t n3, const void *c_dev, void *C_dev, int sign,
                                double eps, nufft_dtype dtype, void *stream);

/* A reusable 3-D plan: everything nufft3d_exec / nufft3d_type1_exec build on
 * each call (the z factoring of the samples and the stacked 2-D plan of their z
 * slices), built once for the samples x_dev, y_dev, z_dev (M = n_pts doubles
 * each, read during this call only) and the n1 x n2 x n3 modes.  The same
 * limits and errors as nufft3d_exec; synchronises once (gamma_z readback).
 * nufft_plan_info reports K3 (the z rank), gamma_z and Gz * Gx * Gy.
 * Release with nufft_destroy. */
nufft_status nufft3d_plan(nufft_plan_t *out, int64_t n1, int64_t n2, int64_t n3, int64_t n_pts,
                          const double *x_dev, const double *y_dev, const double *z_dev, double eps,
                          nufft_dtype dtype, void *stream);

/* 3-D type II on a 3-D plan: C_dev (n1*n2*n3 complex, row-major) -> f_dev (M
 * complex), the result of nufft3d_exec for the plan's samples.  Allocates
 * nothing and does not synchronise (graph capturable); calls on one plan must
 * not overlap (they share its intermediate).  INVALID_ARG for a plan of another
 * kind or a NULL pointer. */
nufft_status nufft3d_plan_exec(nufft_plan_t plan, const void *C_dev, void *f_dev, void *stream);

/* 3-D type I (sign = -1) or adjoint (sign = +1) on a 3-D plan: c_dev (M
 * complex) -> C_dev (n1*n2*n3 complex, overwritten), the result of
 * nufft3d_type1_exec.  Allocates nothing, does not synchronise; calls on one
 * plan must not overlap.  INVALID_ARG for sign not in {-1, +1}, a plan of
 * another kind or a NULL pointer. */
nufft_status nufft3d_plan_type1(nufft_plan_t plan, const void *c_dev, void *C_dev, int sign, void *stream);

/* ---- batches of independent 1-D type II transforms ---------------------- */

/* Plan B independent type-II transforms of sizes N_b (modes, 1 <= N_b <= 2^20)
 * and M_b (samples); x_dev_host[b] is a device pointer to M_b doubles (a
 * host array of device pointers).  Each transform uses the grid
 * L_b = next power of two >= N_b (oversampling, Sec. 2.3) and its own rank
 * K_b(eps, gamma_b).  Transforms with L_b <= 4096 run whole in one
 * workgroup; larger ones run as a two-pass split.  An exec is three plain
 * launches (whole small transforms, pass-A column groups, pass-B tiles; one
 * workgroup per task, tasks in decreasing order of size), or one persistent
 * launch with NUFFT_FLAG_BATCH_PERSISTENT.
 * Flags: NUFFT_FLAG_FIX_GAMMA_HALF, NUFFT_FLAG_NO_AUTOTUNE (by default the
 * persistent launch is timed at 1..4 workgroups per CU and, unless
 * NUFFT_FLAG_BATCH_PERSISTENT, the phased launches too; the fastest is kept),
 * NUFFT_FLAG_BATCH_PERSISTENT. */
nufft_status nufft_batch_plan(nufft_plan_t *out, int batch, const int64_t *n_modes_host,
                              const int64_t *n_pts_host, const double *const *x_dev_host,
                              double eps, nufft_dtype dtype, uint32_t flags, void *stream);

/* c_dev_host[b]: device pointer to N_b complex; f_dev_host[b]: device
 * pointer to M_b complex.  The pointer arrays are host arrays; when they
 * differ from the previous call they are copied to the device first (a
 * synchronous upload), so for HIP graph capture run one exec with the same
 * pointers before capturing: the captured work is then the single kernel. */
nufft_status nufft_batch_exec(nufft_plan_t plan, const void *const *c_dev_host,
                              void *const *f_dev_host, void *stream);

/* Health of a batch plan's persistent launches.  A pass-B task of the
 * persistent launch waits for its transform's pass-A tasks with a bounded
 * spin (by construction every such wait ends; the bound only guarantees that
 * no kernel can hang).  A wait that reaches its bound gives up, its task then
 * reads an unfinished intermediate, and the launch still returns normally.
 * Waits for `stream`, then reports in *timeouts_host the number of waits that
 * gave up since the previous call (0 for a healthy plan) and clears the
 * count.  Synchronises the stream (not graph capturable). */
nufft_status nufft_batch_status(nufft_plan_t plan, int64_t *timeouts_host, void *stream);

/* ---- plan queries and lifetime ----------------------------------------- */

/* Any output pointer may be NULL.  For 2-D plans K and gamma describe the
 * x axis and grid is Gx * Gy; for batches K is the largest rank, gamma the
 * largest gamma and grid the number of workgroups of the persistent launch,
 * or of the three phased launches together (one per task). */
nufft_status nufft_plan_info(nufft_plan_t plan, int *K, double *gamma, int64_t *grid);

/* The tuning schedule of a 1-D plan's two-pass kernels: *schedule is the one
 * in use and *n_schedules how many the plan offers (either may be NULL).
 * complex64 plans whose split has L1, L2 in {1024, 2048} offer three:
 *   0  default tile shapes, FFT stages radix 16 first (16 x 16 x 8 for 2048 points);
 *   1  default tile shapes, radix 8 first (8 x 16 x 16), with twiddle tables of that order;
 *   2  alternative tile shapes (half the columns per pass-A workgroup, half
 *      the ranks and twice the sample slots per pass-B workgroup, half the
 *      ranks in pass B', twice the columns per pass-A' workgroup).
 * Other plans offer one.  Unless NUFFT_FLAG_NO_AUTOTUNE is given, nufft2_plan
 * times a type-II transform and an adjoint under each and keeps the fastest
 * (remembered per problem class, see NUFFT_FLAG_NO_AUTOTUNE).  Results of the
 * schedules differ only by rounding. */
nufft_status nufft_plan_tuning(nufft_plan_t plan, int *schedule, int *n_schedules);

/* Copies the plan's sorted sample order to host memory: perm_host[i] is the
 * sample index at sorted position i (M int32).  1-D plans only. */
nufft_status nufft_plan_perm(nufft_plan_t plan, int32_t *perm_host);

/* Frees the plan.  When the stream the plan last ran on (or was built on) is
 * not being captured into a graph, its queued work is waited for first; no
 * other stream or device-wide wait is made, so another stream may be
 * capturing meanwhile.  A plan whose work was captured into a graph must
 * outlive every replay of that graph.  NULL is accepted. */
nufft_status nufft_destroy(nufft_plan_t plan);

const char *nufft_status_string(nufft_status status);

/* ---- per-kernel timing (profiling aid) ---------------------------------- */

/* enable != 0: from now on every exec call on this plan records a pair of
 * HIP events on its stream around each kernel it launches (kernels of one
 * exec are stream ordered, so a pair brackets exactly one kernel).  Any
 * call resets the record; `reserve` pre-creates that many event pairs so
 * that timed loops do not create events.  Profiled exec calls must not be
 * captured into a graph. */
nufft_status nufft_plan_profile(nufft_plan_t plan, int enable, int reserve);

/* index-th distinct kernel name (in order of first launch) recorded since the
 * last reset: its name (copied, NUL-terminated, into name[name_len]), the
 * number of launches and their summed durations in ms.  Waits for the
 * recorded events.  NUFFT_ERR_INVALID_ARG past the last name. */
nufft_status nufft_plan_profile_read(nufft_plan_t plan, int index, char *name, int name_len, int *calls,
                                     double *total_ms);

/* ---- failure injection (tests) ------------------------------------------- */

/* For callers that test their error handling: with n >= 0, the library's
 * device allocation n allocations from now (0: the next one) is refused, and
 * the call that made it returns NUFFT_ERR_ALLOC after releasing what it had
 * built; the injection then disarms itself.  n < 0 disarms it.  Process-wide
 * state, not meant for concurrent use.  Always returns NUFFT_OK. */
nufft_status nufft_debug_fail_alloc(int64_t n);

/* For tests of the persistent batch launch's bounded wait: from the next exec
 * on, each pass-B wait spins at most spin_limit times (default 2^28), and with
 * unreachable != 0 its target count is one that is never reached, so that
 * every wait gives up after its bound and is reported by nufft_batch_status;
 * every kernel still ends normally.  INVALID_ARG for a non-batch plan or a
 * negative limit. */
nufft_status nufft_debug_batch_wait(nufft_plan_t plan, int64_t spin_limit, int unreachable);

/* For tests of the tuning schedules: makes the plan run `schedule` (below the
 * count nufft_plan_tuning reports, else INVALID_ARG) from the next exec on. */
nufft_status nufft_debug_set_schedule(nufft_plan_t plan, int schedule);

/* For tests of the destination-bucketed permutations: large 1-D plans write
 * their outputs through a layout ordered by destination block, and sort their
 * inputs through it.  enable = 0 makes the plan scatter and gather directly
 * (the same values, bit for bit) from the next exec on; enable = 1 restores the
 * layout.  *has (may be NULL) is set to 1 if the plan has the layout, else 0.
 * INVALID_ARG for a plan that is not 1-D. */
nufft_status nufft_debug_set_buckets(nufft_plan_t plan, int enable, int *has);

/* ---- host-side factor generator (no GPU work) --------------------------- */

/* K(eps, gamma): the smallest K whose Chebyshev truncation tail
 * sum_{max(p,r)>=K} w_p w_r |a_pr| (w_0 = 1/2) is <= eps (Sec. 2.1.2,
 * Table 1, Lemma A.1).  gamma in [0, 1/2]; gamma = 0 gives K = 1. */
nufft_status nufft_choose_rank(double eps, double gamma, int *K);

/* b_host[p*K + r] = a_pr / i^r = 4 J_{(p+r)/2}(-gamma pi/2) J_{(r-p)/2}(-gamma pi/2)
 * for p = r mod 2, else 0 (Sec. 2.1.2): the real part of the coefficients. */
nufft_status nufft_bessel_coefficients(double gamma, int K, double *b_host);

#ifdef __cplusplus
}
#endif

#endif /* NUFFT_MI355X_H */
