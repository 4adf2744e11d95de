// Batched type-II transforms in one persistent launch: descriptors and launchers.
#pragma once

#include "kernels.h"

namespace nufft {

enum { BATCH_SMALL = 0, BATCH_PASS_A = 1, BATCH_PASS_B = 2 };

// Everything a task needs about its transform (device copy, one per member).
template <typename R>
struct BatchDesc {
    int64_t N, M, L;
    int L1, L2, n_pass_a;
    const Factors<R> *fac;          // device copy of the member's factors
    const int32_t *t;               // one-pass members: grid index per sample
    const R *X;                     // one-pass members: perturbation per sample
    const uint32_t *keys;           // two-pass members: sorted keys
    const int32_t *perm;
    const R *Xs;
    const int32_t *off;
    cx_t<R> *Y;                     // two-pass intermediate
    const cx_t<R> *tw1, *tw2, *hi, *lo;
};

// Queue state; zero at plan time, restored to zero by the last workgroup of each launch.
struct BatchCtl {
    int next;        // next task to claim
    int exited;      // workgroups that have left
    int timeouts;    // waits that reached their bound (read and cleared by nufft_batch_status)
    int ntransforms;
    int done_a[1];   // per transform: finished pass-A tasks (ntransforms entries)
};

size_t batch_lds_bytes(int L, int L1, int L2, bool fp32);
int batch_threads();
int batch_small_chunk();
int batch_pass_a_cols(int L2);
int batch_pass_b_points();     // grid points per PASS_B task (runs of whole tiles)
// spin_limit: iterations of a pass-B wait before it gives up (counted in
// ctl->timeouts); unreachable != 0 (tests only) makes every wait's target count
// one that is never reached.
template <typename R>
hipError_t batch_launch(const BatchDesc<R> *descs, const int4 *tasks, int ntasks, BatchCtl *ctl,
                        const cx_t<R> *const *cs, cx_t<R> *const *fs, int grid, size_t lds, int64_t spin_limit,
                        int unreachable, hipStream_t s);
// The same work as three plain launches (SMALL, PASS_A, PASS_B tasks; counts[3]),
// tasks laid out in that order, one workgroup per task.
template <typename R>
hipError_t batch_launch_phased(const BatchDesc<R> *descs, const int4 *tasks, const int *counts,
                               const cx_t<R> *const *cs, cx_t<R> *const *fs, size_t lds, hipStream_t s);
template <typename R>
hipError_t batch_set_lds_limit(size_t lds);

}  // namespace nufft
