"""MI355X-native low-rank nonuniform FFT (Ruiz-Antolin & Townsend, arXiv:1701.04492).

The transforms run in hand-written HIP kernels for gfx950 behind the C ABI of
``include/nufft_mi355x.h`` (``libnufft_mi355x.so``, built in-tree by
``build.py``).  ``binding`` mirrors the C entry points one to one;
``autograd`` wraps the type-II transform for torch.autograd.
"""
from .binding import (  # noqa: F401
    NUFFT_FLAG_BATCH_PERSISTENT, NUFFT_FLAG_FIX_GAMMA_HALF, NUFFT_FLAG_HALF_EXCHANGE, NUFFT_FLAG_NO_AUTOTUNE,
    NUFFT_FLAG_PLAIN_UNFUSED, NufftError, Plan,
    nufft1_exec, nufft1_solve, nufft2_backward, nufft2_exec, nufft2_grad_x, nufft2_plan, nufft2_solve,
    nufft2d3_exec, nufft2d_exec, nufft2d_plan, nufft2d_type1_exec, nufft3_exec, nufft3_exec_noalloc, nufft3d_exec, nufft3d_plan, nufft3d_plan_exec, nufft3d_plan_type1,
    nufft3d_type1_exec,
    nufft_batch_exec, nufft_batch_plan, nufft_batch_status, nufft_bessel_coefficients, nufft_choose_rank,
    nufft_debug_batch_wait, nufft_debug_fail_alloc, nufft_debug_set_schedule, nufft_debug_set_buckets, nufft_plan_tuning,
    nufft_destroy,
    nufft_plan_info, nufft_plan_perm, nufft_plan_profile, nufft_plan_profile_read, nufft_status_string,
)
from .autograd import NufftTypeII, PlanCache, nufft2  # noqa: F401
