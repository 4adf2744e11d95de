"""GPU checks of the destination-bucketed permutations of large 1-D plans.

Pass B writes its outputs (type II, and the x-derivative's per-sample sums)
through a layout ordered by destination block, and the backward and type-I
passes sort their sample-ordered inputs through it.  Only the route of the
values changes: with the layout switched off (direct scatters and gathers)
every result must be the same bit for bit, for every tuning schedule; sampled
rows are also checked against the oracle within the error bound of Sec. 2.4.
"""
import numpy as np
import pytest
import torch

from oracle import nudft as D
from paper_1701_04492_amd import workloads as W

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1701_04492_amd")
DEV = torch.device("cuda:0")
C64, C128 = torch.complex64, torch.complex128
EPS = {C64: 1e-6, C128: 1e-12}


def _has_layout(M, dtype):
    """The plan's rule: blocks of 2^12 to 2^14 samples (2^13 in FP64), about 256 of them,
    and the layout only for 16 to 1024 blocks."""
    top = 14 if dtype == C64 else 13
    b = 12
    while b < top and (M >> b) > 256:
        b += 1
    return 16 <= (M + (1 << b) - 1) >> b <= 1024


def _t(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).to(DEV)


def _run(plan, ct, gt):
    f = P.nufft2_exec(plan, ct)
    gc, gx = P.nufft2_backward(plan, ct, gt)
    t1 = P.nufft1_exec(plan, gt, sign=-1)
    torch.cuda.synchronize()
    return f, gc, gx, t1


# (dtype, N, M): below the 16-block threshold (no layout), 16 blocks with a ragged
# last one, blocks of 2^12, 2^13 and 2^14 samples, many samples per output tile, and
# the full 2^22 size
CASES = [
    (C64, 20000, 15 * (1 << 12)),
    (C64, 1 << 16, 15 * (1 << 12) + 1),
    (C64, 1 << 18, 16 * (1 << 14) + 777),
    (C64, 1 << 12, 1 << 20),
    (C64, 1 << 20, 1 << 21),
    (C64, 1 << 22, 1 << 22),
    (C128, 3000, 15 * (1 << 12)),
    (C128, 1 << 17, 16 * (1 << 13) + 5),
    (C128, 1 << 21, 1 << 21),
]


@pytest.mark.parametrize("dtype,N,M", CASES)
def test_bucketed_equals_direct(dtype, N, M):
    print("buckets", dtype, "N=%d M=%d" % (N, M), flush=True)
    rng = W.rng_for(90)
    x = rng.random(M)
    c, g = W.complex_normal(rng, N), W.complex_normal(rng, M)
    ct, gt = _t(c, dtype), _t(g, dtype)
    plan = P.nufft2_plan(_t(x, torch.float64), N, EPS[dtype], dtype)
    has = P.nufft_debug_set_buckets(plan, True)
    # (only two-pass plans, grids above 4096 points, permute their outputs)
    assert has == (plan.grid > 4096 and _has_layout(M, dtype)), (plan.grid, has)
    _, nsched = P.nufft_plan_tuning(plan)
    for sched in range(nsched):
        P.nufft_debug_set_schedule(plan, sched)
        P.nufft_debug_set_buckets(plan, True)
        on = _run(plan, ct, gt)
        P.nufft_debug_set_buckets(plan, False)
        off = _run(plan, ct, gt)
        for name, a, b in zip(("f", "dL/dc", "dL/dx", "type I"), on, off):
            assert torch.equal(a, b), (sched, name)
    P.nufft_debug_set_buckets(plan, True)
    f, gc, gx, t1 = _run(plan, ct, gt)
    cc, gg = ct.cpu().numpy().astype(np.complex128), gt.cpu().numpy().astype(np.complex128)
    rows = np.unique(np.concatenate([rng.choice(M, 64, replace=False), [0, M - 1]]))
    kq = np.unique(np.concatenate([rng.choice(N, 24, replace=False), [0, N - 1]]))
    err_f = np.abs(f.cpu().numpy()[rows] - D.nudft2(x[rows], cc)).max() / np.abs(cc).sum()
    err_c = np.abs(gc.cpu().numpy()[kq] - D.nudft1(x, gg, N, k=kq, sign=+1)).max() / np.abs(gg).sum()
    err_1 = np.abs(t1.cpu().numpy()[kq] - D.nudft1(x, gg, N, k=kq, sign=-1)).max() / np.abs(gg).sum()
    ref_x = D.grad_x(x[rows], cc, gg[rows])
    bound = 4 * EPS[dtype] * np.abs(gg[rows]) * 2 * np.pi * (np.arange(N) * np.abs(cc)).sum()
    err_x = (np.abs(gx.cpu().numpy()[rows] - ref_x) / bound).max()
    print("   K=%d type II %.2e dL/dc %.2e type I %.2e dL/dx/bound %.2e" % (plan.K, err_f, err_c, err_1, err_x),
          flush=True)
    assert err_f <= 4 * EPS[dtype] and err_c <= 4 * EPS[dtype] and err_1 <= 4 * EPS[dtype]
    assert err_x <= 1.0
