"""GPU parity on the oversampled grids between powers of two (Sec. 2.3,
"Oversampling"): L = 3 * 2^k and 5 * 2^k, whose column transforms take one
radix-3 or radix-5 stage before power-of-two transforms.  Each column length
the kernels offer is planned explicitly (nufft2_plan_grid) and its type II,
adjoint, type I and x-derivative are checked against the FP64 direct sums
(the bar of Sec. 2.4: 4 eps ||c||_1, element by element on all rows at the
small size, on sampled rows and modes above)."""
import numpy as np
import pytest
import torch

from oracle import lowrank as Lr
from oracle import nudft as D
from paper_1701_04492_amd import workloads as W

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1701_04492_amd")
DEV = torch.device("cuda:0")
C64, C128 = torch.complex64, torch.complex128
EPS = {C64: 1e-6, C128: 1e-12}


def _t(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).to(DEV)


# (dtype, N, grid, M, samples): the grid's column length L2 = P Q in the comment
CASES = [
    (C64, 20000, 24576, 30000, "iid"),          # 192 = 3 x 64, L1 = 128; every row checked
    (C128, 20000, 24576, 30000, "iid"),
    (C64, 70000, 98304, 1 << 16, "jitter"),     # 384 = 3 x 128
    (C128, 70000, 98304, 1 << 16, "iid"),
    (C64, 600000, 786432, 1 << 18, "iid"),      # 768 = 3 x 256
    (C64, 1200000, 1572864, 1 << 20, "iid"),    # 1536 = 3 x 512, L1 = 1024
    (C128, 1200000, 1572864, 1 << 18, "jitter"),
    (C64, 70000, 81920, 40000, "iid"),          # 320 = 5 x 64
    (C128, 300000, 327680, 1 << 17, "iid"),     # 640 = 5 x 128
    (C64, 1000000, 1310720, 1 << 20, "jitter"),  # 1280 = 5 x 256
    (C128, 1000000, 1310720, 1 << 18, "iid"),
]


def _samples(rng, M, kind):
    return W.iid_samples(rng, M) if kind == "iid" else W.jittered_samples(rng, M)


@pytest.mark.parametrize("dtype,N,grid,M,kind", CASES)
def test_mixed_grid_against_oracle(dtype, N, grid, M, kind):
    print("mixed grid", dtype, "N=%d L=%d M=%d %s" % (N, grid, M, kind), flush=True)
    rng = W.rng_for(95)
    x = _samples(rng, M, kind)
    c, g = W.complex_normal(rng, N), W.complex_normal(rng, M)
    eps = EPS[dtype]
    plan = P.nufft2_plan(_t(x, torch.float64), N, eps, dtype, grid=grid)
    assert plan.grid == grid
    # gamma and K are those of this grid: X_j = (L x_j - s_j) N / L
    _, _, d = D.grid_assign(x, grid)
    assert plan.gamma == pytest.approx(np.abs(d).max() * N / grid, rel=1e-12, abs=1e-15)
    assert plan.K == Lr.choose_K(eps, plan.gamma)
    ct, gt = _t(c, dtype), _t(g, dtype)
    cc, gg = ct.cpu().numpy().astype(np.complex128), gt.cpu().numpy().astype(np.complex128)
    f = P.nufft2_exec(plan, ct).cpu().numpy()
    gc, gx = P.nufft2_backward(plan, ct, gt)
    t1 = P.nufft1_exec(plan, gt, sign=-1).cpu().numpy()
    gc, gx = gc.cpu().numpy(), gx.cpu().numpy()
    if N * M <= 6e8:
        rows, ks = np.arange(M), np.arange(N)
    else:
        rows = np.unique(np.concatenate([rng.choice(M, 96, replace=False), [0, M - 1]]))
        ks = np.unique(np.concatenate([rng.choice(N, 48, replace=False), [0, N - 1]]))
    err_f = np.abs(f[rows] - D.nudft2(x[rows], cc)).max() / np.abs(cc).sum()
    err_a = np.abs(gc[ks] - D.nudft1(x, gg, N, k=ks, sign=+1)).max() / np.abs(gg).sum()
    err_1 = np.abs(t1[ks] - D.nudft1(x, gg, N, k=ks, sign=-1)).max() / np.abs(gg).sum()
    xr = rows[:512]
    ref_x = D.grad_x(x[xr], cc, gg[xr])
    bound = 4 * eps * np.abs(gg[xr]) * 2 * np.pi * (np.arange(N) * np.abs(cc)).sum()
    err_x = (np.abs(gx[xr] - ref_x) / bound).max()
    print("   K=%d gamma=%.4f type II %.2e adjoint %.2e type I %.2e dL/dx/bound %.2e"
          % (plan.K, plan.gamma, err_f, err_a, err_1, err_x), flush=True)
    assert np.all(np.isfinite(f)) and np.all(np.isfinite(gc)) and np.all(np.isfinite(gx))
    assert err_f <= 4 * eps and err_a <= 4 * eps and err_1 <= 4 * eps and err_x <= 1.0


def test_mixed_grid_lowers_K():
    """A finer grid shrinks the perturbations N (x_j - s_j / L): gamma and K do not
    grow from L = N through 1.25 N and 1.5 N to 2 N, and 2 N needs fewer ranks than N."""
    N, M = 1 << 16, 1 << 16
    x = W.iid_samples(W.rng_for(96), M)
    xt = _t(x, torch.float64)
    ks = {L: P.nufft2_plan(xt, N, 1e-6, C64, P.NUFFT_FLAG_NO_AUTOTUNE, grid=L).K
          for L in (1 << 16, 5 << 14, 3 << 15, 1 << 17)}
    print("K per grid", ks, flush=True)
    assert ks[1 << 16] >= ks[5 << 14] >= ks[3 << 15] >= ks[1 << 17]
    assert ks[1 << 16] > ks[1 << 17]


def test_mixed_grid_bucketed_graph_replay():
    """A 3 * 2^k grid with the destination-bucketed layout: forward and backward captured in
    one HIP graph; every replay, with eager work between replays, gives the eager bits."""
    N, grid, M = 1200000, 1572864, 1 << 20
    rng = W.rng_for(97)
    x = W.iid_samples(rng, M)
    ct = _t(W.complex_normal(rng, N), C64)
    gt = _t(W.complex_normal(rng, M), C64)
    plan = P.nufft2_plan(_t(x, torch.float64), N, 1e-6, C64, grid=grid)
    assert plan.grid == grid and P.nufft_debug_set_buckets(plan, True)
    f = torch.empty(M, dtype=C64, device=DEV)
    gc = torch.empty(N, dtype=C64, device=DEV)
    gx = torch.empty(M, dtype=torch.float64, device=DEV)
    P.nufft2_exec(plan, ct, f)
    P.nufft2_backward(plan, ct, gt, gc, gx)
    torch.cuda.synchronize()
    ref = (f.clone(), gc.clone(), gx.clone())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        P.nufft2_exec(plan, ct, f)
        P.nufft2_backward(plan, ct, gt, gc, gx)
    for rep in range(3):
        for t in (f, gc, gx):
            t.zero_()
        _ = (gt.abs() + 1).sum().item()   # eager work between replays
        graph.replay()
        torch.cuda.synchronize()
        assert all(torch.equal(a, b) for a, b in zip((f, gc, gx), ref)), rep


@pytest.mark.parametrize("dtype", [C64, C128])
@pytest.mark.parametrize("M", [1, 7, 1000])
def test_mixed_grid_edge_cases(dtype, M):
    """N = L on a 3 * 2^k grid (gamma up to 1/2), tiny sample counts, and samples on the
    edges of the period (0, just below 1, negative and beyond 1, the wrap sample s = L):
    every row and mode against the direct sums."""
    N = grid = 24576
    rng = W.rng_for(98)
    x = rng.random(M) * 1.5 - 0.25
    edges = np.array([0.0, 1.0 - 1e-12, -0.25, 1.25, (grid - 0.5) / grid, 0.5 / grid, 1.0 / 3.0])
    x[:min(M, edges.size)] = edges[:min(M, edges.size)]
    c, g = W.complex_normal(rng, N), W.complex_normal(rng, M)
    eps = EPS[dtype]
    plan = P.nufft2_plan(_t(x, torch.float64), N, eps, dtype, grid=grid)
    assert plan.grid == grid
    ct, gt = _t(c, dtype), _t(g, dtype)
    cc, gg = ct.cpu().numpy().astype(np.complex128), gt.cpu().numpy().astype(np.complex128)
    f = P.nufft2_exec(plan, ct).cpu().numpy()
    a = P.nufft1_exec(plan, gt, sign=+1).cpu().numpy()
    t1 = P.nufft1_exec(plan, gt, sign=-1).cpu().numpy()
    err_f = np.abs(f - D.nudft2(x, cc)).max() / np.abs(cc).sum()
    err_a = np.abs(a - D.nudft1(x, gg, N, sign=+1)).max() / np.abs(gg).sum()
    err_1 = np.abs(t1 - D.nudft1(x, gg, N, sign=-1)).max() / np.abs(gg).sum()
    print("   M=%d K=%d type II %.2e adjoint %.2e type I %.2e" % (M, plan.K, err_f, err_a, err_1), flush=True)
    assert err_f <= 4 * eps and err_a <= 4 * eps and err_1 <= 4 * eps
