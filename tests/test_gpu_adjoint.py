"""GPU parity of the type-I / adjoint kernels (Sec. 3.1) and of the gradient
passes behind torch.autograd, against the FP64 oracle."""
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


def _t(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).to(DEV)


def _say(*a):
    print(*a, flush=True)


def check_type1(x, g, N, dtype, sign, kq=None, label=""):
    eps = EPS[dtype]
    _say("type1", label, "N=%d M=%d sign=%d" % (N, x.shape[0], sign), dtype)
    plan = P.nufft2_plan(_t(x, torch.float64), N, eps, dtype)
    gt = _t(g, dtype)
    out = P.nufft1_exec(plan, gt, sign=sign)
    torch.cuda.synchronize()
    out = out.cpu().numpy()
    gg = gt.cpu().numpy().astype(np.complex128)
    if kq is None:
        ref, got = D.nudft1(x, gg, N, sign=sign), out
    else:
        ref, got = D.nudft1(x, gg, N, k=kq, sign=sign), out[kq]
    err = np.abs(got - ref).max() / np.abs(gg).sum()
    _say("   K=%d err/||g||_1 = %.3e" % (plan.K, err))
    assert np.all(np.isfinite(out))
    assert err <= 4 * eps
    return plan, out, err


@pytest.mark.parametrize("dtype", [C64, C128])
@pytest.mark.parametrize("sign", [-1, 1])
@pytest.mark.parametrize("N,M", [(1, 3), (16, 40), (1000, 3001), (4096, 4096), (3000, 200000)])
def test_one_pass(dtype, sign, N, M):
    rng = W.rng_for(30)
    x = rng.random(M) * 2.0 - 0.5
    g = W.complex_normal(rng, M)
    _, _, err = check_type1(x, g, N, dtype, sign, label="one-pass")
    if dtype == C64 and N >= 64:
        # regression gate; a handful of terms does not average the factorisation error down
        assert err < 2e-7


@pytest.mark.parametrize("dtype", [C64, C128])
@pytest.mark.parametrize("sign", [-1, 1])
@pytest.mark.parametrize("N,dist", [(8192, "iid"), (16384, "jitter"), (20000, "iid")])
def test_two_pass(dtype, sign, N, dist):
    x, g = W.type2_case(31, N, N, dist)
    _, _, err = check_type1(x, g, N, dtype, sign, label="two-pass " + dist)
    if dtype == C64:
        assert err < 2e-7


@pytest.mark.parametrize("dtype", [C64, C128])
def test_adjoint_dot_product(dtype):
    """<F2 c, g> = <c, F2^H g> up to the approximation error of both sides."""
    N = 1 << 14
    rng = W.rng_for(32)
    x = rng.random(N)
    c, g = W.complex_normal(rng, N), W.complex_normal(rng, N)
    plan = P.nufft2_plan(_t(x, torch.float64), N, EPS[dtype], dtype)
    f = P.nufft2_exec(plan, _t(c, dtype)).cpu().numpy()
    a = P.nufft1_exec(plan, _t(g, dtype), sign=+1).cpu().numpy()
    lhs, rhs = np.vdot(g, f), np.vdot(a, c)
    assert abs(lhs - rhs) <= 8 * EPS[dtype] * np.abs(c).sum() * np.abs(g).sum()


def test_adjoint_deterministic():
    N = 1 << 16
    x, g = W.type2_case(33, N)
    plan = P.nufft2_plan(_t(x, torch.float64), N, 1e-6, C64)
    gt = _t(g, C64)
    a1 = P.nufft1_exec(plan, gt, sign=+1).cpu()
    a2 = P.nufft1_exec(plan, gt, sign=+1).cpu()
    assert torch.equal(a1, a2)


@pytest.mark.parametrize("dtype", [C64, C128])
@pytest.mark.parametrize("dist", ["iid", "jitter"])
def test_n2p20_sampled(dtype, dist):
    """Type I and adjoint at N = M = 2^20 on both sample distributions of the workload
    (iid uniform, and jittered x_j = (j + U(-1/2, 1/2))/N where every t_j is j or j +- 1)."""
    N = 1 << 20
    x, g = W.type2_case(2, N, N, dist)
    kq = np.sort(np.random.default_rng(5).choice(N, 256, replace=False))
    kq = np.unique(np.concatenate([[0, 1, N // 2, N - 2, N - 1], kq]))
    check_type1(x, g, N, dtype, +1, kq=kq, label="2^20 adjoint " + dist)
    check_type1(x, g, N, dtype, -1, kq=kq, label="2^20 type I " + dist)


def test_n2p23_max_size_sampled():
    """Largest supported grid (N = 2^23, L1 = 4096 tiles): adjoint on sampled outputs."""
    N = 1 << 23
    x, g = W.type2_case(27, N)
    kq = np.sort(np.random.default_rng(6).choice(N, 48, replace=False))
    kq = np.concatenate([[0, 1, N - 1], kq])
    check_type1(x, g, N, C64, +1, kq=kq, label="2^23 adjoint")


# ---- gradients --------------------------------------------------------------

@pytest.mark.parametrize("dist", ["iid", "jitter"])
def test_n2p22_backward_sampled(dist):
    """The backward of the bench step exactly as timed (N = M = 2^22, complex64,
    eps 1e-6, nufft2_backward): dL/dc on sampled modes, dL/dx on sampled samples
    (seeded random ones, every wrap sample, the largest |delta|), and the forward on
    the same samples, for iid and jittered samples."""
    N = 1 << 22
    x, c = W.type2_case(3, N, N, dist)
    g = W.complex_normal(W.rng_for(28), N)
    plan = P.nufft2_plan(_t(x, torch.float64), N, EPS[C64], C64)
    ct, gt = _t(c, C64), _t(g, C64)
    gc, gx = P.nufft2_backward(plan, ct, gt)
    torch.cuda.synchronize()
    gc, gx = gc.cpu().numpy(), gx.cpu().numpy()
    cc, gg = ct.cpu().numpy().astype(np.complex128), gt.cpu().numpy().astype(np.complex128)
    kq = np.sort(np.random.default_rng(11).choice(N, 64, replace=False))
    kq = np.concatenate([[0, 1, N - 1], kq])
    ref_c = D.nudft1(x, gg, N, k=kq, sign=+1)
    err_c = np.abs(gc[kq] - ref_c).max() / np.abs(gg).sum()
    rng = np.random.default_rng(12)
    s, _, d = D.grid_assign(x, N)
    rows = set(rng.choice(N, 64, replace=False).tolist())
    rows.update(np.nonzero(s == N)[0][:16].tolist())
    rows.update(np.argsort(-np.abs(d))[:16].tolist())
    rows = np.array(sorted(rows), dtype=np.int64)
    ref_x = D.grad_x(x[rows], cc, gg[rows])
    bound = 4 * EPS[C64] * np.abs(gg[rows]) * 2 * np.pi * (np.arange(N) * np.abs(cc)).sum()
    f = P.nufft2_exec(plan, ct).cpu().numpy()
    err_f = np.abs(f[rows] - D.nudft2(x[rows], cc)).max() / np.abs(cc).sum()
    _say("2^22 %s backward: K=%d dL/dc err/||g||_1 %.3e, dL/dx max err/bound %.3e, forward err/||c||_1 %.3e"
         % (dist, plan.K, err_c, (np.abs(gx[rows] - ref_x) / bound).max(), err_f))
    assert np.all(np.isfinite(gc)) and np.all(np.isfinite(gx))
    assert err_c <= 4 * EPS[C64]
    assert np.all(np.abs(gx[rows] - ref_x) <= bound)
    assert err_f <= 4 * EPS[C64]


@pytest.mark.parametrize("dtype", [C64, C128])
def test_grad_x_pass(dtype):
    N, M = 4096, 3000
    rng = W.rng_for(34)
    x = rng.random(M)
    c, g = W.complex_normal(rng, N), W.complex_normal(rng, M)
    plan = P.nufft2_plan(_t(x, torch.float64), N, EPS[dtype], dtype)
    ct, gt = _t(c, dtype), _t(g, dtype)
    gx = P.nufft2_grad_x(plan, ct, gt).cpu().numpy()
    cc, gg = ct.cpu().numpy().astype(np.complex128), gt.cpu().numpy().astype(np.complex128)
    ref = D.grad_x(x, cc, gg)
    # |error| <= eps |g_j| 2 pi sum_k k |c_k|  (error bound applied to -2 pi i k c)
    bound = 4 * EPS[dtype] * np.abs(gg) * 2 * np.pi * (np.arange(N) * np.abs(cc)).sum()
    _say("grad_x", dtype, "max err/bound %.3e" % (np.abs(gx - ref) / bound).max())
    assert np.all(np.abs(gx - ref) <= bound)


@pytest.mark.parametrize("dtype", [C64, C128])
def test_many_samples_per_grid_point(dtype):
    """M = 256 N (thousands of samples per output tile): adjoint on sampled k and the
    derivative pass on sampled samples, against the oracle."""
    N, M = 1 << 13, 1 << 21
    rng = W.rng_for(36)
    x = rng.random(M)
    c, g = W.complex_normal(rng, N), W.complex_normal(rng, M)
    plan = P.nufft2_plan(_t(x, torch.float64), N, EPS[dtype], dtype)
    ct, gt = _t(c, dtype), _t(g, dtype)
    cc, gg = ct.cpu().numpy().astype(np.complex128), gt.cpu().numpy().astype(np.complex128)
    gc, gx = P.nufft2_backward(plan, ct, gt)
    # the adjoint's dense tiles are split over several workgroups whose partial rows
    # are added in a fixed order: a second call gives the same bits
    assert torch.equal(gc, P.nufft1_exec(plan, gt, sign=+1))
    assert torch.equal(P.nufft1_exec(plan, gt, sign=-1), P.nufft1_exec(plan, gt, sign=-1))
    kq = np.unique(np.concatenate([rng.choice(N, 40, replace=False), [0, N - 1]]))
    err = np.abs(gc.cpu().numpy()[kq] - D.nudft1(x, gg, N, k=kq, sign=+1)).max() / np.abs(gg).sum()
    rows = np.unique(np.concatenate([rng.choice(M, 300, replace=False), [0, M - 1]]))
    ref = D.grad_x(x[rows], cc, gg[rows])
    bound = 4 * EPS[dtype] * np.abs(gg[rows]) * 2 * np.pi * (np.arange(N) * np.abs(cc)).sum()
    gerr = (np.abs(gx.cpu().numpy()[rows] - ref) / bound).max()
    t1 = P.nufft1_exec(plan, gt, sign=-1).cpu().numpy()
    t1err = np.abs(t1[kq] - D.nudft1(x, gg, N, k=kq, sign=-1)).max() / np.abs(gg).sum()
    _say("M = 256 N", dtype, "adjoint err/||g||_1 %.3e, type I %.3e, grad_x err/bound %.3e" % (err, t1err, gerr))
    assert err <= 4 * EPS[dtype] and t1err <= 4 * EPS[dtype] and gerr <= 1.0


@pytest.mark.parametrize("N,M", [(3000, 2500), (20000, 17000), (1 << 16, 1 << 16)])
@pytest.mark.parametrize("dtype", [C64, C128])
def test_backward_matches_separate_calls(N, M, dtype):
    """nufft2_backward (g sorted once, shared) gives exactly the results of the two separate calls."""
    rng = W.rng_for(35)
    x = rng.random(M)
    c, g = W.complex_normal(rng, N), W.complex_normal(rng, M)
    plan = P.nufft2_plan(_t(x, torch.float64), N, EPS[dtype], dtype)
    ct, gt = _t(c, dtype), _t(g, dtype)
    gc_ref = P.nufft1_exec(plan, gt, sign=+1)
    gx_ref = P.nufft2_grad_x(plan, ct, gt)
    gc, gx = P.nufft2_backward(plan, ct, gt)
    assert torch.equal(gc, gc_ref) and torch.equal(gx, gx_ref)
    gc_only, none_x = P.nufft2_backward(plan, ct, gt, need_x=False)
    none_c, gx_only = P.nufft2_backward(plan, ct, gt, need_c=False)
    assert none_x is None and none_c is None
    assert torch.equal(gc_only, gc_ref) and torch.equal(gx_only, gx_ref)
    _say("backward", N, M, dtype, "identical to separate calls")


def test_autograd_fp64_against_oracle_and_fd():
    """Loss ||f - y||^2 at N = 4096 in FP64: both gradients against the oracle's,
    and the oracle's against central differences of the oracle."""
    N = 4096
    rng = W.rng_for(3)
    x = rng.random(N)
    c, y = W.complex_normal(rng, N), W.complex_normal(rng, N)
    xt = _t(x, torch.float64).requires_grad_(True)
    ct = _t(c, C128).requires_grad_(True)
    yt = _t(y, C128)
    plan = P.nufft2_plan(xt.detach(), N, 1e-12, C128)
    f = P.nufft2(xt, ct, plan)
    loss = ((f - yt).abs() ** 2).sum()
    loss.backward()
    gref = 2.0 * (D.nudft2(x, c) - y)
    gc_ref = D.nudft1(x, gref, N, sign=+1)
    gx_ref = D.grad_x(x, c, gref)
    gc = ct.grad.cpu().numpy()
    gx = xt.grad.cpu().numpy()
    assert np.abs(gc - gc_ref).max() <= 4e-12 * np.abs(gref).sum() + 1e-9
    scale = np.abs(gref) * 2 * np.pi * (np.arange(N) * np.abs(c)).sum()
    assert np.all(np.abs(gx - gx_ref) <= 4e-12 * scale + 1e-8)
    # the oracle's gradient against central differences of the oracle itself
    h = 1e-6 / N
    for j in np.random.default_rng(3).choice(N, 6, replace=False):
        xp, xm = x.copy(), x.copy()
        xp[j] += h
        xm[j] -= h
        fd = (np.sum(np.abs(D.nudft2(xp, c) - y) ** 2) - np.sum(np.abs(D.nudft2(xm, c) - y) ** 2)) / (xp[j] - xm[j])
        assert abs(fd - gx_ref[j]) <= 1e-6 * (abs(gx_ref[j]) + np.abs(gref[j]) * N)


def test_gradcheck_tiny():
    """torch.autograd.gradcheck in FP64 on a tiny transform (eps 1e-14)."""
    N, M = 24, 20
    rng = W.rng_for(35)
    x = _t(rng.random(M), torch.float64).requires_grad_(True)
    c = _t(W.complex_normal(rng, N), C128).requires_grad_(True)
    plan = P.nufft2_plan(x.detach(), N, 1e-14, C128)
    assert torch.autograd.gradcheck(lambda cc: P.nufft2(x.detach(), cc, plan), (c,), eps=1e-6, atol=1e-7)
    # the plan encodes x, so the x-check re-plans at every evaluation
    assert torch.autograd.gradcheck(
        lambda xx: P.nufft2(xx, c.detach(), P.nufft2_plan(xx.detach(), N, 1e-14, C128)), (x,),
        eps=1e-9, atol=1e-5, rtol=1e-4)


@pytest.mark.parametrize("dtype", [C64, C128])
def test_backward_graph_replay(dtype):
    """The fused backward (sort, adjoint, derivative passes) captured in a HIP graph: every
    replay, with eager work between replays, equals the eager result bit for bit."""
    rng = W.rng_for(61)
    N = M = 1 << 16
    x = W.iid_samples(rng, M)
    xt = _t(x, torch.float64)
    c = _t(W.complex_normal(rng, N), dtype)
    g = _t(W.complex_normal(rng, M), dtype)
    plan = P.nufft2_plan(xt, N, EPS[dtype], dtype)
    gc = torch.empty(N, dtype=dtype, device=DEV)
    gx = torch.empty(M, dtype=torch.float64, device=DEV)
    P.nufft2_backward(plan, c, g, gc, gx)
    gc_ref, gx_ref = gc.clone(), gx.clone()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        P.nufft2_backward(plan, c, g, gc, gx)
    for rep in range(3):
        gc.zero_()
        gx.zero_()
        _ = (g.abs() + 1).sum().item()   # eager work between replays
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(gc, gc_ref), rep
        assert torch.equal(gx, gx_ref), rep


@pytest.mark.parametrize("dtype", [C64, C128])
@pytest.mark.parametrize("sign", [-1, 1])
def test_uneven_tiles(dtype, sign):
    """Tiles the per-tile walk of pass B' splits unevenly: one grid point holding 3000
    samples (more than a tile stages in LDS, so the rest of its run is read from
    global memory), 400 points holding 5 copies each, a tile with one sample, long
    stretches of empty tiles and a dense band.  Sampled k against the oracle, and a
    second call gives the same bits."""
    rng = W.rng_for(37)
    x = np.concatenate([
        rng.random(20000) * 0.3,
        np.full(3000, 0.1234567),
        np.repeat(0.3 + rng.random(400) * 0.1, 5),
        [0.7],
        0.75 + rng.random(15000) * 0.05,
    ])
    x = x[rng.permutation(x.shape[0])]
    N = 1 << 15
    g = W.complex_normal(rng, x.shape[0])
    kq = np.unique(np.concatenate([rng.choice(N, 48, replace=False), [0, 1, N // 2, N - 1]]))
    plan, out, _ = check_type1(x, g, N, dtype, sign, kq=kq, label="uneven tiles")
    again = P.nufft1_exec(plan, _t(g, dtype), sign=sign).cpu().numpy()
    assert np.array_equal(out, again)
