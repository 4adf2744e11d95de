"""GPU checks of the C-ABI boundary itself: the plain unfused type I / adjoint
(Sec. 3.1) against the FP64 oracle, conjugated tensor views, the plan/sample
consistency check of the autograd wrapper, the health report of the persistent
batch launch, plan destruction while another stream captures a graph, and the
precision floor of the type III.  Bar: |err| <= 4 eps ||input||_1 per output."""
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
PLAIN = 2


def _t(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).to(DEV)


def _say(*a):
    print(*a, flush=True)


# ---- plain unfused type I / adjoint ---------------------------------------------

@pytest.mark.parametrize("dtype", [C64, C128])
@pytest.mark.parametrize("N,M", [(300, 517), (4096, 5000), (20000, 20000 + 77), (1 << 16, 3000)])
@pytest.mark.parametrize("sign", [-1, 1])
def test_plain_type1_against_oracle(dtype, N, M, sign):
    """One-pass (L <= 4096) and two-pass grids, more and fewer samples than modes."""
    x, _ = W.type2_case(90, N, M)
    g = W.complex_normal(W.rng_for(91), M)
    plan = P.nufft2_plan(_t(x, torch.float64), N, EPS[dtype], dtype, PLAIN)
    gt = _t(g, dtype)
    out = P.nufft1_exec(plan, gt, sign=sign).cpu().numpy()
    gg = gt.cpu().numpy().astype(np.complex128)
    ks = np.unique(np.concatenate([np.random.default_rng(92).choice(N, size=min(N, 400), replace=False),
                                   [0, N - 1]]))
    ref = D.nudft1(x, gg, N, k=ks, sign=sign)
    err = np.abs(out[ks] - ref).max() / np.abs(gg).sum()
    _say("plain type1 sign=%d N=%d M=%d %s K=%d err %.3e" % (sign, N, M, dtype, plan.K, err))
    assert np.all(np.isfinite(out)) and err <= 4 * EPS[dtype]


@pytest.mark.parametrize("dtype", [C64, C128])
def test_plain_matches_fused_adjoint(dtype):
    """The plain and fused adjoints on the same samples agree within the bar (both eps-accurate)."""
    N = 1 << 14
    x, _ = W.type2_case(93, N, N + 5)
    g = W.complex_normal(W.rng_for(94), N + 5)
    xt, gt = _t(x, torch.float64), _t(g, dtype)
    pp = P.nufft2_plan(xt, N, EPS[dtype], dtype, PLAIN)
    pf = P.nufft2_plan(xt, N, EPS[dtype], dtype, P.NUFFT_FLAG_NO_AUTOTUNE)
    a = P.nufft1_exec(pp, gt, sign=+1)
    b = P.nufft1_exec(pf, gt, sign=+1)
    diff = (a - b).abs().max().item() / gt.abs().sum().item()
    _say("plain vs fused adjoint %s: %.3e" % (dtype, diff))
    assert diff <= 8 * EPS[dtype]


@pytest.mark.parametrize("dtype", [C64, C128])
def test_plain_backward_against_oracle(dtype):
    """Both gradients of a real loss on a plain plan: F2^H g and the x-derivative pass."""
    N, M = 5000, 4000
    x, c = W.type2_case(95, N, M)
    g = W.complex_normal(W.rng_for(96), M)
    plan = P.nufft2_plan(_t(x, torch.float64), N, EPS[dtype], dtype, PLAIN)
    ct, gt = _t(c, dtype), _t(g, dtype)
    gc, gx = P.nufft2_backward(plan, ct, gt)
    cc = ct.cpu().numpy().astype(np.complex128)
    gg = gt.cpu().numpy().astype(np.complex128)
    ref_c = D.nudft1(x, gg, N, sign=+1)
    ref_x = D.grad_x(x, cc, gg)
    err_c = np.abs(gc.cpu().numpy() - ref_c).max() / np.abs(gg).sum()
    bound_x = 4 * EPS[dtype] * np.abs(gg) * 2 * np.pi * (np.arange(N) * np.abs(cc)).sum()
    rel_x = (np.abs(gx.cpu().numpy() - ref_x) / bound_x).max()
    _say("plain backward %s: dL/dc err %.3e, dL/dx err / bound %.3f" % (dtype, err_c, rel_x))
    assert err_c <= 4 * EPS[dtype] and rel_x <= 1.0


@pytest.mark.parametrize("dtype", [C64, C128])
def test_plain_autograd_step(dtype):
    """The autograd step (the benchmark's unit) on a plain plan equals the fused plan's within the bar."""
    N = 1 << 13
    x, c = W.type2_case(97, N)
    y = W.complex_normal(W.rng_for(98), N)
    xt, ct, yt = _t(x, torch.float64), _t(c, dtype), _t(y, dtype)
    res = []
    for flags in (PLAIN, P.NUFFT_FLAG_NO_AUTOTUNE):
        plan = P.nufft2_plan(xt, N, EPS[dtype], dtype, flags)
        xg = xt.clone().requires_grad_(True)
        cg = ct.clone().requires_grad_(True)
        loss = torch.view_as_real(P.nufft2(xg, cg, plan) - yt).pow(2).sum()
        loss.backward()
        res.append((cg.grad.clone(), xg.grad.clone()))
    dc = (res[0][0] - res[1][0]).abs().max().item() / res[1][0].abs().max().item()
    dx = (res[0][1] - res[1][1]).abs().max().item() / res[1][1].abs().max().item()
    _say("plain vs fused autograd %s: grad c %.3e, grad x %.3e" % (dtype, dc, dx))
    assert dc < 1e-3 and dx < 1e-3


# ---- conjugated views -------------------------------------------------------------

def test_conjugated_views_are_resolved():
    """c.conj() as input and a loss over f.conj() (torch then hands backward a conjugated g)
    give the results of the materialised tensors, checked against the oracle."""
    N, M = 3000, 2500
    x, c = W.type2_case(99, N, M)
    y = W.complex_normal(W.rng_for(100), M)
    xt, ct, yt = _t(x, torch.float64), _t(c, C128), _t(y, C128)
    plan = P.nufft2_plan(xt, N, 1e-12, C128)
    f = P.nufft2_exec(plan, ct.conj()).cpu().numpy()
    ref = D.nudft2(x, np.conj(c))
    assert np.abs(f - ref).max() <= 4e-12 * np.abs(c).sum()
    # loss = sum Re(conj(f) * w) with a conjugated view of f inside
    w = _t(W.complex_normal(W.rng_for(101), M), C128)
    xg = xt.clone().requires_grad_(True)
    cg = ct.clone().requires_grad_(True)
    fv = P.nufft2(xg, cg, plan)
    (fv.conj() * w).real.sum().backward()
    # dL/dRe f + i dL/dIm f = w (L = Re f . Re w + Im f . Im w)
    gg = w.cpu().numpy()
    ref_c = D.nudft1(x, gg, N, sign=+1)
    ref_x = D.grad_x(x, c, gg)
    err_c = np.abs(cg.grad.cpu().numpy() - ref_c).max() / np.abs(gg).sum()
    bound_x = 4e-12 * np.abs(gg) * 2 * np.pi * (np.arange(N) * np.abs(c)).sum()
    rel_x = (np.abs(xg.grad.cpu().numpy() - ref_x) / bound_x).max()
    _say("conj views: grad c err %.3e, grad x err/bound %.3f" % (err_c, rel_x))
    assert err_c <= 4e-12 and rel_x <= 1.0
    out = torch.empty(M, dtype=C128, device=DEV).conj()
    with pytest.raises(ValueError):
        P.nufft2_exec(plan, ct, out)


def test_autograd_rejects_a_plan_of_other_samples():
    N = 512
    x, c = W.type2_case(102, N)
    xt, ct = _t(x, torch.float64), _t(c, C64)
    plan = P.nufft2_plan(xt, N, 1e-6, C64)
    P.nufft2(xt.clone(), ct, plan)                 # a copy of the planned samples is accepted
    with pytest.raises(ValueError):
        P.nufft2(xt[:-1], ct, plan)                # other samples: a different count
    xt.add_(0.0)   # in-place write: the plan no longer matches x's version
    with pytest.raises(ValueError):
        P.nufft2(xt, ct, plan)


# ---- persistent batch launch: bounded waits are reported ------------------------

def _batch(seed):
    Ns = [700, 9000, 40000, 3000, 70000 // 2]
    rng = W.rng_for(seed)
    xs = [_t(W.iid_samples(rng, n), torch.float64) for n in Ns]
    cs = [_t(W.complex_normal(rng, n), C64) for n in Ns]
    fs = [torch.empty(n, dtype=C64, device=DEV) for n in Ns]
    return Ns, xs, cs, fs


def test_batch_wait_timeouts_are_reported():
    Ns, xs, cs, fs = _batch(103)
    plan = P.nufft_batch_plan(Ns, xs, 1e-6, C64, P.NUFFT_FLAG_BATCH_PERSISTENT | P.NUFFT_FLAG_NO_AUTOTUNE)
    P.nufft_batch_exec(plan, cs, fs)
    assert P.nufft_batch_status(plan) == 0
    ref = [f.clone() for f in fs]
    # every pass-B wait's target made unreachable, a short bound: each gives up, kernels end
    P.nufft_debug_batch_wait(plan, 200, unreachable=True)
    P.nufft_batch_exec(plan, cs, fs)
    n = P.nufft_batch_status(plan)
    _say("forced timeouts reported: %d" % n)
    assert n > 0
    assert P.nufft_batch_status(plan) == 0          # the count was cleared
    P.nufft_debug_batch_wait(plan, 1 << 28, unreachable=False)
    P.nufft_batch_exec(plan, cs, fs)               # the queue state was restored by the last workgroup
    assert P.nufft_batch_status(plan) == 0
    assert all(torch.equal(a, b) for a, b in zip(ref, fs))
    with pytest.raises(P.NufftError):
        P.nufft_debug_batch_wait(plan, -1)


# ---- plan destruction while another stream captures --------------------------------

def test_destroy_during_capture_keeps_the_capture_valid():
    N = 1 << 14
    x, c = W.type2_case(104, N)
    xt, ct = _t(x, torch.float64), _t(c, C64)
    keep = P.nufft2_plan(xt, N, 1e-6, C64)
    doomed = P.nufft2_plan(xt, N, 1e-6, C64)
    P.nufft2_exec(doomed, ct)                      # last used on the current (non-capturing) stream
    f = torch.empty(N, dtype=C64, device=DEV)
    P.nufft2_exec(keep, ct, f)
    torch.cuda.synchronize()
    ref = f.clone()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            P.nufft2_exec(keep, ct, f)
            P.nufft_destroy(doomed)                # not captured, must not disturb the capture
    for rep in range(3):
        f.zero_()
        junk = torch.randn(1 << 18, device=DEV).sum()
        g.replay()
        torch.cuda.synchronize()
        assert junk.isfinite()
        assert torch.equal(f, ref), rep


# ---- type III precision floor --------------------------------------------------

def test_type3_precision_floor():
    """complex64 type III: eps whose composed bound the FP32 inner transforms cannot meet is
    refused; just above it the result meets 4 eps ||c||_1 against the direct sum."""
    M, N = 3000, 2000
    rng = W.rng_for(105)
    x = W.iid_samples(rng, M)
    w = rng.uniform(0, N, N)
    c = W.complex_normal(rng, N)
    xt, wt, ct = _t(x, torch.float64), _t(w, torch.float64), _t(c, C64)
    with pytest.raises(P.NufftError) as e:
        P.nufft3_exec(xt, wt, ct, 1e-7)
    assert e.value.status == 2
    eps = 2e-7
    f = P.nufft3_exec(xt, wt, ct, eps).cpu().numpy()
    cc = ct.cpu().numpy().astype(np.complex128)
    err = np.abs(f - D.nudft3(x, w, cc)).max() / np.abs(cc).sum()
    _say("type3 complex64 eps %g: err %.3e" % (eps, err))
    assert err <= 4 * eps
