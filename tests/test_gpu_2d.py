"""GPU parity of the 2-D type-II transform and its adjoint (Sec. 4) against the
FP64 direct sums, with the bound 4 eps ||C||_1 (eps split in half per axis)."""
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


def _polar(rng, m):
    r, th = 0.5 * rng.random(m), 2 * np.pi * rng.random(m)
    return 0.5 + r * np.cos(th), 0.5 + r * np.sin(th)


def run_2d(x, y, C, dtype, rows=None, kq=None, g=None, label=""):
    n1, n2 = C.shape
    M = x.shape[0]
    eps = EPS[dtype]
    print("2d", label, "n1=%d n2=%d M=%d" % (n1, n2, M), dtype, flush=True)
    plan = P.nufft2d_plan(_t(x, torch.float64), _t(y, torch.float64), n1, n2, eps, dtype)
    Ct = _t(C.ravel(), dtype)
    f = torch.empty(M, dtype=dtype, device=DEV)
    P.nufft2d_exec(plan, Ct, f, 0)
    torch.cuda.synchronize()
    f = f.cpu().numpy()
    Cc = Ct.cpu().numpy().astype(np.complex128).reshape(n1, n2)
    if rows is None:
        ref, got = D.nudft2d(x, y, Cc), f
    else:
        ref, got = D.nudft2d(x[rows], y[rows], Cc), f[rows]
    err = np.abs(got - ref).max() / np.abs(Cc).sum()
    print("   forward err/||C||_1 = %.3e" % err, flush=True)
    assert np.all(np.isfinite(f)) and err <= 4 * eps
    if g is not None:
        gt = _t(g, dtype)
        out = torch.empty(n1 * n2, dtype=dtype, device=DEV)
        P.nufft2d_exec(plan, out, gt, 1)
        torch.cuda.synchronize()
        out = out.cpu().numpy().reshape(n1, n2)
        gg = gt.cpu().numpy().astype(np.complex128)
        if kq is None:
            k1, k2 = np.meshgrid(np.arange(n1), np.arange(n2), indexing="ij")
            k1, k2 = k1.ravel(), k2.ravel()
        else:
            k1, k2 = kq
        ref = D.nudft2d_adj(x, y, gg, k1, k2)
        aerr = np.abs(out[k1, k2] - ref).max() / np.abs(gg).sum()
        print("   adjoint err/||g||_1 = %.3e" % aerr, flush=True)
        assert np.all(np.isfinite(out)) and aerr <= 4 * eps
    return plan


@pytest.mark.parametrize("dtype", [C64, C128])
@pytest.mark.parametrize("n1,n2,M,dist", [(16, 16, 50, "iid"), (32, 24, 500, "polar"), (64, 64, 3000, "polar"),
                                          (200, 130, 4000, "iid"), (5, 300, 700, "iid")])
def test_2d_small(dtype, n1, n2, M, dist):
    rng = W.rng_for(50)
    x, y = _polar(rng, M) if dist == "polar" else (rng.random(M) * 2 - 0.5, rng.random(M))
    C = W.complex_normal(rng, n1 * n2).reshape(n1, n2)
    g = W.complex_normal(rng, M)
    run_2d(x, y, C, dtype, g=g, label=dist)


def test_2d_dot_product():
    rng = W.rng_for(51)
    n1, n2, M = 128, 96, 20000
    x, y = _polar(rng, M)
    C = W.complex_normal(rng, n1 * n2).reshape(n1, n2)
    g = W.complex_normal(rng, M)
    plan = P.nufft2d_plan(_t(x, torch.float64), _t(y, torch.float64), n1, n2, 1e-12, C128)
    f = torch.empty(M, dtype=C128, device=DEV)
    P.nufft2d_exec(plan, _t(C.ravel(), C128), f, 0)
    a = torch.empty(n1 * n2, dtype=C128, device=DEV)
    P.nufft2d_exec(plan, a, _t(g, C128), 1)
    lhs = np.vdot(g, f.cpu().numpy())
    rhs = np.vdot(a.cpu().numpy(), C.ravel())
    assert abs(lhs - rhs) <= 8e-12 * np.abs(C).sum() * np.abs(g).sum()


def test_2d_polar_full_size_sampled():
    """The 1024 x 1024, M = 2^20 polar workload: sampled outputs of both directions."""
    x, y, C = W.polar_case(5)
    rng = np.random.default_rng(52)
    M = x.shape[0]
    r = np.hypot(x - 0.5, y - 0.5)
    # 448 seeded rows, the 64 samples nearest the centre (the densest cells), the ends
    rows = np.unique(np.concatenate([rng.choice(M, 448, replace=False), np.argsort(r)[:64], [0, M - 1]]))
    assert rows.size >= 512
    g = W.complex_normal(W.rng_for(53), M)
    k1 = np.concatenate([[0, 1023, 512, 0, 1023], rng.integers(0, 1024, 256)])
    k2 = np.concatenate([[0, 1023, 511, 1023, 0], rng.integers(0, 1024, 256)])
    kq = (k1, k2)
    plan = run_2d(x, y, C, C64, rows=rows, kq=kq, g=g, label="polar 1024^2")
    assert plan.K == 10


# ---- 2-D type I (nufft2d_type1_exec) ----------------------------------------------

def run_2d_type1(x, y, n1, n2, g, dtype, kq=None, label=""):
    M = x.shape[0]
    eps = EPS[dtype]
    print("2d type1", label, "n1=%d n2=%d M=%d" % (n1, n2, M), dtype, flush=True)
    plan = P.nufft2d_plan(_t(x, torch.float64), _t(y, torch.float64), n1, n2, eps, dtype)
    gt = _t(g, dtype)
    out = P.nufft2d_type1_exec(plan, gt, sign=-1)
    torch.cuda.synchronize()
    out = out.cpu().numpy().reshape(n1, n2)
    gg = gt.cpu().numpy().astype(np.complex128)
    if kq is None:
        k1, k2 = np.meshgrid(np.arange(n1), np.arange(n2), indexing="ij")
        k1, k2 = k1.ravel(), k2.ravel()
    else:
        k1, k2 = kq
    ref = D.nudft2d_adj(x, y, gg, k1, k2, sign=-1)
    err = np.abs(out[k1, k2] - ref).max() / np.abs(gg).sum()
    print("   type-I err/||c||_1 = %.3e" % err, flush=True)
    assert np.all(np.isfinite(out)) and err <= 4 * eps
    return plan, gt


@pytest.mark.parametrize("dtype", [C64, C128])
@pytest.mark.parametrize("n1,n2,M,dist", [(16, 16, 50, "iid"), (32, 24, 500, "polar"), (64, 64, 3000, "polar"),
                                          (200, 130, 4000, "iid"), (5, 300, 700, "iid")])
def test_2d_type1_small(dtype, n1, n2, M, dist):
    rng = W.rng_for(54)
    x, y = _polar(rng, M) if dist == "polar" else (rng.random(M) * 2 - 0.5, rng.random(M))
    g = W.complex_normal(rng, M)
    plan, gt = run_2d_type1(x, y, n1, n2, g, dtype, label=dist)
    # sign +1 of the new entry point is the adjoint of nufft2d_exec, bit for bit
    a1 = P.nufft2d_type1_exec(plan, gt, sign=+1)
    a2 = torch.empty(n1 * n2, dtype=dtype, device=DEV)
    P.nufft2d_exec(plan, a2, gt, 1)
    assert torch.equal(a1, a2)


def test_2d_type1_transpose_identity():
    rng = W.rng_for(55)
    n1, n2, M = 128, 96, 20000
    x, y = _polar(rng, M)
    C = W.complex_normal(rng, n1 * n2)
    g = W.complex_normal(rng, M)
    plan = P.nufft2d_plan(_t(x, torch.float64), _t(y, torch.float64), n1, n2, 1e-12, C128)
    f = torch.empty(M, dtype=C128, device=DEV)
    P.nufft2d_exec(plan, _t(C, C128), f, 0)
    t = P.nufft2d_type1_exec(plan, _t(g, C128), sign=-1).cpu().numpy()
    lhs = np.sum(g * f.cpu().numpy())
    rhs = np.sum(t * C)
    assert abs(lhs - rhs) <= 8e-12 * np.abs(C).sum() * np.abs(g).sum()


def test_2d_type1_polar_full_size_sampled():
    """The 1024 x 1024, M = 2^20 polar workload, type I on sampled outputs."""
    x, y, _ = W.polar_case(5)
    M = x.shape[0]
    rng = np.random.default_rng(56)
    g = W.complex_normal(W.rng_for(57), M)
    kq = (np.concatenate([[0, 1023, 512, 0, 1023], rng.integers(0, 1024, 256)]),
          np.concatenate([[0, 1023, 511, 1023, 0], rng.integers(0, 1024, 256)]))
    run_2d_type1(x, y, 1024, 1024, g, C64, kq=kq, label="polar 1024^2")


def test_2d_type1_bad_sign():
    x = _t(np.linspace(0, 1, 10), torch.float64)
    plan = P.nufft2d_plan(x, x, 16, 16, 1e-6, C64)
    with pytest.raises(P.NufftError):
        P.nufft2d_type1_exec(plan, torch.zeros(10, dtype=C64, device=DEV), sign=0)
