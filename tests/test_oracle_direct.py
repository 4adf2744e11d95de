"""Pins for the direct-sum oracle (CPU only).

Each check fixes the oracle to something other than itself: 50-digit brute
force, closed forms, the uniform DFT, exact identities between the transform
types, and the worked examples printed in the paper's figures.
"""
import json
import os

import mpmath
import numpy as np
import pytest

from oracle import nudft as D

GOLD = os.path.join(os.path.dirname(__file__), "golden")
mpmath.mp.dps = 50


def _mp_sum(phases, coeffs):
    """sum_k coeffs_k * exp(i * 2 pi * phases_k) in 50-digit arithmetic (phases are mpf)."""
    s = mpmath.mpc(0)
    for ph, cc in zip(phases, coeffs):
        s += mpmath.mpc(cc.real, cc.imag) * mpmath.expjpi(2 * ph)
    return complex(s)


def _rand(rng, n):
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


@pytest.mark.parametrize("N,M,seed", [(1, 1, 0), (5, 7, 1), (16, 16, 2), (13, 9, 3)])
def test_type2_vs_mpmath(N, M, seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1.5, 2.5, M)
    c = _rand(rng, N)
    f = D.nudft2(x, c)
    for j in range(M):
        ref = _mp_sum([-mpmath.mpf(x[j]) * k for k in range(N)], c)
        assert abs(f[j] - ref) <= 4e-16 * np.abs(c).sum()


@pytest.mark.parametrize("sign", [-1, 1])
def test_type1_and_adjoint_vs_mpmath(sign):
    rng = np.random.default_rng(11)
    M, N = 11, 9
    x = rng.random(M)
    c = _rand(rng, M)
    f = D.nudft1(x, c, N, sign=sign)
    for k in range(N):
        ref = _mp_sum([sign * mpmath.mpf(x[j]) * k for j in range(M)], c)
        assert abs(f[k] - ref) <= 4e-16 * np.abs(c).sum()


def test_type3_vs_mpmath():
    rng = np.random.default_rng(12)
    M, N = 8, 10
    x = rng.random(M)
    w = rng.uniform(0, N, N)
    c = _rand(rng, N)
    f = D.nudft3(x, w, c)
    for j in range(M):
        ref = _mp_sum([-mpmath.mpf(x[j]) * mpmath.mpf(w[k]) for k in range(N)], c)
        assert abs(f[j] - ref) <= 4e-16 * np.abs(c).sum()


def test_2d_vs_mpmath():
    rng = np.random.default_rng(13)
    n1, n2, M = 4, 5, 6
    x, y = rng.random(M), rng.random(M)
    C = _rand(rng, n1 * n2).reshape(n1, n2)
    f = D.nudft2d(x, y, C)
    for j in range(M):
        ph = [-(mpmath.mpf(x[j]) * k1 + mpmath.mpf(y[j]) * k2) for k1 in range(n1) for k2 in range(n2)]
        ref = _mp_sum(ph, C.ravel())
        assert abs(f[j] - ref) <= 4e-16 * np.abs(C).sum()
    g = _rand(rng, M)
    k1 = np.array([0, 1, 3, 2]); k2 = np.array([0, 4, 1, 2])
    for sign in (+1, -1):     # adjoint and 2-D type I
        a = D.nudft2d_adj(x, y, g, k1, k2, sign=sign)
        for q in range(4):
            ph = [sign * (mpmath.mpf(x[j]) * int(k1[q]) + mpmath.mpf(y[j]) * int(k2[q])) for j in range(M)]
            assert abs(a[q] - _mp_sum(ph, g)) <= 4e-16 * np.abs(g).sum()


def test_2d_type1_is_transpose_and_adjoint_is_conjugate_transpose():
    """sum_j g_j (F C)_j = sum_k C_k (F^T g)_k and <g, F C> = <F^H g, C> (2-D)."""
    rng = np.random.default_rng(17)
    n1, n2, M = 6, 7, 33
    x, y = rng.random(M) * 3 - 1, rng.random(M)
    C = _rand(rng, n1 * n2).reshape(n1, n2)
    g = _rand(rng, M)
    f = D.nudft2d(x, y, C)
    k1, k2 = np.meshgrid(np.arange(n1), np.arange(n2), indexing="ij")
    t1 = D.nudft2d_adj(x, y, g, k1.ravel(), k2.ravel(), sign=-1)
    ad = D.nudft2d_adj(x, y, g, k1.ravel(), k2.ravel(), sign=+1)
    scale = np.abs(C).sum() * np.abs(g).sum()
    assert abs(np.sum(g * f) - np.sum(C.ravel() * t1)) <= 1e-14 * scale
    assert abs(np.vdot(g, f) - np.vdot(ad, C.ravel())) <= 1e-14 * scale
    assert np.abs(t1 - ad).max() > 1e-2          # the two signs differ for generic samples


def test_type3_2d_vs_mpmath():
    rng = np.random.default_rng(18)
    M, Q = 5, 7
    x, y = rng.random(M), rng.random(M)
    w1, w2 = rng.random(Q) * 9.0, rng.random(Q) * 5.0
    c = _rand(rng, Q)
    f = D.nudft3_2d(x, y, w1, w2, c)
    for j in range(M):
        ph = [-(mpmath.mpf(x[j]) * mpmath.mpf(w1[k]) + mpmath.mpf(y[j]) * mpmath.mpf(w2[k])) for k in range(Q)]
        assert abs(f[j] - _mp_sum(ph, c)) <= 4e-16 * np.abs(c).sum()


def test_type3_2d_reduces_to_type2_and_separates():
    """Integer frequencies: the 2-D type II of the coefficients placed at them.  A product
    set of frequencies with a product coefficient: the product of two 1-D type IIIs."""
    rng = np.random.default_rng(19)
    M, n1, n2 = 40, 6, 5
    x, y = rng.random(M), rng.random(M)
    k1, k2 = rng.integers(0, n1, 30), rng.integers(0, n2, 30)
    c = _rand(rng, 30)
    C = np.zeros((n1, n2), np.complex128)
    np.add.at(C, (k1, k2), c)
    f = D.nudft3_2d(x, y, k1.astype(np.float64), k2.astype(np.float64), c)
    assert np.abs(f - D.nudft2d(x, y, C)).max() <= 1e-13 * np.abs(c).sum()
    a1, a2 = rng.random(4) * 7.3, rng.random(3) * 2.9
    ca, cb = _rand(rng, 4), _rand(rng, 3)
    W1, W2 = np.meshgrid(a1, a2, indexing="ij")
    CC = np.outer(ca, cb)
    g = D.nudft3_2d(x, y, W1.ravel(), W2.ravel(), CC.ravel())
    ref = D.nudft3(x, a1, ca) * D.nudft3(y, a2, cb)
    assert np.abs(g - ref).max() <= 1e-13 * np.abs(CC).sum()


def test_3d_vs_mpmath_and_separable():
    rng = np.random.default_rng(20)
    n1, n2, n3, M = 3, 4, 2, 5
    x, y, z = rng.random(M) * 2 - 0.5, rng.random(M), rng.random(M)
    C = _rand(rng, n1 * n2 * n3).reshape(n1, n2, n3)
    f = D.nudft3d(x, y, z, C)
    for j in range(M):
        ph = [-(mpmath.mpf(x[j]) * a + mpmath.mpf(y[j]) * b + mpmath.mpf(z[j]) * c)
              for a in range(n1) for b in range(n2) for c in range(n3)]
        assert abs(f[j] - _mp_sum(ph, C.ravel())) <= 4e-16 * np.abs(C).sum()
    # a product coefficient gives the product of three 1-D type IIs
    a, b, c = _rand(rng, 5), _rand(rng, 3), _rand(rng, 4)
    P3 = np.einsum("i,j,k->ijk", a, b, c)
    g = D.nudft3d(x, y, z, P3)
    assert np.abs(g - D.nudft2(x, a) * D.nudft2(y, b) * D.nudft2(z, c)).max() <= 1e-14 * np.abs(P3).sum()
    # one mode along z: the 2-D type II
    C1 = _rand(rng, 12).reshape(3, 4, 1)
    assert np.abs(D.nudft3d(x, y, z, C1) - D.nudft2d(x, y, C1[:, :, 0])).max() <= 1e-14 * np.abs(C1).sum()


@pytest.mark.parametrize("sign", [-1, +1])
def test_3d_type1_and_adjoint_vs_mpmath(sign):
    rng = np.random.default_rng(21)
    M = 6
    x, y, z = rng.random(M) * 2 - 0.5, rng.random(M), rng.random(M) * 3
    g = _rand(rng, M)
    k1, k2, k3 = np.array([0, 2, 1, 3]), np.array([0, 1, 3, 2]), np.array([0, 1, 2, 4])
    a = D.nudft3d_adj(x, y, z, g, k1, k2, k3, sign=sign)
    for q in range(4):
        ph = [sign * (mpmath.mpf(x[j]) * int(k1[q]) + mpmath.mpf(y[j]) * int(k2[q]) + mpmath.mpf(z[j]) * int(k3[q]))
              for j in range(M)]
        assert abs(a[q] - _mp_sum(ph, g)) <= 4e-16 * np.abs(g).sum()


def test_3d_type1_transpose_adjoint_and_separable():
    """sum_j g_j (F C)_j = sum_k C_k (F^T g)_k and <g, F C> = <F^H g, C> against the 3-D
    type II; samples on a product grid with a product weight give the product of three
    1-D type Is; one z mode at z = 0 gives the 2-D type I."""
    rng = np.random.default_rng(22)
    n1, n2, n3, M = 4, 3, 5, 29
    x, y, z = rng.random(M) * 3 - 1, rng.random(M), rng.random(M)
    C = _rand(rng, n1 * n2 * n3).reshape(n1, n2, n3)
    g = _rand(rng, M)
    K1, K2, K3 = (k.ravel() for k in np.meshgrid(np.arange(n1), np.arange(n2), np.arange(n3), indexing="ij"))
    f = D.nudft3d(x, y, z, C)
    t1 = D.nudft3d_adj(x, y, z, g, K1, K2, K3, sign=-1)
    ad = D.nudft3d_adj(x, y, z, g, K1, K2, K3, sign=+1)
    scale = np.abs(C).sum() * np.abs(g).sum()
    assert abs(np.sum(g * f) - np.sum(C.ravel() * t1)) <= 1e-14 * scale
    assert abs(np.vdot(g, f) - np.vdot(ad, C.ravel())) <= 1e-14 * scale
    assert np.abs(t1 - ad).max() > 1e-2
    xa, yb, zc = rng.random(3), rng.random(4) * 2, rng.random(2) - 0.5
    wa, wb, wc = _rand(rng, 3), _rand(rng, 4), _rand(rng, 2)
    X, Y, Z = (v.ravel() for v in np.meshgrid(xa, yb, zc, indexing="ij"))
    W = np.einsum("i,j,k->ijk", wa, wb, wc).ravel()
    for sign in (-1, +1):
        got = D.nudft3d_adj(X, Y, Z, W, K1, K2, K3, sign=sign).reshape(n1, n2, n3)
        ref = np.einsum("i,j,k->ijk", D.nudft1(xa, wa, n1, sign=sign), D.nudft1(yb, wb, n2, sign=sign),
                        D.nudft1(zc, wc, n3, sign=sign))
        assert np.abs(got - ref).max() <= 1e-14 * np.abs(W).sum()
    k1, k2 = np.meshgrid(np.arange(n1), np.arange(n2), indexing="ij")
    got = D.nudft3d_adj(x, y, np.zeros(M), g, k1.ravel(), k2.ravel(), np.zeros(n1 * n2, np.int64), sign=+1)
    assert np.abs(got - D.nudft2d_adj(x, y, g, k1.ravel(), k2.ravel(), sign=+1)).max() <= 1e-14 * np.abs(g).sum()


def test_large_phase_exact_reduction():
    """At k ~ 2^20 a plain fl(x*k) loses ~1e-10 of phase; the oracle must not."""
    rng = np.random.default_rng(14)
    x = rng.random(3)
    N = 1 << 20
    ks = np.array([N - 1, N - 7, 123457, 999983], dtype=np.int64)
    c = np.zeros(N, np.complex128)
    c[ks] = [1.0, -2.0 + 0.5j, 0.25j, 3.0]
    f = D.nudft2(x, c)
    for j in range(3):
        ref = _mp_sum([-mpmath.mpf(x[j]) * int(k) for k in ks], c[ks])
        assert abs(f[j] - ref) <= 1e-15 * np.abs(c).sum()


def test_unit_coefficient_closed_form():
    """c = e_m gives f_j = exp(-2 pi i x_j m)."""
    rng = np.random.default_rng(15)
    x = rng.random(20)
    N, m = 64, 37
    c = np.zeros(N, np.complex128)
    c[m] = 1.0
    f = D.nudft2(x, c)
    for j in range(20):
        assert abs(f[j] - complex(mpmath.expjpi(-2 * mpmath.mpf(x[j]) * m))) < 1e-15


def test_dirichlet_closed_form():
    """c = 1 gives f_j = (1 - exp(-2 pi i N x_j)) / (1 - exp(-2 pi i x_j))."""
    rng = np.random.default_rng(16)
    N = 100
    x = rng.random(30) + 1e-3
    f = D.nudft2(x, np.ones(N))
    for j in range(30):
        xm = mpmath.mpf(x[j])
        ref = (1 - mpmath.expjpi(-2 * N * xm)) / (1 - mpmath.expjpi(-2 * xm))
        assert abs(f[j] - complex(ref)) <= 1e-14


@pytest.mark.parametrize("N", [1, 2, 4])
def test_uniform_tiny_is_exact(N):
    """x_j = j/N with N | 4: all twiddles are 0 / +-1 / +-i, so the oracle equals
    the exact integer DFT bit for bit."""
    rng = np.random.default_rng(17)
    c = (rng.integers(-9, 10, N) + 1j * rng.integers(-9, 10, N)).astype(np.complex128)
    f = D.nudft2(np.arange(N) / N, c)
    jk = np.outer(np.arange(N), np.arange(N)) % N
    w = np.array([1, -1j, -1, 1j])[(4 * jk) // N]
    exact = (w * c[None, :]).sum(axis=1)
    assert np.array_equal(f, exact)


@pytest.mark.parametrize("N", [8, 96, 1000, 1024])
def test_uniform_equals_fft(N):
    """Fully uniform case x_j = j/N, w_k = k: the NUDFT is the DFT (Sec. 1)."""
    rng = np.random.default_rng(N)
    c = _rand(rng, N)
    f = D.nudft2(np.arange(N) / N, c)
    # FFT rounding, plus (N not a power of two) the rounding of j/N itself:
    # |x - j/N| <= 2^-54 moves term k by at most 2 pi k 2^-54.
    tol = (10 * 2.0 ** -53 * np.log2(N) + 2 * np.pi * N * 2.0 ** -54) * np.abs(c).sum()
    assert np.abs(f - np.fft.fft(c)).max() <= tol
    if N & (N - 1) == 0:
        assert np.abs(f - np.fft.fft(c)).max() <= 10 * 2.0 ** -53 * np.log2(N) * np.abs(c).sum()


def test_periodicity_bitwise():
    """x -> x + 1 leaves every term unchanged; with dyadic x the shift is exact,
    so the exact phase reduction must give identical results."""
    rng = np.random.default_rng(18)
    x = rng.integers(0, 1 << 20, 16) / float(1 << 20)
    c = _rand(rng, 300)
    assert np.array_equal(D.nudft2(x, c), D.nudft2(x + 1.0, c))
    assert np.array_equal(D.nudft2(x, c), D.nudft2(x - 3.0, c))


def test_linearity():
    rng = np.random.default_rng(19)
    x = rng.random(40)
    a, b = _rand(rng, 50), _rand(rng, 50)
    lhs = D.nudft2(x, 2.0 * a - 0.5j * b)
    rhs = 2.0 * D.nudft2(x, a) - 0.5j * D.nudft2(x, b)
    assert np.abs(lhs - rhs).max() < 1e-13


def test_type1_is_transpose_and_adjoint_is_conjugate_transpose():
    """Sec. 3.1: F1 = F2^T; and <F2 c, g> = <c, F2^H g>."""
    rng = np.random.default_rng(20)
    M, N = 70, 50
    x = rng.random(M)
    c, g = _rand(rng, N), _rand(rng, M)
    F2c = D.nudft2(x, c)
    F2Hg = D.nudft1(x, g, N, sign=+1)
    F2Tg = D.nudft1(x, g, N, sign=-1)
    assert abs(np.vdot(g, F2c) - np.vdot(F2Hg, c)) < 1e-12 * np.abs(g).sum() * np.abs(c).sum()
    assert abs(np.dot(g, F2c) - np.dot(F2Tg, c)) < 1e-12 * np.abs(g).sum() * np.abs(c).sum()
    assert np.abs(F2Hg - np.conj(D.nudft1(x, np.conj(g), N, sign=-1))).max() < 1e-13


def test_type3_with_integer_frequencies_is_type2():
    rng = np.random.default_rng(21)
    x = rng.random(33)
    c = _rand(rng, 40)
    assert np.abs(D.nudft3(x, np.arange(40.0), c) - D.nudft2(x, c)).max() < 1e-13


def test_2d_separable():
    """C = a b^T factorises the 2-D sum into two 1-D type-II sums."""
    rng = np.random.default_rng(22)
    x, y = rng.random(25), rng.random(25)
    a, b = _rand(rng, 12), _rand(rng, 9)
    f = D.nudft2d(x, y, np.outer(a, b))
    ref = D.nudft2(x, a) * D.nudft2(y, b)
    assert np.abs(f - ref).max() < 1e-12


def test_grad_x_matches_finite_differences():
    """grad_x of L = ||f - y||^2: central differences of the oracle itself."""
    rng = np.random.default_rng(23)
    N, M = 64, 20
    x = rng.random(M)
    c, yv = _rand(rng, N), _rand(rng, M)
    g = 2.0 * (D.nudft2(x, c) - yv)
    gx = D.grad_x(x, c, g)
    h = 1e-6 / N
    for j in range(M):
        xp, xm = x.copy(), x.copy()
        xp[j] += h
        xm[j] -= h
        Lp = np.sum(np.abs(D.nudft2(xp, c) - yv) ** 2)
        Lm = np.sum(np.abs(D.nudft2(xm, c) - yv) ** 2)
        fd = (Lp - Lm) / (xp[j] - xm[j])
        assert abs(fd - gx[j]) <= 1e-5 * (abs(gx[j]) + 2 * np.pi * N * np.abs(c).sum())


def test_grad_c_is_adjoint():
    """grad_c of L = ||f - y||^2 equals F2^H g: check against directional derivatives."""
    rng = np.random.default_rng(24)
    N, M = 16, 12
    x = rng.random(M)
    c, yv = _rand(rng, N), _rand(rng, M)
    g = 2.0 * (D.nudft2(x, c) - yv)
    gc = D.nudft1(x, g, N, sign=+1)
    h = 1e-6
    for k in range(N):
        for e, comp in ((1.0, "re"), (1j, "im")):
            cp, cm = c.copy(), c.copy()
            cp[k] += h * e
            cm[k] -= h * e
            fd = (np.sum(np.abs(D.nudft2(x, cp) - yv) ** 2)
                  - np.sum(np.abs(D.nudft2(x, cm) - yv) ** 2)) / (2 * h)
            ref = gc[k].real if comp == "re" else gc[k].imag
            assert abs(fd - ref) < 1e-6 * (1 + abs(ref))


def test_fig1_assignment():
    g = json.load(open(os.path.join(GOLD, "fig1_assignment.json")))
    N = g["N"]
    x = np.array(g["x_times_N"]) / N
    s, t, d = D.grid_assign(x, N)
    assert s.tolist() == g["s"] and t.tolist() == g["t"]
    assert np.all(np.abs(d) <= 0.5)


def test_fig5_assignment():
    g = json.load(open(os.path.join(GOLD, "fig5_assignment.json")))
    x = np.array(g["x_times_n"]) / g["n1"]
    y = np.array(g["y_times_n"]) / g["n2"]
    sx, tx, _ = D.grid_assign(x, g["n1"])
    sy, ty, _ = D.grid_assign(y, g["n2"])
    assert sx.tolist() == g["sx"] and sy.tolist() == g["sy"]
    assert tx.tolist() == g["tx"] and ty.tolist() == g["ty"]


def test_grid_assign_edges():
    N = 10
    # ties go to even; negative samples wrap; x = 1 maps to s = N, t = 0
    x = np.array([0.05, 0.15, 0.25, -0.04, -0.06, 1.0, 0.999, 2.31, -1.0])
    s, t, d = D.grid_assign(x, N)
    nx = N * x
    assert s.tolist() == [int(v) for v in np.rint(nx)]
    assert s[5] == 10 and t[5] == 0
    assert t.tolist() == [int(v) % N for v in s]
    assert np.all((t >= 0) & (t < N))
    assert np.all(np.abs(d) <= 0.5)
    # delta is the single-rounding residual: exact here for a power of two grid
    x2 = np.random.default_rng(3).random(1000)
    s2, t2, d2 = D.grid_assign(x2, 1024)
    assert np.array_equal(d2, 1024 * x2 - s2)
    with pytest.raises(ValueError):
        D.grid_assign(np.array([0.1, np.nan]), 8)
    with pytest.raises(ValueError):
        D.grid_assign(np.array([np.inf]), 8)
