"""Pins for the method oracle (the paper's algorithm in numpy FP64), CPU only.

The Chebyshev/Bessel expansion is pinned to the function it expands
(exp(-iXY) on a dense grid), K to the values printed in Table 1, the Bessel
values to 50-digit mpmath, and every transform to the direct-sum oracle within
the paper's error bound.
"""
import json
import os

import mpmath
import numpy as np
import pytest

from oracle import lowrank as L
from oracle import nudft as D

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rand(rng, n):
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


def test_bessel_library_values_vs_mpmath():
    mpmath.mp.dps = 50
    from scipy.special import jv
    for g in (1 / 32, 0.25, 0.5):
        z = -g * np.pi / 2
        for n in range(-12, 13):
            ref = float(mpmath.besselj(n, mpmath.mpf(z)))
            assert abs(jv(n, z) - ref) <= 1e-16 + 1e-14 * abs(ref)


def test_coefficient_structure():
    """a_pr vanishes for p+r odd and is i^r times a real number (Sec. 2.1.2)."""
    a = L.chebyshev_coefficients(0.5, 12)
    for p in range(12):
        for r in range(12):
            if (p + r) % 2:
                assert a[p, r] == 0
            else:
                b = a[p, r] / (1j ** r)
                assert abs(b.imag) <= 1e-15 * abs(b) + 1e-300
    # gamma = 0: only a_00 = 4 survives (A is all ones)
    a0 = L.chebyshev_coefficients(0.0, 6)
    assert a0[0, 0] == 4.0 and np.count_nonzero(a0) == 1


@pytest.mark.parametrize("gamma", [1 / 32, 1 / 8, 0.3, 0.5])
@pytest.mark.parametrize("K", [3, 6, 10, 15])
def test_expansion_reproduces_exponential(gamma, K):
    """Lemma A.1: sup |exp(-iXY) - sum'sum' a_pr exp(-i pi X) T_p(X/gamma) T_r(Y/pi-1)|
    over [-gamma,gamma] x [0,2pi] is at most the truncation tail."""
    X = np.linspace(-gamma, gamma, 201)
    Y = np.linspace(0, 2 * np.pi, 801)
    a = L.chebyshev_coefficients(gamma, K)
    w = np.ones(K); w[0] = 0.5
    Tx = L.chebyshev_T(K, X / gamma)            # [p, X]
    Ty = L.chebyshev_T(K, Y / np.pi - 1.0)      # [r, Y]
    approx = np.exp(-1j * np.pi * X)[:, None] * ((w[:, None] * Tx).T @ (a * w[None, :]) @ Ty)
    err = np.abs(np.exp(-1j * np.outer(X, Y)) - approx).max()
    assert err <= L.tail_bound(gamma, K) * (1 + 1e-6) + 1e-14
    # the tail bound is not vacuous: within a modest factor of the observed sup
    if err > 1e-13:
        assert L.tail_bound(gamma, K) <= 50 * err


def test_wrong_phase_sign_fails():
    """The proof of Lemma A.1 prints exp(+i pi x); with it the expansion is wrong."""
    gamma, K = 0.5, 12
    X = np.linspace(-gamma, gamma, 51)
    Y = np.linspace(0, 2 * np.pi, 101)
    a = L.chebyshev_coefficients(gamma, K)
    w = np.ones(K); w[0] = 0.5
    core = (w[:, None] * L.chebyshev_T(K, X / gamma)).T @ (a * w[None, :]) @ L.chebyshev_T(K, Y / np.pi - 1)
    exact = np.exp(-1j * np.outer(X, Y))
    assert np.abs(exact - np.exp(-1j * np.pi * X)[:, None] * core).max() < 1e-9
    assert np.abs(exact - np.exp(+1j * np.pi * X)[:, None] * core).max() > 0.5


def test_table1_single_and_half_rows():
    tab = json.load(open(os.path.join(GOLD, "table1_K.json")))
    for row in ("single", "half"):
        eps = tab["rows"][row]["eps"]
        got = [L.choose_K(eps, g) for g in tab["gamma"]]
        assert got == tab["rows"][row]["K"], row


def test_table1_double_row_at_1e14():
    tab = json.load(open(os.path.join(GOLD, "table1_K.json")))
    got = [L.choose_K(1e-14, g) for g in tab["gamma"]]
    assert got == tab["rows"]["double"]["K"]


def test_explicit_K_formula_is_a_valid_upper_bound():
    """eq. (ExplicitK) is loose but must still meet the working accuracy."""
    for eps in (1e-4, 1e-6, 1e-9, 1e-12):
        for g in (1 / 32, 1 / 8, 1 / 2):
            Ke = L.explicit_K(eps, g)
            assert Ke >= L.choose_K(eps, g)
            assert L.tail_bound(g, Ke) <= eps


def test_K_values_for_the_workloads():
    assert L.choose_K(1e-6, 0.5) == 10
    assert L.choose_K(1e-12, 0.5) == 15
    assert L.choose_K(5e-7, 0.5) == 10


@pytest.mark.parametrize("eps", [1e-4, 1e-6, 1e-9, 1e-12])
@pytest.mark.parametrize("dist", ["iid", "jitter", "worst_grid"])
def test_type2_within_error_bound(eps, dist):
    """Error bound after Fig. 3: |f_j - f~_j| <= ||A - A_K||_max ||c||_1 <= eps ||c||_1."""
    rng = np.random.default_rng(31)
    N = 512
    if dist == "iid":
        x = rng.random(N)
    elif dist == "jitter":
        x = (np.arange(N) + rng.uniform(-0.5, 0.5, N)) / N
    else:   # Sec. 2.4 "worst grid" with gamma = 1/8
        j = np.arange(N)
        x = np.where(j <= N // 2, (j + 0.125) / N, (j - 0.125) / N)
    c = _rand(rng, N)
    p = L.Plan(x, N, eps)
    err = np.abs(p.type2(c) - D.nudft2(x, c)).max()
    assert err <= eps * np.abs(c).sum()
    if dist == "worst_grid":
        assert abs(p.gamma - 0.125) < 1e-12


def test_uniform_gives_single_fft():
    """gamma = 0: K = 1 and the method is one FFT (Sec. 1, Sec. 2.4)."""
    rng = np.random.default_rng(32)
    N = 256
    c = _rand(rng, N)
    p = L.Plan(np.arange(N) / N, N, 1e-12)
    assert p.K == 1 and p.gamma == 0.0
    assert np.abs(p.type2(c) - np.fft.fft(c)).max() < 1e-12


@pytest.mark.parametrize("eps", [1e-6, 1e-12])
def test_type1_and_adjoint_within_bound(eps):
    rng = np.random.default_rng(33)
    M, N = 300, 256
    x = rng.random(M)
    g = _rand(rng, M)
    p = L.Plan(x, N, eps)
    assert np.abs(p.type1(g) - D.nudft1(x, g, N, sign=-1)).max() <= eps * np.abs(g).sum()
    assert np.abs(p.adjoint(g) - D.nudft1(x, g, N, sign=+1)).max() <= eps * np.abs(g).sum()


@pytest.mark.parametrize("N,grid", [(300, 512), (257, 512), (1000, 1024)])
def test_oversampled_grid(N, grid):
    """Sec. 2.3 oversampling: FFTs of size M >= N with |X| <= N/(2M)."""
    rng = np.random.default_rng(N)
    x = rng.random(N)
    c = _rand(rng, N)
    p = L.Plan(x, N, 1e-6, grid=grid)
    assert p.gamma <= N / (2 * grid) + 1e-15
    assert np.abs(p.type2(c) - D.nudft2(x, c)).max() <= 1e-6 * np.abs(c).sum()


def test_type3_within_bound():
    rng = np.random.default_rng(34)
    N, M = 128, 100
    x = rng.random(M)
    x[:3] = [1 - 1e-4, 0.9999, 0.99995]      # samples that round to s = N
    w = rng.uniform(0, N, N)
    c = _rand(rng, N)
    f = L.nufft3(x, w, c, 1e-9)
    assert np.abs(f - D.nudft3(x, w, c)).max() <= 1e-9 * np.abs(c).sum()


def test_2d_within_bound():
    rng = np.random.default_rng(35)
    n1, n2, M = 32, 24, 200
    r, th = 0.5 * rng.random(M), 2 * np.pi * rng.random(M)
    x, y = 0.5 + r * np.cos(th), 0.5 + r * np.sin(th)
    C = _rand(rng, n1 * n2).reshape(n1, n2)
    p = L.Plan2D(x, y, n1, n2, 1e-6)
    assert np.abs(p.type2(C) - D.nudft2d(x, y, C)).max() <= 1e-6 * np.abs(C).sum()
    g = _rand(rng, M)
    k1, k2 = np.meshgrid(np.arange(n1), np.arange(n2), indexing="ij")
    ref = D.nudft2d_adj(x, y, g, k1.ravel(), k2.ravel()).reshape(n1, n2)
    assert np.abs(p.adjoint(g) - ref).max() <= 1e-6 * np.abs(g).sum()
