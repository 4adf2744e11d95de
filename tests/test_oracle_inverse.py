"""Pins of the inverse type-II oracle (Sec. 3.3) against dense linear algebra and
closed forms: no GPU."""
import numpy as np
import pytest

from oracle import inverse as I
from paper_1701_04492_amd import workloads as W


def _jittered(n, gamma, seed):
    rng = np.random.default_rng(seed)
    return (np.arange(n) + gamma * rng.uniform(-1.0, 1.0, n)) / n


def test_toeplitz_column_is_first_column_of_normal_matrix():
    x = _jittered(37, 0.3, 1)
    F = I.dense_matrix(x, 37)
    A = F.conj().T @ F
    tau = I.toeplitz_column(x, 37)
    assert np.allclose(tau, A[:, 0], rtol=0, atol=1e-11)
    # Hermitian Toeplitz: constant diagonals, first row = conj(first column)
    for m in range(1, 37):
        assert np.allclose(np.diag(A, -m), tau[m], atol=1e-11)
        assert np.allclose(np.diag(A, m), np.conj(tau[m]), atol=1e-11)


@pytest.mark.parametrize("n", [1, 2, 16, 45])
def test_circulant_product_equals_dense_product(n):
    x = _jittered(n, 0.4, 2)
    rng = np.random.default_rng(3)
    c = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    F = I.dense_matrix(x, n)
    lam = I.circulant_eigenvalues(I.toeplitz_column(x, n))
    assert np.allclose(I.toeplitz_matvec(lam, c), F.conj().T @ (F @ c), rtol=0, atol=1e-10 * n)


def test_equispaced_samples_one_iteration():
    """gamma = 0: F2 = F, F^* F = N I, CG converges in one iteration (Sec. 3.3)."""
    n = 64
    x = np.arange(n) / n
    rng = np.random.default_rng(4)
    c = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    f = I.dense_matrix(x, n) @ c
    sol, it, res = I.cg_normal(x, f, n, tol=1e-12)
    assert it == 1
    assert np.allclose(sol, c, atol=1e-12 * np.abs(c).max() * n)


@pytest.mark.parametrize("n,m,gamma", [(64, 64, 1 / 8), (100, 150, 0.3), (200, 200, 1 / 32)])
def test_cg_matches_dense_least_squares(n, m, gamma):
    if m == n:
        x = _jittered(n, gamma, 5)
    else:
        x = np.sort(np.random.default_rng(5).random(m))
    rng = np.random.default_rng(6)
    c = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    f = I.dense_matrix(x, n) @ c
    sol, it, res = I.cg_normal(x, f, n, tol=1e-13, max_iter=2000)
    ref = I.lstsq(x, f, n)
    assert res <= 1e-13
    assert np.abs(sol - ref).max() <= 1e-8 * np.abs(ref).max()
    assert np.abs(sol - c).max() <= 1e-8 * np.abs(c).max()


def test_wrong_conjugation_in_embedding_fails():
    """Planted mistake: the first row taken equal to the first column (no conjugate)
    gives a wrong product, so the Hermitian reading is load-bearing."""
    n = 20
    x = _jittered(n, 0.4, 7)
    tau = I.toeplitz_column(x, n)
    col = np.zeros(2 * n, np.complex128)
    col[:n] = tau
    col[n + 1:] = tau[1:][::-1]
    c = np.random.default_rng(8).standard_normal(n) + 0j
    pad = np.zeros(2 * n, np.complex128)
    pad[:n] = c
    wrong = np.fft.ifft(np.fft.fft(col) * np.fft.fft(pad))[:n]
    F = I.dense_matrix(x, n)
    assert np.abs(wrong - F.conj().T @ (F @ c)).max() > 1e-3


def test_iterations_stay_small_for_small_perturbation():
    """Sec. 3.3 / Fig. 4: for 0 < gamma < 1/4 the iteration count stays small as N grows."""
    its = []
    for n in (128, 512, 2048):
        x = _jittered(n, 1 / 8, 9)
        rng = np.random.default_rng(10)
        f = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        _, it, res = I.cg_normal(x, f, n, tol=1e-12, max_iter=200)
        assert res <= 1e-12
        its.append(it)
    assert max(its) <= 40
