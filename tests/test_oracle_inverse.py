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


# ---- inverse type I (Sec. 3.3, the type-I analogue) ------------------------------

def test_type1_gram_matrix_is_conjugate_toeplitz():
    """F1 F1^* = conj(F2^* F2): Hermitian Toeplitz with first column conj(tau)."""
    n, m = 29, 41
    x = np.random.default_rng(11).random(m)
    F1 = I.dense_matrix_type1(x, n)
    G = F1 @ F1.conj().T
    tau = I.toeplitz_column(x, n)
    assert np.allclose(G[:, 0], np.conj(tau), rtol=0, atol=1e-11)
    F2 = I.dense_matrix(x, n)
    assert np.allclose(G, np.conj(F2.conj().T @ F2), rtol=0, atol=1e-11)


@pytest.mark.parametrize("n,m,gamma", [(64, 64, 1 / 8), (90, 160, 0.3), (256, 256, 1 / 32)])
def test_cg_type1_matches_dense_minimum_norm(n, m, gamma):
    if m == n:
        x = _jittered(n, gamma, 12)
    else:
        x = np.sort(np.random.default_rng(12).random(m))
    f = W.complex_normal(W.rng_for(13), n)
    sol, it, res = I.cg_type1(x, f, n, tol=1e-13, max_iter=2000)
    ref = I.lstsq_type1(x, f, n)
    assert res <= 1e-13
    assert np.abs(sol - ref).max() <= 1e-8 * np.abs(ref).max()
    # it solves the system (to the conditioning of the random-sample Gram matrix),
    # and (M > N) the solution lies in the range of F1^*
    F1 = I.dense_matrix_type1(x, n)
    assert np.abs(F1 @ sol - f).max() <= 1e-7 * np.abs(f).max()
    if m > n:
        z = np.linalg.lstsq(F1.conj().T, sol, rcond=None)[0]
        assert np.abs(F1.conj().T @ z - sol).max() <= 1e-9 * np.abs(sol).max()


def test_type1_equispaced_is_inverse_fft():
    """gamma = 0: F1 = F (the DFT), F F^* = N I, one CG iteration and c = ifft(f)."""
    n = 128
    x = np.arange(n) / n
    f = W.complex_normal(W.rng_for(14), n)
    sol, it, _ = I.cg_type1(x, f, n, tol=1e-12)
    assert it == 1
    assert np.abs(sol - np.fft.ifft(f)).max() <= 1e-13 * np.abs(f).max()


def test_type1_unconjugated_column_fails():
    """Planted mistake: the type-II column tau (instead of conj(tau)) gives a wrong Gram product."""
    n, m = 24, 40
    x = np.random.default_rng(15).random(m)
    y = W.complex_normal(W.rng_for(16), n)
    F1 = I.dense_matrix_type1(x, n)
    right = F1 @ (F1.conj().T @ y)
    good = I.toeplitz_matvec(I.circulant_eigenvalues(np.conj(I.toeplitz_column(x, n))), y)
    wrong = I.toeplitz_matvec(I.circulant_eigenvalues(I.toeplitz_column(x, n)), y)
    assert np.abs(good - right).max() <= 1e-10 * np.abs(right).max()
    assert np.abs(wrong - right).max() > 1e-3 * np.abs(right).max()
