"""The inverse type-II and type-I transforms of Sec. 3.3, in plain numpy FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Steps in the paper's
order:

* The inverse NUDFT-II solves F2 c = f (M >= N samples; least squares when
  M > N) by the conjugate gradient method on the normal equations
  F2^* F2 c = F2^* f.
* F2^* F2 is Toeplitz: its (j, k) entry depends on j - k only,
  tau_{j-k} = sum_p exp(+2 pi i x_p (j - k)).  Its first column tau_m,
  0 <= m < N, is F2^* applied to the all-ones vector; the first row holds
  tau_{-m} = conj(tau_m) (the matrix is Hermitian -- the footnote of Sec. 3.3
  calls the first row and column "the same", which holds up to conjugation).
* A Toeplitz matrix-vector product is one FFT and one inverse FFT of size 2N
  through the circulant matrix whose first column is
  [tau_0, ..., tau_{N-1}, 0, conj(tau_{N-1}), ..., conj(tau_1)].
* Inverse type I: F1 = F2^T (type I of Sec. 3.1 with x_j = w_j / N) maps M
  values to N; for M >= N its inverse (minimum-norm when M > N) is
  F1^* (F1 F1^*)^{-1}, and F1 F1^* = conj(F2^* F2) is again Hermitian
  Toeplitz, with first column conj(tau).  CG runs on F1 F1^* y = f and
  c = F1^* y.

Readings where the paper leaves a choice: the embedding uses 2N points with one zero
(any value there gives the same product); CG stops when the residual of the
normal equations falls below tol times the norm of their right-hand side
F2^* f, or after max_iter iterations, and starts from c = 0; the type-I
solve stops on ||f - F1 F1^* y|| <= tol ||f|| and starts from y = 0.
"""
import numpy as np

from . import nudft as _direct


def dense_matrix(x, n_modes):
    """F2 of eq. (2): (F2)_{jk} = exp(-2 pi i x_j k), from the definition (small sizes only)."""
    x = np.asarray(x, np.float64)
    k = np.arange(n_modes, dtype=np.float64)
    return np.exp(-2j * np.pi * np.outer(x, k))


def toeplitz_column(x, n_modes):
    """tau_m = sum_p exp(+2 pi i x_p m), m < N: the first column of F2^* F2 (the adjoint of ones)."""
    x = np.asarray(x, np.float64)
    return _direct.nudft1(x, np.ones(x.shape[0], np.complex128), n_modes, sign=+1)


def circulant_eigenvalues(tau):
    """FFT of the first column of the 2N-point circulant matrix that embeds the Toeplitz matrix."""
    n = tau.shape[0]
    col = np.zeros(2 * n, np.complex128)
    col[:n] = tau
    col[n + 1:] = np.conj(tau[1:][::-1])
    return np.fft.fft(col)


def toeplitz_matvec(lam, c):
    """(F2^* F2) c via the circulant embedding: first N entries of ifft(lam * fft([c, 0]))."""
    n = c.shape[0]
    pad = np.zeros(2 * n, np.complex128)
    pad[:n] = c
    return np.fft.ifft(lam * np.fft.fft(pad))[:n]


def _cg(apply, b, tol, max_iter):
    """Plain conjugate gradients for a Hermitian positive definite operator, from zero."""
    y = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rs = np.vdot(r, r).real
    bn = np.sqrt(np.vdot(b, b).real)
    it = 0
    if bn == 0.0:
        return y, 0, 0.0
    while it < max_iter and np.sqrt(rs) > tol * bn:
        ap = apply(p)
        alpha = rs / np.vdot(p, ap).real
        y = y + alpha * p
        r = r - alpha * ap
        rs_new = np.vdot(r, r).real
        p = r + (rs_new / rs) * p
        rs = rs_new
        it += 1
    return y, it, np.sqrt(rs) / bn


def cg_normal(x, f, n_modes, tol=1e-12, max_iter=500):
    """Sec. 3.3: conjugate gradients on F2^* F2 c = F2^* f with the fast Toeplitz product.
    Returns (c, iterations, relative residual of the normal equations)."""
    x = np.asarray(x, np.float64)
    f = np.asarray(f, np.complex128)
    b = _direct.nudft1(x, f, n_modes, sign=+1)
    lam = circulant_eigenvalues(toeplitz_column(x, n_modes))
    return _cg(lambda v: toeplitz_matvec(lam, v), b, tol, max_iter)


def lstsq(x, f, n_modes):
    """Least-squares solution of F2 c = f from the dense matrix (small sizes only)."""
    return np.linalg.lstsq(dense_matrix(x, n_modes), np.asarray(f, np.complex128), rcond=None)[0]


def dense_matrix_type1(x, n_modes):
    """F1 = F2^T, the type I of Sec. 3.1: (F1)_{kj} = exp(-2 pi i x_j k) (small sizes only)."""
    return dense_matrix(x, n_modes).T


def cg_type1(x, f, n_modes, tol=1e-12, max_iter=500):
    """Sec. 3.3, the type-I analogue: c = F1^* y with F1 F1^* y = f solved by CG; F1 F1^* =
    conj(F2^* F2) is applied through the circulant embedding of conj(tau).
    Returns (c, iterations, relative residual ||f - F1 F1^* y|| / ||f||)."""
    x = np.asarray(x, np.float64)
    f = np.asarray(f, np.complex128)
    lam = circulant_eigenvalues(np.conj(toeplitz_column(x, n_modes)))
    y, it, res = _cg(lambda v: toeplitz_matvec(lam, v), f, tol, max_iter)
    # c_j = sum_k y_k exp(+2 pi i x_j k) = conj of the type II of conj(y)
    c = np.conj(_direct.nudft2(x, np.conj(y)))
    return c, it, res


def lstsq_type1(x, f, n_modes):
    """Minimum-norm solution of F1 c = f from the dense matrix (small sizes only)."""
    return np.linalg.lstsq(dense_matrix_type1(x, n_modes), np.asarray(f, np.complex128), rcond=None)[0]
