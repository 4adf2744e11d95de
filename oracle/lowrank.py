"""The paper's low-rank NUFFT written out in plain numpy FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).  This follows the steps
of arXiv:1701.04492 in the paper's order and notation so that it can be read
against the text:

* Sec. 2.2: s = round(N x), t = mod(s, N), perturbation N(x - s/N) in [-1/2, 1/2].
* Sec. 2.1.2 / Appendix A, Lemma A.1: the bivariate Chebyshev expansion
  exp(-i X Y) = sum'_p sum'_r a_pr exp(-i pi X) T_p(X/gamma) T_r(Y/pi - 1) on
  [-gamma, gamma] x [0, 2 pi], with a_pr = 4 i^r J_{(p+r)/2}(-gamma pi/2) J_{(r-p)/2}(-gamma pi/2)
  for p = r mod 2 (zero otherwise); primes halve the first term.
* Rank-K factors: u_r(j) = sum'_p a_pr exp(-i pi X_j) T_p(X_j/gamma),
  v_r(k) = T_r(2k/N - 1) with v_0 halved (Sec. 2.1.2).
* Sec. 2.3 vectorized two-step form: X = I(t,:) F [D_{v_0} c | ... | D_{v_{K-1}} c],
  f = [D_{u_0} X_0 | ... ] 1.
* Sec. 3.1 type I as the transpose, Sec. 3.2 type III, Sec. 4 2-D type II.

Readings where the paper is silent or inconsistent:
* K is the smallest integer whose full truncation tail
  sum_{max(p,r) >= K} w_p w_r |a_pr| (w_0 = 1/2, else 1) is at most eps.  The
  tail in the proof of Lemma A.1 keeps only p >= K and r >= K, which misses the
  terms with one index below K; the full tail is the rigorous bound.
* The phase factor is exp(-i pi X) (as in Sec. 2.1.2 and Lemma A.1's
  statement); the proof's exp(+i pi x) is a sign slip.
* Oversampled grid of size M >= N (Sec. 2.3, "Oversampling"): s = round(M x),
  X_j = (M x_j - s_j) N / M, so |X_j| <= N/(2M) and v_r still runs over k < N.
* gamma = 0 means every X_j = 0: K = 1 and X/gamma is read as 0, which gives
  u_0 v_0 = a_00/4 = 1 exactly (the trivial approximation of Sec. 2.1.2).
"""
import numpy as np
from scipy.special import jv, lambertw

from . import nudft as _direct

_TAIL_P = 64   # the tail sums run to p, r < 64; |a_pr| < 1e-60 beyond


def chebyshev_coefficients(gamma, size):
    """a_pr for 0 <= p, r < size (Sec. 2.1.2, Lemma A.1), complex128 array [p, r]."""
    a = np.zeros((size, size), np.complex128)
    z = -gamma * np.pi / 2.0
    for p in range(size):
        for r in range(size):
            if (p - r) % 2 == 0:
                a[p, r] = 4.0 * (1j ** r) * jv((p + r) // 2, z) * jv((r - p) // 2, z)
    return a


def _weights(size):
    w = np.ones(size)
    w[0] = 0.5
    return w


def tail_bound(gamma, K):
    """sum over max(p, r) >= K of w_p w_r |a_pr| -- the bound on
    sup |exp(-iXY) - A_K| that follows from |T_p| <= 1 and |exp(i theta)| = 1."""
    a = np.abs(chebyshev_coefficients(gamma, _TAIL_P))
    w = _weights(_TAIL_P)
    wa = a * w[:, None] * w[None, :]
    return float(wa.sum() - wa[:K, :K].sum())


def choose_K(eps, gamma, k_max=40):
    """Smallest K >= 1 with tail_bound(gamma, K) <= eps (reading of Sec. 2.1.2 / Table 1)."""
    if gamma == 0.0:
        return 1
    a = np.abs(chebyshev_coefficients(gamma, _TAIL_P))
    w = _weights(_TAIL_P)
    wa = a * w[:, None] * w[None, :]
    total = wa.sum()
    for K in range(1, k_max + 1):
        if total - wa[:K, :K].sum() <= eps:
            return K
    raise ValueError("eps too small for the rank limit")


def explicit_K(eps, gamma):
    """The paper's closed-form K of eq. (ExplicitK): max(3, ceil(5 gamma e^{W(log(140/eps)/(5 gamma))}))."""
    w = lambertw(np.log(140.0 / eps) / (5.0 * gamma)).real
    return max(3, int(np.ceil(5.0 * gamma * np.exp(w))))


def chebyshev_T(n, z):
    """T_0..T_{n-1} at z by the three-term recurrence; returns array [n, len(z)]."""
    z = np.asarray(z, dtype=np.float64)
    T = np.empty((n,) + z.shape)
    T[0] = 1.0
    if n > 1:
        T[1] = z
    for p in range(2, n):
        T[p] = 2.0 * z * T[p - 1] - T[p - 2]
    return T


def factors(X, gamma, K, n_modes):
    """U (M x K) and V (N x K) with A_K = U V^T (Sec. 2.1.2):
    u_r = sum'_p a_pr exp(-i pi X) T_p(X/gamma),  v_r(k) = T_r(2k/N - 1), v_0 halved."""
    X = np.asarray(X, dtype=np.float64)
    a = chebyshev_coefficients(gamma, K)
    a[0, :] *= 0.5                                   # prime on the p-sum
    z = X / gamma if gamma > 0 else np.zeros_like(X)
    Tp = chebyshev_T(K, z)                           # [p, j]
    U = np.exp(-1j * np.pi * X)[:, None] * (Tp.T @ a)   # [j, r]
    k = np.arange(n_modes, dtype=np.float64)
    V = chebyshev_T(K, 2.0 * k / n_modes - 1.0).T    # [k, r]
    V[:, 0] *= 0.5                                   # prime on the r-sum
    return U, V


class Plan:
    """Planning stage of Sec. 2.3: gamma, t, K and the factors U, V."""

    def __init__(self, x, n_modes, eps, grid=None, gamma=None):
        self.N = int(n_modes)
        self.M = int(grid) if grid is not None else self.N
        if self.M < self.N:
            raise ValueError("grid must have at least n_modes points")
        self.s, self.t, d = _direct.grid_assign(x, self.M)
        self.X = d * (self.N / self.M)
        self.gamma = float(np.max(np.abs(self.X))) if gamma is None else float(gamma)
        self.K = choose_K(eps, self.gamma)
        self.U, self.V = factors(self.X, self.gamma, self.K, self.N)

    def _fft_cols(self, W, inverse=False):
        Wp = np.zeros((self.M, W.shape[1]), np.complex128)
        Wp[: self.N] = W
        return self.M * np.fft.ifft(Wp, axis=0) if inverse else np.fft.fft(Wp, axis=0)

    def type2(self, c):
        """Sec. 2.3 two-step form: X = I(t,:) F [D_v c], f = [D_u X] 1."""
        W = self.V * np.asarray(c, np.complex128)[:, None]
        Xr = self._fft_cols(W)[self.t, :]
        return (self.U * Xr).sum(axis=1)

    def _spread(self, w):
        G = np.zeros((self.M, self.K), np.complex128)
        np.add.at(G, self.t, w)
        return G

    def type1(self, c):
        """Sec. 3.1: f = sum_r D_{v_r} F^T I(:,t) D_{u_r} c, F^T = F (the transpose of type II)."""
        G = self._spread(self.U * np.asarray(c, np.complex128)[:, None])
        Y = np.fft.fft(G, axis=0)[: self.N]
        return (self.V * Y).sum(axis=1)

    def adjoint(self, g):
        """Conjugate transpose of type II: sum_r D_{v_r} F^H I(:,t) D_{conj u_r} g."""
        G = self._spread(np.conj(self.U) * np.asarray(g, np.complex128)[:, None])
        Y = self.M * np.fft.ifft(G, axis=0)[: self.N]
        return (self.V * Y).sum(axis=1)


def nufft2(x, c, eps, grid=None):
    return Plan(x, len(c), eps, grid).type2(c)


def nufft1(x, c, n_modes, eps, grid=None):
    return Plan(x, n_modes, eps, grid).type1(c)


def nufft3(x, w, c, eps):
    """Sec. 3.2: F3 = A o B o F1(t,:) on the grid of size N = len(w), x in [0,1), w in [0,N).
    A_jk = exp(-2 pi i (x_j - s_j/N) w_k) ~ sum_r u_r(j) v_r(w_k/N);
    B_jk = (1 - d_j) + d_j exp(-2 pi i w_k), d_j = (s_j - t_j)/N in {0, 1};
    F1 is the type-I matrix (F1)_{nk} = exp(-2 pi i n w_k / N)."""
    x = np.asarray(x, np.float64)
    w = np.asarray(w, np.float64)
    c = np.asarray(c, np.complex128)
    N = w.shape[0]
    s, t, d = _direct.grid_assign(x, N)
    gamma = float(np.max(np.abs(d)))
    K = choose_K(eps / 2.0, gamma)
    a = chebyshev_coefficients(gamma, K)
    a[0, :] *= 0.5
    z = d / gamma if gamma > 0 else np.zeros_like(d)
    U = np.exp(-1j * np.pi * d)[:, None] * (chebyshev_T(K, z).T @ a)
    V = chebyshev_T(K, 2.0 * w / N - 1.0).T
    V[:, 0] *= 0.5
    wrap = (s - t) != 0
    inner = Plan(w / N, N, eps / (4.0 * K))         # type I on samples w/N, N modes
    f = np.zeros(x.shape[0], np.complex128)
    for r in range(K):
        y = inner.type1(V[:, r] * c)
        term = y[t]
        if wrap.any():
            y2 = inner.type1(V[:, r] * np.exp(-2j * np.pi * w) * c)
            term = np.where(wrap, y2[t], term)
        f += U[:, r] * term
    return f


class Plan2D:
    """Sec. 4: 2-D type II on an N1 x N2 grid (x pairs with k1, y with k2), eps split in half."""

    def __init__(self, x, y, n1, n2, eps):
        self.px = Plan(x, n1, eps / 2.0)
        self.py = Plan(y, n2, eps / 2.0)
        self.n1, self.n2 = int(n1), int(n2)

    def type2(self, C):
        C = np.asarray(C, np.complex128)
        px, py = self.px, self.py
        f = np.zeros(px.t.shape[0], np.complex128)
        for r1 in range(px.K):
            Ck = C * px.V[:, r1][:, None]
            H = np.fft.fft(Ck, axis=0)                        # k1 -> n1, reused for all r2
            for r2 in range(py.K):
                G = np.fft.fft(H * py.V[:, r2][None, :], axis=1)
                f += px.U[:, r1] * py.U[:, r2] * G[px.t, py.t]
        return f

    def adjoint(self, g):
        g = np.asarray(g, np.complex128)
        px, py = self.px, self.py
        out = np.zeros((self.n1, self.n2), np.complex128)
        for r1 in range(px.K):
            for r2 in range(py.K):
                G = np.zeros((self.n1, self.n2), np.complex128)
                np.add.at(G, (px.t, py.t), np.conj(px.U[:, r1] * py.U[:, r2]) * g)
                Y = self.n1 * self.n2 * np.fft.ifft2(G)
                out += px.V[:, r1][:, None] * py.V[:, r2][None, :] * Y
        return out
