"""ctypes front end of the C oracle: direct FP64 NUDFT sums and grid assignment.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Each function is the
plain definition of a transform of arXiv:1701.04492; see ``nudft.c`` for the
arithmetic (exact phase reduction, compensated Dot2 sums).
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None
_i64 = ctypes.c_int64
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int64)


def _load():
    global _lib
    if _lib is None:
        path = _build.build()
        lib = ctypes.CDLL(path)
        lib.oracle_nudft2.argtypes = [_i64, _dp, _i64, _dp, _dp]
        lib.oracle_nudft1.argtypes = [_i64, _dp, _dp, _i64, _ip, ctypes.c_int, _dp]
        lib.oracle_nudft3.argtypes = [_i64, _dp, _dp, _i64, _dp, _dp]
        lib.oracle_nudft2d.argtypes = [_i64, _i64, _dp, _i64, _dp, _dp, _dp]
        lib.oracle_nudft2d_adj.argtypes = [_i64, _dp, _dp, _dp, _i64, _ip, _ip, ctypes.c_int, _dp]
        lib.oracle_nudft3_2d.argtypes = [_i64, _dp, _dp, _dp, _i64, _dp, _dp, _dp]
        lib.oracle_nudft3d.argtypes = [_i64, _i64, _i64, _dp, _i64, _dp, _dp, _dp, _dp]
        lib.oracle_nudft3d_adj.argtypes = [_i64, _dp, _dp, _dp, _dp, _i64, _ip, _ip, _ip, ctypes.c_int, _dp]
        lib.oracle_grid_assign.argtypes = [_i64, _i64, _dp, _ip, _ip, _dp]
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        lib.oracle_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def _p(a):
    return a.ctypes.data_as(_dp)


def _pi(a):
    return a.ctypes.data_as(_ip)


def set_threads(n):
    _load().oracle_set_threads(int(n))


def max_threads():
    return int(_load().oracle_max_threads())


def nudft2(x, c):
    """Type II, Sec. 1 eq. (2): f_j = sum_{k<N} c_k exp(-2 pi i x_j k)."""
    x, c = _f64(x), _c128(c)
    f = np.empty(x.shape[0], np.complex128)
    rc = _load().oracle_nudft2(c.shape[0], _p(c.view(np.float64)), x.shape[0], _p(x),
                               _p(f.view(np.float64)))
    assert rc == 0
    return f


def nudft1(x, c, n_modes, k=None, sign=-1):
    """Type I (Sec. 3.1, sign=-1) or adjoint of type II (sign=+1):
    f_k = sum_j c_j exp(sign 2 pi i x_j k), for k in ``k`` (default 0..n_modes-1)."""
    x, c = _f64(x), _c128(c)
    if k is None:
        k = np.arange(n_modes, dtype=np.int64)
    k = np.ascontiguousarray(k, dtype=np.int64)
    f = np.empty(k.shape[0], np.complex128)
    rc = _load().oracle_nudft1(x.shape[0], _p(x), _p(c.view(np.float64)), k.shape[0], _pi(k),
                               int(sign), _p(f.view(np.float64)))
    assert rc == 0
    return f


def nudft3(x, w, c):
    """Type III, Sec. 3.2: f_j = sum_k c_k exp(-2 pi i x_j w_k)."""
    x, w, c = _f64(x), _f64(w), _c128(c)
    f = np.empty(x.shape[0], np.complex128)
    rc = _load().oracle_nudft3(w.shape[0], _p(w), _p(c.view(np.float64)), x.shape[0], _p(x),
                               _p(f.view(np.float64)))
    assert rc == 0
    return f


def nudft3d(x, y, z, C):
    """3-D type II (Sec. 4's construction with a third axis):
    f_j = sum_{k1,k2,k3} C[k1,k2,k3] exp(-2 pi i (k1 x_j + k2 y_j + k3 z_j))."""
    x, y, z, C = _f64(x), _f64(y), _f64(z), _c128(C)
    n1, n2, n3 = C.shape
    f = np.empty(x.shape[0], np.complex128)
    rc = _load().oracle_nudft3d(n1, n2, n3, _p(C.view(np.float64)), x.shape[0], _p(x), _p(y), _p(z),
                                _p(f.view(np.float64)))
    assert rc == 0
    return f


def nudft3d_adj(x, y, z, g, k1, k2, k3, sign=+1):
    """Adjoint of the 3-D type II (sign=+1), or the 3-D type I, its transpose (sign=-1), at
    coefficient indices (k1_q, k2_q, k3_q): out_q = sum_j g_j exp(sign 2 pi i (k1_q x_j + k2_q y_j + k3_q z_j))."""
    x, y, z, g = _f64(x), _f64(y), _f64(z), _c128(g)
    k1, k2, k3 = (np.ascontiguousarray(k, dtype=np.int64) for k in (k1, k2, k3))
    out = np.empty(k1.shape[0], np.complex128)
    rc = _load().oracle_nudft3d_adj(x.shape[0], _p(x), _p(y), _p(z), _p(g.view(np.float64)), k1.shape[0],
                                    _pi(k1), _pi(k2), _pi(k3), int(sign), _p(out.view(np.float64)))
    assert rc == 0
    return out


def nudft3_2d(x, y, w1, w2, c):
    """2-D type III (Sec. 3.2 per axis): f_j = sum_k c_k exp(-2 pi i (x_j w1_k + y_j w2_k))."""
    x, y, w1, w2, c = _f64(x), _f64(y), _f64(w1), _f64(w2), _c128(c)
    f = np.empty(x.shape[0], np.complex128)
    rc = _load().oracle_nudft3_2d(w1.shape[0], _p(w1), _p(w2), _p(c.view(np.float64)), x.shape[0], _p(x), _p(y),
                                  _p(f.view(np.float64)))
    assert rc == 0
    return f


def nudft2d(x, y, C):
    """2-D type II, Sec. 4: f_j = sum_{k1,k2} C[k1,k2] exp(-2 pi i (k1 x_j + k2 y_j))."""
    x, y, C = _f64(x), _f64(y), _c128(C)
    n1, n2 = C.shape
    f = np.empty(x.shape[0], np.complex128)
    rc = _load().oracle_nudft2d(n1, n2, _p(C.view(np.float64)), x.shape[0], _p(x), _p(y),
                                _p(f.view(np.float64)))
    assert rc == 0
    return f


def nudft2d_adj(x, y, g, k1, k2, sign=+1):
    """Adjoint of 2-D type II (sign=+1), or the 2-D type I, its transpose (sign=-1),
    at coefficient indices (k1_q, k2_q): out_q = sum_j g_j exp(sign 2 pi i (k1_q x_j + k2_q y_j))."""
    x, y, g = _f64(x), _f64(y), _c128(g)
    k1 = np.ascontiguousarray(k1, dtype=np.int64)
    k2 = np.ascontiguousarray(k2, dtype=np.int64)
    out = np.empty(k1.shape[0], np.complex128)
    rc = _load().oracle_nudft2d_adj(x.shape[0], _p(x), _p(y), _p(g.view(np.float64)),
                                    k1.shape[0], _pi(k1), _pi(k2), int(sign), _p(out.view(np.float64)))
    assert rc == 0
    return out


def grad_x(x, c, g):
    """Gradient in x of a real loss L(f), given g_j = dL/dRe(f_j) + i dL/dIm(f_j)
    (torch's convention for complex tensors).  Calculus on eq. (2) gives
    d f_j / d x_j = sum_k (-2 pi i k) c_k exp(-2 pi i x_j k), so
    grad_x_j = Re(conj(g_j) * d f_j / d x_j).  (The gradient in c is the adjoint
    transform of g: ``nudft1(x, g, N, sign=+1)``.)"""
    c = _c128(c)
    k = np.arange(c.shape[0], dtype=np.float64)
    dfdx = nudft2(x, -2j * np.pi * k * c)
    return np.real(np.conj(_c128(g)) * dfdx)


def grid_assign(x, n):
    """Sec. 2.2: s = round(n x) (ties to even), t = s mod n, delta = n x - s (one rounding)."""
    x = _f64(x)
    m = x.shape[0]
    s = np.empty(m, np.int64)
    t = np.empty(m, np.int64)
    d = np.empty(m, np.float64)
    rc = _load().oracle_grid_assign(int(n), m, _p(x), _pi(s), _pi(t), _p(d))
    if rc != 0:
        raise ValueError("grid_assign: non-finite sample or bad grid size")
    return s, t, d
