"""Thin ctypes binding of ``libnufft_mi355x.so``: one Python function per C
entry point of ``include/nufft_mi355x.h``, same names, argument marshalling
only (tensor -> device pointer, torch's current HIP stream -> hipStream_t).
Every transform runs in the library's HIP kernels; there is no fallback: if
the library is not built, importing this module raises.
"""
import ctypes
import os
import re
import sys

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnufft_mi355x.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "nufft_mi355x.h")

NUFFT_C64, NUFFT_C128 = 0, 1
NUFFT_FLAG_FIX_GAMMA_HALF = 1
NUFFT_FLAG_PLAIN_UNFUSED = 2
NUFFT_FLAG_NO_AUTOTUNE = 4
NUFFT_FLAG_HALF_EXCHANGE = 8
NUFFT_FLAG_BATCH_PERSISTENT = 16
STATUS = {0: "NUFFT_OK", 1: "NUFFT_ERR_INVALID_ARG", 2: "NUFFT_ERR_UNSUPPORTED", 3: "NUFFT_ERR_ALLOC",
          4: "NUFFT_ERR_NONFINITE", 5: "NUFFT_ERR_HIP"}

if not os.path.exists(LIB_PATH):
    raise ImportError("libnufft_mi355x.so is not built (run paper_1701_04492_amd/build.py "
                      "or __graft_entry__.build()); there is no CPU fallback")

_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_u32 = ctypes.c_uint32
_int = ctypes.c_int
_dbl = ctypes.c_double
lib = ctypes.CDLL(LIB_PATH)
_sig = {
    "nufft2_plan": [ctypes.POINTER(_vp), _i64, _i64, _vp, _dbl, _int, _u32, _vp],
    "nufft2_plan_grid": [ctypes.POINTER(_vp), _i64, _i64, _vp, _dbl, _int, _u32, _i64, _vp],
    "nufft2_exec": [_vp, _vp, _vp, _vp],
    "nufft1_exec": [_vp, _vp, _vp, _int, _vp],
    "nufft2_grad_x": [_vp, _vp, _vp, _vp, _vp],
    "nufft2_backward": [_vp, _vp, _vp, _vp, _vp, _vp],
    "nufft2_solve": [_vp, _vp, _vp, _dbl, _int, ctypes.POINTER(_int), ctypes.POINTER(_dbl), _vp],
    "nufft1_solve": [_vp, _vp, _vp, _dbl, _int, ctypes.POINTER(_int), ctypes.POINTER(_dbl), _vp],
    "nufft3_exec": [_i64, _vp, _i64, _vp, _vp, _vp, _dbl, _int, _vp],
    "nufft3_exec_noalloc": [_i64, _vp, _i64, _vp, _vp, _vp, _dbl, _int, _vp],
    "nufft2d3_exec": [_i64, _vp, _vp, _i64, _vp, _vp, _i64, _i64, _vp, _vp, _dbl, _int, _vp],
    "nufft3d_exec": [_i64, _vp, _vp, _vp, _i64, _i64, _i64, _vp, _vp, _dbl, _int, _vp],
    "nufft3d_type1_exec": [_i64, _vp, _vp, _vp, _i64, _i64, _i64, _vp, _vp, _int, _dbl, _int, _vp],
    "nufft3d_plan": [ctypes.POINTER(_vp), _i64, _i64, _i64, _i64, _vp, _vp, _vp, _dbl, _int, _vp],
    "nufft3d_plan_exec": [_vp, _vp, _vp, _vp],
    "nufft3d_plan_type1": [_vp, _vp, _vp, _int, _vp],
    "nufft2d_plan": [ctypes.POINTER(_vp), _i64, _i64, _i64, _vp, _vp, _dbl, _int, _u32, _vp],
    "nufft2d_exec": [_vp, _vp, _vp, _int, _vp],
    "nufft2d_type1_exec": [_vp, _vp, _vp, _int, _vp],
    "nufft_batch_plan": [ctypes.POINTER(_vp), _int, _vp, _vp, _vp, _dbl, _int, _u32, _vp],
    "nufft_batch_exec": [_vp, _vp, _vp, _vp],
    "nufft_plan_info": [_vp, ctypes.POINTER(_int), ctypes.POINTER(_dbl), ctypes.POINTER(_i64)],
    "nufft_plan_perm": [_vp, _vp],
    "nufft_destroy": [_vp],
    "nufft_status_string": [_int],
    "nufft_plan_profile": [_vp, _int, _int],
    "nufft_plan_profile_read": [_vp, _int, ctypes.c_char_p, _int, ctypes.POINTER(_int), ctypes.POINTER(_dbl)],
    "nufft_debug_fail_alloc": [_i64],
    "nufft_batch_status": [_vp, ctypes.POINTER(_i64), _vp],
    "nufft_plan_tuning": [_vp, ctypes.POINTER(_int), ctypes.POINTER(_int)],
    "nufft_debug_set_schedule": [_vp, _int],
    "nufft_debug_set_buckets": [_vp, _int, ctypes.POINTER(_int)],
    "nufft_debug_batch_wait": [_vp, _i64, _int],
    "nufft_choose_rank": [_dbl, _dbl, ctypes.POINTER(_int)],
    "nufft_bessel_coefficients": [_dbl, _int, _vp],
}
for _n, _a in _sig.items():
    _f = getattr(lib, _n)
    _f.argtypes = _a
    _f.restype = _int
lib.nufft_status_string.restype = ctypes.c_char_p


def header_functions():
    """Names of the functions declared in include/nufft_mi355x.h."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:nufft_status|const char \*)\s*(\w+)\s*\(", txt, re.M)))


class NufftError(RuntimeError):
    def __init__(self, status, where):
        self.status = int(status)
        super().__init__("%s: %s (%s)" % (where, STATUS.get(self.status, "?"),
                                          lib.nufft_status_string(self.status).decode()))


def _check(st, where):
    if st != 0:
        raise NufftError(st, where)


def _stream(dev):
    return _vp(torch.cuda.current_stream(dev).cuda_stream)


def _res(t):
    """An input with its lazy conjugate / negative bits materialised: such a view shares
    the unconjugated storage, so its raw pointer would carry the wrong values."""
    if isinstance(t, torch.Tensor) and (t.is_conj() or t.is_neg()):
        return t.resolve_conj().resolve_neg()
    return t


def _dev_tensor(t, dtype, n, name):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise ValueError("%s must be a CUDA (HIP) tensor" % name)
    if t.is_conj() or t.is_neg():
        raise ValueError("%s is a lazily conjugated or negated view; resolve it first" % name)
    if t.dtype != dtype:
        raise ValueError("%s must have dtype %s, got %s" % (name, dtype, t.dtype))
    if n is not None and t.numel() != n:
        raise ValueError("%s must have %d elements, got %d" % (name, n, t.numel()))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return _vp(t.data_ptr())


def _cdtype(dtype):
    if dtype == torch.complex64:
        return NUFFT_C64
    if dtype == torch.complex128:
        return NUFFT_C128
    raise ValueError("dtype must be torch.complex64 or torch.complex128")


class Plan:
    """Owner of a nufft_plan_t; destroyed with the object."""

    def __init__(self, handle, kind, dtype, device, **meta):
        self.handle = handle
        self.kind = kind
        self.dtype = dtype
        self.device = device
        self.__dict__.update(meta)
        K = _int()
        g = _dbl()
        L = _i64()
        _check(lib.nufft_plan_info(self.handle, ctypes.byref(K), ctypes.byref(g), ctypes.byref(L)),
               "nufft_plan_info")
        self.K, self.gamma, self.grid = K.value, g.value, L.value

    def __del__(self):
        h = getattr(self, "handle", None)
        # at interpreter exit the process releases device memory itself
        if h and lib is not None and not sys.is_finalizing():
            lib.nufft_destroy(h)
            self.handle = None


def nufft2_plan(x, n_modes, eps, dtype=torch.complex64, flags=0, grid=None):
    """Plan a 1-D type II / type I transform on samples x (float64 CUDA tensor);
    grid: an explicit FFT grid (nufft2_plan_grid), else chosen and autotuned."""
    M = x.numel()
    px = _dev_tensor(x, torch.float64, None, "x")
    h = _vp()
    if grid is None:
        _check(lib.nufft2_plan(ctypes.byref(h), int(n_modes), M, px, float(eps), _cdtype(dtype), int(flags),
                               _stream(x.device)), "nufft2_plan")
    else:
        _check(lib.nufft2_plan_grid(ctypes.byref(h), int(n_modes), M, px, float(eps), _cdtype(dtype), int(flags),
                                    int(grid), _stream(x.device)), "nufft2_plan_grid")
    return Plan(h, "1d", dtype, x.device, N=int(n_modes), M=M, eps=float(eps), flags=int(flags),
                x_key=(x.data_ptr(), x._version, M))


def nufft2_plan_grid(x, n_modes, eps, dtype, flags, grid):
    return nufft2_plan(x, n_modes, eps, dtype, flags, grid)


def nufft2_exec(plan, c, f=None):
    if f is None:
        f = torch.empty(plan.M, dtype=plan.dtype, device=plan.device)
    c = _res(c)
    _check(lib.nufft2_exec(plan.handle, _dev_tensor(c, plan.dtype, plan.N, "c"),
                           _dev_tensor(f, plan.dtype, plan.M, "f"), _stream(plan.device)), "nufft2_exec")
    return f


def nufft1_exec(plan, c, sign=-1, f=None):
    if f is None:
        f = torch.empty(plan.N, dtype=plan.dtype, device=plan.device)
    c = _res(c)
    _check(lib.nufft1_exec(plan.handle, _dev_tensor(c, plan.dtype, plan.M, "c"),
                           _dev_tensor(f, plan.dtype, plan.N, "f"), int(sign), _stream(plan.device)),
           "nufft1_exec")
    return f


def nufft2_grad_x(plan, c, g, gx=None):
    if gx is None:
        gx = torch.empty(plan.M, dtype=torch.float64, device=plan.device)
    c, g = _res(c), _res(g)
    _check(lib.nufft2_grad_x(plan.handle, _dev_tensor(c, plan.dtype, plan.N, "c"),
                             _dev_tensor(g, plan.dtype, plan.M, "g"),
                             _dev_tensor(gx, torch.float64, plan.M, "gx"), _stream(plan.device)),
           "nufft2_grad_x")
    return gx


def nufft2_backward(plan, c, g, gc=None, gx=None, need_c=True, need_x=True):
    """Both gradients of a real loss through f = F2 c: (F2^H g, Re(conj(g) F2(-2 pi i k c)));
    a gradient that is not needed is returned as None."""
    if not (need_c or need_x):
        raise ValueError("nufft2_backward: nothing requested")
    if need_c and gc is None:
        gc = torch.empty(plan.N, dtype=plan.dtype, device=plan.device)
    if need_x and gx is None:
        gx = torch.empty(plan.M, dtype=torch.float64, device=plan.device)
    c, g = _res(c), _res(g)
    _check(lib.nufft2_backward(plan.handle, _dev_tensor(c, plan.dtype, plan.N, "c") if need_x else None,
                               _dev_tensor(g, plan.dtype, plan.M, "g"),
                               _dev_tensor(gc, plan.dtype, plan.N, "gc") if need_c else None,
                               _dev_tensor(gx, torch.float64, plan.M, "gx") if need_x else None,
                               _stream(plan.device)), "nufft2_backward")
    return (gc if need_c else None), (gx if need_x else None)


def nufft2_solve(plan, f, c=None, tol=1e-6, max_iter=200):
    """Inverse type II (Sec. 3.3): least-squares c with F2 c ~ f, by CG on the normal
    equations.  Returns (c, iterations, relative residual of the normal equations)."""
    if c is None:
        c = torch.empty(plan.N, dtype=plan.dtype, device=plan.device)
    it = _int()
    res = _dbl()
    f = _res(f)
    _check(lib.nufft2_solve(plan.handle, _dev_tensor(f, plan.dtype, plan.M, "f"),
                            _dev_tensor(c, plan.dtype, plan.N, "c"), float(tol), int(max_iter),
                            ctypes.byref(it), ctypes.byref(res), _stream(plan.device)), "nufft2_solve")
    return c, it.value, res.value


def nufft1_solve(plan, f, c=None, tol=1e-6, max_iter=200):
    """Inverse type I (Sec. 3.3): the minimum-norm c with F1 c ~ f (F1 = F2^T), by CG on
    F1 F1^* y = f and c = F1^* y.  Returns (c, iterations, relative residual)."""
    if c is None:
        c = torch.empty(plan.M, dtype=plan.dtype, device=plan.device)
    it = _int()
    res = _dbl()
    f = _res(f)
    _check(lib.nufft1_solve(plan.handle, _dev_tensor(f, plan.dtype, plan.N, "f"),
                            _dev_tensor(c, plan.dtype, plan.M, "c"), float(tol), int(max_iter),
                            ctypes.byref(it), ctypes.byref(res), _stream(plan.device)), "nufft1_solve")
    return c, it.value, res.value


def nufft3_exec(x, w, c, eps, f=None):
    M, N = x.numel(), w.numel()
    c = _res(c)
    if f is None:
        f = torch.empty(M, dtype=c.dtype, device=c.device)
    _check(lib.nufft3_exec(M, _dev_tensor(x, torch.float64, M, "x"), N, _dev_tensor(w, torch.float64, N, "w"),
                           _dev_tensor(c, c.dtype, N, "c"), _dev_tensor(f, c.dtype, M, "f"), float(eps),
                           _cdtype(c.dtype), _stream(c.device)), "nufft3_exec")
    return f


def nufft3_exec_noalloc(x, w, c, eps, f=None):
    """nufft3_exec with every temporary in the library's fixed device scratch (no device
    allocation inside the call; M <= 2^20, N <= 2^15)."""
    M, N = x.numel(), w.numel()
    c = _res(c)
    if f is None:
        f = torch.empty(M, dtype=c.dtype, device=c.device)
    _check(lib.nufft3_exec_noalloc(M, _dev_tensor(x, torch.float64, M, "x"), N,
                                   _dev_tensor(w, torch.float64, N, "w"), _dev_tensor(c, c.dtype, N, "c"),
                                   _dev_tensor(f, c.dtype, M, "f"), float(eps), _cdtype(c.dtype),
                                   _stream(c.device)), "nufft3_exec_noalloc")
    return f


def nufft2d3_exec(x, y, w1, w2, n1, n2, c, eps, f=None):
    """2-D type III: f_j = sum_k c_k exp(-2 pi i (x_j w1_k + y_j w2_k)); x, y in [0, 1),
    w1 in [0, n1), w2 in [0, n2)."""
    M, Q = x.numel(), w1.numel()
    c = _res(c)
    if f is None:
        f = torch.empty(M, dtype=c.dtype, device=c.device)
    _check(lib.nufft2d3_exec(M, _dev_tensor(x, torch.float64, M, "x"), _dev_tensor(y, torch.float64, M, "y"), Q,
                             _dev_tensor(w1, torch.float64, Q, "w1"), _dev_tensor(w2, torch.float64, Q, "w2"),
                             int(n1), int(n2), _dev_tensor(c, c.dtype, Q, "c"), _dev_tensor(f, c.dtype, M, "f"),
                             float(eps), _cdtype(c.dtype), _stream(c.device)), "nufft2d3_exec")
    return f


def nufft3d_exec(x, y, z, C, eps, f=None):
    """3-D type II: f_j = sum_{k1,k2,k3} C[k1,k2,k3] exp(-2 pi i (k1 x_j + k2 y_j + k3 z_j)); C is
    an (n1, n2, n3) complex tensor (row-major)."""
    M = x.numel()
    n1, n2, n3 = C.shape
    Cf = _res(C).reshape(-1)   # held here for the duration of the call
    if f is None:
        f = torch.empty(M, dtype=C.dtype, device=C.device)
    _check(lib.nufft3d_exec(M, _dev_tensor(x, torch.float64, M, "x"), _dev_tensor(y, torch.float64, M, "y"),
                            _dev_tensor(z, torch.float64, M, "z"), int(n1), int(n2), int(n3),
                            _dev_tensor(Cf, C.dtype, n1 * n2 * n3, "C"), _dev_tensor(f, C.dtype, M, "f"),
                            float(eps), _cdtype(C.dtype), _stream(C.device)), "nufft3d_exec")
    return f


def nufft3d_type1_exec(x, y, z, c, shape, eps, sign=-1, C=None):
    """3-D type I (sign=-1) or adjoint (sign=+1):
    C[k1,k2,k3] = sum_j c_j exp(sign 2 pi i (k1 x_j + k2 y_j + k3 z_j)), shape = (n1, n2, n3)."""
    M = x.numel()
    n1, n2, n3 = (int(v) for v in shape)
    c = _res(c)
    if C is None:
        C = torch.empty((n1, n2, n3), dtype=c.dtype, device=c.device)
    _check(lib.nufft3d_type1_exec(M, _dev_tensor(x, torch.float64, M, "x"), _dev_tensor(y, torch.float64, M, "y"),
                                  _dev_tensor(z, torch.float64, M, "z"), n1, n2, n3,
                                  _dev_tensor(c, c.dtype, M, "c"), _dev_tensor(C, c.dtype, n1 * n2 * n3, "C"),
                                  int(sign), float(eps), _cdtype(c.dtype), _stream(c.device)), "nufft3d_type1_exec")
    return C


def nufft3d_plan(x, y, z, shape, eps, dtype=torch.complex64):
    """A reusable 3-D plan for the samples (x, y, z) and the n1 x n2 x n3 modes of ``shape``."""
    M = x.numel()
    n1, n2, n3 = (int(v) for v in shape)
    h = _vp()
    _check(lib.nufft3d_plan(ctypes.byref(h), n1, n2, n3, M, _dev_tensor(x, torch.float64, M, "x"),
                            _dev_tensor(y, torch.float64, M, "y"), _dev_tensor(z, torch.float64, M, "z"),
                            float(eps), _cdtype(dtype), _stream(x.device)), "nufft3d_plan")
    return Plan(h, "3d", dtype, x.device, shape=(n1, n2, n3), M=M, eps=float(eps))


def nufft3d_plan_exec(plan, C, f=None):
    """3-D type II on a 3-D plan: C (n1, n2, n3) -> f (M)."""
    n = plan.shape[0] * plan.shape[1] * plan.shape[2]
    C = _res(C)
    if f is None:
        f = torch.empty(plan.M, dtype=plan.dtype, device=plan.device)
    _check(lib.nufft3d_plan_exec(plan.handle, _dev_tensor(C, plan.dtype, n, "C"),
                                 _dev_tensor(f, plan.dtype, plan.M, "f"), _stream(plan.device)), "nufft3d_plan_exec")
    return f


def nufft3d_plan_type1(plan, c, sign=-1, C=None):
    """3-D type I (sign -1) or adjoint (sign +1) on a 3-D plan: c (M) -> C (n1, n2, n3)."""
    if C is None:
        C = torch.empty(plan.shape, dtype=plan.dtype, device=plan.device)
    n = plan.shape[0] * plan.shape[1] * plan.shape[2]
    c = _res(c)
    _check(lib.nufft3d_plan_type1(plan.handle, _dev_tensor(c, plan.dtype, plan.M, "c"),
                                  _dev_tensor(C, plan.dtype, n, "C"), int(sign), _stream(plan.device)),
           "nufft3d_plan_type1")
    return C


def nufft2d_plan(x, y, n1, n2, eps, dtype=torch.complex64, flags=0):
    M = x.numel()
    h = _vp()
    _check(lib.nufft2d_plan(ctypes.byref(h), int(n1), int(n2), M, _dev_tensor(x, torch.float64, M, "x"),
                            _dev_tensor(y, torch.float64, M, "y"), float(eps), _cdtype(dtype), int(flags),
                            _stream(x.device)), "nufft2d_plan")
    return Plan(h, "2d", dtype, x.device, n1=int(n1), n2=int(n2), M=M, eps=float(eps), flags=int(flags))


def nufft2d_exec(plan, C, f, adjoint=0):
    """adjoint=0: f <- F C (C read); adjoint=1: C <- F^H f (f read).  The output is overwritten."""
    if adjoint:
        f = _res(f)
    else:
        C = _res(C)
    _check(lib.nufft2d_exec(plan.handle, _dev_tensor(C, plan.dtype, plan.n1 * plan.n2, "C"),
                            _dev_tensor(f, plan.dtype, plan.M, "f"), int(adjoint), _stream(plan.device)),
           "nufft2d_exec")


def nufft2d_type1_exec(plan, c, F=None, sign=-1):
    """2-D type I (sign -1) or adjoint (sign +1) on the plan's samples: c (M) -> F (n1*n2)."""
    if F is None:
        F = torch.empty(plan.n1 * plan.n2, dtype=plan.dtype, device=plan.device)
    c = _res(c)
    _check(lib.nufft2d_type1_exec(plan.handle, _dev_tensor(c, plan.dtype, plan.M, "c"),
                                  _dev_tensor(F, plan.dtype, plan.n1 * plan.n2, "F"), int(sign),
                                  _stream(plan.device)), "nufft2d_type1_exec")
    return F


def nufft_batch_plan(n_modes, xs, eps, dtype=torch.complex64, flags=0):
    B = len(xs)
    nm = (ctypes.c_int64 * B)(*[int(n) for n in n_modes])
    npts = (ctypes.c_int64 * B)(*[int(x.numel()) for x in xs])
    ptrs = (ctypes.c_void_p * B)(*[_dev_tensor(x, torch.float64, None, "x").value for x in xs])
    h = _vp()
    _check(lib.nufft_batch_plan(ctypes.byref(h), B, ctypes.cast(nm, _vp), ctypes.cast(npts, _vp),
                                ctypes.cast(ptrs, _vp), float(eps), _cdtype(dtype), int(flags),
                                _stream(xs[0].device)), "nufft_batch_plan")
    return Plan(h, "batch", dtype, xs[0].device, Ns=[int(n) for n in n_modes],
                Ms=[int(x.numel()) for x in xs], eps=float(eps), flags=int(flags))


def nufft_batch_exec(plan, cs, fs):
    B = len(cs)
    cs = [_res(c) for c in cs]
    cp = (ctypes.c_void_p * B)(*[_dev_tensor(c, plan.dtype, n, "c").value for c, n in zip(cs, plan.Ns)])
    fp = (ctypes.c_void_p * B)(*[_dev_tensor(f, plan.dtype, m, "f").value for f, m in zip(fs, plan.Ms)])
    _check(lib.nufft_batch_exec(plan.handle, ctypes.cast(cp, _vp), ctypes.cast(fp, _vp),
                                _stream(plan.device)), "nufft_batch_exec")


def nufft_batch_status(plan):
    """Waits for the current stream and returns the number of persistent-launch waits that
    gave up since the previous call (0 for a healthy plan), clearing the count."""
    n = _i64()
    _check(lib.nufft_batch_status(plan.handle, ctypes.byref(n), _stream(plan.device)), "nufft_batch_status")
    return n.value


def nufft_debug_batch_wait(plan, spin_limit, unreachable=False):
    """Bound of the persistent launch's pass-B waits, and (tests) an unreachable wait target."""
    _check(lib.nufft_debug_batch_wait(plan.handle, int(spin_limit), int(bool(unreachable))),
           "nufft_debug_batch_wait")


def nufft_plan_tuning(plan):
    """(schedule in use, number of schedules the plan offers)."""
    sc, n = _int(), _int()
    _check(lib.nufft_plan_tuning(plan.handle, ctypes.byref(sc), ctypes.byref(n)), "nufft_plan_tuning")
    return sc.value, n.value


def nufft_debug_set_schedule(plan, schedule):
    _check(lib.nufft_debug_set_schedule(plan.handle, int(schedule)), "nufft_debug_set_schedule")


def nufft_debug_set_buckets(plan, enable):
    """Switches the plan's destination-bucketed permutations on or off; returns
    whether the plan has them."""
    has = _int(0)
    _check(lib.nufft_debug_set_buckets(plan.handle, int(bool(enable)), ctypes.byref(has)), "nufft_debug_set_buckets")
    return bool(has.value)


def nufft_plan_info(plan):
    return plan.K, plan.gamma, plan.grid


def nufft_plan_perm(plan):
    out = np.empty(plan.M, np.int32)
    _check(lib.nufft_plan_perm(plan.handle, _vp(out.ctypes.data)), "nufft_plan_perm")
    return out


def nufft_destroy(plan):
    plan.__del__()


def nufft_plan_profile(plan, enable=1, reserve=0):
    _check(lib.nufft_plan_profile(plan.handle, int(enable), int(reserve)), "nufft_plan_profile")


def nufft_plan_profile_read(plan):
    """{kernel name: (launches, total ms)} recorded since the last nufft_plan_profile call."""
    out = {}
    i = 0
    buf = ctypes.create_string_buffer(64)
    while True:
        calls = _int()
        ms = _dbl()
        st = lib.nufft_plan_profile_read(plan.handle, i, buf, 64, ctypes.byref(calls), ctypes.byref(ms))
        if st == 1:
            break
        _check(st, "nufft_plan_profile_read")
        out[buf.value.decode()] = (calls.value, ms.value)
        i += 1
    return out


def nufft_status_string(status):
    return lib.nufft_status_string(int(status)).decode()


def nufft_debug_fail_alloc(n):
    """Refuse the device allocation n allocations from now (n < 0: disarm); for tests of
    error handling."""
    _check(lib.nufft_debug_fail_alloc(int(n)), "nufft_debug_fail_alloc")


def nufft_choose_rank(eps, gamma):
    K = _int()
    _check(lib.nufft_choose_rank(float(eps), float(gamma), ctypes.byref(K)), "nufft_choose_rank")
    return K.value


def nufft_bessel_coefficients(gamma, K):
    b = np.empty(K * K, np.float64)
    _check(lib.nufft_bessel_coefficients(float(gamma), int(K), _vp(b.ctypes.data)), "nufft_bessel_coefficients")
    return b.reshape(K, K)
