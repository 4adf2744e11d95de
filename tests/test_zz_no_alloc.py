"""The allocation-free entry point nufft3_exec_noalloc against nufft3_exec (same
kernels, temporaries in the library's fixed device scratch instead of hipMalloc):
equal results, both within 4 eps ||c||_1 of the FP64 type-III direct sum (Sec. 3.2),
on consecutive calls of decreasing size (the array keeps the previous call's data),
at the largest sizes the scratch serves, and the refusal of larger ones."""
import numpy as np
import pytest
import torch

from oracle import nudft as D
from paper_1701_04492_amd import workloads as W

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1701_04492_amd")
DEV = torch.device("cuda:0")
C64, C128 = torch.complex64, torch.complex128


def _t(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).to(DEV)


def _case(seed, M, N):
    rng = W.rng_for(seed)
    return W.iid_samples(rng, M), rng.uniform(0, N, N), W.complex_normal(rng, N)


def _compare(x, w, c, dtype, eps, rows=None):
    xt, wt, ct = _t(x, torch.float64), _t(w, torch.float64), _t(c, dtype)
    a = P.nufft3_exec_noalloc(xt, wt, ct, eps)
    b = P.nufft3_exec(xt, wt, ct, eps)
    torch.cuda.synchronize()
    same = torch.equal(a, b)
    cc = ct.cpu().numpy().astype(np.complex128)
    rows = np.arange(x.shape[0]) if rows is None else rows
    ref = D.nudft3(x[rows], w, cc)
    err = np.abs(a.cpu().numpy()[rows] - ref).max() / np.abs(cc).sum()
    print("noalloc M=%d N=%d %s eps %g: equal to nufft3_exec %s, err %.3e" % (x.shape[0], w.shape[0], dtype, eps,
                                                                             same, err), flush=True)
    assert same
    assert np.all(np.isfinite(a.cpu().numpy())) and err <= 4 * eps


@pytest.mark.parametrize("dtype,eps", [(C64, 1e-6), (C128, 1e-12)])
def test_noalloc_matches_type3_on_consecutive_calls(dtype, eps):
    # a larger call, then a smaller one reusing the same array
    _compare(*_case(110, 40000, 20000), dtype, eps, rows=np.random.default_rng(1).choice(40000, 300, replace=False))
    _compare(*_case(111, 700, 300), dtype, eps)


def test_noalloc_largest_sizes():
    M, N = 1 << 20, 1 << 15
    x, w, c = _case(112, M, N)
    rows = np.unique(np.concatenate([np.random.default_rng(2).choice(M, 64, replace=False), [0, M - 1]]))
    _compare(x, w, c, C128, 1e-12, rows=rows)


def test_noalloc_refuses_larger_sizes():
    x, w, c = _case(113, (1 << 20) + 1, 16)
    with pytest.raises(P.NufftError) as e:
        P.nufft3_exec_noalloc(_t(x, torch.float64), _t(w, torch.float64), _t(c, C64), 1e-6)
    assert e.value.status == 2
    x, w, c = _case(114, 16, (1 << 15) + 1)
    with pytest.raises(P.NufftError) as e:
        P.nufft3_exec_noalloc(_t(x, torch.float64), _t(w, torch.float64), _t(c, C64), 1e-6)
    assert e.value.status == 2
