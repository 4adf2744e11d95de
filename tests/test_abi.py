"""The C-ABI library loads and exports every declared entry point; host-only
parts (factor generator, argument checks) are checked on the CPU.  No GPU
compute is launched here."""
import ctypes

import numpy as np
import pytest

B = pytest.importorskip("paper_1701_04492_amd.binding")
from oracle import lowrank as L  # noqa: E402


def test_every_declared_symbol_is_exported():
    names = B.header_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(B.lib, n), n


def test_status_strings():
    for st in range(6):
        assert B.nufft_status_string(st)
    assert B.nufft_status_string(99) == "unknown status"


@pytest.mark.parametrize("eps", [9.765625e-4, 1.1920928955078125e-07, 1e-6, 1e-9, 1e-12, 1e-14])
def test_rank_matches_oracle(eps):
    for g in [0.0, 1e-3, 1 / 32, 0.05, 1 / 16, 0.1, 1 / 8, 0.2, 1 / 4, 0.37, 0.5]:
        assert B.nufft_choose_rank(eps, g) == L.choose_K(eps, g), (eps, g)


def test_bessel_coefficients_match_oracle():
    for g in [0.0, 1 / 32, 0.25, 0.5]:
        K = 16
        b = B.nufft_bessel_coefficients(g, K)
        a = L.chebyshev_coefficients(g, K)
        ref = (a / (1j ** np.arange(K))[None, :]).real
        assert np.abs(b - ref).max() <= 1e-15 * max(1.0, np.abs(ref).max())


def test_host_argument_errors():
    with pytest.raises(B.NufftError) as e:
        B.nufft_choose_rank(0.0, 0.5)
    assert e.value.status == 1
    with pytest.raises(B.NufftError):
        B.nufft_choose_rank(1e-6, 0.7)
    with pytest.raises(B.NufftError) as e:
        B.nufft_choose_rank(1e-40, 0.5)
    assert e.value.status == 2
    h = ctypes.c_void_p()
    # rejected before any device work: bad sizes, NULL pointers, eps below the precision floor
    assert B.lib.nufft2_plan(None, 16, 16, ctypes.c_void_p(8), 1e-6, 0, 0, None) == 1
    assert B.lib.nufft2_plan(ctypes.byref(h), 0, 16, ctypes.c_void_p(8), 1e-6, 0, 0, None) == 1
    assert B.lib.nufft2_plan(ctypes.byref(h), 16, 0, ctypes.c_void_p(8), 1e-6, 0, 0, None) == 1
    assert B.lib.nufft2_plan(ctypes.byref(h), 16, 16, None, 1e-6, 0, 0, None) == 1
    assert B.lib.nufft2_plan(ctypes.byref(h), 16, 16, ctypes.c_void_p(8), 1e-9, 0, 0, None) == 2
    assert B.lib.nufft2_plan(ctypes.byref(h), 16, 16, ctypes.c_void_p(8), 1e-16, 1, 0, None) == 2
    assert B.lib.nufft2_plan(ctypes.byref(h), 16, 16, ctypes.c_void_p(8), 1.5, 1, 0, None) == 1
    assert B.lib.nufft2_plan(ctypes.byref(h), 16, 16, ctypes.c_void_p(8), 1e-6, 7, 0, None) == 1
    assert B.lib.nufft2_plan(ctypes.byref(h), 16, 16, ctypes.c_void_p(8), 1e-6, 0, 64, None) == 1
    assert B.lib.nufft2_plan(ctypes.byref(h), 1 << 24 + 1, 16, ctypes.c_void_p(8), 1e-6, 0, 0, None) == 2
    assert B.lib.nufft2_exec(None, None, None, None) == 1
    assert B.lib.nufft1_exec(None, None, None, -1, None) == 1
    assert B.lib.nufft_destroy(None) == 0
