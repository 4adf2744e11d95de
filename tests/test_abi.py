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


def test_plan_grid_argument_errors():
    """Explicit grids the kernels cannot run are refused before any device work."""
    h, p = ctypes.c_void_p(), ctypes.c_void_p(8)
    f = B.lib.nufft2_plan_grid
    assert f(ctypes.byref(h), 1000, 16, p, 1e-6, 0, 0, 0, None) == 1            # no grid
    assert f(ctypes.byref(h), 1000, 16, p, 1e-6, 0, 0, 512, None) == 2          # grid < N
    assert f(ctypes.byref(h), 1000, 16, p, 1e-6, 0, 0, 7 * 4096, None) == 2     # no radix-7 stage
    assert f(ctypes.byref(h), 1000, 16, p, 1e-6, 0, 0, 3072, None) == 2         # mixed only in the two-pass range
    assert f(ctypes.byref(h), 1000, 16, p, 1e-6, 0, 0, 5 * 4096, None) == 2     # 5 x 64 columns need L1 >= 128
    assert f(ctypes.byref(h), 1000, 16, p, 1e-6, 0, 0, 3 << 22, None) == 2      # beyond 2^23
    assert f(ctypes.byref(h), 1000, 16, p, 1e-6, 0, 2, 24576, None) == 2        # plain path: powers of two
    assert f(ctypes.byref(h), 1000, 16, p, 1e-6, 0, 8, 24576, None) == 2        # half exchange: powers of two
    assert f(None, 1000, 16, p, 1e-6, 0, 0, 24576, None) == 1


def test_enum_values_are_pinned():
    """Status codes, dtypes and flag bits as the header declares them (and the binding mirrors)."""
    import re
    txt = open(B.HEADER).read()
    vals = dict((m.group(1), int(m.group(2))) for m in re.finditer(r"(NUFFT_\w+)\s*=\s*(\d+)u?", txt))
    want = {"NUFFT_OK": 0, "NUFFT_ERR_INVALID_ARG": 1, "NUFFT_ERR_UNSUPPORTED": 2, "NUFFT_ERR_ALLOC": 3,
            "NUFFT_ERR_NONFINITE": 4, "NUFFT_ERR_HIP": 5, "NUFFT_C64": 0, "NUFFT_C128": 1,
            "NUFFT_FLAG_FIX_GAMMA_HALF": 1, "NUFFT_FLAG_PLAIN_UNFUSED": 2, "NUFFT_FLAG_NO_AUTOTUNE": 4,
            "NUFFT_FLAG_HALF_EXCHANGE": 8, "NUFFT_FLAG_BATCH_PERSISTENT": 16}
    for k, v in want.items():
        assert vals.get(k) == v, k
        if k.startswith("NUFFT_FLAG") or k.startswith("NUFFT_C"):
            assert getattr(B, k) == v, k
    assert "NUFFT_FLAG_AUTOTUNE" not in vals and "NUFFT_FLAG_PLAIN" not in vals


def test_batch_and_debug_entry_points_reject_bad_handles():
    n = ctypes.c_int64()
    assert B.lib.nufft_batch_status(None, ctypes.byref(n), None) == 1
    assert B.lib.nufft_debug_batch_wait(None, 10, 1) == 1


def test_noalloc_entry_point_refuses_sizes_beyond_its_scratch():
    """Refused on the host before any device work (no GPU needed): M > 2^20 or N > 2^15."""
    p = ctypes.c_void_p(8)
    assert B.lib.nufft3_exec_noalloc((1 << 20) + 1, p, 16, p, p, p, 1e-6, 0, None) == 2
    assert B.lib.nufft3_exec_noalloc(16, p, (1 << 15) + 1, p, p, p, 1e-6, 0, None) == 2
    assert B.lib.nufft3_exec_noalloc(0, p, 16, p, p, p, 1e-6, 0, None) == 1
