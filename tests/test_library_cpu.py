"""Host-side checks of the HIP library (no GPU needed): it loads, exports
every entry point of include/tbs.h, and its host helpers (padded lengths,
wavenumbers, FP64 Hankel functions, self-cell weights, argument validation)
are right."""
import ctypes
import os
import re

import numpy as np
import pytest
import scipy.special

import oracle
import paper_2507_13754_amd as tbs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_header_symbol():
    hdr = open(os.path.join(ROOT, "include", "tbs.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    declared = set(re.findall(r"\b(tbs_[a-z0-9_]+)\s*\(", hdr))
    assert declared == set(tbs.EXPORTS)
    lib = tbs.library()
    for name in declared:
        assert hasattr(lib, name), name
    assert lib.tbs_version() >= 100


@pytest.mark.parametrize("n,pad,m", [(1, 2, 16), (8, 2, 16), (9, 2, 32), (256, 2, 512),
                                     (2048, 2, 4096), (37, 2, 80), (100, 3, 320), (300, 2, 640),
                                     (380, 2, 768), (1247, 2, 2560), (1100, 2, 2560), (1500, 2, 3072)])
def test_padded_length(n, pad, m):
    got = tbs.padded_length(n, pad)
    assert got == m and got >= pad * n - 1 and got % 2 == 0


def test_padded_length_errors():
    with pytest.raises(tbs.TBSError):
        tbs.padded_length(5000, 2)
    with pytest.raises(tbs.TBSError):
        tbs.padded_length(10, 1)


@pytest.mark.parametrize("y", [1.0, 1.5, 1.2])
def test_wavenumber_matches_oracle(y):
    for f in (1e6, 5e6):
        om = 2 * np.pi * f
        a0 = 5.48e-10 if y != 1.0 else 9.2e-7
        assert abs(tbs.wavenumber(om, 1500.0, a0, y) - complex(oracle.wavenumber(om, 1500.0, a0, y))) \
            < 1e-13 * abs(om / 1500)
        for eps in (0.0, 3e4):
            k_lib = tbs.background_k0(om, 1540.0, a0, y, eps)
            k_or = oracle.background_k0(om, 1540.0, a0, y, eps)
            assert abs(k_lib - k_or) < 1e-13 * abs(k_or)


def test_hankel_matches_scipy():
    rng = np.random.default_rng(3)
    worst = 0.0
    for mag in np.concatenate([np.logspace(-6, 4.2, 300), rng.uniform(0.5, 40, 100)]):
        for ang in (0.0, 1e-3, 0.01, 0.1, 0.5):
            z = mag * np.exp(1j * ang)
            if z.imag > 200:
                continue
            h0, h1 = tbs.hankel01(complex(z))
            r0, r1 = scipy.special.hankel1(0, z), scipy.special.hankel1(1, z)
            worst = max(worst, abs(h0 - r0) / abs(r0), abs(h1 - r1) / abs(r1))
    assert worst < 1e-13, worst


@pytest.mark.parametrize("k0", [2 * np.pi / 6 * (1 + 0.004j), 0.9 + 0.2j, 2.5 + 0j, 0.3 + 0.01j, 5 + 0.1j])
@pytest.mark.parametrize("ndim", [2, 3])
def test_self_cell_matches_oracle(k0, ndim):
    w = tbs.self_cell(ndim, k0, 1.0)
    r = oracle.self_cell(k0, 1.0, ndim)
    assert abs(w - r) < 2e-14 * abs(r) * (10 if abs(k0) < 0.5 else 1)


def test_plan_create_rejects_bad_arguments():
    L = tbs.library()
    h = ctypes.c_void_p()
    g = (ctypes.c_int64 * 3)(64, 64, 1)
    k0 = tbs.c128(100.0, 1.0)
    bad = [
        (3 * 0 + 4, g, 1e-3, k0, 2, 0, 1),            # ndim
        (2, g, -1.0, k0, 2, 0, 1),                    # dx
        (2, g, 1e-3, tbs.c128(-1.0, 0.0), 2, 0, 1),   # Re k0 <= 0
        (2, g, 1e-3, tbs.c128(1.0, -1.0), 2, 0, 1),   # Im k0 < 0
        (2, g, 1e-3, k0, 0, 0, 1),                    # padding
        (2, g, 1e-3, k0, 2, 7, 1),                    # dtype
        (2, g, 1e-3, k0, 2, 0, 0),                    # batch
    ]
    for nd, gg, dx, kk, pad, dt, b in bad:
        rc = L.tbs_plan_create(ctypes.byref(h), nd, gg, dx, kk, pad, dt, b, None)
        assert rc == -1, (nd, dx, pad, dt, b)
        assert h.value is None
        assert len(L.tbs_last_error(None)) > 0
    g2 = (ctypes.c_int64 * 3)(5000, 64, 1)
    assert L.tbs_plan_create(ctypes.byref(h), 2, g2, 1e-3, k0, 2, 0, 1, None) == -2


def test_null_safe_entry_points():
    L = tbs.library()
    L.tbs_plan_destroy(None)
    assert L.tbs_solve(None, None, None, 4, None, None) == -1
    assert L.tbs_green_tabulate(None) == -1
    assert L.tbs_status_string(-3) == b"TBS_ERR_OOM"


def test_periodic_plan_rejections():
    """padding 1 makes a periodic plan: 2D only, power-of-two sizes 16..4096."""
    L = tbs.library()
    h = ctypes.c_void_p()
    k = tbs.c128(100.0, 0.0)
    for grid, nd in [((64, 64, 8), 3), ((48, 64, 1), 2), ((64, 8, 1), 2), ((8192, 64, 1), 2)]:
        g = (ctypes.c_int64 * 3)(*grid)
        assert L.tbs_plan_create(ctypes.byref(h), nd, g, 1e-3, k, 1, 0, 1, None) == -2, grid
        assert h.value is None


@pytest.mark.parametrize("n,dx,mu", [(1200, 20e-6, 450), (300, 1e-4, 40), (17, 1e-3, 0)])
def test_abl_profile_matches_oracle(n, dx, mu):
    got = tbs.abl_profile(n, dx, 21.48, mu)
    ref = oracle.abl_profile(n, dx, 21.48, mu)
    assert np.allclose(got, ref, rtol=1e-15, atol=0)
