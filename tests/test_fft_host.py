"""CPU checks of the device FFT building blocks compiled as host code: the
radix-2/3/4/5/8/16 butterflies and the radix plans of every compiled length."""
import ctypes
import os

import numpy as np
import pytest

HC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                  "paper_2507_13754_amd", "_build", "libtbs_hostcheck.so")


@pytest.fixture(scope="module")
def hc():
    if not os.path.exists(HC):
        pytest.fail(f"{HC} missing: run __graft_entry__.build()")
    return ctypes.CDLL(HC)


@pytest.mark.parametrize("R", [2, 3, 4, 5, 8, 16])
@pytest.mark.parametrize("inv", [0, 1])
def test_radix_butterfly(hc, R, inv):
    rng = np.random.default_rng(R + 10 * inv)
    for _ in range(5):
        x = rng.standard_normal(R) + 1j * rng.standard_normal(R)
        inp = np.ascontiguousarray(np.stack([x.real, x.imag], 1).ravel())
        out = np.zeros(2 * R)
        assert hc.tbs_hostcheck_dft(R, inv, inp.ctypes.data_as(ctypes.c_void_p),
                                    out.ctypes.data_as(ctypes.c_void_p)) == 0
        y = out[0::2] + 1j * out[1::2]
        ref = np.fft.ifft(x) * R if inv else np.fft.fft(x)
        assert np.max(np.abs(y - ref)) < 1e-14 * np.max(np.abs(ref)) * R


@pytest.mark.parametrize("M,E", [(16, 4), (32, 4), (64, 4), (128, 8), (256, 8), (512, 8),
                                 (1024, 16), (2048, 16), (4096, 16), (2500, 20), (1000, 40)])
def test_stage_plan(hc, M, E):
    r = (ctypes.c_int * 12)()
    n = hc.tbs_hostcheck_stages(M, E, r)
    radices = [r[i] for i in range(n)]
    assert n > 0 and int(np.prod(radices)) == M
    assert all(E % x == 0 for x in radices)


@pytest.mark.parametrize("M,E", [(16, 4), (48, 12), (96, 12), (160, 20), (320, 20), (640, 40), (768, 24),
                                 (1280, 40), (1536, 24), (2048, 16), (2560, 40), (2560, 20), (3072, 24),
                                 (4096, 16)])
@pytest.mark.parametrize("inv", [0, 1])
def test_stage_data_flow_is_a_dft(hc, M, E, inv):
    """The device transform's hand-over between stages (shared-array exchange
    or in-thread register renaming), emulated on the host, gives the DFT."""
    rng = np.random.default_rng(M + E + inv)
    x = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    inp = np.ascontiguousarray(np.stack([x.real, x.imag], 1).ravel())
    out = np.zeros(2 * M)
    nex, nloc = ctypes.c_int(), ctypes.c_int()
    assert hc.tbs_hostcheck_fft(M, E, inv, inp.ctypes.data_as(ctypes.c_void_p),
                                out.ctypes.data_as(ctypes.c_void_p), ctypes.byref(nex), ctypes.byref(nloc)) == 0
    y = out[0::2] + 1j * out[1::2]
    ref = np.fft.ifft(x) * M if inv else np.fft.fft(x)
    assert np.max(np.abs(y - ref)) < 1e-13 * np.max(np.abs(ref))
    # every stage but the last hands over once; lines with 4+ stages keep the
    # hand-overs after L reaches M/E inside the thread
    r = (ctypes.c_int * 12)()
    n = hc.tbs_hostcheck_stages(M, E, r)
    assert nex.value + nloc.value == n - 1
    if n >= 4:
        assert nloc.value >= 1


@pytest.mark.parametrize("M,E", [(16, 4), (64, 4), (512, 8), (1024, 16), (2048, 16), (4096, 16), (48, 12),
                                 (96, 12), (1536, 12), (3072, 12), (80, 20), (640, 20), (1280, 20),
                                 (2560, 20), (2560, 40), (1536, 24)])
def test_lds_slot_closed_forms(hc, M, E):
    """The LDS slots the device code computes as base + constant offsets equal
    the padded exchange indices they stand for."""
    assert hc.tbs_hostcheck_slots(M, E) == 0


@pytest.mark.parametrize("M,E", [(16, 4), (64, 4), (512, 8), (1024, 16), (2048, 16), (4096, 16), (48, 12),
                                 (96, 12), (768, 12), (1536, 12), (3072, 12), (80, 20), (640, 20),
                                 (1280, 20), (2560, 20), (2560, 40), (1536, 24)])
def test_resident_twiddle_slots(hc, M, E):
    """A pass that keeps its twiddle factors in registers reads, for every
    thread, stage, butterfly and input, the factor the table holds for that
    butterfly: the period of k over the butterflies of a thread is right."""
    assert hc.tbs_hostcheck_twcache(M, E) == 0
