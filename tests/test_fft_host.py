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


@pytest.mark.parametrize("R", [2, 4, 8, 16])
@pytest.mark.parametrize("inv", [0, 1])
def test_first_stage_of_zero_padded_line(hc, R, inv):
    """The pruned first-stage butterflies (inputs R/2.. zero) equal the DFT of
    the zero-padded input; a dropped term or a wrong rotation fails."""
    rng = np.random.default_rng(100 + R + inv)
    for _ in range(5):
        x = rng.standard_normal(R // 2) + 1j * rng.standard_normal(R // 2)
        inp = np.empty(R)
        inp[0::2], inp[1::2] = x.real, x.imag
        out = np.zeros(2 * R)
        assert hc.tbs_hostcheck_dft_half(R, inv, inp.ctypes.data_as(ctypes.c_void_p),
                                         out.ctypes.data_as(ctypes.c_void_p)) == 0
        y = out[0::2] + 1j * out[1::2]
        xp = np.concatenate([x, np.zeros(R // 2)])
        ref = np.fft.ifft(xp) * R if inv else np.fft.fft(xp)
        assert np.max(np.abs(y - ref)) < 1e-14 * max(1.0, np.max(np.abs(ref)))


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


LDS_CASES = [(M, E) for M, E in [(16, 4), (32, 4), (64, 4), (128, 8), (256, 8), (512, 8), (1024, 16),
                                  (2048, 16), (4096, 16), (48, 12), (96, 12), (192, 12), (384, 12), (768, 12),
                                  (1536, 12), (3072, 12), (80, 20), (160, 20), (320, 20), (640, 20),
                                  (1280, 20), (2560, 20), (2560, 40), (1536, 24)]]


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("NL", [1, 2, 4])
@pytest.mark.parametrize("esz", [4, 8, 16])
@pytest.mark.parametrize("M,E", LDS_CASES)
def test_lds_exchange_layout(hc, M, E, esz, NL, kind):
    """The LDS exchange layouts of a pass block of NL lines whose lanes take
    the lines as the column pass (kind 0) or the row pass (kind 1) does, for
    4-byte split halves, FP32 and FP64 complex values: the slots the device
    computes are the layout of the indices they stand for, one element per
    slot, every read finds its element; under the 32-bank model a block of
    one line of 128+ values waits on no bank conflict, where the padded
    layout conflicts on the radix-4 stages of 3*2^a and 5*2^a lines."""
    if kind == 1 and (M // E) % 4:
        pytest.skip("row passes need 4-value column blocks")
    pad, new = ctypes.c_int(), ctypes.c_int()
    assert hc.tbs_hostcheck_xslots(M, E, esz, NL, kind, ctypes.byref(pad), ctypes.byref(new)) == 0
    if NL == 1:
        assert new.value <= pad.value
        if M >= 128:
            assert new.value == 0
        if esz == 8 and (M, E) in ((768, 12), (1536, 12), (640, 20), (1280, 20), (2560, 20)):
            assert pad.value > 0


@pytest.mark.parametrize("M,E", [(16, 4), (64, 4), (512, 8), (1024, 16), (2048, 16), (4096, 16), (48, 12),
                                 (96, 12), (768, 12), (1536, 12), (3072, 12), (80, 20), (640, 20),
                                 (1280, 20), (2560, 20), (2560, 40), (1536, 24)])
def test_resident_twiddle_slots(hc, M, E):
    """A pass that keeps its twiddle factors in registers reads, for every
    thread, stage, butterfly and input, the factor the table holds for that
    butterfly: the period of k over the butterflies of a thread is right."""
    assert hc.tbs_hostcheck_twcache(M, E) == 0


def _bf16_rne(x):
    """Round-to-nearest-even of float32 values to their upper 16 bits."""
    b = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    return ((b + 0x7FFF + lsb) >> 16).astype(np.uint32)


def test_bf16_compensation_storage(hc):
    """The compensation word rounds to nearest, ties to even, keeps sign,
    zero, infinity and NaN, and reads back the rounded value."""
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.standard_normal(4000).astype(np.float32) * 10.0 ** rng.integers(-30, 30, 4000),
                        np.array([0.0, -0.0, np.inf, -np.inf, 1.0, 1.00390625, 1.01171875, 3e-39],
                                 np.float32)]).astype(np.float32)
    n = x.size
    out = np.zeros(n, np.uint32)
    back = np.zeros(n, np.float32)
    hc.tbs_hostcheck_bf16(x.ctypes.data_as(ctypes.c_void_p), ctypes.c_int(n),
                          out.ctypes.data_as(ctypes.c_void_p), back.ctypes.data_as(ctypes.c_void_p))
    assert np.array_equal(out, _bf16_rne(x))
    assert np.array_equal(back.view(np.uint32), out << 16)
    # ties: 1 + 2^-8 rounds down to 1 (even), 1 + 3 * 2^-8 rounds up
    assert back[n - 3] == np.float32(1.0) and back[n - 2] == np.float32(1.015625)
    rel = np.abs(back[:4000] - x[:4000]) / np.abs(x[:4000])
    assert rel.max() <= 2.0 ** -8
    nan = np.array([np.nan], np.float32)
    hc.tbs_hostcheck_bf16(nan.ctypes.data_as(ctypes.c_void_p), ctypes.c_int(1),
                          out.ctypes.data_as(ctypes.c_void_p), back.ctypes.data_as(ctypes.c_void_p))
    assert np.isnan(back[0])


def test_kahan_with_bf16_compensation_keeps_its_accuracy(hc):
    """The row pass's FP32 accumulation step with the compensation stored in
    bfloat16, emulated on the host with the device's rounding: a slowly
    decaying 200-term series sums as accurately as with an FP32 compensation
    and an order of magnitude better than plain FP32 addition."""
    rng = np.random.default_rng(11)
    n, L, rho = 20000, 200, 0.97
    base = rng.standard_normal(n).astype(np.float32)
    terms = [((rng.standard_normal(n) + base) * rho ** k).astype(np.float32) for k in range(L)]
    exact = np.sum(np.array(terms, np.float64), axis=0)

    def store(c):
        out = np.zeros(n, np.uint32)
        back = np.zeros(n, np.float32)
        c = np.ascontiguousarray(c, np.float32)
        hc.tbs_hostcheck_bf16(c.ctypes.data_as(ctypes.c_void_p), ctypes.c_int(n),
                              out.ctypes.data_as(ctypes.c_void_p), back.ctypes.data_as(ctypes.c_void_p))
        return back

    def kahan(q):
        s = np.zeros(n, np.float32)
        c = np.zeros(n, np.float32)
        for t in terms:
            y = (t - c).astype(np.float32)
            tt = (s + y).astype(np.float32)
            c = q(((tt - s).astype(np.float32) - y).astype(np.float32))
            s = tt
        return s

    plain = np.zeros(n, np.float32)
    for t in terms:
        plain = (plain + t).astype(np.float32)

    def err(v):
        return np.linalg.norm(v - exact) / np.linalg.norm(exact)

    e_plain, e32, e16 = err(plain), err(kahan(lambda c: c)), err(kahan(store))
    assert e16 <= 1.05 * e32 + 1e-9
    assert e16 * 8 < e_plain
