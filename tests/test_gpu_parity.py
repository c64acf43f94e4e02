"""Parity of the HIP path with the FP64 oracle (GPU).

Every comparison is element by element on the same seeded inputs: relative L2
of the complex field per right-hand side, <= 1e-12 for the FP64 plan and
<= 1e-5 for the FP32 (Kahan) plan, the tolerances of the measurement plan.
"""
import math
import warnings

import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-12, "c64": 1e-5}


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def tdt(name):
    return torch.complex128 if name == "c128" else torch.complex64


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def per_rhs_rel(a, b):
    return max(rel(a[i], b[i]) for i in range(a.shape[0]))


def gpu_solve(dev, shape, dx, k0, s, V, L, dt, spectrum=None):
    import paper_2507_13754_amd as tbs
    s = np.asarray(s)
    if s.ndim == len(shape):
        s = s[None]
    plan = tbs.Plan(shape, dx, k0, dtype=tdt(dt), batch=s.shape[0])
    if spectrum is not None:
        plan.import_spectrum(spectrum)
    else:
        plan.tabulate()
    Vt = None if V is None else torch.from_numpy(np.ascontiguousarray(V)).to(dev, tdt(dt))
    p, res = plan.solve(torch.from_numpy(np.ascontiguousarray(s)).to(dev, tdt(dt)), Vt, L, residual=True)
    out = p.cpu().numpy().astype(np.complex128)
    plan.close()
    return out, res


def small_case(shape, seed, contrast=0.05):
    dx = 1.0
    k0 = 2 * np.pi / 6.0 * (1 + 0.01j)
    V = contrast * (k0 * k0).real * workloads.random_field(shape, seed)
    s = workloads.random_field((2,) + tuple(shape), seed + 1)
    return dx, k0, V, s


# ------------------------------------------------------------- spectrum ------

@pytest.mark.parametrize("shape", [(256, 256), (37, 23), (9, 10, 12)])
def test_green_spectrum_matches_oracle(dev, shape):
    import paper_2507_13754_amd as tbs
    case = workloads.plain2d(n=256)
    k0 = oracle.background_k0(case.omega, case.c0, case.alpha0, case.y)
    dx = case.dx
    plan = tbs.Plan(shape, dx, k0, dtype=torch.complex128).tabulate()
    Mx, My, Mz = plan.padded
    mshape = (Mz, My, Mx) if len(shape) == 3 else (My, Mx)
    full = oracle.green_spectrum(k0, dx, shape, mshape) / np.prod(mshape)
    if len(shape) == 2:
        ref = full[: My // 2 + 1, : Mx // 2 + 1].T
    else:
        ref = np.transpose(full[: Mz // 2 + 1, : My // 2 + 1, : Mx // 2 + 1], (2, 1, 0))
    got = plan.export_spectrum()
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
    plan.close()


# ---------------------------------------------------------- full config 1 ----

@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_plain2d_full_size(dev, dt):
    """256^2, 16 terms, GRF medium, 32-element line source."""
    import paper_2507_13754_amd as tbs
    case = workloads.plain2d()
    k0 = oracle.background_k0(case.omega, case.c0, case.alpha0, case.y)
    V = oracle.potential(case.c, case.omega, case.c0, case.alpha0, case.y)
    p_ref, r_ref = oracle.solve(k0, case.dx, case.sources, V, case.nterms)
    plan = tbs.Plan(case.grid, case.dx, tbs.background_k0(case.omega, case.c0, case.alpha0, case.y),
                    dtype=tdt(dt)).tabulate()
    Vg = plan.potential(torch.from_numpy(case.c).to(dev), case.omega, case.c0, case.alpha0, case.y)
    assert rel(Vg.cpu().numpy(), V) < (1e-13 if dt == "c128" else 1e-6)
    p, res = plan.solve(torch.from_numpy(case.sources).to(dev, tdt(dt)), Vg, case.nterms, residual=True)
    err = per_rhs_rel(p.cpu().numpy().astype(np.complex128), p_ref)
    assert err <= TOL[dt], err
    assert np.allclose(res, r_ref, rtol=1e-9 if dt == "c128" else 1e-3, atol=0)
    plan.close()


# ----------------------------------------------------------- ragged grids ----

@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("shape", [(37, 23), (5, 64), (64, 3), (1, 1), (130, 70), (17, 200)])
def test_ragged_2d(dev, shape, dt):
    dx, k0, V, s = small_case(shape, seed=sum(shape))
    L = 6
    p_ref, r_ref = oracle.solve(k0, dx, s, V, L)
    p, res = gpu_solve(dev, shape, dx, k0, s, V, L, dt)
    assert per_rhs_rel(p, p_ref) <= TOL[dt]
    assert np.allclose(res, r_ref, rtol=1e-9 if dt == "c128" else 1e-3)


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_long_slowly_converging_series(dev, dt):
    """150 terms of a series that contracts by about 0.87 per term: the
    compensated FP32 sum (compensation stored as bfloat16) and the FP64 sum
    against the oracle, and the series converged."""
    shape = (96, 96)
    dx, k0, V, s = small_case(shape, seed=7, contrast=0.2)
    s = s[:1]
    L = 150
    p_ref, r_ref = oracle.solve(k0, dx, s, V, L)
    assert r_ref[0, 60] < 1e-3 and r_ref[0, -1] < 1e-8
    p, res = gpu_solve(dev, shape, dx, k0, s, V, L, dt)
    assert per_rhs_rel(p, p_ref) <= TOL[dt]


def _bf16(x):
    """Round-to-nearest-even of float32 values to bfloat16 (as float32)."""
    b = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def test_compensated_sum_beats_plain_fp32(dev):
    """An 8000-term series whose terms stay near 1e-4 of the running sum (in
    norm): one potential cell V(x0) = v at a spot the first term barely
    reaches, so GV is rank one with eigenvalue v W(0) = 0.99995 e^{2i} and
    u_n = lambda^{n-1} u_1.  The spectrum is the oracle's rounded to FP32
    values (imported on both sides) and v an FP32 value, so device and oracle
    apply the same operator.  The device's sum of terms 1..L-1 (p_L - p_1 on
    the device) must match the oracle's to 5e-8 of |p|; the same FP32 terms
    summed without compensation (host emulation) miss it by more than 2e-7,
    with the compensation stored as bfloat16 (host emulation) by less than
    5e-8."""
    import paper_2507_13754_amd as tbs
    n, L = 48, 8000
    dx = 1.0
    k0 = 2 * np.pi / 8 + 0.15j
    G = oracle.GreenOperator(k0, dx, (n, n))
    M = G.mshape[0]
    q = (G.ghat / (M * M)).astype(np.complex64).astype(np.complex128)
    f = np.minimum(np.arange(M), M - np.arange(M))
    full = q[f][:, f] * (M * M)             # even, FP32-representable after / M^2
    G.ghat = full
    xs, x0 = (6, 6), (40, 40)
    d0 = np.zeros((n, n), complex)
    d0[x0] = 1.0
    W0 = G(d0)[x0]
    v = complex(np.complex64(0.99995 * np.exp(2.0j) / W0))
    V = np.zeros((n, n), complex)
    V[x0] = v
    s = np.zeros((1, n, n), complex)
    s[(0,) + xs] = 1.0
    terms = [G(s)[0]]
    for _ in range(L - 1):
        terms.append(G(V * terms[-1]))
    tail = np.sum(terms[1:], axis=0)        # sum of u_1 .. u_{L-1}, FP64
    assert 3e-5 < np.linalg.norm(terms[1]) / np.linalg.norm(terms[0]) < 3e-4
    p1, _ = gpu_solve(dev, (n, n), dx, k0, s, V, 1, "c64", spectrum=full)
    pL, _ = gpu_solve(dev, (n, n), dx, k0, s, V, L, "c64", spectrum=full)
    ref = p1[0] + tail
    dev_err = rel(pL[0], ref)
    # host emulation of the FP32 summation of the FP32-rounded terms
    plain = p1[0].astype(np.complex64)
    sr, si = plain.real.copy(), plain.imag.copy()
    cr, ci = np.zeros_like(sr), np.zeros_like(si)
    for t in terms[1:]:
        t32 = t.astype(np.complex64)
        plain = (plain + t32).astype(np.complex64)
        for sv, cv, xv in ((sr, cr, t32.real), (si, ci, t32.imag)):
            y = (xv - cv).astype(np.float32)
            tt = (sv + y).astype(np.float32)
            cv[:] = _bf16((tt - sv).astype(np.float32) - y)
            sv[:] = tt
    plain_err = rel(plain.astype(np.complex128), ref)
    kahan_err = rel((sr + 1j * si).astype(np.complex128), ref)
    print(f"compensated sum: device {dev_err:.2e}, host plain FP32 {plain_err:.2e}, "
          f"host bf16-compensated {kahan_err:.2e}", flush=True)
    bound = 5e-8
    assert kahan_err <= bound
    assert plain_err >= 4 * bound
    assert dev_err <= bound


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("shape", [(9, 10, 12), (16, 16, 16), (5, 3, 33)])
def test_ragged_3d(dev, shape, dt):
    dx, k0, V, s = small_case(shape, seed=sum(shape), contrast=0.03)
    L = 5
    p_ref, r_ref = oracle.solve(k0, dx, s, V, L)
    p, res = gpu_solve(dev, shape, dx, k0, s, V, L, dt)
    assert per_rhs_rel(p, p_ref) <= TOL[dt]


@pytest.mark.parametrize("L", [1, 2, 3])
def test_short_series(dev, L):
    dx, k0, V, s = small_case((20, 30), seed=5)
    p_ref, r_ref = oracle.solve(k0, dx, s, V, L)
    p, res = gpu_solve(dev, (20, 30), dx, k0, s, V, L, "c128")
    assert per_rhs_rel(p, p_ref) <= 1e-12
    assert np.allclose(res, r_ref, rtol=1e-10)


# -------------------------------------------------------------- properties --

@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_zero_potential_gives_first_term(dev, dt):
    dx, k0, V, s = small_case((24, 40), seed=7)
    p1, r1 = gpu_solve(dev, (24, 40), dx, k0, s, None, 1, dt)
    p5, r5 = gpu_solve(dev, (24, 40), dx, k0, s, None, 5, dt)
    assert np.array_equal(p1, p5)
    assert np.all(r5[:, 0] == 1.0) and np.all(r5[:, 1:] == 0.0)
    G = oracle.GreenOperator(k0, dx, (24, 40))
    assert per_rhs_rel(p1, G(s)) <= TOL[dt]


def test_batch_equals_single_bitwise(dev):
    dx, k0, V, s = small_case((33, 47), seed=11)
    s3 = np.concatenate([s, workloads.random_field((1, 33, 47), 99)])
    pb, rb = gpu_solve(dev, (33, 47), dx, k0, s3, V, 7, "c128")
    for b in range(3):
        p1, r1 = gpu_solve(dev, (33, 47), dx, k0, s3[b], V, 7, "c128")
        assert np.array_equal(pb[b], p1[0])
        assert np.array_equal(rb[b], r1[0])


def test_reciprocity(dev):
    """Field at B from a point source at A equals the field at A from B, for
    any V and L (W is even, so every truncated term operator is symmetric)."""
    shape = (48, 40)
    dx, k0, V, _ = small_case(shape, seed=13)
    a, b = (5, 7), (40, 31)
    s = np.zeros((2,) + shape, np.complex128)
    s[(0,) + a] = 1.0
    s[(1,) + b] = 1.0
    p, _ = gpu_solve(dev, shape, dx, k0, s, V, 9, "c128")
    assert abs(p[(0,) + b] - p[(1,) + a]) <= 1e-12 * abs(p[(0,) + b])


def test_injected_spectrum_isolates_fft_path(dev):
    """With the oracle's own spectrum injected, the remaining difference is the
    device FFT/passes alone."""
    import paper_2507_13754_amd as tbs
    shape = (50, 60)
    dx, k0, V, s = small_case(shape, seed=17)
    Mx = tbs.padded_length(60)
    My = tbs.padded_length(50)
    full = oracle.green_spectrum(k0, dx, shape, (My, Mx))
    p_ref, _ = oracle.solve(k0, dx, s, V, 6, mshape=(My, Mx))
    p, _ = gpu_solve(dev, shape, dx, k0, s, V, 6, "c128", spectrum=full)
    assert per_rhs_rel(p, p_ref) <= 1e-13


def test_deterministic(dev):
    dx, k0, V, s = small_case((64, 64), seed=19)
    p1, r1 = gpu_solve(dev, (64, 64), dx, k0, s, V, 8, "c64")
    p2, r2 = gpu_solve(dev, (64, 64), dx, k0, s, V, 8, "c64")
    assert np.array_equal(p1, p2) and np.array_equal(r1, r2)


# ---------------------------------------------------------- failure paths ---

def test_nonfinite_input_warns(dev):
    import paper_2507_13754_amd as tbs
    dx, k0, V, s = small_case((32, 32), seed=23)
    V = V.copy()
    V[10, 10] = np.nan
    with warnings.catch_warnings(record=True) as w:
        warnings.simplefilter("always")
        p, res = gpu_solve(dev, (32, 32), dx, k0, s, V, 4, "c128")
    assert any(issubclass(x.category, tbs.TBSWarning) and "NONFINITE" in str(x.message) for x in w)
    assert not np.all(np.isfinite(res))


def test_diverging_series_warns(dev):
    import paper_2507_13754_amd as tbs
    dx, k0, V, s = small_case((24, 24), seed=29)
    A = oracle.dense_operator(k0, dx, (24, 24))
    V = V * (1.5 / oracle.spectral_radius(A, V))
    with warnings.catch_warnings(record=True) as w:
        warnings.simplefilter("always")
        gpu_solve(dev, (24, 24), dx, k0, s, V, 40, "c128")
    assert any(issubclass(x.category, tbs.TBSWarning) and "DIVERGING" in str(x.message) for x in w)


@pytest.mark.parametrize("shape", [(2048, 300), (700, 1000)])
def test_autotuned_plan_is_bitwise_identical(dev, shape):
    """The autotuner only changes block shapes: the field is bitwise equal."""
    import paper_2507_13754_amd as tbs
    dx, k0, V, s = small_case(shape, seed=37)
    s = s[:1]
    L = 4
    base = tbs.Plan(shape, dx, k0, dtype=torch.complex64).tabulate()
    tuned = tbs.Plan(shape, dx, k0, dtype=torch.complex64).tabulate()
    nr, nc = tuned.autotune()
    assert nr in (2, 4) and nc in (1, 2, 4)
    sd = torch.from_numpy(s).to(dev, torch.complex64)
    Vd = torch.from_numpy(V).to(dev, torch.complex64)
    p0, r0 = base.solve(sd, Vd, L, residual=True)
    p1, r1 = tuned.solve(sd, Vd, L, residual=True)
    assert torch.equal(p0, p1)
    assert np.allclose(r0, r1, rtol=1e-13, atol=0)
    base.close()
    tuned.close()


@pytest.mark.parametrize("shape", [(70, 50, 60), (130, 40, 34)])
def test_autotuned_3d_plan_is_bitwise_identical(dev, shape):
    """3D plans tune the z lines per block of the z convolution; the field is
    bitwise equal to the default shape's and the choice is reported."""
    import paper_2507_13754_amd as tbs
    dx, k0, V, s = small_case(shape, seed=41)
    s = s[:1]
    L = 4
    base = tbs.Plan(shape, dx, k0, dtype=torch.complex64).tabulate()
    tuned = tbs.Plan(shape, dx, k0, dtype=torch.complex64).tabulate()
    _, nc = tuned.autotune()
    assert nc in (1, 2, 4)
    sd = torch.from_numpy(s).to(dev, torch.complex64)
    Vd = torch.from_numpy(V).to(dev, torch.complex64)
    p0, r0 = base.solve(sd, Vd, L, residual=True)
    p1, r1 = tuned.solve(sd, Vd, L, residual=True)
    assert torch.equal(p0, p1)
    assert np.allclose(r0, r1, rtol=1e-13, atol=0)
    base.close()
    tuned.close()
