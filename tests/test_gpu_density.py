"""The density-contrast term (div(gamma grad psi), conservative differences)
in the GPU series against the oracle's series with the same term."""
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


def blob(shape, amp, centre, r2):
    """amp exp(-|i - centre|^2 / r2) on a 2D or 3D grid of cells."""
    idx = np.indices(shape)
    d2 = sum((idx[a] - centre[a]) ** 2 for a in range(len(shape)))
    return amp * np.exp(-d2 / r2)


def case(shape, seed):
    dx = 1.0
    k0 = 2 * np.pi / 6.0 * (1 + 0.01j)
    V = 0.04 * (k0 * k0).real * workloads.random_field(shape, seed)
    centre = [n / 2 for n in shape[:-1]] + [shape[-1] / 3]
    gam = blob(shape, 0.08, centre, shape[0])
    s = workloads.random_field((2,) + tuple(shape), seed + 1)
    return dx, k0, V, gam, s


def gpu(dev, shape, dx, k0, s, V, gam, L, dt):
    import paper_2507_13754_amd as tbs
    plan = tbs.Plan(shape, dx, k0, dtype=tdt(dt), batch=s.shape[0]).tabulate()
    if gam is not None:
        plan.density_contrast(torch.from_numpy(gam).to(dev))
    Vt = None if V is None else torch.from_numpy(V).to(dev, tdt(dt))
    p, r = plan.solve(torch.from_numpy(s).to(dev, tdt(dt)), Vt, L, residual=True)
    out = p.cpu().numpy().astype(np.complex128)
    plan.close()
    return out, r


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("shape", [(37, 23), (64, 96), (130, 70), (9, 10, 12), (12, 7, 16), (5, 3, 20)])
def test_density_series_matches_oracle(dev, shape, dt):
    dx, k0, V, gam, s = case(shape, sum(shape))
    L = 7
    p_ref, r_ref = oracle.solve_density(k0, dx, s, V, gam, L)
    p, r = gpu(dev, shape, dx, k0, s, V, gam, L, dt)
    assert max(rel(p[b], p_ref[b]) for b in range(2)) <= TOL[dt]
    assert np.allclose(r, r_ref, rtol=1e-9 if dt == "c128" else 1e-3, atol=0)


def test_density_only_no_potential(dev):
    """V = NULL with a density contrast: the terms are G(-div(gamma grad u))."""
    shape = (48, 40)
    dx, k0, V, gam, s = case(shape, 5)
    p_ref, _ = oracle.solve_density(k0, dx, s, np.zeros(shape), gam, 6)
    p, _ = gpu(dev, shape, dx, k0, s, None, gam, 6, "c128")
    assert max(rel(p[b], p_ref[b]) for b in range(2)) <= 1e-12


def test_zero_density_is_the_plain_series(dev):
    """gamma = 0 reproduces the plain series to rounding (the product V u is
    formed in another pass, so the compiler may fuse it differently)."""
    shape = (50, 44)
    dx, k0, V, _, s = case(shape, 9)
    a, ra = gpu(dev, shape, dx, k0, s, V, np.zeros(shape), 6, "c128")
    b, rb = gpu(dev, shape, dx, k0, s, V, None, 6, "c128")
    assert max(rel(a[i], b[i]) for i in range(2)) <= 1e-14


def test_density_512_fp32(dev):
    """A 512^2 absorbing medium with a 10 % density blob, 20 terms, FP32."""
    import paper_2507_13754_amd as tbs
    c = workloads.plain2d(n=512, nterms=20)
    k0 = oracle.background_k0(c.omega, c.c0, c.alpha0, c.y)
    V = oracle.potential(c.c, c.omega, c.c0, c.alpha0, c.y)
    gam = blob((512, 512), 0.1, (300, 256), 400.0)
    p_ref, _ = oracle.solve_density(k0, c.dx, c.sources, V, gam, c.nterms)
    plan = tbs.Plan(c.grid, c.dx, tbs.background_k0(c.omega, c.c0, c.alpha0, c.y),
                    dtype=torch.complex64).tabulate()
    plan.density_contrast(torch.from_numpy(gam).to(dev))
    Vg = plan.potential(torch.from_numpy(c.c).to(dev), c.omega, c.c0, c.alpha0, c.y)
    p = plan.solve(torch.from_numpy(c.sources).to(dev, torch.complex64), Vg, c.nterms)
    assert rel(p.cpu().numpy().astype(np.complex128)[0], p_ref[0]) <= 1e-5
    plan.close()


def test_density_3d_fp32_medium(dev):
    """A 64^3 grid at 6 points per wavelength with a 5 % density blob and a
    2 % speed medium, 12 terms, FP32 against the oracle."""
    import paper_2507_13754_amd as tbs
    n = 64
    f = 3e6
    dx = workloads.C0 / f / 6
    om = 2 * np.pi * f
    a0, y = workloads.alpha0_si(0.75, 1.5), 1.5
    c = workloads.small_medium((n, n, n), dx, 0.02, seed=71)
    gam = blob((n, n, n), 0.05, (n / 2, n / 2, n / 3), 60.0)
    s = np.zeros((1, n, n, n), np.complex128)
    s[0, 8, n // 2, 20:44:3] = 1.0 / dx ** 3
    k0 = oracle.background_k0(om, workloads.C0, a0, y)
    V = oracle.potential(c, om, workloads.C0, a0, y)
    p_ref, _ = oracle.solve_density(k0, dx, s, V, gam, 12)
    plan = tbs.Plan((n, n, n), dx, tbs.background_k0(om, workloads.C0, a0, y), dtype=torch.complex64).tabulate()
    plan.density_contrast(torch.from_numpy(gam).to(dev))
    Vg = plan.potential(torch.from_numpy(c).to(dev), om, workloads.C0, a0, y)
    p = plan.solve(torch.from_numpy(s).to(dev, torch.complex64), Vg, 12)
    assert rel(p.cpu().numpy().astype(np.complex128)[0], p_ref[0]) <= 1e-5
    plan.close()


def test_density_refusals(dev):
    import paper_2507_13754_amd as tbs
    plan = tbs.Plan((16, 16), 1.0, 1.0 + 0.1j, padding=1, dtype=torch.complex64)
    with pytest.raises(tbs.TBSError) as e:
        plan.density_contrast(torch.zeros((16, 16), dtype=torch.float64, device=dev))
    assert e.value.status == -2
    plan.close()
    shape = (20, 24)
    plan = tbs.Plan(shape, 1.0, 1.0 + 0.1j, dtype=torch.complex64).tabulate()
    plan.density_contrast(torch.zeros(shape, dtype=torch.float64, device=dev))
    z = torch.zeros((1,) + shape, dtype=torch.complex64, device=dev)
    with pytest.raises(tbs.TBSError) as e:
        plan.adjoint(z, z[0], 3, z)
    assert e.value.status == -2
    plan.close()
