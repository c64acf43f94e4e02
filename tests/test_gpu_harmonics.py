"""Chained higher harmonics (fundamental, then harmonics 2..5 one by one, each
driven by the sum-frequency source of the lower ones) against the oracle
chain, FP64 <= 1e-12 and FP32 <= 1e-5 relative L2."""
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


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("shape", [(44, 38), (9, 12, 10)])
def test_harmonics_up_to_fifth(dev, dt, shape, errlog):
    import paper_2507_13754_amd as tbs
    f0 = 1e6
    om = 2 * np.pi * f0
    nh = 5
    dx = workloads.C0 / (nh * f0) / 6
    c = workloads.small_medium(shape, dx, 0.02, seed=61)
    a0, y = workloads.alpha0_si(0.75, 1.5), 1.5
    rho, BA = workloads.RHO0, 5.0
    s = np.zeros((1,) + shape, np.complex128)
    s[(0,) + tuple(n // 3 for n in shape)] = 1e6 / dx ** 2    # p1 ~ 1e5 Pa (far from FP32 limits)
    L = 5
    # oracle chain
    ref = []
    for n in range(1, nh + 1):
        kn = oracle.background_k0(n * om, workloads.C0, a0, y)
        Vn = oracle.potential(c, n * om, workloads.C0, a0, y)
        src = s if n == 1 else oracle.harmonic_source_n(ref, n, c, om, rho, BA)
        ref.append(oracle.solve(kn, dx, src, Vn, L)[0])
    # device chain
    cd = torch.from_numpy(c).to(dev)
    got = []
    for n in range(1, nh + 1):
        plan = tbs.Plan(shape, dx, tbs.background_k0(n * om, workloads.C0, a0, y), dtype=tdt(dt)).tabulate()
        if n == 1:
            src = torch.from_numpy(s).to(dev, tdt(dt))
        else:
            src = plan.harmonic_source_n(n, got, cd, om, rho, BA)
            S_dev = oracle.harmonic_source_n([g.cpu().numpy().astype(np.complex128) for g in got],
                                             n, c, om, rho, BA)
            # the source kernel itself, on the device's own lower harmonics
            assert rel(src.cpu().numpy(), S_dev) <= (1e-14 if dt == "c128" else 1e-6)
        got.append(plan.solve(src, plan.potential(cd, n * om, workloads.C0, a0, y), L))
        plan.close()
        assert errlog(f"psi_{n}", rel(got[-1].cpu().numpy(), ref[n - 1]), TOL[dt]) <= TOL[dt], n
    assert all(np.linalg.norm(r) > 0 for r in ref)


def test_harmonic_source_n_two_equals_second_harmonic(dev):
    import paper_2507_13754_amd as tbs
    shape = (16, 20)
    p1 = torch.from_numpy(workloads.random_field((2,) + shape, 81)).to(dev)
    c = torch.from_numpy(1540.0 * (1 + 0.02 * workloads.random_field(shape, 82).real)).to(dev)
    plan = tbs.Plan(shape, 1e-4, 1.0 + 0.1j, dtype=torch.complex128, batch=2)
    a = plan.harmonic_source(p1, c, 1e6, 1000.0, 7.0)
    b = plan.harmonic_source_n(2, [p1], c, 1e6, 1000.0, 7.0)
    assert torch.allclose(a, b, rtol=1e-15, atol=0)
    plan.close()


def _paper_chain(dev, n, dtype, scaled, counts=None):
    """Fundamental and harmonics 2..5 of the paper's homogeneous setup scaled
    to n^2 (Sec. 3.1; B/A = 5, rho = 1000), each iterated to the paper's
    tolerance, or for the given iteration counts (tol 0).  scaled: the
    sources of the harmonics come from tbs_harmonic_source_scaled, and field
    h holds psi_h 2^exps[h-1]."""
    import paper_2507_13754_amd as tbs
    case = workloads.paper_periodic("homogeneous", n)
    c_map = torch.from_numpy(case.c).to(dev)
    prof = torch.from_numpy(tbs.abl_profile(n, case.dx, case.zeta, case.mu_cells)).to(dev)
    fields, exps, its = [], [], []
    for h in range(1, 6):
        k = h * case.omega / case.c0
        eps = case.eps_factor * k * k
        plan = tbs.Plan((n, n), case.dx, k, padding=1, dtype=dtype)
        plan.green_periodic(eps)
        V = plan.potential(c_map, h * case.omega, case.c0, 0.0, 1.0, eps)
        if h == 1:
            src, e = torch.from_numpy(case.sources).to(dev, dtype), 0
        elif scaled:
            src, e = plan.harmonic_source_scaled(h, fields, exps, c_map, case.omega, 1000.0, 5.0)
        else:
            src, e = plan.harmonic_source_n(h, fields, c_map, case.omega, 1000.0, 5.0), 0
        tol, mi = (case.tol, case.max_iter) if counts is None else (0.0, counts[h - 1])
        psi, it, _ = plan.iterate(src, V, prof, prof, case.check_row, tol, mi)
        plan.close()
        fields.append(psi)
        exps.append(e)
        its.append(it)
    return fields, exps, its


@pytest.mark.filterwarnings("ignore:tbs_iterate")
def test_fp32_paper_chain_to_fifth_harmonic(dev, errlog):
    """The nonlinear chain of Table 3 on the 256^2 scaled setup, where the 4th
    and 5th harmonics (about 1e-35 and 1e-46) lie below or at the edge of the
    FP32 range: with power-of-two scaled sources the FP32 chain stops within
    one iteration of the FP64 one at every order, and, run for the FP64
    counts, matches the FP64 fields to 1e-5 (relative L2)."""
    n = 256
    f64, e64, it64 = _paper_chain(dev, n, torch.complex128, scaled=False)
    assert all(it < 2000 for it in it64)
    # the scaled FP64 chain is the unscaled one times 2^e (exact up to rounding)
    g64, ge64, git64 = _paper_chain(dev, n, torch.complex128, scaled=True)
    assert git64 == it64
    for h in range(5):
        a = g64[h].cpu().numpy() * 2.0 ** (-ge64[h])
        assert rel(a, f64[h].cpu().numpy()) <= 1e-12, h
    # the paper's stopping rule in FP32
    _, _, it32 = _paper_chain(dev, n, torch.complex64, scaled=True)
    assert all(abs(a - b) <= 1 for a, b in zip(it32, it64)), (it32, it64)
    # FP32 fields at the FP64 counts
    f32, e32, _ = _paper_chain(dev, n, torch.complex64, scaled=True, counts=it64)
    assert min(e32[1:]) > 20   # the harmonics were scaled up
    for h in range(5):
        a = f32[h].cpu().numpy().astype(np.complex128) * 2.0 ** (-e32[h])
        assert errlog(f"psi_{h + 1}", rel(a, f64[h].cpu().numpy()), 1e-5) <= 1e-5, h


def test_fp64_paper_chain_matches_oracle(dev):
    """The same chain (64^2 scaled setup) against the oracle's iteration of
    Algorithm 1 with the oracle's sum-frequency sources."""
    n = 64
    case = workloads.paper_periodic("homogeneous", n)
    mask = oracle.abl_mask((n, n), case.dx, case.zeta, case.mu_cells)
    ref = []
    its = []
    for h in range(1, 6):
        k = h * case.omega / case.c0
        eps = case.eps_factor * k * k
        g = oracle.periodic_green_spectrum(k, eps, case.dx, (n, n))
        V = oracle.potential(case.c, h * case.omega, case.c0, 0.0, 1.0, eps)
        src = case.sources[0] if h == 1 else \
            oracle.harmonic_source_n([f[None] for f in ref], h, case.c, case.omega, 1000.0, 5.0)[0]
        psi, it, _ = oracle.paper_iterate(g, src, V, mask=mask, check_row=case.check_row, tol=case.tol,
                                          max_iter=case.max_iter)
        ref.append(psi)
        its.append(it)
    got, exps, git = _paper_chain(dev, n, torch.complex128, scaled=True)
    assert git == its
    for h in range(5):
        a = got[h].cpu().numpy()[0] * 2.0 ** (-exps[h])
        assert rel(a, ref[h]) <= 1e-11, h
