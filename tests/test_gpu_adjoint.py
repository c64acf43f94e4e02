"""GPU adjoint, misfit gradient and second-harmonic chain against the oracle
(FP64 <= 1e-12, FP32 <= 1e-5 relative L2; FD agreement <= 1e-4)."""
import math

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


def to_dev(a, dev, dt):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev, tdt(dt))


@pytest.mark.parametrize("flags", [0, 1], ids=["store", "recompute"])
@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("shape,L", [((21, 34), 6), ((40, 40), 1), ((40, 40), 2), ((6, 7, 9), 4),
                                     ((16, 20), 25), ((18, 12), 13)])
def test_adjoint_series_matches_oracle(dev, dt, shape, L, flags, errlog):
    """Both adjoint modes: all partial sums stored, or sqrt(2L)-spaced
    checkpoints with segment recomputation (L = 13, 25: several segments)."""
    import paper_2507_13754_amd as tbs
    dx = 1.0
    k0 = 2 * np.pi / 6 * (1 + 0.02j)
    V = 0.05 * (k0 * k0).real * workloads.random_field(shape, 3)
    s = workloads.random_field((2,) + shape, 4)
    q = workloads.random_field((2,) + shape, 5)
    G = oracle.GreenOperator(k0, dx, shape)
    ref = np.stack([oracle.adjoint_series_gradient(G, s[b], V, L, q[b]) for b in range(2)])
    plan = tbs.Plan(shape, dx, k0, dtype=tdt(dt), batch=2).tabulate()
    g = plan.adjoint(to_dev(s, dev, dt), to_dev(V, dev, dt), L, to_dev(q, dev, dt), flags=flags)
    g = g.cpu().numpy().astype(np.complex128)
    if L == 1:
        assert np.all(g == 0)
    else:
        tol = TOL[dt]
        assert errlog("gradient", max(rel(g[b], ref[b]) for b in range(2)), tol) <= tol
    plan.close()


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_adjoint_store_reuses_one_plan_for_growing_L(dev, dt):
    """One plan, stored partial sums, L = 4, then 5 (the slot buffer must grow
    by the running-sum slot too), then 3: each against the oracle."""
    import paper_2507_13754_amd as tbs
    shape = (20, 18)
    k0 = 2 * np.pi / 6 * (1 + 0.02j)
    V = 0.05 * (k0 * k0).real * workloads.random_field(shape, 11)
    s = workloads.random_field((2,) + shape, 12)
    q = workloads.random_field((2,) + shape, 13)
    G = oracle.GreenOperator(k0, 1.0, shape)
    plan = tbs.Plan(shape, 1.0, k0, dtype=tdt(dt), batch=2).tabulate()
    for L in (4, 5, 3):
        ref = np.stack([oracle.adjoint_series_gradient(G, s[b], V, L, q[b]) for b in range(2)])
        g = plan.adjoint(to_dev(s, dev, dt), to_dev(V, dev, dt), L, to_dev(q, dev, dt), flags=0)
        g = g.cpu().numpy().astype(np.complex128)
        assert max(rel(g[b], ref[b]) for b in range(2)) <= TOL[dt], L
    plan.close()


def test_adjoint_dot_product_fd_fp64(dev):
    """Re sum dV g_V equals the central difference of Re<q, p_L(V + h dV)>,
    both from the GPU FP64 path."""
    import paper_2507_13754_amd as tbs
    shape = (30, 26)
    k0 = 2 * np.pi / 6 * (1 + 0.02j)
    V = 0.05 * (k0 * k0).real * workloads.random_field(shape, 7)
    dV = workloads.random_field(shape, 8)
    s = workloads.random_field((1,) + shape, 9)
    q = workloads.random_field((1,) + shape, 10)
    L = 7
    plan = tbs.Plan(shape, 1.0, k0, dtype=torch.complex128).tabulate()
    g = plan.adjoint(to_dev(s, dev, "c128"), to_dev(V, dev, "c128"), L, to_dev(q, dev, "c128"))
    lin = np.sum(dV * g.cpu().numpy()[0]).real
    h = 1e-6
    fp = np.vdot(q, plan.solve(to_dev(s, dev, "c128"), to_dev(V + h * dV, dev, "c128"), L).cpu().numpy()).real
    fm = np.vdot(q, plan.solve(to_dev(s, dev, "c128"), to_dev(V - h * dV, dev, "c128"), L).cpu().numpy()).real
    assert abs((fp - fm) / (2 * h) - lin) <= 1e-7 * abs(lin)
    plan.close()


def _misfit_setup(dev, dt, n=48, nfreq=2, nsrc=3, nrec=12, nterms=6):
    from paper_2507_13754_amd.autograd import MisfitProblem
    prob = workloads.adjoint2d(n=n, nfreq=nfreq, nsrc=nsrc, nrec=nrec, nterms=nterms)
    rec = prob.receivers
    flat = rec[:, 0] * n + rec[:, 1]
    p_obs = []
    for f in prob.freqs:
        om = 2 * np.pi * f
        k0 = oracle.background_k0(om, workloads.C0, prob.alpha0, prob.y)
        V = oracle.potential(prob.c_true, om, workloads.C0, prob.alpha0, prob.y)
        p, _ = oracle.solve(k0, prob.dx, prob.sources, V, prob.nterms)
        p_obs.append(p[(slice(None),) + tuple(rec.T)])
    mp = MisfitProblem((n, n), prob.dx, prob.freqs, workloads.C0, prob.alpha0, prob.y,
                       to_dev(prob.sources, dev, dt), torch.from_numpy(flat).to(dev),
                       [to_dev(p, dev, dt) for p in p_obs], prob.nterms, dtype=tdt(dt))
    return prob, rec, p_obs, mp


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_misfit_gradient_matches_oracle(dev, dt, errlog):
    from paper_2507_13754_amd.autograd import TBSMisfit
    prob, rec, p_obs, mp = _misfit_setup(dev, dt)
    J_ref, g_ref = oracle.misfit_gradient(prob.c_model, prob.freqs, prob.dx, workloads.C0, prob.alpha0,
                                          prob.y, prob.sources, rec, p_obs, prob.nterms)
    c = torch.from_numpy(prob.c_model).to(dev).requires_grad_(True)
    J = TBSMisfit.apply(c, mp)
    J.backward()
    tj, tg = (1e-11, 1e-10) if dt == "c128" else (1e-5, 1e-5)
    assert errlog("J", abs(J.item() - J_ref) / J_ref, tj) <= tj
    assert errlog("grad", rel(c.grad.cpu().numpy(), g_ref), tg) <= tg
    mp.close()


def test_misfit_gradient_finite_differences(dev):
    """Autograd gradient (FP32 adjoint) against central FD of the FP64 GPU
    misfit at sampled pixels, h = 1e-6 c0: agreement <= 1e-4 of max |grad|."""
    from paper_2507_13754_amd.autograd import TBSMisfit
    prob, rec, p_obs, mp32 = _misfit_setup(dev, "c64")
    _, _, _, mp64 = _misfit_setup(dev, "c128")
    c = torch.from_numpy(prob.c_model).to(dev).requires_grad_(True)
    TBSMisfit.apply(c, mp32).backward()
    g = c.grad.cpu().numpy()
    h = 1e-6 * workloads.C0
    rng = np.random.default_rng(55)
    pix = [(int(a), int(b)) for a, b in zip(rng.integers(10, 38, 8), rng.integers(10, 38, 8))]
    for (iy, ix) in pix:
        cp = prob.c_model.copy(); cp[iy, ix] += h
        cm = prob.c_model.copy(); cm[iy, ix] -= h
        with torch.no_grad():
            Jp = TBSMisfit.apply(torch.from_numpy(cp).to(dev), mp64).item()
            Jm = TBSMisfit.apply(torch.from_numpy(cm).to(dev), mp64).item()
        fd = (Jp - Jm) / (2 * h)
        assert abs(fd - g[iy, ix]) <= 1e-4 * np.max(np.abs(g)), (iy, ix, fd, g[iy, ix])
    mp32.close()
    mp64.close()


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_misfit_sums_receivers_sharing_a_cell(dev, dt):
    """q = R^H (R p - p_obs) adds the residuals of receivers on one cell."""
    import paper_2507_13754_amd as tbs
    shape = (16, 20)
    p = workloads.random_field((2,) + shape, 41)
    rec = np.array([[3, 4], [3, 4], [10, 7], [3, 4], [15, 19]], dtype=np.int64)
    p_obs = workloads.random_field((2, len(rec)), 42)
    J_ref, q_ref = oracle.receiver_misfit(p, rec, p_obs)
    plan = tbs.Plan(shape, 1.0, 1.0 + 0.1j, dtype=tdt(dt), batch=2)
    flat = torch.from_numpy(rec[:, 0] * shape[1] + rec[:, 1]).to(dev)
    q, J = plan.misfit(to_dev(p, dev, dt), flat, to_dev(p_obs, dev, dt))
    assert abs(J.item() - J_ref) <= TOL[dt] * J_ref
    assert rel(q.cpu().numpy(), q_ref) <= TOL[dt]
    plan.close()


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("shape", [(40, 36), (10, 12, 14)])
def test_second_harmonic_chain(dev, dt, shape, errlog):
    """p1 at omega, S2 = -xi (2 omega)^2 p1^2 / 2, p2 at 2 omega (the paper's
    Sec. 2.3.4 scheme, sum term only) against the oracle chain."""
    import paper_2507_13754_amd as tbs
    f = 3e6
    om = 2 * np.pi * f
    dx = workloads.C0 / f / 6
    c = workloads.small_medium(shape, dx, 0.02, seed=31)
    a0, y = workloads.alpha0_si(0.75, 1.5), 1.5
    s = np.zeros((1,) + shape, np.complex128)
    s[(0,) + tuple(n // 3 for n in shape)] = 1.0 / dx ** len(shape)
    L = 5
    k1 = oracle.background_k0(om, workloads.C0, a0, y)
    p1, _ = oracle.solve(k1, dx, s, oracle.potential(c, om, workloads.C0, a0, y), L)
    S2 = oracle.harmonic_source(p1, c, om, workloads.RHO0, 7.0)
    k2 = oracle.background_k0(2 * om, workloads.C0, a0, y)
    p2, _ = oracle.solve(k2, dx, S2, oracle.potential(c, 2 * om, workloads.C0, a0, y), L)

    cd = torch.from_numpy(c).to(dev)
    pl1 = tbs.Plan(shape, dx, tbs.background_k0(om, workloads.C0, a0, y), dtype=tdt(dt)).tabulate()
    pl2 = tbs.Plan(shape, dx, tbs.background_k0(2 * om, workloads.C0, a0, y), dtype=tdt(dt)).tabulate()
    g1 = pl1.solve(to_dev(s, dev, dt), pl1.potential(cd, om, workloads.C0, a0, y), L)
    gS = pl1.harmonic_source(g1, cd, om, workloads.RHO0, 7.0)
    assert errlog("S2", rel(gS.cpu().numpy(), S2), TOL[dt]) <= TOL[dt]
    g2 = pl2.solve(gS, pl2.potential(cd, 2 * om, workloads.C0, a0, y), L)
    assert errlog("p2", rel(g2.cpu().numpy(), p2), TOL[dt]) <= TOL[dt]
    pl1.close()
    pl2.close()


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("shape", [(21, 34), (6, 7, 9)])
def test_adjoint_field_matches_oracle(dev, dt, shape):
    """TBS_ADJ_SERIES_ONLY: A_L^H q = sum_m (G^H conj(V))^m G^H q against the
    oracle's series with G^H and conj(V), and <A_L s, q> = <s, A_L^H q>."""
    import paper_2507_13754_amd as tbs
    k0 = 2 * np.pi / 6 * (1 + 0.02j)
    V = 0.05 * (k0 * k0).real * workloads.random_field(shape, 13)
    s = workloads.random_field((2,) + shape, 14)
    q = workloads.random_field((2,) + shape, 15)
    L = 6
    G = oracle.GreenOperator(k0, 1.0, shape)
    ref, _ = oracle.born_series(lambda f: G(f, adjoint=True), q, np.conj(V), L)
    plan = tbs.Plan(shape, 1.0, k0, dtype=tdt(dt), batch=2).tabulate()
    w = plan.adjoint(None, to_dev(V, dev, dt), L, to_dev(q, dev, dt), flags=tbs.TBS_ADJ_SERIES_ONLY)
    w = w.cpu().numpy().astype(np.complex128)
    assert max(rel(w[b], ref[b]) for b in range(2)) <= TOL[dt]
    if dt == "c128":
        p = plan.solve(to_dev(s, dev, dt), to_dev(V, dev, dt), L).cpu().numpy()
        for b in range(2):
            lhs, rhs = np.vdot(q[b], p[b]), np.vdot(w[b], s[b])
            assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    plan.close()
