"""Parity at the measured workloads' full sizes, in the launch configuration
the benchmark times (FP32 plans with autotuned block shapes, the broadband
batch as one grouped graph): against the FP64 oracle where it runs in
seconds, otherwise on sampled right-hand sides or a shortened series."""
import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def test_absorb2d_full_size(dev):
    """2048^2, 30 terms, FP32 + Kahan with the autotuned block shapes."""
    import paper_2507_13754_amd as tbs
    case = workloads.absorb2d()
    k0 = oracle.background_k0(case.omega, case.c0, case.alpha0, case.y)
    V = oracle.potential(case.c, case.omega, case.c0, case.alpha0, case.y)
    p_ref, r_ref = oracle.solve(k0, case.dx, case.sources, V, case.nterms)
    plan = tbs.Plan(case.grid, case.dx, tbs.background_k0(case.omega, case.c0, case.alpha0, case.y),
                    dtype=torch.complex64).tabulate()
    plan.autotune()
    Vg = plan.potential(torch.from_numpy(case.c).to(dev), case.omega, case.c0, case.alpha0, case.y)
    p, r = plan.solve(torch.from_numpy(case.sources).to(dev, torch.complex64), Vg, case.nterms, residual=True)
    assert rel(p.cpu().numpy().astype(np.complex128)[0], p_ref[0]) <= 1e-5
    assert np.allclose(r, r_ref, rtol=1e-3, atol=0)
    plan.close()


def test_broadband_full_batch_sampled(dev):
    """All 48 grids (312^2 .. 1247^2, 16 RHS, 25 terms) in one batch; the
    largest grid's first and last steering angles against the oracle."""
    import paper_2507_13754_amd as tbs
    plans, srcs, pots = [], [], []
    for i in range(len(workloads.BROADBAND_FREQS)):
        c = workloads.broadband(i)
        p = tbs.Plan(c.grid, c.dx, tbs.background_k0(c.omega, c.c0, c.alpha0, c.y),
                     dtype=torch.complex64, batch=c.sources.shape[0]).tabulate()
        p.autotune()
        plans.append(p)
        srcs.append(torch.from_numpy(c.sources).to(dev, torch.complex64))
        pots.append(p.potential(torch.from_numpy(c.c).to(dev), c.omega, c.c0, c.alpha0, c.y))
    batch = tbs.Batch(plans)
    outs = batch.solve(srcs, pots, 25)
    c = workloads.broadband(47)
    assert c.grid == (1247, 1247) and plans[-1].padded[0] == 2560
    k0 = oracle.background_k0(c.omega, c.c0, c.alpha0, c.y)
    V = oracle.potential(c.c, c.omega, c.c0, c.alpha0, c.y)
    got = outs[-1].cpu().numpy().astype(np.complex128)
    for b in (0, 15):
        p_ref, _ = oracle.solve(k0, c.dx, c.sources[b:b + 1], V, c.nterms)
        assert rel(got[b], p_ref[0]) <= 1e-5, b
    batch.close()
    for p in plans:
        p.close()


def test_harmonic3d_full_size(dev):
    """256^3 at 3 MHz: the first two terms against the oracle; the full 24-term
    fundamental, the source and the 24-term 6 MHz solve of the FP32 plan
    against the FP64 plan (both parity-tested against the oracle at small
    sizes)."""
    import paper_2507_13754_amd as tbs
    case = workloads.harmonic3d()
    k0 = oracle.background_k0(case.omega, case.c0, case.alpha0, case.y)
    V = oracle.potential(case.c, case.omega, case.c0, case.alpha0, case.y)
    p_ref, _ = oracle.solve(k0, case.dx, case.sources, V, 2)
    cd = torch.from_numpy(case.c).to(dev)
    res = {}
    for dt in (torch.complex64, torch.complex128):
        pl1 = tbs.Plan(case.grid, case.dx, tbs.background_k0(case.omega, case.c0, case.alpha0, case.y),
                       dtype=dt).tabulate()
        V1 = pl1.potential(cd, case.omega, case.c0, case.alpha0, case.y)
        s = torch.from_numpy(case.sources).to(dev, dt)
        if dt == torch.complex64:
            two = pl1.solve(s, V1, 2).cpu().numpy().astype(np.complex128)
            assert rel(two[0], p_ref[0]) <= 1e-5
        p1 = pl1.solve(s, V1, case.nterms)
        S2 = pl1.harmonic_source(p1, cd, case.omega, case.rho, case.BA)
        pl1.close()
        om2 = 2 * case.omega
        pl2 = tbs.Plan(case.grid, case.dx, tbs.background_k0(om2, case.c0, case.alpha0, case.y),
                       dtype=dt).tabulate()
        p2 = pl2.solve(S2, pl2.potential(cd, om2, case.c0, case.alpha0, case.y), case.nterms)
        res[dt] = (p1.cpu().numpy().astype(np.complex128), p2.cpu().numpy().astype(np.complex128))
        pl2.close()
        del p1, p2, S2
        torch.cuda.empty_cache()
    a, b = res[torch.complex64], res[torch.complex128]
    assert rel(a[0], b[0]) <= 1e-5 and rel(a[1], b[1]) <= 1e-5


def test_adjoint2d_full_size_one_case(dev, errlog):
    """1024^2, 25 terms: the FP32 adjoint gradient with recomputation (the
    benchmark's setting) for one frequency and one source against the
    oracle's adjoint."""
    import paper_2507_13754_amd as tbs
    prob = workloads.adjoint2d()
    f = prob.freqs[len(prob.freqs) // 2]
    om = 2 * np.pi * f
    s = prob.sources[3:4]
    k0 = oracle.background_k0(om, workloads.C0, prob.alpha0, prob.y)
    V = oracle.potential(prob.c_model, om, workloads.C0, prob.alpha0, prob.y)
    q = workloads.random_field((1,) + prob.grid, 91)
    G = oracle.GreenOperator(k0, prob.dx, prob.grid)
    ref = oracle.adjoint_series_gradient(G, s[0], V, prob.nterms, q[0])
    plan = tbs.Plan(prob.grid, prob.dx, tbs.background_k0(om, workloads.C0, prob.alpha0, prob.y),
                    dtype=torch.complex64).tabulate()
    Vg = plan.potential(torch.from_numpy(prob.c_model).to(dev), om, workloads.C0, prob.alpha0, prob.y)
    g = plan.adjoint(torch.from_numpy(s).to(dev, torch.complex64), Vg, prob.nterms,
                     torch.from_numpy(q).to(dev, torch.complex64), flags=tbs.TBS_ADJ_RECOMPUTE)
    assert errlog("gradient", rel(g.cpu().numpy().astype(np.complex128)[0], ref), 1e-5) <= 1e-5
    plan.close()
