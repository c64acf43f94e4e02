"""Chained higher harmonics (fundamental, then harmonics 2..5 one by one, each
driven by the sum-frequency source of the lower ones) against the oracle
chain, FP64 <= 1e-12 and FP32 <= 1e-5 relative L2 (x3 for the chain)."""
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
def test_harmonics_up_to_fifth(dev, dt, shape):
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
        assert rel(got[-1].cpu().numpy(), ref[n - 1]) <= TOL[dt] * 3, n
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
