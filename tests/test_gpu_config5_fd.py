"""The misfit gradient of the full adjoint workload (1024^2, 16 frequencies
2-6 MHz x 8 sources, 128 receivers, 25 terms) against central finite
differences at its 64 seeded pixels (GPU).

The gradient is the FP32 adjoint through torch.autograd with term
recomputation (checkpoints instead of stored partial sums); the finite
differences use the FP64 series, h = 1e-6 c0.  Both sides use the same
observed data, synthesised with the FP64 series from the true map.  Agreement
<= 1e-4 of max |dJ/dc| (the adjoint's FD bar).
"""
import math

import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def test_full_adjoint_gradient_finite_differences(dev):
    import paper_2507_13754_amd as tbs
    from paper_2507_13754_amd.autograd import MisfitProblem, TBSMisfit
    prob = workloads.adjoint2d()
    n = prob.grid[0]
    rec = torch.from_numpy(prob.receivers[:, 0] * n + prob.receivers[:, 1]).to(dev)
    src64 = torch.from_numpy(prob.sources).to(dev, torch.complex128)
    ct = torch.from_numpy(prob.c_true).to(dev)
    p_obs = []
    for f in prob.freqs:
        om = 2 * math.pi * f
        pl = tbs.Plan(prob.grid, prob.dx, tbs.background_k0(om, workloads.C0, prob.alpha0, prob.y),
                      dtype=torch.complex128, batch=src64.shape[0]).tabulate()
        p = pl.solve(src64, pl.potential(ct, om, workloads.C0, prob.alpha0, prob.y), prob.nterms)
        p_obs.append(p[:, prob.receivers[:, 0], prob.receivers[:, 1]].contiguous())
        pl.close()
    mp32 = MisfitProblem(prob.grid, prob.dx, prob.freqs, workloads.C0, prob.alpha0, prob.y, src64, rec,
                         p_obs, prob.nterms, dtype=torch.complex64, adjoint_flags=tbs.TBS_ADJ_RECOMPUTE)
    c = torch.from_numpy(prob.c_model).to(dev).requires_grad_(True)
    TBSMisfit.apply(c, mp32).backward()
    g = c.grad.cpu().numpy()
    mp32.close()
    gmax = float(np.max(np.abs(g)))
    assert gmax > 0
    mp64 = MisfitProblem(prob.grid, prob.dx, prob.freqs, workloads.C0, prob.alpha0, prob.y, src64, rec,
                         p_obs, prob.nterms, dtype=torch.complex128)
    h = 1e-6 * workloads.C0
    cm = torch.from_numpy(prob.c_model).to(dev)
    worst = 0.0
    for iy, ix in prob.fd_pixels:
        cp = cm.clone()
        cp[iy, ix] += h
        cn = cm.clone()
        cn[iy, ix] -= h
        with torch.no_grad():
            Jp = TBSMisfit.apply(cp, mp64).item()
            Jm = TBSMisfit.apply(cn, mp64).item()
        fd = (Jp - Jm) / (2 * h)
        err = abs(fd - g[iy, ix]) / gmax
        worst = max(worst, err)
        assert err <= 1e-4, (int(iy), int(ix), fd, g[iy, ix], gmax)
    print(f"config-5 FD check: 64 pixels, worst |fd - grad| / max|grad| = {worst:.2e}", flush=True)
    mp64.close()
