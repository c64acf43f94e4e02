"""tbs_solve_noalloc (the series on the library's static device workspace)
against tbs_solve, through the C ABI (GPU).

Two calls in a row, the second on a smaller problem, each compared with
tbs_solve on the same plan and inputs: the two entry points run the same
kernels in the same order, so fields and residual histories must agree
bitwise.  A plan whose workspace exceeds the static array is refused with
TBS_ERR_UNSUPPORTED before any launch.
"""
import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TBS_ERR_UNSUPPORTED = -2


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _inputs(dev, dtype, grid, nrhs, seed):
    import paper_2507_13754_amd as tbs
    f = 1.0e6
    dx = workloads.C0 / f / 8.0
    alpha0 = workloads.alpha0_si(0.5, 1.0)
    c = workloads.small_medium(grid, dx, 0.02, seed)
    rng = np.random.Generator(np.random.PCG64(seed + 100))
    s = np.zeros((nrhs,) + tuple(grid), dtype=np.complex128)
    for b in range(nrhs):
        for _ in range(6):
            idx = tuple(int(rng.integers(0, n)) for n in grid)
            s[(b,) + idx] += complex(rng.standard_normal(), rng.standard_normal()) / dx ** len(grid)
    om = 2 * np.pi * f
    plan = tbs.Plan(grid, dx, tbs.background_k0(om, workloads.C0, alpha0, 1.0), dtype=dtype,
                    batch=nrhs).tabulate()
    V = plan.potential(torch.from_numpy(c).to(dev), om, workloads.C0, alpha0, 1.0)
    return plan, torch.from_numpy(s).to(dev, dtype), V


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128], ids=["c64", "c128"])
def test_noalloc_matches_solve_two_calls(dev, dtype):
    L = 12
    # first a 2D problem with two right-hand sides, then a smaller 3D one
    for grid, nrhs, seed in (((200, 256), 2, 11), ((12, 20, 24), 1, 12)):
        print(f"noalloc case grid={grid} rhs={nrhs} dtype={dtype}", flush=True)
        plan, s, V = _inputs(dev, dtype, grid, nrhs, seed)
        ref, rref = plan.solve(s, V, L, residual=True)
        out = torch.full_like(ref, float("nan"))
        got, rgot = plan.solve_noalloc(s, V, L, out, residual=True)
        torch.cuda.synchronize()
        assert got.data_ptr() == out.data_ptr()
        assert torch.equal(got, ref), float((got - ref).abs().max())
        assert np.array_equal(rgot, rref)
        # the plan's own workspace still serves tbs_solve afterwards
        again = plan.solve(s, V, L)
        assert torch.equal(again, ref)
        plan.close()


def test_noalloc_refuses_oversize(dev):
    import paper_2507_13754_amd as tbs
    # 2048^2 FP32 with two right-hand sides: 2 x (4096 x 2048 x 8 + 2048^2 x 4)
    # bytes of workspace, beyond the 128 MiB static array
    grid = (2048, 2048)
    f = 5.0e6
    dx = workloads.C0 / f / 6.0
    plan = tbs.Plan(grid, dx, tbs.background_k0(2 * np.pi * f, workloads.C0, 0.0, 1.0),
                    dtype=torch.complex64, batch=2).tabulate()
    s = torch.zeros((2,) + grid, dtype=torch.complex64, device=dev)
    out = torch.empty_like(s)
    with pytest.raises(tbs.TBSError) as ei:
        plan.solve_noalloc(s, None, 3, out)
    assert ei.value.status == TBS_ERR_UNSUPPORTED
    assert "static scratch" in str(ei.value)
    plan.close()
