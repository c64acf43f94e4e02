"""Batched multi-grid solves (grouped launches + recorded graph) against the
oracle and against single-plan solves; mixed-radix padded lengths."""
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


# frequency indices whose 1.2 cm grids pad to 3*2^a, 5*2^a and 2^a lengths,
# two of them sharing a length (one grouped launch)
FREQS = [0, 9, 20, 30, 31, 47]


def cases(nangles=3, nterms=6):
    return [workloads.broadband(i, nangles=nangles, nterms=nterms, extent=0.012) for i in FREQS]


def build(dev, cs, dt):
    import paper_2507_13754_amd as tbs
    plans, srcs, pots = [], [], []
    for c in cs:
        k0 = tbs.background_k0(c.omega, c.c0, c.alpha0, c.y)
        p = tbs.Plan(c.grid, c.dx, k0, dtype=tdt(dt), batch=c.sources.shape[0]).tabulate()
        plans.append(p)
        srcs.append(torch.from_numpy(c.sources).to(dev, tdt(dt)))
        pots.append(p.potential(torch.from_numpy(c.c).to(dev), c.omega, c.c0, c.alpha0, c.y))
    return plans, srcs, pots


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_batch_matches_oracle(dev, dt):
    import paper_2507_13754_amd as tbs
    cs = cases()
    plans, srcs, pots = build(dev, cs, dt)
    lengths = sorted({p.padded[0] for p in plans})
    odd = {m // (m & -m) for m in lengths}
    assert odd >= {1, 3, 5} and len(lengths) < len(plans)   # all families, one shared length
    batch = tbs.Batch(plans)
    outs, res = batch.solve(srcs, pots, cs[0].nterms, residual=True)
    row = 0
    for c, o in zip(cs, outs):
        k0 = oracle.background_k0(c.omega, c.c0, c.alpha0, c.y)
        V = oracle.potential(c.c, c.omega, c.c0, c.alpha0, c.y)
        p_ref, r_ref = oracle.solve(k0, c.dx, c.sources, V, c.nterms)
        got = o.cpu().numpy().astype(np.complex128)
        err = max(rel(got[b], p_ref[b]) for b in range(got.shape[0]))
        assert err <= TOL[dt], (c.name, err)
        assert np.allclose(res[row:row + got.shape[0]], r_ref, rtol=1e-9 if dt == "c128" else 1e-3)
        row += got.shape[0]
    batch.close()


def test_batch_equals_single_plan_solves_and_replays(dev):
    import paper_2507_13754_amd as tbs
    cs = cases(nangles=2, nterms=5)
    plans, srcs, pots = build(dev, cs, "c64")
    batch = tbs.Batch(plans)
    outs = batch.solve(srcs, pots, 5)
    first = [o.clone() for o in outs]
    for p, s, v, o in zip(plans, srcs, pots, first):
        single = p.solve(s, v, 5)
        assert torch.equal(single, o)
    # replay of the recorded graph with the same buffers
    outs2 = batch.solve(srcs, pots, 5, outs=outs)
    for a, b in zip(first, outs2):
        assert torch.equal(a, b)
    # new contents in the same buffers: the replay reads them
    for s in srcs:
        s.mul_(2.0)
    outs3 = batch.solve(srcs, pots, 5, outs=outs)
    for a, b in zip(first, outs3):
        assert torch.allclose(b, 2.0 * a, rtol=1e-6, atol=0)
    batch.close()


def test_full_size_smallest_broadband_grid(dev):
    """The 2 MHz grid of the broadband workload at full size (312^2, 16 angles,
    25 terms, padded 640) in FP32 against the oracle."""
    import paper_2507_13754_amd as tbs
    c = workloads.broadband(0)
    plans, srcs, pots = build(dev, [c], "c64")
    assert plans[0].padded[0] == 640
    outs = tbs.Batch(plans).solve(srcs, pots, c.nterms)
    k0 = oracle.background_k0(c.omega, c.c0, c.alpha0, c.y)
    V = oracle.potential(c.c, c.omega, c.c0, c.alpha0, c.y)
    p_ref, _ = oracle.solve(k0, c.dx, c.sources, V, c.nterms)
    got = outs[0].cpu().numpy().astype(np.complex128)
    assert max(rel(got[b], p_ref[b]) for b in range(16)) <= TOL["c64"]


def test_batch_rerecords_after_member_plan_grows(dev):
    """A member plan solved alone with more terms reallocates its norm partials;
    the next batch solve with the old pointers must re-record, not replay into
    the freed buffer.  Tuning a plan that belongs to a live batch is refused."""
    import paper_2507_13754_amd as tbs
    cs = cases(nangles=2, nterms=4)
    plans, srcs, pots = build(dev, cs, "c64")
    batch = tbs.Batch(plans)
    outs = batch.solve(srcs, pots, 4)
    first = [o.clone() for o in outs]
    # a much longer single solve grows plans[0]'s partials past the batch's L
    plans[0].solve(srcs[0], pots[0], 40)
    torch.cuda.synchronize()
    outs2, res = batch.solve(srcs, pots, 4, outs=outs, residual=True)
    for a, b in zip(first, outs2):
        assert torch.equal(a, b)
    assert np.all(np.isfinite(res))
    with pytest.raises(tbs.TBSError):
        plans[1].autotune()
    batch.close()
    plans[1].autotune()          # allowed again once the batch is gone
    for p in plans:
        p.close()


def test_launch_chains_are_bitwise_one(dev, monkeypatch):
    """Several launch chains (the tiles of each set going to 2, 3 (the
    default) or 4 streams in turn) against one chain (TBS_BATCH_CHAINS=1):
    the same kernels on the same data, bitwise, replays included."""
    import paper_2507_13754_amd as tbs
    cs = cases(nangles=2, nterms=6) + [workloads.broadband(40, nangles=4, nterms=6)]
    plans, srcs, pots = build(dev, cs, "c64")
    monkeypatch.setenv("TBS_BATCH_CHAINS", "1")
    one = tbs.Batch(plans)
    ref, rref = one.solve(srcs, pots, 6, residual=True)
    ref = [o.clone() for o in ref]
    one.close()
    for k in ("2", None, "4"):
        if k is None:
            monkeypatch.delenv("TBS_BATCH_CHAINS")
        else:
            monkeypatch.setenv("TBS_BATCH_CHAINS", k)
        many = tbs.Batch(plans)
        outs, res = many.solve(srcs, pots, 6, residual=True)
        for a, b in zip(ref, outs):
            assert torch.equal(a, b), k
        for a, b in zip(rref, res):
            assert np.array_equal(a, b), k
        outs2 = many.solve(srcs, pots, 6, outs=outs)
        for a, b in zip(ref, outs2):
            assert torch.equal(a, b), k
        many.close()
    for p in plans:
        p.close()


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_batch_autotune_is_bitwise_neutral_and_cached(dev, tmp_path, monkeypatch, dt):
    """tbs_batch_autotune times the grouped launches' block shapes and the
    number of launch chains and regroups: the fields after tuning equal the
    untuned ones bitwise (every
    block shape of a length keeps its twiddle factors where the default shape
    does, 2560 lines with 1, 2 or 4 columns and 2 or 4 rows per block
    included), and the choices land in the TBS_TUNE_CACHE file."""
    import paper_2507_13754_amd as tbs
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("TBS_TUNE_CACHE", str(cache))
    cs = cases(nangles=2, nterms=5) + [workloads.broadband(40, nangles=2, nterms=5)]
    plans, srcs, pots = build(dev, cs, dt)
    batch = tbs.Batch(plans)
    ref = [o.clone() for o in batch.solve(srcs, pots, 5)]
    outs = [torch.empty_like(o) for o in ref]
    batch.autotune(srcs, pots, outs)
    got = batch.solve(srcs, pots, 5, outs=outs)
    for a, b in zip(ref, got):
        assert torch.equal(a, b)
    batch.close()
    lines = cache.read_text().splitlines() if cache.exists() else []
    # only lengths with more than one candidate shape are timed and stored
    assert all(" = " in ln and ln.split()[0] in ("batchrow", "batchcol", "batchchains") for ln in lines)
    assert any(ln.startswith("batchchains ") for ln in lines)
    for p in plans:
        p.close()


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_tile_schedules_are_bitwise_one_set(dev, monkeypatch, dt):
    """The cache-sized schedule (right-hand sides cut into tiles, tiles packed
    into sets that run their whole series one after the other, the tiles of
    a set alternating between two streams) against all plans as one set of
    whole plans on one stream: the same arithmetic per right-hand side,
    bitwise, with the residual histories; uneven tiles (5 RHS in tiles of
    3 + 2 and 4 + 1) and many small sets included, with one grid of the full
    broadband size."""
    import paper_2507_13754_amd as tbs
    cs = cases(nangles=3, nterms=5) + [workloads.broadband(40, nangles=5, nterms=5)]
    plans, srcs, pots = build(dev, cs, dt)
    monkeypatch.setenv("TBS_BATCH_CACHE_MB", "0")
    monkeypatch.setenv("TBS_BATCH_CHAINS", "1")
    whole = tbs.Batch(plans)
    ref, rref = whole.solve(srcs, pots, 5, residual=True)
    ref = [o.clone() for o in ref]
    whole.close()
    monkeypatch.delenv("TBS_BATCH_CHAINS")
    for cap, trhs in (("0", "2"), ("200", "4"), ("256", "2"), ("20", "3"), ("1", "1")):
        monkeypatch.setenv("TBS_BATCH_CACHE_MB", cap)
        monkeypatch.setenv("TBS_BATCH_TILE_RHS", trhs)
        tiled = tbs.Batch(plans)
        outs, res = tiled.solve(srcs, pots, 5, residual=True)
        for a, b in zip(ref, outs):
            assert torch.equal(a, b)
        for a, b in zip(rref, res):
            assert np.array_equal(a, b)
        tiled.close()
    for p in plans:
        p.close()


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_every_block_shape_is_bitwise_one(dev, monkeypatch, dt):
    """Every block shape the tuners choose from (TBS_BATCH_SHAPE: 2 or 4 rows
    and 1, 2 or 4 columns per block) gives the default shape's fields
    bitwise: a length keeps its twiddle factors where its default shape does,
    whatever the shape (lines of 512, 640 and 768, and a full-size grid with
    2560 lines).  The residual histories are FP64 sums of per-block partial
    norms, so another number of rows per block changes their summation order:
    equal to 1e-13."""
    import paper_2507_13754_amd as tbs
    cs = cases(nangles=2, nterms=5) + [workloads.broadband(40, nangles=2, nterms=5)]
    plans, srcs, pots = build(dev, cs, dt)
    base = tbs.Batch(plans)
    ref, rref = base.solve(srcs, pots, 5, residual=True)
    ref = [o.clone() for o in ref]
    base.close()
    for shape in ("2,1", "4,2", "2,4", "4,1"):
        fresh, fsrcs, fpots = build(dev, cs, dt)
        monkeypatch.setenv("TBS_BATCH_SHAPE", shape)
        b = tbs.Batch(fresh)
        outs, res = b.solve(fsrcs, fpots, 5, residual=True)
        for a, g in zip(ref, outs):
            assert torch.equal(a, g), shape
        for a, g in zip(rref, res):
            assert np.allclose(a, g, rtol=1e-13, atol=0), shape
        b.close()
        monkeypatch.delenv("TBS_BATCH_SHAPE")
        for p in fresh:
            p.close()
    for p in plans:
        p.close()
