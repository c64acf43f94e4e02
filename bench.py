#!/usr/bin/env python3
"""Throughput of the Born-series hot path on one MI355X.

One step = one full L-term solve (every row and column pass of every term)
of one batch of right-hand sides, with inputs already resident in HBM.
value = physical grid points x summed terms x RHS / step time
(grid-point.terms/s), for the FP32 (Kahan) plan; the plain FP64 plan is timed
beside it on the same input and its accuracy gap is stated.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published
METRIC = "Born grid-point·terms/s + HBM GB/s frac, FP32 batched vs FP64 plain, 1 GPU"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_sources_hash() -> str:
    h = hashlib.sha256()
    for f in ("tbs_passes.hpp", "tbs_fft.hpp", "tbs_internal.hpp"):
        with open(os.path.join(ROOT, "paper_2507_13754_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def pass_bytes(kind: str, ndim: int, N, M, B: int, esz: int, kahan: bool, ghat_bytes: int) -> int:
    """Algorithmic HBM bytes of one launch of a pass: every array the pass
    must read or write, once.  N, M: (x, y, z) physical / padded sizes."""
    P = N[0] * N[1] * N[2]
    rows = N[1] * N[2]
    X = B * rows * M[0] * esz                 # x-spectral intermediate
    acc_rw = B * P * esz * (3 if kahan else 2)   # p read + write (and Kahan c, bf16 pairs: half size)
    if kind == "row_first":
        return B * P * esz + X
    if kind == "row_mid":
        return 2 * X + P * esz + acc_rw
    if kind == "row_last":
        return X + acc_rw
    if kind == "col_conv":
        if ndim == 2:
            return 2 * X + ghat_bytes
        return 2 * B * M[0] * M[1] * N[2] * esz + ghat_bytes
    if kind in ("col_fwd", "col_inv"):
        return X + B * M[0] * M[1] * N[2] * esz
    raise ValueError(kind)


# Non-packed FP32 vector peak of MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2 flops
# (FMA) x 2.4 GHz.  (The published 157.3 TFLOP/s counts packed FP32, which
# these kernels do not issue; FP64 vector is the same 78.6.)
VALU_PEAK_TFLOPS = 78.6


def pass_flops(kind: str, ndim: int, N, M, B: int) -> float:
    """Algorithmic floating-point work of one launch of a pass: 5 n log2 n per
    complex FFT of length n (the radix-2 count) and 6 per complex product."""
    def fft(n):
        return 5.0 * n * math.log2(n)
    rows = N[1] * N[2]
    if kind in ("row_first", "row_last"):
        return float(B * rows * fft(M[0]))
    if kind == "row_mid":
        return float(B * rows * (2 * fft(M[0]) + 6 * N[0]))
    if kind == "col_conv":
        if ndim == 2:
            return float(B * M[0] * (2 * fft(M[1]) + 6 * M[1]))
        return float(B * M[0] * M[1] * (2 * fft(M[2]) + 6 * M[2]))
    if kind in ("col_fwd", "col_inv"):
        return float(B * M[0] * N[2] * fft(M[1]))
    raise ValueError(kind)


def step_bytes(ndim, N, M, B, esz, kahan, ghat_bytes, L) -> int:
    f = lambda k: pass_bytes(k, ndim, N, M, B, esz, kahan, ghat_bytes)  # noqa: E731
    total = f("row_first") + (L - 1) * f("row_mid") + f("row_last") + L * f("col_conv")
    if ndim == 3:
        total += L * (f("col_fwd") + f("col_inv"))
    return total


def make_workload(name: str):
    import workloads
    if name == "absorb2d":
        case = workloads.absorb2d()
        desc = ("absorb2d: 2048x2048 grid, dx=lambda/6 at 5 MHz, 111 Gaussian blobs c0 +-3%, "
                "0.75 dB/(MHz^1.5 cm) y=1.5 with dispersion, 64-element line array, 30 terms, 1 RHS")
    elif name == "plain2d":
        case = workloads.plain2d()
        desc = "plain2d: 256x256, dx=lambda/8 at 1 MHz, 1% GRF, 0.5 dB/cm/MHz y=1, 32 elements, 16 terms"
    else:
        raise SystemExit(f"unknown workload {name}")
    return case, desc


def time_solves(plan, s, V, L, out, steps, warmup):
    import torch
    for _ in range(warmup):
        plan.solve(s, V, L, out=out)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        plan.solve(s, V, L, out=out)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / steps, wall / steps * 1e3


def profile_passes(plan, s, V, L, out, steps):
    import paper_2507_13754_amd as tbs
    plan.profile(True)
    for _ in range(steps):
        plan.solve(s, V, L, out=out)
    prof = plan.profile_read()
    plan.profile(False)
    return prof


def cpu_baseline(case, budget_s: float):
    """The FP64 oracle on the host: the same series on the same input for as
    many terms as fit the time budget (spectrum tabulation excluded)."""
    import oracle
    k0 = oracle.background_k0(case.omega, case.c0, case.alpha0, case.y)
    V = oracle.potential(case.c, case.omega, case.c0, case.alpha0, case.y)
    G = oracle.GreenOperator(k0, case.dx, case.grid)
    t0 = time.perf_counter()
    G(case.sources)
    t_apply = time.perf_counter() - t0
    nterms = int(max(1, min(case.nterms, budget_s // max(t_apply, 1e-3))))
    t0 = time.perf_counter()
    oracle.born_series(G, case.sources, V, nterms)
    t = time.perf_counter() - t0
    gpt = case.points * nterms * case.sources.shape[0]
    return {
        "value": gpt / t,
        "unit": "grid-point·terms/s",
        "cores": int(oracle.tbs_oracle.WORKERS),
        "kind": "oracle",
        "sample": f"{case.name}: first {nterms} of {case.nterms} terms, {case.sources.shape[0]} RHS, "
                  f"FP64 numpy/scipy.fft, {t:.1f} s",
    }


def read_counters(workload: str, kernel: str):
    path = os.path.join(ROOT, "profiles", f"counters_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("sources_sha256_16") != kernel_sources_hash():
        return None
    return d.get("traffic_bytes_per_launch")


def grid_step_bytes(grid, padded, B, esz, kahan, L):
    N = (grid[-1], grid[-2], grid[-3] if len(grid) == 3 else 1)
    M = (padded[0], padded[1], padded[2] if len(grid) == 3 else 1)
    g = (M[0] // 2 + 1) * (M[1] // 2 + 1) * ((M[2] // 2 + 1) if len(grid) == 3 else 1) * esz
    return step_bytes(len(grid), N, M, B, esz, kahan, g, L)


def run_broadband(dev, steps: int, warmup: int, fp64: bool, cpu_seconds: float, tune: bool = True):
    """48 frequencies (2-8 MHz) on their own lambda/6 grids over 4 x 4 cm, 16
    steering angles each, 25 terms: one batch, replayed as one graph."""
    import torch
    import workloads
    import paper_2507_13754_amd as tbs
    out = {}
    for name, dtype in (("c64", torch.complex64), ("c128", torch.complex128)):
        if name == "c128" and not fp64:
            continue
        plans, srcs, pots, gpts, nbytes = [], [], [], 0, 0
        t0 = time.perf_counter()
        for i in range(len(workloads.BROADBAND_FREQS)):
            c = workloads.broadband(i)
            k0 = tbs.background_k0(c.omega, c.c0, c.alpha0, c.y)
            p = tbs.Plan(c.grid, c.dx, k0, dtype=dtype, batch=c.sources.shape[0]).tabulate()
            if tune:
                p.autotune()
            plans.append(p)
            srcs.append(torch.from_numpy(c.sources).to(dev, dtype))
            pots.append(p.potential(torch.from_numpy(c.c).to(dev), c.omega, c.c0, c.alpha0, c.y))
            gpts += c.points * c.nterms * c.sources.shape[0]
            nbytes += grid_step_bytes(c.grid, p.padded, c.sources.shape[0], 8 if name == "c64" else 16,
                                      name == "c64", c.nterms)
            L = c.nterms
            del c
        log(f"[bench] broadband {name}: 48 plans built in {time.perf_counter() - t0:.1f} s")
        batch = tbs.Batch(plans)
        outs = batch.solve(srcs, pots, L)
        ms, wall = time_solves_fn(lambda: batch.solve(srcs, pots, L, outs=outs), steps, warmup)
        log(f"[bench] broadband {name}: {ms:.2f} ms/step")
        out[name] = dict(ms=ms, value=gpts / (ms * 1e-3), bytes=nbytes,
                         GBps=nbytes / (ms * 1e-3) / 1e9, outs=[o.cpu() for o in outs],
                         lengths=sorted({p.padded[0] for p in plans}))
        batch.close()
        for p in plans:
            p.close()
        del srcs, pots, outs
        torch.cuda.empty_cache()
    res = {"workload": "broadband: 48 frequencies 2-8 MHz, lambda/6 grids over 4x4 cm (312^2..1247^2), "
                       "16 steering angles each, 25 terms, one recorded graph per solve",
           "value": out["c64"]["value"], "unit": "grid-point·terms/s", "ms_per_step": out["c64"]["ms"],
           "alg_bytes_per_step": out["c64"]["bytes"], "achieved_GBps": out["c64"]["GBps"],
           "frac": out["c64"]["GBps"] / HBM_PEAK_GBS, "padded_lengths": out["c64"]["lengths"]}
    if "c128" in out:
        errs = []
        for a, b in zip(out["c64"]["outs"], out["c128"]["outs"]):
            a = a.numpy().astype(np.complex128)
            b = b.numpy()
            errs.append(max(float(np.linalg.norm(a[k] - b[k]) / np.linalg.norm(b[k])) for k in range(a.shape[0])))
        res["fp64_plain"] = {"value": out["c128"]["value"], "ms_per_step": out["c128"]["ms"],
                             "achieved_GBps": out["c128"]["GBps"], "frac": out["c128"]["GBps"] / HBM_PEAK_GBS}
        res["speedup_fp32_vs_fp64"] = out["c128"]["ms"] / out["c64"]["ms"]
        res["rel_l2_fp32_vs_fp64_max"] = max(errs)
    if cpu_seconds > 0:
        res["cpu_baseline"] = cpu_baseline(workloads.broadband(0), cpu_seconds)
    return res


def time_solves_fn(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps, (time.perf_counter() - t0) / steps * 1e3


def run_harmonic3d(dev, steps: int, warmup: int, fp64: bool):
    """256^3 at lambda/6 (3 MHz), 3D blob tissue; fundamental (24 terms), the
    second-harmonic source, then the 6 MHz solve (24 terms).  One step = both
    series and the source kernel."""
    import torch
    import workloads
    import paper_2507_13754_amd as tbs
    c = workloads.harmonic3d()
    cd = torch.from_numpy(c.c).to(dev)
    om = c.omega
    res = {"workload": "harmonic3d: 256^3 grid, dx=lambda/6 at 3 MHz, 11 3D blobs c0 +-2%, rho=1000, B/A=7, "
                       "fundamental 24 terms + second harmonic (6 MHz) 24 terms"}
    outs = {}
    for name, dtype in (("c64", torch.complex64), ("c128", torch.complex128)):
        if name == "c128" and not fp64:
            continue
        p1 = tbs.Plan(c.grid, c.dx, tbs.background_k0(om, c.c0, c.alpha0, c.y), dtype=dtype).tabulate()
        p2 = tbs.Plan(c.grid, c.dx, tbs.background_k0(2 * om, c.c0, c.alpha0, c.y), dtype=dtype).tabulate()
        V1 = p1.potential(cd, om, c.c0, c.alpha0, c.y)
        V2 = p2.potential(cd, 2 * om, c.c0, c.alpha0, c.y)
        s = torch.from_numpy(c.sources).to(dev, dtype)
        f1 = torch.empty_like(s)
        S2 = torch.empty_like(s)
        f2 = torch.empty_like(s)

        def step():
            p1.solve(s, V1, c.nterms, out=f1)
            p1.harmonic_source(f1, cd, om, c.rho, c.BA, out=S2)
            p2.solve(S2, V2, c.nterms, out=f2)

        ms, _ = time_solves_fn(step, steps, warmup)
        esz = 8 if name == "c64" else 16
        nb = 2 * grid_step_bytes(c.grid, p1.padded, 1, esz, name == "c64", c.nterms)
        gpt = 2 * c.points * c.nterms
        log(f"[bench] harmonic3d {name}: {ms:.2f} ms/step")
        outs[name] = (f1.cpu(), f2.cpu())
        entry = {"value": gpt / (ms * 1e-3), "ms_per_step": ms, "alg_bytes_per_step": nb,
                 "achieved_GBps": nb / (ms * 1e-3) / 1e9, "frac": nb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
        if name == "c64":
            res.update(entry)
            res["unit"] = "grid-point·terms/s"
        else:
            res["fp64_plain"] = entry
        p1.close()
        p2.close()
        del s, f1, S2, f2
        torch.cuda.empty_cache()
    if "c128" in outs:
        for k, nm in ((0, "fundamental"), (1, "harmonic")):
            a = outs["c64"][k].numpy().astype(np.complex128)
            b = outs["c128"][k].numpy()
            res[f"rel_l2_fp32_vs_fp64_{nm}"] = float(np.linalg.norm(a - b) / np.linalg.norm(b))
        res["speedup_fp32_vs_fp64"] = res["fp64_plain"]["ms_per_step"] / res["ms_per_step"]
    return res


def run_density(dev, steps: int, warmup: int):
    """absorb2d (2048^2, 30 terms, FP32) with a density contrast: the blob map
    of the medium scaled to gamma_rho = 3 x the speed contrast.  Per term the
    field is kept in space between two row passes: alg. bytes 104 + 24 B per
    grid-point-term (u written and read, gamma read)."""
    import torch
    import workloads
    import paper_2507_13754_amd as tbs
    case = workloads.absorb2d()
    gam = 3.0 * np.abs(case.c / case.c0 - 1.0)
    plan = tbs.Plan(case.grid, case.dx, tbs.background_k0(case.omega, case.c0, case.alpha0, case.y),
                    dtype=torch.complex64).tabulate()
    plan.autotune()
    plan.density_contrast(torch.from_numpy(gam).to(dev))
    V = plan.potential(torch.from_numpy(case.c).to(dev), case.omega, case.c0, case.alpha0, case.y)
    s = torch.from_numpy(case.sources).to(dev, torch.complex64)
    out = torch.empty_like(s)
    ms, _ = time_solves(plan, s, V, case.nterms, out, steps, warmup)
    plan.close()
    gpt = case.points * case.nterms
    nbytes = 128.0 * gpt
    log(f"[bench] density2d: {ms:.3f} ms/step")
    return {"workload": "absorb2d (2048^2, 30 terms) with a density contrast gamma_rho = 3 |c/c0 - 1|",
            "ms_per_step": ms, "value": gpt / (ms * 1e-3), "unit": "grid-point·terms/s",
            "alg_bytes_per_step": nbytes, "achieved_GBps": nbytes / (ms * 1e-3) / 1e9,
            "frac": nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}


# the paper's Table 3 (iterations, seconds on its RTX 4060), context only
PAPER_TABLE3 = {
    "homogeneous": (135, 5.0), "absorbing": (133, 8.0), "absorbing-dispersive": (132, 11.0),
    "inhomogeneous vs=1350": (134, 7.0), "inhomogeneous vs=1650": (134, 7.0),
    "inhomogeneous vs=1800": (134, 7.0), "harmonic 2": (228, 9.0), "harmonic 3": (306, 12.0),
    "harmonic 4": (368, 15.0), "harmonic 5": (416, 16.0),
}


def run_paper(dev, n: int = 4096, fp64: bool = False):
    """The paper's own periodic scheme on its 4096^2 setups (Sec. 3.1,
    Algorithm 1): the linear media of Table 3 and the nonlinear chain up to
    the 5th harmonic (B/A = 5), each iterated to the paper's tolerance 1e-5.
    Time = the whole tbs_iterate call (spectrum tabulated before), wall clock
    after a device sync; alg. bytes per iteration: row pass 40 B/pt (X r+w,
    psi0, psi, V) + column pass 16 B/pt + the folded spectrum (FP32).  With
    the paper's source strength the 5th harmonic is ~1e-39 in these units,
    below FP32's normal range: the FP32 run stalls there and the FP64 run is
    the one to read for the nonlinear chain."""
    import torch
    import workloads
    import paper_2507_13754_amd as tbs
    dtype = torch.complex128 if fp64 else torch.complex64
    esz = 16 if fp64 else 8
    out = {}

    def iterate(case, k, eps, src, vv, V):
        plan = tbs.Plan((n, n), case.dx, k, padding=1, dtype=dtype)
        plan.green_periodic(eps, vv)
        prof = torch.from_numpy(tbs.abl_profile(n, case.dx, case.zeta, case.mu_cells)).to(dev)
        psi = torch.empty((1, n, n), dtype=dtype, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, it, errs = plan.iterate(src, V, prof, prof, case.check_row, case.tol, case.max_iter, out=psi)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        plan.close()
        return psi, it, sec

    def record(name, it, sec, with_v):
        per_pt = (5 if with_v else 4) * esz + 2 * esz + esz * (n // 2 + 1) ** 2 / n ** 2
        nbytes = per_pt * n * n * it
        ref = PAPER_TABLE3.get(name)
        out[name] = {"iterations": it, "seconds": sec, "ms_per_iteration": 1e3 * sec / max(it, 1),
                     "alg_GBps": nbytes / sec / 1e9,
                     "paper_iterations": ref[0] if ref else None,
                     "paper_seconds_rtx4060": ref[1] if ref else None}
        log(f"[bench] paper {'c128' if fp64 else 'c64'} {name}: {it} iterations, {sec * 1e3:.1f} ms")

    media = [("homogeneous", "homogeneous", 1650.0), ("absorbing", "absorbing", 1650.0),
             ("absorbing-dispersive", "absorbing-dispersive", 1650.0)]
    media += [(f"inhomogeneous vs={vs:.0f}", "inhomogeneous", vs) for vs in (1350.0, 1650.0, 1800.0)]
    for name, kind, vs in media:
        case = workloads.paper_periodic(kind, n, vs=vs)
        k = case.omega / case.c0
        eps = case.eps_factor * k * k
        src = torch.from_numpy(case.sources).to(dev, dtype)
        vv, V = None, None
        if case.alpha0:
            vv = tbs.kspace_potential(case.alpha0, case.nu, case.c0, case.omega)
            if not case.dispersion:
                vv.eta = 0.0
        else:
            tmp = tbs.Plan((n, n), case.dx, k, padding=1, dtype=dtype)
            V = tmp.potential(torch.from_numpy(case.c).to(dev), case.omega, case.c0, 0.0, 1.0, eps)
            tmp.close()
        psi, it, sec = iterate(case, k, eps, src, vv, V)
        record(name, it, sec, V is not None)
        del psi, src, V
    # nonlinear: fundamental, then harmonics 2..5 from the sum-frequency sources
    case = workloads.paper_periodic("homogeneous", n)
    c_map = torch.from_numpy(case.c).to(dev)
    fields = []
    for h in range(1, 6):
        k = h * case.omega / case.c0
        eps = case.eps_factor * k * k
        aux = tbs.Plan((n, n), case.dx, k, padding=1, dtype=dtype)
        V = aux.potential(c_map, h * case.omega, case.c0, 0.0, 1.0, eps)
        src = (torch.from_numpy(case.sources).to(dev, dtype) if h == 1
               else aux.harmonic_source_n(h, fields, c_map, case.omega, 1000.0, 5.0))
        aux.close()
        psi, it, sec = iterate(case, k, eps, src, None, V)
        if h > 1:
            record(f"harmonic {h}", it, sec, True)
        fields.append(psi)
        del V, src
    del fields
    torch.cuda.empty_cache()
    total = sum(v["seconds"] for v in out.values())
    paper_total = sum(v["paper_seconds_rtx4060"] for v in out.values())
    return {"workload": f"paper periodic scheme, {n}^2, dx = 20 um, 1007080 Hz, eps = 0.8 k^2, "
                        "501-element line, sigmoid layer, tol 1e-5 (Sec. 3.1, Algorithm 1, Table 3)",
            "dtype": "c128" if fp64 else "c64", "media": out, "total_seconds": total,
            "paper_total_seconds_rtx4060": paper_total}


def run_adjoint2d(dev, steps: int, warmup: int):
    """One misfit gradient: 1024^2, 16 frequencies (2-6 MHz) x 8 sources, 128
    receivers, 25 terms, FP32 adjoint through torch.autograd (forward series,
    misfit, adjoint series paired with stored partial sums)."""
    import torch
    import workloads
    import paper_2507_13754_amd as tbs
    from paper_2507_13754_amd.autograd import MisfitProblem, TBSMisfit
    prob = workloads.adjoint2d()
    n = prob.grid[0]
    rec = torch.from_numpy(prob.receivers[:, 0] * n + prob.receivers[:, 1]).to(dev)
    src = torch.from_numpy(prob.sources).to(dev, torch.complex64)
    ct = torch.from_numpy(prob.c_true).to(dev)
    # observed data from the true map with the same library
    p_obs = []
    for f in prob.freqs:
        om = 2 * math.pi * f
        pl = tbs.Plan(prob.grid, prob.dx, tbs.background_k0(om, workloads.C0, prob.alpha0, prob.y),
                      batch=src.shape[0]).tabulate()
        p = pl.solve(src, pl.potential(ct, om, workloads.C0, prob.alpha0, prob.y), prob.nterms)
        p_obs.append(p[:, prob.receivers[:, 0], prob.receivers[:, 1]].contiguous())
        pl.close()
    mp = MisfitProblem(prob.grid, prob.dx, prob.freqs, workloads.C0, prob.alpha0, prob.y, src, rec,
                       p_obs, prob.nterms)
    c = torch.from_numpy(prob.c_model).to(dev)

    def step():
        cc = c.clone().requires_grad_(True)
        TBSMisfit.apply(cc, mp).backward()
        return cc.grad

    ms, _ = time_solves_fn(step, steps, warmup)
    nsrc = src.shape[0]
    P = n * n
    # forward solve, adjoint's forward replay and adjoint series: 3 series of L terms
    gpt = 3 * P * prob.nterms * nsrc * len(prob.freqs)
    log(f"[bench] adjoint2d: {ms:.1f} ms per gradient")
    mp.close()
    return {"workload": "adjoint2d: 1024^2, 16 frequencies 2-6 MHz x 8 sources, 128 receivers, 25 terms, "
                        "FP32 gradient via torch.autograd", "ms_per_gradient": ms,
            "value": gpt / (ms * 1e-3), "unit": "grid-point·terms/s (3 series per (f, s))"}


# ------------------------------------------------------------------------------
# rocprofv3 summaries (text under profiles/): parse the CSV output of a
# --kernel-trace --stats run, or of two --pmc runs (FETCH_SIZE, WRITE_SIZE) of
# this same script with --calib-copy, and write the per-kernel figures.

KIND_KERNELS = {  # pass kind -> (kernel template name, OP template argument or None)
    "row_mid": ("k_row_pass<", None),
    "col_conv": ("k_col_pass<", 0),
}


def _kernel_matches(name: str, kind: str) -> bool:
    stem, op = KIND_KERNELS[kind]
    if stem not in name:
        return False
    if op is None:
        return True
    args = name.split(stem, 1)[1].split(">", 1)[0].split(",")
    return len(args) >= 5 and args[4].strip() == str(op)


def _csv(path):
    import csv
    with open(path, newline="") as fh:
        return list(csv.DictReader(fh))


def summarize_trace(src: str, out: str, command: str, title: str):
    """Per-kernel durations from <src>/run_kernel_trace.csv into a markdown table."""
    rows = _csv(os.path.join(src, "run_kernel_trace.csv"))
    agg = {}
    for r in rows:
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        a = agg.setdefault(r["Kernel_Name"], dict(n=0, tot=0.0, mn=1e30, mx=0.0, lds=r.get("LDS_Block_Size", ""),
                                                  grid=r.get("Grid_Size_X", ""), block=r.get("Workgroup_Size_X", ""),
                                                  vgpr=r.get("VGPR_Count", ""), scr=r.get("Scratch_Size", "")))
        a["n"] += 1
        a["tot"] += d
        a["mn"] = min(a["mn"], d)
        a["mx"] = max(a["mx"], d)
    lines = [f"# rocprofv3 kernel trace: {title}", "", "Command (repository root as working directory):", "",
             "    " + command, "",
             "Per-kernel durations (us) from the kernel trace of that run.", "",
             "| kernel | calls | total us | avg us | min us | max us | LDS B | VGPR | scratch | grid | block |",
             "|---|---|---|---|---|---|---|---|---|---|---|"]
    for k, a in sorted(agg.items(), key=lambda kv: -kv[1]["tot"]):
        lines.append(f"| `{k}` | {a['n']} | {a['tot']:.1f} | {a['tot'] / a['n']:.2f} | {a['mn']:.2f} | "
                     f"{a['mx']:.2f} | {a['lds']} | {a['vgpr']} | {a['scr']} | {a['grid']} | {a['block']} |")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    log(f"[bench] wrote {out}")


def summarize_counters(src: str, workload: str, command: str):
    """FETCH_SIZE / WRITE_SIZE per dispatch (KiB) from <src>/fetch and
    <src>/write, scaled by what the same counters read for the 256 MiB
    calibration copy, into profiles/counters_<kind>_<workload>.json (+ .md)."""
    import statistics
    vals = {}
    for kind, ctr in (("fetch", "FETCH_SIZE"), ("write", "WRITE_SIZE")):
        for r in _csv(os.path.join(src, kind, "run_counter_collection.csv")):
            if r["Counter_Name"] == ctr:
                vals.setdefault(kind, []).append((r["Kernel_Name"], int(r["Grid_Size"]), float(r["Counter_Value"])))
    calib = 256 * 1024  # KiB read and written by the calibration copy
    factor = {}
    for kind in ("fetch", "write"):
        copies = [v for n, g, v in vals[kind] if "copyBuffer" in n]
        big = max(copies)
        sel = [v for v in copies if v > 0.4 * big]
        factor[kind] = calib / statistics.median(sel)
    out = {}
    md = [f"# HBM traffic counters: {workload}", "", "Commands (repository root as working directory):", "",
          "    " + command, "",
          "FETCH_SIZE and WRITE_SIZE in KiB per dispatch (median over dispatches), scaled by the",
          f"calibration copy of 256 MiB: read factor {factor['fetch']:.3f}, write factor {factor['write']:.3f}.", "",
          "| pass kind | dispatches | FETCH KiB | WRITE KiB | scaled bytes / launch |", "|---|---|---|---|---|"]
    for kind in KIND_KERNELS:
        f = [v for n, g, v in vals["fetch"] if _kernel_matches(n, kind)]
        w = [v for n, g, v in vals["write"] if _kernel_matches(n, kind)]
        if not f or not w:
            continue
        fk, wk = statistics.median(f), statistics.median(w)
        traffic = 1024.0 * (fk * factor["fetch"] + wk * factor["write"])
        out[kind] = traffic
        md.append(f"| {kind} | {len(f)} | {fk:.1f} | {wk:.1f} | {traffic:.4g} |")
        with open(os.path.join(ROOT, "profiles", f"counters_{kind}_{workload}.json"), "w") as fh:
            json.dump({"kind": kind, "workload": workload, "sources_sha256_16": kernel_sources_hash(),
                       "fetch_kib_median": fk, "write_kib_median": wk, "read_factor": factor["fetch"],
                       "write_factor": factor["write"], "traffic_bytes_per_launch": traffic,
                       "command": command}, fh, indent=1)
    md += ["", f"Kernel sources hash: {kernel_sources_hash()} (bench.py reports the traffic only while it matches)."]
    with open(os.path.join(ROOT, "profiles", f"counters_{workload}.md"), "w") as fh:
        fh.write("\n".join(md) + "\n")
    log(f"[bench] counters: {out}")


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="absorb2d", choices=["absorb2d", "plain2d"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="skip the block-shape autotuner")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (counter calibration)")
    ap.add_argument("--extra", default="broadband,harmonic3d,adjoint2d,density2d,paper",
                    help="comma-separated side workloads reported in the same line ('' for none)")
    ap.add_argument("--summarize-trace", metavar="DIR",
                    help="write a kernel-trace summary of a rocprofv3 CSV run (no GPU work)")
    ap.add_argument("--summarize-counters", metavar="DIR",
                    help="write traffic summaries of FETCH_SIZE/WRITE_SIZE runs (no GPU work)")
    ap.add_argument("--summary-out", default=None)
    ap.add_argument("--summary-command", default="")
    ap.add_argument("--summary-title", default="")
    args = ap.parse_args()
    if args.summarize_trace:
        summarize_trace(args.summarize_trace, args.summary_out, args.summary_command, args.summary_title)
        return
    if args.summarize_counters:
        summarize_counters(args.summarize_counters, args.workload, args.summary_command)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        log("bench.py measures one GPU: this build runs the hot path on a single MI355X "
            "(frequencies/sources would shard across GPUs with no communication); use --gpus 1")
        sys.exit(2)

    import torch
    import paper_2507_13754_amd as tbs

    dev = torch.device("cuda:0")
    log(f"[bench] building workload {args.workload}")
    case, desc = make_workload(args.workload)
    L = case.nterms
    B = case.sources.shape[0]
    k0 = tbs.background_k0(case.omega, case.c0, case.alpha0, case.y)
    c_dev = torch.from_numpy(case.c).to(dev)

    res = {}
    for name, dtype in (("c64", torch.complex64), ("c128", torch.complex128)):
        if name == "c128" and args.no_fp64:
            continue
        log(f"[bench] {name}: plan + tabulation")
        t0 = time.perf_counter()
        plan = tbs.Plan(case.grid, case.dx, k0, dtype=dtype, batch=B).tabulate()
        t_tab = time.perf_counter() - t0
        shapes = plan.autotune() if not args.no_tune else None
        V = plan.potential(c_dev, case.omega, case.c0, case.alpha0, case.y)
        s = torch.from_numpy(case.sources).to(dev, dtype)
        out = torch.empty((B,) + case.grid, dtype=dtype, device=dev)
        steps = args.steps if name == "c64" else max(3, args.steps // 2)
        ms_ev, ms_wall = time_solves(plan, s, V, L, out, steps, args.warmup)
        log(f"[bench] {name}: {ms_ev:.3f} ms/step (events), {ms_wall:.3f} ms/step (wall)")
        prof_steps = max(3, steps // 2)
        prof = profile_passes(plan, s, V, L, out, prof_steps)
        _, r = plan.solve(s, V, L, out=out, residual=True)
        res[name] = dict(plan=plan, out=out.clone(), ms=ms_ev, ms_wall=ms_wall, prof=prof,
                         t_tab=t_tab, steps=steps, prof_steps=prof_steps, resid=r, shapes=shapes)
        if args.calib_copy and name == "c64":
            a = torch.empty(256 * 1024 * 1024 // 4, dtype=torch.float32, device=dev).fill_(1.0)
            bb = torch.empty_like(a)
            for _ in range(3):
                bb.copy_(a)
            torch.cuda.synchronize()
            log("[bench] calibration copy of 256 MiB done (3 launches)")

    P = case.points
    r32 = res["c64"]
    plan32 = r32["plan"]
    N = (case.grid[-1], case.grid[-2], case.grid[-3] if len(case.grid) == 3 else 1)
    Mx, My, Mz = plan32.padded
    M = (Mx, My, Mz)
    ndim = len(case.grid)

    def roofline(rr, esz, kahan):
        ghat_bytes = (Mx // 2 + 1) * (My // 2 + 1) * ((Mz // 2 + 1) if ndim == 3 else 1) * esz
        kinds = {k: v for k, v in rr["prof"].items() if v[1] > 0}
        dom = max(kinds, key=lambda k: kinds[k][0])
        avg_ms = kinds[dom][0] / kinds[dom][1]
        nbytes = pass_bytes(dom, ndim, N, M, B, esz, kahan, ghat_bytes)
        ach = nbytes / (avg_ms * 1e-3) / 1e9
        passes = {k: {"avg_us": 1e3 * v[0] / v[1], "launches_per_step": v[1] / rr["prof_steps"],
                      "alg_bytes": pass_bytes(k, ndim, N, M, B, esz, kahan, ghat_bytes),
                      "GBps": pass_bytes(k, ndim, N, M, B, esz, kahan, ghat_bytes) / (v[0] / v[1] * 1e-3) / 1e9}
                  for k, v in kinds.items()}
        sb = step_bytes(ndim, N, M, B, esz, kahan, ghat_bytes, L)
        return dom, nbytes, avg_ms, ach, passes, sb

    dom, nbytes, avg_ms, ach, passes32, sb32 = roofline(r32, 8, True)
    traffic = read_counters(args.workload, dom)
    for k, v in passes32.items():
        v["alg_flops"] = pass_flops(k, ndim, N, M, B)
        v["TFLOPs"] = v["alg_flops"] / (v["avg_us"] * 1e-6) / 1e12
    # the column convolution is bound by vector ALU work, the row passes by HBM
    if dom == "col_conv":
        tf = passes32[dom]["TFLOPs"]
        roof = {"bound": "alu", "achieved": tf, "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": tf / VALU_PEAK_TFLOPS, "traffic": traffic, "kernel": dom,
                "alg_flops_per_launch": passes32[dom]["alg_flops"], "alg_bytes_per_launch": nbytes,
                "hbm_GBps": ach, "avg_launch_ms": avg_ms}
    else:
        roof = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": ach / HBM_PEAK_GBS, "traffic": traffic, "kernel": dom,
                "alg_bytes_per_launch": nbytes, "avg_launch_ms": avg_ms}
    value = P * L * B / (r32["ms"] * 1e-3)
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "grid-point·terms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "grid": list(case.grid), "padded": [Mx, My] + ([Mz] if ndim == 3 else []),
                   "nterms": L, "rhs": B, "dx_m": case.dx, "freq_hz": case.freq,
                   "plan_dtype": "complex64 + Kahan-compensated sum (compensation stored as bf16)"},
        "roofline": roof,
        "step_roofline": {"alg_bytes_per_step": sb32, "achieved_GBps": sb32 / (r32["ms"] * 1e-3) / 1e9,
                          "frac": sb32 / (r32["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                          "bytes_per_gpt": sb32 / (P * L * B)},
        "passes": passes32,
        "ms_per_step_wall": r32["ms_wall"],
        "tabulation_s": r32["t_tab"],
        "autotuned_block_shapes": r32["shapes"],
        "residual_last": float(np.max(r32["resid"][:, -1])),
    }
    if "c128" in res:
        r64 = res["c128"]
        p32 = r32["out"].cpu().numpy().astype(np.complex128)
        p64 = r64["out"].cpu().numpy()
        err = max(float(np.linalg.norm(p32[b] - p64[b]) / np.linalg.norm(p64[b])) for b in range(B))
        _, _, _, ach64, passes64, sb64 = roofline(r64, 16, False)
        line["fp64_plain"] = {"value": P * L * B / (r64["ms"] * 1e-3), "ms_per_step": r64["ms"],
                              "step_GBps": sb64 / (r64["ms"] * 1e-3) / 1e9,
                              "step_frac": sb64 / (r64["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                              "passes": passes64}
        line["speedup_fp32_vs_fp64"] = r64["ms"] / r32["ms"]
        line["rel_l2_fp32_vs_fp64"] = err
    if not args.no_cpu_baseline:
        log(f"[bench] CPU oracle baseline (~{args.cpu_seconds:.0f} s)")
        line["cpu_baseline"] = cpu_baseline(case, args.cpu_seconds)
    for r in res.values():
        r["plan"].close()
    del res
    torch.cuda.empty_cache()
    extras = [e for e in args.extra.split(",") if e]
    if extras:
        line["side_workloads"] = {}
    if "broadband" in extras:
        line["side_workloads"]["broadband"] = run_broadband(
            dev, max(2, args.steps // 5), 1, not args.no_fp64,
            0.0 if args.no_cpu_baseline else min(args.cpu_seconds, 10.0), not args.no_tune)
    if "harmonic3d" in extras:
        line["side_workloads"]["harmonic3d"] = run_harmonic3d(dev, max(2, args.steps // 4), 1, not args.no_fp64)
    if "adjoint2d" in extras:
        line["side_workloads"]["adjoint2d"] = run_adjoint2d(dev, 2, 1)
    if "density2d" in extras:
        line["side_workloads"]["density2d"] = run_density(dev, max(3, args.steps // 2), 1)
    if "paper" in extras:
        line["side_workloads"]["paper"] = {"c64": run_paper(dev)}
        if not args.no_fp64:
            line["side_workloads"]["paper"]["c128"] = run_paper(dev, fp64=True)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
