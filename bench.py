#!/usr/bin/env python3
"""Throughput of the Born-series hot path on one MI355X.

Headline workload: the batched broadband solve.  48 frequencies (2-8 MHz),
each on its own lambda/6 grid over 4 x 4 cm (312^2 ... 1247^2), 16 steering
angles per frequency, 25 terms, all grids in one batch replayed as one
recorded HIP graph.  One step = one full 25-term solve of every grid and
right-hand side, inputs resident in HBM.

value = physical grid points x summed terms x right-hand sides / step time
(grid-point.terms/s) of the FP32 (complex64, Kahan-compensated sum) batch;
the plain FP64 batch runs beside it on the same input, and the speedup is
stated with the FP32-vs-FP64 relative L2 error of the fields.

HBM bytes: the streaming-convolution model per summed term and right-hand
side, with M the smallest 5-smooth length >= 2N - 1 (padding beyond that
counts against the kernels):
  FP32 + compensation: 32 N_y M_x + 32 P + (8 P + 2 M_x M_y) / B
  FP64:                64 N_y M_x + 32 P + (16 P + 4 M_x M_y) / B
(the x-spectral intermediate read and written by the row and by the column
pass; the sum and its compensation read and written; the potential and the
folded spectrum shared by the B right-hand sides).  Per pass: row pass
16 N_y M_x + 32 P + 8 P / B (FP32), column convolution 16 N_y M_x +
2 M_x M_y / B; the first row pass reads the source (8 P) and writes the
intermediate, the last one reads it and updates the sum.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import platform
import re
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published
# FP32 vector peak of the code path: 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x
# 2.4 GHz.  The published 157.3 TFLOP/s counts packed (two-wide) FP32
# instructions, which these kernels are compiled without.
VALU_FP32_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
METRIC = "Born grid-point·terms/s + HBM GB/s frac, FP32 batched vs FP64 plain, 1 GPU"
UNIT = "grid-point·terms/s"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_sources_hash() -> str:
    h = hashlib.sha256()
    for f in ("tbs_passes.hpp", "tbs_fft.hpp", "tbs_internal.hpp"):
        with open(os.path.join(ROOT, "paper_2507_13754_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


# ------------------------------------------------------------------ bytes ---

def smooth5(n: int) -> int:
    """Smallest 5-smooth integer >= n."""
    m = max(1, n)
    while True:
        x = m
        for p in (2, 3, 5):
            while x % p == 0:
                x //= p
        if x == 1:
            return m
        m += 1


def min_padded(n: int) -> int:
    return smooth5(2 * n - 1)


def pass_bytes_2d(kind: str, nx: int, ny: int, B: int, fp64: bool, mx: int = 0, my: int = 0) -> float:
    """Algorithmic HBM bytes of one launch of a 2D pass over one grid with B
    right-hand sides (model in the module docstring; mx, my default to the
    smallest 5-smooth padded lengths)."""
    mx = mx or min_padded(nx)
    my = my or min_padded(ny)
    P = nx * ny
    esz = 16 if fp64 else 8
    X = ny * mx * esz                  # one sweep of the intermediate, one RHS
    acc = 2 * P * esz + (0 if fp64 else 2 * P * 8)   # sum r+w (+ compensation r+w at 8 B/pt per way)
    ghat = (mx // 2 + 1) * (my // 2 + 1) * esz
    if kind == "row_first":
        return B * (P * esz + X)
    if kind == "row_mid":
        return B * (2 * X + acc) + P * esz
    if kind == "row_last":
        return B * (X + acc)
    if kind == "col_conv":
        return B * 2 * X + ghat
    raise ValueError(kind)


def series_bytes_2d(nx, ny, B, L, fp64, mx=0, my=0) -> float:
    f = lambda k: pass_bytes_2d(k, nx, ny, B, fp64, mx, my)  # noqa: E731
    return f("row_first") + (L - 1) * f("row_mid") + f("row_last") + L * f("col_conv")


def pass_bytes_3d(kind: str, N, M, B: int, fp64: bool) -> float:
    """3D passes (x row pass, y forward, z convolution, y inverse)."""
    nx, ny, nz = N
    mx, my, mz = M
    P = nx * ny * nz
    esz = 16 if fp64 else 8
    A = B * ny * nz * mx * esz          # x-spectral intermediate
    Y = B * my * nz * mx * esz          # y-spectral intermediate
    acc = B * (2 * P * esz + (0 if fp64 else 2 * P * 8))
    if kind == "row_first":
        return B * P * esz + A
    if kind == "row_mid":
        return 2 * A + acc + P * esz
    if kind == "row_last":
        return A + acc
    if kind in ("col_fwd", "col_inv"):
        return A + Y
    if kind == "col_conv":
        return 2 * Y + (mx // 2 + 1) * (my // 2 + 1) * (mz // 2 + 1) * esz
    raise ValueError(kind)


VALU_PEAK_TFLOPS = 78.6   # non-packed FP32 FMA: 256 CU x 4 SIMD x 16 lanes x 2 x 2.4 GHz


def col_conv_flops_2d(nx, ny, B, M) -> float:
    """Radix-2 count (5 n log2 n per complex FFT, 6 per complex product) of
    one 2D column-convolution launch at the compiled length M (both axes)."""
    return float(B * M * (2 * 5.0 * M * math.log2(M) + 6 * M))


# ---------------------------------------------------------------- timing ---

def time_fn(fn, steps, warmup):
    """Event time of `steps` calls after `warmup` untimed ones, bracketed by
    device synchronisation; returns (ms per call, wall ms per call)."""
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


def rel_l2(a, b) -> float:
    """max over right-hand sides (leading axis) of ||a - b|| / ||b||."""
    a = np.asarray(a).astype(np.complex128)
    b = np.asarray(b).astype(np.complex128)
    return max(float(np.linalg.norm(a[k] - b[k]) / np.linalg.norm(b[k])) for k in range(a.shape[0]))


def cpu_info():
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return model, os.cpu_count(), usable


# ------------------------------------------------------- counter records ---

def read_counters(kernel_re: str):
    """HBM traffic per term of the kernel whose name matches kernel_re (all
    its dispatches of one term, every set of tiles), from the counter summary
    under profiles/ (two rocprofv3 --pmc runs, FETCH_SIZE then WRITE_SIZE,
    scaled by a plain copy's readings); None when the kernel sources or the
    batch schedule changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "counters_broadband.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("sources_sha256_16") != kernel_sources_hash():
        return None
    for name, v in d.get("kernels", {}).items():
        if re.search(kernel_re, name) and "traffic_bytes_per_term" in v:
            return v["traffic_bytes_per_term"]
    return None


# ------------------------------------------------------------- headline ---

def group_kernel_re(kind: str, M: int, shape: int) -> str:
    """Name pattern of the grouped kernel of a profile entry."""
    stem = "k_row_pass_group" if kind.startswith("row") else "k_col_pass_group"
    return rf"{stem}<float, {M}, \d+, {shape}, "


def group_kernel_name(e) -> str:
    stem = "k_row_pass_group" if e["kind"].startswith("row") else "k_col_pass_group"
    return f"{stem}<float, {e['length']}, ..., {e['shape']}, ...>"


def run_broadband(dev, steps: int, warmup: int, fp64: bool, tune: bool, counters_only: bool = False):
    """The headline: 48 frequencies on their own grids, 16 steering angles
    each, 25 terms, one batch replayed as one recorded graph."""
    import torch
    import workloads
    import paper_2507_13754_amd as tbs
    res = {}
    geo = []
    for name, dtype in (("c64", torch.complex64), ("c128", torch.complex128)):
        if name == "c128" and not fp64:
            continue
        plans, srcs, pots, gpts = [], [], [], 0
        t0 = time.perf_counter()
        for i in range(len(workloads.BROADBAND_FREQS)):
            c = workloads.broadband(i)
            k0 = tbs.background_k0(c.omega, c.c0, c.alpha0, c.y)
            p = tbs.Plan(c.grid, c.dx, k0, dtype=dtype, batch=c.sources.shape[0]).tabulate()
            plans.append(p)
            srcs.append(torch.from_numpy(c.sources).to(dev, dtype))
            pots.append(p.potential(torch.from_numpy(c.c).to(dev), c.omega, c.c0, c.alpha0, c.y))
            gpts += c.points * c.nterms * c.sources.shape[0]
            if name == "c64":
                geo.append((c.grid[1], c.grid[0], c.sources.shape[0], p.padded[0], p.padded[1]))
            L = c.nterms
            del c
        batch = tbs.Batch(plans)
        outs = [torch.empty((p.batch,) + p.shape, dtype=dtype, device=dev) for p in plans]
        if tune:
            batch.autotune(srcs, pots, outs)
        t_build = time.perf_counter() - t0
        log(f"[bench] broadband {name}: 48 plans built (tabulated{', batch tuned' if tune else ''}) "
            f"in {t_build:.1f} s")
        outs = batch.solve(srcs, pots, L, outs=outs)
        if counters_only:  # counter collection: two replays of the recorded graph, nothing else
            batch.solve(srcs, pots, L, outs=outs)
            torch.cuda.synchronize()
            batch.close()
            return None
        ms, wall = time_fn(lambda: batch.solve(srcs, pots, L, outs=outs), steps, warmup)
        log(f"[bench] broadband {name}: {ms:.2f} ms/step ({wall:.2f} wall)")
        fp = name == "c128"
        nbytes = sum(series_bytes_2d(nx, ny, B, L, fp) for nx, ny, B, _, _ in geo)
        nbytes_compiled = sum(series_bytes_2d(nx, ny, B, L, fp, mx, my) for nx, ny, B, mx, my in geo)
        r = {"ms": ms, "wall_ms": wall, "value": gpts / (ms * 1e-3), "bytes": nbytes,
             "bytes_compiled": nbytes_compiled, "gpts": gpts, "build_s": t_build}
        # per-launch event timing of the same series (no graph replay while
        # profiled), on a one-chain batch over the same plans and tuned shapes:
        # all tiles of a set in one launch, the launches one after the other,
        # so that each kernel's time is its own (the solve above runs the
        # set's tiles on several streams side by side)
        prev = os.environ.get("TBS_BATCH_CHAINS")
        os.environ["TBS_BATCH_CHAINS"] = "1"
        pbatch = tbs.Batch(plans)
        if prev is None:
            del os.environ["TBS_BATCH_CHAINS"]
        else:
            os.environ["TBS_BATCH_CHAINS"] = prev
        pbatch.profile(True)
        nprof = max(2, min(3, steps))
        for _ in range(nprof):
            pbatch.solve(srcs, pots, L, outs=outs)
        prof = pbatch.profile_read()
        pbatch.close()
        # one entry per kernel (pass kind, FFT length, lines per block): the
        # batch splits the grids of one length between its two launch chains,
        # i.e. two grouped launches of the same kernel per term
        agg = {}
        for e in prof:
            if e["launches"] == 0:
                continue
            a = agg.setdefault((e["kind"], e["length"], e["shape"]),
                               {"members": [], "member_rhs": [], "ms": 0.0, "launches": 0, "groups": 0})
            a["members"] += e["members"]
            a["member_rhs"] += e["member_rhs"]
            a["ms"] += e["ms"]
            a["launches"] += e["launches"]
            a["groups"] += 1
        entries = []
        for (kind, length, shape), e in agg.items():
            # a tile of r of a grid's B right-hand sides carries r / B of that
            # grid's algorithmic bytes (potential and spectrum once per grid)
            tiles = list(zip(e["members"], e["member_rhs"]))
            bl = sum(pass_bytes_2d(kind, geo[i][0], geo[i][1], geo[i][2], fp) * r / geo[i][2] for i, r in tiles)
            blc = sum(pass_bytes_2d(kind, geo[i][0], geo[i][1], geo[i][2], fp, geo[i][3], geo[i][4]) * r / geo[i][2]
                      for i, r in tiles)
            per_term = e["launches"] / e["groups"] / nprof         # launches of one group per step
            t_term = e["ms"] / nprof / per_term                   # all groups of this kernel, one term
            # column convolutions: radix-2 FLOP count at the smallest 5-smooth length
            fl = (sum(col_conv_flops_2d(geo[i][0], geo[i][1], r, min_padded(geo[i][0])) for i, r in tiles)
                  if kind == "col_conv" else 0.0)
            entries.append({"kind": kind, "length": length, "shape": shape, "grids": len(set(e["members"])),
                            "alg_flops_per_term": fl,
                            "tiles": len(tiles), "rhs": sum(r for _, r in tiles),
                            "launches_per_step": e["launches"] / nprof, "grouped_launches_per_term": e["groups"],
                            "avg_launch_ms": e["ms"] / e["launches"], "ms_per_term": t_term,
                            "ms_per_step": e["ms"] / nprof, "alg_bytes_per_term": bl,
                            "alg_bytes_per_term_at_compiled_length": blc,
                            "GBps": bl / (t_term * 1e-3) / 1e9})
        entries.sort(key=lambda x: -x["ms_per_step"])
        r["kernels"] = entries
        r["profiled_ms_per_step"] = sum(x["ms_per_step"] for x in entries)
        r["outs"] = [o.cpu() for o in outs]
        res[name] = r
        batch.close()
        for p in plans:
            p.close()
        del srcs, pots, outs
        torch.cuda.empty_cache()
    r32 = res["c64"]

    def roofline(k):
        """The kernel's roofline: HBM bytes for the row passes, FP32 VALU
        FLOPs for the column convolutions (issue-bound: two transforms per
        16 B of traffic per value; SQ counters in profiles/)."""
        desc = (f"{group_kernel_name(k)}: {k['kind']}, FFT length {k['length']}, {k['grids']} grids "
                f"({k['rhs']} RHS in {k['tiles']} tiles) in {k['grouped_launches_per_term']} grouped launches per term")
        common = {"kernel": desc, "ms_per_term": k["ms_per_term"], "avg_launch_ms": k["avg_launch_ms"],
                  "launches_per_step": k["launches_per_step"], "alg_bytes_per_term": k["alg_bytes_per_term"],
                  "traffic": read_counters(group_kernel_re(k["kind"], k["length"], k["shape"]))}
        if k["kind"] == "col_conv":
            a = k["alg_flops_per_term"] / (k["ms_per_term"] * 1e-3) / 1e12
            return {"bound": "alu", "achieved": a, "peak": VALU_FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": a / VALU_FP32_PEAK_TFLOPS, "alg_flops_per_term": k["alg_flops_per_term"],
                    "hbm_GBps": k["GBps"], **common}
        return {"bound": "hbm", "achieved": k["GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": k["GBps"] / HBM_PEAK_GBS, **common}

    dom = r32["kernels"][0]
    roof = roofline(dom)
    row_dom = next(k for k in r32["kernels"] if k["kind"].startswith("row"))
    r32["roofline_row_pass"] = roofline(row_dom)
    out = {"r32": r32, "roofline": roof, "L": L, "geo": geo}
    if "c128" in res:
        r64 = res["c128"]
        out["r64"] = r64
        errs = [rel_l2(a.numpy(), b.numpy()) for a, b in zip(r32["outs"], r64["outs"])]
        out["rel_l2_fp32_vs_fp64_max"] = max(errs)
        out["rel_l2_fp32_vs_fp64_per_grid"] = errs
    return out


def cpu_baseline_broadband(budget_s: float, gpu_outs32=None, gpu_outs64=None):
    """The FP64 oracle on the host's cores, on a bounded sample of the
    broadband batch: (a) a larger grid (frequency 40 of 48, 1107^2, all 16
    right-hand sides) for as many terms as fit the budget, timed; (b) the
    whole 25-term solve of the smallest grid, compared with the GPU fields."""
    import oracle
    import workloads
    model, ncpu, usable = cpu_info()
    c = workloads.broadband(40)
    k0 = oracle.background_k0(c.omega, c.c0, c.alpha0, c.y)
    V = oracle.potential(c.c, c.omega, c.c0, c.alpha0, c.y)
    G = oracle.GreenOperator(k0, c.dx, c.grid)
    t0 = time.perf_counter()
    G(c.sources)
    t_apply = time.perf_counter() - t0
    nterms = int(max(1, min(c.nterms, budget_s // max(t_apply, 1e-3))))
    t0 = time.perf_counter()
    oracle.born_series(G, c.sources, V, nterms)
    t = time.perf_counter() - t0
    gpt = c.points * nterms * c.sources.shape[0]
    out = {"value": gpt / t, "unit": UNIT, "cores": int(oracle.tbs_oracle.WORKERS), "kind": "oracle",
           "sample": f"broadband frequency 40 of 48 ({c.freq / 1e6:.3f} MHz, {c.grid[1]}x{c.grid[0]} grid, "
                     f"{c.sources.shape[0]} RHS): first {nterms} of {c.nterms} terms, FP64 numpy + scipy.fft "
                     f"({oracle.tbs_oracle.WORKERS} FFT threads), {t:.1f} s",
           "cpu_model": model, "host_cpus": ncpu, "usable_cpus": usable}
    if gpu_outs32 is not None:
        c0 = workloads.broadband(0)
        k00 = oracle.background_k0(c0.omega, c0.c0, c0.alpha0, c0.y)
        V0 = oracle.potential(c0.c, c0.omega, c0.c0, c0.alpha0, c0.y)
        t0 = time.perf_counter()
        p_ref, _ = oracle.solve(k00, c0.dx, c0.sources, V0, c0.nterms)
        t0 = time.perf_counter() - t0
        acc = {"grid": f"{c0.grid[1]}x{c0.grid[0]}, {c0.sources.shape[0]} RHS, {c0.nterms} terms",
               "oracle_s": t0, "fp32": rel_l2(gpu_outs32[0].numpy(), p_ref)}
        if gpu_outs64 is not None:
            acc["fp64"] = rel_l2(gpu_outs64[0].numpy(), p_ref)
        out["rel_l2_gpu_vs_oracle"] = acc
    return out


# ------------------------------------------------------- side workloads ---

def run_absorb2d(dev, steps: int, warmup: int, fp64: bool, tune: bool):
    """2048^2 at lambda/6 (5 MHz), 111-blob absorbing-dispersive medium, 30
    terms, one right-hand side: the FP32 plan and the plain FP64 plan, with
    per-pass event timing."""
    import torch
    import workloads
    import paper_2507_13754_amd as tbs
    case = workloads.absorb2d()
    L = case.nterms
    k0 = tbs.background_k0(case.omega, case.c0, case.alpha0, case.y)
    c_dev = torch.from_numpy(case.c).to(dev)
    out = {"workload": "absorb2d: 2048x2048 grid, dx=lambda/6 at 5 MHz, 111 Gaussian blobs c0 +-3%, "
                       "0.75 dB/(MHz^1.5 cm) y=1.5 with dispersion, 64-element line array, 30 terms, 1 RHS",
           "unit": UNIT}
    fields = {}
    nx, ny = case.grid[1], case.grid[0]
    for name, dtype in (("c64", torch.complex64), ("c128", torch.complex128)):
        if name == "c128" and not fp64:
            continue
        plan = tbs.Plan(case.grid, case.dx, k0, dtype=dtype).tabulate()
        shapes = plan.autotune() if tune else None
        V = plan.potential(c_dev, case.omega, case.c0, case.alpha0, case.y)
        s = torch.from_numpy(case.sources).to(dev, dtype)
        o = torch.empty((1,) + case.grid, dtype=dtype, device=dev)
        ms, _ = time_fn(lambda: plan.solve(s, V, L, out=o), steps, warmup)
        plan.profile(True)
        for _ in range(3):
            plan.solve(s, V, L, out=o)
        prof = plan.profile_read()
        plan.profile(False)
        fp = name == "c128"
        passes = {}
        M = plan.padded[0]
        for k, (tms, cnt) in prof.items():
            if cnt == 0:
                continue
            b = pass_bytes_2d(k, nx, ny, 1, fp)
            passes[k] = {"avg_us": 1e3 * tms / cnt, "alg_bytes": b, "GBps": b / (tms / cnt * 1e-3) / 1e9}
        passes["col_conv"]["TFLOPs_alg"] = col_conv_flops_2d(nx, ny, 1, M) / (passes["col_conv"]["avg_us"] * 1e-6) / 1e12
        sb = series_bytes_2d(nx, ny, 1, L, fp)
        e = {"ms_per_step": ms, "value": case.points * L / (ms * 1e-3),
             "step_GBps": sb / (ms * 1e-3) / 1e9, "frac": sb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
             "passes": passes, "autotuned_block_shapes": shapes}
        log(f"[bench] absorb2d {name}: {ms:.3f} ms/step")
        if name == "c64":
            out.update(e)
        else:
            out["fp64_plain"] = e
        fields[name] = o.cpu().numpy()
        plan.close()
        del s, V, o
        torch.cuda.empty_cache()
    if "c128" in fields:
        out["rel_l2_fp32_vs_fp64"] = rel_l2(fields["c64"], fields["c128"])
        out["speedup_fp32_vs_fp64"] = out["fp64_plain"]["ms_per_step"] / out["ms_per_step"]
    return out


def run_harmonic3d(dev, steps: int, warmup: int, fp64: bool, tune: bool):
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
                       "fundamental 24 terms + second harmonic (6 MHz) 24 terms", "unit": UNIT}
    outs = {}
    N = (c.grid[2], c.grid[1], c.grid[0])
    for name, dtype in (("c64", torch.complex64), ("c128", torch.complex128)):
        if name == "c128" and not fp64:
            continue
        p1 = tbs.Plan(c.grid, c.dx, tbs.background_k0(om, c.c0, c.alpha0, c.y), dtype=dtype).tabulate()
        p2 = tbs.Plan(c.grid, c.dx, tbs.background_k0(2 * om, c.c0, c.alpha0, c.y), dtype=dtype).tabulate()
        shapes = [p1.autotune()[1], p2.autotune()[1]] if tune else None  # z lines per block
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

        ms, _ = time_fn(step, steps, warmup)
        fp = name == "c128"
        M = tuple(p1.padded)
        per = lambda k: pass_bytes_3d(k, N, M, 1, fp)  # noqa: E731
        L = c.nterms
        nb = 2 * (per("row_first") + (L - 1) * per("row_mid") + per("row_last")
                  + L * (per("col_fwd") + per("col_conv") + per("col_inv")))
        gpt = 2 * c.points * c.nterms
        log(f"[bench] harmonic3d {name}: {ms:.2f} ms/step")
        outs[name] = (f1.cpu().numpy(), f2.cpu().numpy())
        entry = {"value": gpt / (ms * 1e-3), "ms_per_step": ms, "alg_bytes_per_step": nb,
                 "achieved_GBps": nb / (ms * 1e-3) / 1e9, "frac": nb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                 "autotuned_z_lines_per_block": shapes}
        if name == "c64":
            res.update(entry)
        else:
            res["fp64_plain"] = entry
        p1.close()
        p2.close()
        del s, f1, S2, f2
        torch.cuda.empty_cache()
    if "c128" in outs:
        for k, nm in ((0, "fundamental"), (1, "harmonic")):
            res[f"rel_l2_fp32_vs_fp64_{nm}"] = rel_l2(outs["c64"][k], outs["c128"][k])
        res["speedup_fp32_vs_fp64"] = res["fp64_plain"]["ms_per_step"] / res["ms_per_step"]
    return res


def run_density(dev, steps: int, warmup: int, fp64: bool):
    """absorb2d (2048^2, 30 terms) with a density contrast: the blob map of
    the medium: gamma_rho = |c / c0 - 1| (up to 3 %).  Per term the
    field is kept in space between two row passes (u written and read, gamma
    read: + 24 B per grid-point.term over the plain FP32 series)."""
    import torch
    import workloads
    import paper_2507_13754_amd as tbs
    case = workloads.absorb2d()
    gam = torch.from_numpy(np.abs(case.c / case.c0 - 1.0)).to(dev)
    nx, ny = case.grid[1], case.grid[0]
    res = {"workload": "absorb2d (2048^2, 30 terms) with a density contrast gamma_rho = |c/c0 - 1|",
           "unit": UNIT}
    fields = {}
    for name, dtype in (("c64", torch.complex64), ("c128", torch.complex128)):
        if name == "c128" and not fp64:
            continue
        plan = tbs.Plan(case.grid, case.dx, tbs.background_k0(case.omega, case.c0, case.alpha0, case.y),
                        dtype=dtype).tabulate()
        plan.density_contrast(gam)
        V = plan.potential(torch.from_numpy(case.c).to(dev), case.omega, case.c0, case.alpha0, case.y)
        s = torch.from_numpy(case.sources).to(dev, dtype)
        o = torch.empty_like(s)
        ms, _ = time_fn(lambda: plan.solve(s, V, case.nterms, out=o), steps, warmup)
        plan.close()
        gpt = case.points * case.nterms
        nb = series_bytes_2d(nx, ny, 1, case.nterms, name == "c128") + \
            (case.nterms - 1) * case.points * (2 * (16 if name == "c128" else 8) + 8)
        log(f"[bench] density2d {name}: {ms:.3f} ms/step")
        e = {"ms_per_step": ms, "value": gpt / (ms * 1e-3), "alg_bytes_per_step": nb,
             "achieved_GBps": nb / (ms * 1e-3) / 1e9, "frac": nb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
        if name == "c64":
            res.update(e)
        else:
            res["fp64_plain"] = e
        fields[name] = o.cpu().numpy()
        del s, V, o
        torch.cuda.empty_cache()
    if "c128" in fields:
        res["rel_l2_fp32_vs_fp64"] = rel_l2(fields["c64"], fields["c128"])
        res["speedup_fp32_vs_fp64"] = res["fp64_plain"]["ms_per_step"] / res["ms_per_step"]
    return res


def run_adjoint2d(dev, steps: int, warmup: int, fp64: bool):
    """One misfit gradient: 1024^2, 16 frequencies (2-6 MHz) x 8 sources, 128
    receivers, 25 terms, FP32 through torch.autograd with term recomputation
    (checkpoints every ceil(sqrt(2L)) terms instead of all partial sums); the
    FP64 gradient (stored partial sums) beside it for the accuracy."""
    import torch
    import workloads
    import paper_2507_13754_amd as tbs
    from paper_2507_13754_amd.autograd import MisfitProblem, TBSMisfit
    prob = workloads.adjoint2d()
    n = prob.grid[0]
    rec = torch.from_numpy(prob.receivers[:, 0] * n + prob.receivers[:, 1]).to(dev)
    ct = torch.from_numpy(prob.c_true).to(dev)
    c = torch.from_numpy(prob.c_model).to(dev)
    res = {"workload": "adjoint2d: 1024^2, 16 frequencies 2-6 MHz x 8 sources, 128 receivers, 25 terms, "
                       "misfit gradient via torch.autograd (forward, forward replay with checkpoints, adjoint)",
           "unit": "grid-point·terms/s (3 series per (f, s))"}
    grads = {}
    for name, dtype, flags in (("c64", torch.complex64, tbs.TBS_ADJ_RECOMPUTE),
                               ("c128", torch.complex128, tbs.TBS_ADJ_STORE)):
        if name == "c128" and not fp64:
            continue
        src = torch.from_numpy(prob.sources).to(dev, dtype)
        p_obs = []
        for f in prob.freqs:
            om = 2 * math.pi * f
            pl = tbs.Plan(prob.grid, prob.dx, tbs.background_k0(om, workloads.C0, prob.alpha0, prob.y),
                          dtype=dtype, batch=src.shape[0]).tabulate()
            p = pl.solve(src, pl.potential(ct, om, workloads.C0, prob.alpha0, prob.y), prob.nterms)
            p_obs.append(p[:, prob.receivers[:, 0], prob.receivers[:, 1]].contiguous())
            pl.close()
        mp = MisfitProblem(prob.grid, prob.dx, prob.freqs, workloads.C0, prob.alpha0, prob.y, src, rec,
                           p_obs, prob.nterms, dtype=dtype, adjoint_flags=flags)

        def step():
            cc = c.clone().requires_grad_(True)
            TBSMisfit.apply(cc, mp).backward()
            return cc.grad

        ms, _ = time_fn(step, steps if name == "c64" else 1, warmup if name == "c64" else 0)
        grads[name] = step().cpu().numpy()
        dev_bytes = max(p.device_bytes for p in mp.plans)
        nsrc = src.shape[0]
        gpt = 3 * n * n * prob.nterms * nsrc * len(prob.freqs)
        log(f"[bench] adjoint2d {name}: {ms:.1f} ms per gradient")
        e = {"ms_per_gradient": ms, "value": gpt / (ms * 1e-3),
             "adjoint_mode": "recompute" if flags == tbs.TBS_ADJ_RECOMPUTE else "store",
             "plan_device_bytes_max": dev_bytes}
        if name == "c64":
            res.update(e)
        else:
            res["fp64_plain"] = e
        mp.close()
        del src, p_obs
        torch.cuda.empty_cache()
    if "c128" in grads:
        g32, g64 = grads["c64"], grads["c128"]
        res["rel_l2_grad_fp32_vs_fp64"] = float(np.linalg.norm(g32 - g64) / np.linalg.norm(g64))
        res["max_err_grad_fp32_vs_fp64_over_max"] = float(np.max(np.abs(g32 - g64)) / np.max(np.abs(g64)))
    return res


# the paper's Table 3 (iterations, seconds on its RTX 4060), context only
PAPER_TABLE3 = {
    "homogeneous": (135, 5.0), "absorbing": (133, 8.0), "absorbing-dispersive": (132, 11.0),
    "inhomogeneous vs=1350": (134, 7.0), "inhomogeneous vs=1650": (134, 7.0),
    "inhomogeneous vs=1800": (134, 7.0), "harmonic 2": (228, 9.0), "harmonic 3": (306, 12.0),
    "harmonic 4": (368, 15.0), "harmonic 5": (416, 16.0),
}


def run_paper(dev, n: int, fp64: bool):
    """The paper's own periodic scheme on its 4096^2 setups (Sec. 3.1,
    Algorithm 1): the linear media of Table 3 and the nonlinear chain up to
    the 5th harmonic (B/A = 5), each iterated to the paper's tolerance 1e-5,
    in FP32 and in FP64; the FP32 fields are compared with the FP64 ones.
    Time = the whole tbs_iterate call (spectrum tabulated before), wall clock
    after a device sync; alg. bytes per iteration: row pass 40 B/pt (X r+w,
    psi0, psi, V) + column pass 16 B/pt + the folded spectrum (FP32)."""
    import torch
    import workloads
    import paper_2507_13754_amd as tbs
    out = {}
    fields = {}

    def iterate(case, k, eps, src, vv, V, dtype):
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

    for name, dtype in (("c64", torch.complex64), ("c128", torch.complex128)):
        if name == "c128" and not fp64:
            continue
        esz = 16 if name == "c128" else 8
        rec = {}

        def record(label, it, sec, with_v):
            per_pt = (5 if with_v else 4) * esz + 2 * esz + esz * (n // 2 + 1) ** 2 / n ** 2
            ref = PAPER_TABLE3.get(label)
            rec[label] = {"iterations": it, "seconds": sec, "ms_per_iteration": 1e3 * sec / max(it, 1),
                          "alg_GBps": per_pt * n * n * it / sec / 1e9,
                          "paper_iterations": ref[0] if ref else None,
                          "paper_seconds_rtx4060": ref[1] if ref else None}
            log(f"[bench] paper {name} {label}: {it} iterations, {sec * 1e3:.1f} ms")

        media = [("homogeneous", "homogeneous", 1650.0), ("absorbing", "absorbing", 1650.0),
                 ("absorbing-dispersive", "absorbing-dispersive", 1650.0)]
        media += [(f"inhomogeneous vs={vs:.0f}", "inhomogeneous", vs) for vs in (1350.0, 1650.0, 1800.0)]
        for label, kind, vs in media:
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
            psi, it, sec = iterate(case, k, eps, src, vv, V, dtype)
            record(label, it, sec, V is not None)
            fields[(name, label)] = psi.cpu().numpy()
            del psi, src, V
        # nonlinear: fundamental, then harmonics 2..5 from the sum-frequency
        # sources; field h is kept as psi_h 2^e_h (the 5th harmonic is about
        # 1e-39 here, below the FP32 range), the source of order h scaled so
        # that its largest part lies in [1, 2)
        case = workloads.paper_periodic("homogeneous", n)
        c_map = torch.from_numpy(case.c).to(dev)
        chain, exps = [], []
        for h in range(1, 6):
            k = h * case.omega / case.c0
            eps = case.eps_factor * k * k
            aux = tbs.Plan((n, n), case.dx, k, padding=1, dtype=dtype)
            V = aux.potential(c_map, h * case.omega, case.c0, 0.0, 1.0, eps)
            if h == 1:
                src, e = torch.from_numpy(case.sources).to(dev, dtype), 0
            else:
                src, e = aux.harmonic_source_scaled(h, chain, exps, c_map, case.omega, 1000.0, 5.0)
            aux.close()
            psi, it, sec = iterate(case, k, eps, src, None, V, dtype)
            if h > 1:
                record(f"harmonic {h}", it, sec, True)
                rec[f"harmonic {h}"]["scale_exponent"] = e
                fields[(name, f"harmonic {h}")] = psi.cpu().numpy().astype(np.complex128) * 2.0 ** (-e)
            chain.append(psi)
            exps.append(e)
            del V, src
        del chain
        torch.cuda.empty_cache()
        total = sum(v["seconds"] for v in rec.values())
        out[name] = {"media": rec, "total_seconds": total,
                     "paper_total_seconds_rtx4060": sum(v["paper_seconds_rtx4060"] for v in rec.values())}
    if "c128" in out:
        for label in out["c64"]["media"]:
            out["c64"]["media"][label]["rel_l2_vs_fp64"] = rel_l2(fields[("c64", label)], fields[("c128", label)])
    out["workload"] = (f"paper periodic scheme, {n}^2, dx = 20 um, 1007080 Hz, eps = 0.8 k^2, 501-element line, "
                       "sigmoid layer, tol 1e-5 (Sec. 3.1, Algorithm 1, Table 3)")
    return out


# ------------------------------------------------------------------------------
# rocprofv3 summaries (text under profiles/): a --kernel-trace --stats run, or
# two --pmc runs (FETCH_SIZE, WRITE_SIZE) of this script with --calib-copy.

def _csv(path):
    import csv
    with open(path, newline="") as fh:
        return list(csv.DictReader(fh))


def summarize_trace(src: str, out: str, command: str, title: str, skip_before: str = ""):
    """Per-kernel durations from <src>/run_kernel_trace.csv into a markdown
    table (dispatches before the first kernel whose name contains skip_before
    are left out: autotuning and warm-up of other workloads)."""
    rows = _csv(os.path.join(src, "run_kernel_trace.csv"))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    if skip_before:
        first = next((i for i, r in enumerate(rows) if skip_before in r["Kernel_Name"]), 0)
        rows = rows[first:]
    agg = {}
    for r in rows:
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        a = agg.setdefault(r["Kernel_Name"], dict(n=0, tot=0.0, mn=1e30, mx=0.0, lds=r.get("LDS_Block_Size", ""),
                                                  vgpr=r.get("VGPR_Count", ""), scr=r.get("Scratch_Size", ""),
                                                  block=r.get("Workgroup_Size_X", "")))
        a["n"] += 1
        a["tot"] += d
        a["mn"] = min(a["mn"], d)
        a["mx"] = max(a["mx"], d)
    lines = [f"# rocprofv3 kernel trace: {title}", "", "Command (repository root as working directory):", "",
             "    " + command, "",
             "Per-kernel durations (us) from the kernel trace of that run"
             + (f", from the first `{skip_before}` dispatch on." if skip_before else "."), "",
             "| kernel | calls | total us | avg us | min us | max us | LDS B | VGPR | scratch | block |",
             "|---|---|---|---|---|---|---|---|---|---|"]
    for k, a in sorted(agg.items(), key=lambda kv: -kv[1]["tot"]):
        lines.append(f"| `{k}` | {a['n']} | {a['tot']:.1f} | {a['tot'] / a['n']:.2f} | {a['mn']:.2f} | "
                     f"{a['mx']:.2f} | {a['lds']} | {a['vgpr']} | {a['scr']} | {a['block']} |")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    log(f"[bench] wrote {out}")


def summarize_counters(src: str, command: str, nplans: int = 48, nterms: int = 25):
    """FETCH_SIZE / WRITE_SIZE (KiB) of every grouped pass kernel from
    <src>/fetch and <src>/write, scaled by what the same counters read for the
    256 MiB calibration copy, per term: summed over all dispatches of the
    kernel and divided by the solves of the run (one norm reduction per plan
    and solve) times the passes per solve (nterms column passes, nterms + 1
    row passes: first, middle and last averaged).  Into
    profiles/counters_broadband.json (+ .md).  Run with the block shapes taken
    from a TBS_TUNE_CACHE file, so that no tuning launches are counted."""
    vals = {}
    for kind, ctr in (("fetch", "FETCH_SIZE"), ("write", "WRITE_SIZE")):
        for r in _csv(os.path.join(src, kind, "run_counter_collection.csv")):
            if r["Counter_Name"] == ctr:
                vals.setdefault(kind, []).append((r["Kernel_Name"], float(r["Counter_Value"])))
    calib = 256 * 1024  # KiB read and written by the calibration copy
    factor = {}
    for kind in ("fetch", "write"):
        copies = [v for n, v in vals[kind] if "copyBuffer" in n]
        big = max(copies)
        factor[kind] = calib / statistics.median([v for v in copies if v > 0.4 * big])
    solves = {k: sum(1 for n, _ in vals[k] if "k_finish_norms" in n) / nplans for k in vals}
    names = sorted({n for n, _ in vals["fetch"] if "_pass_group<" in n})
    kernels = {}
    md = ["# HBM traffic counters: broadband batch (48 grids x 16 RHS, 25 terms)", "",
          "Commands (repository root as working directory):", "", "    " + command, "",
          "FETCH_SIZE and WRITE_SIZE in KiB summed over every dispatch of each kernel (all sets of",
          f"tiles), per term: divided by the {solves['fetch']:.0f} solves of the run times {nterms} column passes",
          f"or {nterms + 1} row passes per solve (first, middle and last row passes averaged); scaled by the",
          f"256 MiB calibration copy: read factor {factor['fetch']:.3f}, write factor {factor['write']:.3f}.", "",
          "| kernel | dispatches | FETCH KiB / term | WRITE KiB / term | scaled bytes / term |", "|---|---|---|---|---|"]
    for n in names:
        f = [v for k, v in vals["fetch"] if k == n]
        w = [v for k, v in vals["write"] if k == n]
        if not f or not w:
            continue
        per = (nterms if "k_col_pass" in n else nterms + 1)
        fk = sum(f) / (solves["fetch"] * per)
        wk = sum(w) / (solves["write"] * per)
        traffic = 1024.0 * (fk * factor["fetch"] + wk * factor["write"])
        kernels[n] = {"dispatches": len(f), "fetch_kib_per_term": fk, "write_kib_per_term": wk,
                      "traffic_bytes_per_term": traffic}
        md.append(f"| `{n}` | {len(f)} | {fk:.1f} | {wk:.1f} | {traffic:.4g} |")
    with open(os.path.join(ROOT, "profiles", "counters_broadband.json"), "w") as fh:
        json.dump({"workload": "broadband", "sources_sha256_16": kernel_sources_hash(),
                   "read_factor": factor["fetch"], "write_factor": factor["write"], "solves": solves,
                   "kernels": kernels, "command": command}, fh, indent=1)
    md += ["", f"Kernel sources hash: {kernel_sources_hash()} (bench.py reports the traffic only while it matches)."]
    with open(os.path.join(ROOT, "profiles", "counters_broadband.md"), "w") as fh:
        fh.write("\n".join(md) + "\n")
    log(f"[bench] counters of {len(kernels)} kernels written")


# ------------------------------------------------------------------ main ---

def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="skip the block-shape autotuner")
    ap.add_argument("--counters-only", action="store_true",
                    help="build the FP32 broadband batch, replay it twice and exit (for --pmc runs; "
                         "with --calib-copy, the calibration copy after it)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (counter calibration)")
    ap.add_argument("--extra", default="absorb2d,harmonic3d,adjoint2d,density2d,paper",
                    help="comma-separated side workloads reported in the same line ('' for none)")
    ap.add_argument("--paper-n", type=int, default=4096)
    ap.add_argument("--summarize-trace", metavar="DIR",
                    help="write a kernel-trace summary of a rocprofv3 CSV run (no GPU work)")
    ap.add_argument("--summarize-counters", metavar="DIR",
                    help="write traffic summaries of FETCH_SIZE/WRITE_SIZE runs (no GPU work)")
    ap.add_argument("--summary-out", default=None)
    ap.add_argument("--summary-command", default="")
    ap.add_argument("--summary-title", default="")
    ap.add_argument("--summary-skip-before", default="")
    args = ap.parse_args()
    if args.summarize_trace:
        summarize_trace(args.summarize_trace, args.summary_out, args.summary_command, args.summary_title,
                        args.summary_skip_before)
        return
    if args.summarize_counters:
        summarize_counters(args.summarize_counters, args.summary_command)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        log("bench.py measures one GPU: this build runs the hot path on a single MI355X "
            "(frequencies and sources would shard across GPUs with no communication); use --gpus 1")
        sys.exit(2)

    import torch
    dev = torch.device("cuda:0")
    fp64 = not args.no_fp64
    tune = not args.no_tune
    bb = run_broadband(dev, args.steps, args.warmup, fp64 and not args.counters_only, tune, args.counters_only)
    if args.calib_copy:
        a = torch.empty(256 * 1024 * 1024 // 4, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        log("[bench] calibration copy of 256 MiB done (3 launches)")
    if args.counters_only:
        return
    r32 = bb["r32"]
    L = bb["L"]
    B = bb["geo"][0][2]
    lengths = sorted({g[3] for g in bb["geo"]})
    line = {
        "metric": METRIC,
        "value": r32["value"],
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "broadband: 48 frequencies 2-8 MHz (f_i = 2 + 6 i/47 MHz), each on its own "
                               "lambda/6 grid over 4 x 4 cm (312^2 .. 1247^2), 16-blob absorbing-dispersive "
                               "medium, 64-element array with 16 steering angles (-30..30 deg) per frequency, "
                               "25 terms, one batch (right-hand sides in tiles of 2, cache-sized sets run one "
                               "after another, the tiles of a set on three streams) replayed as one recorded "
                               "HIP graph",
                   "grids": len(bb["geo"]), "rhs_per_grid": B, "nterms": L,
                   "physical_points": int(sum(g[0] * g[1] for g in bb["geo"])),
                   "padded_lengths": lengths,
                   "plan_dtype": "complex64 + Kahan-compensated sum (compensation stored as bf16)"},
        "roofline": bb["roofline"],
        "roofline_row_pass": r32["roofline_row_pass"],
        "step_roofline": {"alg_bytes_per_step": r32["bytes"],
                          "achieved_GBps": r32["bytes"] / (r32["ms"] * 1e-3) / 1e9,
                          "frac": r32["bytes"] / (r32["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                          "bytes_per_gpt": r32["bytes"] / r32["gpts"],
                          "alg_bytes_per_step_at_compiled_lengths": r32["bytes_compiled"]},
        "kernels": r32["kernels"],
        "profiled_ms_per_step": r32["profiled_ms_per_step"],
        "ms_per_step_wall": r32["wall_ms"],
        "plan_build_s": r32["build_s"],
    }
    if "r64" in bb:
        r64 = bb["r64"]
        line["fp64_plain"] = {"value": r64["value"], "ms_per_step": r64["ms"],
                              "step_GBps": r64["bytes"] / (r64["ms"] * 1e-3) / 1e9,
                              "frac": r64["bytes"] / (r64["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                              "kernels": r64["kernels"][:4]}
        line["speedup_fp32_vs_fp64"] = r64["ms"] / r32["ms"]
        line["rel_l2_fp32_vs_fp64"] = bb["rel_l2_fp32_vs_fp64_max"]
    if not args.no_cpu_baseline:
        log(f"[bench] CPU oracle baseline (~{args.cpu_seconds:.0f} s + the smallest grid's full solve)")
        line["cpu_baseline"] = cpu_baseline_broadband(args.cpu_seconds, r32["outs"],
                                                      bb["r64"]["outs"] if "r64" in bb else None)
    del bb
    torch.cuda.empty_cache()
    extras = [e for e in args.extra.split(",") if e]
    if extras:
        line["side_workloads"] = {}
    sw = line.get("side_workloads", {})
    if "absorb2d" in extras:
        sw["absorb2d"] = run_absorb2d(dev, max(10, args.steps), args.warmup, fp64, tune)
    if "harmonic3d" in extras:
        sw["harmonic3d"] = run_harmonic3d(dev, max(2, args.steps // 4), 1, fp64, tune)
    if "adjoint2d" in extras:
        sw["adjoint2d"] = run_adjoint2d(dev, 2, 1, fp64)
    if "density2d" in extras:
        sw["density2d"] = run_density(dev, max(3, args.steps // 2), 1, fp64)
    if "paper" in extras:
        sw["paper"] = run_paper(dev, args.paper_n, fp64)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
