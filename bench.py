#!/usr/bin/env python3
"""Throughput of the semi-implicit PIC hot path on one MI355X.

Metric: particle-steps/s of gather + alpha_p + J-hat/M deposit + push (with
the per-step re-sort), on the 2D double Harris sheet 1024 x 512 cells, 64
particles per cell per species (67,108,864 particles), FP32-mixed (headline)
and FP64.  Every timed step is a full step of the scheme: deposit, FP64 GMRES
field solve (relative tolerance 1e-10), push + re-sort, FP64 energy.  The
metric's time is the GPU time of the deposit and push calls (HIP events on
the stream the library launches on); the field solve and the energy
diagnostic are timed and reported separately.  Inputs are generated on the host, copied to HBM,
and are resident before the timed region starts.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
One JSON line is printed on stdout.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_bytes(name, wl, prec, n, nbins, ncells):
    """Algorithmic bytes of one launch of a kernel: what it must read and
    write at least once (particle state, grid fields, per-cell moments)."""
    T = 4 if prec == "mixed" else 8
    d = wl.dim
    noff = 27 if d == 3 else 9
    grid = 24  # one FP64 3-vector per node or cell
    if name == "deposit_cells":
        # in: particle state (offsets, momentum, weight) + B^n; out: the
        # per-cell moments (81 + 12 per cell in 2D, 243 + 24 in 3D)
        nmom = 93 if d == 2 else 267
        return n * (d + 4) * T + ncells * grid + ncells * nmom * T
    if name == "assemble_nodes":
        # in: per-cell moments; out: J-hat and M at nodes (FP64)
        nmom = 93 if d == 2 else 267
        return ncells * nmom * T + ncells * (grid + 8 * 9 * noff)
    if name == "push_count":
        # first pass of push + re-sort: in: offsets + (momentum, weight)
        # records, E_theta, B^n; out: 1-byte move code (+ per-bin counts)
        return n * ((d + 4) * T + 1) + 2 * ncells * grid
    if name == "push_scatter":
        # second pass: in: the records, move codes, E_theta, B^n; out: the
        # pushed records in the new order
        return n * (2 * (d + 4) * T + 1) + 2 * ncells * grid
    if name == "push":
        # push in place without re-sort: in and out the records
        return n * 2 * (d + 4) * T + 2 * ncells * grid
    return None


# library timing names -> HIP kernel symbols (for the committed counter summaries)
KERNEL_SYMBOL = {"deposit_cells": "k_deposit_cells", "assemble_nodes": "k_assemble", "push_count": "k_push",
                 "push_scatter": "k_push_scatter", "sort_offsets": "k_sort_offsets"}


def device_code_sha256(lib_path=None):
    """sha256 of the GPU code objects built into the library (its
    .hip_fatbin ELF section): identifies the kernels that ran, and does not
    change with edits that leave the compiled kernels alone."""
    import hashlib
    import struct

    if lib_path is None:
        lib_path = os.path.join(ROOT, "paper_2509_11100_amd", "librelsim.so")
    data = open(lib_path, "rb").read()
    shoff = struct.unpack_from("<Q", data, 0x28)[0]
    shentsize, shnum, shstrndx = struct.unpack_from("<HHH", data, 0x3A)

    def section(i):
        name, _, _, _, off, size = struct.unpack_from("<IIQQQQ", data, shoff + i * shentsize)
        return name, off, size

    _, stroff, _ = section(shstrndx)
    for i in range(shnum):
        name, off, size = section(i)
        end = data.index(b"\0", stroff + name)
        if data[stroff + name:end] == b".hip_fatbin":
            return hashlib.sha256(data[off:off + size]).hexdigest()
    return None


def measured_traffic(tag, kernel):
    """HBM bytes per dispatch from the committed rocprofv3 counter summary,
    or None when the kernels changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % tag)
    if not os.path.exists(path):
        return None
    js = json.load(open(path))
    code = device_code_sha256()
    if code is None or js.get("device_code_sha256") != code:
        return None
    k = js["kernels"].get(KERNEL_SYMBOL.get(kernel, kernel))
    return None if k is None else k["hbm_bytes"]


def run_energy_conserving(prec, wl, host, steps, warmup, rtol, group=0):
    """Whole energy-conserving steps (relsim.Step(energy_conserving=True):
    fixed-point passes of deposit, solve and relsim_gamma_mean, then the
    push) on the same workload: wall time per step, passes per step and the
    relative energy change over the timed steps.  Not the headline metric."""
    import numpy as np
    import torch

    from paper_2509_11100_amd import relsim

    n = host["w"].shape[0]
    ctx = relsim.Context(dim=wl.dim, nx=wl.nx, ny=wl.ny, nz=wl.nz if wl.dim == 3 else 1, dx=wl.dx, dt=wl.dt,
                         precision=prec, q=wl.q, m=wl.m, max_particles=n, gmres_rtol=rtol, gmres_restart=30,
                         gmres_maxit=5000, group=group)
    parts = relsim.Particles(ctx).load(host["cell"], host["species"], host["off"], host["u"], host["w"],
                                       host["bin_start"])
    step = relsim.Step(ctx, parts, torch.as_tensor(host["E"]).cuda(), torch.as_tensor(host["B"]).cuda(),
                       energy_conserving=True)
    step(warmup)
    W0 = step.energy()
    passes = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
        passes.append(step.picard_iters)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    W1 = step.energy()
    del step, parts, ctx
    torch.cuda.empty_cache()
    return {"precision": prec, "particle_steps_per_s": n * steps / wall, "ms_per_step": 1e3 * wall / steps,
            "picard_tol": 1e-12 if prec == "fp64" else 1e-6, "passes_per_step": float(np.mean(passes)),
            "rel_energy_change": float(abs(W1[3] - W0[3]) / W0[3])}


def run_precision(prec, wl, host, steps, warmup, rtol, want_kernels=True, group=0):
    import numpy as np
    import torch

    from paper_2509_11100_amd import relsim

    n = host["w"].shape[0]
    ctx = relsim.Context(dim=wl.dim, nx=wl.nx, ny=wl.ny, nz=wl.nz if wl.dim == 3 else 1, dx=wl.dx, dt=wl.dt,
                         precision=prec, q=wl.q, m=wl.m, max_particles=n, gmres_rtol=rtol, gmres_restart=30,
                         gmres_maxit=5000, group=group)
    parts = relsim.Particles(ctx).load(host["cell"], host["species"], host["off"], host["u"], host["w"],
                                       host["bin_start"])
    E = torch.as_tensor(host["E"]).cuda()
    B = torch.as_tensor(host["B"]).cuda()
    nb = [ctx.grid(), ctx.grid()]
    Eth = ctx.grid()
    J = ctx.grid()
    M = ctx.mass_matrix()
    W0 = relsim.energy(ctx, parts, E, B)
    st = torch.cuda.current_stream()

    def one_step(E, B, E1, B1, ev=None):
        if ev is not None:
            ev[0].record(st)
        relsim.timing_enable(ctx, ev is not None and want_kernels)
        relsim.deposit_moments(ctx, parts, B, J, M)
        relsim.timing_enable(ctx, False)
        if ev is not None:
            ev[1].record(st)
        _, _, _, it, rr = relsim.field_solve(ctx, M, J, E, B, Eth, E1, B1)
        if ev is not None:
            ev[2].record(st)
        relsim.timing_enable(ctx, ev is not None and want_kernels)
        relsim.push(ctx, parts, Eth, B, resort=True)
        relsim.timing_enable(ctx, False)
        if ev is not None:
            ev[3].record(st)
        W = relsim.energy(ctx, parts, E1, B1)
        if ev is not None:
            ev[4].record(st)
        return it, rr, W

    for _ in range(warmup):
        one_step(E, B, nb[0], nb[1])
        E, nb[0] = nb[0], E
        B, nb[1] = nb[1], B
    relsim.timing_reset(ctx)
    Wstart = relsim.energy(ctx, parts, E, B)
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(steps)]
    iters = []
    energies = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        it, rr, W = one_step(E, B, nb[0], nb[1], evs[k])
        iters.append(it)
        energies.append(W)
        E, nb[0] = nb[0], E
        B, nb[1] = nb[1], B
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    Wend = relsim.energy(ctx, parts, E, B)
    dep = sum(e[0].elapsed_time(e[1]) for e in evs)
    sol = sum(e[1].elapsed_time(e[2]) for e in evs)
    pus = sum(e[2].elapsed_time(e[3]) for e in evs)
    ene = sum(e[3].elapsed_time(e[4]) for e in evs)
    hot_steps = sorted(e[0].elapsed_time(e[1]) + e[2].elapsed_time(e[3]) for e in evs)
    kern = relsim.timing_read(ctx)
    hot = dep + pus
    res = {
        "precision": prec,
        "particles": n,
        "value": n * steps / (hot * 1e-3),
        "hot_ms_per_step": hot / steps,
        "hot_ms_median_step": hot_steps[len(hot_steps) // 2],
        "deposit_ms_per_step": dep / steps,
        "push_sort_ms_per_step": pus / steps,
        "solve_ms_per_step": sol / steps,
        "energy_ms_per_step": ene / steps,
        "wall_ms_per_step": 1e3 * wall / steps,
        "gmres_iters_per_step": sum(iters) / steps,
        "energy_start": list(map(float, Wstart)),
        "energy_end": list(map(float, Wend)),
        "energy_drift_per_step": float((Wend[3] - Wstart[3]) / W0[3] / steps),
        "energy_drift_max_abs_per_step": float(max(abs(b[3] - a[3]) for a, b in zip([Wstart] + energies[:-1],
                                                                                        energies)) / W0[3]),
        "kernels": {k: {"ms_per_launch": v[0] / max(v[1], 1), "launches": v[1]} for k, v in kern.items()},
    }
    del parts, ctx, E, B, nb, Eth, J, M
    torch.cuda.empty_cache()
    return res


def device_copy_bandwidth(nbytes=1 << 30, reps=10):
    """Achievable HBM bandwidth on this GPU: a device-to-device copy of 1 GiB
    (read + write bytes over time), the practical ceiling beside the 8 TB/s
    specification."""
    import torch

    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record()
    for _ in range(reps):
        b.copy_(a)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / reps
    del a, b
    return 2 * nbytes / (ms * 1e-3) / 1e9


def path_bytes_per_particle(wl, prec, n, nbins, ncells):
    """Algorithmic bytes per particle-step of this design (deposit + push +
    re-sort, as separate kernels) and the single-pass minimum (one read and
    one write of the particle state plus the per-step grid traffic: M and
    J-hat written once, E_theta and B^n read once)."""
    T = 4 if prec == "mixed" else 8
    d = wl.dim
    noff = 27 if d == 3 else 9
    this = sum(kernel_bytes(k, wl, prec, n, nbins, ncells) for k in
               ("deposit_cells", "assemble_nodes", "push_count", "push_scatter")) / n
    state = (d + 4) * T
    grid = ncells * (8 * 9 * noff + 3 * 24) / n
    return this, 2 * state + grid


def cpu_baseline(wl, host, nsample):
    """The CPU oracle (serial C, FP64) on the first nsample particles of the
    same workload: deposit (S1-S3) + push (S6), one step."""
    import numpy as np

    import oracle

    g = oracle.Grid(dim=wl.dim, nx=wl.nx, ny=wl.ny, nz=wl.nz if wl.dim == 3 else 1, dx=wl.dx, dy=wl.dx, dz=wl.dx,
                    dt=wl.dt, q=wl.q, m=wl.m)
    c = host["cell"][:nsample].astype(np.int64)
    off = host["off"][:, :nsample]
    xs = [((c % wl.nx) + off[0]) * wl.dx, (((c // wl.nx) % wl.ny) + off[1]) * wl.dx]
    if wl.dim == 3:
        xs.append(((c // (wl.nx * wl.ny)) + off[2]) * wl.dx)
    x = np.stack(xs)
    u = np.ascontiguousarray(host["u"][:, :nsample])
    w = np.ascontiguousarray(host["w"][:nsample])
    sp = host["species"][:nsample].astype(np.int32)
    oracle.build(force=False)
    t = time.perf_counter()
    oracle.deposit(g, x, u, w, sp, host["B"])
    oracle.push(g, x, u, sp, host["E"], host["B"])
    dt = time.perf_counter() - t
    return {"value": nsample / dt, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": "first %d particles (bin order) of the same workload, one step of deposit (S1-S3) + push (S6), "
                      "serial C FP64, %.1f s" % (nsample, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="harris2d_1024x512")
    ap.add_argument("--precision", default="both", choices=["both", "mixed", "fp64"])
    ap.add_argument("--group", type=int, default=0, help="lanes per cell in the deposit and energy kernels (0 = automatic)")
    ap.add_argument("--rtol", type=float, default=1e-10)
    ap.add_argument("--cpu-sample", type=int, default=10_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--energy-conserving", action="store_true",
                    help="also time the energy-conserving step (reported beside the headline, not in it)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run one device copy of this size (for counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU; the multi-GPU path is not built. Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2509_11100_amd import _lib, harris

    _lib.load()  # fail loudly before the long input generation
    wl = harris.workload(args.workload)
    log("generating %s: %d particles" % (wl.name, wl.nparticles))
    t = time.perf_counter()
    host = harris.make_particles(wl, workers=min(16, os.cpu_count() or 1))
    host["E"], host["B"] = harris.make_fields(wl)
    log("inputs ready in %.1f s" % (time.perf_counter() - t))
    torch.cuda.set_device(0)

    if args.copy_probe_mib:
        a = torch.empty(args.copy_probe_mib << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    copy_gbs = device_copy_bandwidth()

    precs = ["mixed", "fp64"] if args.precision == "both" else [args.precision]
    results = {}
    for p in precs:
        log("running %s: %d warmup + %d timed steps" % (p, args.warmup, args.steps))
        results[p] = run_precision(p, wl, host, args.steps, args.warmup, args.rtol, group=args.group)
        log("%s: %.4g particle-steps/s, hot %.3f ms/step, solve %.3f ms/step" % (
            p, results[p]["value"], results[p]["hot_ms_per_step"], results[p]["solve_ms_per_step"]))

    head = results[precs[0]]
    n = head["particles"]
    nbins = wl.ncells * wl.nspecies
    # dominant particle kernel of the headline run, and its HBM roofline
    cand = {k: v for k, v in head["kernels"].items() if kernel_bytes(k, wl, head["precision"], n, nbins, wl.ncells)}
    roof = None
    if cand:
        dom = max(cand, key=lambda k: cand[k]["ms_per_launch"] * cand[k]["launches"])
        byt = kernel_bytes(dom, wl, head["precision"], n, nbins, wl.ncells)
        ach = byt / (cand[dom]["ms_per_launch"] * 1e-3) / 1e9
        roof = {"kernel": dom, "bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(ach / PEAK_HBM_GBS, 4),
                "traffic": measured_traffic("%s_%s" % (wl.name, head["precision"]), dom),
                "bytes_per_launch": byt, "ms_per_launch": round(cand[dom]["ms_per_launch"], 4)}
        per_kernel = {}
        for k, v in cand.items():
            b = kernel_bytes(k, wl, head["precision"], n, nbins, wl.ncells)
            per_kernel[k] = round(b / (v["ms_per_launch"] * 1e-3) / 1e9, 1)
        roof["achieved_by_kernel_GBs"] = per_kernel
        roof["measured_copy_GBs"] = round(copy_gbs, 1)
        roof["frac_of_measured_copy"] = round(ach / copy_gbs, 4)
        this, fused = path_bytes_per_particle(wl, head["precision"], n, nbins, wl.ncells)
        roof["path"] = {
            "bytes_per_particle_step": round(this, 2),
            "achieved_GBs": round(head["value"] * this / 1e9, 1),
            "frac": round(head["value"] * this / 1e9 / PEAK_HBM_GBS, 4),
            "single_pass_min_bytes_per_particle_step": round(fused, 2),
            "frac_single_pass_min": round(head["value"] * fused / 1e9 / PEAK_HBM_GBS, 4),
        }

    ec = None
    if args.energy_conserving:
        ec = {}
        for p in precs:
            log("running the energy-conserving step, %s" % p)
            ec[p] = run_energy_conserving(p, wl, host, args.steps, args.warmup, args.rtol, group=args.group)
            log("%s energy-conserving: %.3f ms/step, %.1f passes/step, |dW|/W %.2e" % (
                p, ec[p]["ms_per_step"], ec[p]["passes_per_step"], ec[p]["rel_energy_change"]))

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on %d particles" % args.cpu_sample)
        cpu = cpu_baseline(wl, host, min(args.cpu_sample, n))

    out = {
        "metric": "particle-steps/sec (gather+alpha_p+M/J deposit+push), FP32-mixed vs FP64, at 1e-5 rel err",
        "value": head["value"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["wall_ms_per_step"],
        "hot_path_ms_per_step": head["hot_ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if head["precision"] == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": "%s: %dD double Harris sheet %s cells, %d particles/cell/species, %d particles, "
                               "dt = 0.5 dx/c, GMRES rtol %g" % (
                                   wl.name, wl.dim, "x".join(str(v) for v in (wl.nx, wl.ny, wl.nz)[:wl.dim]), wl.ppc,
                                   n, args.rtol),
                   "precision": head["precision"], "parallelism": "single GPU"},
        "results": results,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    if ec is not None:
        out["energy_conserving"] = ec
    if "mixed" in results and "fp64" in results:
        out["mixed_over_fp64"] = results["mixed"]["value"] / results["fp64"]["value"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
