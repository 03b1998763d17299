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

A second workload, the 3D double Harris sheet 128 x 64 x 64 cells x 16
particles per cell per species (16,777,216 particles, 27-offset mass matrix),
is timed the same way after the headline and reported under "secondary".

The CPU-baseline leg runs the oracle (plain C, FP64) on the host: once on one
thread over a bounded sample, once on every host core over the whole
workload (one thread per chunk of particles, private J-hat/M copies summed in
a fixed order), and it reports the error of every GPU result against the
oracle on the same inputs: J-hat and M at sampled nodes, the pushed
particles at a sample followed through the re-sort, and the FP64 energy.

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


def kernel_bytes(name, wl, prec, n, nbins, ncells, mb=8):
    """Algorithmic bytes of one launch of a kernel: what it must read and
    write at least once (particle state, grid fields, per-cell moments); mb
    is the bytes of one stored value of M (8, or 4 with mass_fp32)."""
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
        # in: per-cell moments; out: J-hat (FP64) and the stored half of M
        # at nodes (5 of the 9 node-pair blocks in 2D, 14 of 27 in 3D)
        nmom = 93 if d == 2 else 267
        return ncells * nmom * T + ncells * (grid + mb * 9 * (noff // 2 + 1))
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


def measured_valu(tag, kernel):
    """VALU issue of a kernel from the committed rocprofv3 counter summary
    (busy fraction, lane use, clock, VALU instructions per 64 particles), or
    None when the kernels changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "valu_%s.json" % tag)
    if not os.path.exists(path):
        return None
    js = json.load(open(path))
    code = device_code_sha256()
    if code is None or js.get("device_code_sha256") != code:
        return None
    return js["kernels"].get(KERNEL_SYMBOL.get(kernel, kernel))


def run_energy_conserving(prec, wl, host, steps, warmup, rtol, group=0, secant=False, mass_fp32=False):
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
                         gmres_maxit=5000, group=group, mass_fp32=mass_fp32)
    parts = relsim.Particles(ctx).load(host["cell"], host["species"], host["off"], host["u"], host["w"],
                                       host["bin_start"])
    step = relsim.Step(ctx, parts, torch.as_tensor(host["E"]).cuda(), torch.as_tensor(host["B"]).cuda(),
                       energy_conserving=True, secant=secant)
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
            "picard_tol": 1e-12 if prec == "fp64" else 1e-6, "fixed_point": "secant" if secant else "plain",
            "mass_matrix": "fp32" if mass_fp32 else "fp64",
            "passes_per_step": float(np.mean(passes)),
            "rel_energy_change": float(abs(W1[3] - W0[3]) / W0[3])}


def run_precision(prec, wl, host, steps, warmup, rtol, want_kernels=True, group=0, mass_fp32=False):
    import numpy as np
    import torch

    from paper_2509_11100_amd import relsim

    n = host["w"].shape[0]
    ctx = relsim.Context(dim=wl.dim, nx=wl.nx, ny=wl.ny, nz=wl.nz if wl.dim == 3 else 1, dx=wl.dx, dt=wl.dt,
                         precision=prec, q=wl.q, m=wl.m, max_particles=n, gmres_rtol=rtol, gmres_restart=30,
                         gmres_maxit=5000, group=group, mass_fp32=mass_fp32)
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
        # S7 with the kinetic part the push summed (no pass over the particles)
        W = relsim.energy_pushed(ctx, E1, B1)
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
        "mass_matrix": "fp32" if mass_fp32 else "fp64",
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


def path_bytes_per_particle(wl, prec, n, nbins, ncells, mb=8):
    """Algorithmic bytes per particle-step of this design (deposit + push +
    re-sort, as separate kernels) and the fused minimum of a step: one read
    and one write of each particle's offsets, momentum and weight (the mixed
    state counted with a 4-byte cell index beside its FP32 values), plus the
    grid traffic of a step with push and the next deposit in one pass: M and
    J-hat written once, E_theta, B^n and B^{n+1} read once per node.  M is
    counted with all 9 (2D) or 27 (3D) blocks per node, as the roofline
    target was set, although the library writes only the unique half."""
    T = 4 if prec == "mixed" else 8
    d = wl.dim
    noff = 27 if d == 3 else 9
    this = sum(kernel_bytes(k, wl, prec, n, nbins, ncells, mb) for k in
               ("deposit_cells", "assemble_nodes", "push_count", "push_scatter")) / n
    state = (d + 4) * T
    grid = ncells * (8 * 9 * noff + 24 + 3 * 24) / n
    return this, 2 * state + (4 if prec == "mixed" else 0) + grid


def sample_nodes_and_particles(wl, host, seed=7):
    """The sampled outputs compared with the oracle: about 150 random nodes
    plus the box corners and the sheet centres (their J-hat and M depend only
    on the particles of the cells around them), and about 20,000 random
    particles followed through the re-sort."""
    import numpy as np

    rng = np.random.default_rng(seed)
    N = wl.ncells
    nodes = np.unique(np.concatenate([rng.integers(0, N, 150), [0, wl.nx - 1, N - 1],
                                      [wl.nx * (wl.ny // 4), wl.nx * (3 * wl.ny // 4)]]))
    i, j, k = nodes % wl.nx, (nodes // wl.nx) % wl.ny, nodes // (wl.nx * wl.ny)
    cells = []
    for a in range(1 << wl.dim):
        ii = (i - (a & 1)) % wl.nx
        jj = (j - ((a >> 1) & 1)) % wl.ny
        kk = (k - ((a >> 2) & 1)) % wl.nz if wl.dim == 3 else 0
        cells.append(ii + wl.nx * (jj + wl.ny * kk))
    cells = np.unique(np.concatenate(cells))
    S = wl.nspecies
    b = host["bin_start"]
    around = np.concatenate([np.arange(b[c * S], b[c * S + S]) for c in cells])
    n = host["w"].shape[0]
    parts = np.unique(np.concatenate([np.random.default_rng(seed + 4).integers(0, n, 20000), [0, n - 1]]))
    return nodes, around, parts


def gpu_sampled_results(prec, wl, host, rtol):
    """One deposit, solve and push + re-sort of the initial state on a fresh
    context (outside any timed region), read back at the sampled nodes and
    particles, plus the energy of the initial state."""
    import numpy as np
    import torch

    from paper_2509_11100_amd import relsim

    n = host["w"].shape[0]
    nodes, _, sel = sample_nodes_and_particles(wl, host)
    ctx = relsim.Context(dim=wl.dim, nx=wl.nx, ny=wl.ny, nz=wl.nz if wl.dim == 3 else 1, dx=wl.dx, dt=wl.dt,
                         precision=prec, q=wl.q, m=wl.m, max_particles=n, gmres_rtol=rtol, gmres_restart=30,
                         gmres_maxit=5000)
    parts = relsim.Particles(ctx).load(host["cell"], host["species"], host["off"], host["u"], host["w"],
                                       host["bin_start"])
    E = torch.as_tensor(host["E"]).cuda()
    B = torch.as_tensor(host["B"]).cuda()
    W = relsim.energy(ctx, parts, E, B)
    J, M = relsim.deposit_moments(ctx, parts, B)
    nt = torch.as_tensor(nodes, device=J.device)
    out = {"W": W, "J": J[:, nt].cpu().numpy(), "M": _all_blocks_at(wl, M, nodes)}
    Eth, _, _, _, _ = relsim.field_solve(ctx, M, J, E, B)
    del J, M
    perm = torch.empty(n, dtype=torch.int32, device=E.device)
    relsim.push(ctx, parts, Eth, B, resort=True, new_index=perm)
    out["clamps"] = relsim.placement_clamps(ctx)
    new = perm[torch.as_tensor(sel, device=E.device)].long()
    del perm
    out["cell"] = parts.cell[new].cpu().numpy()
    out["off"] = np.stack([o[new].cpu().numpy().astype(np.float64) for o in parts.off])
    out["u"] = np.stack([c[new].cpu().numpy().astype(np.float64) for c in parts.u])
    out["E_theta"] = Eth.cpu().numpy()
    del parts, ctx, E, B, Eth
    torch.cuda.empty_cache()
    return out


def _all_blocks_at(wl, M, nodes):
    """The 9 (2D) or 27 (3D) node-pair blocks of some nodes, [noff][9][n],
    from the library's stored half (offsets o >= c at the node itself; o < c
    is slot c - o of the node at offset o)."""
    import numpy as np
    import torch

    noff = 27 if wl.dim == 3 else 9
    c = noff // 2
    nodes = np.asarray(nodes)
    nz = wl.nz if wl.dim == 3 else 1
    i, j, k = nodes % wl.nx, (nodes // wl.nx) % wl.ny, nodes // (wl.nx * wl.ny)
    out = []
    for o in range(noff):
        dx, dy, dz = o % 3 - 1, (o // 3) % 3 - 1, (o // 9 - 1 if wl.dim == 3 else 0)
        nb = (i + dx) % wl.nx + wl.nx * (((j + dy) % wl.ny) + wl.ny * ((k + dz) % nz))
        slot, ids = (o - c, nodes) if o >= c else (c - o, nb)
        out.append(M[slot][:, torch.as_tensor(ids, device=M.device)].cpu().numpy())
    return np.stack(out)


def _oracle_grid(wl):
    import oracle

    return oracle.Grid(dim=wl.dim, nx=wl.nx, ny=wl.ny, nz=wl.nz if wl.dim == 3 else 1, dx=wl.dx, dy=wl.dx, dz=wl.dx,
                       dt=wl.dt, q=wl.q, m=wl.m)


def _positions(wl, cell, off):
    import numpy as np

    c = np.asarray(cell, dtype=np.int64)
    xs = [((c % wl.nx) + off[0]) * wl.dx, (((c // wl.nx) % wl.ny) + off[1]) * wl.dx]
    if wl.dim == 3:
        xs.append(((c // (wl.nx * wl.ny)) + off[2]) * wl.dx)
    return np.stack(xs)


def _errors(a, b):
    import numpy as np

    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return {"normwise": float(np.linalg.norm(a - b) / np.linalg.norm(b)),
            "max_abs_over_max_ref": float(np.abs(a - b).max() / np.abs(b).max())}


def oracle_errors(prec, wl, host, gpu):
    """Error of the GPU results against the oracle on the same inputs (the
    mixed run's inputs rounded to FP32 and promoted for the oracle)."""
    import numpy as np

    import oracle

    def r(a):
        a = np.asarray(a, dtype=np.float64)
        return a.astype(np.float32).astype(np.float64) if prec == "mixed" else a

    g = _oracle_grid(wl)
    nodes, around, sel = sample_nodes_and_particles(wl, host)
    sp = host["species"].astype(np.int32)
    Jr, Mr = oracle.deposit_nodes(g, _positions(wl, host["cell"][around], r(host["off"][:, around])),
                                  r(host["u"][:, around]), r(host["w"][around]), sp[around], host["B"], nodes)
    x0 = _positions(wl, host["cell"][sel], r(host["off"][:, sel]))
    xr, ur = oracle.push(g, x0, r(host["u"][:, sel]), sp[sel], gpu["E_theta"], host["B"])
    L = np.array(g.L)[:, None]
    dx = _positions(wl, gpu["cell"], gpu["off"]) - xr
    dx -= L * np.round(dx / L)
    disp = xr - x0
    disp -= L * np.round(disp / L)
    Wr = oracle.energy(g, r(host["u"]), r(host["w"]), sp, host["E"], host["B"])
    W = gpu["W"]
    return {
        "J_sampled_nodes": _errors(gpu["J"], Jr),
        "M_sampled_nodes": _errors(gpu["M"], Mr),
        "u_pushed_sampled": _errors(gpu["u"], ur),
        "x_pushed_sampled_over_displacement": {
            "normwise": float(np.linalg.norm(dx) / np.linalg.norm(disp)),
            "max_abs_over_max_ref": float(np.abs(dx).max() / np.abs(disp).max())},
        # relative to each part, or to the total where the part is zero (E^0 = 0)
        "energy_rel": {k: float(abs(W[i] - Wr[i]) / (abs(Wr[i]) if Wr[i] != 0 else abs(Wr[3]))) for i, k in
                       enumerate(("kinetic", "electric", "magnetic", "total"))},
        "placement_clamps": int(gpu["clamps"]),
        "samples": {"nodes": int(nodes.size), "particles": int(sel.size)},
    }


def host_cores():
    """Host cores this process may use, capped at 16 (the host share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(wl, host, nsample, all_cores=True):
    """The CPU oracle (plain C, FP64) on the same work as the metric, deposit
    (S1-S3) + push (S6), one step: on one thread over the first nsample
    particles, and on every host core over all particles (one thread per
    contiguous chunk; the C calls release the interpreter lock; each chunk
    deposits into its own J-hat/M, summed in chunk order)."""
    import concurrent.futures as cf

    import numpy as np

    import oracle

    g = _oracle_grid(wl)
    oracle.build(force=False)
    n_all = host["w"].shape[0]
    sp_all = host["species"].astype(np.int32)

    def work(lo, hi):
        x = _positions(wl, host["cell"][lo:hi], host["off"][:, lo:hi])
        u = np.ascontiguousarray(host["u"][:, lo:hi])
        J, M = oracle.deposit(g, x, u, np.ascontiguousarray(host["w"][lo:hi]), sp_all[lo:hi], host["B"])
        oracle.push(g, x, u, sp_all[lo:hi], host["E"], host["B"])
        return J, M

    nsample = min(nsample, n_all)
    t = time.perf_counter()
    work(0, nsample)
    dt1 = time.perf_counter() - t
    out = {"value": nsample / dt1, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
           "sample": "first %d particles (bin order) of the same workload, one step of deposit (S1-S3) + push (S6), "
                     "plain C FP64 on one thread, %.1f s" % (nsample, dt1)}
    if all_cores:
        cores = host_cores()
        bounds = np.linspace(0, n_all, cores + 1).astype(np.int64)
        t = time.perf_counter()
        with cf.ThreadPoolExecutor(max_workers=cores) as ex:
            res = list(ex.map(lambda k: work(int(bounds[k]), int(bounds[k + 1])), range(cores)))
        J, M = res[0]
        for Jk, Mk in res[1:]:
            J += Jk
            M += Mk
        dtn = time.perf_counter() - t
        del res, J, M
        out["all_cores"] = {"value": n_all / dtn, "unit": "particle-steps/s", "cores": cores, "kind": "oracle",
                            "sample": "all %d particles of the workload, one step of deposit + push, %d threads "
                                      "(one chunk each, private J-hat/M summed in chunk order), %.1f s"
                                      % (n_all, cores, dtn)}
    return out


def roofline_of(res, wl, copy_gbs):
    """HBM roofline of the dominant particle kernel of a timed run, and of the
    whole path."""
    prec = res["precision"]
    n = res["particles"]
    nbins = wl.ncells * wl.nspecies
    mb = 4 if res.get("mass_matrix") == "fp32" else 8
    cand = {k: v for k, v in res["kernels"].items() if kernel_bytes(k, wl, prec, n, nbins, wl.ncells, mb)}
    if not cand:
        return None
    dom = max(cand, key=lambda k: cand[k]["ms_per_launch"] * cand[k]["launches"])
    byt = kernel_bytes(dom, wl, prec, n, nbins, wl.ncells, mb)
    # the committed counter summaries were taken with M stored in FP64
    tag = "%s_%s" % (wl.name, prec) if mb == 8 else None
    ach = byt / (cand[dom]["ms_per_launch"] * 1e-3) / 1e9
    roof = {"kernel": dom, "bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(ach / PEAK_HBM_GBS, 4),
            "traffic": measured_traffic(tag, dom) if tag else None,
            "valu": measured_valu(tag, dom) if tag else None,
            "bytes_per_launch": byt, "ms_per_launch": round(cand[dom]["ms_per_launch"], 4)}
    per_kernel = {}
    for k, v in cand.items():
        b = kernel_bytes(k, wl, prec, n, nbins, wl.ncells, mb)
        per_kernel[k] = round(b / (v["ms_per_launch"] * 1e-3) / 1e9, 1)
    roof["achieved_by_kernel_GBs"] = per_kernel
    roof["measured_copy_GBs"] = round(copy_gbs, 1)
    roof["frac_of_measured_copy"] = round(ach / copy_gbs, 4)
    this, fused = path_bytes_per_particle(wl, prec, n, nbins, wl.ncells, mb)
    roof["path"] = {
        "bytes_per_particle_step": round(this, 2),
        "achieved_GBs": round(res["value"] * this / 1e9, 1),
        "frac": round(res["value"] * this / 1e9 / PEAK_HBM_GBS, 4),
        "fused_min_bytes_per_particle_step": round(fused, 2),
        "frac_fused_min": round(res["value"] * fused / 1e9 / PEAK_HBM_GBS, 4),
        "particle_steps_per_s_at_half_of_peak_fused": round(0.5 * PEAK_HBM_GBS * 1e9 / fused, -7),
    }
    return roof


def make_inputs(name):
    from paper_2509_11100_amd import harris

    wl = harris.workload(name)
    log("generating %s: %d particles" % (wl.name, wl.nparticles))
    t = time.perf_counter()
    host = harris.make_particles(wl, workers=host_cores())
    host["E"], host["B"] = harris.make_fields(wl)
    log("inputs ready in %.1f s" % (time.perf_counter() - t))
    return wl, host


def workload_label(wl, n, rtol):
    return "%s: %dD double Harris sheet %s cells, %d particles/cell/species, %d particles, dt = 0.5 dx/c, " \
           "GMRES rtol %g" % (wl.name, wl.dim, "x".join(str(v) for v in (wl.nx, wl.ny, wl.nz)[:wl.dim]), wl.ppc, n,
                              rtol)


def run_adjoint(steps, rtol=1e-14):
    """The adjoint of `steps` FP64 steps of the 256 x 128 double Harris sheet
    (32 particles per cell per species, 2,097,152 particles): the gradient of
    the field energy after the steps with respect to the initial E and B
    (autograd.field_energy_after, per-step checkpoints), timed against the
    same steps run forward without gradients.  Returns ms per step."""
    import numpy as np
    import torch

    from paper_2509_11100_amd import autograd, harris, relsim

    wl = harris.workload("harris2d_256x128")
    p = harris.make_particles(wl)
    E0, Bh = harris.make_fields(wl, eps=0.0)
    n = p["w"].shape[0]
    ctx = relsim.Context(dim=2, nx=wl.nx, ny=wl.ny, dx=wl.dx, dy=wl.dx, dt=wl.dt, precision="fp64", q=wl.q, m=wl.m,
                         max_particles=n, gmres_rtol=rtol)
    parts = relsim.Particles(ctx).load(p["cell"], p["species"], p["off"], p["u"], p["w"], p["bin_start"])
    st = autograd.Stepper(ctx)
    base = [t.clone() for t in (parts.cell, parts.bin_start, parts.w)]
    off0 = torch.stack([t.clone() for t in parts.off])
    u0 = torch.stack([t.clone() for t in parts.u])

    def dev(a):
        return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()

    E = dev(E0)
    B = dev(Bh) + wl.eps * dev(harris.seed_direction(wl))
    out = None
    for rep in range(2):  # the first pass warms up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        with torch.no_grad():
            off, u, Ee, Bb, c, b, w = off0, u0, E, B, *base
            for _ in range(steps):
                off, u, Ee, Bb, c, b, w = autograd.StepFn.apply(st, off, u, Ee, Bb, c, b, w)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        Eg = E.clone().requires_grad_(True)
        Bg = B.clone().requires_grad_(True)
        F = autograd.field_energy_after(st, off0, u0, Eg, Bg, *base, steps)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        F.backward()
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        out = {"particles": n, "steps": steps, "forward_ms_per_step": 1e3 * (t1 - t0) / steps,
               "checkpointed_forward_ms_per_step": 1e3 * (t2 - t1) / steps,
               "backward_ms_per_step": 1e3 * (t3 - t2) / steps, "grad_B_norm": float(Bg.grad.norm())}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="harris2d_1024x512")
    ap.add_argument("--secondary", default="harris3d_128x64x64",
                    help="second workload timed after the headline ('none' to skip)")
    ap.add_argument("--secondary-steps", type=int, default=10)
    ap.add_argument("--precision", default="both", choices=["both", "mixed", "fp64"])
    ap.add_argument("--group", type=int, default=0, help="lanes per cell in the deposit and energy kernels (0 = automatic)")
    ap.add_argument("--rtol", type=float, default=1e-10)
    ap.add_argument("--cpu-sample", type=int, default=10_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle leg (its timings and the errors against it)")
    ap.add_argument("--energy-conserving", action="store_true",
                    help="also time the energy-conserving step (reported beside the headline, not in it)")
    ap.add_argument("--secant", action="store_true",
                    help="the energy-conserving step's fixed point with per-particle secant steps")
    ap.add_argument("--mass-fp32", action="store_true",
                    help="mixed precision with the mass matrix stored in FP32 (the default stores it in FP64)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run one device copy of this size (for counter calibration)")
    ap.add_argument("--adjoint", type=int, default=0, metavar="K",
                    help="instead of the step, time the adjoint of K FP64 steps of the 256 x 128 sheet")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU; the multi-GPU path is not built. Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if args.adjoint > 0:
        import torch

        from paper_2509_11100_amd import _lib

        _lib.load()
        torch.cuda.set_device(0)
        res = run_adjoint(args.adjoint)
        log("adjoint of %d steps: forward %.2f ms/step, backward %.2f ms/step" % (
            args.adjoint, res["forward_ms_per_step"], res["backward_ms_per_step"]))
        print(json.dumps({"metric": "adjoint ms per step (gradient of the field energy after K steps)",
                          "config": {"workload": "harris2d_256x128, 2D double Harris sheet 256x128 cells, "
                                                 "32 particles/cell/species, FP64"}, **res}), flush=True)
        return

    import torch

    from paper_2509_11100_amd import _lib

    _lib.load()  # fail loudly before the long input generation
    wl, host = make_inputs(args.workload)
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
        results[p] = run_precision(p, wl, host, args.steps, args.warmup, args.rtol, group=args.group,
                                   mass_fp32=args.mass_fp32 and p == "mixed")
        log("%s: %.4g particle-steps/s, hot %.3f ms/step, solve %.3f ms/step" % (
            p, results[p]["value"], results[p]["hot_ms_per_step"], results[p]["solve_ms_per_step"]))
    head = results[precs[0]]
    n = head["particles"]
    roof = roofline_of(head, wl, copy_gbs)
    # the GPU results the oracle leg checks (fresh context, untimed)
    samples = {p: gpu_sampled_results(p, wl, host, args.rtol) for p in precs} if not args.no_cpu_baseline else {}

    ec = None
    if args.energy_conserving:
        ec = {}
        for p in precs:
            log("running the energy-conserving step, %s" % p)
            ec[p] = run_energy_conserving(p, wl, host, args.steps, args.warmup, args.rtol, group=args.group,
                                          secant=args.secant, mass_fp32=args.mass_fp32 and p == "mixed")
            log("%s energy-conserving: %.3f ms/step, %.1f passes/step, |dW|/W %.2e" % (
                p, ec[p]["ms_per_step"], ec[p]["passes_per_step"], ec[p]["rel_energy_change"]))

    secondary = None
    if args.secondary != "none":
        wl2, host2 = make_inputs(args.secondary)
        secondary = {"config": {"workload": workload_label(wl2, host2["w"].shape[0], args.rtol)}, "results": {}}
        samples2 = {}
        for p in precs:
            log("running %s on %s: %d warmup + %d timed steps" % (p, wl2.name, min(args.warmup, 2),
                                                                  args.secondary_steps))
            r2 = run_precision(p, wl2, host2, args.secondary_steps, min(args.warmup, 2), args.rtol, group=args.group,
                               mass_fp32=args.mass_fp32 and p == "mixed")
            r2["roofline"] = roofline_of(r2, wl2, copy_gbs)
            secondary["results"][p] = r2
            log("%s %s: %.4g particle-steps/s, hot %.3f ms/step" % (wl2.name, p, r2["value"], r2["hot_ms_per_step"]))
            if not args.no_cpu_baseline:
                samples2[p] = gpu_sampled_results(p, wl2, host2, args.rtol)
        if "mixed" in secondary["results"] and "fp64" in secondary["results"]:
            secondary["mixed_over_fp64"] = secondary["results"]["mixed"]["value"] / secondary["results"]["fp64"]["value"]

    cpu = None
    if not args.no_cpu_baseline:
        # the oracle leg: its errors against every GPU result, then its timings
        log("oracle: errors of the GPU results")
        for p in precs:
            results[p]["oracle_error"] = oracle_errors(p, wl, host, samples[p])
            log("%s vs oracle: %s" % (p, json.dumps(results[p]["oracle_error"])))
        if secondary is not None:
            for p in precs:
                secondary["results"][p]["oracle_error"] = oracle_errors(p, wl2, host2, samples2[p])
            del host2
        log("timing the CPU oracle: %d particles on one thread, all particles on %d threads"
            % (args.cpu_sample, host_cores()))
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
        "config": {"workload": workload_label(wl, n, args.rtol), "precision": head["precision"],
                   "parallelism": "single GPU"},
        "results": results,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    if "oracle_error" in head:
        out["oracle_error"] = head["oracle_error"]
    if ec is not None:
        out["energy_conserving"] = ec
    if "mixed" in results and "fp64" in results:
        out["mixed_over_fp64"] = results["mixed"]["value"] / results["fp64"]["value"]
    if secondary is not None:
        out["secondary"] = secondary
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
