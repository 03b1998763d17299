"""Momentum spectra of the nonlinear reconnection runs (Sec. 3.2, Sec. 4.2,
Table 2): the spectrum of the background population's proper speed u/c, its
power-law slope and its high-energy cutoff, and a driver for the fiducial
run (sigma_ci = 100, L_x = L_y = 50 d_i,C) on one GPU.

Readings.  The spectrum is f(u) = dN/du, the number of physical particles
(macro-particle weights) per unit proper speed u = gamma v / c, histogrammed
in logarithmic bins; its slope is alpha = d ln f / d ln u, fitted by least
squares in log-log over the window the paper quotes for the run (electrons
of the fiducial case: u/c in [100, 4000], that is [0.01, 0.4] sigma_ce).
The cutoff u_max is where the spectrum, followed upward from the fit
window's lower end, first falls below the fitted power law by a factor e.
sigma_ce = sigma_ci m_i / m_e.

The diagnostics run on the GPU state through torch (a histogram per
snapshot); they are analysis, not part of the step.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time
from typing import Dict, Optional, Sequence

import numpy as np

from . import harris

# logarithmic bins of u/c: 0.01 .. 1e6, 40 per decade
EDGES = np.logspace(-2.0, 6.0, 8 * 40 + 1)


def spectrum(u: np.ndarray, w: np.ndarray, edges: np.ndarray = EDGES) -> np.ndarray:
    """dN/du in the bins `edges` from proper speeds u (n,) and weights w (n,)."""
    counts, _ = np.histogram(u, bins=edges, weights=w)
    return counts / np.diff(edges)


def centres(edges: np.ndarray = EDGES) -> np.ndarray:
    """Geometric bin centres."""
    return np.sqrt(edges[1:] * edges[:-1])


def fit_power_law(uc: np.ndarray, f: np.ndarray, u1: float, u2: float):
    """Least-squares slope and amplitude of ln f against ln u over the bins
    with u1 <= u <= u2 and f > 0: f ~ amp u^alpha.  Returns (alpha, amp)."""
    sel = (uc >= u1) & (uc <= u2) & (f > 0)
    if sel.sum() < 2:
        return float("nan"), float("nan")
    x, y = np.log(uc[sel]), np.log(f[sel])
    alpha, lnamp = np.polyfit(x, y, 1)
    return float(alpha), float(math.exp(lnamp))


def local_slope(uc: np.ndarray, f: np.ndarray, span: int = 8) -> np.ndarray:
    """d ln f / d ln u by a centred difference over +-span bins (nan where
    f vanishes)."""
    out = np.full(f.shape, np.nan)
    lf = np.where(f > 0, np.log(np.where(f > 0, f, 1.0)), np.nan)
    lu = np.log(uc)
    out[span:-span] = (lf[2 * span:] - lf[:-2 * span]) / (lu[2 * span:] - lu[:-2 * span])
    return out


def cutoff(uc: np.ndarray, f: np.ndarray, alpha: float, amp: float, u1: float) -> float:
    """The first u >= u1 at which f drops below amp u^alpha / e (the last
    bin centre before it), or the largest populated bin if it never does."""
    start = np.searchsorted(uc, u1)
    for i in range(start, uc.size):
        if f[i] < amp * uc[i] ** alpha / math.e:
            return float(uc[i - 1]) if i > start else float(uc[i])
    nz = np.nonzero(f > 0)[0]
    return float(uc[nz[-1]]) if nz.size else float("nan")


def analyse(f: np.ndarray, u1: float, u2: float, sigma: float, edges: np.ndarray = EDGES) -> Dict[str, float]:
    """Slope over [u1, u2], cutoff, and the cutoff in units of sigma."""
    uc = centres(edges)
    alpha, amp = fit_power_law(uc, f, u1, u2)
    umax = cutoff(uc, f, alpha, amp, u1) if np.isfinite(alpha) else float("nan")
    peak = float(uc[int(np.argmax(f * uc))]) if f.any() else float("nan")
    return {"alpha": alpha, "u_max": umax, "u_max_over_sigma": umax / sigma, "u_peak": peak}


def sigma_ce(wl: harris.Workload) -> float:
    """Cold electron magnetisation sigma_ce = B0^2 / (4 pi n_b m_e c^2)."""
    return wl.harris.B0 ** 2 / (4.0 * math.pi * wl.nb_over_n0 * harris.N0 * min(wl.m))


def device_spectra(parts, species: Sequence[int], edges: np.ndarray = EDGES) -> Dict[int, np.ndarray]:
    """dN/du of the given species of a device particle set (relsim.Particles),
    computed on the device: the proper speed of every particle of a species
    (its bins' ranges), histogrammed by its logarithm."""
    import torch

    S = parts.ctx.nspecies
    bs = parts.bin_start.long()
    u = torch.stack([c.double() for c in parts.u])
    w = parts.w.double()
    counts = bs[1:] - bs[:-1]
    sp_of = torch.repeat_interleave(torch.arange(counts.numel(), device=bs.device) % S, counts)
    ledges = torch.as_tensor(np.log(edges), device=u.device)
    out = {}
    for s in species:
        sel = sp_of == s
        us = torch.sqrt((u[:, sel] ** 2).sum(0))
        lu = torch.log(torch.clamp(us, min=1e-300))
        idx = torch.bucketize(lu, ledges, right=True) - 1
        ok = (idx >= 0) & (idx < edges.size - 1)
        h = torch.zeros(edges.size - 1, dtype=torch.float64, device=u.device)
        h.index_add_(0, idx[ok], w[sel][ok])
        out[s] = h.cpu().numpy() / np.diff(edges)
    return out


def run(steps: Optional[int] = None, snapshots: Sequence[float] = (0, 1, 2, 3, 4, 5, 6, 7, 7.77),
        precision: str = "mixed", energy_conserving: bool = True, rtol: float = 1e-10,
        workers: int = 16, log=sys.stdout, secant: bool = True, out: Optional[str] = None,
        mass_fp32: bool = False, **overrides) -> Dict:
    """The fiducial Table 2 run: spectra of the background electrons and
    ions at the given times (t c / L_y), the energy history, and the slope
    and cutoff of the last electron spectrum.  With `out`, the record is
    written as JSON after every snapshot."""
    import torch

    from . import relsim

    wl = harris.workload("reconnection2d_625x625", **overrides)
    Ly = 0.5 * wl.ny * wl.dx
    tcl = wl.dt / Ly  # t c / L_y per step
    nsteps = wl.steps if steps is None else steps
    t0 = time.time()
    p = harris.make_particles(wl, workers=workers)
    E, B = harris.make_fields(wl)
    n = p["w"].shape[0]
    print("generated %d particles in %.1f s" % (n, time.time() - t0), file=log, flush=True)
    ctx = relsim.Context(dim=2, nx=wl.nx, ny=wl.ny, dx=wl.dx, dt=wl.dt, precision=precision, q=wl.q, m=wl.m,
                         max_particles=n, gmres_rtol=rtol, gmres_restart=30, gmres_maxit=5000,
                         mass_fp32=mass_fp32)
    parts = relsim.Particles(ctx).load(p["cell"], p["species"], p["off"], p["u"], p["w"], p["bin_start"])
    del p
    # the fixed point of this sheet converges slowly (about a factor 0.4 per
    # pass at sigma_ci = 100): allow many passes, and count the steps that
    # still miss the tolerance instead of stopping the run
    step = relsim.Step(ctx, parts, torch.as_tensor(E).cuda(), torch.as_tensor(B).cuda(),
                       energy_conserving=energy_conserving, picard_maxit=60, allow_unconverged=True,
                       secant=secant)
    S = wl.nspecies
    bg = (S - 2, S - 1)  # background ion and electron species
    sce = sigma_ce(wl)
    sci = sce * min(wl.m) / max(wl.m)
    marks = sorted(set(int(round(t / tcl)) for t in snapshots if round(t / tcl) <= nsteps) | {nsteps})
    rec = {"workload": wl.name, "particles": n, "precision": precision, "mass_fp32": bool(mass_fp32),
           "energy_conserving": energy_conserving,
           "fixed_point": "secant" if secant else "plain",
           "dt": wl.dt, "dx": wl.dx, "sigma_ce": sce, "sigma_ci": sci, "edges": EDGES.tolist(), "snapshots": []}
    W0 = step.energy()
    k = 0
    passes, unconverged = 0, 0
    tstart = tlast = time.time()
    for mark in marks:
        while k < mark:
            step()
            k += 1
            passes += step.picard_iters
            unconverged += 0 if step.picard_converged else 1
            now = time.time()
            if k % 100 == 0 or now - tlast > 20.0:
                tlast = now
                print("  step %d: %.1f fixed-point passes per step so far, %d unconverged, %.1f s" % (
                    k, passes / k, unconverged, now - tstart), file=log, flush=True)
        torch.cuda.synchronize()
        W = step.energy()
        sp = device_spectra(parts, bg)
        snap = {"step": k, "t_c_over_Ly": k * tcl, "W": [float(x) for x in W],
                "energy_error": float(abs(W[3] - W0[3]) / W0[3]), "f_e": sp[bg[1]].tolist(), "f_i": sp[bg[0]].tolist(),
                "picard_iters": int(step.picard_iters), "gmres_iters": int(step.iters)}
        snap["electrons"] = analyse(sp[bg[1]], 100.0, 0.4 * sce, sce)
        snap["ions"] = analyse(sp[bg[0]], 1.5, 0.4 * sci, sci)
        rec["snapshots"].append(snap)
        rec["seconds"] = time.time() - tstart
        rec["picard_passes_per_step"] = passes / max(k, 1)
        rec["picard_unconverged_steps"] = unconverged
        if out:
            with open(out, "w") as fh:
                json.dump(rec, fh)
        print("step %d t c/L_y %.2f |dW|/W %.2e alpha_e %.3f u_max/sigma_ce %.3f alpha_i %.3f (%.1f s)" % (
            k, k * tcl, snap["energy_error"], snap["electrons"]["alpha"], snap["electrons"]["u_max_over_sigma"],
            snap["ions"]["alpha"], time.time() - tstart), file=log, flush=True)
    rec["ms_per_step"] = 1e3 * rec["seconds"] / max(k, 1)
    if out:
        with open(out, "w") as fh:
            json.dump(rec, fh)
    return rec


def main(argv=None):
    ap = argparse.ArgumentParser(description="Table 2 fiducial run: background spectra, slope and cutoff")
    ap.add_argument("--steps", type=int, default=None, help="default: to t c / L_y = 7.77")
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--standard", action="store_true", help="the standard step (gbar = gamma(u^n))")
    ap.add_argument("--plain", action="store_true",
                    help="plain fixed-point passes (default: per-particle secant steps)")
    ap.add_argument("--mass-fp32", action="store_true", help="mixed precision with M stored in FP32")
    ap.add_argument("--out", default=None, help="write the record as JSON")
    ap.add_argument("--nx", type=int, default=None)
    ap.add_argument("--ny", type=int, default=None)
    ap.add_argument("--ppc", type=int, default=None, help="background particles per cell per species")
    ap.add_argument("--ppc-sheet", type=int, default=None)
    args = ap.parse_args(argv)
    over = {k: v for k, v in (("nx", args.nx), ("ny", args.ny), ("ppc", args.ppc), ("ppc_sheet", args.ppc_sheet))
            if v is not None}
    rec = run(args.steps, precision=args.precision, energy_conserving=not args.standard, secant=not args.plain,
              out=args.out, mass_fp32=args.mass_fp32, **over)
    last = rec["snapshots"][-1]
    print(json.dumps({"t_c_over_Ly": last["t_c_over_Ly"], "energy_error": last["energy_error"],
                      "electrons": last["electrons"], "ions": last["ions"], "ms_per_step": rec["ms_per_step"]}))


if __name__ == "__main__":
    main()
