"""The relativistic tearing run (Sec. 3.1) and its growth-rate diagnostic.

Runs the electron-ion double Harris sheet of the tearing study
(``harris.WORKLOADS["tearing2d_200x102"]``: m_i/m_e = 100, T = 10 m_e c^2,
u_d/c = 0.05, a = 20 rho_Le,R, dx = 5 rho_Le,R, dt omega_pe0 = 0.758, 256
particles per cell per species, no background, no seed, a box of
1000 x 510 rho_Le,R) on the GPU path, one
whole step (deposit, field solve, push with re-sort) at a time, and records
every ``every`` steps:

* the energy of B_y in each Fourier mode m along x (k = 2 pi m / X for the
  box length X), summed over y, and its low-pass sum over 0 < k a < 1, the
  quantity the paper fits;
* the total energy (kinetic + electric + magnetic, FP64).

The growth rate is the slope of ln(low-pass energy) / 2 fitted over
t gamma_th in [0.5, 1.5] (the paper's standard window); gamma_th, which also
sets the time unit, is the linear theory of Sec. 2 (gamma_th a / c with
f(k) = ka (1 - k^2 a^2)) at its maximum, ka = 1/sqrt(3).  Each box mode gets
its own fit over the same window; k_max a is the mode with the largest one.

Usage (GPU): python -m paper_2509_11100_amd.tearing --steps 45000 --every 100
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np
from typing import Optional

from . import harris


def gamma_theory(ka: float, u_d: float, Gamma_d: float, theta_i: float) -> float:
    """gamma_th a / c of the tearing mode at k a (Sec. 2): relativistic
    electrons, non-relativistic ions of temperature theta_i = T / (m_i c^2)."""
    f = ka * (1.0 - ka * ka)
    corr = 2.0 / (1.0 + 2.0 ** 1.75 * theta_i ** 0.25 / math.sqrt(math.pi))
    return 2.0 * math.sqrt(2.0) / math.pi * f * u_d ** 1.5 / Gamma_d ** 2.5 * corr


def gamma_max(wl: harris.Workload) -> float:
    """gamma_th a / c at the fastest-growing k a = 1/sqrt(3)."""
    hp = wl.harris
    return gamma_theory(1.0 / math.sqrt(3.0), hp.u_d, hp.Gamma_d, hp.T / max(wl.m))


def box_modes(wl: harris.Workload):
    """(m, k a, gamma_th a / c) of the box modes along x with 0 < k a < 1."""
    hp = wl.harris
    X = wl.nx * wl.dx
    theta_i = hp.T / max(wl.m)
    out = []
    m = 1
    while True:
        ka = 2.0 * math.pi * m * hp.a / X
        if ka >= 1.0:
            break
        out.append((m, ka, gamma_theory(ka, hp.u_d, hp.Gamma_d, theta_i)))
        m += 1
    return out


def mode_energies(B, wl: harris.Workload, mmax: int):
    """Energy of B_y in the modes m = 1..mmax along x, summed over y:
    V / (8 pi) sum_j 2 |F_m(j)|^2 / nx (Parseval, one-sided transform)."""
    import torch

    by = B[1].view(wl.ny, wl.nx)
    F = torch.fft.rfft(by, dim=1)
    p = (F.real ** 2 + F.imag ** 2).sum(dim=0)[1:mmax + 1]
    V = wl.dx * wl.dx
    return (p * (2.0 / wl.nx) * V / (8.0 * math.pi)).cpu().numpy()


def fit_growth(t: np.ndarray, e: np.ndarray, t0: float, t1: float) -> float:
    """Slope of ln(e) / 2 over t in [t0, t1] (least squares)."""
    sel = (t >= t0) & (t <= t1) & (e > 0)
    if sel.sum() < 3:
        return float("nan")
    A = np.stack([t[sel], np.ones(int(sel.sum()))], axis=1)
    slope = np.linalg.lstsq(A, np.log(e[sel]), rcond=None)[0][0]
    return 0.5 * float(slope)


def summarize(wl: harris.Workload, rec: dict, window=(0.5, 1.5)) -> dict:
    """Growth rates (gamma a / c) and energy errors from the records of run():
    the low-pass fit, one fit per box mode, k_max a (the mode with the
    largest fitted rate), the dominant mode at t gamma_th = 1.5, the largest
    relative energy error up to t gamma_th = 1 and the error at the end."""
    hp = wl.harris
    modes = box_modes(wl)
    gth = gamma_max(wl)
    t = np.asarray(rec["t_gamma_th"])
    low = np.asarray(rec["lowpass"])
    em = np.asarray(rec["modes"])
    Wt = np.asarray(rec["W"])[:, 3]
    # the fits give the rate in units of gamma_th
    gm = fit_growth(t, low, *window) * gth
    per_mode = [fit_growth(t, em[:, i], *window) * gth for i in range(len(modes))]
    fastest = int(np.nanargmax(per_mode)) if np.isfinite(per_mode).any() else 0
    dominant = int(np.argmax(em[int(np.argmin(np.abs(t - 1.5)))]))
    err1 = float(np.max(np.abs(Wt[t <= 1.0] - Wt[0])) / Wt[0])
    return {
        "workload": wl.name, "ppc": wl.ppc, "dt_wpe": wl.dt, "a": hp.a, "rho_Le_R": hp.u_d * hp.a,
        "box_modes": [{"m": m, "ka": ka, "gamma_th_a_over_c": g} for m, ka, g in modes],
        "gamma_th_a_over_c": gth, "fit_window_t_gamma_th": list(window),
        "gamma_m_a_over_c_lowpass": gm, "gamma_m_a_over_c_per_mode": per_mode,
        "k_max_a": modes[fastest][1], "dominant_ka_at_t_gamma_th_1.5": modes[dominant][1],
        "energy_error_max_to_t_gamma_th_1": err1,
        "energy_error_end": float(abs(Wt[-1] - Wt[0]) / Wt[0]),
        "t_gamma_th_end": float(t[-1]),
    }


def run(steps: int, every: int, precision: str = "fp64", rtol: float = 1e-10, seed=None, log=sys.stdout,
        energy_conserving: bool = False, picard_tol: Optional[float] = None, **overrides):
    import torch

    from . import relsim

    wl = harris.workload("tearing2d_200x102", **overrides)
    hp = wl.harris
    modes = box_modes(wl)
    t_unit = hp.a / gamma_max(wl)  # 1 / gamma_th in time units (c = 1)
    p = harris.make_particles(wl, seed=seed)
    E, B = harris.make_fields(wl)
    n = p["w"].shape[0]
    ctx = relsim.Context(dim=2, nx=wl.nx, ny=wl.ny, dx=wl.dx, dt=wl.dt, precision=precision, q=wl.q, m=wl.m,
                         max_particles=n, gmres_rtol=rtol, gmres_restart=30, gmres_maxit=5000)
    parts = relsim.Particles(ctx).load(p["cell"], p["species"], p["off"], p["u"], p["w"], p["bin_start"])
    step = relsim.Step(ctx, parts, torch.as_tensor(E).cuda(), torch.as_tensor(B).cuda(),
                       energy_conserving=energy_conserving, picard_tol=picard_tol)
    mmax = len(modes)
    rec = {"step": [], "t_gamma_th": [], "lowpass": [], "modes": [], "W": [], "gmres_iters": [], "picard_iters": []}

    def record(k):
        em = mode_energies(step.B, wl, mmax)
        W = step.energy()
        rec["step"].append(k)
        rec["t_gamma_th"].append(k * wl.dt / t_unit)
        rec["modes"].append([float(x) for x in em])
        rec["lowpass"].append(float(em.sum()))
        rec["W"].append([float(x) for x in W])
        rec["gmres_iters"].append(int(step.iters))
        rec["picard_iters"].append(int(step.picard_iters))

    t0 = time.time()
    record(0)
    k = 0
    while k < steps:
        nstep = min(every, steps - k)
        step(nstep)
        k += nstep
        record(k)
        if k % (every * 50) == 0 or k == steps:
            print("step %d  t gamma_th %.3f  low-pass %.3e  |W - W0|/W0 %.2e  %.1f s"
                  % (k, rec["t_gamma_th"][-1], rec["lowpass"][-1],
                     abs(rec["W"][-1][3] - rec["W"][0][3]) / rec["W"][0][3], time.time() - t0), file=log, flush=True)
    torch.cuda.synchronize()
    wall = time.time() - t0
    summary = summarize(wl, rec)
    summary.update({"precision": precision, "energy_conserving": energy_conserving, "particles": int(n), "steps": steps,
                    "wall_s": wall, "ms_per_step": 1e3 * wall / max(steps, 1)})
    return summary, rec


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--steps", type=int, default=None, help="default: to t gamma_th = --t-end")
    ap.add_argument("--t-end", type=float, default=2.0, help="run length in units of 1 / gamma_th")
    ap.add_argument("--every", type=int, default=100)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--rtol", type=float, default=1e-10)
    ap.add_argument("--seed", type=int, default=None)
    ap.add_argument("--energy-conserving", action="store_true",
                    help="gbar = (gamma^n + gamma^{n+1})/2 by fixed-point iteration (exact energy)")
    ap.add_argument("--picard-tol", type=float, default=None, help="default 1e-12 (FP64), 1e-6 (mixed)")
    ap.add_argument("--ppc", type=int, default=None, help="particles per cell per species (default 256)")
    ap.add_argument("--dt-wpe", type=float, default=None, help="time step in 1 / omega_pe0 (default 0.758)")
    ap.add_argument("--dx-rho", type=float, default=None,
                    help="cell size in rho_Le,R (default 5); the box stays 1000 x 510 rho_Le,R, rounded to cells")
    ap.add_argument("--out", default=None, help="write the summary and the records as JSON")
    args = ap.parse_args(argv)
    over = {k: v for k, v in (("ppc", args.ppc), ("dt_wpe", args.dt_wpe)) if v is not None}
    if args.dx_rho is not None:
        over.update(dx_over_a=args.dx_rho / 20.0, nx=int(round(1000.0 / args.dx_rho)),
                    ny=int(round(510.0 / args.dx_rho)))
    if args.steps is None:
        wl = harris.workload("tearing2d_200x102", **over)
        args.steps = int(math.ceil(args.t_end * wl.harris.a / gamma_max(wl) / wl.dt))
    summary, rec = run(args.steps, args.every, args.precision, args.rtol, args.seed,
                       energy_conserving=args.energy_conserving, picard_tol=args.picard_tol, **over)
    print(json.dumps(summary))
    if args.out:
        with open(args.out, "w") as f:
            json.dump({"summary": summary, "records": rec}, f)
    return 0


if __name__ == "__main__":
    sys.exit(main())
