"""The tearing run's set-up and diagnostics (Sec. 2, Sec. 3.1, Sec. 4.1,
Table 1): the growth-rate theory against the value the paper prints, the box
modes against the paper's mode numbering, the low-pass mode energies against
Parseval on a single cosine, the fit on an exact exponential, and the
electron-ion loading against the Maxwell-Juettner moments."""
import json
import math
import os

import numpy as np
import pytest
import torch
from scipy.special import kv

from paper_2509_11100_amd import harris, tearing

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_parameters.json")))["tearing_growth"]
WL = harris.workload("tearing2d_200x102")


def test_theory_growth_rate_matches_the_printed_value():
    g = tearing.gamma_max(WL)
    assert abs(g - GOLD["printed_gamma_th_a_over_c"]) < GOLD["printed_digits_tol"]
    # the maximum of f(k) = ka (1 - k^2 a^2) is at ka = 1/sqrt(3)
    hp = WL.harris
    ti = hp.T / max(WL.m)
    k0 = 1.0 / math.sqrt(3.0)
    for d in (1e-3, 1e-2, 0.1):
        assert tearing.gamma_theory(k0 + d, hp.u_d, hp.Gamma_d, ti) < g
        assert tearing.gamma_theory(k0 - d, hp.u_d, hp.Gamma_d, ti) < g
    # cold ions: the ion correction factor tends to 2
    assert abs(tearing.gamma_theory(k0, hp.u_d, hp.Gamma_d, 1e-16) / tearing.gamma_theory(k0, hp.u_d, hp.Gamma_d, ti)
               - (1.0 + 2.0 ** 1.75 * ti ** 0.25 / math.sqrt(math.pi))) < 1e-3


def test_box_modes_follow_the_paper_mode_numbering():
    modes = {m: ka for m, ka, _ in tearing.box_modes(WL)}
    for m, ka in GOLD["mode_ka"].items():
        assert round(modes[int(m)], 1) == ka
    assert round(modes[1], 1) == GOLD["printed_smallest_kmax_a"]
    assert max(modes) == 7 and all(0 < ka < 1 for ka in modes.values())


def test_mode_energies_are_parseval_on_a_cosine():
    nx, ny, dx = WL.nx, WL.ny, WL.dx
    x = (np.arange(nx) + 0.5) * dx
    A, m = 0.37, 4
    by = np.tile(A * np.cos(2 * math.pi * m * x / (nx * dx)) + 1.5, (ny, 1))
    B = torch.zeros(3, nx * ny, dtype=torch.float64)
    B[1] = torch.as_tensor(by.reshape(-1))
    e = tearing.mode_energies(B, WL, 7)
    direct = ((by - 1.5) ** 2).sum() * dx * dx / (8 * math.pi)
    assert abs(e[m - 1] - direct) < 1e-12 * direct
    assert np.all(np.delete(e, m - 1) < 1e-20 * direct)


def test_fit_recovers_an_exact_exponential_inside_the_window():
    t = np.linspace(0, 3, 301)
    e = 2.5 * np.exp(2 * 0.8 * t)
    e[t > 1.6] *= 7.0     # outside the window: ignored
    e[t < 0.4] *= 0.1
    assert abs(tearing.fit_growth(t, e, 0.5, 1.5) - 0.8) < 1e-12


def test_electron_ion_loading_moments():
    wl = harris.workload("tearing2d_200x102", nx=4, ppc=64)
    p = harris.make_particles(wl)
    sp, w, u = p["species"], p["w"], p["u"]
    hp = wl.harris
    assert np.count_nonzero(sp == 0) == np.count_nonzero(sp == 1) == wl.ncells * wl.ppc
    # pair loading: equal weight of ions and electrons in every cell
    wi = np.bincount(p["cell"][sp == 0], w[sp == 0], wl.ncells)
    we = np.bincount(p["cell"][sp == 1], w[sp == 1], wl.ncells)
    np.testing.assert_allclose(wi, we, rtol=1e-12)
    # total number: two sheets of integral 2 a n0 per unit length along x
    X = wl.nx * wl.dx
    assert abs(wi.sum() / (2 * 2 * hp.a * hp.n0 * X) - 1) < 0.02
    gam = np.sqrt(1 + (u * u).sum(0))   # u is the proper velocity gamma v / c
    y = (p["cell"] // wl.nx + p["off"][1]) * wl.dx - 0.5 * wl.ny * wl.dx
    for s, (tol_g, tol_u) in enumerate([(0.005, 0.15), (0.02, 0.3)]):
        th = hp.T / wl.m[s]
        # lab-frame moments of a drifting Maxwell-Juettner gas per particle:
        # <gamma> = Gamma_d h - theta / Gamma_d and <u_drift> = u_d h, with
        # h = K3(1/theta) / K2(1/theta) the enthalpy per unit rest energy
        h = kv(3, 1 / th) / kv(2, 1 / th)
        sel = sp == s
        assert abs(gam[sel].mean() / (hp.Gamma_d * h - th / hp.Gamma_d) - 1) < tol_g
        # drift: ions along +z on the upper sheet, electrons along -z
        sgn = np.where(y[sel] > 0, 1.0, -1.0) * (1.0 if wl.q[s] > 0 else -1.0)
        uz = (sgn * u[2][sel]).mean()
        assert abs(uz / (hp.u_d * h) - 1) < tol_u
