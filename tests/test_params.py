"""Parameter calculator against the worked values the paper prints
(tests/golden/paper_parameters.json, each entry citing its section)."""
import json
import math
import os

import numpy as np

from paper_2509_11100_amd import harris, params

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_parameters.json")))


def test_tearing_larmor_ratio():
    t = GOLD["tearing_setup"]
    # a / rho_Le,R = c / u_d  and  a / rho_Li,C = v_Ti / u_d
    assert abs(1.0 / params.larmor_relativistic_over_a(t["u_d"]) - t["a_over_rho_LeR"]) < 1e-12
    r = 1.0 / params.larmor_classical_over_a(t["T_over_me"], t["mass_ratio"], t["u_d"])
    assert round(r, 2) == t["printed_a_over_rho_LiC"]


def test_osiris_courant_number():
    t = GOLD["osiris_timestep"]
    T = 10.0
    rho = params.larmor_relativistic(T, 1.0, 0.05, harris.N0)
    dx = t["dx_over_rho_LeR"] * rho
    assert abs(t["dt_omega_pe0"] / dx - t["printed_dt_c_over_dx"]) < t["printed_tol"]


def test_sigma_convention_and_density_ratio():
    t = GOLD["nonlinear_fiducial"]
    mi = t["mass_ratio"]
    T = t["T_over_me"]
    ratio = params.n0_over_nb_for_sigma(t["sigma_ci"], T, mi, t["u_d"])
    assert round(ratio, 1) == t["printed_n0_over_nb"]
    # consistency: B0 from pressure balance with that ratio gives sigma_ci back
    n0 = harris.N0
    nb = n0 / ratio
    Gd = params.gamma_from_proper(t["u_d"])
    hp = params.harris(n0, T, t["u_d"] / Gd)
    assert abs(params.sigma_cold(hp.B0, nb, mi) - t["sigma_ci"]) < 1e-9
    # hot electron magnetisation with h = 4T
    assert abs(params.sigma_hot(hp.B0, nb, T) - t["printed_sigma_he"]) < 1e-9
    # 2 L_y / (sigma_ce rho_0e) at L_y = 50 d_i,C
    sce = params.sigma_cold(hp.B0, nb, 1.0)
    di = params.inertial_length_classical(mi, nb)
    rho0e = params.nominal_larmor(hp.B0, 1.0)
    assert abs(2 * t["L_over_di"] * di / (sce * rho0e) - t["printed_2L_over_sigma_rho0e"]) < 1e-9


def test_harris_balance_and_ampere_in_code_units():
    hp = params.harris(harris.N0, 1.0, 0.3)
    assert abs(hp.Gamma_d - 1.0 / math.sqrt(1 - 0.09)) < 1e-15
    # pressure balance: B0^2/(8 pi) = (2 n0) T / Gamma_d
    assert abs(hp.B0 ** 2 / (8 * math.pi) - 2 * harris.N0 * 1.0 / hp.Gamma_d) < 1e-14
    # Ampere: c B0 / a = 4 pi e (2 n0) v_d
    assert abs(hp.B0 / hp.a - 4 * math.pi * 2 * harris.N0 * 0.3) < 1e-14
    assert abs(hp.B0 - 1.953396) < 1e-6 and abs(hp.a - 3.255660) < 1e-6


def test_harris_fields_reverse_and_seed_is_divergence_free():
    wl = harris.workload("harris2d_64x32")
    E, B = harris.make_fields(wl)
    bx = B[0].reshape(wl.ny, wl.nx)[:, 0]
    hp = wl.harris
    assert bx[wl.ny // 2] > 0.99 * hp.B0 and bx[0] < -0.99 * hp.B0 and bx[-1] < -0.99 * hp.B0
    by = B[1].reshape(wl.ny, wl.nx)
    assert np.allclose(by, by[0:1, :])
    assert abs(by.max() - wl.eps * hp.B0 * math.cos(math.pi / wl.nx)) < 1e-12
    assert np.all(E == 0)


def test_harris_particles_layout_and_moments():
    wl = harris.workload("harris2d_64x32")
    p = harris.make_particles(wl)
    n = wl.nparticles
    assert p["off"].shape == (2, n) and p["u"].shape == (3, n)
    assert np.all((p["off"] >= 0) & (p["off"] < 1))
    bins = p["cell"].astype(np.int64) * 2 + p["species"]
    assert np.all(np.diff(bins) >= 0)
    assert np.array_equal(np.searchsorted(bins, np.arange(wl.ncells * 2 + 1)), p["bin_start"])
    # total charge is zero and total sheet current matches Ampere's law
    q = np.asarray(wl.q)[p["species"]]
    assert abs((q * p["w"]).sum()) < 1e-9 * p["w"].sum()
    g = np.sqrt(1 + (p["u"] ** 2).sum(0))
    y = ((p["cell"] // wl.nx) + p["off"][1]) * wl.dx - 0.5 * wl.ny * wl.dx
    upper = y > 0
    Jz_up = (q * p["w"] * p["u"][2] / g)[upper].sum()
    # sheet current per unit length in x: integral of J_z dy = c B0 (2) / (4 pi) ... per box width X
    X = wl.nx * wl.dx
    expect = 2 * wl.harris.B0 * X / (4 * math.pi)
    assert abs(Jz_up - expect) < 0.05 * expect
