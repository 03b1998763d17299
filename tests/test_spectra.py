"""CPU pins of the spectrum diagnostics and of the Table 2 workload (Sec. 3.2,
Sec. 4.2, Table 2): a histogram that conserves the weight, slope and cutoff
recovered from power laws whose slope and cutoff are known, and the loading
of the fiducial sheet (magnetisation, sizes, populations)."""
import math

import numpy as np
import pytest

from paper_2509_11100_amd import harris, spectra


def test_spectrum_integrates_to_the_total_weight():
    rng = np.random.default_rng(1)
    u = 10 ** rng.uniform(-1.5, 5.5, 100000)
    w = rng.random(100000)
    f = spectra.spectrum(u, w)
    np.testing.assert_allclose((f * np.diff(spectra.EDGES)).sum(), w.sum(), rtol=1e-12)


def test_fit_is_exact_on_a_noise_free_power_law():
    uc = spectra.centres()
    f = 3.7 * uc ** -1.35
    alpha, amp = spectra.fit_power_law(uc, f, 100.0, 4000.0)
    assert abs(alpha + 1.35) < 1e-10 and abs(amp - 3.7) < 1e-8
    # no cutoff inside the populated range: the largest bin
    assert spectra.cutoff(uc, f, alpha, amp, 100.0) == uc[-1]


@pytest.mark.parametrize("alpha", [-1.1, -1.35, -1.5])
def test_slope_and_cutoff_of_a_sampled_power_law(alpha):
    """Samples of f(u) ~ u^alpha exp(-u / u_c), u_c = 2e4 (power law on
    [10, 2e5] thinned with probability exp(-u/u_c)): the fit over [30, 1000]
    recovers alpha within 0.03 and the point where f falls a factor e below
    the fit lands within 30 % of u_c."""
    rng = np.random.default_rng(int(-100 * alpha))
    n = 4_000_000
    a1 = alpha + 1.0
    lo, hi, uc = 10.0, 2e5, 2e4
    u = (lo ** a1 + rng.random(n) * (hi ** a1 - lo ** a1)) ** (1.0 / a1)  # inverse CDF of u^alpha
    u = u[rng.random(n) < np.exp(-u / uc)]
    f = spectra.spectrum(u, np.ones(u.size))
    res = spectra.analyse(f, 30.0, 1000.0, sigma=1e5)
    assert abs(res["alpha"] - alpha) < 0.03, res
    assert 0.7 * uc < res["u_max"] < 1.3 * uc, res
    assert abs(res["u_max_over_sigma"] - res["u_max"] / 1e5) < 1e-15


def test_local_slope_of_a_power_law():
    uc = spectra.centres()
    s = spectra.local_slope(uc, uc ** -2.0)
    np.testing.assert_allclose(s[8:-8], -2.0, rtol=1e-10)


def test_fiducial_workload_matches_the_paper():
    """Sec. 3.2: sigma_ci = 100 with n0/n_b = 269.3, a/d_e,C = 0.5 from
    pressure balance and Ampere's law at T = 10 m_e c^2 and u_d/c = 0.4,
    L_x = L_y = 500 d_e,C at dx = 1.6 d_e,C, dt omega_pe = 0.96; 16 and 256
    particles per cell per species in the background and the sheet."""
    wl = harris.workload("reconnection2d_625x625")
    hp = wl.harris
    assert abs(1.0 / wl.nb_over_n0 - 269.26) < 0.01
    sci = hp.B0 ** 2 / (4 * math.pi * wl.nb_over_n0 * harris.N0 * 100.0)
    assert abs(sci - 100.0) < 1e-9
    assert abs(spectra.sigma_ce(wl) - 1e4) < 1e-6
    assert abs(hp.a / wl.de_C - 0.5) < 1e-3
    assert abs(hp.u_d - 0.4) < 1e-12
    assert abs(wl.dx / wl.de_C - 1.6) < 1e-12
    assert abs(0.5 * wl.ny * wl.dx / wl.de_C - 500.0) < 1e-9
    assert abs(wl.dt * math.sqrt(wl.nb_over_n0) - 0.96) < 1e-12  # omega_pe0 = 1 in code units
    assert wl.ppc_of_species == (256, 256, 16, 16)
    # the sheet populations fill the 6 rows around each sheet where n0 sech^2
    # reaches 1e-6 n0; with no cut, every cell
    rows = np.nonzero(wl.sheet_rows())[0]
    np.testing.assert_array_equal(rows, [153, 154, 155, 156, 157, 158, 466, 467, 468, 469, 470, 471])
    assert wl.nparticles == 625 * 625 * 32 + 12 * 625 * 512
    assert harris.workload("reconnection2d_625x625", sheet_cut=0.0).nparticles == 625 * 625 * 544


def test_separate_population_loading():
    """A cut-down fiducial sheet: bin layout by species, each population
    neutral on its own, background weights uniform, sheet weights carrying
    n0 sech^2, drifts of opposite sign for the two charges."""
    wl = harris.workload("reconnection2d_625x625", nx=8, ny=24, ppc=4, ppc_sheet=256)
    p = harris.make_particles(wl, workers=2)
    S = 4
    key = p["cell"].astype(np.int64) * S + p["species"]
    assert np.all(np.diff(key) >= 0)
    np.testing.assert_array_equal(p["bin_start"], np.searchsorted(key, np.arange(wl.ncells * S + 1)))
    q = np.asarray(wl.q)[p["species"]]
    for pop in ((0, 1), (2, 3)):
        sel = np.isin(p["species"], pop)
        assert abs((q[sel] * p["w"][sel]).sum()) <= 1e-12 * p["w"][sel].sum()
    bgw = p["w"][p["species"] >= 2]
    np.testing.assert_allclose(bgw, wl.nb_over_n0 * harris.N0 * wl.dx ** 2 / 4, rtol=1e-14)
    # the sheet's total weight is the integral of n0 sech^2 over the box
    Y = wl.ny * wl.dx
    sheet_w = p["w"][p["species"] == 1].sum()
    assert abs(sheet_w - harris.N0 * 2 * 2 * wl.harris.a * wl.nx * wl.dx) < 0.05 * sheet_w
    # sheet ions and electrons drift in opposite z directions on one sheet
    ys = ((p["cell"] // wl.nx) + p["off"][1]) * wl.dx - 0.5 * Y
    up = ys > 0
    uz_i = p["u"][2][(p["species"] == 0) & up]
    uz_e = p["u"][2][(p["species"] == 1) & up]
    assert uz_i.mean() * uz_e.mean() < 0
