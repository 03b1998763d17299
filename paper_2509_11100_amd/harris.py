"""Seeded synthetic inputs: the double relativistic Harris sheet.

This module only prepares inputs.  It holds none of the particle or field
arithmetic of the semi-implicit step, and it imports nothing else from this
package besides the parameter calculator, so both the GPU path and the CPU
checker can take their inputs from here.

Setup (Schoeffler et al. 2025, Sec. 2):
  * two current sheets at y = +-L_y/2 in a periodic box y in [-L_y, L_y),
    i.e. the sheets sit at +-Y/4 for a box of height Y = 2 L_y;
  * each sheet: counter-drifting Maxwell-Juettner (MJ) populations boosted
    along +-z with drift speed v_d, density n0 sech^2((y -+ L_y/2)/a);
  * a uniform background of density n_b at rest;
  * B0 from pressure balance and a from Ampere's law (params.harris).

The paper prints the double-sheet B_x profile with a sign garble (its form is
3 B0 at y = 0 and does not reverse).  The profile used here reverses at both
sheets: B_x = B0 [tanh((y + L_y/2)/a) - tanh((y - L_y/2)/a) - 1].

The paper's tearing runs grow from noise; the workloads add a seed
delta B_y = eps B0 cos(2 pi x / X) at cell centres, uniform in y (and z), which
is divergence-free on the grid.  The particles do not depend on eps.

Loading: per cell and species, half the macro-particles belong to the sheet
population and half to the background; positions are uniform in the cell and
shared by the species (pair loading, exact charge neutrality); the
weight carries the density, w = n(y_p) V / (particles of that population per
cell).  A sheet particle drifts with the sign of the nearer sheet; positrons
(species 0, q = +1) drift along +z on the upper sheet and electrons (species 1,
q = -1) along -z.  MJ momenta come from an inverse-CDF table of
u^2 exp(-(gamma - 1)/theta); the drift boost uses the flipping method of
Zenitani (2015).

Layout of the generated particles: sorted by bin = cell * nspecies + species,
cells in natural order (i + nx (j + ny k)), so ``bin_start`` is known up front.
In 3D every z-layer of cells draws from its own stream (PCG64 seeded with
(seed, layer)), so layers can be generated in parallel or one at a time.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Dict, Optional

import numpy as np

from . import params as _params

N0 = 1.0 / (4.0 * math.pi)   # omega_pe0 = 1 with c = m_e = e = 1


@dataclass(frozen=True)
class Workload:
    """One synthetic double-Harris workload (sizes and physics knobs)."""

    name: str
    dim: int
    nx: int
    ny: int
    nz: int
    dx_over_a: float          # cell size in units of the sheet half thickness a
    ppc: int                  # macro-particles per cell per species
    cfl: float = 0.5          # dt = cfl * dx / c
    theta_s: float = 1.0      # sheet temperature T / (m_e c^2); species s samples T / (m_s c^2)
    beta_d: float = 0.3       # sheet drift speed
    nb_over_n0: float = 0.1   # background density ratio
    theta_b: float = 0.1      # background temperature T_b / (m_e c^2)
    eps: float = 0.01         # delta B_y seed amplitude / B0
    seed: int = 0
    steps: int = 10
    q: tuple = (1.0, -1.0)
    m: tuple = (1.0, 1.0)
    dt_wpe: Optional[float] = None  # if set, dt = dt_wpe / omega_pe0 (overrides cfl)
    # Separate populations (the nonlinear runs of Sec. 3.2): if ppc_sheet is
    # set, the sheet and the background are loaded as separate species, the
    # sheet ones first (q and m list both, e.g. ion sheet, electron sheet,
    # ion background, electron background), with ppc_sheet particles per
    # cell for each sheet species and ppc for each background species.
    ppc_sheet: Optional[int] = None
    # ... loaded only in the cells where the sheet density reaches sheet_cut
    # n0 somewhere in the cell (0: in every cell)
    sheet_cut: float = 0.0
    dx_over_de: Optional[float] = None  # if set, dx in units of d_e,C (background density; overrides dx_over_a)
    dt_wpb: Optional[float] = None      # if set, dt times the background omega_pe (overrides cfl and dt_wpe)

    @property
    def nspecies(self) -> int:
        return len(self.q)

    @property
    def ncells(self) -> int:
        return self.nx * self.ny * (self.nz if self.dim == 3 else 1)

    @property
    def split(self) -> bool:
        """Sheet and background loaded as separate species."""
        return self.ppc_sheet is not None

    @property
    def ppc_of_species(self) -> tuple:
        """Particles per cell of every species."""
        if not self.split:
            return (self.ppc,) * self.nspecies
        h = self.nspecies // 2
        return (self.ppc_sheet,) * h + (self.ppc,) * h

    @property
    def ppc_total(self) -> int:
        return int(sum(self.ppc_of_species))

    def sheet_rows(self) -> np.ndarray:
        """Separate populations: True for the cell rows (y index) that hold
        sheet particles (where n0 sech^2 of either sheet reaches sheet_cut
        n0 somewhere in the row)."""
        ny, dx = self.ny, self.dx
        Y = ny * dx
        lo = np.arange(ny) * dx - 0.5 * Y
        hi = lo + dx
        a = self.harris.a
        keep = np.zeros(ny, bool)
        for ys in (-0.25 * Y, 0.25 * Y):  # the two sheets, at +-L_y/2
            d = np.maximum(0.0, np.maximum(lo - ys, ys - hi))  # distance of the row from the sheet centre
            keep |= _sech2(d / a) >= self.sheet_cut
        return keep

    def counts(self) -> np.ndarray:
        """Particles per (cell, species), shape (ncells, nspecies)."""
        c = np.tile(np.asarray(self.ppc_of_species, dtype=np.int64), (self.ncells, 1))
        if self.split and self.sheet_cut > 0:
            assert self.dim == 2, "separate populations are a 2D loading"
            rows = self.sheet_rows()
            j = (np.arange(self.ncells) // self.nx) % self.ny
            c[~rows[j], : self.nspecies // 2] = 0
        return c

    @property
    def nparticles(self) -> int:
        if self.split and self.sheet_cut > 0:
            return int(self.counts().sum())
        return self.ncells * self.ppc_total

    @property
    def de_C(self) -> float:
        """Classical electron inertial length with the background density
        (the paper's d_e,C; electron mass 1)."""
        return math.sqrt(1.0 / (4.0 * math.pi * self.nb_over_n0 * N0))

    @property
    def harris(self) -> _params.HarrisParams:
        return _params.harris(N0, self.theta_s, self.beta_d)

    @property
    def dx(self) -> float:
        if self.dx_over_de is not None:
            return self.dx_over_de * self.de_C
        return self.dx_over_a * self.harris.a

    @property
    def dt(self) -> float:
        # omega_pe0 = 1 in these units (n0 = N0, m_e = e = c = 1); the
        # background omega_pe is sqrt(n_b / n0) of it
        if self.dt_wpb is not None:
            return self.dt_wpb / math.sqrt(self.nb_over_n0)
        return self.dt_wpe if self.dt_wpe is not None else self.cfl * self.dx

    @property
    def sigma_c(self) -> float:
        """Cold magnetisation of the background (derived, not imposed)."""
        return _params.sigma_cold(self.harris.B0, self.nb_over_n0 * N0, self.m[0])


# The workloads: 2D 64x32 (small, all parities), 2D 1024x512 (throughput),
# 2D 256x128 (adjoint), 3D 128x64x64, 3D 256x128x128 and 3D 512x256x256
# (536,870,912 particles: the particle count and mass-matrix size stated for
# the large 3D run).
WORKLOADS: Dict[str, Workload] = {
    "harris2d_64x32": Workload("harris2d_64x32", 2, 64, 32, 1, 0.5, 16, seed=1, steps=10),
    "harris2d_1024x512": Workload("harris2d_1024x512", 2, 1024, 512, 1, 1.0, 64, seed=2, steps=100),
    "harris2d_256x128": Workload("harris2d_256x128", 2, 256, 128, 1, 0.5, 32, seed=3, steps=20),
    "harris3d_128x64x64": Workload("harris3d_128x64x64", 3, 128, 64, 64, 0.5, 16, seed=4, steps=50),
    "harris3d_256x128x128": Workload("harris3d_256x128x128", 3, 256, 128, 128, 0.5, 8, seed=5, steps=20),
    "harris3d_512x256x256": Workload("harris3d_512x256x256", 3, 512, 256, 256, 0.5, 8, seed=6, steps=20),
    # The relativistic tearing run (Sec. 3.1, fiducial RelSIM case): ions and
    # electrons, m_i/m_e = 100, T = 10 m_e c^2 for both, u_d/c = 0.05, no
    # background, a / rho_Le,R = 20 (rho_Le,R = u_d a / c), dx = 5 rho_Le,R =
    # a / 4, dt omega_pe0 = 0.758, 256 particles per cell per species, no seed
    # (the instability grows from the particle noise).  Species 0: ions.
    # The box is 1000 x 510 rho_Le,R = 200 x 102 cells: 510 = twice the sheet
    # distance; along x the period is the one the mode numbering of Sec. 4.1
    # and the k_max a column of Table 1 imply (m = 4 at ka ~ 0.5, modes down
    # to ka ~ 0.1, so ka = 0.1257 m), twice the stated 2 L_x.
    "tearing2d_200x102": Workload("tearing2d_200x102", 2, 200, 102, 1, 0.25, 256, theta_s=10.0,
                                  beta_d=0.05 / math.sqrt(1.0 + 0.05 ** 2), nb_over_n0=0.0, eps=0.0, seed=7,
                                  steps=45000, q=(1.0, -1.0), m=(100.0, 1.0), dt_wpe=0.758),
}


# The fiducial nonlinear run of Table 2 (Sec. 3.2): ions and electrons,
# m_i/m_e = 100, T = 10 m_e c^2 for both species and both populations, proper
# drift u_d/c = 0.4, sigma_ci = 100 (n0/n_b = 269.26 from pressure balance;
# Ampere's law then gives a = 0.50 d_e,C), L_x = L_y = 50 d_i,C = 500 d_e,C
# (a box of 2 L_x x 2 L_y = 625 x 625 cells at dx = 1.6 d_e,C), dt omega_pe
# = 0.96, 256 sheet and 16 background particles per cell per species, no
# seed, to t c / L_y = 7.77 (4,047 steps).  Species: ion sheet, electron
# sheet, ion background, electron background.  The sheet particles fill the
# rows where the sheet density reaches 1e-6 n0 (6 rows per sheet at a = dx /
# 3.2; the density left out is below 3e-4 of the background): 16,340,000
# particles (sheet_cut = 0 puts 256 in every cell: 212,500,000).
_B_D_F3 = 0.4 / math.sqrt(1.0 + 0.4 ** 2)
_NB_F3 = 1.0 / _params.n0_over_nb_for_sigma(100.0, 10.0, 100.0, 0.4)
WORKLOADS["reconnection2d_625x625"] = Workload(
    "reconnection2d_625x625", 2, 625, 625, 1, 0.0, 16, theta_s=10.0, beta_d=_B_D_F3, nb_over_n0=_NB_F3,
    theta_b=10.0, eps=0.0, seed=8, steps=4047, q=(1.0, -1.0, 1.0, -1.0), m=(100.0, 1.0, 100.0, 1.0),
    ppc_sheet=256, sheet_cut=1e-6, dx_over_de=1.6, dt_wpb=0.96)


def workload(name: str, **overrides) -> Workload:
    wl = WORKLOADS[name]
    return replace(wl, **overrides) if overrides else wl


# ----------------------------------------------------------------------------
# Maxwell-Juettner sampling
# ----------------------------------------------------------------------------
def _mj_table(theta: float, npts: int = 1 << 15):
    gmax = 1.0 + 60.0 * theta
    umax = math.sqrt(gmax * gmax - 1.0)
    u = np.linspace(0.0, umax, npts)
    g = np.sqrt(1.0 + u * u)
    f = u * u * np.exp(-(g - 1.0) / theta)
    cdf = np.concatenate([[0.0], np.cumsum(0.5 * (f[1:] + f[:-1]) * np.diff(u))])
    cdf /= cdf[-1]
    return cdf, u


def sample_mj(rng: np.random.Generator, theta: float, n: int) -> np.ndarray:
    """Isotropic MJ momenta (u = gamma v / c), shape (3, n)."""
    cdf, ut = _mj_table(theta)
    umag = np.interp(rng.random(n), cdf, ut)
    cz = 2.0 * rng.random(n) - 1.0
    ph = 2.0 * math.pi * rng.random(n)
    sz = np.sqrt(np.maximum(0.0, 1.0 - cz * cz))
    return np.stack([umag * sz * np.cos(ph), umag * sz * np.sin(ph), umag * cz])


def boost_z(rng: np.random.Generator, u: np.ndarray, beta: np.ndarray) -> np.ndarray:
    """Boost rest-frame momenta along z by beta (array), flipping method."""
    g = np.sqrt(1.0 + (u * u).sum(axis=0))
    Gd = 1.0 / np.sqrt(1.0 - beta * beta)
    uz = u[2].copy()
    flip = -beta * uz / g > rng.random(u.shape[1])
    uz[flip] = -uz[flip]
    out = u.copy()
    out[2] = Gd * (uz + beta * g)
    return out


# ----------------------------------------------------------------------------
# Particles and fields
# ----------------------------------------------------------------------------
def _sech2(x: np.ndarray) -> np.ndarray:
    """sech^2 without overflow: 4 e^{-2|x|} / (1 + e^{-2|x|})^2."""
    e = np.exp(-2.0 * np.abs(x))
    return 4.0 * e / (1.0 + e) ** 2


def _sheet_momenta(wl: Workload, rng: np.random.Generator, species: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Drifting MJ momenta of sheet particles: temperature T / (m_s c^2),
    boosted along z by the drift speed with the sign of the nearer sheet and
    of the charge."""
    n = species.size
    us = np.empty((3, n))
    ms = np.asarray(wl.m)[species]
    for mv in sorted(set(wl.m)):
        sel = ms == mv
        if sel.any():
            us[:, sel] = sample_mj(rng, wl.theta_s / mv, int(sel.sum()))
    qv = np.asarray(wl.q)[species]
    beta = wl.beta_d * np.sign(y) * np.sign(qv)
    beta[beta == 0] = wl.beta_d
    return boost_z(rng, us, beta)


def _background_momenta(wl: Workload, rng: np.random.Generator, species: np.ndarray) -> np.ndarray:
    """MJ momenta at rest, temperature T_b / (m_s c^2)."""
    ub = np.empty((3, species.size))
    ms = np.asarray(wl.m)[species]
    for mv in sorted(set(wl.m)):
        sel = ms == mv
        if sel.any():
            ub[:, sel] = sample_mj(rng, wl.theta_b / mv, int(sel.sum()))
    return ub


def _generate_split(wl: Workload, rng: np.random.Generator, c0: int, c1: int) -> Dict[str, np.ndarray]:
    """Cells [c0, c1) of a workload with separate populations: per cell, the
    sheet species (ppc_sheet each) and then the background species (ppc
    each).  Within a population every species shares the positions (pair
    loading: each population is exactly neutral)."""
    hp = wl.harris
    S = wl.nspecies
    h = S // 2
    dx = wl.dx
    Y = wl.ny * dx
    Ly = 0.5 * Y
    V = dx * dx * (dx if wl.dim == 3 else 1.0)
    cnt = wl.counts()[c0:c1]                      # (cells, species)
    per = cnt.sum(1)
    cbeg = np.concatenate([[0], np.cumsum(per)])  # first particle of each cell
    n = int(cbeg[-1])
    cell = np.repeat(np.arange(c0, c1, dtype=np.int32), per)
    species = np.repeat(np.tile(np.arange(S, dtype=np.uint8), c1 - c0), cnt.reshape(-1))
    off = np.empty((wl.dim, n))
    w = np.empty(n)
    u = np.empty((3, n))
    # a population's positions are drawn once per cell and shared by its
    # species; the species of a cell sit one after the other
    start = np.zeros(c1 - c0, dtype=np.int64)     # first slot of the current species in each cell
    for pop in (0, 1):
        npp = cnt[:, pop * h]
        tot = int(npp.sum())
        pos = rng.random((wl.dim, tot))
        k = np.arange(tot) - np.repeat(np.concatenate([[0], np.cumsum(npp)[:-1]]), npp)  # index in the cell
        cidx = np.repeat(np.arange(c1 - c0), npp)
        for _ in range(h):
            off[:, cbeg[cidx] + start[cidx] + k] = pos
            start += npp
    j = (cell.astype(np.int64) // wl.nx) % wl.ny
    y = (j + off[1]) * dx - 0.5 * Y
    sheet = species < h
    dens = N0 * (_sech2((y[sheet] - 0.5 * Ly) / hp.a) + _sech2((y[sheet] + 0.5 * Ly) / hp.a))
    w[sheet] = dens * V / wl.ppc_sheet
    w[~sheet] = wl.nb_over_n0 * N0 * V / wl.ppc
    u[:, sheet] = _sheet_momenta(wl, rng, species[sheet], y[sheet])
    u[:, ~sheet] = _background_momenta(wl, rng, species[~sheet])
    return {"cell": cell, "species": species, "off": off, "u": u, "w": w}


def _generate(wl: Workload, rng: np.random.Generator, c0: int, c1: int) -> Dict[str, np.ndarray]:
    """Particles of cells [c0, c1) drawn from rng (bin order, no bin_start)."""
    if wl.split:
        return _generate_split(wl, rng, c0, c1)
    hp = wl.harris
    S, ppc = wl.nspecies, wl.ppc
    nc = c1 - c0
    n = nc * S * ppc
    # half the particles of a cell belong to the sheet and half to the
    # background; without a background all of them belong to the sheet
    n_sheet = ppc // 2 if wl.nb_over_n0 > 0 else ppc
    n_bg = ppc - n_sheet
    dx = wl.dx
    Y = wl.ny * dx
    Ly = 0.5 * Y
    V = dx * dx * (dx if wl.dim == 3 else 1.0)

    p = np.arange(n, dtype=np.int64)
    cell = (c0 + p // (S * ppc)).astype(np.int32)
    species = ((p // ppc) % S).astype(np.uint8)
    k_in = p % ppc
    is_sheet = k_in < n_sheet

    # pair loading: every species gets the same positions (and hence the
    # same weights), so the initial state is exactly charge neutral
    off1 = rng.random((wl.dim, nc, 1, ppc))
    off = np.broadcast_to(off1, (wl.dim, nc, S, ppc)).reshape(wl.dim, n).copy()
    j = (cell.astype(np.int64) // wl.nx) % wl.ny
    y = (j + off[1]) * dx - 0.5 * Y           # physical y in [-Y/2, Y/2)

    dens_sheet = N0 * (_sech2((y - 0.5 * Ly) / hp.a) + _sech2((y + 0.5 * Ly) / hp.a))
    w = np.where(is_sheet, dens_sheet * V / n_sheet, wl.nb_over_n0 * N0 * V / max(n_bg, 1))

    u = np.empty((3, n))
    ns = int(is_sheet.sum())
    masses = sorted(set(wl.m))
    if len(masses) == 1:
        # one mass (the pair plasma): one draw for all sheet particles
        us = sample_mj(rng, wl.theta_s / masses[0], ns)
    else:
        # the same temperature T for every species: theta = T / (m_s c^2)
        us = np.empty((3, ns))
        msh = np.asarray(wl.m)[species[is_sheet]]
        for mv in masses:
            sel = msh == mv
            us[:, sel] = sample_mj(rng, wl.theta_s / mv, int(sel.sum()))
    qv = np.asarray(wl.q)[species[is_sheet]]
    beta = wl.beta_d * np.sign(y[is_sheet]) * np.sign(qv)
    beta[beta == 0] = wl.beta_d
    u[:, is_sheet] = boost_z(rng, us, beta)
    if n - ns > 0:
        mbg = np.asarray(wl.m)[species[~is_sheet]]
        ub = np.empty((3, n - ns))
        for mv in sorted(set(wl.m)):
            sel = mbg == mv
            ub[:, sel] = sample_mj(rng, wl.theta_b / mv, int(sel.sum()))
        u[:, ~is_sheet] = ub
    return {"cell": cell, "species": species, "off": off, "u": u, "w": w}


def layer_rng(seed: int, k: int) -> np.random.Generator:
    """The stream of z-layer k of a 3D workload."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, k])))


def make_layers(wl: Workload, k0: int, k1: int, seed: Optional[int] = None) -> Dict[str, np.ndarray]:
    """Particles of the z-layers [k0, k1) of a 3D workload, in bin order.

    ``bin_start`` covers the bins of those layers and starts at 0.
    """
    assert wl.dim == 3 and 0 <= k0 <= k1 <= wl.nz
    seed = wl.seed if seed is None else seed
    nxy = wl.nx * wl.ny
    parts = [_generate(wl, layer_rng(seed, k), k * nxy, (k + 1) * nxy) for k in range(k0, k1)]
    out = {key: np.concatenate([q[key] for q in parts], axis=-1) for key in ("cell", "species", "off", "u", "w")}
    out["bin_start"] = _uniform_bins((k1 - k0) * nxy * wl.nspecies, wl.ppc_of_species)
    return out


def _uniform_bins(nbins: int, ppc) -> np.ndarray:
    """bin_start of nbins bins holding ppc particles each (ppc an int, or the
    per-species counts repeated cell after cell)."""
    if np.ndim(ppc) == 0:
        counts = np.full(nbins, ppc, dtype=np.int64)
    else:
        counts = np.tile(np.asarray(ppc, dtype=np.int64), nbins // len(ppc))
    bin_start = np.zeros(nbins + 1, dtype=np.int64)
    np.cumsum(counts, out=bin_start[1:])
    return bin_start.astype(np.int32)


def make_particles(wl: Workload, seed: Optional[int] = None, workers: int = 1) -> Dict[str, np.ndarray]:
    """Generate the bin-sorted particle state in FP64.

    Returns a dict with ``cell`` (int32, natural cell index), ``species``
    (uint8), ``off`` (dim, n) offsets in [0,1), ``u`` (3, n), ``w`` (n), and
    ``bin_start`` (int32, ncells * nspecies + 1).  3D workloads are generated
    layer by layer (``workers`` > 1: in that many threads; numpy releases the
    interpreter lock in the array work).
    """
    seed = wl.seed if seed is None else seed
    if wl.dim == 2 and wl.split:
        # separate populations: blocks of rows, each from its own stream,
        # generated independently (in `workers` threads) into one array
        rows = max(1, min(wl.ny, (1 << 21) // max(1, wl.nx * wl.ppc_total)))
        nblk = (wl.ny + rows - 1) // rows
        cnt = wl.counts()
        n = int(cnt.sum())
        out = {"cell": np.empty(n, np.int32), "species": np.empty(n, np.uint8), "off": np.empty((2, n)),
               "u": np.empty((3, n)), "w": np.empty(n)}
        row_start = np.concatenate([[0], np.cumsum(cnt.reshape(wl.ny, -1).sum(1))])

        def put_rows(b):
            j0, j1 = b * rows, min(wl.ny, (b + 1) * rows)
            q = _generate_split(wl, layer_rng(seed, b), j0 * wl.nx, j1 * wl.nx)
            sl = slice(int(row_start[j0]), int(row_start[j1]))
            for key in ("cell", "species", "w"):
                out[key][sl] = q[key]
            out["off"][:, sl] = q["off"]
            out["u"][:, sl] = q["u"]

        if workers > 1:
            from concurrent.futures import ThreadPoolExecutor

            with ThreadPoolExecutor(workers) as ex:
                list(ex.map(put_rows, range(nblk)))
        else:
            for b in range(nblk):
                put_rows(b)
        out["bin_start"] = np.concatenate([[0], np.cumsum(cnt.reshape(-1))]).astype(np.int32)
        return out
    if wl.dim == 2:
        out = _generate(wl, np.random.Generator(np.random.PCG64(seed)), 0, wl.ncells)
        out["bin_start"] = _uniform_bins(wl.ncells * wl.nspecies, wl.ppc_of_species)
        return out
    n = wl.nparticles
    out = {"cell": np.empty(n, np.int32), "species": np.empty(n, np.uint8), "off": np.empty((3, n)),
           "u": np.empty((3, n)), "w": np.empty(n)}
    per = wl.nx * wl.ny * wl.ppc_total

    def put(k):
        q = make_layers(wl, k, k + 1, seed)
        sl = slice(k * per, (k + 1) * per)
        for key in ("cell", "species", "w"):
            out[key][sl] = q[key]
        out["off"][:, sl] = q["off"]
        out["u"][:, sl] = q["u"]

    if workers > 1:
        from concurrent.futures import ThreadPoolExecutor

        with ThreadPoolExecutor(workers) as ex:
            list(ex.map(put, range(wl.nz)))
    else:
        for k in range(wl.nz):
            put(k)
    out["bin_start"] = _uniform_bins(wl.ncells * wl.nspecies, wl.ppc_of_species)
    return out


def make_fields(wl: Workload, eps: Optional[float] = None):
    """Initial E (zero, at nodes) and B (at cell centres), both (3, ncells) FP64."""
    eps = wl.eps if eps is None else eps
    hp = wl.harris
    dx = wl.dx
    nx, ny = wl.nx, wl.ny
    nz = wl.nz if wl.dim == 3 else 1
    Y = ny * dx
    X = nx * dx
    Ly = 0.5 * Y
    yc = (np.arange(ny) + 0.5) * dx - 0.5 * Y
    xc = (np.arange(nx) + 0.5) * dx
    bx = hp.B0 * (np.tanh((yc + 0.5 * Ly) / hp.a) - np.tanh((yc - 0.5 * Ly) / hp.a) - 1.0)
    by = eps * hp.B0 * np.cos(2.0 * math.pi * xc / X)
    B = np.zeros((3, nz, ny, nx))
    B[0] = bx[None, :, None]
    B[1] = by[None, None, :]
    E = np.zeros((3, nz * ny * nx))
    return E, B.reshape(3, -1).copy()


def seed_direction(wl: Workload) -> np.ndarray:
    """d B / d eps: the seed pattern B0 cos(2 pi x / X) in B_y, shape (3, ncells)."""
    _, B1 = make_fields(wl, eps=1.0)
    _, B0 = make_fields(wl, eps=0.0)
    return B1 - B0
