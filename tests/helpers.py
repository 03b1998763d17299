"""Test-side glue: build oracle grids from workloads, convert the (cell, offset)
particle representation into physical positions, and small random inputs."""
from __future__ import annotations

import numpy as np

import oracle
from paper_2509_11100_amd import harris


def grid_of(wl: harris.Workload, nonrel: bool = False, theta: float = 0.5) -> oracle.Grid:
    return oracle.Grid(dim=wl.dim, nx=wl.nx, ny=wl.ny, nz=wl.nz if wl.dim == 3 else 1,
                       dx=wl.dx, dy=wl.dx, dz=wl.dx, dt=wl.dt, c=1.0, theta=theta,
                       nonrel=nonrel, q=wl.q, m=wl.m)


def positions(g: oracle.Grid, cell, off) -> np.ndarray:
    """Physical positions x[dim][n] from linear cell index and offsets."""
    cell = np.asarray(cell, dtype=np.int64)
    off = np.asarray(off, dtype=np.float64)
    i = cell % g.nx
    j = (cell // g.nx) % g.ny
    k = cell // (g.nx * g.ny)
    h = [g.dx, g.dy, g.dz]
    ijk = [i, j, k]
    return np.stack([(ijk[d] + off[d]) * h[d] for d in range(g.dim)])


def cell_and_offset(g: oracle.Grid, x):
    """Inverse of positions() (floor convention)."""
    h = [g.dx, g.dy, g.dz]
    ext = [g.nx, g.ny, g.nz]
    idx = []
    offs = []
    for d in range(g.dim):
        s = x[d] / h[d]
        fl = np.floor(s)
        offs.append(s - fl)
        idx.append(np.mod(fl.astype(np.int64), ext[d]))
    cell = idx[0] + g.nx * idx[1]
    if g.dim == 3:
        cell = cell + g.nx * g.ny * idx[2]
    return cell, np.stack(offs)


def periodic_diff(g: oracle.Grid, xa, xb) -> np.ndarray:
    """Minimum-image difference of two position arrays."""
    out = []
    for d in range(g.dim):
        L = g.L[d]
        dd = np.asarray(xa[d]) - np.asarray(xb[d])
        out.append(dd - L * np.round(dd / L))
    return np.stack(out)


def random_state(g: oracle.Grid, n: int, rng: np.random.Generator, umax: float = 2.0, bmax: float = 1.0,
                 emax: float = 0.5):
    """Random particles anywhere in the box plus random fields."""
    x = np.stack([rng.random(n) * g.L[d] for d in range(g.dim)])
    u = (2.0 * rng.random((3, n)) - 1.0) * umax
    w = 0.5 + rng.random(n)
    sp = rng.integers(0, len(g.q), n).astype(np.int32)
    B = (2.0 * rng.random((3, g.N)) - 1.0) * bmax
    E = (2.0 * rng.random((3, g.N)) - 1.0) * emax
    return x, u, w, sp, E, B


def normwise(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / (den if den > 0 else 1.0))


def maxrel(a, b) -> float:
    """max |a - b| / max |b| (the elementwise measure beside the normwise one)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.abs(b).max() if b.size else 0.0
    return float(np.abs(a - b).max() / (den if den > 0 else 1.0)) if a.size else 0.0


def check_rel(a, b, tol: float, what: str = ""):
    """Gate both ||a - b|| / ||b|| and max |a - b| / max |b| at tol; returns
    the two errors."""
    nw, mx = normwise(a, b), maxrel(a, b)
    assert nw < tol, "%s normwise %.3e >= %.1e" % (what, nw, tol)
    assert mx < tol, "%s max-abs/max-ref %.3e >= %.1e" % (what, mx, tol)
    return nw, mx


def check_disp(dx, disp, tol: float, what: str = "positions"):
    """Position error relative to the displacement of the step, normwise and
    as max |dx| / max |displacement|."""
    dx = np.asarray(dx, dtype=np.float64)
    disp = np.asarray(disp, dtype=np.float64)
    nw = float(np.linalg.norm(dx) / np.linalg.norm(disp))
    mx = float(np.abs(dx).max() / np.abs(disp).max()) if dx.size else 0.0
    assert nw < tol, "%s normwise %.3e >= %.1e" % (what, nw, tol)
    assert mx < tol, "%s max-abs/max-displacement %.3e >= %.1e" % (what, mx, tol)
    return nw, mx
