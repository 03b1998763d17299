"""GPU-side test glue: contexts and particle sets built from the same seeded
inputs the oracle receives."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from tests.helpers import positions


def need_gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def make_ctx(g: oracle.Grid, precision: str, max_particles: int, rtol: float = 1e-13, **kw):
    from paper_2509_11100_amd import relsim

    return relsim.Context(dim=g.dim, nx=g.nx, ny=g.ny, nz=g.nz if g.dim == 3 else 1, dx=g.dx, dy=g.dy, dz=g.dz,
                          dt=g.dt, c=g.c, theta=g.theta, precision=precision, q=tuple(g.q), m=tuple(g.m),
                          max_particles=max(int(max_particles), 1), gmres_rtol=rtol,
                          nonrelativistic=g.nonrel, **kw)


def load(ctx, cell, species, off, u, w, bin_start=None):
    from paper_2509_11100_amd import relsim

    return relsim.Particles(ctx).load(cell, species, off, u, w, bin_start)


def rounded(precision: str, a):
    """The values a mixed-precision run actually holds (teacher forcing)."""
    a = np.asarray(a, dtype=np.float64)
    return a.astype(np.float32).astype(np.float64) if precision == "mixed" else a


def host_state(g: oracle.Grid, parts):
    """Front particle state on the host, with oracle positions."""
    cell, sp, off, u, w, bs = parts.to_host()
    off64 = off.astype(np.float64)
    return {"cell": cell, "species": sp, "off": off64, "u": u.astype(np.float64), "w": w.astype(np.float64),
            "bin_start": bs, "x": positions(g, cell, off64)}


def random_cells(g: oracle.Grid, n: int, rng, umax=2.0, empty_frac=0.0):
    """Random particles with (cell, offset) coordinates; optionally leave a
    fraction of the cells empty (ragged occupancy)."""
    ncell = g.N
    allowed = np.arange(ncell)
    if empty_frac > 0:
        allowed = allowed[rng.random(ncell) >= empty_frac]
        if allowed.size == 0:
            allowed = np.arange(1)
    cell = rng.choice(allowed, n).astype(np.int32)
    off = rng.random((g.dim, n))
    u = (2 * rng.random((3, n)) - 1) * umax
    w = 0.5 + rng.random(n)
    sp = rng.integers(0, len(g.q), n).astype(np.uint8)
    return cell, sp, off, u, w
