"""The stored half of the mass matrix (CPU): the test-side index bookkeeping
that rebuilds the full [noff][9][N] layout from the slots the library keeps,
checked against the oracle's full deposit and against exactly symmetric
synthetic blocks."""
import numpy as np
import pytest

import oracle
from tests.helpers import full_at_nodes, full_from_half, m_centre, random_state, stored_half


def grid(dim):
    return oracle.Grid(dim=dim, nx=5, ny=4, nz=3 if dim == 3 else 1, dx=1.0, dy=0.9, dz=1.1, dt=0.4)


def pair_blocks(g):
    """Blocks that depend only on the unordered node pair {n, n + delta}:
    exactly M_{g,g'} = M_{g',g}, and different for every pair."""
    nz = g.nz if g.dim == 3 else 1
    idx = np.arange(g.N)
    i, j, k = idx % g.nx, (idx // g.nx) % g.ny, idx // (g.nx * g.ny)
    M = np.empty((g.noff, 9, g.N))
    for o in range(g.noff):
        dx, dy, dz = o % 3 - 1, (o // 3) % 3 - 1, (o // 9 - 1 if g.dim == 3 else 0)
        nb = (i + dx) % g.nx + g.nx * (((j + dy) % g.ny) + g.ny * ((k + dz) % nz))
        lo, hi = np.minimum(idx, nb), np.maximum(idx, nb)
        for q in range(9):
            M[o, q] = (lo * 1000 + hi) * 10 + q
    return M


@pytest.mark.parametrize("dim", [2, 3])
def test_half_layout_rebuilds_exactly_symmetric_blocks(dim):
    g = grid(dim)
    M = pair_blocks(g)
    assert stored_half(M).shape == (g.noff // 2 + 1, 9, g.N)
    np.testing.assert_array_equal(full_from_half(g, stored_half(M)), M)
    nodes = np.array([0, 3, g.N - 1, g.N // 2])
    np.testing.assert_array_equal(full_at_nodes(g, lambda h, ids: stored_half(M)[h][:, ids], nodes), M[:, :, nodes])


@pytest.mark.parametrize("dim", [2, 3])
def test_half_layout_rebuilds_the_oracle_deposit(dim):
    g = grid(dim)
    rng = np.random.default_rng(5 + dim)
    x, u, w, sp, E, B = random_state(g, 300, rng, bmax=3.0)
    J, M = oracle.deposit(g, x, u, w, sp, B)
    Mf = full_from_half(g, stored_half(M))
    # equal up to the rounding order of the weight product
    np.testing.assert_allclose(Mf, M, rtol=1e-14, atol=1e-15 * np.abs(M).max())
    np.testing.assert_allclose(oracle.apply_A(g, Mf, E), oracle.apply_A(g, M, E), rtol=1e-13, atol=1e-13)


def test_centre_slot_is_the_zero_offset():
    for dim in (2, 3):
        g = grid(dim)
        o = m_centre(g)
        assert (o % 3, (o // 3) % 3, (o // 9 if dim == 3 else 1)) == (1, 1, 1)
