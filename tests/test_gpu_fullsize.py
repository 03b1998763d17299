"""Parity at the full workload sizes, in the launch configuration bench.py
times (automatic lane groups, re-sort every step), on sampled outputs the
oracle computes one by one:

* deposit (S1-S3): J-hat and the 9/27 M blocks of sampled nodes, from the
  oracle run on exactly the particles of the cells around those nodes;
* push (S6 + re-sort): sampled particles followed through the re-sort by
  their new index, against the oracle push of the same particles; plus the
  global bin order of the re-sorted state (a property that holds at any
  size);
* energy (S7): the full FP64 diagnostic against the oracle.

Workloads: the 2D double Harris sheet 1024 x 512 cells x 64 particles per
cell per species (67,108,864 particles) and the 3D sheets 128 x 64 x 64 x 16
(16,777,216 particles) and 256 x 128 x 128 x 8 (67,108,864 particles), in
both precisions.  (The 536,870,912-particle 3D sheet is in
test_gpu_zlarge.py.)  Inputs are the seeded generator's; the mixed path
is teacher-forced (the oracle receives the FP32-rounded particle state).
Tolerances as in test_gpu_parity: 1e-12 (FP64) and 1e-5 (mixed), both
normwise and as max |error| / max |reference|.  The energy sums are gated at
1e-12 relative in both precisions: the oracle sums with compensation (exact
to a few ulps whatever the number of terms) and the GPU in fixed-order blocks
(error about 50 ulps at 5e8 terms); in mixed precision both sum the same
FP32-held state in FP64.
"""
import os

import numpy as np
import pytest

import oracle
from paper_2509_11100_amd import harris
from tests.gpu_helpers import load, make_ctx, need_gpu, rounded
from tests.helpers import check_disp, check_rel, full_at_nodes, grid_of, normwise, periodic_diff, positions

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "mixed": 1e-5}
WORKLOADS = ["harris2d_1024x512", "harris3d_128x64x64", "harris3d_256x128x128"]
_CACHE = {}
WORKERS = min(16, os.cpu_count() or 1)


def inputs(name):
    # kept for the whole module (about 4 GB of host memory per 67M particles)
    if name not in _CACHE:
        wl = harris.workload(name)
        p = harris.make_particles(wl, workers=WORKERS)
        E, B = harris.make_fields(wl)
        _CACHE[name] = (wl, p, E, B)
    return _CACHE[name]


def cuda_grid(a):
    import torch

    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def cells_around_nodes(g, nodes):
    """The 2^dim cells having each node as a corner (cell = node - corner)."""
    i, j, k = nodes % g.nx, (nodes // g.nx) % g.ny, nodes // (g.nx * g.ny)
    out = []
    for a in range(1 << g.dim):
        ii = (i - (a & 1)) % g.nx
        jj = (j - ((a >> 1) & 1)) % g.ny
        kk = (k - ((a >> 2) & 1)) % g.nz if g.dim == 3 else 0
        out.append(ii + g.nx * (jj + g.ny * kk))
    return np.unique(np.concatenate(out))


def particles_of_cells(p, cells, S):
    b = p["bin_start"]
    idx = [np.arange(b[c * S], b[c * S + S]) for c in cells]
    return np.concatenate(idx) if idx else np.zeros(0, np.int64)


def check_deposit(wl, p, B, ctx, parts, precision):
    """J-hat and M of sampled nodes against the oracle on the particles of
    the cells around them."""
    from paper_2509_11100_amd import relsim
    import torch

    g = grid_of(wl)
    J, M = relsim.deposit_moments(ctx, parts, cuda_grid(B))
    rng = np.random.default_rng(7)
    # sampled nodes: random ones, the grid corners and the sheet centres
    nodes = np.unique(np.concatenate([rng.integers(0, g.N, 150), [0, g.nx - 1, g.N - 1],
                                      [g.nx * (g.ny // 4), g.nx * (3 * g.ny // 4)]]))
    sel = particles_of_cells(p, cells_around_nodes(g, nodes), len(wl.q))
    off = rounded(precision, p["off"][:, sel])
    x = positions(g, p["cell"][sel], off)
    Jr, Mr = oracle.deposit_nodes(g, x, rounded(precision, p["u"][:, sel]), rounded(precision, p["w"][sel]),
                                  p["species"][sel].astype(np.int32), B, nodes)
    nt = torch.as_tensor(nodes, device=J.device)
    Jg = J[:, nt].cpu().numpy()
    # every block of the sampled nodes: the stored half at the node, the
    # mirrored half from the neighbours' slots
    Mg = full_at_nodes(g, lambda h, ids: M[h][:, torch.as_tensor(ids, device=M.device)].cpu().numpy(), nodes)
    check_rel(Jg, Jr, TOL[precision])
    check_rel(Mg, Mr, TOL[precision])
    return J, M


def check_push(wl, p, E, B, ctx, parts, J, M, precision):
    """Sampled particles followed through push + re-sort by their new index
    against the oracle push; the whole re-sorted state in bin order."""
    import torch
    from paper_2509_11100_amd import relsim

    g = grid_of(wl)
    n = p["w"].shape[0]
    S = len(wl.q)
    Bt = cuda_grid(B)
    # E_theta from the GPU's own deposit and solve (the oracle takes it as input)
    Eth, _, _, it, rr = relsim.field_solve(ctx, M, J, cuda_grid(E), Bt)
    del J, M
    perm = torch.empty(n, dtype=torch.int32, device=Bt.device)
    relsim.push(ctx, parts, Eth, Bt, resort=True, new_index=perm)
    # the re-sort placed no particle on a face by a rounding difference
    assert relsim.placement_clamps(ctx) == 0
    # the kinetic energy the push summed equals a separate pass over the
    # pushed state (itself checked against the oracle by test_fullsize_energy)
    Wp = relsim.energy_pushed(ctx, Eth, Bt)
    np.testing.assert_allclose(Wp, relsim.energy(ctx, parts, Eth, Bt), rtol=1e-12)
    rng = np.random.default_rng(11)
    old = np.unique(np.concatenate([rng.integers(0, n, 20000), [0, n - 1]]))
    new = perm[torch.as_tensor(old, device=perm.device)].cpu().numpy().astype(np.int64)
    del perm
    assert np.unique(new).size == new.size and new.min() >= 0 and new.max() < n
    newt = torch.as_tensor(new, device=Bt.device)
    cell1 = parts.cell[newt].cpu().numpy()
    off1 = np.stack([parts.off[d][newt].cpu().numpy().astype(np.float64) for d in range(g.dim)])
    u1 = np.stack([parts.u[d][newt].cpu().numpy().astype(np.float64) for d in range(3)])
    w1 = parts.w[newt].cpu().numpy().astype(np.float64)
    # oracle push of the same particles (teacher-forced state, GPU E_theta)
    off0 = rounded(precision, p["off"][:, old])
    x0 = positions(g, p["cell"][old], off0)
    u0 = rounded(precision, p["u"][:, old])
    xr, ur = oracle.push(g, x0, u0, p["species"][old].astype(np.int32), Eth.cpu().numpy(), B)
    check_rel(u1, ur, TOL[precision])
    dx = periodic_diff(g, positions(g, cell1, off1), xr)
    disp = periodic_diff(g, xr, x0)
    check_disp(dx, disp, TOL[precision])
    np.testing.assert_array_equal(w1, rounded(precision, p["w"][old]))
    assert np.all((off1 >= 0) & (off1 < 1))
    # the whole re-sorted state is in bin order and bin_start matches it
    key = parts.cell.cpu().numpy().astype(np.int64) * S + parts.species().cpu().numpy()
    assert np.all(np.diff(key) >= 0)
    np.testing.assert_array_equal(parts.bin_start.cpu().numpy(), np.searchsorted(key, np.arange(g.N * S + 1)))


def check_energy(wl, p, E, B, ctx, parts, precision):
    """The FP64 energy diagnostic against the oracle's."""
    from paper_2509_11100_amd import relsim

    g = grid_of(wl)
    n = p["w"].shape[0]
    W = relsim.energy(ctx, parts, cuda_grid(E), cuda_grid(B))
    Wr = oracle.energy(g, rounded(precision, p["u"]), rounded(precision, p["w"]), p["species"].astype(np.int32), E,
                       B)
    # the oracle's sums are compensated (a few ulps whatever the number of
    # terms); the GPU's blocked fixed-order sums stay within about 50 ulps
    eps = np.finfo(np.float64).eps
    # a part that is zero (E^0 = 0) must come out exactly zero
    rel = [abs(W[k] - Wr[k]) / abs(Wr[k]) if Wr[k] != 0 else abs(W[k]) for k in range(3)]
    print("%s %s energy rel. errors: kinetic %.2e electric %.2e magnetic %.2e (%d particles)"
          % (wl.name, precision, rel[0], rel[1], rel[2], n))
    for k in range(3):
        assert rel[k] <= 1e-12, (k, rel[k])
    np.testing.assert_allclose(W[3], W[0] + W[1] + W[2], rtol=4 * eps)


def setup(name, precision, **kw):
    wl, p, E, B = inputs(name)
    g = grid_of(wl)
    ctx = make_ctx(g, precision, p["w"].shape[0], rtol=1e-10, **kw)
    parts = load(ctx, p["cell"], p["species"], p["off"], p["u"], p["w"], p["bin_start"])
    return wl, p, E, B, ctx, parts


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
@pytest.mark.parametrize("name", WORKLOADS)
def test_fullsize_deposit_sampled_nodes(name, precision):
    need_gpu()
    wl, p, E, B, ctx, parts = setup(name, precision)
    check_deposit(wl, p, B, ctx, parts, precision)
    del parts, ctx


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
@pytest.mark.parametrize("name", WORKLOADS)
def test_fullsize_push_resort_sampled_particles(name, precision):
    need_gpu()
    wl, p, E, B, ctx, parts = setup(name, precision)
    J, M = check_deposit(wl, p, B, ctx, parts, precision)
    check_push(wl, p, E, B, ctx, parts, J, M, precision)
    del J, M, parts, ctx


@pytest.mark.parametrize("name", ["harris2d_1024x512", "harris3d_256x128x128"])
def test_fullsize_fp32_mass_matrix(name):
    """Mixed precision with M stored in FP32 (mass_fp32): the sampled nodes'
    blocks, then the solve on that M and the push + re-sort of the sampled
    particles, against the oracle at the mixed tolerance."""
    need_gpu()
    wl, p, E, B, ctx, parts = setup(name, "mixed", mass_fp32=True)
    J, M = check_deposit(wl, p, B, ctx, parts, "mixed")
    assert M.dtype.itemsize == 4
    check_push(wl, p, E, B, ctx, parts, J, M, "mixed")
    del J, M, parts, ctx


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
@pytest.mark.parametrize("name", WORKLOADS)
def test_fullsize_energy(name, precision):
    need_gpu()
    wl, p, E, B, ctx, parts = setup(name, precision)
    check_energy(wl, p, E, B, ctx, parts, precision)
    del parts, ctx

