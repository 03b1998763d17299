"""GPU (HIP) path against the CPU oracle, through the C ABI.

Tolerances (normwise relative, ||gpu - oracle|| / ||oracle||, on identical
inputs: the mixed-precision path's inputs are rounded to FP32 and the oracle
receives those rounded values in FP64):
  FP64 path          1e-12
  mixed path         1e-5 for moments, fields and particles
Integer and layout results (sort order, bin_start, cell ids) are bit-exact.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2509_11100_amd import harris
from tests.gpu_helpers import host_state, load, make_ctx, need_gpu, random_cells, rounded
from tests.helpers import (cell_and_offset, check_disp, check_rel, full_from_half, grid_of, normwise, periodic_diff,
                           positions, stored_half)

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "mixed": 1e-5}


def grids():
    return {
        "2d_7x5": oracle.Grid(dim=2, nx=7, ny=5, dx=1.1, dy=0.9, dt=0.45),
        "2d_3x3": oracle.Grid(dim=2, nx=3, ny=3, dx=1.0, dy=1.0, dt=0.4),
        # 143 cells: two full 64-cell moment blocks and a partial one
        "2d_13x11": oracle.Grid(dim=2, nx=13, ny=11, dx=1.0, dy=0.8, dt=0.4),
        "3d_5x4x3": oracle.Grid(dim=3, nx=5, ny=4, nz=3, dx=1.1, dy=0.9, dz=1.2, dt=0.4),
        "3d_3x3x3": oracle.Grid(dim=3, nx=3, ny=3, nz=3, dx=1.0, dy=1.0, dz=1.0, dt=0.4),
        # larger 3D grids (many segments and tiles per row and layer)
        "3d_32x4x3": oracle.Grid(dim=3, nx=32, ny=4, nz=3, dx=1.1, dy=0.9, dz=1.2, dt=0.4),
        "3d_32x8x40": oracle.Grid(dim=3, nx=32, ny=8, nz=40, dx=1.0, dy=1.1, dz=0.9, dt=0.4),
        # the field kernels' node order: rows of two 64-node chunks, the
        # second partial; in 3D z-slabs of 4 planes (nz a multiple of 4)
        "2d_70x9": oracle.Grid(dim=2, nx=70, ny=9, dx=1.0, dy=0.9, dt=0.4),
        "3d_70x6x8": oracle.Grid(dim=3, nx=70, ny=6, nz=8, dx=1.0, dy=0.9, dz=1.1, dt=0.4),
    }


def g_cells(gname):
    return grids()[gname].N


def torch_grid(a):
    import torch

    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def setup_random(gname, precision, n, seed, empty_frac=0.2, bmax=2.0, emax=0.5, umax=2.0, **kw):
    g = grids()[gname]
    rng = np.random.default_rng(seed)
    cell, sp, off, u, w = random_cells(g, n, rng, umax=umax, empty_frac=empty_frac)
    B = (2 * rng.random((3, g.N)) - 1) * bmax
    E = (2 * rng.random((3, g.N)) - 1) * emax
    ctx = make_ctx(g, precision, n, **kw)
    parts = load(ctx, cell, sp, off, u, w)
    return g, ctx, parts, B, E


def mode(name):
    """precision and context options of a test mode: fp64, mixed (M stored
    in FP64) or mixed-m32 (M stored in FP32)"""
    return ("mixed", dict(mass_fp32=True)) if name == "mixed-m32" else (name, {})


# ----------------------------------------------------------------------------
# a1: general sort (bit-exact against a stable sort by bin)
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("gname", ["2d_7x5", "3d_5x4x3"])
def test_general_sort_is_stable_sort_by_bin(gname, precision):
    need_gpu()
    g = grids()[gname]
    rng = np.random.default_rng(11)
    n = 3001
    cell, sp, off, u, w = random_cells(g, n, rng, empty_frac=0.3)
    ctx = make_ctx(g, precision, n)
    parts = load(ctx, cell, sp, off, u, w)
    st = host_state(g, parts)
    S = len(g.q)
    order = np.argsort(cell.astype(np.int64) * S + sp, kind="stable")
    np.testing.assert_array_equal(st["cell"], cell[order])
    np.testing.assert_array_equal(st["species"], sp[order])
    np.testing.assert_array_equal(st["off"], rounded(precision, off[:, order]))
    np.testing.assert_array_equal(st["u"], rounded(precision, u[:, order]))
    np.testing.assert_array_equal(st["w"], rounded(precision, w[order]))
    bins = cell.astype(np.int64) * S + sp
    np.testing.assert_array_equal(st["bin_start"], np.searchsorted(np.sort(bins), np.arange(g.N * S + 1)))


# ----------------------------------------------------------------------------
# a2-a4: deposit
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("gname", ["2d_7x5", "2d_3x3", "2d_13x11", "3d_5x4x3", "3d_3x3x3", "3d_32x4x3", "3d_32x8x40"])
def test_deposit_parity(gname, precision):
    need_gpu()
    g, ctx, parts, B, E = setup_random(gname, precision, 2500 if g_cells(gname) < 1000 else 40000, 21)
    from paper_2509_11100_amd import relsim

    J, M = relsim.deposit_moments(ctx, parts, torch_grid(B))
    st = host_state(g, parts)
    Jr, Mr = oracle.deposit(g, st["x"], st["u"], st["w"], st["species"], B)
    J, M = J.cpu().numpy(), M.cpu().numpy()
    check_rel(J, Jr, TOL[precision])
    # the stored half against the oracle's blocks of the same offsets, and
    # the mirrored half (read from the neighbours' slots) against the
    # oracle's own, separately summed, blocks of the other offsets
    assert M.shape == (g.noff // 2 + 1, 9, g.N)
    check_rel(M, stored_half(Mr), TOL[precision], "stored M")
    check_rel(full_from_half(g, M), Mr, TOL[precision], "full M")


@pytest.mark.parametrize("gname", ["2d_13x11", "3d_32x8x40"])
def test_fp32_mass_matrix_is_the_fp64_one_rounded(gname):
    """mass_fp32 stores the same FP64 sums rounded to FP32: on the same
    particles the two contexts' M agree bit for bit after rounding the FP64
    one, and Jhat is identical.  Each context refuses the other's M."""
    need_gpu()
    import ctypes as C

    import torch

    from paper_2509_11100_amd import relsim

    g, ctx, parts, B, E = setup_random(gname, "mixed", 40000, 23)
    ctx32 = make_ctx(g, "mixed", 40000, mass_fp32=True)
    parts32 = load(ctx32, *parts.to_host()[:5])
    J, M = relsim.deposit_moments(ctx, parts, torch_grid(B))
    J32, M32 = relsim.deposit_moments(ctx32, parts32, torch_grid(B))
    assert M.dtype == torch.float64 and M32.dtype == torch.float32
    assert torch.equal(J, J32)
    assert torch.equal(M.to(torch.float32), M32)
    # each context takes only its own storage type, and M aligned to it
    from paper_2509_11100_amd._lib import RELSIM_EINVAL

    with pytest.raises(ValueError):
        relsim.apply_A(ctx, M32, torch_grid(E))
    with pytest.raises(ValueError):
        relsim.deposit_moments(ctx32, parts32, torch_grid(B), J32, M)
    parts.s.n = parts.n
    Bt = torch_grid(B)
    rc = ctx.lib.relsim_deposit_moments(ctx.handle, C.byref(parts.s), Bt.data_ptr(), J.data_ptr(), M.data_ptr() + 4)
    assert rc == RELSIM_EINVAL


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("group", [4, 8, 16, 32, 64])
def test_deposit_every_lane_group_width(group, precision):
    """Cells with far more particles than lanes (many rounds) and empty cells,
    at every lane-group width of the 2D deposit (the automatic choice takes
    4 lanes on the FP64 bench sheet) and of the kinetic-energy kernel."""
    need_gpu()
    g = grids()["2d_7x5"]
    rng = np.random.default_rng(5)
    n = 4000
    cell, sp, off, u, w = random_cells(g, n, rng, empty_frac=0.5)
    cell[: n // 2] = 3       # one crowded cell
    B = (2 * rng.random((3, g.N)) - 1) * 2.0
    E = (2 * rng.random((3, g.N)) - 1) * 0.5
    ctx = make_ctx(g, precision, n, group=group)
    parts = load(ctx, cell, sp, off, u, w)
    from paper_2509_11100_amd import relsim

    J, M = relsim.deposit_moments(ctx, parts, torch_grid(B))
    st = host_state(g, parts)
    Jr, Mr = oracle.deposit(g, st["x"], st["u"], st["w"], st["species"], B)
    check_rel(J.cpu().numpy(), Jr, TOL[precision])
    check_rel(full_from_half(g, M.cpu().numpy()), Mr, TOL[precision])
    W = relsim.energy(ctx, parts, torch_grid(E), torch_grid(B))
    np.testing.assert_allclose(W, oracle.energy(g, st["u"], st["w"], st["species"], E, B), rtol=1e-12)


def test_deposit_with_no_particles():
    need_gpu()
    g = grids()["2d_7x5"]
    ctx = make_ctx(g, "fp64", 16)
    e = np.zeros(0)
    parts = load(ctx, np.zeros(0, np.int32), np.zeros(0, np.uint8), np.zeros((2, 0)), np.zeros((3, 0)), e)
    from paper_2509_11100_amd import relsim

    J, M = relsim.deposit_moments(ctx, parts, torch_grid(np.ones((3, g.N))))
    assert float(J.abs().max()) == 0.0 and float(M.abs().max()) == 0.0
    Ek = relsim.energy(ctx, parts, torch_grid(np.zeros((3, g.N))), torch_grid(np.ones((3, g.N))))
    assert Ek[0] == 0.0 and abs(Ek[2] - g.V / (8 * math.pi) * 3 * g.N) < 1e-12


# ----------------------------------------------------------------------------
# a5: field operators and solve
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("md", ["fp64", "mixed", "mixed-m32"])
@pytest.mark.parametrize("gname", ["2d_7x5", "3d_5x4x3", "3d_3x3x3", "2d_70x9", "3d_70x6x8"])
def test_field_operators(gname, md):
    """Curls, A and A^T against the oracle on the library's own M (an FP32
    M is promoted exactly for the oracle; the products are FP64 on both
    sides)."""
    need_gpu()
    precision, kw = mode(md)
    g, ctx, parts, B, E = setup_random(gname, precision, 800, 31, **kw)
    from paper_2509_11100_amd import relsim

    J, M = relsim.deposit_moments(ctx, parts, torch_grid(B))
    assert M.dtype == ctx.mass_dtype
    Mh = full_from_half(g, M.cpu().numpy().astype(np.float64))
    c1 = relsim.curl_nc(ctx, torch_grid(E)).cpu().numpy()
    c2 = relsim.curl_cn(ctx, torch_grid(B)).cpu().numpy()
    check_rel(c1, oracle.curl_nc(g, E), 1e-13)
    check_rel(c2, oracle.curl_cn(g, B), 1e-13)
    A = relsim.apply_A(ctx, M, torch_grid(E)).cpu().numpy()
    check_rel(A, oracle.apply_A(g, Mh, E), 1e-13)
    # the transposed operator (the same kernel with every block transposed)
    # against the transpose of the oracle's sparse matrix
    AT = relsim.apply_AT(ctx, M, torch_grid(E)).cpu().numpy()
    check_rel(AT, (oracle.A_matrix(g, Mh).T @ E.reshape(-1)).reshape(3, g.N), 1e-13)


@pytest.mark.parametrize("md", ["fp64", "mixed", "mixed-m32"])
@pytest.mark.parametrize("gname", ["2d_7x5", "3d_5x4x3", "3d_70x6x8"])
def test_field_solve_parity(gname, md):
    """S4-S5 against the oracle's direct solve of the same system (the
    library's Jhat and M, M stored in FP64 or FP32; the solve is FP64)."""
    need_gpu()
    precision, kw = mode(md)
    g, ctx, parts, B, E = setup_random(gname, precision, 1500, 41, **kw)
    from paper_2509_11100_amd import relsim

    J, M = relsim.deposit_moments(ctx, parts, torch_grid(B))
    Eth, E1, B1, it, rr = relsim.field_solve(ctx, M, J, torch_grid(E), torch_grid(B))
    assert rr <= 1e-13 and it > 0
    Jh, Mh = J.cpu().numpy(), full_from_half(g, M.cpu().numpy().astype(np.float64))
    r = oracle.rhs(g, E, B, Jh)
    ref = oracle.solve(g, Mh, r)
    E1r, B1r = oracle.field_update(g, E, B, ref)
    check_rel(Eth.cpu().numpy(), ref, 1e-12)
    check_rel(E1.cpu().numpy(), E1r, 1e-12)
    check_rel(B1.cpu().numpy(), B1r, 1e-12)


@pytest.mark.parametrize("restart", [5, 30])
def test_field_solve_from_a_guess(restart):
    """relsim_field_solve_guess: started from the converged E_theta it takes
    no Arnoldi step and returns the same fields bit for bit; started from a
    perturbed E^n it converges to the oracle's solution."""
    need_gpu()
    import torch

    g, ctx0, parts, B, E = setup_random("3d_5x4x3", "fp64", 1500, 45)
    from paper_2509_11100_amd import relsim

    ctx = make_ctx(g, "fp64", 1500, rtol=1e-13, gmres_restart=restart)
    parts = load(ctx, *parts.to_host()[:5])
    J, M = relsim.deposit_moments(ctx, parts, torch_grid(B))
    Eth, E1, B1, it, rr = relsim.field_solve(ctx, M, J, torch_grid(E), torch_grid(B))
    assert it > 0 and rr <= 1e-13
    Eg = Eth.clone()
    Eth2, E12, B12, it2, rr2 = relsim.field_solve(ctx, M, J, torch_grid(E), torch_grid(B), E_theta=Eg, guess=True)
    assert it2 == 0 and rr2 == rr
    assert torch.equal(Eth2, Eth) and torch.equal(E12, E1) and torch.equal(B12, B1)
    rng = np.random.default_rng(7)
    Eg = torch_grid(E + 0.01 * rng.standard_normal(E.shape))
    Eth3, E13, B13, it3, rr3 = relsim.field_solve(ctx, M, J, torch_grid(E), torch_grid(B), E_theta=Eg, guess=True)
    assert rr3 <= 1e-13
    Jh, Mh = J.cpu().numpy(), full_from_half(g, M.cpu().numpy())
    ref = oracle.solve(g, Mh, oracle.rhs(g, E, B, Jh))
    E1r, B1r = oracle.field_update(g, E, B, ref)
    check_rel(Eth3.cpu().numpy(), ref, 1e-12)
    check_rel(E13.cpu().numpy(), E1r, 1e-12)
    check_rel(B13.cpu().numpy(), B1r, 1e-12)


def test_field_solve_with_a_long_restart_cycle():
    """GMRES(64) to 1e-15 on a 3D grid: Arnoldi steps past the 32nd of a
    cycle take the unfused second Gram-Schmidt pass."""
    need_gpu()
    g, ctx0, parts, B, E = setup_random("3d_5x4x3", "fp64", 1500, 47)
    from paper_2509_11100_amd import relsim

    ctx = make_ctx(g, "fp64", 1500, rtol=1e-15, gmres_restart=64)
    parts = load(ctx, *parts.to_host()[:5])
    J, M = relsim.deposit_moments(ctx, parts, torch_grid(B))
    Eth, E1, B1, it, rr = relsim.field_solve(ctx, M, J, torch_grid(E), torch_grid(B), allow_unconverged=True)
    print("GMRES(64) to 1e-15: %d Arnoldi steps, relative residual %.3e" % (it, rr))
    Jh, Mh = J.cpu().numpy(), full_from_half(g, M.cpu().numpy())
    ref = oracle.solve(g, Mh, oracle.rhs(g, E, B, Jh))
    check_rel(Eth.cpu().numpy(), ref, 1e-13)


def test_field_solve_reports_non_convergence():
    need_gpu()
    g, ctx0, parts, B, E = setup_random("2d_7x5", "fp64", 500, 43)
    from paper_2509_11100_amd import _lib, relsim

    ctx = make_ctx(g, "fp64", 500, rtol=1e-15, gmres_maxit=2, gmres_restart=2)
    parts = load(ctx, *parts.to_host()[:5])
    J, M = relsim.deposit_moments(ctx, parts, torch_grid(B))
    with pytest.raises(_lib.RelsimError) as ei:
        relsim.field_solve(ctx, M, J, torch_grid(E), torch_grid(B))
    assert ei.value.code == _lib.RELSIM_ENOTCONVERGED
    out = relsim.field_solve(ctx, M, J, torch_grid(E), torch_grid(B), allow_unconverged=True)
    assert out[3] == 2 and out[4] > 1e-15


# ----------------------------------------------------------------------------
# a6 (+a1): push and the incremental re-sort
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("gname", ["2d_7x5", "2d_3x3", "3d_5x4x3", "3d_3x3x3"])
def test_push_parity(gname, precision):
    need_gpu()
    g, ctx, parts, B, E = setup_random(gname, precision, 2500, 51)
    from paper_2509_11100_amd import relsim

    st0 = host_state(g, parts)
    relsim.push(ctx, parts, torch_grid(E), torch_grid(B), resort=False)
    st1 = host_state(g, parts)
    # without re-sort the offsets are relative to the old cell, in [-1, 2)
    x_gpu = positions(g, st0["cell"], st1["off"])
    for d in range(g.dim):
        x_gpu[d] = np.mod(x_gpu[d], g.L[d])
    xr, ur = oracle.push(g, st0["x"], st0["u"], st0["species"], E, B)
    check_rel(st1["u"], ur, TOL[precision])
    dxp = periodic_diff(g, x_gpu, xr)
    disp = periodic_diff(g, xr, st0["x"])
    check_disp(dxp, disp, TOL[precision])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("gname", ["2d_7x5", "2d_3x3", "3d_5x4x3", "3d_3x3x3"])
def test_push_resort_is_the_stable_sort_of_the_moved_particles(gname, precision):
    need_gpu()
    g, ctx, parts, B, E = setup_random(gname, precision, 3000, 61, umax=3.0)
    from paper_2509_11100_amd import relsim

    # the same push without re-sort gives the moved state in the old order
    ctx2 = make_ctx(g, precision, 3000)
    p2 = load(ctx2, *parts.to_host())
    relsim.push(ctx2, p2, torch_grid(E), torch_grid(B), resort=False)
    s2 = host_state(g, p2)
    n = parts.n
    keys = ["xy", "uw", "bin_start"] + (["z"] if g.dim == 3 else [])
    before = {k: parts.sets[parts.front][k].clone() for k in keys}
    relsim.push(ctx, parts, torch_grid(E), torch_grid(B), resort=True)
    # the push with re-sort only reads the front set: after the swap the
    # back set holds the state before the push
    back = parts.sets[1 - parts.front]
    for k in keys:
        m = None if k == "bin_start" else n
        np.testing.assert_array_equal(back[k][:m].cpu().numpy(), before[k][:m].cpu().numpy())
    st = host_state(g, parts)
    dt = np.float32 if precision == "mixed" else np.float64
    off = p2.to_host()[2].astype(dt)
    cell = s2["cell"].astype(np.int64)
    ext = [g.nx, g.ny, g.nz]
    coords = [cell % g.nx, (cell // g.nx) % g.ny, cell // (g.nx * g.ny)]
    for d in range(g.dim):
        f = off[d]
        m = np.where(f >= 1, 1, np.where(f < 0, -1, 0))
        f = (f - m.astype(dt)).astype(dt)
        edge = (m == -1) & (f == dt(1))
        f[edge] = 0
        m[edge] = 0
        off[d] = f
        coords[d] = (coords[d] + m) % ext[d]
    newcell = coords[0] + g.nx * coords[1] + (g.nx * g.ny * coords[2] if g.dim == 3 else 0)
    S = len(g.q)
    sp = s2["species"].astype(np.int64)
    order = np.argsort(newcell * S + sp, kind="stable")
    np.testing.assert_array_equal(st["cell"], newcell[order])
    np.testing.assert_array_equal(st["species"], sp[order])
    np.testing.assert_array_equal(st["off"], off[:, order].astype(np.float64))
    np.testing.assert_array_equal(st["u"], s2["u"][:, order])
    np.testing.assert_array_equal(st["w"], s2["w"][order])
    np.testing.assert_array_equal(st["bin_start"], np.searchsorted(np.sort(newcell * S + sp), np.arange(g.N * S + 1)))
    assert np.all((st["off"] >= 0) & (st["off"] < 1))


SPECIES = {
    1: ((-1.0,), (1.0,)),
    3: ((1.0, -1.0, 2.0), (1.0, 1.0, 25.0)),
    8: ((1.0, -1.0, 2.0, -2.0, 0.5, -0.5, 1.0, -3.0), (1.0, 1.0, 4.0, 9.0, 0.25, 2.0, 100.0, 7.0)),
}


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("ns", [1, 3, 8])
@pytest.mark.parametrize("gname", ["2d_7x5", "3d_5x4x3"])
def test_species_counts_other_than_two(gname, ns, precision):
    """The kernels special-case two species; 1, 3 and 8 species take the
    general path of the bin bounds (deposit, push + re-sort, energy)."""
    need_gpu()
    import dataclasses

    import torch

    from paper_2509_11100_amd import relsim

    q, m = SPECIES[ns]
    g = dataclasses.replace(grids()[gname], q=q, m=m)
    rng = np.random.default_rng(70 + ns)
    n = 3000
    cell, sp, off, u, w = random_cells(g, n, rng, umax=2.5, empty_frac=0.2)
    B = (2 * rng.random((3, g.N)) - 1) * 2.0
    E = (2 * rng.random((3, g.N)) - 1) * 0.5
    ctx = make_ctx(g, precision, n)
    parts = load(ctx, cell, sp, off, u, w)
    st = host_state(g, parts)
    J, M = relsim.deposit_moments(ctx, parts, torch_grid(B))
    Jr, Mr = oracle.deposit(g, st["x"], st["u"], st["w"], st["species"], B)
    check_rel(J.cpu().numpy(), Jr, TOL[precision])
    check_rel(full_from_half(g, M.cpu().numpy()), Mr, TOL[precision])
    W = relsim.energy(ctx, parts, torch_grid(E), torch_grid(B))
    Wr = oracle.energy(g, st["u"], st["w"], st["species"], E, B)
    np.testing.assert_allclose(W, Wr, rtol=1e-12)
    perm = torch.empty(n, dtype=torch.int32, device="cuda")
    relsim.push(ctx, parts, torch_grid(E), torch_grid(B), resort=True, new_index=perm)
    s1 = host_state(g, parts)
    # every particle's pushed state, found through the new index
    new = perm.cpu().numpy().astype(np.int64)
    assert np.array_equal(np.sort(new), np.arange(n))
    xr, ur = oracle.push(g, st["x"], st["u"], st["species"], E, B)
    check_rel(s1["u"][:, new], ur, TOL[precision])
    disp = periodic_diff(g, xr, st["x"])
    check_disp(periodic_diff(g, s1["x"][:, new], xr), disp, TOL[precision])
    np.testing.assert_array_equal(s1["species"][new], st["species"])
    np.testing.assert_array_equal(s1["w"][new], st["w"])
    # bin order, bin_start, and stability (equal bins keep their old order)
    key = s1["cell"].astype(np.int64) * ns + s1["species"]
    assert np.all(np.diff(key) >= 0)
    np.testing.assert_array_equal(s1["bin_start"], np.searchsorted(key, np.arange(g.N * ns + 1)))
    for b in np.unique(key):
        src = np.nonzero(key[new] == b)[0]
        assert np.all(np.diff(new[src]) > 0)


SEGMENT_GRIDS = {
    "2d_256x64": oracle.Grid(dim=2, nx=256, ny=64, dx=1.0, dy=0.9, dt=0.4),
    "3d_32x32x16": oracle.Grid(dim=3, nx=32, ny=32, nz=16, dx=1.0, dy=0.9, dz=1.1, dt=0.4),
}


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("ns", [2, 3])
@pytest.mark.parametrize("gname", ["2d_256x64", "3d_32x32x16"])
def test_push_passes_over_multi_cell_segments(gname, ns, precision):
    """Grids large enough (16384 cells, about 16 particles per cell, a fifth
    of the cells empty) that the push passes give each wave a segment of
    several cells, so the lanes of one round push particles of different
    cells and bins.  The pushed state must be the oracle's, bit for bit the
    in-place push's, and stably sorted by bin."""
    need_gpu()
    import dataclasses

    import torch

    from paper_2509_11100_amd import relsim

    g = SEGMENT_GRIDS[gname]
    if ns != 2:
        q, m = SPECIES[ns]
        g = dataclasses.replace(g, q=q, m=m)
    rng = np.random.default_rng(90 + ns)
    n = 16 * g.N * 4 // 5
    cell, sp, off, u, w = random_cells(g, n, rng, umax=2.5, empty_frac=0.2)
    B = (2 * rng.random((3, g.N)) - 1) * 2.0
    E = (2 * rng.random((3, g.N)) - 1) * 0.5
    ctx = make_ctx(g, precision, n)
    parts = load(ctx, cell, sp, off, u, w)
    st = host_state(g, parts)
    ctx2 = make_ctx(g, precision, n)
    p2 = load(ctx2, *parts.to_host())
    relsim.push(ctx2, p2, torch_grid(E), torch_grid(B), resort=False)
    s2 = host_state(g, p2)
    perm = torch.empty(n, dtype=torch.int32, device="cuda")
    relsim.push(ctx, parts, torch_grid(E), torch_grid(B), resort=True, new_index=perm)
    s1 = host_state(g, parts)
    new = perm.cpu().numpy().astype(np.int64)
    assert np.array_equal(np.sort(new), np.arange(n))
    np.testing.assert_array_equal(s1["u"][:, new], s2["u"])
    np.testing.assert_array_equal(s1["w"][new], st["w"])
    np.testing.assert_array_equal(s1["species"][new], st["species"])
    xr, ur = oracle.push(g, st["x"], st["u"], st["species"], E, B)
    check_rel(s1["u"][:, new], ur, TOL[precision])
    disp = periodic_diff(g, xr, st["x"])
    check_disp(periodic_diff(g, s1["x"][:, new], xr), disp, TOL[precision])
    key = s1["cell"].astype(np.int64) * len(g.q) + s1["species"]
    assert np.all(np.diff(key) >= 0)
    np.testing.assert_array_equal(s1["bin_start"], np.searchsorted(key, np.arange(g.N * len(g.q) + 1)))
    # stability: the particles of a bin keep their old relative order
    order = np.argsort(key[new], kind="stable")
    np.testing.assert_array_equal(new[order], np.arange(n))


def test_push_flags_a_move_of_more_than_one_cell():
    need_gpu()
    # |v| < c, so a move of more than one cell needs c dt > dx: here c dt = 2.7 dx
    g = oracle.Grid(dim=2, nx=7, ny=5, dx=1.1, dy=0.9, dt=3.0)
    ctx = make_ctx(g, "fp64", 4)
    cell = np.array([0, 1, 2, 3], np.int32)
    off = np.full((2, 4), 0.5)
    u = np.zeros((3, 4))
    u[0, 2] = 1e3                        # this one moves about 2.7 cells along x
    w = np.ones(4)
    sp = np.zeros(4, np.uint8)
    from paper_2509_11100_amd import _lib, relsim

    parts = load(ctx, cell, sp, off, u, w)
    E = np.zeros((3, g.N))
    relsim.push(ctx, parts, torch_grid(E), torch_grid(np.zeros((3, g.N))), resort=True)
    with pytest.raises(_lib.RelsimError) as ei:
        relsim.energy(ctx, parts, torch_grid(E), torch_grid(np.zeros((3, g.N))))
    assert ei.value.code == _lib.RELSIM_ERANGE


def test_push_flags_a_move_class_beyond_the_16_bit_counters():
    """70,000 particles of one species resting in one cell: their (bin, move)
    class exceeds the 16-bit re-sort counters, which is reported (and the
    scatter stays inside the arrays); the next sort of a smaller state works."""
    need_gpu()
    g = oracle.Grid(dim=2, nx=7, ny=5, dx=1.1, dy=0.9, dt=0.4)
    n = 70000
    ctx = make_ctx(g, "mixed", n)
    cell = np.full(n, 3, np.int32)
    off = np.full((2, n), 0.5)
    u = np.zeros((3, n))
    w = np.ones(n)
    sp = np.zeros(n, np.uint8)
    from paper_2509_11100_amd import _lib, relsim

    parts = load(ctx, cell, sp, off, u, w)
    Z = torch_grid(np.zeros((3, g.N)))
    relsim.push(ctx, parts, Z, Z, resort=True)
    with pytest.raises(_lib.RelsimError) as ei:
        relsim.energy(ctx, parts, Z, Z)
    assert ei.value.code == _lib.RELSIM_ERANGE
    # the flag is cleared once reported; a valid state pushes cleanly
    parts = load(ctx, cell[:100], sp[:100], off[:, :100], u[:, :100], w[:100])
    relsim.push(ctx, parts, Z, Z, resort=True)
    relsim.energy(ctx, parts, Z, Z)
    np.testing.assert_array_equal(parts.cell.cpu().numpy(), cell[:100])


# ----------------------------------------------------------------------------
# a7: energy
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("gname", ["2d_7x5", "3d_5x4x3"])
def test_energy_parity(gname, precision):
    need_gpu()
    g, ctx, parts, B, E = setup_random(gname, precision, 2000, 71)
    from paper_2509_11100_amd import relsim

    W = relsim.energy(ctx, parts, torch_grid(E), torch_grid(B))
    st = host_state(g, parts)
    Wr = oracle.energy(g, st["u"], st["w"], st["species"], E, B)
    np.testing.assert_allclose(W, Wr, rtol=1e-12)


# ----------------------------------------------------------------------------
# end to end: the 64x32 double Harris sheet, 10 steps
# ----------------------------------------------------------------------------
def harris_inputs(name="harris2d_64x32", **over):
    wl = harris.workload(name, **over)
    p = harris.make_particles(wl)
    E, B = harris.make_fields(wl)
    return wl, p, E, B


def run_gpu_steps(wl, p, E, B, precision, steps, rtol=1e-13):
    from paper_2509_11100_amd import relsim

    g = grid_of(wl)
    ctx = make_ctx(g, precision, p["w"].shape[0], rtol=rtol)
    parts = load(ctx, p["cell"], p["species"], p["off"], p["u"], p["w"], p["bin_start"])
    step = relsim.Step(ctx, parts, torch_grid(E), torch_grid(B))
    hist = [step.energy()]
    for _ in range(steps):
        step()
        hist.append(step.energy())
    return ctx, parts, step.E.cpu().numpy(), step.B.cpu().numpy(), np.array(hist)


def run_oracle_steps(g, x, u, w, sp, E, B, steps):
    hist = [oracle.energy(g, u, w, sp, E, B)]
    for _ in range(steps):
        out = oracle.step(g, x, u, w, sp, E, B)
        x, u, E, B = out["x"], out["u"], out["E"], out["B"]
        hist.append(out["W"])
    return x, u, E, B, np.array(hist)


def test_harris_end_to_end_fp64_ten_steps():
    need_gpu()
    wl, p, E, B = harris_inputs()
    g = grid_of(wl)
    steps = wl.steps
    ctx, parts, Eg, Bg, Wg = run_gpu_steps(wl, p, E, B, "fp64", steps)
    x0 = positions(g, p["cell"], p["off"])
    xr, ur, Er, Br, Wr = run_oracle_steps(g, x0, p["u"], p["w"], p["species"].astype(np.int32), E, B, steps)
    # multi-step comparison: the particles are re-sorted on the GPU, so compare
    # the sorted multisets through the fields and the energy history
    assert normwise(Eg, Er) < 1e-9
    assert normwise(Bg, Br) < 1e-9
    np.testing.assert_allclose(Wg, Wr, rtol=1e-10)
    st = host_state(g, parts)
    cr, offr = cell_and_offset(g, xr)
    order_r = np.lexsort((np.round(ur[2], 9), np.round(ur[1], 9), np.round(ur[0], 9), p["species"], cr))
    order_g = np.lexsort((np.round(st["u"][2], 9), np.round(st["u"][1], 9), np.round(st["u"][0], 9), st["species"],
                          st["cell"]))
    assert normwise(st["u"][:, order_g], ur[:, order_r]) < 1e-9


def test_harris_mixed_energy_drift_matches_oracle():
    """Mixed precision: per-step energy change relative to W0 within 1e-4 of
    the FP64 oracle's (teacher-forced: the oracle starts from the FP32-rounded
    particle state)."""
    need_gpu()
    wl, p, E, B = harris_inputs()
    g = grid_of(wl)
    steps = 5
    pr = dict(p)
    pr["off"] = rounded("mixed", p["off"])
    pr["u"] = rounded("mixed", p["u"])
    pr["w"] = rounded("mixed", p["w"])
    ctx, parts, Eg, Bg, Wg = run_gpu_steps(wl, pr, E, B, "mixed", steps)
    x0 = positions(g, pr["cell"], pr["off"])
    xr, ur, Er, Br, Wr = run_oracle_steps(g, x0, pr["u"], pr["w"], pr["species"].astype(np.int32), E, B, steps)
    dg = np.diff(Wg[:, 3]) / Wg[0, 3]
    dr = np.diff(Wr[:, 3]) / Wr[0, 3]
    assert np.abs(dg - dr).max() <= 1e-4
    assert normwise(Bg, Br) < 1e-5
    print("mixed 5-step drift vs oracle: E %.2e B %.2e W %.2e" % (normwise(Eg, Er), normwise(Bg, Br),
                                                                   np.abs(dg - dr).max()))


def test_tearing_electron_ion_end_to_end_fp64():
    """The electron-ion tearing sheet (m_i/m_e = 100, T = 10 m_e c^2, no
    background) cut to 8 x 102 cells and 4 particles per cell per species:
    five whole FP64 steps against the oracle."""
    need_gpu()
    wl, p, E, B = harris_inputs("tearing2d_200x102", nx=8, ppc=4)
    g = grid_of(wl)
    steps = 5
    ctx, parts, Eg, Bg, Wg = run_gpu_steps(wl, p, E, B, "fp64", steps)
    x0 = positions(g, p["cell"], p["off"])
    xr, ur, Er, Br, Wr = run_oracle_steps(g, x0, p["u"], p["w"], p["species"].astype(np.int32), E, B, steps)
    assert normwise(Eg, Er) < 1e-9
    assert normwise(Bg, Br) < 1e-9
    np.testing.assert_allclose(Wg, Wr, rtol=1e-10)


# ----------------------------------------------------------------------------
# energy-conserving variant: gbar per particle
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("gname", ["2d_7x5", "3d_5x4x3"])
def test_energy_conserving_passes(gname, precision):
    """relsim_deposit_moments_ec, relsim_gamma_mean and relsim_push_ec with a
    given gbar against the oracle's deposit and push with that gbar."""
    need_gpu()
    import torch

    from paper_2509_11100_amd import relsim

    g = grids()[gname]
    rng = np.random.default_rng(90)
    n = 3000
    cell, sp, off, u, w = random_cells(g, n, rng, umax=2.5, empty_frac=0.2)
    B = (2 * rng.random((3, g.N)) - 1) * 2.0
    E = (2 * rng.random((3, g.N)) - 1) * 0.5
    ctx = make_ctx(g, precision, n)
    parts = load(ctx, cell, sp, off, u, w)
    st = host_state(g, parts)
    g0 = np.sqrt(1 + (st["u"] ** 2).sum(0))
    gb = rounded(precision, g0 * (1 + 0.05 * rng.random(n)))
    gbar = torch.as_tensor(gb, dtype=ctx.dtype, device="cuda")
    J, M = relsim.deposit_moments(ctx, parts, torch_grid(B), gbar=gbar)
    Jr, Mr = oracle.deposit(g, st["x"], st["u"], st["w"], st["species"], B, gb)
    check_rel(J.cpu().numpy(), Jr, TOL[precision])
    check_rel(full_from_half(g, M.cpu().numpy()), Mr, TOL[precision])
    # the fixed-point pass, with the given gbar and from gamma(u^n)
    xr, ur = oracle.push(g, st["x"], st["u"], st["species"], E, B, gb)
    nxt = 0.5 * (g0 + np.sqrt(1 + (ur ** 2).sum(0)))
    for given in (True, False):
        gn = torch.empty(n, dtype=ctx.dtype, device="cuda")
        ch = relsim.gamma_mean(ctx, parts, torch_grid(E), torch_grid(B), gbar if given else None, gn)
        if given:
            ref_next, ref_in = nxt, gb
        else:
            _, u0 = oracle.push(g, st["x"], st["u"], st["species"], E, B)
            ref_next, ref_in = 0.5 * (g0 + np.sqrt(1 + (u0 ** 2).sum(0))), g0
        np.testing.assert_allclose(gn.cpu().numpy(), ref_next, rtol=TOL[precision])
        ref_ch = np.max(np.abs(ref_next - ref_in) / ref_in)
        assert abs(ch - ref_ch) <= 1e-3 * ref_ch + TOL[precision]
    # the state is untouched by the fixed-point pass
    st2 = host_state(g, parts)
    assert np.array_equal(st2["u"], st["u"]) and np.array_equal(st2["x"], st["x"])
    perm = torch.empty(n, dtype=torch.int32, device="cuda")
    relsim.push(ctx, parts, torch_grid(E), torch_grid(B), resort=True, new_index=perm, gbar=gbar)
    s1 = host_state(g, parts)
    new = perm.cpu().numpy().astype(np.int64)
    check_rel(s1["u"][:, new], ur, TOL[precision])
    disp = periodic_diff(g, xr, st["x"])
    check_disp(periodic_diff(g, s1["x"][:, new], xr), disp, TOL[precision])


def secant_reference(g, Fg, gp, rp):
    """The per-particle secant step written out in FP64 (numpy) from the
    stored history gp, rp: the root of the line through the last two
    residuals r = F(g) - g where its slope lies in [-10, -0.1] and the step
    is measurable, else the plain update; the result is clamped to
    gamma >= 1."""
    gd = g.astype(np.float64)
    r = Fg.astype(np.float64) - gd
    dg = gd - gp.astype(np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        slope = (r - rp.astype(np.float64)) / np.where(dg == 0.0, 1.0, dg)
        use = (np.abs(dg) > 1e-12 * gd) & (slope <= -0.1) & (slope >= -10.0)
        nxt = np.where(use, gd - r / np.where(use, slope, 1.0), gd + r)
    return np.where(nxt < 1.0, 1.0, nxt), gd, r, use


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_gamma_secant_matches_its_definition(precision):
    """relsim_gamma_secant on 1,000,003 particles (a ragged tail) over two
    passes: the first only records g and r (in the particle type: g exactly,
    r rounded); the second takes the secant step where the slope is in range
    and the plain update elsewhere (equal inputs, slopes outside [-10, -0.1]
    and on both ends of it, steps below 1 clamped).  The branch is decided in
    FP64 on both sides, from the stored history."""
    need_gpu()
    import torch

    from paper_2509_11100_amd import relsim

    n = 1_000_003
    g = grids()["2d_7x5"]
    ctx = make_ctx(g, precision, n)
    dt = np.float64 if precision == "fp64" else np.float32
    rng = np.random.default_rng(31)
    g0 = (1 + 3 * rng.random(n)).astype(dt)
    F0 = (g0 + 0.1 * (2 * rng.random(n) - 1)).astype(dt)
    # second pass: a chosen slope (F1 - g1) - (F0 - g0) = s (g1 - g0)
    g1 = F0.copy()
    s = rng.choice([-0.05, -0.1, -0.5, -9.0, -10.0, -20.0, 0.3], n)
    r0 = F0.astype(np.float64) - g0
    F1 = (g1 + r0 + s * (g1.astype(np.float64) - g0)).astype(dt)
    g1[:1000] = g0[:1000]                      # no step: plain update
    F1[1000:2000] = 0.5                        # clamped to 1 where the plain update falls below
    dev = lambda a: torch.as_tensor(a).cuda()
    gp = torch.empty(n, dtype=ctx.dtype, device="cuda")
    rp = torch.empty_like(gp)
    Fd = dev(F0.copy())
    relsim.gamma_secant(ctx, dev(g0), Fd, gp, rp, True)
    np.testing.assert_array_equal(Fd.cpu().numpy(), F0)
    np.testing.assert_array_equal(gp.cpu().numpy(), g0)
    # F0 lies within a factor 2 of g0: the residual is exact in either type
    np.testing.assert_array_equal(rp.cpu().numpy().astype(np.float64), r0)
    gp0, rp0 = gp.cpu().numpy(), rp.cpu().numpy()
    Fd = dev(F1.copy())
    relsim.gamma_secant(ctx, dev(g1), Fd, gp, rp, False)
    ref, gref, rref, took = secant_reference(g1, F1, gp0, rp0)
    got = Fd.cpu().numpy()
    np.testing.assert_allclose(got, ref.astype(dt), rtol=1e-15 if precision == "fp64" else 1.2e-7, atol=0)
    np.testing.assert_array_equal(gp.cpu().numpy(), gref.astype(dt))
    np.testing.assert_array_equal(rp.cpu().numpy(), rref.astype(dt))
    # every branch was taken
    assert took.sum() > n // 3 and (~took).sum() > n // 3 and (got == 1.0).sum() >= 500


@pytest.mark.parametrize("secant", [False, True])
def test_energy_conserving_steps_match_oracle_and_conserve_energy(secant):
    """Three energy-conserving FP64 steps of the 64 x 32 pair sheet (sheet
    temperature kT = m c^2, relativistic; time centring theta = 1/2) against
    the oracle's fixed point; the energy stays constant to the iteration's
    tolerance where the standard step drifts.  With per-particle secant
    steps the same fixed point is reached."""
    need_gpu()
    from paper_2509_11100_amd import relsim

    wl, p, E, B = harris_inputs()
    g = grid_of(wl)
    steps = 3
    ctx = make_ctx(g, "fp64", p["w"].shape[0], rtol=1e-13)
    parts = load(ctx, p["cell"], p["species"], p["off"], p["u"], p["w"], p["bin_start"])
    step = relsim.Step(ctx, parts, torch_grid(E), torch_grid(B), energy_conserving=True, picard_tol=1e-14,
                       secant=secant)
    W = [step.energy()]
    passes = []
    for _ in range(steps):
        step()
        assert step.picard_change <= 1e-14 and step.picard_iters < 30
        passes.append(step.picard_iters)
        W.append(step.energy())
    print("secant %s: passes per step %s" % (secant, passes))
    W = np.array(W)
    x = positions(g, p["cell"], p["off"])
    u, Er, Br = p["u"], E, B
    sp = p["species"].astype(np.int32)
    Wr = [oracle.energy(g, u, p["w"], sp, Er, Br)]
    for _ in range(steps):
        out = oracle.step_ec(g, x, u, p["w"], sp, Er, Br, tol=1e-14)
        x, u, Er, Br = out["x"], out["u"], out["E"], out["B"]
        Wr.append(out["W"])
    Wr = np.array(Wr)
    assert normwise(step.E.cpu().numpy(), Er) < 1e-9
    assert normwise(step.B.cpu().numpy(), Br) < 1e-9
    np.testing.assert_allclose(W, Wr, rtol=1e-10)
    assert np.abs(W[:, 3] - W[0, 3]).max() < 1e-12 * W[0, 3]
    print("energy-conserving steps: |dW|/W %.2e, passes %d" % (np.abs(W[:, 3] - W[0, 3]).max() / W[0, 3],
                                                              step.picard_iters))


def test_energy_conserving_argument_checks():
    """relsim_gamma_mean refuses an output that aliases its input and a
    misaligned gbar; relsim_gamma_secant refuses aliased, misaligned, null or
    oversized arrays; the binding refuses arrays of the wrong type or length.
    All are caught on the host before any kernel runs."""
    need_gpu()
    import ctypes as C

    import torch

    from paper_2509_11100_amd import relsim
    from paper_2509_11100_amd._lib import RELSIM_EINVAL, RelsimError

    g = grids()["2d_7x5"]
    rng = np.random.default_rng(91)
    n = 500
    cell, sp, off, u, w = random_cells(g, n, rng, umax=2.0, empty_frac=0.0)
    ctx = make_ctx(g, "fp64", n)
    parts = load(ctx, cell, sp, off, u, w)
    E, B = torch_grid(np.zeros((3, g.N))), torch_grid(np.ones((3, g.N)))
    gb = torch.ones(n + 1, dtype=torch.float64, device="cuda")
    with pytest.raises(RelsimError) as ei:
        relsim.gamma_mean(ctx, parts, E, B, gb, gb)
    assert ei.value.code == RELSIM_EINVAL
    parts.s.n = parts.n
    rc = ctx.lib.relsim_gamma_mean(ctx.handle, C.byref(parts.s), E.data_ptr(), B.data_ptr(), gb.data_ptr() + 4,
                                   gb.data_ptr(), C.byref(C.c_double()))
    assert rc == RELSIM_EINVAL
    with pytest.raises(ValueError):
        relsim.deposit_moments(ctx, parts, B, gbar=torch.ones(n, dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError):
        relsim.push(ctx, parts, E, B, gbar=torch.ones(n - 1, dtype=torch.float64, device="cuda"))
    # relsim_gamma_secant: aliased pair, misaligned history, too many
    # particles, null arrays; and the binding's type check
    h = torch.ones(n + 1, dtype=torch.float64, device="cuda")
    lib, hd = ctx.lib, ctx.handle
    assert lib.relsim_gamma_secant(hd, n, gb.data_ptr(), gb.data_ptr(), h.data_ptr(), h.data_ptr(), 1) == RELSIM_EINVAL
    assert lib.relsim_gamma_secant(hd, n, gb.data_ptr(), h.data_ptr(), h.data_ptr() + 4, h.data_ptr(), 1) \
        == RELSIM_EINVAL
    assert lib.relsim_gamma_secant(hd, n + 10**6, gb.data_ptr(), h.data_ptr(), h.data_ptr(), h.data_ptr(), 1) \
        == RELSIM_EINVAL
    assert lib.relsim_gamma_secant(hd, n, gb.data_ptr(), None, h.data_ptr(), h.data_ptr(), 1) == RELSIM_EINVAL
    with pytest.raises(ValueError):
        relsim.gamma_secant(ctx, gb[:n], h[:n], torch.ones(n, dtype=torch.float32, device="cuda"), h[:n], True)
