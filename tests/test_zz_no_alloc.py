"""relsim_energy_noalloc, the allocation-free energy diagnostic, through the
C ABI against relsim_energy (same kernels, same reduction order: equal bit
for bit) and the oracle (1e-12), on two calls in a row, the second with a
smaller input on another grid; and its refusal of a grid beyond its scratch.
"""
import numpy as np
import pytest

import oracle
from paper_2509_11100_amd import harris
from tests.gpu_helpers import host_state, load, make_ctx, need_gpu, random_cells
from tests.helpers import grid_of

pytestmark = pytest.mark.gpu


def torch_grid(a):
    import torch

    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _case_harris(precision):
    wl = harris.workload("harris2d_64x32")
    p = harris.make_particles(wl)
    E, B = harris.make_fields(wl)
    rng = np.random.default_rng(3)
    E = E + (2 * rng.random(E.shape) - 1) * 0.05  # E^0 = 0 in the workload; make every part nonzero
    g = grid_of(wl)
    ctx = make_ctx(g, precision, p["w"].shape[0])
    parts = load(ctx, p["cell"], p["species"], p["off"], p["u"], p["w"], p["bin_start"])
    return g, ctx, parts, E, B


def _case_small(precision):
    g = oracle.Grid(dim=3, nx=5, ny=4, nz=3, dx=1.1, dy=0.9, dz=1.2, dt=0.4)
    rng = np.random.default_rng(8)
    cell, sp, off, u, w = random_cells(g, 700, rng, umax=2.0, empty_frac=0.2)
    B = (2 * rng.random((3, g.N)) - 1) * 2.0
    E = (2 * rng.random((3, g.N)) - 1) * 0.5
    ctx = make_ctx(g, precision, 700)
    parts = load(ctx, cell, sp, off, u, w)
    return g, ctx, parts, E, B


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_energy_noalloc_matches_relsim_energy_on_two_calls(precision):
    need_gpu()
    import torch

    from paper_2509_11100_amd import relsim

    out = torch.full((4,), float("nan"), dtype=torch.float64, device="cuda")
    for make in (_case_harris, _case_small):  # the second input is smaller
        g, ctx, parts, E, B = make(precision)
        Et, Bt = torch_grid(E), torch_grid(B)
        relsim.energy_noalloc(ctx, parts, Et, Bt, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        ref = relsim.energy(ctx, parts, Et, Bt)
        np.testing.assert_array_equal(got, ref)
        st = host_state(g, parts)
        np.testing.assert_allclose(got, oracle.energy(g, st["u"], st["w"], st["species"], E, B), rtol=1e-12)
        assert got[1] > 0 and got[2] > 0
        del parts, ctx


def test_energy_noalloc_refuses_a_grid_beyond_its_scratch():
    """16.7M cells need about 2.1M kinetic partials, beyond the 4 MiB of
    scratch: refused on the host before any kernel runs (the field arrays are
    never read, so small stand-ins are passed)."""
    need_gpu()
    import torch

    from paper_2509_11100_amd import _lib, relsim

    small = make_ctx(oracle.Grid(dim=2, nx=7, ny=5), "fp64", 16)
    parts = load(small, np.zeros(0, np.int32), np.zeros(0, np.uint8), np.zeros((2, 0)), np.zeros((3, 0)),
                 np.zeros(0))
    p = _lib.relsim_params()
    C = __import__("ctypes")
    C.memmove(C.addressof(p), C.addressof(small.params), C.sizeof(p))
    p.nx, p.ny = 4096, 4096
    dummy = torch.zeros(12, dtype=torch.float64, device="cuda")
    with pytest.raises(_lib.RelsimError) as ei:
        relsim.energy_noalloc(p, parts, dummy, dummy, dummy[:4])
    assert ei.value.code == _lib.RELSIM_ERANGE
