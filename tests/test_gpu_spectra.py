"""GPU checks for the nonlinear reconnection run (Sec. 3.2, Table 2): the
fiducial sheet cut down to 16 x 24 cells (separate sheet and background
species, n0/n_b = 269.3, T = 10 m_e c^2, m_i/m_e = 100) stepped on the GPU
against the oracle, and the spectra computed on the device against the same
histogram on the host."""
import numpy as np
import pytest

import oracle
from paper_2509_11100_amd import harris, spectra
from tests.gpu_helpers import host_state, load, make_ctx, need_gpu
from tests.helpers import grid_of, normwise, positions

pytestmark = pytest.mark.gpu


def torch_grid(a):
    import torch

    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def small_sheet():
    wl = harris.workload("reconnection2d_625x625", nx=16, ny=24, ppc=4, ppc_sheet=8)
    p = harris.make_particles(wl, workers=2)
    E, B = harris.make_fields(wl)
    return wl, p, E, B


@pytest.mark.parametrize("energy_conserving,secant", [(False, False), (True, False), (True, True)])
def test_reconnection_sheet_steps_match_the_oracle(energy_conserving, secant):
    """Three FP64 steps (standard, and energy-conserving with the fixed
    point to 1e-13: plain and per-particle secant) of the
    cut-down fiducial sheet: fields and energy against the oracle's steps."""
    need_gpu()
    from paper_2509_11100_amd import relsim

    wl, p, E, B = small_sheet()
    g = grid_of(wl)
    ctx = make_ctx(g, "fp64", p["w"].shape[0], rtol=1e-13)
    parts = load(ctx, p["cell"], p["species"], p["off"], p["u"], p["w"], p["bin_start"])
    step = relsim.Step(ctx, parts, torch_grid(E), torch_grid(B), energy_conserving=energy_conserving,
                       picard_tol=1e-13 if energy_conserving else None, picard_maxit=80, secant=secant)
    steps = 3
    Wg = [step.energy()]
    passes = []
    for _ in range(steps):
        step()
        passes.append(step.picard_iters)
        Wg.append(step.energy())
    print("energy-conserving %s, secant %s: passes %s" % (energy_conserving, secant, passes))
    x = positions(g, p["cell"], p["off"])
    u, Er, Br = p["u"], E, B
    sp = p["species"].astype(np.int32)
    Wr = [oracle.energy(g, u, p["w"], sp, Er, Br)]
    for _ in range(steps):
        out = (oracle.step_ec(g, x, u, p["w"], sp, Er, Br, tol=1e-13) if energy_conserving
               else oracle.step(g, x, u, p["w"], sp, Er, Br))
        x, u, Er, Br = out["x"], out["u"], out["E"], out["B"]
        Wr.append(out["W"])
    assert normwise(step.E.cpu().numpy(), Er) < 1e-9
    assert normwise(step.B.cpu().numpy(), Br) < 1e-9
    np.testing.assert_allclose(np.array(Wg), np.array(Wr), rtol=1e-10)
    if energy_conserving:
        Wg = np.array(Wg)
        assert np.abs(Wg[:, 3] - Wg[0, 3]).max() < 1e-11 * Wg[0, 3]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_device_spectra_equal_the_host_histogram(precision):
    need_gpu()
    import torch

    from paper_2509_11100_amd import relsim

    wl, p, E, B = small_sheet()
    g = grid_of(wl)
    ctx = make_ctx(g, precision, p["w"].shape[0])
    parts = load(ctx, p["cell"], p["species"], p["off"], p["u"], p["w"], p["bin_start"])
    relsim.push(ctx, parts, torch_grid(E), torch_grid(B), resort=True)
    st = host_state(g, parts)
    got = spectra.device_spectra(parts, (2, 3))
    for s in (2, 3):
        sel = st["species"] == s
        u = np.sqrt((st["u"][:, sel] ** 2).sum(0))
        ref = spectra.spectrum(u, st["w"][sel])
        np.testing.assert_allclose(got[s], ref, rtol=1e-12, atol=1e-300)
        assert (got[s] * np.diff(spectra.EDGES)).sum() == pytest.approx(st["w"][sel].sum(), rel=1e-12)
