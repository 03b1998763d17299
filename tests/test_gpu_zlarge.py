"""Parity at the largest workload: the 3D double Harris sheet 512 x 256 x 256
cells x 8 particles per cell per species (536,870,912 particles; a 65 GB
FP64 mass matrix and about 190 GB of HBM in all), FP32-mixed, in the launch
configuration bench.py times.  One context runs the energy diagnostic, the
deposit (sampled nodes), the solve and push + re-sort (sampled particles,
global bin order) in turn, with the same checks and tolerances as
test_gpu_fullsize.  The module is named to be collected last: it needs most
of the GPU's memory.
"""
import pytest

from paper_2509_11100_amd import harris
from tests.gpu_helpers import load, make_ctx, need_gpu
from tests.helpers import grid_of
from tests.test_gpu_fullsize import WORKERS, _CACHE, check_deposit, check_energy, check_push

pytestmark = pytest.mark.gpu


def test_fullsize_3d_512x256x256_mixed():
    need_gpu()
    import torch

    _CACHE.clear()
    torch.cuda.empty_cache()
    name, precision = "harris3d_512x256x256", "mixed"
    wl = harris.workload(name)
    p = harris.make_particles(wl, workers=WORKERS)
    E, B = harris.make_fields(wl)
    print("generated", p["w"].shape[0], "particles", flush=True)
    g = grid_of(wl)
    ctx = make_ctx(g, precision, p["w"].shape[0], rtol=1e-10)
    parts = load(ctx, p["cell"], p["species"], p["off"], p["u"], p["w"], p["bin_start"])
    print("loaded; GPU memory in use %.1f GB" % (torch.cuda.memory_allocated() / 1e9), flush=True)
    check_energy(wl, p, E, B, ctx, parts, precision)
    print("energy checked", flush=True)
    J, M = check_deposit(wl, p, B, ctx, parts, precision)
    print("deposit checked", flush=True)
    check_push(wl, p, E, B, ctx, parts, J, M, precision)
    print("push checked", flush=True)
    del J, M, parts, ctx
    torch.cuda.empty_cache()
