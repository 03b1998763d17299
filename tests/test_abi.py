"""C ABI checks that need no GPU: the library loads, exports every function
declared in include/relsim.h, and rejects bad parameters before any device
work; bench.py refuses more than one GPU."""
import ctypes as C
import os
import re
import subprocess
import sys

import pytest

from paper_2509_11100_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "relsim.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(relsim_[A-Za-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    lib = _lib.load()
    names = declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_lib.exported_symbols())


def base_params():
    p = _lib.relsim_params()
    p.dim, p.nx, p.ny, p.nz = 2, 8, 6, 1
    p.dx = p.dy = p.dz = 1.0
    p.dt, p.c, p.theta = 0.5, 1.0, 0.5
    p.precision = _lib.RELSIM_FP64
    p.nspecies = 2
    p.q[0], p.q[1] = 1.0, -1.0
    p.m[0], p.m[1] = 1.0, 1.0
    p.max_particles = 1000
    p.gmres_rtol, p.gmres_restart, p.gmres_maxit = 1e-10, 30, 100
    return p


@pytest.mark.parametrize("field,value", [("nx", 2), ("ny", 0), ("dim", 4), ("theta", 0.3), ("theta", 1.5),
                                         ("dt", 0.0), ("dt", float("nan")), ("precision", 7), ("nspecies", 0),
                                         ("nspecies", 9), ("gmres_restart", 65), ("gmres_maxit", 0),
                                         ("group", 12), ("max_particles", -1), ("max_particles", 1 << 31)])
def test_invalid_parameters_are_rejected(field, value):
    lib = _lib.load()
    p = base_params()
    assert lib.relsim_workspace_bytes(C.byref(p)) > 0
    setattr(p, field, value)
    assert lib.relsim_workspace_bytes(C.byref(p)) == 0
    h = C.c_void_p()
    assert lib.relsim_init(C.byref(p), None, None, 0, C.byref(h)) == _lib.RELSIM_EINVAL


def test_fp32_mass_matrix_needs_mixed_precision():
    lib = _lib.load()
    p = base_params()
    p.mass_fp32 = 1
    assert lib.relsim_workspace_bytes(C.byref(p)) == 0
    p.precision = _lib.RELSIM_MIXED
    assert lib.relsim_workspace_bytes(C.byref(p)) > 0
    p.mass_fp32 = 2
    assert lib.relsim_workspace_bytes(C.byref(p)) == 0


def test_3d_needs_nz_of_three():
    lib = _lib.load()
    p = base_params()
    p.dim, p.nz = 3, 2
    assert lib.relsim_workspace_bytes(C.byref(p)) == 0
    p.nz = 3
    assert lib.relsim_workspace_bytes(C.byref(p)) > 0


def test_workspace_too_small_is_rejected():
    lib = _lib.load()
    p = base_params()
    nb = lib.relsim_workspace_bytes(C.byref(p))
    h = C.c_void_p()
    assert lib.relsim_init(C.byref(p), None, C.c_void_p(16), nb - 1, C.byref(h)) == _lib.RELSIM_EINVAL


def test_error_strings():
    lib = _lib.load()
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert len(lib.relsim_strerror(code)) > 0
        assert lib.relsim_strerror(code) != b"unknown error"
    assert lib.relsim_strerror(-99) == b"unknown error"
    assert lib.relsim_last_error(None) == b"no context"


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
