"""CPU FP64 oracle of the relativistic semi-implicit PIC step.

TEST INFRASTRUCTURE ONLY.  Only the tests, the package's ``smoke()`` check and
the benchmark's ``cpu_baseline`` leg may import this package.  It shares no
code with the HIP library and never imports it.

The per-particle and stencil loops live in ``relsim_oracle.c`` (plain serial
C, FP64); this module compiles it with gcc on first use, wraps it with ctypes,
and adds the linear solve (S4) as a sparse direct factorisation of the
assembled operator (SciPy/SuperLU), or restarted GMRES from SciPy for systems
too large to factor.  See ``relsim_oracle.c`` for the equations followed.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "relsim_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle into ``oracle/liboracle.so`` (gcc, -O2, portable)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-D_GNU_SOURCE", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class OCfg(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double), ("dt", C.c_double),
        ("c", C.c_double), ("theta", C.c_double),
        ("nonrel", C.c_int32), ("nspecies", C.c_int32),
        ("q", C.c_double * 8), ("m", C.c_double * 8),
    ]


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build(force=False)
            lib = C.CDLL(_LIB)
            dp = C.POINTER(C.c_double)
            ip = C.POINTER(C.c_int32)
            lp = C.POINTER(C.c_long)
            cp = C.POINTER(OCfg)
            L = C.c_long
            sig = {
                "oracle_alpha": [dp, dp],
                "oracle_gather_B": [cp, L, dp, dp, dp],
                "oracle_gather_E": [cp, L, dp, dp, dp],
                "oracle_alphas": [cp, L, dp, dp, ip, dp, dp],
                "oracle_deposit": [cp, L, dp, dp, dp, ip, dp, dp, dp, dp],
                "oracle_deposit_nodes": [cp, L, dp, dp, dp, ip, dp, L, lp, dp, dp],
                "oracle_curl_nc": [cp, dp, dp],
                "oracle_curl_cn": [cp, dp, dp],
                "oracle_apply_M": [cp, dp, dp, dp],
                "oracle_apply_A": [cp, dp, dp, dp],
                "oracle_rhs": [cp, dp, dp, dp, dp],
                "oracle_field_update": [cp, dp, dp, dp, dp, dp],
                "oracle_push": [cp, L, dp, dp, ip, dp, dp, dp],
                "oracle_energy": [cp, L, dp, dp, ip, dp, dp, dp],
            }
            for name, args in sig.items():
                fn = getattr(lib, name)
                fn.argtypes = args
                fn.restype = C.c_int if name == "oracle_deposit_nodes" else None
            _lib = lib
    return _lib


@dataclass
class Grid:
    """Grid and step parameters (periodic box, Gaussian units)."""

    dim: int
    nx: int
    ny: int
    nz: int = 1
    dx: float = 1.0
    dy: float = 1.0
    dz: float = 1.0
    dt: float = 0.5
    c: float = 1.0
    theta: float = 0.5
    nonrel: bool = False
    q: Sequence[float] = (1.0, -1.0)
    m: Sequence[float] = (1.0, 1.0)

    @property
    def N(self) -> int:
        return self.nx * self.ny * (self.nz if self.dim == 3 else 1)

    @property
    def noff(self) -> int:
        return 27 if self.dim == 3 else 9

    @property
    def V(self) -> float:
        return self.dx * self.dy * (self.dz if self.dim == 3 else 1.0)

    @property
    def L(self):
        return [self.nx * self.dx, self.ny * self.dy, (self.nz if self.dim == 3 else 1) * self.dz][: self.dim]

    def cfg(self) -> OCfg:
        o = OCfg()
        o.dim, o.nx, o.ny = self.dim, self.nx, self.ny
        o.nz = self.nz if self.dim == 3 else 1
        o.dx, o.dy, o.dz, o.dt, o.c, o.theta = self.dx, self.dy, self.dz, self.dt, self.c, self.theta
        o.nonrel = 1 if self.nonrel else 0
        o.nspecies = len(self.q)
        for i, (qq, mm) in enumerate(zip(self.q, self.m)):
            o.q[i] = qq
            o.m[i] = mm
        return o


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(C.POINTER(C.c_int32))


def alpha(b) -> np.ndarray:
    """S2 rotation operator for a normalised field b (3,) -> (3, 3)."""
    lib = _load()
    bb, pb = _d(np.asarray(b, dtype=np.float64).reshape(3))
    out, po = _d(np.zeros(9))
    lib.oracle_alpha(pb, po)
    return out.reshape(3, 3)


def gather_B(g: Grid, x, B) -> np.ndarray:
    lib = _load()
    x, px = _d(x)
    B, pB = _d(B)
    n = x.shape[1]
    out, po = _d(np.zeros((3, n)))
    cfg = g.cfg()
    lib.oracle_gather_B(C.byref(cfg), n, px, pB, po)
    return out


def gather_E(g: Grid, x, E) -> np.ndarray:
    lib = _load()
    x, px = _d(x)
    E, pE = _d(E)
    n = x.shape[1]
    out, po = _d(np.zeros((3, n)))
    cfg = g.cfg()
    lib.oracle_gather_E(C.byref(cfg), n, px, pE, po)
    return out


def alphas(g: Grid, x, u, species, B) -> np.ndarray:
    lib = _load()
    x, px = _d(x)
    u, pu = _d(u)
    sp, ps = _i(species)
    B, pB = _d(B)
    n = x.shape[1]
    out, po = _d(np.zeros((9, n)))
    cfg = g.cfg()
    lib.oracle_alphas(C.byref(cfg), n, px, pu, ps, pB, po)
    return out


def _gbar(gbar, n):
    if gbar is None:
        return None, None
    gb = np.ascontiguousarray(gbar, dtype=np.float64).reshape(n)
    return gb, gb.ctypes.data_as(C.POINTER(C.c_double))


def deposit(g: Grid, x, u, w, species, B, gbar=None):
    """S1-S3: returns (Jhat [3][N], M [noff][9][N]).  ``gbar`` (n,), if
    given, replaces gamma(u^n) in S2-S3 (the energy-conserving variant)."""
    lib = _load()
    x, px = _d(x)
    u, pu = _d(u)
    w, pw = _d(w)
    sp, ps = _i(species)
    B, pB = _d(B)
    n = x.shape[1]
    J, pJ = _d(np.zeros((3, g.N)))
    M, pM = _d(np.zeros((g.noff, 9, g.N)))
    cfg = g.cfg()
    gb, pg = _gbar(gbar, n)
    lib.oracle_deposit(C.byref(cfg), n, px, pu, pw, ps, pB, pg, pJ, pM)
    return J, M


def deposit_nodes(g: Grid, x, u, w, species, B, nodes):
    """S1-S3 for a sample of nodes: (Jhat [3][ns], M [noff][9][ns]), the
    columns ``nodes`` of deposit()'s result, bit for bit.  Node ids must be
    distinct and in [0, N)."""
    lib = _load()
    x, px = _d(x)
    u, pu = _d(u)
    w, pw = _d(w)
    sp, ps = _i(species)
    B, pB = _d(B)
    nodes = np.ascontiguousarray(nodes, dtype=np.int64)
    ns = nodes.shape[0]
    n = x.shape[1]
    J, pJ = _d(np.zeros((3, ns)))
    M, pM = _d(np.zeros((g.noff, 9, ns)))
    cfg = g.cfg()
    rc = lib.oracle_deposit_nodes(C.byref(cfg), n, px, pu, pw, ps, pB, ns,
                                  nodes.ctypes.data_as(C.POINTER(C.c_long)), pJ, pM)
    if rc == -2:
        raise ValueError("deposit_nodes: node ids must be distinct and in [0, N)")
    if rc != 0:
        raise MemoryError("deposit_nodes: slot table allocation failed")
    return J, M


def curl_nc(g: Grid, E) -> np.ndarray:
    lib = _load()
    E, pE = _d(E)
    out, po = _d(np.zeros((3, g.N)))
    cfg = g.cfg()
    lib.oracle_curl_nc(C.byref(cfg), pE, po)
    return out


def curl_cn(g: Grid, B) -> np.ndarray:
    lib = _load()
    B, pB = _d(B)
    out, po = _d(np.zeros((3, g.N)))
    cfg = g.cfg()
    lib.oracle_curl_cn(C.byref(cfg), pB, po)
    return out


def apply_M(g: Grid, M, xv) -> np.ndarray:
    lib = _load()
    M, pM = _d(M)
    xv, px = _d(xv)
    out, po = _d(np.zeros((3, g.N)))
    cfg = g.cfg()
    lib.oracle_apply_M(C.byref(cfg), pM, px, po)
    return out


def apply_A(g: Grid, M, xv) -> np.ndarray:
    lib = _load()
    M, pM = _d(M)
    xv, px = _d(xv)
    out, po = _d(np.zeros((3, g.N)))
    cfg = g.cfg()
    lib.oracle_apply_A(C.byref(cfg), pM, px, po)
    return out


def rhs(g: Grid, En, Bn, J) -> np.ndarray:
    lib = _load()
    En, pE = _d(En)
    Bn, pB = _d(Bn)
    J, pJ = _d(J)
    out, po = _d(np.zeros((3, g.N)))
    cfg = g.cfg()
    lib.oracle_rhs(C.byref(cfg), pE, pB, pJ, po)
    return out


def field_update(g: Grid, En, Bn, Eth):
    lib = _load()
    En, pE = _d(En)
    Bn, pB = _d(Bn)
    Eth, pT = _d(Eth)
    E1, p1 = _d(np.zeros((3, g.N)))
    B1, p2 = _d(np.zeros((3, g.N)))
    cfg = g.cfg()
    lib.oracle_field_update(C.byref(cfg), pE, pB, pT, p1, p2)
    return E1, B1


def push(g: Grid, x, u, species, Eth, Bn, gbar=None):
    """S6: returns new (x, u); inputs are not modified.  ``gbar`` as in
    deposit()."""
    lib = _load()
    x = np.array(x, dtype=np.float64, order="C", copy=True)
    u = np.array(u, dtype=np.float64, order="C", copy=True)
    px = x.ctypes.data_as(C.POINTER(C.c_double))
    pu = u.ctypes.data_as(C.POINTER(C.c_double))
    sp, ps = _i(species)
    Eth, pE = _d(Eth)
    Bn, pB = _d(Bn)
    cfg = g.cfg()
    gb, pg = _gbar(gbar, x.shape[1])
    lib.oracle_push(C.byref(cfg), x.shape[1], px, pu, ps, pE, pB, pg)
    return x, u


def energy(g: Grid, u, w, species, E, B) -> np.ndarray:
    """S7: (kinetic, electric, magnetic, total), each sum compensated
    (correct to a few ulps whatever the number of terms)."""
    lib = _load()
    u, pu = _d(u)
    w, pw = _d(w)
    sp, ps = _i(species)
    E, pE = _d(E)
    B, pB = _d(B)
    out, po = _d(np.zeros(4))
    cfg = g.cfg()
    lib.oracle_energy(C.byref(cfg), u.shape[1], pu, pw, ps, pE, pB, po)
    return out


# ----------------------------------------------------------------------------
# S4: the linear solve
# ----------------------------------------------------------------------------
def _diff_matrix(g: Grid, d: int, to_centres: bool):
    """Sparse N x N averaged difference along dim d (same stencil as the C
    code, written here as index arithmetic): nodes -> centres if to_centres,
    centres -> nodes otherwise; zero for the ignorable z direction in 2D."""
    import scipy.sparse as sp

    N = g.N
    nz = g.nz if g.dim == 3 else 1
    ext = (g.nx, g.ny, nz)
    h = (g.dx, g.dy, g.dz)[d]
    active = [0, 1] + ([2] if g.dim == 3 else [])
    if d not in active:
        return sp.csr_matrix((N, N))
    trans = [e for e in active if e != d]
    idx = np.arange(N)
    coord = [idx % g.nx, (idx // g.nx) % g.ny, idx // (g.nx * g.ny)]

    def lin(c):
        return (c[0] % ext[0]) + ext[0] * ((c[1] % ext[1]) + ext[1] * (c[2] % ext[2]))

    rows, cols, vals = [], [], []
    ncorner = 1 << len(trans)
    for t in range(ncorner):
        o = [0, 0, 0]
        for bit, e in enumerate(trans):
            o[e] = (t >> bit) & 1
        sgn = 1 if to_centres else -1
        hi = [coord[e] + sgn * o[e] + (1 if (to_centres and e == d) else 0) for e in range(3)]
        lo = [coord[e] + sgn * o[e] - (1 if (not to_centres and e == d) else 0) for e in range(3)]
        rows += [idx, idx]
        cols += [lin(hi), lin(lo)]
        vals += [np.full(N, 1.0 / (ncorner * h)), np.full(N, -1.0 / (ncorner * h))]
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))


def curl_matrix(g: Grid, to_centres: bool):
    """Sparse C_NC (to_centres) or C_CN: curl = (dy Fz - dz Fy, dz Fx - dx Fz, dx Fy - dy Fx)."""
    import scipy.sparse as sp

    D = [_diff_matrix(g, d, to_centres) for d in range(3)]
    Z = sp.csr_matrix((g.N, g.N))
    return sp.bmat([[Z, -D[2], D[1]], [D[2], Z, -D[0]], [-D[1], D[0], Z]], format="csr")


def M_matrix(g: Grid, M):
    """Expand the stencil mass matrix M [noff][9][N] into a sparse 3N x 3N matrix."""
    import scipy.sparse as sp

    N = g.N
    nz = g.nz if g.dim == 3 else 1
    gi = np.arange(N)
    i = gi % g.nx
    j = (gi // g.nx) % g.ny
    k = gi // (g.nx * g.ny)
    rows, cols, vals = [], [], []
    for off in range(g.noff):
        dx, dy, dz = off % 3 - 1, (off // 3) % 3 - 1, off // 9 - 1
        gj = ((i + dx) % g.nx) + g.nx * (((j + dy) % g.ny) + g.ny * ((k + dz) % nz))
        for r in range(3):
            for c in range(3):
                rows.append(r * N + gi)
                cols.append(c * N + gj)
                vals.append(np.asarray(M[off, 3 * r + c]))
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(3 * N, 3 * N))


def A_matrix(g: Grid, M):
    """Sparse S4 operator I + (c th dt)^2 C_CN C_NC + 4 pi th dt M."""
    import scipy.sparse as sp

    Cnc = curl_matrix(g, True)
    Ccn = curl_matrix(g, False)
    a = g.c * g.theta * g.dt
    b = 4.0 * np.pi * g.theta * g.dt
    return (sp.identity(3 * g.N, format="csr") + (a * a) * (Ccn @ Cnc) + b * M_matrix(g, M)).tocsc()


def solve(g: Grid, M, r, direct_limit: int = 200_000, rtol: float = 1e-13, x0=None):
    """Solve A E_th = r.  Sparse LU below ``direct_limit`` unknowns, else SciPy GMRES(30)."""
    import scipy.sparse.linalg as sla

    r = np.asarray(r, dtype=np.float64).reshape(-1)
    if 3 * g.N <= direct_limit:
        A = A_matrix(g, M)
        return sla.spsolve(A, r).reshape(3, g.N)
    A = sla.LinearOperator((3 * g.N, 3 * g.N), matvec=lambda v: apply_A(g, M, v.reshape(3, g.N)).reshape(-1))
    x, info = sla.gmres(A, r, x0=None if x0 is None else np.asarray(x0).reshape(-1), rtol=rtol, restart=30, maxiter=2000)
    if info != 0:
        raise RuntimeError("oracle GMRES did not converge (info=%d)" % info)
    return x.reshape(3, g.N)


def step(g: Grid, x, u, w, species, E, B, direct_limit: int = 200_000, rtol: float = 1e-13):
    """One full step S1-S7.  Returns a dict with the new state and intermediates."""
    J, M = deposit(g, x, u, w, species, B)
    r = rhs(g, E, B, J)
    Eth = solve(g, M, r, direct_limit=direct_limit, rtol=rtol, x0=E)
    E1, B1 = field_update(g, E, B, Eth)
    x1, u1 = push(g, x, u, species, Eth, B)
    W = energy(g, u1, w, species, E1, B1)
    return {"J": J, "M": M, "rhs": r, "E_theta": Eth, "E": E1, "B": B1, "x": x1, "u": u1, "W": W}


def gamma(g: Grid, u) -> np.ndarray:
    """Lorentz factor sqrt(1 + |u|^2/c^2) per particle (1 when non-relativistic)."""
    u = np.asarray(u, dtype=np.float64)
    if g.nonrel:
        return np.ones(u.shape[1])
    return np.sqrt(1.0 + (u * u).sum(0) / (g.c * g.c))


def step_ec(g: Grid, x, u, w, species, E, B, tol: float = 1e-13, maxit: int = 50,
            direct_limit: int = 200_000, rtol: float = 1e-13):
    """One energy-conserving step: S1-S6 with gbar = (gamma(u^n) + gamma(u^{n+1}))/2,
    found by fixed-point (Picard) iteration from gbar = gamma(u^n).  Each pass
    deposits with the current gbar, solves, pushes, and forms the next gbar
    from the pushed momenta; it stops once max |gbar_next - gbar| / gbar <=
    tol and keeps that pass's fields and particles.  Returns step()'s dict plus
    ``gbar`` (the value the kept pass used), ``iters`` and ``change``."""
    g0 = gamma(g, u)
    gbar = g0.copy()
    for it in range(1, maxit + 1):
        J, M = deposit(g, x, u, w, species, B, gbar)
        r = rhs(g, E, B, J)
        Eth = solve(g, M, r, direct_limit=direct_limit, rtol=rtol, x0=E)
        x1, u1 = push(g, x, u, species, Eth, B, gbar)
        nxt = 0.5 * (g0 + gamma(g, u1))
        change = float(np.max(np.abs(nxt - gbar) / gbar)) if gbar.size else 0.0
        if change <= tol or it == maxit:
            break
        gbar = nxt
    E1, B1 = field_update(g, E, B, Eth)
    W = energy(g, u1, w, species, E1, B1)
    return {"J": J, "M": M, "rhs": r, "E_theta": Eth, "E": E1, "B": B1, "x": x1, "u": u1, "W": W,
            "gbar": gbar, "iters": it, "change": change}
