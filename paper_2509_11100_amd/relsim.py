"""Thin Python binding of librelsim over torch device tensors.

Each function carries the name of the C entry point it calls and only
marshals arguments: every step of the path runs in the library's HIP kernels.
PyTorch provides the device memory and the stream (the stream current at
context creation is the one every call enqueues on).
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import RelsimError


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


class Context:
    """A librelsim context: parameters, caller-owned workspace, stream."""

    def __init__(self, *, dim: int, nx: int, ny: int, nz: int = 1, dx: float, dy: Optional[float] = None,
                 dz: Optional[float] = None, dt: float, c: float = 1.0, theta: float = 0.5,
                 precision: str = "fp64", q: Sequence[float] = (1.0, -1.0), m: Sequence[float] = (1.0, 1.0),
                 max_particles: int, gmres_rtol: float = 1e-10, gmres_restart: int = 30, gmres_maxit: int = 3000,
                 nonrelativistic: bool = False, group: int = 0, mass_fp32: bool = False, device: str = "cuda"):
        self.lib = _lib.load()
        p = _lib.relsim_params()
        p.dim, p.nx, p.ny, p.nz = dim, nx, ny, (nz if dim == 3 else 1)
        p.dx = dx
        p.dy = dx if dy is None else dy
        p.dz = dx if dz is None else dz
        p.dt, p.c, p.theta = dt, c, theta
        if precision not in ("fp64", "mixed"):
            raise ValueError("precision must be 'fp64' or 'mixed'")
        p.precision = _lib.RELSIM_FP64 if precision == "fp64" else _lib.RELSIM_MIXED
        p.nspecies = len(q)
        for i, (qq, mm) in enumerate(zip(q, m)):
            p.q[i] = qq
            p.m[i] = mm
        p.max_particles = int(max_particles)
        p.gmres_rtol, p.gmres_restart, p.gmres_maxit = gmres_rtol, gmres_restart, gmres_maxit
        p.nonrelativistic = 1 if nonrelativistic else 0
        p.group = group
        if mass_fp32 and precision != "mixed":
            raise ValueError("mass_fp32 needs mixed precision")
        p.mass_fp32 = 1 if mass_fp32 else 0
        self.mass_dtype = torch.float32 if mass_fp32 else torch.float64
        self.params = p
        self.precision = precision
        dev = torch.device(device)
        if dev.type == "cuda" and dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        nbytes = self.lib.relsim_workspace_bytes(C.byref(p))
        if nbytes == 0:
            raise RelsimError(_lib.RELSIM_EINVAL, "invalid parameters")
        self.workspace = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        rc = self.lib.relsim_init(C.byref(p), C.c_void_p(self.stream.cuda_stream), C.c_void_p(self.workspace.data_ptr()),
                                  C.c_size_t(int(nbytes)), C.byref(h))
        if rc != 0:
            raise RelsimError(rc, self.lib.relsim_strerror(rc).decode())
        self.handle = h

    # ---- shapes ----
    @property
    def dim(self) -> int:
        return self.params.dim

    @property
    def ncells(self) -> int:
        return self.params.nx * self.params.ny * (self.params.nz if self.params.dim == 3 else 1)

    @property
    def nspecies(self) -> int:
        return self.params.nspecies

    @property
    def noff(self) -> int:
        return 27 if self.params.dim == 3 else 9

    @property
    def m_slots(self) -> int:
        """Stored node-pair blocks of M per node: the offsets from the centre
        on in the offset order (M_{g,g'} = M_{g',g}, so the other half is the
        same blocks seen from the other node)."""
        return self.noff // 2 + 1

    @property
    def dtype(self) -> torch.dtype:
        return torch.float64 if self.precision == "fp64" else torch.float32

    def check(self, rc: int) -> int:
        if rc != 0:
            raise RelsimError(rc, "%s: %s" % (self.lib.relsim_strerror(rc).decode(),
                                              self.lib.relsim_last_error(self.handle).decode()))
        return rc

    def grid(self) -> torch.Tensor:
        return torch.zeros((3, self.ncells), dtype=torch.float64, device=self.device)

    def mass_matrix(self) -> torch.Tensor:
        """The stored half of M, [m_slots][9][N]: FP64, or FP32 for a
        context made with mass_fp32."""
        return torch.empty((self.m_slots, 9, self.ncells), dtype=self.mass_dtype, device=self.device)

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self.lib.relsim_finalize(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Particles:
    """Double-buffered particle state on the device: per set, in 2D xy
    [cap][2] (offsets x, y) and uw [cap][4] (momentum, weight); in 3D one
    record tensor xy [cap][8] (offsets x, y, z, 0, momentum, weight), with
    uw and z kept as strided views of it; cell ids and bin starts.  `off`,
    `u` and `w` are strided views."""

    def __init__(self, ctx: Context, capacity: Optional[int] = None):
        self.ctx = ctx
        cap = int(ctx.params.max_particles if capacity is None else capacity)
        if cap > ctx.params.max_particles:
            raise ValueError("capacity exceeds the context's max_particles")
        dev, dt = ctx.device, ctx.dtype
        nb = ctx.ncells * ctx.nspecies
        self.capacity = cap
        self.sets = []
        for _ in range(2):
            st = {"bin_start": torch.zeros(nb + 1, dtype=torch.int32, device=dev),
                  "cell": torch.zeros(max(cap, 1), dtype=torch.int32, device=dev)}
            if ctx.dim == 3:
                rec = torch.zeros((max(cap, 1), 8), dtype=dt, device=dev)
                st.update(xy=rec, uw=rec[:, 4:8], z=rec[:, 2])
            else:
                st.update(xy=torch.zeros((max(cap, 1), 2), dtype=dt, device=dev),
                          uw=torch.zeros((max(cap, 1), 4), dtype=dt, device=dev), z=None)
            self.sets.append(st)
        self.species_in = torch.zeros(max(cap, 1), dtype=torch.uint8, device=dev)
        self.s = _lib.relsim_particles()
        self.front = 0
        self.n = 0
        self._bind()

    def _bind(self):
        f, b = self.sets[self.front], self.sets[1 - self.front]
        s = self.s
        s.n = self.n
        s.bin_start, s.cell = f["bin_start"].data_ptr(), f["cell"].data_ptr()
        s.bin_start_back, s.cell_back = b["bin_start"].data_ptr(), b["cell"].data_ptr()
        s.xy, s.xy_back = f["xy"].data_ptr(), b["xy"].data_ptr()
        two = self.ctx.dim == 2  # in 3D the records are all in xy
        s.uw = f["uw"].data_ptr() if two else None
        s.uw_back = b["uw"].data_ptr() if two else None
        s.z = s.z_back = None
        s.species = self.species_in.data_ptr()

    def _sync_front(self):
        """After a call that may have swapped the sets inside the C struct."""
        self.front = 0 if self.s.xy == self.sets[0]["xy"].data_ptr() else 1
        self._bind()

    def load(self, cell, species, off, u, w, bin_start=None):
        """Copy host (numpy) particles in; sorts on the device unless bin_start is given."""
        n = int(np.asarray(w).shape[0])
        if n > self.capacity:
            raise ValueError("too many particles for this buffer")
        f = self.sets[self.front]
        dt = self.ctx.dtype
        dev = self.ctx.device
        self.n = n
        f["cell"][:n].copy_(torch.as_tensor(np.asarray(cell, dtype=np.int32)).to(dev))
        self.species_in[:n].copy_(torch.as_tensor(np.asarray(species, dtype=np.uint8)).to(dev))
        offs = np.asarray(off)
        uu = np.asarray(u)
        for d in range(self.ctx.dim):
            f["xy"][:n, d].copy_(torch.as_tensor(offs[d]).to(dev, dt))
        for k in range(3):
            f["uw"][:n, k].copy_(torch.as_tensor(uu[k]).to(dev, dt))
        f["uw"][:n, 3].copy_(torch.as_tensor(np.asarray(w)).to(dev, dt))
        self._bind()
        if bin_start is None:
            sort(self.ctx, self)
        else:
            f["bin_start"].copy_(torch.as_tensor(np.asarray(bin_start, dtype=np.int32)).to(dev))
        return self

    # front views (first n entries)
    @property
    def bin_start(self) -> torch.Tensor:
        return self.sets[self.front]["bin_start"]

    @property
    def cell(self) -> torch.Tensor:
        """Cell id per particle, written from the bin ranges on access
        (relsim_fill_cells): the push does not maintain it."""
        self.s.n = self.n
        self.ctx.check(self.ctx.lib.relsim_fill_cells(self.ctx.handle, C.byref(self.s)))
        return self.sets[self.front]["cell"][: self.n]

    @property
    def off(self):
        f = self.sets[self.front]
        return [f["xy"][: self.n, d] for d in range(self.ctx.dim)]

    @property
    def u(self):
        f = self.sets[self.front]
        return [f["uw"][: self.n, k] for k in range(3)]

    @property
    def w(self) -> torch.Tensor:
        return self.sets[self.front]["uw"][: self.n, 3]

    def species(self) -> torch.Tensor:
        """Species id of every front particle, from the bin layout."""
        bs = self.bin_start.long()
        counts = bs[1:] - bs[:-1]
        ids = torch.arange(counts.numel(), device=bs.device) % self.ctx.nspecies
        return torch.repeat_interleave(ids, counts)

    def to_host(self):
        """Front state as numpy (cell, species, off, u, w, bin_start)."""
        return (self.cell.cpu().numpy(), self.species().cpu().numpy().astype(np.uint8),
                np.stack([t.cpu().numpy() for t in self.off]), np.stack([t.cpu().numpy() for t in self.u]),
                self.w.cpu().numpy(), self.bin_start.cpu().numpy())


# ---------------------------------------------------------------------------
# entry points (names follow include/relsim.h)
# ---------------------------------------------------------------------------
def _grid_ok(ctx: Context, *ts):
    for t in ts:
        if t is None:
            continue
        if t.device != ctx.device or t.dtype != torch.float64 or not t.is_contiguous():
            raise ValueError("grid arrays must be contiguous float64 tensors on the context device")


def _mass_ok(ctx: Context, M):
    # the stored half of the node-pair blocks, [m_slots][9][N], in M's storage type
    if M.device != ctx.device or M.dtype != ctx.mass_dtype or not M.is_contiguous():
        raise ValueError("M must be a contiguous %s tensor on the context device" % ctx.mass_dtype)
    if M.numel() < ctx.m_slots * 9 * ctx.ncells:
        raise ValueError("M must hold [%d][9][%d] values" % (ctx.m_slots, ctx.ncells))


def sort(ctx: Context, parts: Particles) -> None:
    """relsim_sort"""
    parts.s.n = parts.n
    ctx.check(ctx.lib.relsim_sort(ctx.handle, C.byref(parts.s)))
    parts._sync_front()


def _gbar_ok(ctx: Context, parts: "Particles", *ts):
    for t in ts:
        if t is not None and (t.device != ctx.device or t.dtype != ctx.dtype or not t.is_contiguous()
                              or t.numel() < parts.n):
            raise ValueError("gbar arrays must be contiguous tensors of the particle type with at least n elements")


def deposit_moments(ctx: Context, parts: Particles, B: torch.Tensor, J: Optional[torch.Tensor] = None,
                    M: Optional[torch.Tensor] = None, gbar: Optional[torch.Tensor] = None):
    """relsim_deposit_moments -> (Jhat [3][N], M [m_slots][9][N]); with gbar
    (per particle, particle type), relsim_deposit_moments_ec"""
    J = ctx.grid() if J is None else J
    M = ctx.mass_matrix() if M is None else M
    _grid_ok(ctx, B, J)
    _mass_ok(ctx, M)
    parts.s.n = parts.n
    if gbar is None:
        ctx.check(ctx.lib.relsim_deposit_moments(ctx.handle, C.byref(parts.s), _ptr(B), _ptr(J), _ptr(M)))
    else:
        _gbar_ok(ctx, parts, gbar)
        ctx.check(ctx.lib.relsim_deposit_moments_ec(ctx.handle, C.byref(parts.s), _ptr(B), _ptr(gbar), _ptr(J),
                                                    _ptr(M)))
    return J, M


def gamma_mean(ctx: Context, parts: Particles, E_theta: torch.Tensor, B: torch.Tensor,
               gbar: Optional[torch.Tensor], gbar_next: torch.Tensor) -> float:
    """relsim_gamma_mean: gbar_next = (gamma(u^n) + gamma(u^{n+1}))/2 with
    u^{n+1} pushed using gbar (None: gamma(u^n)); returns max |gbar_next -
    gbar| / gbar"""
    _grid_ok(ctx, E_theta, B)
    _gbar_ok(ctx, parts, gbar, gbar_next)
    parts.s.n = parts.n
    out = C.c_double(0.0)
    ctx.check(ctx.lib.relsim_gamma_mean(ctx.handle, C.byref(parts.s), _ptr(E_theta), _ptr(B), _ptr(gbar),
                                        _ptr(gbar_next), C.byref(out)))
    return out.value


def placement_clamps(ctx: Context) -> int:
    """relsim_placement_clamps: particles the re-sort placed on a face of
    their counted cell since the last call (expected 0)"""
    out = C.c_int64(0)
    ctx.check(ctx.lib.relsim_placement_clamps(ctx.handle, C.byref(out)))
    return out.value


def field_solve(ctx: Context, M, J, E, B, E_theta=None, E1=None, B1=None, allow_unconverged: bool = False,
                guess: bool = False):
    """relsim_field_solve -> (E_theta, E^{n+1}, B^{n+1}, iterations, relative
    residual); with guess=True, relsim_field_solve_guess (GMRES starts from
    the E_theta given)"""
    if guess and E_theta is None:
        raise ValueError("guess=True needs E_theta (the initial guess)")
    E_theta = ctx.grid() if E_theta is None else E_theta
    E1 = ctx.grid() if E1 is None else E1
    B1 = ctx.grid() if B1 is None else B1
    _grid_ok(ctx, J, E, B, E_theta, E1, B1)
    _mass_ok(ctx, M)
    it = C.c_int32(0)
    rr = C.c_double(0.0)
    fn = ctx.lib.relsim_field_solve_guess if guess else ctx.lib.relsim_field_solve
    rc = fn(ctx.handle, _ptr(M), _ptr(J), _ptr(E), _ptr(B), _ptr(E_theta), _ptr(E1), _ptr(B1), C.byref(it),
            C.byref(rr))
    if not (allow_unconverged and rc == _lib.RELSIM_ENOTCONVERGED):
        ctx.check(rc)
    return E_theta, E1, B1, it.value, rr.value


def push(ctx: Context, parts: Particles, E_theta: torch.Tensor, B: torch.Tensor, resort: bool = True,
         new_index: Optional[torch.Tensor] = None, gbar: Optional[torch.Tensor] = None) -> None:
    """relsim_push (with resort: the pushed state goes into the back buffers
    in the new order and the sets swap, leaving the old state in the back
    set; new_index, int32 [n], receives each old particle's new position);
    with gbar, relsim_push_ec"""
    _grid_ok(ctx, E_theta, B)
    if new_index is not None and (new_index.dtype != torch.int32 or new_index.numel() < parts.n):
        raise ValueError("new_index must be an int32 tensor of at least n elements")
    parts.s.n = parts.n
    if gbar is None:
        ctx.check(ctx.lib.relsim_push(ctx.handle, C.byref(parts.s), _ptr(E_theta), _ptr(B), 1 if resort else 0,
                                      _ptr(new_index)))
    else:
        _gbar_ok(ctx, parts, gbar)
        ctx.check(ctx.lib.relsim_push_ec(ctx.handle, C.byref(parts.s), _ptr(E_theta), _ptr(B), _ptr(gbar),
                                         1 if resort else 0, _ptr(new_index)))
    parts._sync_front()


def apply_AT(ctx: Context, M: torch.Tensor, x: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """relsim_apply_AT"""
    out = ctx.grid() if out is None else out
    _grid_ok(ctx, x, out)
    _mass_ok(ctx, M)
    ctx.check(ctx.lib.relsim_apply_AT(ctx.handle, _ptr(M), _ptr(x), _ptr(out)))
    return out


def _f64(ctx: Context, *ts):
    for t in ts:
        if t.device != ctx.device or t.dtype != torch.float64 or not t.is_contiguous():
            raise ValueError("adjoint arrays must be contiguous float64 tensors on the context device")


def push_adjoint(ctx: Context, state: Particles, E_theta, B, new_index, lam_x_in, lam_u_in, lam_x_out, lam_u_out,
                 lam_E_theta, lam_B) -> None:
    """relsim_push_adjoint (lam_E_theta and lam_B are accumulated into)"""
    _f64(ctx, E_theta, B, lam_x_in, lam_u_in, lam_x_out, lam_u_out, lam_E_theta, lam_B)
    state.s.n = state.n
    ctx.check(ctx.lib.relsim_push_adjoint(ctx.handle, C.byref(state.s), _ptr(E_theta), _ptr(B), _ptr(new_index),
                                          _ptr(lam_x_in), _ptr(lam_u_in), _ptr(lam_x_out), _ptr(lam_u_out),
                                          _ptr(lam_E_theta), _ptr(lam_B)))


def field_solve_adjoint(ctx: Context, M, lam_E_theta, lam_E1, lam_B1, mu, lam_E, lam_B):
    """relsim_field_solve_adjoint -> (iterations, relative residual); lam_E, lam_B accumulated into"""
    _f64(ctx, M, lam_E_theta, lam_E1, lam_B1, mu, lam_E, lam_B)
    _mass_ok(ctx, M)
    it = C.c_int32(0)
    rr = C.c_double(0.0)
    ctx.check(ctx.lib.relsim_field_solve_adjoint(ctx.handle, _ptr(M), _ptr(lam_E_theta), _ptr(lam_E1), _ptr(lam_B1),
                                                 _ptr(mu), _ptr(lam_E), _ptr(lam_B), C.byref(it), C.byref(rr)))
    return it.value, rr.value


def deposit_adjoint(ctx: Context, state: Particles, B, E_theta, mu, lam_x, lam_u, lam_B) -> None:
    """relsim_deposit_adjoint (all three outputs accumulated into)"""
    _f64(ctx, B, E_theta, mu, lam_x, lam_u, lam_B)
    state.s.n = state.n
    ctx.check(ctx.lib.relsim_deposit_adjoint(ctx.handle, C.byref(state.s), _ptr(B), _ptr(E_theta), _ptr(mu),
                                             _ptr(lam_x), _ptr(lam_u), _ptr(lam_B)))


def energy(ctx: Context, parts: Particles, E: torch.Tensor, B: torch.Tensor) -> np.ndarray:
    """relsim_energy -> (kinetic, electric, magnetic, total)"""
    _grid_ok(ctx, E, B)
    out = (C.c_double * 4)()
    parts.s.n = parts.n
    ctx.check(ctx.lib.relsim_energy(ctx.handle, C.byref(parts.s), _ptr(E), _ptr(B), out))
    return np.array(list(out))


def energy_pushed(ctx: Context, E: torch.Tensor, B: torch.Tensor) -> np.ndarray:
    """relsim_energy_pushed -> (kinetic, electric, magnetic, total) of the
    state the last push with re-sort wrote (its kinetic part summed by that
    push)"""
    _grid_ok(ctx, E, B)
    out = (C.c_double * 4)()
    ctx.check(ctx.lib.relsim_energy_pushed(ctx.handle, _ptr(E), _ptr(B), out))
    return np.array(list(out))


def energy_noalloc(params, parts: Particles, E: torch.Tensor, B: torch.Tensor,
                   out: Optional[torch.Tensor] = None, stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
    """relsim_energy_noalloc: the S7 energy without a context or workspace,
    written asynchronously into out (4 float64 on the device: kinetic,
    electric, magnetic, total).  params: a Context or its relsim_params."""
    p = params.params if isinstance(params, Context) else params
    dev = E.device
    out = torch.empty(4, dtype=torch.float64, device=dev) if out is None else out
    for t in (E, B, out):
        if t.dtype != torch.float64 or not t.is_contiguous() or t.device != dev:
            raise ValueError("E, B and out must be contiguous float64 tensors on one device")
    st = torch.cuda.current_stream(dev) if stream is None else stream
    parts.s.n = parts.n
    rc = _lib.load().relsim_energy_noalloc(C.byref(p), C.c_void_p(st.cuda_stream), C.byref(parts.s), _ptr(E),
                                           _ptr(B), _ptr(out))
    if rc == _lib.RELSIM_ERANGE:
        raise RelsimError(rc, "relsim_energy_noalloc: the grid needs more than the 4 MiB of per-device scratch "
                              "(about 520,000 kinetic partials, one per 64/group cells)")
    if rc != _lib.RELSIM_OK:
        raise RelsimError(rc, "relsim_energy_noalloc: %s" % _lib.load().relsim_strerror(rc).decode())
    return out


class _SecantMix:
    """Per-particle secant steps for the fixed point g = F(g) through
    relsim_gamma_secant: with the residual r = F(g) - g of this pass and the
    last, each particle's next input is g - r (g - g_prev) / (r - r_prev),
    the root of the line through its last two residuals, where that line
    falls with a slope in [-10, -0.1] (an estimated contraction dF/dg in [-9,
    0.9]); elsewhere (first pass, a flat or rising residual, a step too small
    to measure) the plain update F(g).  Each particle's gbar is nearly its own
    scalar fixed point (the field couples them weakly), so a per-particle
    secant follows each one's own contraction rate.  The fixed point, the
    stopping test and the final push are those of the plain iteration."""

    def __init__(self, ctx: Context):
        self.ctx = ctx
        self.g_prev = self.r_prev = None

    def __call__(self, g: torch.Tensor, Fg: torch.Tensor) -> None:
        """g: the pass's input, Fg: its output; Fg is overwritten with the
        next input."""
        first = self.g_prev is None
        if first:
            self.g_prev = torch.empty(g.numel(), dtype=g.dtype, device=g.device)
            self.r_prev = torch.empty_like(self.g_prev)
        gamma_secant(self.ctx, g, Fg, self.g_prev, self.r_prev, first)


def gamma_secant(ctx: Context, gbar: torch.Tensor, gbar_next: torch.Tensor, g_prev: torch.Tensor,
                 r_prev: torch.Tensor, first: bool) -> None:
    """relsim_gamma_secant: gbar_next (the plain update F(gbar)) is replaced
    by the per-particle secant step; g_prev, r_prev (n elements of the
    particle type) carry the last pass's input and residual; first only
    records them."""
    n = gbar.numel()
    for t in (gbar, gbar_next):
        if t.device != ctx.device or t.dtype != ctx.dtype or not t.is_contiguous() or t.numel() < n:
            raise ValueError("gbar arrays must be contiguous tensors of the particle type")
    for t in (g_prev, r_prev):
        if t.device != ctx.device or t.dtype != ctx.dtype or not t.is_contiguous() or t.numel() < n:
            raise ValueError("g_prev and r_prev must be contiguous tensors of the particle type, n elements")
    ctx.check(ctx.lib.relsim_gamma_secant(ctx.handle, C.c_int64(n), _ptr(gbar), _ptr(gbar_next), _ptr(g_prev),
                                          _ptr(r_prev), 1 if first else 0))


class PicardNotConverged(RuntimeError):
    """The energy-conserving step's fixed point did not reach its tolerance."""

    def __init__(self, iters: int, change: float, tol: float):
        super().__init__("energy-conserving step: gbar change %.3e after %d passes (tolerance %.1e)"
                         % (change, iters, tol))
        self.iters, self.change, self.tol = iters, change, tol


class Step:
    """Advances a particle state and its fields by whole steps n -> n+1:
    relsim_deposit_moments (S1-S3), relsim_field_solve (S4-S5) and
    relsim_push with re-sort (S6 + a1), in that order, on the context's
    stream.  Holds E^n and B^n (copies of the tensors given) and the per-step
    grid arrays (J-hat, M, E_theta and the next fields), allocated once.

    energy_conserving=True takes gbar = (gamma^n + gamma^{n+1})/2 in place
    of gamma(u^n) (exact energy conservation when relativistic): each step
    iterates deposit -> solve -> relsim_gamma_mean from gbar = gamma(u^n)
    until the largest relative change of gbar is at most picard_tol (or
    picard_maxit passes), then pushes with the gbar of the last pass.  The
    default tolerance is 1e-12 in FP64 and 1e-6 in mixed precision (FP32
    particles round gbar at about 6e-8).  The iteration starts from one
    relsim_gamma_mean pass with the known E^n in place of E_theta (no
    deposit or solve), which lands nearer the fixed point than gamma(u^n);
    the fixed point itself does not depend on the start.
    picard_iters / picard_change hold the last step's passes and change.

    If the change is still above picard_tol after picard_maxit passes, or
    is not finite, the step raises PicardNotConverged before pushing (the
    state and fields stay at step n), since energy would then not be
    conserved to the stated tolerance; with allow_unconverged=True a finite
    change only clears picard_converged and the step goes on.

    secant=True replaces the plain update by per-particle
    secant steps (each particle's next gbar from the line through its last
    two residuals, see _SecantMix).

    warm_start=True (the default) starts each pass's GMRES after the first
    from the previous pass's E_theta (relsim_field_solve_guess); the solve's
    tolerance is unchanged."""

    def __init__(self, ctx: Context, parts: Particles, E: torch.Tensor, B: torch.Tensor,
                 energy_conserving: bool = False, picard_tol: Optional[float] = None, picard_maxit: int = 30,
                 allow_unconverged: bool = False, warm_start: bool = True, secant: bool = False):
        _grid_ok(ctx, E, B)
        self.ctx, self.parts = ctx, parts
        self.E, self.B = E.clone(), B.clone()
        self.J, self.M = ctx.grid(), ctx.mass_matrix()
        self.E_theta = ctx.grid()
        self._E1, self._B1 = ctx.grid(), ctx.grid()
        self.iters, self.rel_resid = 0, 0.0
        self.energy_conserving = energy_conserving
        if picard_tol is None:
            picard_tol = 1e-12 if ctx.precision == "fp64" else 1e-6
        self.picard_tol, self.picard_maxit = picard_tol, picard_maxit
        self.allow_unconverged = allow_unconverged
        self.warm_start = bool(warm_start)
        self.secant = bool(secant)
        self.picard_iters, self.picard_change, self.picard_converged = 0, 0.0, True
        self._pushed = False
        if energy_conserving:
            cap = max(parts.n, 1)
            self._gb = [torch.empty(cap, dtype=ctx.dtype, device=ctx.device) for _ in range(2)]

    def _solve(self, gbar, guess: bool = False):
        deposit_moments(self.ctx, self.parts, self.B, self.J, self.M, gbar=gbar)
        _, _, _, self.iters, self.rel_resid = field_solve(self.ctx, self.M, self.J, self.E, self.B, self.E_theta,
                                                          self._E1, self._B1, guess=guess)

    def __call__(self, steps: int = 1) -> "Step":
        for _ in range(steps):
            gbar = None
            if self.energy_conserving:
                gamma_mean(self.ctx, self.parts, self.E, self.B, None, self._gb[0])
                gbar, nxt = self._gb[0], 1
                mix = _SecantMix(self.ctx) if self.secant else None
                for it in range(1, self.picard_maxit + 1):
                    # after the first pass GMRES starts from the last pass's E_theta
                    self._solve(gbar, guess=self.warm_start and it > 1)
                    self.picard_change = gamma_mean(self.ctx, self.parts, self.E_theta, self.B, gbar, self._gb[nxt])
                    self.picard_iters = it
                    if self.picard_change <= self.picard_tol or it == self.picard_maxit:
                        break
                    if mix is not None:
                        # the mixed input overwrites F(g_k) in place
                        mix(gbar[: self.parts.n], self._gb[nxt][: self.parts.n])
                    gbar, nxt = self._gb[nxt], 1 - nxt
                self.picard_converged = self.picard_change <= self.picard_tol
                if not self.picard_converged and (not self.allow_unconverged or not np.isfinite(self.picard_change)):
                    raise PicardNotConverged(self.picard_iters, self.picard_change, self.picard_tol)
            else:
                self._solve(None)
            push(self.ctx, self.parts, self.E_theta, self.B, resort=True, gbar=gbar)
            self._pushed = True
            self.E, self._E1 = self._E1, self.E
            self.B, self._B1 = self._B1, self.B
        return self

    def energy(self) -> np.ndarray:
        """S7 of the current state: (kinetic, electric, magnetic, total); after
        a step, relsim_energy_pushed (the kinetic sum formed by the push),
        before the first, relsim_energy"""
        if self._pushed:
            return energy_pushed(self.ctx, self.E, self.B)
        return energy(self.ctx, self.parts, self.E, self.B)


def curl_nc(ctx: Context, x: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """relsim_curl_nc"""
    out = ctx.grid() if out is None else out
    _grid_ok(ctx, x, out)
    ctx.check(ctx.lib.relsim_curl_nc(ctx.handle, _ptr(x), _ptr(out)))
    return out


def curl_cn(ctx: Context, x: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """relsim_curl_cn"""
    out = ctx.grid() if out is None else out
    _grid_ok(ctx, x, out)
    ctx.check(ctx.lib.relsim_curl_cn(ctx.handle, _ptr(x), _ptr(out)))
    return out


def apply_A(ctx: Context, M: torch.Tensor, x: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """relsim_apply_A"""
    out = ctx.grid() if out is None else out
    _grid_ok(ctx, x, out)
    _mass_ok(ctx, M)
    ctx.check(ctx.lib.relsim_apply_A(ctx.handle, _ptr(M), _ptr(x), _ptr(out)))
    return out


def timing_enable(ctx: Context, on: bool = True) -> None:
    """relsim_timing_enable"""
    ctx.check(ctx.lib.relsim_timing_enable(ctx.handle, 1 if on else 0))


def timing_reset(ctx: Context) -> None:
    """relsim_timing_reset"""
    ctx.check(ctx.lib.relsim_timing_reset(ctx.handle))


def timing_read(ctx: Context) -> dict:
    """relsim_timing_read -> {kernel: (total_ms, launches)}"""
    cap = 64
    names = (C.c_char * 48 * cap)()
    ms = (C.c_double * cap)()
    cnt = (C.c_int64 * cap)()
    n = ctx.lib.relsim_timing_read(ctx.handle, cap, C.cast(names, C.c_void_p), ms, cnt)
    if n < 0:
        ctx.check(n)
    return {names[i].value.decode(): (ms[i], cnt[i]) for i in range(n)}
