"""Independent PyTorch (CPU, FP64) implementation of one semi-implicit step,
differentiable by torch autograd: the reference gradient for the adjoint.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Same equations as the
C oracle (S1-S6 of ``relsim_oracle.c``), written with tensor operations on
physical positions: CIC weights from floor(), the J-hat/M deposit assembled
densely (3N x 3N, component-major rows r*N + g), the curl matrices from
``oracle.curl_matrix``, and a dense solve.  Meant for small grids only.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import Grid, curl_matrix


def _dense(sp_matrix) -> torch.Tensor:
    return torch.as_tensor(sp_matrix.toarray(), dtype=torch.float64)


class TorchStep:
    def __init__(self, g: Grid):
        self.g = g
        self.Cnc = _dense(curl_matrix(g, True))
        self.Ccn = _dense(curl_matrix(g, False))
        self.q = torch.tensor(list(g.q), dtype=torch.float64)
        self.m = torch.tensor(list(g.m), dtype=torch.float64)

    def _cic(self, x: torch.Tensor, shift: float):
        """Corner node indices (2^dim, n) and weights (2^dim, n), differentiable in x."""
        g = self.g
        h = [g.dx, g.dy, g.dz]
        ext = [g.nx, g.ny, g.nz if g.dim == 3 else 1]
        base, frac = [], []
        for d in range(g.dim):
            s = x[d] / h[d] - shift
            fl = torch.floor(s.detach())
            base.append(fl.long())
            frac.append(s - fl)
        idx, wts = [], []
        for a in range(1 << g.dim):
            o = [(a >> d) & 1 for d in range(g.dim)]
            w = torch.ones_like(x[0])
            lin = torch.zeros_like(base[0])
            mul = 1
            for d in range(g.dim):
                w = w * (frac[d] if o[d] else 1.0 - frac[d])
                lin = lin + mul * torch.remainder(base[d] + o[d], ext[d])
                mul *= ext[d]
            idx.append(lin)
            wts.append(w)
        return torch.stack(idx), torch.stack(wts)

    def _gather(self, F: torch.Tensor, idx, wts):
        return torch.stack([(wts * F[k][idx]).sum(0) for k in range(3)])

    def _alpha(self, b: torch.Tensor) -> torch.Tensor:
        """(n, 3, 3) alpha = (I - [b]x + b b^T)/(1 + b^2)."""
        n = b.shape[1]
        bx, by, bz = b[0], b[1], b[2]
        z = torch.zeros_like(bx)
        cross = torch.stack([torch.stack([z, -bz, by], -1), torch.stack([bz, z, -bx], -1),
                             torch.stack([-by, bx, z], -1)], -2)
        eye = torch.eye(3, dtype=torch.float64).expand(n, 3, 3)
        outer = b.T[:, :, None] * b.T[:, None, :]
        return (eye - cross + outer) / (1.0 + (b * b).sum(0))[:, None, None]

    def step(self, x, u, w, sp, E, B):
        """One step; x [dim][n], u [3][n], E/B [3][N] tensors; returns (x', u', E', B', E_theta)."""
        g = self.g
        N = g.N
        c = g.c
        th = g.theta
        spi = torch.as_tensor(np.asarray(sp), dtype=torch.long)
        q = self.q[spi]
        m = self.m[spi]
        beta = q * g.dt / (2.0 * m)
        idn, wn = self._cic(x, 0.0)
        idc, wc = self._cic(x, 0.5)
        Bp = self._gather(B, idc, wc)
        gb = torch.ones_like(u[0]) if g.nonrel else torch.sqrt(1.0 + (u * u).sum(0) / (c * c))
        b = beta * Bp / (gb * c)
        al = self._alpha(b)                                   # (n, 3, 3)
        V = g.V
        cJ = w * q / V
        cM = w * q * beta / (V * gb)
        v = torch.einsum("pij,jp->ip", al, u) / gb            # alpha u / gbar
        # J-hat
        J = torch.zeros(3 * N, dtype=torch.float64)
        for a in range(idn.shape[0]):
            for k in range(3):
                J = J.index_add(0, k * N + idn[a], cJ * wn[a] * v[k])
        # dense M
        Md = torch.zeros(9 * N * N, dtype=torch.float64)
        for a in range(idn.shape[0]):
            for bb in range(idn.shape[0]):
                ww = cM * wn[a] * wn[bb]
                for r in range(3):
                    for cc in range(3):
                        flat = (r * N + idn[a]) * (3 * N) + (cc * N + idn[bb])
                        Md = Md.index_add(0, flat, ww * al[:, r, cc])
        Md = Md.reshape(3 * N, 3 * N)
        aa = c * th * g.dt
        bm = 4.0 * math.pi * th * g.dt
        A = torch.eye(3 * N, dtype=torch.float64) + aa * aa * (self.Ccn @ self.Cnc) + bm * Md
        rhs = E.reshape(-1) + aa * (self.Ccn @ B.reshape(-1)) - bm * J
        Eth = torch.linalg.solve(A, rhs).reshape(3, N)
        B1 = B - c * g.dt * (self.Cnc @ Eth.reshape(-1)).reshape(3, N)
        E1 = (Eth - (1.0 - th) * E) / th
        Ep = self._gather(Eth, idn, wn)
        ub = torch.einsum("pij,jp->ip", al, u + beta * Ep)
        un = 2.0 * ub - u
        gn = torch.ones_like(u[0]) if g.nonrel else torch.sqrt(1.0 + (un * un).sum(0) / (c * c))
        L = torch.tensor(g.L, dtype=torch.float64)[:, None]
        xn = x + g.dt * un[: g.dim] / gn
        xn = xn - L * torch.floor(xn.detach() / L)
        return xn, un, E1, B1, Eth

    def field_energy(self, E, B):
        return self.g.V / (8.0 * math.pi) * ((E * E).sum() + (B * B).sum())
