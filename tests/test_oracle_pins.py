"""Pins of the CPU oracle against facts the method and the mathematics fix.

Each test names the property it checks.  Together they are chosen so that a
dropped term, a wrong sign or index, or a transposed operand anywhere in the
oracle fails at least one of them:

  rotation operator   alpha solves (I + [b]x) ubar = v; 2 alpha - I is a rotation
  gather/push         exact gyration angle 2 atan(Omega dt/2); exact E x B drift
  deposit             partition of unity; cold-plasma closed form; dense
                      brute-force assembly; node-pair symmetry and PSD; the
                      sampled-node deposit equals the full deposit's columns
  energy              one particle's closed form (relativistic and not); the
                      compensated sums exact for many equal terms
  curls               transpose pair; curl of a gradient vanishes; second-order
                      convergence to the analytic curl
  field solve         vacuum wave phase 2 atan(c dt sin(k dx/2)/dx) with exact
                      amplitude; direct LU vs GMRES; sym(A) >= I
  coupled step        cold plasma oscillation phase 2 atan(omega_p dt/2) and
                      exact energy (non-relativistic); relativistic
                      energy-budget identity
"""
import math

import numpy as np
import pytest

import oracle
from tests.helpers import normwise, random_state


def small_grid(dim=2, nonrel=False, **kw):
    base = dict(dim=dim, nx=4, ny=3, nz=3 if dim == 3 else 1, dx=1.1, dy=0.9, dz=1.3, dt=0.4, nonrel=nonrel)
    base.update(kw)
    return oracle.Grid(**base)


# ----------------------------------------------------------------------------
# rotation operator
# ----------------------------------------------------------------------------
def test_alpha_solves_implicit_rotation_and_is_a_cayley_map():
    rng = np.random.default_rng(1)
    for _ in range(50):
        b = rng.standard_normal(3) * rng.choice([1e-3, 0.3, 2.0, 30.0])
        al = oracle.alpha(b)
        cross = np.array([[0, -b[2], b[1]], [b[2], 0, -b[0]], [-b[1], b[0], 0]])
        # ubar - ubar x b = v  <=>  (I + [b]x) ubar = v : alpha is that inverse
        np.testing.assert_allclose(al @ (np.eye(3) + cross), np.eye(3), atol=1e-13)
        R = 2.0 * al - np.eye(3)
        np.testing.assert_allclose(R @ R.T, np.eye(3), atol=1e-13)
        assert abs(np.linalg.det(R) - 1.0) < 1e-12
        np.testing.assert_allclose(al @ b, b, rtol=1e-13, atol=1e-15)
        ev = np.sort(np.linalg.eigvalsh(0.5 * (al + al.T)))
        bb = b @ b
        np.testing.assert_allclose(ev, [1 / (1 + bb), 1 / (1 + bb), 1.0], rtol=1e-12)
        # rotation angle of 2 alpha - I is 2 atan|b|
        ang = math.acos(max(-1.0, min(1.0, (np.trace(R) - 1.0) / 2.0)))
        assert abs(ang - 2.0 * math.atan(math.sqrt(bb))) < 1e-7


# ----------------------------------------------------------------------------
# gather + push in analytic fields
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("q", [1.0, -1.0])
def test_gyration_angle_and_orbit_radius(q):
    g = small_grid(q=(q,), m=(1.7,), dt=0.3)
    Bz = 1.9
    B = np.zeros((3, g.N))
    B[2] = Bz
    E = np.zeros((3, g.N))
    u0 = np.array([[1.3], [-0.4], [0.7]])
    x = np.array([[1.234], [0.567]])
    sp = np.zeros(1, dtype=np.int32)
    gam = math.sqrt(1 + (u0 ** 2).sum())
    Omega = q * Bz / (g.m[0] * gam * g.c)
    phi = 2.0 * math.atan(abs(Omega) * g.dt / 2.0)
    xs, us = [x.copy()], [u0.copy()]
    u = u0
    for _ in range(9):
        x, u = oracle.push(g, x, u, sp, E, B)
        xs.append(x.copy())
        us.append(u.copy())
    for a, b in zip(us[:-1], us[1:]):
        a2, b2 = a[:2, 0], b[:2, 0]
        ang = math.atan2(a2[0] * b2[1] - a2[1] * b2[0], a2 @ b2)
        assert abs(ang + math.copysign(phi, q * Bz)) < 1e-12
        assert abs(np.linalg.norm(a) - np.linalg.norm(b)) < 1e-12
        assert abs(a[2, 0] - b[2, 0]) < 1e-14
    # unwrap positions and check they lie on a circle of radius dt|v_perp|/(2 sin(phi/2))
    L = np.array(g.L)[:, None]
    P = [xs[0][:, 0]]
    for k in range(1, len(xs)):
        d = xs[k][:, 0] - xs[k - 1][:, 0]
        d -= L[:, 0] * np.round(d / L[:, 0])
        P.append(P[-1] + d)
    P = np.array(P)
    R = g.dt * np.linalg.norm(u0[:2, 0]) / gam / (2.0 * math.sin(phi / 2.0))
    # centre from the first three points
    A = 2 * np.array([P[1] - P[0], P[2] - P[0]])
    rhs = np.array([P[1] @ P[1] - P[0] @ P[0], P[2] @ P[2] - P[0] @ P[0]])
    ctr = np.linalg.solve(A, rhs)
    np.testing.assert_allclose(np.linalg.norm(P - ctr, axis=1), R, rtol=1e-11)


def test_exb_drift_is_an_exact_fixed_point():
    g = small_grid(q=(1.0, -1.0), m=(1.0, 3.0), dt=0.7)
    Bz, Ey = 2.0, 1.2
    B = np.zeros((3, g.N)); B[2] = Bz
    E = np.zeros((3, g.N)); E[1] = Ey
    vE = g.c * Ey / Bz               # (E x B)/B^2 along +x
    gE = 1.0 / math.sqrt(1 - vE * vE)
    n = 6
    rng = np.random.default_rng(3)
    x = np.stack([rng.random(n) * g.L[0], rng.random(n) * g.L[1]])
    u = np.zeros((3, n)); u[0] = gE * vE
    sp = np.array([0, 1, 0, 1, 0, 1], dtype=np.int32)
    x1, u1 = oracle.push(g, x, u, sp, E, B)
    np.testing.assert_allclose(u1, u, atol=1e-14)
    d = x1 - x
    d -= np.array(g.L)[:, None] * np.round(d / np.array(g.L)[:, None])
    np.testing.assert_allclose(d[0], g.dt * vE, rtol=1e-13)
    np.testing.assert_allclose(d[1], 0.0, atol=1e-14)


# ----------------------------------------------------------------------------
# deposit
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("dim", [2, 3])
def test_partition_of_unity_sums(dim):
    g = small_grid(dim)
    rng = np.random.default_rng(10 + dim)
    x, u, w, sp, E, B = random_state(g, 200, rng)
    J, M = oracle.deposit(g, x, u, w, sp, B)
    al = oracle.alphas(g, x, u, sp, B).reshape(3, 3, -1)
    gb = np.sqrt(1 + (u * u).sum(0))
    q = np.asarray(g.q)[sp]
    m = np.asarray(g.m)[sp]
    beta = q * g.dt / (2 * m)
    v = np.einsum("ijp,jp->ip", al, u) / gb
    np.testing.assert_allclose(g.V * J.sum(axis=1), (w * q * v).sum(axis=1), rtol=1e-12, atol=1e-12)
    Msum = g.V * M.sum(axis=(0, 2)).reshape(3, 3)
    ref = np.einsum("p,ijp->ij", w * q * beta / gb, al)
    np.testing.assert_allclose(Msum, ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("dim", [2, 3])
def test_cold_uniform_plasma_row_sums(dim):
    """Same offsets in every cell, u = 0, B = 0: sum_g' M_gg' = dt omega_p^2/(8 pi) I."""
    g = small_grid(dim, q=(1.0, -1.0), m=(1.0, 4.0))
    rng = np.random.default_rng(7)
    ppc = 3
    offs = rng.random((dim, ppc))
    nz = g.nz if dim == 3 else 1
    cells = np.arange(g.N)
    ci, cj, ck = cells % g.nx, (cells // g.nx) % g.ny, cells // (g.nx * g.ny)
    h = [g.dx, g.dy, g.dz]
    xs, sps = [], []
    n_s = [0.8, 0.8]            # density per species
    for s in range(2):
        for k in range(ppc):
            xs.append(np.stack([(c + offs[d, k]) * h[d] for d, c in enumerate([ci, cj, ck][:dim])]))
            sps.append(np.full(g.N, s))
    x = np.concatenate(xs, axis=1)
    sp = np.concatenate(sps).astype(np.int32)
    w = np.array([n_s[s] * g.V / ppc for s in sp])
    u = np.zeros((3, x.shape[1]))
    B = np.zeros((3, g.N))
    J, M = oracle.deposit(g, x, u, w, sp, B)
    wp2 = sum(4 * math.pi * n_s[s] * g.q[s] ** 2 / g.m[s] for s in range(2))
    rows = M.sum(axis=0).reshape(3, 3, g.N)
    for gi in range(g.N):
        np.testing.assert_allclose(rows[:, :, gi], g.dt * wp2 / (8 * math.pi) * np.eye(3), atol=1e-14)
    assert np.abs(J).max() == 0.0


def _brute_force(g, x, u, w, sp):
    """Dense assembly with no offset bookkeeping: weights of every node and
    centre from the CIC hat function with minimum-image distances."""
    N = g.N
    nz = g.nz if g.dim == 3 else 1
    idx = np.arange(N)
    coord = [idx % g.nx, (idx // g.nx) % g.ny, idx // (g.nx * g.ny)]
    ext = [g.nx, g.ny, nz]
    h = [g.dx, g.dy, g.dz]

    def hat(p, shift):
        W = np.ones(N)
        for d in range(g.dim):
            s = x[d, p] / h[d] - (coord[d] + shift)
            s -= ext[d] * np.round(s / ext[d])
            W *= np.maximum(0.0, 1.0 - np.abs(s))
        return W

    return hat


@pytest.mark.parametrize("shape", [(2, 3, 3, 1), (2, 4, 4, 1), (2, 5, 3, 1), (3, 3, 3, 3), (3, 3, 4, 3)])
def test_dense_brute_force_assembly(shape):
    dim, nx, ny, nz = shape
    g = small_grid(dim, nx=nx, ny=ny, nz=nz)
    rng = np.random.default_rng(sum(shape))
    x, u, w, sp, E, B = random_state(g, 40, rng, bmax=3.0)
    hat = _brute_force(g, x, u, w, sp)
    N = g.N
    Md = np.zeros((3 * N, 3 * N))
    Jd = np.zeros(3 * N)
    for p in range(x.shape[1]):
        Wn = hat(p, 0.0)
        Wc = hat(p, 0.5)
        Bp = B @ Wc
        s = sp[p]
        gb = math.sqrt(1 + u[:, p] @ u[:, p])
        beta = g.q[s] * g.dt / (2 * g.m[s])
        b = beta * Bp / (gb * g.c)
        cross = np.array([[0, -b[2], b[1]], [b[2], 0, -b[0]], [-b[1], b[0], 0]])
        al = np.linalg.inv(np.eye(3) + cross)
        cM = w[p] * g.q[s] * beta / (g.V * gb)
        cJ = w[p] * g.q[s] / g.V
        Md += cM * np.kron(al, np.outer(Wn, Wn))
        Jd += cJ * np.kron(al @ u[:, p] / gb, Wn)
    J, M = oracle.deposit(g, x, u, w, sp, B)
    Ms = oracle.M_matrix(g, M).toarray()
    np.testing.assert_allclose(Ms, Md, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(J.reshape(-1), Jd, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("dim", [2, 3])
def test_mass_matrix_symmetry_and_psd(dim):
    g = small_grid(dim, nx=4, ny=4, nz=3)
    rng = np.random.default_rng(20 + dim)
    x, u, w, sp, E, B = random_state(g, 150, rng, bmax=4.0)
    J, M = oracle.deposit(g, x, u, w, sp, B)
    nz = g.nz if dim == 3 else 1
    idx = np.arange(g.N)
    i, j, k = idx % g.nx, (idx // g.nx) % g.ny, idx // (g.nx * g.ny)
    for off in range(g.noff):
        dx, dy, dz = off % 3 - 1, (off // 3) % 3 - 1, off // 9 - 1
        opp = (1 - dx) + 3 * (1 - dy) + (9 * (1 - dz) if dim == 3 else 0)
        gj = (i + dx) % g.nx + g.nx * (((j + dy) % g.ny) + g.ny * ((k + dz) % nz))
        # M_{g,g'} = M_{g',g} (same weight product, same alpha; equal up to
        # the rounding order of the weight product)
        np.testing.assert_allclose(M[off][:, idx], M[opp][:, gj], rtol=1e-14, atol=1e-16)
    Ms = oracle.M_matrix(g, M).toarray()
    ev = np.linalg.eigvalsh(0.5 * (Ms + Ms.T))
    assert ev.min() > -1e-13 * ev.max()
    # with B = 0 every alpha is the identity and the matrix is symmetric
    J0, M0 = oracle.deposit(g, x, u, w, sp, np.zeros_like(B))
    M0s = oracle.M_matrix(g, M0).toarray()
    np.testing.assert_allclose(M0s, M0s.T, rtol=1e-14, atol=1e-16)
    # while with B != 0 the skew parts of alpha make it non-symmetric
    assert np.abs(Ms - Ms.T).max() > 1e-3 * np.abs(Ms).max()


# ----------------------------------------------------------------------------
# curls
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("dim", [2, 3])
def test_curl_pair_is_a_transpose_and_annihilates_gradients(dim):
    g = small_grid(dim, nx=5, ny=4, nz=3)
    Cnc = oracle.curl_matrix(g, True)
    Ccn = oracle.curl_matrix(g, False)
    assert abs(Ccn - Cnc.T).max() == 0.0
    rng = np.random.default_rng(5)
    E = rng.standard_normal((3, g.N))
    B = rng.standard_normal((3, g.N))
    np.testing.assert_allclose(oracle.curl_nc(g, E).ravel(), Cnc @ E.ravel(), atol=1e-13)
    np.testing.assert_allclose(oracle.curl_cn(g, B).ravel(), Ccn @ B.ravel(), atol=1e-13)
    # gradients built from the same averaged differences
    phi = rng.standard_normal(g.N)
    Gnc = np.stack([oracle._diff_matrix(g, d, True) @ phi for d in range(3)])
    Gcn = np.stack([oracle._diff_matrix(g, d, False) @ phi for d in range(3)])
    assert np.abs(oracle.curl_cn(g, Gnc)).max() < 1e-12
    assert np.abs(oracle.curl_nc(g, Gcn)).max() < 1e-12


def test_curl_converges_to_analytic_curl_at_second_order():
    errs = []
    for n in (16, 32):
        g = oracle.Grid(dim=3, nx=n, ny=n, nz=n, dx=1.0 / n, dy=1.0 / n, dz=1.0 / n)
        idx = np.arange(g.N)
        i, j, k = idx % n, (idx // n) % n, idx // (n * n)
        X, Y, Z = i / n, j / n, k / n
        tp = 2 * math.pi
        F = np.stack([np.sin(tp * Y) * np.cos(tp * Z), np.sin(tp * Z) * np.cos(tp * X), np.sin(tp * X) * np.cos(tp * Y)])
        # analytic curl at centres
        Xc, Yc, Zc = X + 0.5 / n, Y + 0.5 / n, Z + 0.5 / n
        cx = -tp * np.sin(tp * Xc) * np.sin(tp * Yc) - tp * np.cos(tp * Zc) * np.cos(tp * Xc)
        cy = -tp * np.sin(tp * Yc) * np.sin(tp * Zc) - tp * np.cos(tp * Xc) * np.cos(tp * Yc)
        cz = -tp * np.sin(tp * Zc) * np.sin(tp * Xc) - tp * np.cos(tp * Yc) * np.cos(tp * Zc)
        num = oracle.curl_nc(g, F)
        errs.append(np.abs(num - np.stack([cx, cy, cz])).max())
    order = math.log2(errs[0] / errs[1])
    assert errs[1] < 0.2 and 1.8 < order < 2.3, (errs, order)


# ----------------------------------------------------------------------------
# field solve
# ----------------------------------------------------------------------------
def test_vacuum_wave_phase_and_amplitude():
    n, ny = 24, 3
    g = oracle.Grid(dim=2, nx=n, ny=ny, dx=0.7, dy=0.5, dt=0.9)
    kx = 2 * math.pi * 3 / (n * g.dx)
    idx = np.arange(g.N)
    i = idx % n
    xn = i * g.dx
    xc = (i + 0.5) * g.dx
    E = np.zeros((3, g.N)); B = np.zeros((3, g.N))
    E[1] = np.cos(kx * xn)
    B[2] = 0.3 * np.sin(kx * xc)
    M = np.zeros((g.noff, 9, g.N)); J = np.zeros((3, g.N))

    def amps(E, B):
        a = (E[1] * np.exp(-1j * kx * xn)).sum()
        b = (B[2] * np.exp(-1j * kx * xc)).sum()
        return a + b, a - b

    p0, m0 = amps(E, B)
    W0 = (E ** 2).sum() + (B ** 2).sum()
    steps = 7
    for _ in range(steps):
        r = oracle.rhs(g, E, B, J)
        Eth = oracle.solve(g, M, r)
        E, B = oracle.field_update(g, E, B, Eth)
    p1, m1 = amps(E, B)
    phi = 2 * math.atan(g.c * g.dt * math.sin(kx * g.dx / 2) / g.dx)
    np.testing.assert_allclose(p1, p0 * np.exp(-1j * steps * phi), rtol=1e-11)
    np.testing.assert_allclose(m1, m0 * np.exp(1j * steps * phi), rtol=1e-11)
    assert abs((E ** 2).sum() + (B ** 2).sum() - W0) < 1e-12 * W0


@pytest.mark.parametrize("dim", [2, 3])
def test_direct_and_gmres_agree_and_sym_A_dominates_identity(dim):
    g = small_grid(dim, nx=5, ny=4, nz=3, dt=0.8)
    rng = np.random.default_rng(30 + dim)
    x, u, w, sp, E, B = random_state(g, 300, rng, bmax=3.0)
    J, M = oracle.deposit(g, x, u, w, sp, B)
    r = oracle.rhs(g, E, B, J)
    e1 = oracle.solve(g, M, r)
    e2 = oracle.solve(g, M, r, direct_limit=0, rtol=1e-14)
    assert normwise(e2, e1) < 1e-12
    A = oracle.A_matrix(g, M).toarray()
    np.testing.assert_allclose(A @ e1.ravel(), r.ravel(), atol=1e-12)
    # the matrix-free operator matches the assembled one
    v = rng.standard_normal((3, g.N))
    np.testing.assert_allclose(oracle.apply_A(g, M, v).ravel(), A @ v.ravel(), atol=1e-12)
    ev = np.linalg.eigvalsh(0.5 * (A + A.T))
    assert ev.min() > 1.0 - 1e-12


# ----------------------------------------------------------------------------
# coupled step
# ----------------------------------------------------------------------------
def test_cold_plasma_oscillation_nonrelativistic():
    g = oracle.Grid(dim=2, nx=4, ny=3, dx=1.0, dy=1.0, dt=0.6, nonrel=True, q=(1.0, -1.0), m=(1.0, 1.0))
    ppc = 2
    n_s = 0.5
    rng = np.random.default_rng(4)
    offs = rng.random((2, ppc))
    cells = np.arange(g.N)
    ci, cj = cells % g.nx, cells // g.nx
    xs, sps = [], []
    for s in range(2):
        for k in range(ppc):
            xs.append(np.stack([(ci + offs[0, k]) * g.dx, (cj + offs[1, k]) * g.dy]))
            sps.append(np.full(g.N, s))
    x = np.concatenate(xs, axis=1)
    sp = np.concatenate(sps).astype(np.int32)
    w = np.full(x.shape[1], n_s * g.V / ppc)
    U0 = 0.05
    u = np.zeros((3, x.shape[1])); u[0] = np.where(sp == 0, U0, -U0)
    E = np.zeros((3, g.N)); B = np.zeros((3, g.N))
    wp = math.sqrt(2 * 4 * math.pi * n_s / 1.0)
    z0 = E[0].mean() + 1j * wp * U0
    W0 = oracle.energy(g, u, w, sp, E, B)[3]
    steps = 6
    for _ in range(steps):
        out = oracle.step(g, x, u, w, sp, E, B)
        x, u, E, B = out["x"], out["u"], out["E"], out["B"]
        assert abs(out["W"][3] - W0) < 1e-13 * W0
    np.testing.assert_allclose(E[0], E[0].mean(), atol=1e-13)
    U = u[0][sp == 0].mean()
    z = E[0].mean() + 1j * wp * U
    phi = 2 * math.atan(wp * g.dt / 2)
    np.testing.assert_allclose(z, z0 * np.exp(1j * steps * phi), rtol=1e-11)


@pytest.mark.parametrize("dim", [2, 3])
def test_relativistic_energy_budget_identity(dim):
    g = small_grid(dim, nx=5, ny=4, nz=3, dt=0.5)
    rng = np.random.default_rng(40 + dim)
    x, u, w, sp, E, B = random_state(g, 400, rng, umax=3.0, bmax=1.5, emax=0.4)
    W0 = oracle.energy(g, u, w, sp, E, B)
    out = oracle.step(g, x, u, w, sp, E, B)
    W1 = out["W"]
    Ep = oracle.gather_E(g, x, out["E_theta"])
    ubar = 0.5 * (u + out["u"])
    g0 = np.sqrt(1 + (u * u).sum(0))
    g1 = np.sqrt(1 + (out["u"] ** 2).sum(0))
    q = np.asarray(g.q)[sp]
    pred = (w * q * g.dt * (Ep * ubar).sum(0) * (2.0 / (g0 + g1) - 1.0 / g0)).sum()
    dW = W1[3] - W0[3]
    assert abs(dW - pred) < 1e-12 * W0[3], (dW, pred)
    # the budget term is not negligible here, so the identity is a real check
    assert abs(pred) > 1e-6 * W0[3]


def test_nonrelativistic_energy_conserved_to_solver_tolerance():
    g = small_grid(2, nx=6, ny=5, dt=0.5, nonrel=True)
    rng = np.random.default_rng(50)
    x, u, w, sp, E, B = random_state(g, 300, rng, umax=0.3, bmax=1.0, emax=0.2)
    W0 = oracle.energy(g, u, w, sp, E, B)[3]
    for _ in range(5):
        out = oracle.step(g, x, u, w, sp, E, B)
        x, u, E, B = out["x"], out["u"], out["E"], out["B"]
        assert abs(out["W"][3] - W0) < 1e-13 * W0


@pytest.mark.parametrize("dim", [2, 3])
def test_energy_conserving_variant_conserves_energy_when_relativistic(dim):
    """gbar = (gamma^n + gamma^{n+1})/2 zeroes the budget term of the identity
    above: the fixed point conserves W to solver tolerance where the standard
    step does not."""
    g = small_grid(dim, nx=5, ny=4, nz=3, dt=0.5)
    rng = np.random.default_rng(60 + dim)
    x, u, w, sp, E, B = random_state(g, 400, rng, umax=3.0, bmax=1.5, emax=0.4)
    W0 = oracle.energy(g, u, w, sp, E, B)[3]
    std = oracle.step(g, x, u, w, sp, E, B)
    assert abs(std["W"][3] - W0) > 1e-6 * W0
    for _ in range(3):
        out = oracle.step_ec(g, x, u, w, sp, E, B, tol=1e-15)
        assert out["iters"] < 50 and out["change"] <= 1e-15
        # the kept pass is self-consistent and conserves energy
        g0 = np.sqrt(1 + (u * u).sum(0))
        g1 = np.sqrt(1 + (out["u"] ** 2).sum(0))
        np.testing.assert_allclose(out["gbar"], 0.5 * (g0 + g1), rtol=2e-15)
        assert abs(out["W"][3] - W0) < 1e-12 * W0, (out["W"][3] - W0) / W0
        x, u, E, B = out["x"], out["u"], out["E"], out["B"]


def test_energy_conserving_variant_reduces_to_the_standard_step():
    """With gbar = gamma(u^n) given explicitly, deposit and push are the
    standard ones; without relativity gbar plays no part and step_ec is step."""
    g = small_grid(2, nx=5, ny=4, dt=0.5)
    rng = np.random.default_rng(70)
    x, u, w, sp, E, B = random_state(g, 300, rng, umax=3.0, bmax=1.5, emax=0.4)
    g0 = oracle.gamma(g, u)
    J0, M0 = oracle.deposit(g, x, u, w, sp, B)
    J1, M1 = oracle.deposit(g, x, u, w, sp, B, g0)
    assert np.array_equal(J0, J1) and np.array_equal(M0, M1)
    assert all(np.array_equal(a, b) for a, b in zip(oracle.push(g, x, u, sp, E, B), oracle.push(g, x, u, sp, E, B, g0)))
    gn = small_grid(2, nx=5, ny=4, dt=0.5, nonrel=True)
    a = oracle.step(gn, x, 0.1 * u, w, sp, E, B)
    b = oracle.step_ec(gn, x, 0.1 * u, w, sp, E, B)
    assert b["iters"] == 1
    for k in ("E", "B", "x", "u", "W"):
        assert np.array_equal(a[k], b[k])


# ----------------------------------------------------------------------------
# sampled-node deposit (the reference of the full-size parity checks)
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("shape", [(2, 3, 3, 1), (2, 7, 5, 1), (3, 3, 3, 3), (3, 5, 4, 3)])
def test_deposit_nodes_equals_the_full_deposit_columns(shape):
    """deposit_nodes adds, into each sampled node, the same terms in the same
    particle order as deposit (itself pinned by the dense brute force above),
    so its result is those columns bit for bit, for any sample of nodes."""
    dim, nx, ny, nz = shape
    g = small_grid(dim, nx=nx, ny=ny, nz=nz)
    rng = np.random.default_rng(300 + nx * ny * nz)
    x, u, w, sp, E, B = random_state(g, 700, rng, umax=3.0, bmax=2.0)
    J, M = oracle.deposit(g, x, u, w, sp, B)
    for nodes in (np.arange(g.N), rng.permutation(g.N)[: max(1, g.N // 3)], np.array([g.N - 1, 0])):
        Jn, Mn = oracle.deposit_nodes(g, x, u, w, sp, B, nodes)
        np.testing.assert_array_equal(Jn, J[:, nodes])
        np.testing.assert_array_equal(Mn, M[:, :, nodes])
    # no particles: exact zeros
    Jn, Mn = oracle.deposit_nodes(g, x[:, :0], u[:, :0], w[:0], sp[:0], B, np.arange(g.N))
    assert not Jn.any() and not Mn.any()


def test_deposit_nodes_rejects_repeated_or_out_of_range_nodes():
    g = small_grid(2, nx=4, ny=3)
    rng = np.random.default_rng(5)
    x, u, w, sp, E, B = random_state(g, 50, rng)
    for bad in ([0, 3, 3], [g.N], [-1]):
        with pytest.raises(ValueError):
            oracle.deposit_nodes(g, x, u, w, sp, B, np.array(bad))


# ----------------------------------------------------------------------------
# S7 energy sums
# ----------------------------------------------------------------------------
def test_kinetic_energy_of_one_particle_closed_form():
    """w m c^2 (gamma - 1) with |u| = 5 c (gamma = sqrt 26), and w m |u|^2 / 2
    without relativity; fields enter as V/(8 pi) sum |F|^2."""
    g = small_grid(2, nx=3, ny=3, c=2.0, q=(1.0, -1.0), m=(3.0, 0.5))
    u = np.array([[3.0 * 2.0], [0.0], [4.0 * 2.0]])
    w = np.array([0.7])
    E = np.zeros((3, g.N))
    B = np.zeros((3, g.N))
    E[1, 4] = 2.0
    B[2, 0] = 3.0
    W = oracle.energy(g, u, w, np.array([1], np.int32), E, B)
    assert abs(W[0] - 0.7 * 0.5 * 4.0 * (math.sqrt(26.0) - 1.0)) <= 4e-16 * W[0]
    assert abs(W[1] - g.V / (8 * math.pi) * 4.0) <= 4e-16 * W[1]
    assert abs(W[2] - g.V / (8 * math.pi) * 9.0) <= 4e-16 * W[2]
    gn = small_grid(2, nx=3, ny=3, c=2.0, q=(1.0, -1.0), m=(3.0, 0.5), nonrel=True)
    Wn = oracle.energy(gn, u, w, np.array([1], np.int32), E, B)
    assert abs(Wn[0] - 0.5 * 0.7 * 0.5 * 100.0) <= 4e-16 * Wn[0]


def test_energy_sums_are_exact_for_many_equal_terms():
    """Many equal terms: the sum is n times one term (computed once, in
    exact integer multiples) to a few ulps, whatever n.  A plain running sum
    drifts by about n/2 ulps here (shown beside it), so this pins the
    compensated summation the full-size energy checks rely on."""
    n = 1 << 21
    g = small_grid(2, nx=1024, ny=1024)
    u = np.tile(np.array([[0.1], [0.3], [0.7]]), (1, n))
    w = np.full(n, 0.1)
    sp = np.zeros(n, np.int32)
    E = np.full((3, g.N), 0.1)
    B = np.full((3, g.N), 0.3)
    W = oracle.energy(g, u, w, sp, E, B)
    uu = 0.1 * 0.1 + 0.3 * 0.3 + 0.7 * 0.7
    term = 0.1 * 1.0 * uu / (math.sqrt(1.0 + uu) + 1.0)
    eps = np.finfo(np.float64).eps
    assert abs(W[0] - n * term) <= 4 * eps * n * term
    assert abs(W[1] - g.V / (8 * math.pi) * (3 * g.N) * (0.1 * 0.1)) <= 8 * eps * W[1]
    assert abs(W[2] - g.V / (8 * math.pi) * (3 * g.N) * (0.3 * 0.3)) <= 8 * eps * W[2]
    naive = np.cumsum(np.full(n, term))[-1]
    assert abs(naive - n * term) > 100 * eps * n * term
