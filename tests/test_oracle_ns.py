"""Pins of the oracle's momentum step (sections 2, 3.2, 4.2.3, 4.3 and 4.4), CPU only.

- Pressure solve: equals the zero-mean solution of the 5/7-point Laplacian with zero flux through
  the box walls, assembled cell by cell here and solved with a sparse direct solver.
- Convective and viscous operators: second-order convergence to the analytic div(u u_a) and
  div(mu (grad u + grad u^T)) of smooth fields with the wall symmetries of no-slip box walls
  (tangential velocity odd, normal velocity zero, viscosity even), in 2D and 3D.
- A parallel channel flow driven by a body force follows the one-dimensional forward-Euler
  recurrence of the viscous term with the no-slip images, assembled independently.
- The projection leaves a discretely divergence-free velocity (to round-off) with a density ratio
  of 10, a viscosity ratio of 5 and an immersed wall: the pressure equation and the correction are
  consistent with each other whatever the pressure history.
- A drop at rest: the pressure balancing the capillary force jumps by 1/(Re Ca R) across the
  interface (Laplace), which fixes the capillary coefficient.
- Staggered-cell volume fractions of a flat wall: closed form.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import workloads as W
from oracle import ns
from oracle.geometry import build_tables, face_fractions, volume_fraction
from oracle.solver import OracleState


def _lin(n, idx):
    """Linear cell index, x fastest."""
    out = 0
    mul = 1
    for a in range(len(n)):
        out += idx[a] * mul
        mul *= n[a]
    return out


@pytest.mark.parametrize("n", [(8, 6), (6, 4, 5)])
def test_poisson_equals_assembled_neumann_laplacian(n):
    d = len(n)
    h = 0.25
    grid = W.Grid(n, (0.0,) * d, tuple(h * v for v in n))
    N = int(np.prod(n))
    rows, cols, vals = [], [], []
    for c in range(N):
        idx = []
        r = c
        for a in range(d):
            idx.append(r % n[a])
            r //= n[a]
        for a in range(d):
            for s in (-1, 1):
                q = list(idx)
                q[a] += s
                if a < d - 1:
                    q[a] %= n[a]
                elif q[a] < 0 or q[a] >= n[a]:
                    continue                  # no flux through a box wall
                rows += [c, c]
                cols += [_lin(n, q), c]
                vals += [1.0 / h ** 2, -1.0 / h ** 2]
    L = sp.csr_matrix((vals, (rows, cols)), shape=(N, N))
    rng = np.random.default_rng(5)
    R = rng.standard_normal(N)
    R -= R.mean()
    A = sp.bmat([[L, np.ones((N, 1))], [np.ones((1, N)), None]]).tocsc()
    ref = spla.spsolve(A, np.concatenate([R, [0.0]]))[:N]
    got = ns.poisson_solve(R.reshape(tuple(reversed(n))), grid).reshape(-1)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
    assert abs(got.mean()) <= 1e-14 * np.max(np.abs(ref))


def _fields_2d(X, Y):
    u = np.sin(2 * np.pi * X) * np.sin(2 * np.pi * Y)
    v = np.cos(2 * np.pi * X) * np.sin(np.pi * Y)
    mu = 1.0 + 0.3 * np.cos(2 * np.pi * X) * np.cos(2 * np.pi * Y)
    return [u, v], mu


def _fields_3d(X, Y, Z):
    u = np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y) * np.sin(2 * np.pi * Z)
    v = np.cos(2 * np.pi * X) * np.sin(4 * np.pi * Y) * np.sin(2 * np.pi * Z)
    w = np.cos(2 * np.pi * X) * np.cos(2 * np.pi * Y) * np.sin(np.pi * Z)
    mu = 1.0 + 0.3 * np.cos(2 * np.pi * X) * np.sin(2 * np.pi * Y) * np.cos(2 * np.pi * Z)
    return [u, v, w], mu


def _analytic(fields, X, a, d):
    """div(u u_a) and div(mu (grad u + grad u^T))_a at points X by central differences of the
    analytic fields with a tiny step (independent of the staggered discretisation)."""
    e = 1e-5

    def at(P):
        return fields(*P)

    def dd(fun, b):
        Pp = list(X)
        Pm = list(X)
        Pp[b] = Pp[b] + e
        Pm[b] = Pm[b] - e
        return (fun(Pp) - fun(Pm)) / (2 * e)

    conv = sum(dd(lambda P: at(P)[0][a] * at(P)[0][b], b) for b in range(d))

    def stress(P, b):
        def du(q, k):                      # d u_q / d x_k at P
            Pp = list(P)
            Pm = list(P)
            Pp[k] = Pp[k] + e
            Pm[k] = Pm[k] - e
            return (at(Pp)[0][q] - at(Pm)[0][q]) / (2 * e)
        return at(P)[1] * (du(a, b) + du(b, a))

    visc = 0.0
    for b in range(d):
        Pp = list(X)
        Pm = list(X)
        Pp[b] = Pp[b] + 1e-4
        Pm[b] = Pm[b] - 1e-4
        visc = visc + (stress(Pp, b) - stress(Pm, b)) / 2e-4
    return conv, visc


@pytest.mark.parametrize("d", [2, 3])
def test_convective_and_viscous_operators_are_second_order(d):
    errs = []
    for m in (16, 32):
        n = (m,) * d
        grid = W.Grid(n, (0.0,) * d, (1.0,) * d)
        h = grid.h
        cc = W.cell_centres(grid)
        cc = [np.broadcast_to(c, grid.shape) for c in cc]
        fields = _fields_2d if d == 2 else _fields_3d
        faces = []
        for a in range(d):
            P = [cc[b] + (0.5 * h if b == a else 0.0) for b in range(d)]
            faces.append(fields(*P)[0][a])
        mu = fields(*cc)[1]
        N = ns.convective(faces, grid)
        V = ns.viscous(faces, mu, grid)
        e = []
        for a in range(d):
            P = [cc[b] + (0.5 * h if b == a else 0.0) for b in range(d)]
            conv, visc = _analytic(fields, P, a, d)
            sl = (slice(0, -1),) if a == d - 1 else (slice(None),)   # the top wall faces are fixed
            e.append(np.max(np.abs(N[a] - conv)[sl]))
            e.append(np.max(np.abs(V[a] - visc)[sl]))
        errs.append(np.array(e))
    ratio = errs[0] / errs[1]
    assert np.all(ratio > 3.3), (errs, ratio)


def _channel(ny=16, nx=8, steps=40, g=1.0):
    grid = W.Grid((nx, ny), (0.0, 0.0), (nx / ny, 1.0))
    prm = W.Params(Cn=0.05, Pe=10.0, Re=10.0, Ca=0.1, dt=2e-4, navier_stokes=True, body_force=(g, 0.0))
    T = build_tables(grid, [], prm)
    C0 = -np.ones(grid.shape)
    o = OracleState(grid, prm, T, C0, face_alpha=[np.ones(grid.shape)] * 2)
    o.step(steps)
    return grid, prm, o


def test_channel_flow_follows_the_1d_viscous_recurrence():
    grid, prm, o = _channel()
    ny, h, nu = grid.n[1], grid.h, 1.0 / prm.Re
    u = np.zeros(ny)
    for _ in range(40):
        up = np.concatenate([[-u[0]], u, [-u[-1]]])          # no-slip images
        u = u + prm.dt * (nu * (up[2:] - 2 * u + up[:-2]) / h ** 2 + 1.0)
    got = o.faces[0]
    assert np.max(np.abs(got - u[:, None])) <= 1e-13 * np.max(np.abs(u))
    assert np.max(np.abs(o.faces[1])) <= 1e-13
    assert np.max(np.abs(o.p)) <= 1e-10


def _drop_case(nx=64, ny=32, theta=70.0):
    grid = W.Grid((nx, ny), (0.0, 0.0), (2.0, 1.0))
    prm = W.Params(Cn=0.03, Pe=50.0, Re=20.0, Ca=0.2, theta_deg=theta, slip_length=0.02, dt=1e-4,
                   navier_stokes=True, rho1=0.1, rho2=1.0, mu1=0.2, mu2=1.0, body_force=(0.0, -0.5))
    shapes = [W.Shape(W.HALFPLANE, (0.0, 0.2, 0.0, 0.0, 1.0, 0.0))]
    T = build_tables(grid, shapes, prm)
    fa = face_fractions(grid, shapes, prm)
    C0, _ = W.droplet_field(grid, (1.0, 0.25), 0.3, prm.Cn, 1e-3, 7)
    rng = np.random.default_rng(11)
    faces = [0.2 * rng.standard_normal(grid.shape) for _ in range(2)]
    return grid, prm, T, fa, C0, faces


def test_projection_is_divergence_free():
    grid, prm, T, fa, C0, faces = _drop_case()
    o = OracleState(grid, prm, T, C0, faces, face_alpha=fa)
    for _ in range(4):
        o.step(1)
        div = ns.divergence(o.faces, grid)
        scale = max(np.max(np.abs(f)) for f in o.faces) / grid.h
        assert np.max(np.abs(div)) <= 1e-11 * scale, np.max(np.abs(div)) / scale
        assert abs(o.p.mean()) <= 1e-12 * np.max(np.abs(o.p))
    assert np.max(np.abs(o.p)) > 0.0


def test_laplace_pressure_of_a_drop():
    """The jump converges at second order in h/Cn; its Richardson limit from Cn/h = 1.28 and
    2.56 is the Laplace value."""
    from oracle.solver import chemical_potential
    R = 0.25
    jumps = []
    for n in (128, 256):
        grid = W.Grid((n, n), (0.0, 0.0), (1.0, 1.0))
        prm = W.Params(Cn=0.01, Pe=100.0, Re=2.0, Ca=0.5, navier_stokes=True)
        C, _ = W.droplet_field(grid, (0.5, 0.5), R, prm.Cn, 0.0, None)
        T = build_tables(grid, [], prm)
        phi = chemical_potential(C, grid, T, prm.Cn)
        f = ns.capillary_force(phi, C, grid, ns.capillary_coefficient(prm))
        p = ns.poisson_solve(ns.divergence(f, grid), grid)
        jumps.append(p[n // 2, n // 2] - p[2, 2])
    want = 1.0 / (prm.Re * prm.Ca * R)
    limit = (4.0 * jumps[1] - jumps[0]) / 3.0
    assert abs(jumps[1] / want - 1.0) < 0.02, (jumps, want)
    assert abs(limit / want - 1.0) < 0.003, (jumps, limit, want)


def test_staggered_fractions_of_a_flat_wall():
    grid = W.Grid((16, 32), (0.0, 0.0), (0.5, 1.0))
    h = grid.h
    yw = 19.25 * h
    shapes = [W.Shape(W.HALFPLANE, (0.0, yw, 0.0, 0.0, 1.0, 0.0))]
    prm = W.Params(Cn=0.05, Pe=10.0)
    fx, fy = face_fractions(grid, shapes, prm)
    cell = volume_fraction(grid, shapes, 100)[0]
    assert np.array_equal(fx, cell)
    col = np.zeros(32)
    col[19] = 1.0                     # the staggered cell [19.5h, 20.5h) is all fluid
    col[20:] = 1.0
    col[18] = 0.25                    # [18.5h, 19.5h) holds 0.25h of fluid
    assert np.allclose(fy, col[:, None], atol=0, rtol=0)
    assert np.allclose(cell[19], 0.75) and np.all(cell[20:] == 1.0) and np.all(cell[:19] == 0.0)
