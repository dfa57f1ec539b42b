"""Pins of the oracle at the immersed wall, CPU only.

- The wall condition dphi/dn = 0 (Eq. WallBCS; end of section 4.2.2) in the semi-implicit step:
  near flat and sinusoidal walls the semi-implicit and the explicit schemes converge to each other
  as dt falls (section 3 finds their differences negligible), and the droplet keeps its volume
  (section 5 reports less than 0.3 % change).  The convergence order follows from the step's
  structure: with the ghost condition on the explicit chemical potential, what is left is the
  stabilisation S (C^(n+1) - C~) at the ghosts, where C^(n+1) - C~ is O(dt) and S grows as
  dt^(-1/2), so the gap closes as dt^(1/2): at least a factor 1.8 for dt / 4 (2 with 10 % slack).
- The static fill when the mirror value leaves [-1, 1]: the wall value is the pure phase.
- The dynamic fill's wall-advection term u_I . grad_t C_I and the capillary bracket Kc of
  Eq. UpdateVtan, on linear fields where both are known in closed form.
- The central difference at the box walls reflects the field as the Laplacian does.
- Young's relation: a flat-wall droplet with the momentum step on relaxes to the cap of theta
  (2 degrees at Cn/h = 1.28, fixed before the runs); 90 degrees misses it on this grid (see there).
"""
import dataclasses
import math

import numpy as np
import pytest

import workloads as W
from oracle.geometry import build_tables
from oracle.solver import OracleState, gradient_at, mirror_value

SQ2 = math.sqrt(2.0)


def _near_wall_fluid(grid, T):
    """Fluid cells (alpha > 0) with a ghost face neighbour: the first fluid row."""
    ghost = np.zeros(grid.cells, bool)
    ghost[T.gidx] = True
    gm = ghost.reshape(grid.shape)
    nb = np.zeros_like(gm)
    nb[1:] |= gm[:-1]
    nb[:-1] |= gm[1:]
    nb |= np.roll(gm, 1, 1) | np.roll(gm, -1, 1)
    return nb & (T.alpha.reshape(grid.shape) > 0) & ~gm


@pytest.mark.parametrize("kind,bound", [("flat", 5e-4), ("sin", 2e-3)])
def test_semi_implicit_converges_to_explicit_near_immersed_walls(kind, bound):
    case = W.small_case(64, 32, theta_deg=60.0, kind=kind)
    T = build_tables(case.grid, case.shapes, case.params)
    C0, faces = case.initial_fields()
    row = _near_wall_fluid(case.grid, T)
    gaps = []
    for dt in (4e-6, 1e-6):
        out = []
        for ex in (False, True):
            o = OracleState(case.grid, dataclasses.replace(case.params, dt=dt, explicit=ex), T, C0, faces)
            o.step(int(round(4e-4 / dt)))
            out.append(o.C)
        gaps.append(np.max(np.abs(out[0] - out[1])[row]))
    assert np.max(np.abs(out[1] - C0)[row]) > 0.01           # the near-wall field did move
    assert gaps[1] <= bound and gaps[0] / gaps[1] >= 1.8, gaps


def _droplet_volume(C, alpha):
    return float(np.sum(alpha * (1.0 + C) * 0.5))


@pytest.mark.parametrize("theta", [60.0, 120.0])
def test_droplet_keeps_its_volume_and_energy_decays(theta):
    """The flat-wall droplet of the 128 x 64 workload over 2000 steps: droplet volume within
    0.3 % (section 5), free energy non-increasing."""
    case = W.config1()
    prm = dataclasses.replace(case.params, theta_deg=theta)
    T = build_tables(case.grid, case.shapes, prm)
    C0, faces = case.initial_fields()
    o = OracleState(case.grid, prm, T, C0, faces)
    al = T.alpha.reshape(case.grid.shape)
    v0 = _droplet_volume(o.C, al)
    F = [o.diagnostics()["free_energy"]]
    for _ in range(5):
        o.step(400)
        F.append(o.diagnostics()["free_energy"])
        assert abs(_droplet_volume(o.C, al) / v0 - 1.0) <= 3e-3
    assert all(b <= a for a, b in zip(F, F[1:])), F


@pytest.mark.parametrize("theta", [60.0, 120.0])
def test_low_peclet_droplet_does_not_drain_through_the_wall(theta):
    """At Pe = 10 the chemical potential of the solid's interior, left unconditioned, would drive
    C through the ghost layer (tens of percent of the droplet in 4000 steps).  With dphi/dn = 0 at
    the ghosts the droplet keeps its volume to 2 %."""
    case = W.small_case(64, 32, theta_deg=theta, kind="flat")
    prm = dataclasses.replace(case.params, Pe=10.0)
    T = build_tables(case.grid, case.shapes, prm)
    C0, faces = case.initial_fields()
    o = OracleState(case.grid, prm, T, C0, faces)
    al = T.alpha.reshape(case.grid.shape)
    v0 = _droplet_volume(o.C, al)
    o.step(4000)
    assert abs(_droplet_volume(o.C, al) / v0 - 1.0) <= 2e-2


@pytest.mark.parametrize("value", [1.2, -1.3])
@pytest.mark.parametrize("theta", [30.0, 120.0])
def test_static_fill_beyond_the_pure_phases_sets_the_wall_to_the_pure_phase(value, theta):
    """The exact integration artanh C_I = artanh C_M + b is taken with C_M clipped to [-1, 1]; a
    pure phase is a fixed point of the wall relation (dC/dn = 0 at C = +-1), so a mirror value
    past +-1 makes C_I the pure phase exactly and the ghost carries the overshoot:
    C_G = ((gamma + 1) sign(C_M) - C_M)/gamma."""
    case = W.small_case(64, 32, kind="sin", theta_deg=theta)
    T = build_tables(case.grid, case.shapes, case.params)
    st = OracleState(case.grid, case.params, T, np.zeros(case.grid.shape))
    CG = st.fill_C(np.full(case.grid.shape, value), initial=False)
    g = T.gamma
    s = math.copysign(1.0, value)
    assert np.max(np.abs(CG - ((g + 1.0) * s - value) / g)) <= 1e-14
    assert np.max(np.abs((g * CG + value) / (g + 1.0) - s)) <= 1e-14


def _on_centre_case(**kw):
    """Flat wall on a cell face (y = 4h) with d1 = 1.5h, d2 = 1h: M, IP1 and IP2 fall on cell
    centres, so the mirror value of a linear field is exact and the wall value, the normal and
    tangential derivatives at I are those of the field."""
    g = W.Grid((32, 16), (0.0, 0.0), (2.0, 1.0))
    h = g.h
    prm = W.Params(Cn=0.05, Pe=10.0, d1_cells=1.5, d2_cells=1.0, **kw)
    shapes = [W.Shape(W.HALFPLANE, (0.0, 4 * h, 0.0, 0.0, 1.0, 0.0))]
    T = build_tables(g, shapes, prm)
    x = (np.arange(32) + 0.5) * h
    y = (np.arange(16) + 0.5) * h
    return g, prm, T, x, y


def _linear(x, y, c0=0.1, gx=0.3, gy=0.2):
    return c0 + gx * (x - 1.0) + gy * (y - 0.25)


def _interior(T, lo=0.6, hi=1.4):
    """Ghosts whose stencils stay clear of the periodic wrap (a linear field is not periodic)."""
    Gx = T.points["G"][0]
    return (Gx > lo) & (Gx < hi)


def test_dynamic_fill_rate_on_a_linear_field_under_uniform_flow():
    """C = c0 + gx (x - 1) + gy (y - yw): at I the wall value, dC/dn = gy and grad_t C = (gx, 0)
    are exact, and a uniform flow (U, 0) gives u_I . grad_t C_I = U gx, so one dynamic update is
    C_I <- C_I + dt [-U gx + Vs (Cn gy + cos(theta)(1 - C(I)^2)/sqrt2)] (Eq. WallBCS_recast)."""
    Vs, th, U = 40.0, 70.0, 0.8
    g, prm, T, x, y = _on_centre_case(theta_deg=th, Vs=Vs, dt=1e-4)
    C = _linear(x[None, :], y[:, None])
    faces = [np.full(g.shape, U), np.zeros(g.shape)]
    st = OracleState(g, prm, T, C, faces)
    st.faces = faces            # the initial velocity fill changed the faces next to the ghosts
    CI0 = st.CI.copy()
    st.fill_C(C.copy(), initial=False)
    Ix, Iy = T.points["I"]
    CIx = _linear(Ix, Iy)
    rate = -U * 0.3 + Vs * (prm.Cn * 0.2 + math.cos(math.radians(th)) * (1.0 - CIx ** 2) / SQ2)
    m = _interior(T)
    assert m.sum() >= 8
    assert np.max(np.abs((st.CI - (CI0 + prm.dt * rate))[m])) <= 1e-13


def test_dynamic_fill_wall_advection_on_a_tilted_wall():
    """On any wall a linear field has grad C = g at G and at M (the weights sum to one) and a
    uniform flow u has u_I = u, so the advection term of the dynamic update is exactly
    u . (g - (g . n) n): two flows differ by dt (u1 - u2) . (g - (g . n) n) in C_I."""
    case = W.small_case(64, 32, kind="tilted", theta_deg=70.0, Vs=40.0)
    grid = case.grid
    T = build_tables(grid, case.shapes, case.params)
    xs = W.cell_centres(grid)
    gvec = np.array([0.3, -0.2])
    C = 0.1 + gvec[0] * (xs[0] - 1.0) + gvec[1] * (xs[1] - 0.5) + 0.0 * xs[0] * xs[1]
    C = np.ascontiguousarray(np.broadcast_to(C, grid.shape))
    out = []
    for u in ((0.7, -0.4), (-0.2, 0.5)):
        faces = [np.full(grid.shape, u[0]), np.full(grid.shape, u[1])]
        st = OracleState(grid, case.params, T, C, faces)
        st.faces = faces
        st.CI[:] = 0.0
        st.fill_C(C.copy(), initial=False)
        out.append(st.CI.copy())
    n = T.normal
    gt = gvec[:, None] - (gvec @ n)[None, :] * n
    du = np.array([0.7 - (-0.2), -0.4 - 0.5])
    expect = -case.params.dt * (du @ gt)
    m = _interior(T, 0.5, 1.5) & (T.points["G"][1] < 0.8)
    assert m.sum() >= 8
    assert np.max(np.abs((out[0] - out[1] - expect)[m])) <= 1e-14


@pytest.mark.parametrize("ls", [1e12, 0.01])
def test_capillary_bracket_on_a_linear_field(ls):
    """Kc = [(3/(2 sqrt2)) Cn dC/dn + cos(theta) g'(C_I)]/Ca, g'(C) = 3(1 - C^2)/4 (Eq. UpdateVtan)
    with the fluid at rest: V_tG = -Kc grad_t C_I ls (gamma + 1) dn / (mu (ls + gamma dn)), which
    for ls -> infinity is the balance (V_tM - V_tG)/((1 + gamma) dn) = Kc grad_t C_I / mu."""
    th, Ca, mu = 65.0, 0.05, 2.0
    g, prm, T, x, y = _on_centre_case(theta_deg=th, Vs=30.0, Ca=Ca, mu=mu, slip_length=ls)
    C = _linear(x[None, :], y[:, None])
    st = OracleState(g, prm, T, C, [np.zeros(g.shape), np.zeros(g.shape)])
    st.faces = [np.zeros(g.shape), np.zeros(g.shape)]
    st.fill_velocity(C)
    Ix, Iy = T.points["I"]
    CIx = _linear(Ix, Iy)
    Kc = ((3.0 / (2.0 * SQ2)) * prm.Cn * 0.2 + 0.75 * math.cos(math.radians(th)) * (1.0 - CIx ** 2)) / Ca
    gam, dn = T.gamma, T.dn
    VtG = -Kc * 0.3 * ls * (gam + 1.0) * dn / (mu * (ls + gam * dn))
    m = _interior(T)
    assert m.sum() >= 8
    assert np.max(np.abs((st.last_uG[0] - VtG)[m])) <= 1e-12 * (1.0 + np.max(np.abs(VtG)))
    assert np.max(np.abs(st.last_uG[1][m])) <= 1e-14               # no normal velocity
    if ls > 1.0:
        assert np.max(np.abs((-st.last_uG[0] / ((1.0 + gam) * dn) - Kc * 0.3 / mu)[m])) <= 1e-9


def test_gradient_reflects_at_the_box_walls():
    """At the first and last cell of the bounded axis the neighbour outside the box is the cell
    itself (f_-1 = f_0), the reflection the Laplacian uses: dC/dy = (f_1 - f_0)/(2h) there."""
    g = W.Grid((8, 6), (0.0, 0.0), (1.0, 0.75))
    f = np.arange(48, dtype=np.float64).reshape(6, 8) ** 1.5
    ff = f.reshape(-1)
    lin = np.array([3, 8 * 5 + 2, 8 * 2 + 7])
    gr = gradient_at(ff, g, lin)
    h = g.h
    assert gr[1][0] == (f[1, 3] - f[0, 3]) / (2 * h)
    assert gr[1][1] == (f[5, 2] - f[4, 2]) / (2 * h)
    assert gr[1][2] == (f[3, 7] - f[1, 7]) / (2 * h)
    assert gr[0][2] == (f[2, 0] - f[2, 6]) / (2 * h)              # periodic wrap along x


def _relaxed_cap(theta, steps=3000, yw=0.1):
    """Flat-wall droplet with the momentum step on (128 x 64, Cn/h = 1.28, matched fluids), released
    as a half disc (apparent angle 90 degrees) and relaxed; returns the cap-fit angle."""
    from oracle.geometry import face_fractions
    from paper_2104_00350_amd import angle
    grid = W.Grid((128, 64), (0.0, 0.0), (2.0, 1.0))
    prm = W.Params(Cn=0.02, Pe=100.0, Re=10.0, Ca=0.05, theta_deg=theta, slip_length=0.05, dt=2e-4,
                   navier_stokes=True)
    shapes = [W.Shape(W.HALFPLANE, (0.0, yw, 0.0, 0.0, 1.0, 0.0))]
    T = build_tables(grid, shapes, prm)
    C0, faces = W.droplet_field(grid, (1.0, yw), 0.3, prm.Cn, 0.0, None)
    o = OracleState(grid, prm, T, C0, faces, face_alpha=face_fractions(grid, shapes, prm))
    o.step(steps)
    m = angle.measure_cap(o.C, grid.lo, grid.hi, W.HALFPLANE, shapes[0].p, prm.Cn)
    return m["mean"]


@pytest.mark.parametrize("theta", [
    60.0,
    pytest.param(90.0, marks=pytest.mark.xfail(strict=True, reason=(
        "measured 87.1 degrees: at h = 1/64 the relaxed angle depends on where the wall cuts the "
        "cells (88.9, 87.1, 90.0, 92.4 degrees for the wall at 6.0, 6.4, 6.5, 6.75 cells; 88.6 and 91.6 "
        "with the fluid at rest at Pe = 2), and the error shrinks with h (91.0 degrees at h = 1/128)"))),
    120.0])
def test_flat_wall_droplet_relaxes_to_the_cap_of_theta(theta):
    """Young's relation (section 2) makes a droplet on a flat wall relax to a circular cap that meets
    the wall at the prescribed angle.  Tolerance fixed before the runs: 2 degrees at Cn/h = 1.28."""
    assert abs(_relaxed_cap(theta) - theta) <= 2.0
