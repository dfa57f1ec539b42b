"""Pins of the oracle's explicit Adams-Bashforth step (Eq. ExpCH), CPU only.

- A small Fourier mode with the fluid at rest follows the scalar AB2 recurrence of its linearised
  rate exactly (the cubic term is ~1e-18 relative at amplitude 1e-9).
- Without immersed walls the update is a sum of discrete divergences: the mass of the box is
  conserved to round-off, with advection on.
- Without immersed walls the explicit and the semi-implicit schemes discretise the same equation:
  their difference shrinks at the semi-implicit stabilisation's first order as dt falls.  (Near an
  immersed wall they converge too, more slowly: tests/test_oracle_wall.py.)
- The chemical potential is C^3 - C in the interior of a linear field; ghosts carry the mirror value.
"""
import dataclasses
import math

import numpy as np
import pytest

import workloads as W
from oracle.geometry import build_tables
from oracle.solver import OracleState, chemical_potential, mirror_value


def _box(nx=64, ny=16, L=2.0):
    g = W.Grid((nx, ny), (0.0, 0.0), (L, L * ny / nx))
    return g


@pytest.mark.parametrize("m", [1, 5, 17])
def test_fourier_mode_follows_the_ab2_recurrence(m):
    g = _box()
    prm = W.Params(Cn=0.02, Pe=100.0, dt=2e-5, explicit=True)
    T = build_tables(g, [], prm)
    x = (np.arange(g.n[0]) + 0.5) * g.h
    C0 = 1e-9 * np.cos(2 * math.pi * m * x / 2.0)[None, :] * np.ones((g.n[1], 1))
    o = OracleState(g, prm, T, C0)
    N = 300
    o.step(N)
    lam = -(4.0 / g.h ** 2) * math.sin(math.pi * m / g.n[0]) ** 2   # the discrete Laplacian's eigenvalue
    rate = (1.0 / prm.Pe) * lam * (-1.0 - prm.Cn ** 2 * lam)         # lap(-C - Cn^2 lap C) / Pe
    a0, a1 = 1.0, 1.0 + prm.dt * rate                                 # forward Euler start
    for _ in range(N - 1):
        a0, a1 = a1, a1 + prm.dt * rate * (1.5 * a1 - 0.5 * a0)
    assert np.max(np.abs(o.C - a1 * C0)) <= 1e-13 * np.max(np.abs(C0))


def test_mass_is_conserved_without_immersed_walls():
    g = _box()
    rng = np.random.default_rng(3)
    C0 = 0.5 * np.tanh(rng.standard_normal(g.shape))
    faces = [0.3 * rng.standard_normal(g.shape) for _ in range(2)]
    prm = W.Params(Cn=0.02, Pe=100.0, dt=1e-5, explicit=True)
    o = OracleState(g, prm, build_tables(g, [], prm), C0, faces)
    m0 = o.C.sum()
    o.step(200)
    assert np.max(np.abs(o.C - C0)) > 0.05                  # the field did move
    assert abs(o.C.sum() - m0) <= 1e-13 * abs(m0)


def test_converges_to_the_semi_implicit_scheme_without_immersed_walls():
    g = W.Grid((64, 32), (0.0, 0.0), (2.0, 1.0))
    x = (np.arange(64) + 0.5) * g.h
    y = (np.arange(32) + 0.5) * g.h
    X, Y = np.meshgrid(x, y)
    C0 = np.tanh((0.3 - np.hypot(X - 1.0, Y - 0.4)) / (math.sqrt(2) * 0.03))
    rng = np.random.default_rng(5)
    faces = [0.5 * rng.standard_normal(g.shape) for _ in range(2)]
    base = W.Params(Cn=0.03, Pe=100.0, dt=1e-5)
    T = build_tables(g, [], base)
    diff = []
    for dt in (4e-6, 1e-6):
        out = []
        for ex in (False, True):
            o = OracleState(g, dataclasses.replace(base, dt=dt, explicit=ex), T, C0, faces)
            o.step(int(round(4e-4 / dt)))
            out.append(o.C)
        diff.append(np.max(np.abs(out[0] - out[1])))
    assert np.max(np.abs(out[1] - C0)) > 0.04
    assert diff[1] <= 1e-4 and diff[0] / diff[1] >= 3.0, diff


def test_chemical_potential_interior_and_ghosts():
    case = W.small_case(64, 32, kind="sin", theta_deg=60.0)
    g = case.grid
    T = build_tables(g, case.shapes, case.params)
    y = (np.arange(g.n[1]) + 0.5) * g.h
    C = (0.3 * y - 0.1)[:, None] * np.ones((1, g.n[0]))   # linear in y: zero discrete Laplacian inside
    phi = chemical_potential(C, g, T, case.params.Cn)
    ghost = np.zeros(g.cells, dtype=bool)
    ghost[T.gidx] = True
    inner = ~ghost.reshape(g.shape)
    inner[0] = inner[-1] = False                           # box-wall rows reflect
    assert np.max(np.abs((phi - (C ** 3 - C))[inner])) <= 1e-13
    ref = C ** 3 - C
    assert np.max(np.abs(phi.reshape(-1)[T.gidx] - mirror_value(ref.reshape(-1), T))) <= 1e-13
