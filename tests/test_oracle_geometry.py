"""Pins of the oracle's geometry preprocessing (section 4.1) against closed forms. CPU only."""
import math

import numpy as np
import pytest

import workloads as W
from oracle.geometry import GeometryError, build_tables, volume_fraction


def _clip_area(x0, y0, h, px, py, nx, ny):
    """Exact area of the square [x0,x0+h]x[y0,y0+h] on the fluid side (x-p).n >= 0 of a line."""
    poly = [(x0, y0), (x0 + h, y0), (x0 + h, y0 + h), (x0, y0 + h)]
    f = lambda q: (q[0] - px) * nx + (q[1] - py) * ny
    out = []
    for k in range(4):
        a, b = poly[k], poly[(k + 1) % 4]
        fa, fb = f(a), f(b)
        if fa >= 0:
            out.append(a)
        if (fa >= 0) != (fb >= 0):
            t = fa / (fa - fb)
            out.append((a[0] + t * (b[0] - a[0]), a[1] + t * (b[1] - a[1])))
    if len(out) < 3:
        return 0.0
    s = 0.0
    for k in range(len(out)):
        s += out[k][0] * out[(k + 1) % len(out)][1] - out[(k + 1) % len(out)][0] * out[k][1]
    return abs(s) / 2


def test_flat_wall_tables_closed_form():
    c = W.config1()
    T = build_tables(c.grid, c.shapes, c.params)
    h = c.grid.h
    # wall at y = 0.1 = 6.4 h: rows 0..5 solid, row 6 has 60 of 100 subgrid rows fluid
    assert np.all(T.alpha[:6] == 0.0) and np.all(T.alpha[7:] == 1.0)
    assert np.all(T.alpha[6] == 0.6)
    assert T.n_ghost == 128
    assert np.all(T.gidx // 128 == 5)
    assert np.all(T.normal[0] == 0.0) and np.all(T.normal[1] == 1.0)
    assert np.allclose(T.dn, 0.1 - 5.5 * h, rtol=0, atol=1e-14)
    assert np.allclose(T.points["I"][1], 0.1, rtol=0, atol=1e-14)
    assert np.allclose(T.gamma, 2.0 * h / T.dn, rtol=1e-14)


def _check_colinear(T, grid):
    P = T.points
    n = T.normal
    for key in ("I", "M", "IP1", "IP2"):
        v = P[key] - P["G"]
        along = (v * n).sum(axis=0)
        perp = v - along * n
        assert np.max(np.abs(perp)) <= 1e-13
    assert np.allclose(np.sqrt(((P["M"] - P["I"]) ** 2).sum(0)), T.d1, rtol=0, atol=1e-13)
    assert np.allclose(np.sqrt(((P["IP1"] - P["M"]) ** 2).sum(0)), T.d2, rtol=0, atol=1e-13)
    assert np.allclose(np.sqrt(((P["IP2"] - P["IP1"]) ** 2).sum(0)), T.d2, rtol=0, atol=1e-13)


@pytest.mark.parametrize("kind", ["flat", "tilted", "sin", "circle"])
def test_points_colinear_and_averaging_points_fluid(kind):
    c = W.small_case(64, 32, kind=kind)
    T = build_tables(c.grid, c.shapes, c.params)
    assert T.n_ghost > 0
    _check_colinear(T, c.grid)
    cs = T.csolid.reshape(-1)
    assert not np.any(cs[T.ap[T.w > 0]])          # every weighted averaging point is fluid
    assert np.allclose(T.w.sum(axis=1), 1.0, rtol=0, atol=1e-14)
    assert np.all(T.dn > 0) and np.all(T.dn < 1.5 * c.grid.h)
    # every ghost is solid with a fluid face neighbour; every such cell is a ghost
    assert np.all(cs[T.gidx])


def test_tilted_half_plane_volume_fraction_and_normals():
    """alpha of a 15-degree wall within the subgrid resolution of the exact clipped area.

    The normal from the 3x3 corner-gradient stencil of alpha is exact only for
    axis-aligned walls; for an oblique straight wall it deviates by a few degrees
    (alpha is a nonlinear function of the distance to the wall), so the bound is
    0.08 per component (about 4.5 degrees)."""
    c = W.small_case(64, 32, kind="tilted")
    g = c.grid
    h = g.h
    p = c.shapes[0].p
    alpha, _ = volume_fraction(g, c.shapes, 100)
    worst = 0.0
    for j in range(g.n[1]):
        for i in range(g.n[0]):
            ex = _clip_area(i * h, j * h, h, p[0], p[1], p[3], p[4]) / (h * h)
            worst = max(worst, abs(alpha[j, i] - ex))
    assert worst <= 0.02
    T = build_tables(g, c.shapes, c.params)
    nn = np.array([p[3], p[4]]) / math.hypot(p[3], p[4])
    x = T.points["G"][0]
    away = (x > 0.3) & (x < 1.7)          # the half-plane is not periodic: skip the seam at x = 0
    err = np.abs(T.normal[:, away] - nn[:, None]).max()
    assert err <= 0.08


def test_sphere_normals_are_radial():
    c = W.small_case_3d(32)
    T = build_tables(c.grid, c.shapes, c.params)
    G = T.points["G"]
    radial = G / np.sqrt((G * G).sum(0))
    cosang = (T.normal * radial).sum(0)
    assert np.degrees(np.arccos(np.clip(cosang.min(), -1, 1))) < 6.0
    _check_colinear(T, c.grid)
    assert T.ap.shape[1] == 7


def test_on_centre_interpolation_point_gets_one_hot_weight():
    """Wall on a cell face, d1 = 1.5h, d2 = h: IP1 and IP2 fall on cell centres."""
    g = W.Grid((32, 16), (0.0, 0.0), (2.0, 1.0))
    h = g.h
    prm = W.Params(Cn=0.05, Pe=10.0, d1_cells=1.5, d2_cells=1.0)
    T = build_tables(g, [W.Shape(W.HALFPLANE, (0.0, 4 * h, 0.0, 0.0, 1.0, 0.0))], prm)
    assert np.allclose(T.dn, 0.5 * h)
    assert np.all(T.w[:, 0, :] == 1.0)
    assert np.all(T.ap[0, 0] == T.gidx + 3 * 32) and np.all(T.ap[1, 0] == T.gidx + 4 * 32)


def test_ghost_touching_box_wall_is_rejected():
    g = W.Grid((16, 8), (0.0, 0.0), (1.0, 0.5))
    prm = W.Params(Cn=0.05, Pe=10.0)
    with pytest.raises(GeometryError):
        build_tables(g, [W.Shape(W.HALFPLANE, (0.0, 0.05, 0.0, 0.0, 1.0, 0.0))], prm)
