"""Pins of the contact-angle measurement (host analysis) with synthetic interfaces of known angle.

CPU only: straight interfaces meeting a flat or a sinusoidal wall at a prescribed angle (the
measurement is exact for them up to the sampling of C on cells) and circular caps on a flat
wall (exact contact angle known in closed form)."""
import math

import numpy as np
import pytest

from paper_2104_00350_amd import angle as A

SQ2 = math.sqrt(2.0)


def _grid(nx=512, ny=256, L=4.0, H=2.0):
    h = L / nx
    x = (np.arange(nx) + 0.5) * h
    y = (np.arange(ny) + 0.5) * h
    return np.meshgrid(x, y), (0.0, 0.0), (L, H)


def _wedge_droplet(X, Y, pL, tL, pR, tR, theta, Cn):
    """C > 0 between two straight interfaces leaving the wall at pL, pR (tangents tL, tR point
    into the droplet along the wall), each at angle theta to its tangent."""
    def line_dist(p, t, sign):
        c, s = math.cos(theta), math.sin(theta)
        # rotate the wall tangent by theta towards the fluid side (left turn for the left line,
        # right turn for the right one, so both rotate away from the wall)
        u = (t[0] * c - sign * t[1] * s, sign * t[0] * s + t[1] * c)
        return sign * ((X - p[0]) * u[1] - (Y - p[1]) * u[0])
    sL = line_dist(pL, tL, 1.0)
    sR = line_dist(pR, tR, -1.0)
    return np.tanh(np.minimum(sL, sR) / (SQ2 * Cn))


@pytest.mark.parametrize("theta", [40.0, 90.0, 140.0])
def test_straight_interfaces_on_a_flat_wall(theta):
    (X, Y), lo, hi = _grid()
    yw, Cn = 0.3, 0.01
    th = math.radians(theta)
    C = _wedge_droplet(X, Y, (1.6, yw), (1.0, 0.0), (2.6, yw), (-1.0, 0.0), th, Cn)
    r = A.measure(C, lo, hi, A.HALFPLANE, (0.0, yw, 0.0, 0.0, 1.0, 0.0), Cn)
    assert abs(r["left"] - theta) < 0.05 and abs(r["right"] - theta) < 0.05, r
    assert abs(r["left_x"] - 1.6) < 1e-3 and abs(r["right_x"] - 2.6) < 1e-3


@pytest.mark.parametrize("theta", [50.0, 100.0, 135.0])
def test_straight_interfaces_on_a_sinusoidal_wall(theta):
    (X, Y), lo, hi = _grid()
    p = (0.3, 0.1, 0.5, 0.0)
    k = 2 * math.pi / p[2]
    yw = lambda s: p[0] + p[1] * math.sin(k * s)
    dyw = lambda s: p[1] * k * math.cos(k * s)
    Cn = 0.01
    th = math.radians(theta)
    xL, xR = 1.93, 2.31
    tL = np.array([1.0, dyw(xL)]); tL /= np.linalg.norm(tL)
    tR = -np.array([1.0, dyw(xR)]); tR /= np.linalg.norm(tR)
    C = _wedge_droplet(X, Y, (xL, yw(xL)), tL, (xR, yw(xR)), tR, th, Cn)
    C = np.where(Y > p[0] + p[1] * np.sin(k * X), C, -1.0)        # solid side: outside the droplet
    r = A.measure(C, lo, hi, A.SINUSOID, p, Cn)
    # the crossings carry the bilinear-interpolation error of C sampled at Cn/h = 1.28, which the
    # quadratic extrapolation to the wall amplifies to about 0.2 degree at most
    assert abs(r["left"] - theta) < 0.25 and abs(r["right"] - theta) < 0.25, r


@pytest.mark.parametrize("theta", [45.0, 90.0, 120.0])
def test_circular_cap_on_a_flat_wall(theta):
    (X, Y), lo, hi = _grid()
    yw, Cn, R = 0.3, 0.01, 0.5
    yc = yw - R * math.cos(math.radians(theta))
    C = np.tanh((R - np.hypot(X - 2.0, Y - yc)) / (SQ2 * Cn))
    r = A.measure(C, lo, hi, A.HALFPLANE, (0.0, yw, 0.0, 0.0, 1.0, 0.0), Cn)
    assert abs(r["mean"] - theta) < 0.3, r
    assert abs(r["left"] - r["right"]) < 0.02


def test_coarser_sampling_of_the_same_interface_agrees():
    """The same physical droplet sampled at h and 2h measures within 0.1 degree."""
    out = []
    for nx in (512, 1024):
        (X, Y), lo, hi = _grid(nx, nx // 2)
        yw, Cn, R = 0.3, 0.01, 0.5
        yc = yw - R * math.cos(math.radians(70.0))
        C = np.tanh((R - np.hypot(X - 2.0, Y - yc)) / (SQ2 * Cn))
        out.append(A.measure(C, lo, hi, A.HALFPLANE, (0.0, yw, 0.0, 0.0, 1.0, 0.0), Cn)["mean"])
    assert abs(out[0] - out[1]) < 0.1, out


# ---- circular-cap (equilibrium) measurement ---------------------------------------------------

def _tangent_angle(c, R, P, t_wall_into_drop):
    """Angle (degrees) through the droplet between the wall tangent pointing into the droplet and
    the circle's tangent at P pointing away from the wall (both as unit vectors)."""
    rad = (P - c) / R
    tc = np.array([-rad[1], rad[0]])                     # one of the two circle tangents
    # the interface tangent leaving the wall points to the fluid side of the wall
    n_up = np.array([-t_wall_into_drop[1], t_wall_into_drop[0]])
    if n_up[1] < 0:
        n_up = -n_up
    if tc @ n_up < 0:
        tc = -tc
    return math.degrees(math.acos(np.clip(tc @ t_wall_into_drop, -1.0, 1.0)))


def _circle_wall_hits(c, R, yw):
    """Brute force: the two circle points where y - yw(x) changes sign nearest the circle's lowest
    point on each side, refined by bisection in the polar angle."""
    psi = np.linspace(-math.pi / 2, 3 * math.pi / 2, 400001)
    f = c[1] + R * np.sin(psi) - yw(c[0] + R * np.cos(psi))
    top = np.argmax(f)
    hits = []
    for rng in (range(top, len(psi) - 1), range(top, 0, -1)):
        for i in rng:
            j = i + 1 if rng.step == 1 else i - 1
            if (f[i] > 0) != (f[j] > 0):
                a, b = psi[i], psi[j]
                for _ in range(80):
                    m = 0.5 * (a + b)
                    if (c[1] + R * math.sin(m) - yw(c[0] + R * math.cos(m)) > 0) == (f[i] > 0):
                        a = m
                    else:
                        b = m
                hits.append(np.array([c[0] + R * math.cos(a), c[1] + R * math.sin(a)]))
                break
    return hits          # [left, right]


@pytest.mark.parametrize("theta", [30.0, 60.0, 90.0, 120.0, 150.0])
def test_cap_fit_on_a_flat_wall(theta):
    """Closed form: a cap of radius R whose centre sits R cos(theta) below the wall meets it at theta."""
    (X, Y), lo, hi = _grid()
    yw, Cn, R = 0.3, 0.01, 0.5
    yc = yw - R * math.cos(math.radians(theta))
    C = np.tanh((R - np.hypot(X - 2.0, Y - yc)) / (SQ2 * Cn))
    C = np.where(Y > yw, C, -1.0)
    r = A.measure_cap(C, lo, hi, A.HALFPLANE, (0.0, yw, 0.0, 0.0, 1.0, 0.0), Cn)
    # bilinear sampling of C at Cn/h = 1.28 leaves ~0.005 h rms on the crossings; extrapolating a
    # short arc (theta = 30) to the wall turns that into a few hundredths of a degree
    assert abs(r["left"] - theta) < 0.05 and abs(r["right"] - theta) < 0.05, r
    half = R * math.sin(math.radians(theta))
    assert abs(r["left_x"] - (2.0 - half)) < 1e-3 and abs(r["right_x"] - (2.0 + half)) < 1e-3, r


@pytest.mark.parametrize("cy,R", [(0.35, 0.45), (0.55, 0.4), (0.62, 0.36)])
def test_cap_fit_on_a_sinusoidal_wall(cy, R):
    """A circle cut by the sinusoid: the contact points and angles come from a brute-force
    intersection and the tangent vectors, independent of the routine's formula."""
    (X, Y), lo, hi = _grid()
    p = (0.3, 0.1, 0.5, 0.0)
    k = 2 * math.pi / p[2]
    yw = lambda s: p[0] + p[1] * np.sin(k * s)
    dyw = lambda s: p[1] * k * np.cos(k * s)
    Cn = 0.01
    c = np.array([2.07, cy])
    C = np.tanh((R - np.hypot(X - c[0], Y - c[1])) / (SQ2 * Cn))
    C = np.where(Y > yw(X), C, -1.0)
    r = A.measure_cap(C, lo, hi, A.SINUSOID, p, Cn)
    PL, PR = _circle_wall_hits(c, R, yw)
    tL = np.array([1.0, dyw(PL[0])]); tL /= np.linalg.norm(tL)
    tR = -np.array([1.0, dyw(PR[0])]); tR /= np.linalg.norm(tR)
    want_L, want_R = _tangent_angle(c, R, PL, tL), _tangent_angle(c, R, PR, tR)
    assert abs(r["left_x"] - PL[0]) < 2e-3 and abs(r["right_x"] - PR[0]) < 2e-3, (r, PL, PR)
    assert abs(r["left"] - want_L) < 0.05 and abs(r["right"] - want_R) < 0.05, (r, want_L, want_R)


def test_cap_fit_ignores_a_film_beside_the_droplet():
    """A liquid film 0.06 thick along the wall, joined to the droplet beyond its right contact line,
    puts crossings on the film surface; they are trimmed from the fit."""
    (X, Y), lo, hi = _grid()
    p = (0.3, 0.1, 0.5, 0.0)
    k = 2 * math.pi / p[2]
    ywX = p[0] + p[1] * np.sin(k * X)
    Cn, R = 0.01, 0.45
    c = np.array([2.07, 0.55])
    drop = (R - np.hypot(X - c[0], Y - c[1])) / (SQ2 * Cn)
    ref = np.where(Y > ywX, np.tanh(drop), -1.0)
    b = A.measure_cap(ref, lo, hi, A.SINUSOID, p, Cn)
    film = np.where((X > b["right_x"] - 0.05) & (X < b["right_x"] + 0.35), (0.06 - (Y - ywX)) / (SQ2 * Cn), -10.0)
    C = np.where(Y > ywX, np.tanh(np.maximum(drop, film)), -1.0)
    a = A.measure_cap(C, lo, hi, A.SINUSOID, p, Cn)
    assert a["points"] < b["points"] - 10, (a, b)
    assert abs(a["left"] - b["left"]) < 0.05 and abs(a["right"] - b["right"]) < 0.05, (a, b)


def test_cap_fit_coarser_sampling_agrees():
    out = []
    for nx in (512, 1024):
        (X, Y), lo, hi = _grid(nx, nx // 2)
        yw, Cn, R = 0.3, 0.01, 0.5
        yc = yw - R * math.cos(math.radians(70.0))
        C = np.where(Y > yw, np.tanh((R - np.hypot(X - 2.0, Y - yc)) / (SQ2 * Cn)), -1.0)
        out.append(A.measure_cap(C, lo, hi, A.HALFPLANE, (0.0, yw, 0.0, 0.0, 1.0, 0.0), Cn)["mean"])
    assert abs(out[0] - out[1]) < 0.02, out
