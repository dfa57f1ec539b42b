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
