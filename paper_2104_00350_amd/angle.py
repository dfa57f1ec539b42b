"""Contact-angle measurement of a 2D droplet on a flat or sinusoidal wall (host analysis).

The same routine scores plain coarse, plain fine and corrected coarse runs, so every run is
measured the same way:

* the wall is the analytic curve of the case's shape (half-plane with normal (0, 1), or
  y_w(x) = mean + amp sin(2 pi x / wavelength + phase)); a wall point at abscissa s is
  W(s) = (s, y_w(s)) with unit normal n(s) into the fluid;
* for a set of distances d_j from the wall (a window a few interface widths away from it,
  the same physical window on every grid), the droplet's own C = 0 crossing on the curve
  s -> W(s) + d_j n(s) is found by walking outward from the droplet's centre of mass (so
  films or satellite drops farther out are ignored) and bisecting the sign change of the
  bilinearly interpolated C;
* on each side the crossing points are fitted by a quadratic curve in their own principal
  frame; its intersection with the wall is the contact point, and the angle between the
  curve's tangent there and the wall tangent pointing into the droplet is the contact angle
  (measured through the C > 0 phase, so cos(theta) > 0 means the C > 0 phase wets).

Returns the two angles in degrees and their mean.
"""
from __future__ import annotations

import math
from typing import Dict, Sequence

import numpy as np

HALFPLANE = 1
SINUSOID = 2


class AngleError(RuntimeError):
    pass


def _wall(shape_kind: int, p: Sequence[float]):
    if shape_kind == SINUSOID:
        mean, amp, lam, ph = p[0], p[1], p[2], p[3]
        k = 2.0 * math.pi / lam

        def y(s):
            return mean + amp * np.sin(k * s + ph)

        def dy(s):
            return amp * k * np.cos(k * s + ph)
        return y, dy
    if shape_kind == HALFPLANE:
        if abs(p[3]) > 1e-12 or abs(p[4] - 1.0) > 1e-12:
            raise AngleError("only half-planes with normal (0, 1) are supported")
        y0 = p[1]
        return (lambda s: y0 + 0.0 * np.asarray(s)), (lambda s: 0.0 * np.asarray(s))
    raise AngleError(f"unsupported wall kind {shape_kind}")


def _bilinear(C: np.ndarray, lo, h, x, y):
    """C (ny, nx) at points (x, y); periodic in x, clamped in y."""
    ny, nx = C.shape
    fx = (np.asarray(x) - lo[0]) / h - 0.5
    fy = (np.asarray(y) - lo[1]) / h - 0.5
    fy = np.clip(fy, 0.0, ny - 1.000001)
    i0 = np.floor(fx).astype(np.int64)
    j0 = np.floor(fy).astype(np.int64)
    tx = fx - i0
    ty = fy - j0
    i0m = np.mod(i0, nx)
    i1m = np.mod(i0 + 1, nx)
    j1 = np.minimum(j0 + 1, ny - 1)
    return ((1 - tx) * (1 - ty) * C[j0, i0m] + tx * (1 - ty) * C[j0, i1m]
            + (1 - tx) * ty * C[j1, i0m] + tx * ty * C[j1, i1m])


def measure(C: np.ndarray, lo: Sequence[float], hi: Sequence[float], shape_kind: int,
            shape_p: Sequence[float], Cn: float, window=(2.5, 8.5), levels: int = 13) -> Dict[str, float]:
    """Left, right and mean contact angle (degrees) of the C > 0 droplet in C (ny, nx)."""
    C = np.asarray(C, dtype=np.float64)
    ny, nx = C.shape
    h = (hi[0] - lo[0]) / nx
    L = hi[0] - lo[0]
    yw, dyw = _wall(shape_kind, shape_p)

    def point(s, d):
        t = dyw(s)
        inv = 1.0 / np.sqrt(1.0 + t * t)
        return s - d * t * inv, yw(s) + d * inv           # W(s) + d n(s), n = (-y', 1)/|.|

    # droplet centre of mass along x (fluid cells with C > 0)
    xs = lo[0] + (np.arange(nx) + 0.5) * h
    ys = lo[1] + (np.arange(ny) + 0.5) * h
    fluid = ys[:, None] > yw(xs)[None, :]
    wgt = np.where(fluid & (C > 0), C, 0.0)
    if wgt.sum() <= 0:
        raise AngleError("no droplet (C > 0) above the wall")
    xc = float((wgt.sum(axis=0) * xs).sum() / wgt.sum())

    ds = Cn * np.linspace(window[0], window[1], levels)
    out = {}
    for side, sgn in (("left", -1.0), ("right", 1.0)):
        pts = []
        for d in ds:
            step = 0.25 * h
            s_in = xc
            px, py = point(s_in, d)
            if _bilinear(C, lo, h, px, py) <= 0:
                raise AngleError(f"droplet centre not inside C > 0 at distance {d:.4g}")
            found = False
            for k in range(1, int(0.5 * L / step)):
                s_out = xc + sgn * k * step
                px, py = point(s_out, d)
                if _bilinear(C, lo, h, px, py) <= 0:
                    found = True
                    break
                s_in = s_out
            if not found:
                raise AngleError("no C = 0 crossing found on the " + side)
            a, b = s_in, s_out
            for _ in range(40):
                m = 0.5 * (a + b)
                px, py = point(m, d)
                if _bilinear(C, lo, h, px, py) > 0:
                    a = m
                else:
                    b = m
            pts.append(point(0.5 * (a + b), d))
        pts = np.array(pts)                                # (levels, 2)
        # quadratic curve through the crossings in their principal frame, b = c0 + c1 a + c2 a^2
        pm = pts.mean(axis=0)
        _, _, vt = np.linalg.svd(pts - pm)
        e1 = vt[0]
        if (pts[-1] - pts[0]) @ e1 < 0:                    # e1 points away from the wall
            e1 = -e1
        e2 = np.array([-e1[1], e1[0]])
        a_ = (pts - pm) @ e1
        b_ = (pts - pm) @ e2
        c2, c1, c0 = np.polyfit(a_, b_, 2)

        def q(a):
            return pm + a * e1 + (c0 + c1 * a + c2 * a * a) * e2

        def above(a):                                      # height of q(a) above the wall
            x, yv = q(a)
            return yv - yw(x)
        lo_a = a_.min()
        hi_a = lo_a
        span = a_.max() - a_.min()
        while above(lo_a) > 0:                             # walk towards the wall to bracket it
            lo_a -= 0.25 * span
            if lo_a < a_.min() - 4 * span:
                raise AngleError("interface fit does not reach the wall on the " + side)
        for _ in range(60):
            m = 0.5 * (lo_a + hi_a)
            if above(m) > 0:
                hi_a = m
            else:
                lo_a = m
        a0 = 0.5 * (lo_a + hi_a)
        P0 = q(a0)
        ti = e1 + (c1 + 2 * c2 * a0) * e2
        ti /= np.linalg.norm(ti)
        s0 = P0[0]
        tw = np.array([1.0, dyw(s0)])
        tw /= np.linalg.norm(tw)
        if sgn > 0:
            tw = -tw
        out[side] = math.degrees(math.acos(max(-1.0, min(1.0, float(tw @ ti)))))
        out[side + "_x"] = float(s0)
    out["mean"] = 0.5 * (out["left"] + out["right"])
    return out
