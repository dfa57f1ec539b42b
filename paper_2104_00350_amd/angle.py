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

`measure_cap` is the equilibrium measurement: at rest the 2D interface away from the wall's
diffuse layer is a circular arc (uniform pressure jump), so the droplet's C = 0 crossings
farther than a few interface widths from the wall are fitted by one circle, which is then
followed down to its first intersections with the wall curve on each side.  There the angle
through the droplet between wall and interface satisfies cos(theta) = n_w . (P - c) / R,
with n_w the wall normal into the fluid, c and R the circle's centre and radius.  It does not
look at the region near the wall, so the wall's curvature within a few interface widths of the
contact line cannot fold the sampling curves.
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


def _wall_distance(shape_kind: int, p: Sequence[float], x, y):
    """Unsigned distance from points (x, y) above the wall to the wall curve (Newton on the
    nearest-point condition from three seeds, smallest result)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if shape_kind == HALFPLANE:
        return np.abs(y - p[1])
    mean, amp, lam, ph = p[0], p[1], p[2], p[3]
    k = 2.0 * math.pi / lam
    best = np.full(x.shape, np.inf)
    for seed in (0.0, -0.25 * lam, 0.25 * lam):
        s = x + seed
        for _ in range(20):
            yw = mean + amp * np.sin(k * s + ph)
            d1 = amp * k * np.cos(k * s + ph)
            d2 = -amp * k * k * np.sin(k * s + ph)
            f = (s - x) + (yw - y) * d1
            fp = 1.0 + d1 * d1 + (yw - y) * d2
            fp = np.where(fp > 0.1, fp, 0.1)
            s = s - np.clip(f / fp, -0.1 * lam, 0.1 * lam)
        best = np.minimum(best, np.hypot(s - x, mean + amp * np.sin(k * s + ph) - y))
    return best


def _fit_circle(P: np.ndarray):
    """Least-squares circle through points P (m, 2): algebraic fit, then Gauss-Newton on the
    geometric residuals |p - c| - R."""
    A_ = np.column_stack([P[:, 0], P[:, 1], np.ones(len(P))])
    sol, *_ = np.linalg.lstsq(A_, -(P[:, 0] ** 2 + P[:, 1] ** 2), rcond=None)
    c = np.array([-0.5 * sol[0], -0.5 * sol[1]])
    R = math.sqrt(max(c @ c - sol[2], 1e-300))
    for _ in range(20):
        d = P - c
        r = np.hypot(d[:, 0], d[:, 1])
        res = r - R
        J = np.column_stack([-d[:, 0] / r, -d[:, 1] / r, -np.ones(len(P))])
        step, *_ = np.linalg.lstsq(J, -res, rcond=None)
        c = c + step[:2]
        R = R + step[2]
        if np.max(np.abs(step)) < 1e-14 * max(1.0, R):
            break
    res = np.hypot(P[:, 0] - c[0], P[:, 1] - c[1]) - R
    return c, R, res


def measure_cap(C: np.ndarray, lo: Sequence[float], hi: Sequence[float], shape_kind: int,
                shape_p: Sequence[float], Cn: float, min_dist: float = 3.0, rays: int = 720) -> Dict[str, float]:
    """Equilibrium contact angles (degrees) of the C > 0 droplet from a circular-cap fit.

    Crossings C = 0 are found along `rays` rays from the droplet's centre of mass (bisection of
    the bilinearly interpolated C; a ray that enters the solid first has none), and those closer
    than min_dist * Cn to the wall are dropped.  Points farther than 3 median deviations (and two
    cells) from the fitted circle are trimmed and the circle refitted (up to three times), so
    liquid left in a groove does not bend the fit.  Returns left, right, mean, the contact
    abscissas and the rms fit residual over the cell size (`fit_rms_cells`)."""
    C = np.asarray(C, dtype=np.float64)
    ny, nx = C.shape
    h = (hi[0] - lo[0]) / nx
    yw, dyw = _wall(shape_kind, shape_p)
    xs = lo[0] + (np.arange(nx) + 0.5) * h
    ys = lo[1] + (np.arange(ny) + 0.5) * h
    fluid = ys[:, None] > yw(xs)[None, :]
    wgt = np.where(fluid & (C > 0), C, 0.0)
    if wgt.sum() <= 0:
        raise AngleError("no droplet (C > 0) above the wall")
    xc = float((wgt.sum(axis=0) * xs).sum() / wgt.sum())
    yc = float((wgt.sum(axis=1) * ys).sum() / wgt.sum())
    if _bilinear(C, lo, h, xc, yc) <= 0:
        raise AngleError("droplet centre of mass is not inside C > 0")
    dmin = min_dist * Cn
    phi = np.linspace(0.0, 2.0 * math.pi, rays, endpoint=False)
    ux, uy = np.cos(phi), np.sin(phi)
    step = 0.25 * h
    rmax = 0.5 * (hi[0] - lo[0])
    alive = np.ones(rays, dtype=bool)
    r_in = np.zeros(rays)
    r_out = np.full(rays, np.nan)
    r = 0.0
    while alive.any() and r < rmax:
        r += step
        px, py = xc + r * ux, yc + r * uy
        out_box = (py <= lo[1]) | (py >= hi[1])
        solid = np.zeros(rays, dtype=bool)
        idx = np.nonzero(alive & ~out_box)[0]
        solid[idx] = py[idx] <= yw(px[idx])
        alive &= ~(out_box | solid)
        idx = np.nonzero(alive)[0]
        neg = _bilinear(C, lo, h, px[idx], py[idx]) <= 0
        hit = idx[neg]
        r_out[hit] = r
        r_in[hit] = r - step
        alive[hit] = False
    ok = np.isfinite(r_out)
    a, b = r_in[ok], r_out[ok]
    for _ in range(40):
        m = 0.5 * (a + b)
        pos = _bilinear(C, lo, h, xc + m * ux[ok], yc + m * uy[ok]) > 0
        a = np.where(pos, m, a)
        b = np.where(pos, b, m)
    rm = 0.5 * (a + b)
    P = np.column_stack([xc + rm * ux[ok], yc + rm * uy[ok]])
    P = P[_wall_distance(shape_kind, shape_p, P[:, 0], P[:, 1]) >= dmin]
    if len(P) < 12:
        raise AngleError("too few interface points away from the wall")
    keep = np.ones(len(P), dtype=bool)
    for _ in range(3):
        c, R, res = _fit_circle(P[keep])
        res_all = np.hypot(P[:, 0] - c[0], P[:, 1] - c[1]) - R
        mad = np.median(np.abs(res_all[keep] - np.median(res_all[keep])))
        new = np.abs(res_all) <= max(3.0 * 1.4826 * mad, 2.0 * h)
        if new.sum() < 12 or np.array_equal(new, keep):
            break
        keep = new
    c, R, res = _fit_circle(P[keep])
    # follow the circle from the ends of the fitted arc down to the wall on each side
    v = (P[keep] - c) / R
    mid = v.mean(axis=0)
    psi_mid = math.atan2(mid[1], mid[0])
    dpsi = np.angle(np.exp(1j * (np.arctan2(v[:, 1], v[:, 0]) - psi_mid)))

    def below(ps):
        x, y = c[0] + R * math.cos(ps), c[1] + R * math.sin(ps)
        return y - float(yw(x)) <= 0

    out = {}
    dstep = 0.25 * h / R
    for side, start, sgn in (("left", dpsi.max(), 1.0), ("right", dpsi.min(), -1.0)):
        d_in = start
        d_out = None
        d = start
        while abs(d) < math.pi:
            d += sgn * dstep
            if below(psi_mid + d):
                d_out = d
                break
            d_in = d
        if d_out is None:
            raise AngleError("fitted circle does not meet the wall on the " + side)
        for _ in range(60):
            m = 0.5 * (d_in + d_out)
            if below(psi_mid + m):
                d_out = m
            else:
                d_in = m
        ps = psi_mid + 0.5 * (d_in + d_out)
        Px, Py = c[0] + R * math.cos(ps), c[1] + R * math.sin(ps)
        t = float(dyw(Px))
        nw = np.array([-t, 1.0]) / math.sqrt(1.0 + t * t)
        cos_t = float(nw @ ((np.array([Px, Py]) - c) / R))
        out[side] = math.degrees(math.acos(max(-1.0, min(1.0, cos_t))))
        out[side + "_x"] = Px
    out["mean"] = 0.5 * (out["left"] + out["right"])
    out["fit_rms_cells"] = float(np.sqrt(np.mean(res ** 2)) / h)
    out["points"] = int(keep.sum())
    return out
