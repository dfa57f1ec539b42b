"""Oracle geometry preprocessing (one-time, host): volume fraction, normals, ghost tables.

Follows section 4.1 of the paper ("Preliminary computations"):

* volume fraction by counting subgrid points outside the solid (4.1.1);
* wall normal from the corner gradients of the volume fraction, averaged to the
  cell centre and normalised (4.1.1, Eqs. NormalVectors_part1/2);
* ghost, intersect, mirror and interpolation points on the wall normal (4.1.2);
* averaging points and inverse-squared-distance weights of the two
  interpolation points (4.1.4, Eq. "weright averaged").

Readings of silent or garbled passages:

* the normal is m / sqrt(m.m + eps0) with eps0 = 1e-30 (the printed formula
  repeats one component and puts a grid spacing in the numerator);
* the corner gradient divides by the sum of the two adjacent spacings along the
  same axis, averaged over the 2^(d-1) cell pairs;
* subgrid points sit at sub-cell centres, 100 per direction as the paper states
  (in 3D too; configurable);
* a ghost is a solid cell centre with at least one face neighbour whose centre
  is fluid; a ghost touching the bounded (last) axis' box wall is rejected;
* the intersect point is found by marching from the ghost along n in steps of
  h/100 to the first fluid point, then bisecting 60 times (the kept end is the
  fluid one);
* d1 (intersect to mirror) defaults to 2h and d2 to 1.5h (d2 < d1 as the
  paper asks); the interpolation points lie beyond the mirror point:
  IP1 = M + d2 n, IP2 = M + 2 d2 n.  The paper only asks for d1 above half a
  cell diagonal; with d1 near one diagonal and d2 = h/2 the averaging stencil
  of IP1 reaches the ghost's own fluid neighbours and near-wall modes grow for
  strongly wetting angles at Cn/h ~ 1.3;
* the averaging points of an interpolation point are the cell containing it
  and that cell's 2d face neighbours (5 in 2D, 7 in 3D); averaging points whose
  centre is solid are dropped and the remaining weights renormalised; if none
  remains, the nearest fluid centre within 2h carries the whole weight.
"""
from __future__ import annotations

import dataclasses
import itertools
import math
from typing import List, Optional, Sequence

import numpy as np

from workloads import BOX, HALFPLANE, SINUSOID, SPHERE, Grid, Params, Shape

TWO_PI = 6.283185307179586
EPS0 = 1e-30


class GeometryError(RuntimeError):
    pass


# ---------------------------------------------------------------------------
# Shape predicates (solid = True).

def _solid_shape(shape: Shape, X: Sequence[np.ndarray], ndim: int) -> np.ndarray:
    p = shape.padded()
    k = shape.kind
    if k == HALFPLANE:
        s = (X[0] - p[0]) * p[3] + (X[1] - p[1]) * p[4]
        if ndim == 3:
            s = s + (X[2] - p[2]) * p[5]
        return s < 0.0
    if k == SINUSOID:
        yw = p[0] + p[1] * np.sin(TWO_PI * X[0] / p[2] + p[3])
        return X[ndim - 1] < yw
    if k == SPHERE:
        dx = X[0] - p[0]
        dy = X[1] - p[1]
        r2 = dx * dx + dy * dy
        if ndim == 3:
            dz = X[2] - p[2]
            r2 = r2 + dz * dz
        return r2 < p[3] * p[3]
    if k == BOX:
        c, s_ = math.cos(p[4]), math.sin(p[4])
        dx = X[0] - p[0]
        dy = X[1] - p[1]
        q0 = c * dx + s_ * dy
        q1 = -s_ * dx + c * dy
        out = (np.abs(q0) > p[3]) | (np.abs(q1) > p[3])
        if ndim == 3:
            out = out | (np.abs(X[2] - p[2]) > p[3])
        return out
    raise GeometryError(f"unknown shape kind {k}")


def wrap_periodic(grid: Grid, X: Sequence[np.ndarray]) -> List[np.ndarray]:
    """Shift points lying outside the box by one period along the periodic axes."""
    out = []
    for a in range(grid.ndim):
        x = np.asarray(X[a], dtype=np.float64)
        if a < grid.ndim - 1:
            L = grid.hi[a] - grid.lo[a]
            x = np.where(x >= grid.hi[a], x - L, np.where(x < grid.lo[a], x + L, x))
        out.append(x)
    return out


def solid(grid: Grid, shapes: Sequence[Shape], X: Sequence[np.ndarray]) -> np.ndarray:
    """Union of the shapes' solid regions, evaluated at (periodically wrapped) points."""
    Xw = wrap_periodic(grid, X)
    if not shapes:
        return np.zeros(np.broadcast(*Xw).shape, dtype=bool)
    out = None
    for s in shapes:
        v = _solid_shape(s, Xw, grid.ndim)
        out = v if out is None else (out | v)
    return out


def _may_be_cut(shape: Shape, Xc: Sequence[np.ndarray], grid: Grid) -> np.ndarray:
    """Conservative test: can the cell centred at Xc hold both solid and fluid points?"""
    h = grid.h
    d = grid.ndim
    hd = 0.5 * h * math.sqrt(d)
    m = 1e-9 * h
    p = shape.padded()
    k = shape.kind
    if k == HALFPLANE:
        nn = math.sqrt(sum(p[3 + a] ** 2 for a in range(d)))
        s = sum((Xc[a] - p[a]) * p[3 + a] for a in range(d)) / nn
        return np.abs(s) <= hd + m
    if k == SPHERE:
        r = np.sqrt(sum((Xc[a] - p[a]) ** 2 for a in range(d)))
        return np.abs(r - p[3]) <= hd + m
    if k == SINUSOID:
        lip = TWO_PI * abs(p[1]) / p[2]
        yw = p[0] + p[1] * np.sin(TWO_PI * Xc[0] / p[2] + p[3])
        return np.abs(Xc[d - 1] - yw) <= 0.5 * h + 0.5 * lip * h + m
    if k == BOX:
        c, s_ = math.cos(p[4]), math.sin(p[4])
        dx = Xc[0] - p[0]
        dy = Xc[1] - p[1]
        q = [np.abs(c * dx + s_ * dy) - p[3], np.abs(-s_ * dx + c * dy) - p[3]]
        if d == 3:
            q.append(np.abs(Xc[2] - p[2]) - p[3])
        outside = np.sqrt(sum(np.maximum(qq, 0.0) ** 2 for qq in q))
        inside = np.minimum(np.maximum.reduce(q), 0.0)
        return np.abs(outside + inside) <= hd + m
    raise GeometryError(f"unknown shape kind {k}")


def default_subgrid(grid: Grid, params: Params) -> int:
    if params.subgrid > 0:
        return int(params.subgrid)
    return 100


def cell_index_coords(grid: Grid):
    """Full arrays of integer cell indices per axis (x first), in field layout."""
    idx = np.indices(grid.shape)
    return [idx[grid.ndim - 1 - a] for a in range(grid.ndim)]


def centre_coords(grid: Grid, I: Sequence[np.ndarray]) -> List[np.ndarray]:
    return [grid.lo[a] + (I[a] + 0.5) * grid.h for a in range(grid.ndim)]


def volume_fraction(grid: Grid, shapes: Sequence[Shape], subgrid: int, face_axis: Optional[int] = None):
    """Fluid volume fraction alpha of every cell and the centre solid mask (section 4.1.1).

    alpha = (number of subgrid points outside the solid) / subgrid^d, counted
    in cells that the wall may cut; other cells are wholly solid or fluid and
    take 0 or 1 from their centre.  With ``face_axis`` = a the control volumes
    are the staggered cells of the faces normal to axis a (each cell shifted by
    h/2 along a), the other three of the four volume fractions the section
    asks for on a staggered grid.
    """
    d = grid.ndim
    h = grid.h
    I = cell_index_coords(grid)
    Xc = centre_coords(grid, I)
    off = [0.0] * d
    if face_axis is not None:
        off[face_axis] = 0.5 * h
        Xc = [Xc[a] + off[a] for a in range(d)]
    csolid = solid(grid, shapes, Xc)
    alpha = np.where(csolid, 0.0, 1.0)
    cut = np.zeros(grid.shape, dtype=bool)
    for s in shapes:
        cut |= _may_be_cut(s, Xc, grid)
    flat_cut = np.flatnonzero(cut)
    n = int(subgrid)
    hs = h / n
    sub = (np.arange(n, dtype=np.float64) + 0.5) * hs
    per_cell = n ** d
    chunk = max(1, 4_000_000 // per_cell)
    aflat = alpha.reshape(-1)
    Iflat = [ii.reshape(-1) for ii in I]
    for c0 in range(0, flat_cut.size, chunk):
        cells = flat_cut[c0:c0 + chunk]
        X = []
        for a in range(d):
            base = grid.lo[a] + Iflat[a][cells].astype(np.float64) * h + off[a]
            shp = [1] * (d + 1)
            shp[1 + a] = n
            X.append(base.reshape((cells.size,) + (1,) * d) + sub.reshape(shp))
        inside = solid(grid, shapes, [np.broadcast_to(x, [cells.size] + [n] * d) for x in X])
        fluid_count = (~inside).reshape(cells.size, -1).sum(axis=1)
        aflat[cells] = fluid_count / float(per_cell)
    return alpha, csolid


def face_fractions(grid: Grid, shapes: Sequence[Shape], params: Params) -> List[np.ndarray]:
    """Fluid volume fractions of the face-centred staggered cells, one field per axis
    (entry c of field a belongs to the face between cell c and c + e_a)."""
    n = default_subgrid(grid, params)
    return [volume_fraction(grid, shapes, n, face_axis=a)[0] for a in range(grid.ndim)]


@dataclasses.dataclass
class GhostTables:
    """Per-ghost tables (structure of arrays), sorted by the ghost's linear cell index.

    ap/w have shape (2, K, G): averaging points and weights of IP1 and IP2.
    Unused averaging slots carry weight 0 and repeat a used index.
    """

    gidx: np.ndarray          # (G,) int64 linear cell index, x fastest
    normal: np.ndarray        # (d, G) unit wall normal pointing into the fluid
    dn: np.ndarray            # (G,) ghost-to-intersect distance
    gamma: np.ndarray         # (G,) d1 / dn
    ap: np.ndarray            # (2, K, G) int64
    w: np.ndarray             # (2, K, G) float64
    alpha: np.ndarray         # cell volume fraction (field layout)
    csolid: np.ndarray        # cell-centre solid mask (field layout)
    points: dict              # 'G','I','M','IP1','IP2' -> (d, G) coordinates
    d1: float
    d2: float

    @property
    def n_ghost(self) -> int:
        return int(self.gidx.size)

    @property
    def n_ap(self) -> int:
        return int(self.ap.shape[1])


def _alpha_at(grid: Grid, alpha: np.ndarray, cells: Sequence[np.ndarray]) -> np.ndarray:
    """alpha at integer cell indices (x first), periodic wrap on periodic axes."""
    idx = []
    for a in range(grid.ndim):
        c = cells[a]
        if a < grid.ndim - 1:
            c = np.mod(c, grid.n[a])
        elif np.any((c < 0) | (c >= grid.n[a])):
            raise GeometryError("normal stencil leaves the box along the bounded axis")
        idx.append(c)
    return alpha[tuple(reversed(idx))]


def wall_normals(grid: Grid, alpha: np.ndarray, gcell: np.ndarray) -> np.ndarray:
    """Unit normals at the given cells from corner gradients of alpha (Eqs. NormalVectors_part1/2).

    A corner gradient component is the one-cell difference of alpha across the
    corner, averaged over the 2^(d-1) cell pairs that share the corner, divided
    by h; the cell value is the mean over its 2^d corners.
    """
    d = grid.ndim
    h = grid.h
    G = gcell.shape[1]
    m = np.zeros((d, G))
    for s in itertools.product((0, 1), repeat=d):
        mc = np.zeros((d, G))
        for t in itertools.product((0, 1), repeat=d):
            cells = [gcell[a] + s[a] - 1 + t[a] for a in range(d)]
            av = _alpha_at(grid, alpha, cells)
            for a in range(d):
                mc[a] += av if t[a] == 1 else -av
        mc /= (2 ** (d - 1)) * h
        m += mc
    m /= 2 ** d
    nrm = np.sqrt((m * m).sum(axis=0) + EPS0)
    return m / nrm


def _points_solid(grid, shapes, P):
    return solid(grid, shapes, [P[a] for a in range(grid.ndim)])


def build_tables(grid: Grid, shapes: Sequence[Shape], params: Params) -> GhostTables:
    """Geometry preprocessing P1-P9 (section 4.1): the permanent per-ghost arrays."""
    d = grid.ndim
    h = grid.h
    nsub = default_subgrid(grid, params)
    alpha, csolid = volume_fraction(grid, shapes, nsub)

    # ghosts: solid centres with a fluid face neighbour
    fluid = ~csolid
    has_fluid_nb = np.zeros_like(csolid)
    for a in range(d):
        ax = d - 1 - a
        if a < d - 1:
            has_fluid_nb |= np.roll(fluid, 1, axis=ax) | np.roll(fluid, -1, axis=ax)
        else:
            up = np.zeros_like(fluid)
            dn_ = np.zeros_like(fluid)
            sl_hi = [slice(None)] * d
            sl_lo = [slice(None)] * d
            sl_hi[ax] = slice(0, -1)
            sl_lo[ax] = slice(1, None)
            up[tuple(sl_hi)] = fluid[tuple(sl_lo)]
            dn_[tuple(sl_lo)] = fluid[tuple(sl_hi)]
            has_fluid_nb |= up | dn_
    ghost = csolid & has_fluid_nb
    gidx = np.flatnonzero(ghost).astype(np.int64)
    G = gidx.size
    unr = np.unravel_index(gidx, grid.shape)
    gcell = np.stack([unr[d - 1 - a] for a in range(d)]).astype(np.int64)
    last = gcell[d - 1]
    if G and (np.any(last == 0) or np.any(last == grid.n[d - 1] - 1)):
        raise GeometryError("a ghost point touches the box wall of the bounded axis")

    n = wall_normals(grid, alpha, gcell)
    Gp = np.stack([grid.lo[a] + (gcell[a] + 0.5) * h for a in range(d)])

    # intersect point: march along n, then bisect
    delta = h / 100.0
    kmax = 1000
    kfound = np.zeros(G, dtype=np.int64)
    active = np.ones(G, dtype=bool)
    for k in range(1, kmax + 1):
        if not active.any():
            break
        ia = np.flatnonzero(active)
        P = Gp[:, ia] + (k * delta) * n[:, ia]
        out = ~_points_solid(grid, shapes, P)
        done = ia[out]
        kfound[done] = k
        active[done] = False
    if active.any():
        raise GeometryError("marching along the normal found no fluid within 10 cells")
    tlo = (kfound - 1) * delta
    thi = kfound * delta
    for _ in range(60):
        tm = 0.5 * (tlo + thi)
        P = Gp + tm * n
        s = _points_solid(grid, shapes, P)
        tlo = np.where(s, tm, tlo)
        thi = np.where(s, thi, tm)
    Ip = Gp + thi * n
    dn = np.sqrt(((Ip - Gp) ** 2).sum(axis=0))

    d1 = (params.d1_cells if params.d1_cells > 0 else 2.0) * h
    d2 = (params.d2_cells if params.d2_cells > 0 else 1.5) * h
    Mp = Ip + d1 * n
    IP1 = Mp + d2 * n
    IP2 = Mp + (2.0 * d2) * n
    gamma = d1 / dn

    K = 2 * d + 1
    ap = np.zeros((2, K, G), dtype=np.int64)
    w = np.zeros((2, K, G))
    for j, IPp in enumerate((IP1, IP2)):
        ap[j], w[j] = _averaging(grid, csolid, IPp, K)

    pts = {"G": Gp, "I": Ip, "M": Mp, "IP1": IP1, "IP2": IP2}
    return GhostTables(gidx, n, dn, gamma, ap, w, alpha, csolid, pts, d1, d2)


def _linear(grid: Grid, cells: Sequence[np.ndarray]) -> np.ndarray:
    lin = np.zeros_like(cells[0])
    stride = 1
    for a in range(grid.ndim):
        lin = lin + cells[a] * stride
        stride *= grid.n[a]
    return lin


def _averaging(grid: Grid, csolid: np.ndarray, IPp: np.ndarray, K: int):
    """Averaging points and normalised 1/h^2 weights of one interpolation point per ghost."""
    d = grid.ndim
    h = grid.h
    G = IPp.shape[1]
    cstar = np.stack([np.floor((IPp[a] - grid.lo[a]) / h).astype(np.int64) for a in range(d)])
    offs = [np.zeros(d, dtype=np.int64)]
    for a in range(d):
        for sgn in (-1, 1):
            o = np.zeros(d, dtype=np.int64)
            o[a] = sgn
            offs.append(o)
    idx = np.zeros((K, G), dtype=np.int64)
    hk = np.zeros((K, G))
    valid = np.zeros((K, G), dtype=bool)
    csflat = csolid.reshape(-1)
    for s, o in enumerate(offs):
        u = cstar + o[:, None]
        ok = np.ones(G, dtype=bool)
        wrapped = []
        for a in range(d):
            if a < d - 1:
                wrapped.append(np.mod(u[a], grid.n[a]))
            else:
                ok &= (u[a] >= 0) & (u[a] < grid.n[a])
                wrapped.append(np.clip(u[a], 0, grid.n[a] - 1))
        lin = _linear(grid, wrapped)
        ok &= ~csflat[lin]
        xap = [grid.lo[a] + (u[a] + 0.5) * h for a in range(d)]
        dist2 = np.zeros(G)
        for a in range(d):
            dd = IPp[a] - xap[a]
            dist2 = dist2 + dd * dd
        idx[s] = lin
        hk[s] = np.sqrt(dist2)
        valid[s] = ok
    w = np.zeros((K, G))
    for g in range(G):
        vs = [s for s in range(K) if valid[s, g]]
        if not vs:
            lin = _fallback(grid, csflat, IPp[:, g], cstar[:, g])
            idx[:, g] = lin
            w[0, g] = 1.0
            continue
        near = [s for s in vs if hk[s, g] < 1e-12 * h]
        if near:
            w[near[0], g] = 1.0
        else:
            inv = [1.0 / (hk[s, g] * hk[s, g]) for s in vs]
            q = 0.0
            for v in inv:
                q += v
            for s, v in zip(vs, inv):
                w[s, g] = v / q
        first = idx[vs[0], g]
        for s in range(K):
            if not valid[s, g]:
                idx[s, g] = first
    return idx, w


def _fallback(grid, csflat, ip, cstar):
    d = grid.ndim
    h = grid.h
    best = None
    for o in itertools.product(range(-2, 3), repeat=d):
        u = [int(cstar[a]) + o[d - 1 - a] for a in range(d)]
        if not (0 <= u[d - 1] < grid.n[d - 1]):
            continue
        wr = [u[a] % grid.n[a] if a < d - 1 else u[a] for a in range(d)]
        lin = int(_linear(grid, [np.int64(v) for v in wr]))
        if csflat[lin]:
            continue
        dist2 = 0.0
        for a in range(d):
            dd = ip[a] - (grid.lo[a] + (u[a] + 0.5) * h)
            dist2 += dd * dd
        dist = math.sqrt(dist2)
        if dist <= 2.0 * h and (best is None or dist < best[0]):
            best = (dist, lin)
    if best is None:
        raise GeometryError("an interpolation point has no fluid averaging point within 2h")
    return best[1]
