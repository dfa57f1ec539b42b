"""Reference of the learned wall-band correction (test infrastructure only).

Not part of the paper: the correction is an extension of the method (a coarse 2D run corrected
near the wall by a small convolutional network).  This module states what the device library
computes, in plain NumPy with float64 arithmetic, and rounds to BF16 (round to nearest even)
exactly where the device stores BF16 values, so that the two agree to float32 accumulation
order.  It shares no code with the library.

Network (per cell of a 2D grid, x fastest, periodic along x, zeros outside the box along y for
every layer's input):
  X  = [C, phi, clip(dist / (band h), -2, 2), n_x, n_y]            features (BF16)
  h1 = tanh(W1 * X + b1)          32 channels (BF16)
  h2 = tanh(W2 * h1 + b2)         32 channels (BF16)
  dC = s (W3 * h2 + b3)
"*" is the 3x3 cross-correlation out(x, y) = sum_{ky,kx} W[ky][kx] in(x + kx - 1, y + ky - 1).
The correction applies in the band 0 < dist <= band h, |C| < 0.9, limited so that C + dC stays
inside [-1, 1].
Parameter vector: W1[9][32][16] (tap = 3 ky + kx, out, in; inputs 5..15 unused), b1[32],
W2[9][32][32], b2[32], W3[9][32], b3.
"""
from __future__ import annotations

import math
from typing import Dict, List, Sequence, Tuple

import numpy as np

TS, HX, E1, E2, CIN, NFEAT, CH = 16, 22, 20, 18, 16, 5, 32
OFF_W1 = 0
OFF_B1 = OFF_W1 + 9 * CH * CIN
OFF_W2 = OFF_B1 + CH
OFF_B2 = OFF_W2 + 9 * CH * CH
OFF_W3 = OFF_B2 + CH
OFF_B3 = OFF_W3 + 9 * CH
NPARAM = OFF_B3 + 1


# -- BF16 -----------------------------------------------------------------------------------
def bf16(x) -> np.ndarray:
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def unpack(params: np.ndarray, round_weights: bool = True) -> Dict[str, np.ndarray]:
    """Weights as (tap, out, in) arrays (BF16-rounded unless told otherwise), biases as given."""
    p = np.asarray(params, dtype=np.float32).astype(np.float64)
    r = bf16 if round_weights else (lambda a: a)
    return {
        "W1": r(p[OFF_W1:OFF_B1]).reshape(9, CH, CIN)[:, :, :NFEAT],
        "b1": p[OFF_B1:OFF_W2],
        "W2": r(p[OFF_W2:OFF_B2]).reshape(9, CH, CH),
        "b2": p[OFF_B2:OFF_W3],
        "W3": r(p[OFF_W3:OFF_B3]).reshape(9, CH),
        "b3": p[OFF_B3],
    }


# -- wall field -----------------------------------------------------------------------------
def wall_field(n: Tuple[int, int], lo, hi, shapes) -> Tuple[np.ndarray, np.ndarray]:
    """Signed distance to the wall (> 0 in the fluid, minimum over the shapes) and the unit
    normal into the fluid at the nearest wall point, on the cell centres of a 2D grid."""
    nx, ny = n
    h = (hi[0] - lo[0]) / nx
    x = lo[0] + (np.arange(nx) + 0.5) * h
    y = lo[1] + (np.arange(ny) + 0.5) * h
    X, Y = np.meshgrid(x, y)
    best = np.full(X.shape, np.inf)
    bn = np.zeros((2,) + X.shape)
    for sh in shapes:
        p = sh.p
        if sh.kind == 1:        # half-plane: point p[0:2], normal p[3:5]
            nn = math.hypot(p[3], p[4])
            n0, n1 = p[3] / nn, p[4] / nn
            sd = (X - p[0]) * n0 + (Y - p[1]) * n1
            N0, N1 = np.full(X.shape, n0), np.full(X.shape, n1)
        elif sh.kind == 3:      # circle
            dx, dy = X - p[0], Y - p[1]
            r = np.hypot(dx, dy)
            sd = r - p[3]
            N0, N1 = dx / r, dy / r
        elif sh.kind == 2:      # sinusoid y = p0 + p1 sin(2 pi x / p2 + p3)
            sd, N0, N1 = _sinusoid_distance(X, Y, p)
        else:
            raise ValueError("unsupported wall shape")
        take = sd < best
        best = np.where(take, sd, best)
        bn[0] = np.where(take, N0, bn[0])
        bn[1] = np.where(take, N1, bn[1])
    return best, bn


def _sinusoid_distance(X, Y, p):
    A, lam, ph = p[1], p[2], p[3]
    k = 2 * math.pi / lam
    yw = lambda s: p[0] + A * np.sin(k * s + ph)
    # dense search over one wavelength around each point, then Newton on the squared distance
    offs = lam * (np.arange(64) + 0.5) / 64 - 0.5 * lam
    S = X[..., None] + offs
    D2 = (S - X[..., None]) ** 2 + (yw(S) - Y[..., None]) ** 2
    s = np.take_along_axis(S, np.argmin(D2, axis=-1)[..., None], axis=-1)[..., 0]
    for _ in range(60):
        sn, cs = np.sin(k * s + ph), np.cos(k * s + ph)
        f1 = A * k * cs
        f2 = -A * k * k * sn
        g = (s - X) + (p[0] + A * sn - Y) * f1
        gp = 1 + f1 * f1 + (p[0] + A * sn - Y) * f2
        s = s - g / gp
    d = np.hypot(s - X, yw(s) - Y)
    sd = np.where(Y >= yw(X), d, -d)
    f1 = A * k * np.cos(k * s + ph)
    nn = np.sqrt(1 + f1 * f1)
    return sd, -f1 / nn, 1.0 / nn


# -- features, forward ----------------------------------------------------------------------
def features(C, phi, dist, nrm, band_h: float) -> np.ndarray:
    """(5, ny, nx) BF16 features; arithmetic in float32 as on the device."""
    d32 = np.asarray(dist, np.float32) * np.float32(1.0 / band_h)
    f = [np.asarray(C, np.float32), np.asarray(phi, np.float32),
         np.clip(d32, np.float32(-2), np.float32(2)),
         np.asarray(nrm[0], np.float32), np.asarray(nrm[1], np.float32)]
    return np.stack([bf16(v) for v in f])


def limit(C, dC) -> np.ndarray:
    """The applied correction keeps C + dC inside [-1, 1] (float32 result, as stored)."""
    return (np.clip(C + dC, -1.0, 1.0) - C).astype(np.float32).astype(np.float64)


def band_mask(C, dist, band_h: float) -> np.ndarray:
    d = np.asarray(dist, np.float32).astype(np.float64)
    return (d > 0) & (d <= band_h) & (np.abs(C) < 0.9)


def _shift(a, dx, dy):
    """a[..., y + dy, x + dx] with x periodic and zeros outside the box along y."""
    out = np.roll(a, -dx, axis=-1)
    if dy == 0:
        return out
    res = np.zeros_like(out)
    if dy > 0:
        res[..., :-dy, :] = out[..., dy:, :]
    else:
        res[..., -dy:, :] = out[..., :dy, :]
    return res


def conv3x3(W, inp):
    """W (9, out, in), inp (in, ny, nx) -> (out, ny, nx), float64 sums."""
    out = np.zeros((W.shape[1],) + inp.shape[1:])
    for t in range(9):
        ky, kx = divmod(t, 3)
        out += np.einsum("oi,iyx->oyx", W[t], _shift(inp, kx - 1, ky - 1))
    return out


def forward(params, X, out_scale: float, rounding: bool = True):
    """Full-grid forward: returns dC (ny, nx) and the activations."""
    P = unpack(params, rounding)
    r = bf16 if rounding else (lambda a: a)
    h1 = r(np.tanh(conv3x3(P["W1"], X) + P["b1"][:, None, None]))
    h2 = r(np.tanh(conv3x3(P["W2"], h1) + P["b2"][:, None, None]))
    out = out_scale * (conv3x3(P["W3"][:, None, :], h2)[0] + P["b3"])
    return out, h1, h2


# -- training on stored tiles ---------------------------------------------------------------
def tile_gradient(params, Xt, Yt, Mt, ty0: int, ny: int, out_scale: float, inv_count: float,
                  rounding: bool = True):
    """Loss and gradient of sum_cells M (dC - Y)^2 inv_count for one stored tile.

    Xt (16, 22, 22) is the feature patch of the tile whose first row is ty0 (patch rows
    ty0 - 3 .. ty0 + 18); the tile forward shrinks 22 -> 20 -> 18 -> 16 and zeroes h1/h2 rows
    outside the box.  With `rounding` the backward signals that the device stores in BF16 (the
    pre-activation signals of both hidden layers) are rounded the same way."""
    P = unpack(params, rounding)
    r = bf16 if rounding else (lambda a: a)
    X = np.asarray(Xt, np.float64)[:NFEAT]

    def valid(W, inp, m):                 # (9, o, i), (i, m+2, m+2) -> (o, m, m)
        out = np.zeros((W.shape[1], m, m))
        for t in range(9):
            ky, kx = divmod(t, 3)
            out += np.einsum("oi,iyx->oyx", W[t], inp[:, ky:ky + m, kx:kx + m])
        return out

    rows1 = ty0 - 2 + np.arange(E1)
    rows2 = ty0 - 1 + np.arange(E2)
    in1 = ((rows1 >= 0) & (rows1 < ny)).astype(float)[None, :, None]
    in2 = ((rows2 >= 0) & (rows2 < ny)).astype(float)[None, :, None]
    h1 = r(np.tanh(valid(P["W1"], X, E1) + P["b1"][:, None, None]) * in1)
    h2 = r(np.tanh(valid(P["W2"], h1, E2) + P["b2"][:, None, None]) * in2)
    out = out_scale * (valid(P["W3"][:, None, :], h2, TS)[0] + P["b3"])
    diff = out - Yt
    loss = float(np.sum(Mt * diff * diff) * inv_count)
    g3 = 2 * inv_count * Mt * diff * out_scale                     # d loss / d (W3 * h2 + b3)
    grad = np.zeros(NPARAM)
    dW3 = np.zeros((9, CH))
    dh2 = np.zeros((CH, E2, E2))
    for t in range(9):
        ky, kx = divmod(t, 3)
        dW3[t] = np.einsum("yx,cyx->c", g3, h2[:, ky:ky + TS, kx:kx + TS])
        dh2[:, ky:ky + TS, kx:kx + TS] += P["W3"][t][:, None, None] * g3[None]
    G2 = r(dh2 * (1 - h2 * h2) * in2)
    dW2 = np.zeros((9, CH, CH))
    dh1 = np.zeros((CH, E1, E1))
    for t in range(9):
        ky, kx = divmod(t, 3)
        dW2[t] = np.einsum("oyx,iyx->oi", G2, h1[:, ky:ky + E2, kx:kx + E2])
        dh1[:, ky:ky + E2, kx:kx + E2] += np.einsum("oi,oyx->iyx", P["W2"][t], G2)
    G1 = r(dh1 * (1 - h1 * h1) * in1)
    dW1 = np.zeros((9, CH, CIN))
    for t in range(9):
        ky, kx = divmod(t, 3)
        dW1[t, :, :NFEAT] = np.einsum("oyx,iyx->oi", G1, X[:, ky:ky + E1, kx:kx + E1])
    grad[OFF_W1:OFF_B1] = dW1.reshape(-1)
    grad[OFF_B1:OFF_W2] = G1.sum(axis=(1, 2))
    grad[OFF_W2:OFF_B2] = dW2.reshape(-1)
    grad[OFF_B2:OFF_W3] = G2.sum(axis=(1, 2))
    grad[OFF_W3:OFF_B3] = dW3.reshape(-1)
    grad[OFF_B3] = g3.sum()
    return loss, grad, out


def adam(params, m, v, g, t: int, lr: float, b1=0.9, b2=0.999, eps=1e-8):
    """One bias-corrected Adam step (returns new params, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def patch(field: np.ndarray, tx0: int, ty0: int) -> np.ndarray:
    """22x22 patch of a (c, ny, nx) field around tile (tx0, ty0); zeros outside the box."""
    c, ny, nx = field.shape
    out = np.zeros((c, HX, HX))
    for py in range(HX):
        gy = ty0 - 3 + py
        if 0 <= gy < ny:
            out[:, py, :] = field[:, gy, (tx0 - 3 + np.arange(HX)) % nx]
    return out


def band_tiles(dist, band_h: float) -> List[Tuple[int, int]]:
    """16x16 tiles (x0, y0), row-major, holding a cell with 0 < dist <= band_h."""
    ny, nx = dist.shape
    out = []
    for ty in range(0, ny, TS):
        for tx in range(0, nx, TS):
            d = dist[ty:ty + TS, tx:tx + TS]
            if np.any((d > 0) & (d <= band_h)):
                out.append((tx, ty))
    return out
