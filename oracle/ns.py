"""Oracle Navier-Stokes coupling: explicit momentum step, volume penalisation, variable-density
pressure projection (sections 2, 3.2, 4.2.3, 4.3 and 4.4, Eqs. NS equation, PredictionExp, Penalization2,
PressurePoisson, correction).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Non-dimensional form (lengths in domain units, velocity scale U, time L/U, density and
viscosity relative to the reference fluid of Re = rho U L / mu):

    du/dt + div(u u) = (1/rho~) [ -grad p + (1/Re) div(mu~ (grad u + grad u^T))
                                  + kappa phi grad C ] + g,      div u = 0,

    rho~(C) = ((C + 1) rho2 - (C - 1) rho1)/2,  mu~(C) = ((C + 1) mu2 - (C - 1) mu1)/2,
    phi = C^3 - C - Cn^2 lap C  (the chemical potential of the order-parameter step),
    kappa = 3 / (2 sqrt2 Re Ca Cn).

Reading of kappa: the paper's free energy carries the factor 3/(2 sqrt2) in the order-parameter
equation and in the wall condition but not in the printed momentum equation.  With the factor the
planar tanh profile carries exactly the surface tension sigma, so a drop of radius R has the
Laplace jump 1/(Re Ca R) in these units, which is what the tests pin.

Staggered (MAC) grid: face field a holds u_a on the face between cell c and c + e_a.  Periodic
axes wrap.  On the bounded (last) axis the box walls are no-slip: the normal face velocity on
both walls is zero (the top wall face is stored and kept at zero, the bottom one is implicit), the
tangential velocity is reflected with a sign change across the wall, the pressure gradient
through the wall is zero, and cell-centred scalars (C, mu) are reflected.

One coupled step (the block diagram of Fig. Chart, end of section 4):
 1. order-parameter step with the current velocity (semi-implicit: the advecting velocity is the
    extrapolation 2u^n - u^(n-1) of Appendix A.1; explicit: u^n), ghost fill of C;
 2. phi, rho~, mu~ from C^(n+1);
 3. prediction u* (Eq. PredictionExp): Adams-Bashforth for the convective term, the viscous and
    capillary terms with u^n and C^(n+1) (the printed 3/2 - 1/2 combinations of one and the same
    quantity reduce to that quantity), the body force constant in time;
    the first step uses forward Euler for the convective term;
 4. penalisation u** = alpha_face u* (Eq. Penalization2, stationary walls);
 5. velocity ghost fill on u** (section 4.3, the existing slip / no-penetration fill);
 6. pressure (Eq. PressurePoisson) with rho0 = min(rho1, rho2), p^ = 2p^n - p^(n-1), solved with
    the cosine / Fourier eigen-decomposition of the discrete Laplacian (zero-mean solution);
 7. correction (Eq. correction) on every face except the box-wall faces.
"""
from __future__ import annotations

import math
from typing import List, Sequence

import numpy as np
import scipy.fft as sfft

from workloads import Grid, Params

from .solver import WORKERS, _shift, eigenvalues

SQRT2 = math.sqrt(2.0)


def capillary_coefficient(params: Params) -> float:
    """kappa = 3 / (2 sqrt2 Re Ca Cn): the capillary force per unit phi grad C."""
    return 3.0 / (2.0 * SQRT2 * params.Re * params.Ca * params.Cn)


def density(C: np.ndarray, params: Params) -> np.ndarray:
    """rho~(C) of section 2 (rho2 at C = +1, rho1 at C = -1)."""
    return 0.5 * ((C + 1.0) * params.rho2 - (C - 1.0) * params.rho1)


def viscosity(C: np.ndarray, params: Params) -> np.ndarray:
    """mu~(C) of section 2."""
    return 0.5 * ((C + 1.0) * params.mu2 - (C - 1.0) * params.mu1)


def _wall(grid: Grid, a: int) -> bool:
    return a == grid.ndim - 1


def _mask_top(grid: Grid, a: int, f: np.ndarray) -> np.ndarray:
    """Face field a with its box-wall faces (top row of the bounded axis) set to zero."""
    if not _wall(grid, a):
        return f
    g = f.copy()
    g[-1] = 0.0
    return g


def _shift_odd(f: np.ndarray, grid: Grid, a: int, s: int) -> np.ndarray:
    """f[c + s e_a] with a tangential no-slip image across the bounded axis' walls: the value
    beyond a wall is minus the value in the first cell row (zero on the wall itself)."""
    out = _shift(f, grid, a, s, "reflect")
    if _wall(grid, a):
        if s == 1:
            out[-1] = -f[-1]
        else:
            out[0] = -f[0]
    return out


def face_mean(f: np.ndarray, grid: Grid, a: int) -> np.ndarray:
    """Cell-centred scalar averaged onto the faces normal to a (reflected across box walls)."""
    return 0.5 * (f + _shift(f, grid, a, 1, "reflect"))


def face_gradient(p: np.ndarray, grid: Grid) -> List[np.ndarray]:
    """Discrete gradient on the faces: (p[c + e_a] - p[c]) / h, zero through the box walls."""
    return [_mask_top(grid, a, (_shift(p, grid, a, 1, "reflect") - p) / grid.h) for a in range(grid.ndim)]


def divergence(faces: Sequence[np.ndarray], grid: Grid) -> np.ndarray:
    """Discrete divergence at the cell centres; the normal velocity on the box walls is zero."""
    out = np.zeros_like(faces[0])
    for a in range(grid.ndim):
        u = _mask_top(grid, a, faces[a])
        out = out + (u - _shift(u, grid, a, -1, "zero"))
    return out / grid.h


def convective(faces: Sequence[np.ndarray], grid: Grid) -> List[np.ndarray]:
    """Conservative central convective term div(u u_a) on the faces of each axis a.

    Along a itself the momentum flux u_a u_a sits at the cell centres, with u_a there the mean of
    the cell's two faces; across another axis b it sits on the edge between the four faces, as
    the product of the two-point means of u_a along b and of u_b along a.  No flux crosses the
    box walls (u_b = 0 there)."""
    d = grid.ndim
    h = grid.h
    U = [_mask_top(grid, a, faces[a]) for a in range(d)]
    out = []
    for a in range(d):
        ua = U[a]
        acc = np.zeros_like(ua)
        for b in range(d):
            if b == a:
                uc = 0.5 * (_shift(ua, grid, a, -1, "zero") + ua)
                P = uc * uc
                acc = acc + (_shift(P, grid, a, 1, "reflect") - P) / h
            else:
                E = 0.5 * (ua + _shift(ua, grid, b, 1, "reflect")) * 0.5 * (U[b] + _shift(U[b], grid, a, 1, "zero"))
                if _wall(grid, b):
                    E[-1] = 0.0
                acc = acc + (E - _shift(E, grid, b, -1, "zero")) / h
        out.append(_mask_top(grid, a, acc))
    return out


def viscous(faces: Sequence[np.ndarray], mu: np.ndarray, grid: Grid) -> List[np.ndarray]:
    """div(mu (grad u + grad u^T)) on the faces of each axis a (second-order central).

    Normal stress 2 mu du_a/dx_a at the cell centres with the cell's mu; shear stress
    mu (du_a/dx_b + du_b/dx_a) on the edges with mu the mean of the four cells around the edge.
    On a box wall the tangential velocity has the no-slip image and du_b/dx_a = 0."""
    d = grid.ndim
    h = grid.h
    U = [_mask_top(grid, a, faces[a]) for a in range(d)]
    out = []
    for a in range(d):
        ua = U[a]
        tn = 2.0 * mu * (ua - _shift(ua, grid, a, -1, "zero")) / h
        acc = (_shift(tn, grid, a, 1, "reflect") - tn) / h
        for b in range(d):
            if b == a:
                continue
            ma = _shift(mu, grid, a, 1, "reflect")
            me = 0.25 * (mu + ma + _shift(mu, grid, b, 1, "reflect") + _shift(ma, grid, b, 1, "reflect"))
            dua = (_shift_odd(ua, grid, b, 1) - ua) / h if _wall(grid, b) else (_shift(ua, grid, b, 1, "reflect") - ua) / h
            dub = (_shift(U[b], grid, a, 1, "zero") - U[b]) / h
            tau = me * (dua + dub)
            if _wall(grid, b):
                # edge on the bottom wall (below row 0): no-slip image, u_b = 0 along the wall
                mb = 0.5 * (mu[0] + ma[0])
                below = mb * (ua[0] - (-ua[0])) / h
                prev = _shift(tau, grid, b, -1, "zero")
                prev[0] = below
            else:
                prev = _shift(tau, grid, b, -1, "zero")
            acc = acc + (tau - prev) / h
        out.append(_mask_top(grid, a, acc))
    return out


def capillary_force(phi: np.ndarray, C: np.ndarray, grid: Grid, kappa: float) -> List[np.ndarray]:
    """kappa phi grad C on the faces: phi averaged onto the face times the one-cell difference of C."""
    out = []
    for a in range(grid.ndim):
        f = kappa * face_mean(phi, grid, a) * (_shift(C, grid, a, 1, "reflect") - C) / grid.h
        out.append(_mask_top(grid, a, f))
    return out


def poisson_solve(R: np.ndarray, grid: Grid) -> np.ndarray:
    """Zero-mean p with lap_h p = R - mean(R), lap_h = div(face_gradient) (Neumann through the box
    walls), by the cosine transform along the bounded axis and Fourier transforms along the
    periodic ones (the route the paper names for Eq. PressurePoisson)."""
    d = grid.ndim
    lam = eigenvalues(grid)
    X = sfft.dct(R, type=2, axis=0, workers=WORKERS)
    X = sfft.rfft(X, axis=-1, workers=WORKERS)
    if d == 3:
        X = sfft.fft(X, axis=1, workers=WORKERS)
    nx = grid.n[0]
    lx = lam[0][: nx // 2 + 1]
    if d == 2:
        L = lam[1][:, None] + lx[None, :]
    else:
        L = lam[2][:, None, None] + lam[1][None, :, None] + lx[None, None, :]
    L = np.where(L == 0.0, np.inf, L)          # the mean mode (k = 0 on every axis) is dropped
    X = X / L
    if d == 3:
        X = sfft.ifft(X, axis=1, workers=WORKERS)
    X = sfft.irfft(X, n=nx, axis=-1, workers=WORKERS)
    return sfft.idct(X, type=2, axis=0, workers=WORKERS)


def prediction(faces, C, phi, params: Params, grid: Grid, N_prev):
    """u* of Eq. PredictionExp before penalisation; returns (u*, N^n).  N_prev None: first step."""
    d = grid.ndim
    rho = density(C, params)
    mu = viscosity(C, params)
    N = convective(faces, grid)
    Np = N if N_prev is None else N_prev
    V = viscous(faces, mu, grid)
    F = capillary_force(phi, C, grid, capillary_coefficient(params))
    g = list(params.body_force) + [0.0] * 3
    out = []
    for a in range(d):
        rf = face_mean(rho, grid, a)
        u = faces[a] + params.dt * (-(1.5 * N[a] - 0.5 * Np[a]) + (V[a] / params.Re + F[a]) / rf + g[a])
        out.append(_mask_top(grid, a, u))
    return out, N


def pressure_rhs(u2, C, p, p_prev, params: Params, grid: Grid) -> np.ndarray:
    """Right-hand side of Eq. PressurePoisson: div((1 - rho0/rho~) grad p^) + (rho0/dt) div u**."""
    rho0 = min(params.rho1, params.rho2)
    rho = density(C, params)
    ph = 2.0 * p - p_prev
    G = face_gradient(ph, grid)
    flux = [(1.0 - rho0 / face_mean(rho, grid, a)) * G[a] for a in range(grid.ndim)]
    return divergence(flux, grid) + (rho0 / params.dt) * divergence(u2, grid)


def correction(u2, C, p_new, p, p_prev, params: Params, grid: Grid):
    """Eq. correction: u^(n+1) = u** - dt [grad p^(n+1)/rho0 + (1/rho~ - 1/rho0) grad p^]."""
    rho0 = min(params.rho1, params.rho2)
    rho = density(C, params)
    ph = 2.0 * p - p_prev
    Gn = face_gradient(p_new, grid)
    Gh = face_gradient(ph, grid)
    out = []
    for a in range(grid.ndim):
        rf = face_mean(rho, grid, a)
        u = u2[a] - params.dt * (Gn[a] / rho0 + (1.0 / rf - 1.0 / rho0) * Gh[a])
        out.append(_mask_top(grid, a, u))
    return out
