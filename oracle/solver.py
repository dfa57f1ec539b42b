"""Oracle time step: S-stabilised semi-implicit Cahn-Hilliard update plus ghost-cell fills.

Non-dimensional form used throughout (lengths in domain units, eps = Cn,
lambda*M = Cn^2/Pe, psi'(C) = C^3 - C):

    dC/dt + div(u C) = (1/Pe) lap(C^3 - C - Cn^2 lap C)

Time step (Appendix A.1, Eqs. Helmholtz1 and Helmholtz2, with psi read as psi'
in the right-hand side, which is the only reading that reproduces the printed
alpha_s and the bound on S):

    C~ = 2C^n - C^(n-1),  C^ = 2C^n - C^(n-1)/2
    Q  = (Pe/Cn^2) (C^/dt - div_h(u C~)) + lap_h(g),  g = (C~^3 - C~ - S C~)/Cn^2
    (lap_h - a)(lap_h + alpha_s) C* = Q,   a = alpha_s + S/Cn^2

with the wall condition dphi/dn = 0 carried by g at the ghost cells (see rhs)

solved with a cosine transform along the bounded (last) axis (Neumann box
walls) and Fourier transforms along the periodic axes (end of Appendix A.1).
The second-order discrete Laplacian is the one diagonalised by those
transforms.  Then the ghost values of C are overwritten from the contact-angle
condition (section 4.2.2, Eqs. interpolationAtWall ... UpdateC) and the
velocity at faces touching ghosts from the no-penetration and Navier-slip
conditions (section 4.3, Eqs. NoPenetration ... UpdateVandW).
"""
from __future__ import annotations

import math
import os
from typing import List, Optional

import numpy as np
import scipy.fft as sfft

from workloads import Grid, Params

from .geometry import GhostTables

SQRT2 = math.sqrt(2.0)
WORKERS = os.cpu_count() or 1


class ParamError(ValueError):
    pass


def derived_coefficients(params: Params):
    """Stabilisation S, alpha_s and a of the two Helmholtz factors (Appendix A.1).

    S >= eps^2 sqrt(6/(lambda M dt)) = Cn sqrt(6 Pe/dt);
    alpha_s = -(S/(2 Cn^2)) (1 + sqrt(1 - 6 Cn^2 Pe/(dt S^2))) (argument clamped at 0);
    a = alpha_s + S/Cn^2.
    """
    Cn, Pe, dt = params.Cn, params.Pe, params.dt
    S_min = Cn * math.sqrt(6.0 * Pe / dt)
    S = params.S if params.S > 0.0 else S_min
    disc = 1.0 - 6.0 * Cn * Cn * Pe / (dt * S * S)
    if disc < -1e-12:
        raise ParamError(f"S={S} is below the stability bound {S_min}")
    disc = max(disc, 0.0)
    alpha_s = -(S / (2.0 * Cn * Cn)) * (1.0 + math.sqrt(disc))
    a = alpha_s + S / (Cn * Cn)
    return S, alpha_s, a


def eigenvalues(grid: Grid):
    """Eigenvalues of the 1D second-difference operator per axis (x first).

    Periodic axes: -(4/h^2) sin^2(pi k / N), k = 0..N-1.
    Bounded axis with reflecting (Neumann) box walls: -(4/h^2) sin^2(pi k / (2N)).
    """
    h = grid.h
    out = []
    for a in range(grid.ndim):
        N = grid.n[a]
        k = np.arange(N, dtype=np.float64)
        if a < grid.ndim - 1:
            s = np.sin(math.pi * k / N)
        else:
            s = np.sin(math.pi * k / (2.0 * N))
        out.append(-(4.0 / (h * h)) * s * s)
    return out


def spectral_solve(Q: np.ndarray, grid: Grid, alpha_s: float, a: float) -> np.ndarray:
    """Solve (lap_h - a)(lap_h + alpha_s) C = Q on the whole box (Appendix A.1).

    Type-II cosine transform along the bounded axis, real/complex Fourier
    transforms along the periodic axes, a pointwise division by
    (lambda - a)(lambda + alpha_s), and the inverse transforms.
    """
    d = grid.ndim
    lam = eigenvalues(grid)
    X = sfft.dct(Q, type=2, axis=0, workers=WORKERS)
    X = sfft.rfft(X, axis=-1, workers=WORKERS)
    if d == 3:
        X = sfft.fft(X, axis=1, workers=WORKERS)
    nx = grid.n[0]
    lx = lam[0][: nx // 2 + 1]
    if d == 2:
        L = lam[1][:, None] + lx[None, :]
    else:
        L = lam[2][:, None, None] + lam[1][None, :, None] + lx[None, None, :]
    X = X / ((L - a) * (L + alpha_s))
    if d == 3:
        X = sfft.ifft(X, axis=1, workers=WORKERS)
    X = sfft.irfft(X, n=nx, axis=-1, workers=WORKERS)
    return sfft.idct(X, type=2, axis=0, workers=WORKERS)


# ---------------------------------------------------------------------------
# Stencil helpers.  Field arrays have numpy shape reversed(grid.n): grid axis a
# is numpy axis ndim-1-a.  The last grid axis (numpy axis 0) is bounded.

def _shift(f: np.ndarray, grid: Grid, a: int, s: int, mode: str) -> np.ndarray:
    """g[c] = f[c + s e_a]; periodic wrap on periodic axes; on the bounded axis
    out-of-box values are reflected (mode 'reflect') or zero (mode 'zero')."""
    ax = grid.ndim - 1 - a
    if a < grid.ndim - 1:
        return np.roll(f, -s, axis=ax)
    out = np.empty_like(f)
    n = f.shape[ax]
    src = [slice(None)] * f.ndim
    dst = [slice(None)] * f.ndim
    if s == 1:
        dst[ax] = slice(0, n - 1)
        src[ax] = slice(1, n)
        out[tuple(dst)] = f[tuple(src)]
        edge = [slice(None)] * f.ndim
        edge[ax] = slice(n - 1, n)
        out[tuple(edge)] = f[tuple(edge)] if mode == "reflect" else 0.0
    else:
        dst[ax] = slice(1, n)
        src[ax] = slice(0, n - 1)
        out[tuple(dst)] = f[tuple(src)]
        edge = [slice(None)] * f.ndim
        edge[ax] = slice(0, 1)
        out[tuple(edge)] = f[tuple(edge)] if mode == "reflect" else 0.0
    return out


def laplacian(f: np.ndarray, grid: Grid) -> np.ndarray:
    """Second-order 5/7-point Laplacian; periodic axes wrap, box walls reflect (g_-1 = g_0)."""
    acc = np.zeros_like(f)
    for a in range(grid.ndim):
        acc = acc + _shift(f, grid, a, 1, "reflect") + _shift(f, grid, a, -1, "reflect")
    return (acc - 2.0 * grid.ndim * f) / (grid.h * grid.h)


def _box_face_mask(grid: Grid, a: int, f: np.ndarray) -> np.ndarray:
    """Face array with the bounded axis' top box-wall face forced to zero."""
    if a < grid.ndim - 1:
        return f
    g = f.copy()
    g[-1] = 0.0
    return g


def advection(Ct: np.ndarray, faces: List[np.ndarray], grid: Grid) -> np.ndarray:
    """Conservative central advection div_h(u C~) on the staggered grid.

    Face flux F_(c+e_a/2) = u_a (C~_c + C~_(c+e_a)) / 2; the face velocity normal
    to a box wall is zero (no penetration).
    """
    A = np.zeros_like(Ct)
    for a in range(grid.ndim):
        u = _box_face_mask(grid, a, faces[a])
        F = u * (Ct + _shift(Ct, grid, a, 1, "reflect")) * 0.5
        A = A + (F - _shift(F, grid, a, -1, "zero"))
    return A / grid.h


def centred_velocity(faces: List[np.ndarray], grid: Grid) -> List[np.ndarray]:
    """Cell-centred velocity: mean of the two faces of the cell along each axis."""
    out = []
    for a in range(grid.ndim):
        u = _box_face_mask(grid, a, faces[a])
        out.append(0.5 * (_shift(u, grid, a, -1, "zero") + u))
    return out


def _unravel(grid: Grid, lin: np.ndarray) -> List[np.ndarray]:
    out = []
    rem = lin.copy()
    for a in range(grid.ndim):
        out.append(rem % grid.n[a])
        rem = rem // grid.n[a]
    return out


def _ravel(grid: Grid, cells: List[np.ndarray]) -> np.ndarray:
    lin = np.zeros_like(cells[0])
    stride = 1
    for a in range(grid.ndim):
        lin = lin + cells[a] * stride
        stride *= grid.n[a]
    return lin


def gradient_at(f_flat: np.ndarray, grid: Grid, lin: np.ndarray) -> np.ndarray:
    """Central-difference gradient of a cell field at the given linear indices.

    Periodic wrap along periodic axes; reflection (f_-1 = f_0, f_N = f_(N-1))
    at the box walls of the bounded axis.  Returns shape (d,) + lin.shape.
    """
    cells = _unravel(grid, lin)
    out = []
    for a in range(grid.ndim):
        N = grid.n[a]
        cp = list(cells)
        cm = list(cells)
        if a < grid.ndim - 1:
            cp[a] = (cells[a] + 1) % N
            cm[a] = (cells[a] - 1) % N
        else:
            cp[a] = np.minimum(cells[a] + 1, N - 1)
            cm[a] = np.maximum(cells[a] - 1, 0)
        out.append((f_flat[_ravel(grid, cp)] - f_flat[_ravel(grid, cm)]) / (2.0 * grid.h))
    return np.stack(out)


def _idw(values_flat: np.ndarray, T: GhostTables, j: int) -> np.ndarray:
    """Inverse-distance-weighted value at interpolation point j (Eq. 'weright averaged')."""
    return (T.w[j] * values_flat[T.ap[j]]).sum(axis=0)


def mirror_value(values_flat: np.ndarray, T: GhostTables) -> np.ndarray:
    """Mirror value by linear extrapolation Omega_M = 2 Omega_IP1 - Omega_IP2 (Eq. extrapolation)."""
    return 2.0 * _idw(values_flat, T, 0) - _idw(values_flat, T, 1)


def _mirror_grad(f_flat: np.ndarray, grid: Grid, T: GhostTables) -> np.ndarray:
    gm = np.zeros((grid.ndim, T.n_ghost))
    for j, coef in ((0, 2.0), (1, -1.0)):
        g = gradient_at(f_flat, grid, T.ap[j])          # (d, K, G)
        gm = gm + coef * (T.w[j][None] * g).sum(axis=1)
    return gm


def _mirror_centred_velocity(uc: List[np.ndarray], T: GhostTables) -> np.ndarray:
    return np.stack([mirror_value(u.reshape(-1), T) for u in uc])


class OracleState:
    """Order parameter, face velocities and per-ghost state of one run (FP64, host)."""

    def __init__(self, grid: Grid, params: Params, tables: GhostTables,
                 C0: np.ndarray, faces: Optional[List[np.ndarray]] = None,
                 face_alpha: Optional[List[np.ndarray]] = None):
        self.grid = grid
        self.params = params
        self.T = tables
        self.S, self.alpha_s, self.a = derived_coefficients(params)
        self.cos_theta = math.cos(math.radians(params.theta_deg))
        self.C = np.array(C0, dtype=np.float64, copy=True)
        self.faces = [np.zeros(grid.shape) for _ in range(grid.ndim)] if faces is None else \
            [np.array(f, dtype=np.float64, copy=True) for f in faces]
        self.CI = np.zeros(tables.n_ghost)
        self.step_count = 0
        self.Rh = None          # rate of the previous explicit step
        if params.navier_stokes:
            if face_alpha is None:
                raise ParamError("the momentum step needs the staggered-cell volume fractions")
            self.face_alpha = [np.array(f, dtype=np.float64) for f in face_alpha]
            self.Nh = None      # convective term of the previous momentum step
            self.p = np.zeros(grid.shape)
            self.p_prev = np.zeros(grid.shape)
        self.initial_fill()
        self.Cp = self.C.copy()
        self.u_prev = [f.copy() for f in self.faces]

    # -- ghost fill of C -------------------------------------------------------
    def fill_C(self, P: np.ndarray, initial: bool) -> np.ndarray:
        """Ghost values of C from the contact-angle condition (section 4.2.2).

        P is the provisional field: the Helmholtz solution off the ghosts and
        C^_G = 2C^n_G - C^(n-1)_G at the ghosts (Eq. interpolationAtWall).  All
        reads come from P (Jacobi sweep), so the result is order independent.
        Static condition (no contact-line friction, mu_f = 0): Eq. WallBCS loses
        its time derivative and reads (3/(2 sqrt2)) Cn dC/dn + cos(theta) g'(C) = 0,
        g'(C) = 3(1 - C^2)/4, i.e. dC/dn = -cos(theta)(1 - C^2)/(sqrt2 Cn) with n
        pointing into the fluid.  That relation also holds at every point of the
        normal through a straight interface meeting the wall at theta (the
        equilibrium tanh profile), so it is integrated exactly from M back to I:
        artanh C_I = artanh C_M + b, b = d1 cos(theta)/(sqrt2 Cn) = gamma dn cos(theta)/(sqrt2 Cn),
        i.e. C_I = (C_M + t)/(1 + t C_M), t = tanh b, with C_M taken inside [-1, 1]
        (continued smoothly beyond +-1 the map has slope e^(2b) there and the ghost
        feedback diverges at these resolutions; the clip keeps it bounded).  C_G then
        follows from Eq. UpdateC.  (The one-sided slope over d1 with g'
        at C_I or at C_M instead has spurious wall-film steady states and, for
        wetting angles below about 60 degrees at Cn/h ~ 1.3, growing near-wall
        modes.)
        Dynamic condition: C_I advanced by one forward step of
        DC/Dt = Vs [Cn dC/dn + cos(theta)(1 - C_I^2)/sqrt2] (Eq. WallBCS_recast),
        then C_G = ((gamma+1) C_I - C_M)/gamma (Eq. UpdateC).
        """
        T = self.T
        prm = self.params
        Pf = P.reshape(-1)
        PG = Pf[T.gidx]
        gam = T.gamma
        CM = mirror_value(Pf, T)
        CIs = (gam * PG + CM) / (gam + 1.0)
        if prm.Vs <= 0.0:
            t = np.tanh(gam * T.dn * self.cos_theta / (SQRT2 * prm.Cn))
            Mc = np.clip(CM, -1.0, 1.0)
            CI = (Mc + t) / (1.0 + t * Mc)
            return ((gam + 1.0) * CI - CM) / gam
        if initial:
            self.CI = CIs.copy()
            return PG.copy()
        grid = self.grid
        gG = gradient_at(Pf, grid, T.gidx)
        gM = _mirror_grad(Pf, grid, T)
        gI = (gam * gG + gM) / (gam + 1.0)
        gt = gI - (gI * T.normal).sum(axis=0) * T.normal
        uc = centred_velocity(self.faces, grid)
        uG = np.stack([u.reshape(-1)[T.gidx] for u in uc])
        uM = _mirror_centred_velocity(uc, T)
        uI = (gam * uG + uM) / (gam + 1.0)
        dCdn = (CM - PG) / ((1.0 + gam) * T.dn)
        rhs = -(uI * gt).sum(axis=0) + prm.Vs * (prm.Cn * dCdn + self.cos_theta * (1.0 - CIs * CIs) / SQRT2)
        self.CI = self.CI + prm.dt * rhs
        return ((gam + 1.0) * self.CI - CM) / gam

    # -- velocity fill -------------------------------------------------------------
    def fill_velocity(self, Cfin: np.ndarray) -> None:
        """No-penetration and Navier-slip ghost velocities, then faces touching ghosts (section 4.3).

        V_nG = -V_nM/gamma (Eq. NoPenetration);
        V_tG = V_tM (ls - dn)/(ls + gamma dn) - Kc grad_t C_I ls (gamma+1) dn / (mu (ls + gamma dn))
        (Eq. UpdateVtan), Kc = [(3/(2 sqrt2)) Cn dC/dn + cos(theta) g'(C_I)]/Ca for the
        dynamic condition; with mu_f = 0 the wall equation itself sets that bracket
        to zero, so Kc = 0 for the static condition; the ghost velocity is V_nG n + V_tG (vector form of Eq. UpdateVandW, with the
        back-transform sign read so that it inverts Eq. CoordinateTransformation).
        Every face with a ghost on either side becomes the mean of its two
        cell-centred values, taken from the faces as they were before this fill.
        """
        grid = self.grid
        T = self.T
        prm = self.params
        gam, dn, n = T.gamma, T.dn, T.normal
        uc = centred_velocity(self.faces, grid)
        uM = _mirror_centred_velocity(uc, T)
        VnM = (uM * n).sum(axis=0)
        VtM = uM - VnM * n
        VnG = -VnM / gam
        Cf = Cfin.reshape(-1)
        CG = Cf[T.gidx]
        CM = mirror_value(Cf, T)
        CI = (gam * CG + CM) / (gam + 1.0)
        dCdn = (CM - CG) / ((1.0 + gam) * dn)
        gG = gradient_at(Cf, grid, T.gidx)
        gM = _mirror_grad(Cf, grid, T)
        gI = (gam * gG + gM) / (gam + 1.0)
        gt = gI - (gI * n).sum(axis=0) * n
        if prm.Vs <= 0.0:
            Kc = np.zeros_like(CI)
        else:
            Kc = ((3.0 / (2.0 * SQRT2)) * prm.Cn * dCdn + 0.75 * self.cos_theta * (1.0 - CI * CI)) / prm.Ca
        ls = prm.slip_length
        VtG = VtM * ((ls - dn) / (ls + gam * dn)) - Kc * gt * (ls * (gam + 1.0) * dn / (prm.mu * (ls + gam * dn)))
        uG = VnG * n + VtG
        self.last_uG = uG
        ghost = np.zeros(grid.cells, dtype=bool)
        ghost[T.gidx] = True
        ghost = ghost.reshape(grid.shape)
        new_faces = []
        for a in range(grid.ndim):
            ua = uc[a].reshape(-1).copy()
            ua[T.gidx] = uG[a]
            ua = ua.reshape(grid.shape)
            touch = ghost | _shift(ghost, grid, a, 1, "zero").astype(bool)
            if a == grid.ndim - 1:
                touch[-1] = False
            mean = 0.5 * (ua + _shift(ua, grid, a, 1, "zero"))
            new_faces.append(np.where(touch, mean, self.faces[a]))
        self.faces = new_faces

    def initial_fill(self) -> None:
        """Fill the ghosts of the initial field (provisional field = C0), then the velocity."""
        P = self.C.copy()
        CG = self.fill_C(P, initial=True)
        Pf = P.reshape(-1)
        Pf[self.T.gidx] = CG
        self.C = P
        if self.params.velocity_fill or self.params.navier_stokes:
            self.fill_velocity(self.C)

    def rhs(self) -> np.ndarray:
        """Right-hand side Q of the first Helmholtz equation (Eq. Helmholtz1, psi -> psi'),
        with the wall condition dphi/dn = 0 imposed at the ghosts.

        The stabilised step's chemical potential is the explicit part
        phi~ = psi'(C~) - Cn^2 lap_h C~ plus the implicit correction
        (S - Cn^2 lap_h)(C^(n+1) - C~), which vanishes as dt -> 0.  Dividing by Cn^2,
        g = (psi'(C~) - S C~)/Cn^2 is phi~/Cn^2 + (lap_h - S/Cn^2) C~, and the second term
        cancels against the implicit operator.  The end of section 4.2.2 imposes
        dphi/dn = 0 at the ghosts by the mirror value, "in a similar way" as for C; in the
        semi-implicit step that is done on phi~, the part the right-hand side carries:
        g_G <- g_G + (phi~_M - phi~_G)/Cn^2.  phi~ at the averaging points of M uses the
        filled ghost values of C^n and C^(n-1) (Eq. interpolationAtWall's C^_G).  The
        correction term is left to the whole-box solve.
        """
        prm = self.params
        grid = self.grid
        Cn2 = prm.Cn * prm.Cn
        Ct = 2.0 * self.C - self.Cp
        Cc = 2.0 * self.C - 0.5 * self.Cp
        # with the momentum step the advecting velocity is the extrapolation 2u^n - u^(n-1)
        # (Appendix A.1, u~^(n+1)); with frozen faces both are the same field
        uadv = [2.0 * u - up for u, up in zip(self.faces, self.u_prev)] if prm.navier_stokes else self.faces
        A = advection(Ct, uadv, grid)
        g = (Ct * Ct * Ct - Ct - self.S * Ct) / Cn2
        if self.T.n_ghost:
            phit = (Ct * Ct * Ct - Ct - Cn2 * laplacian(Ct, grid)).reshape(-1)
            gf = g.reshape(-1)
            gf[self.T.gidx] += (mirror_value(phit, self.T) - phit[self.T.gidx]) / Cn2
        return (prm.Pe / Cn2) * (Cc / prm.dt - A) + laplacian(g, grid)

    def provisional(self) -> np.ndarray:
        """Helmholtz solution C* of this step on every cell, before any ghost overwrite."""
        return spectral_solve(self.rhs(), self.grid, self.alpha_s, self.a)

    def explicit_rate(self) -> np.ndarray:
        """Rate R^n of the explicit scheme (Eq. ExpCH, non-dimensional).

        dC/dt = -div(u C) + (1/Pe) lap(phi) with phi the chemical potential of
        Eq. Chemical-Potential (ghosts take the mirror value, dphi/dn = 0, as at the end
        of section 4.2.2).  The advection is the conservative central form of the
        semi-implicit path (equal to u . grad C for the divergence-free flows the paper
        considers) evaluated on C^n; the mobility term is the paper's
        (3/(2 sqrt2)) div(M grad phi) in the units of the non-dimensional equation.
        """
        prm = self.params
        phi = chemical_potential(self.C, self.grid, self.T, prm.Cn)
        return -advection(self.C, self.faces, self.grid) + laplacian(phi, self.grid) / prm.Pe

    def explicit_provisional(self) -> np.ndarray:
        """C^(n+1) = C^n + dt (3/2 R^n - 1/2 R^(n-1)) on every cell (second-order
        Adams-Bashforth); the first step has no R^(n-1) and is a forward Euler step.
        Records R^n for the next step."""
        R = self.explicit_rate()
        Rp = R if self.Rh is None else self.Rh
        self.Rh = R
        return self.C + self.params.dt * (1.5 * R - 0.5 * Rp)

    def step(self, nsteps: int = 1) -> None:
        for _ in range(nsteps):
            P = self.explicit_provisional() if self.params.explicit else self.provisional()
            Pf = P.reshape(-1)
            Pf[self.T.gidx] = 2.0 * self.C.reshape(-1)[self.T.gidx] - self.Cp.reshape(-1)[self.T.gidx]
            CG = self.fill_C(P, initial=False)
            Pf[self.T.gidx] = CG
            self.Cp = self.C
            self.C = P
            if self.params.navier_stokes:
                self.momentum_step()
            elif self.params.velocity_fill:
                self.fill_velocity(self.C)
            self.step_count += 1

    # -- momentum ---------------------------------------------------------------------
    def momentum_step(self) -> None:
        """Prediction, penalisation, velocity ghost fill, pressure and correction with the new C
        (sections 4.2.3, 4.3 and 4.4; the operators are in ``oracle.ns``)."""
        from . import ns
        grid = self.grid
        prm = self.params
        phi = chemical_potential(self.C, grid, self.T, prm.Cn)
        us, self.Nh = ns.prediction(self.faces, self.C, phi, prm, grid, self.Nh)
        u_old = self.faces
        self.faces = [self.face_alpha[a] * us[a] for a in range(grid.ndim)]
        self.fill_velocity(self.C)
        u2 = self.faces
        R = ns.pressure_rhs(u2, self.C, self.p, self.p_prev, prm, grid)
        pn = ns.poisson_solve(R, grid)
        self.faces = ns.correction(u2, self.C, pn, self.p, self.p_prev, prm, grid)
        self.u_prev = u_old
        self.p_prev = self.p
        self.p = pn

    # -- diagnostics ------------------------------------------------------------------
    def diagnostics(self) -> dict:
        return diagnostics(self.grid, self.params, self.T.alpha, self.C)


def fill_scalar(f: np.ndarray, T: GhostTables, a: float, b: float, g) -> np.ndarray:
    """Ghost values of any scalar field from the mixed condition a f + b df/dn = g at the wall.

    The ghost-cell procedure of section 4.2.2 applied to a general boundary condition (the
    abstract and the conclusions note that it imposes Dirichlet, Neumann or mixed conditions on
    any field).  With the wall value and the normal derivative taken from the ghost G and the
    mirror point M as in Eq. interpolationAtWall and Eq. ProjectingToNT,
        f_I = (gamma f_G + f_M) / (gamma + 1),   (df/dn)_I = (f_M - f_G) / ((1 + gamma) dn),
    the condition is linear in f_G:
        f_G = ((gamma + 1) g - f_M (a + b/dn)) / (a gamma - b/dn).
    b = 0 is Dirichlet (f_G = ((gamma+1) g - f_M)/gamma, Eq. UpdateC with f_I = g); a = 0 is
    Neumann (f_G = f_M - (gamma+1) dn g; g = 0 gives the mirror value used for phi).  g is a
    scalar or one value per ghost.  Returns a copy of f with the ghosts replaced.
    """
    out = np.array(f, dtype=np.float64, copy=True)
    of = out.reshape(-1)
    fM = mirror_value(np.asarray(f, dtype=np.float64).reshape(-1), T)
    gam, dn = T.gamma, T.dn
    g = np.broadcast_to(np.asarray(g, dtype=np.float64), fM.shape)
    of[T.gidx] = ((gam + 1.0) * g - fM * (a + b / dn)) / (a * gam - b / dn)
    return out


def chemical_potential(C: np.ndarray, grid: Grid, T: GhostTables, Cn: float) -> np.ndarray:
    """phi = C^3 - C - Cn^2 lap_h C on all cells; at ghosts the mirror value (dphi/dn = 0).

    Non-dimensional Eq. Chemical-Potential (phi in units of sigma/eps); the
    ghost treatment is the 'similar way' of the end of section 4.2.2.
    """
    phi = C * C * C - C - Cn * Cn * laplacian(C, grid)
    pf = phi.reshape(-1)
    pf[T.gidx] = mirror_value(pf.copy(), T)
    return phi


def diagnostics(grid: Grid, params: Params, alpha: np.ndarray, C: np.ndarray) -> dict:
    """Mass of the box and of the fluid, free energy and max |C|.

    Free energy (Eqs. FreeEnergy and FreeEnergySolid, non-dimensional, wall term
    as a diffuse surface integral):
      F = h^d sum alpha [ (C^2-1)^2/(4 Cn) + (Cn/2) sum_a (forward difference_a C / h)^2 ]
          - (2 sqrt2/3) cos(theta) h^d sum |grad_h alpha| g(C),   g(C) = (2 + 3C - C^3)/4
    The forward differences are those of the second-order Laplacian (periodic
    wrap; none across a box wall); |grad_h alpha| uses central differences.
    """
    h = grid.h
    vol = h ** grid.ndim
    Cn = params.Cn
    bulk = (C * C - 1.0) ** 2 / (4.0 * Cn)
    grad2 = np.zeros_like(C)
    for a in range(grid.ndim):
        df = (_shift(C, grid, a, 1, "reflect") - C) / h
        grad2 = grad2 + df * df
    F_int = vol * np.sum(alpha * (bulk + 0.5 * Cn * grad2))
    ga2 = np.zeros_like(C)
    for a in range(grid.ndim):
        dg = (_shift(alpha, grid, a, 1, "reflect") - _shift(alpha, grid, a, -1, "reflect")) / (2.0 * h)
        ga2 = ga2 + dg * dg
    gC = (2.0 + 3.0 * C - C * C * C) / 4.0
    cos_t = math.cos(math.radians(params.theta_deg))
    F_wall = -(2.0 * SQRT2 / 3.0) * cos_t * vol * np.sum(np.sqrt(ga2) * gC)
    return {
        "mass_box": float(vol * np.sum(C)),
        "mass_fluid": float(vol * np.sum(alpha * C)),
        "free_energy": float(F_int + F_wall),
        "max_abs_C": float(np.max(np.abs(C))),
    }
