"""Pins of the oracle's Cahn-Hilliard update (Appendix A.1) against closed forms,
brute-force linear algebra and invariants.  CPU only."""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import workloads as W
from oracle.geometry import build_tables
from oracle.solver import (OracleState, ParamError, advection, derived_coefficients,
                           laplacian, spectral_solve)


def _second_difference(N, h, periodic):
    main = -2.0 * np.ones(N)
    off = np.ones(N - 1)
    D = sp.diags([off, main, off], [-1, 0, 1], format="lil")
    if periodic:
        D[0, N - 1] = 1.0
        D[N - 1, 0] = 1.0
    else:  # reflecting box walls: f_-1 = f_0, f_N = f_(N-1)
        D[0, 0] = -1.0
        D[N - 1, N - 1] = -1.0
    return (D / (h * h)).tocsr()


def _assembled_laplacian(grid):
    """Kronecker sum of 1D second differences in the field layout (x fastest)."""
    n = grid.n
    h = grid.h
    mats = [_second_difference(n[a], h, a < grid.ndim - 1) for a in range(grid.ndim)]
    eye = [sp.identity(n[a], format="csr") for a in range(grid.ndim)]
    L = None
    for a in range(grid.ndim):
        # field flat index = sum_a i_a * prod_{b<a} n_b  -> kron order: last axis outermost
        factors = [mats[b] if b == a else eye[b] for b in reversed(range(grid.ndim))]
        M = factors[0]
        for f in factors[1:]:
            M = sp.kron(M, f, format="csr")
        L = M if L is None else L + M
    return L.tocsc()


@pytest.mark.parametrize("n", [(8, 4), (16, 8), (8, 8, 4), (4, 8, 8)])
def test_spectral_solve_matches_direct_sparse_solve(n):
    grid = W.Grid(n, tuple(0.0 for _ in n), tuple(v / 8.0 for v in n))
    prm = W.Params(Cn=0.05, Pe=10.0, dt=1e-3)
    S, al, a = derived_coefficients(prm)
    rng = np.random.default_rng(5)
    Q = rng.standard_normal(grid.shape)
    L = _assembled_laplacian(grid)
    I = sp.identity(L.shape[0], format="csc")
    G = spla.spsolve(L - a * I, Q.reshape(-1))
    C_ref = spla.spsolve(L + al * I, G).reshape(grid.shape)
    C = spectral_solve(Q, grid, al, a)
    assert np.max(np.abs(C - C_ref)) <= 1e-12 * np.max(np.abs(C_ref))


def test_laplacian_matches_assembled_operator():
    grid = W.Grid((16, 8, 4), (0.0, 0.0, 0.0), (2.0, 1.0, 0.5))
    rng = np.random.default_rng(3)
    f = rng.standard_normal(grid.shape)
    ref = (_assembled_laplacian(grid) @ f.reshape(-1)).reshape(grid.shape)
    assert np.max(np.abs(laplacian(f, grid) - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("kx,m", [(0, 0), (3, 0), (0, 5), (7, 2), (8, 15)])
def test_discrete_eigenmode(kx, m):
    """cos(2 pi kx i/Nx + phi) cos(pi m (j+1/2)/Ny) is an eigenvector of lap_h with the
    closed-form eigenvalue; the spectral solve divides it by (lam-a)(lam+alpha_s)."""
    grid = W.Grid((16, 16), (0.0, 0.0), (1.0, 1.0))
    h = grid.h
    i = np.arange(16)[None, :]
    j = np.arange(16)[:, None]
    mode = np.cos(2 * math.pi * kx * i / 16 + 0.3) * np.cos(math.pi * m * (j + 0.5) / 16)
    lam = -(4 / h ** 2) * (math.sin(math.pi * kx / 16) ** 2 + math.sin(math.pi * m / 32) ** 2)
    assert np.max(np.abs(laplacian(mode, grid) - lam * mode)) <= 1e-9 * (1 + abs(lam))
    prm = W.Params(Cn=0.05, Pe=10.0, dt=1e-3)
    _, al, a = derived_coefficients(prm)
    C = spectral_solve((lam - a) * (lam + al) * mode, grid, al, a)
    assert np.max(np.abs(C - mode)) <= 1e-12


@pytest.mark.parametrize("S_factor", [1.0, 1.3, 3.0])
def test_alpha_s_is_root_and_factorisation(S_factor):
    prm = W.Params(Cn=0.02, Pe=100.0, dt=1e-4)
    S_min = prm.Cn * math.sqrt(6 * prm.Pe / prm.dt)
    prm.S = S_factor * S_min
    S, al, a = derived_coefficients(prm)
    Cn2 = prm.Cn ** 2
    c0 = 3 * prm.Pe / (2 * Cn2 * prm.dt)
    assert abs(al * al + (S / Cn2) * al + c0) <= 1e-12 * c0
    for lam in (-1e5, -3.3e3, 0.0):
        assert abs((lam - a) * (lam + al) - (lam * lam - (S / Cn2) * lam + c0)) <= 1e-12 * (lam * lam + c0)


def test_stabilisation_bound_enforced():
    prm = W.Params(Cn=0.02, Pe=100.0, dt=1e-4, S=10.0)   # S_min is about 49
    with pytest.raises(ParamError):
        derived_coefficients(prm)
    prm.S = 0.0
    S, _, _ = derived_coefficients(prm)
    assert abs(S - 0.02 * math.sqrt(6e6)) < 1e-12


def test_uniform_advection_of_a_fourier_mode():
    """Central flux form with a uniform velocity: A = U sin(kh)/h cos(kx) exactly."""
    grid = W.Grid((32, 8), (0.0, 0.0), (1.0, 0.25))
    h = grid.h
    k = 2 * math.pi * 3
    x = (np.arange(32) + 0.5) * h
    C = np.tile(np.sin(k * x), (8, 1))
    U = 0.7
    faces = [np.full(grid.shape, U), np.zeros(grid.shape)]
    A = advection(C, faces, grid)
    ref = U * math.sin(k * h) / h * np.cos(k * x)[None, :]
    assert np.max(np.abs(A - ref)) <= 1e-12 * np.max(np.abs(ref))


def _wall_free_state(grid, prm, C0, faces=None):
    T = build_tables(grid, [], prm)
    return OracleState(grid, prm, T, C0, faces)


def test_single_mode_follows_closed_form_recurrence():
    """No wall, u = 0, amplitude 1e-6: the cubic term is negligible and each mode follows
    C^(n+1) = [(2C^n - C^(n-1)/2) Pe/(Cn^2 dt) + lam (-1 - S)(2C^n - C^(n-1))/Cn^2] / ((lam-a)(lam+alpha_s))."""
    grid = W.Grid((32, 16), (0.0, 0.0), (2.0, 1.0))
    prm = W.Params(Cn=0.05, Pe=50.0, dt=1e-3, velocity_fill=False)
    h = grid.h
    kx, m = 2, 3
    i = np.arange(32)[None, :]
    j = np.arange(16)[:, None]
    mode = np.cos(2 * math.pi * kx * i / 32) * np.cos(math.pi * m * (j + 0.5) / 16)
    lam = -(4 / h ** 2) * (math.sin(math.pi * kx / 32) ** 2 + math.sin(math.pi * m / 32) ** 2)
    st = _wall_free_state(grid, prm, 1e-6 * mode)
    S, al, a = st.S, st.alpha_s, st.a
    Cn2 = prm.Cn ** 2
    cn, cp = 1e-6, 1e-6
    for _ in range(10):
        st.step(1)
        nxt = ((2 * cn - 0.5 * cp) * prm.Pe / (Cn2 * prm.dt) + lam * (-1 - S) * (2 * cn - cp) / Cn2) \
            / ((lam - a) * (lam + al))
        cp, cn = cn, nxt
        assert np.max(np.abs(st.C - cn * mode)) <= 1e-9 * abs(cn)


def test_box_mass_is_conserved_without_wall():
    grid = W.Grid((32, 16), (0.0, 0.0), (2.0, 1.0))
    prm = W.Params(Cn=0.05, Pe=50.0, dt=1e-3, velocity_fill=False)
    rng = np.random.default_rng(9)
    C0 = 0.3 + 0.5 * rng.standard_normal(grid.shape)
    faces = [0.2 * rng.standard_normal(grid.shape) for _ in range(2)]
    st = _wall_free_state(grid, prm, C0, faces)
    m0 = st.C.sum()
    for _ in range(20):
        st.step(1)
        assert abs(st.C.sum() - m0) <= 1e-11 * np.abs(st.C).sum()


def test_free_energy_decays_without_wall():
    """Spinodal decomposition at rest: the discrete free energy never increases."""
    grid = W.Grid((64, 32), (0.0, 0.0), (2.0, 1.0))
    prm = W.Params(Cn=0.04, Pe=20.0, dt=1e-3, theta_deg=90.0, velocity_fill=False)
    rng = np.random.default_rng(4)
    C0 = 0.05 * rng.standard_normal(grid.shape)
    st = _wall_free_state(grid, prm, C0)
    F = [st.diagnostics()["free_energy"]]
    for _ in range(60):
        st.step(1)
        F.append(st.diagnostics()["free_energy"])
    F = np.array(F)
    assert np.all(np.diff(F) <= 1e-12 * np.abs(F[:-1]))
    assert F[-1] < (1.0 - 1e-3) * F[0]
