"""Pins of the oracle's ghost-cell fills (sections 4.2.2 and 4.3) and of the mass identity.

CPU only.  The pins are special cases with known answers (constant and linear
fields, pure phases, the exact tanh wedge that satisfies the continuous
contact-angle condition, the wall balance reached by the dynamic condition, the
no-slip and free-slip
limits of the Navier condition) and the discrete mass identity of the
semi-implicit step.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle.geometry import build_tables
from oracle.solver import OracleState, centred_velocity, mirror_value

SQ2 = math.sqrt(2.0)


def _state(case, C0=None, faces=None):
    T = build_tables(case.grid, case.shapes, case.params)
    if C0 is None:
        C0, f = case.initial_fields()
        faces = f if faces is None else faces
    return OracleState(case.grid, case.params, T, C0, faces), T


@pytest.mark.parametrize("kind", ["flat", "sin", "circle"])
def test_constant_field(kind):
    case = W.small_case(64, 32, kind=kind, theta_deg=90.0)
    st, T = _state(case, C0=np.full(case.grid.shape, 0.37))
    P = np.full(case.grid.shape, 0.37)
    assert np.max(np.abs(mirror_value(P.reshape(-1), T) - 0.37)) <= 1e-15
    CG = st.fill_C(P, initial=False)
    assert np.max(np.abs(CG - 0.37)) <= 1e-12          # 90 degrees: cos(theta) ~ 6e-17


def test_linear_field_mirror_value_exact_for_on_centre_interpolation_points():
    g = W.Grid((32, 16), (0.0, 0.0), (2.0, 1.0))
    h = g.h
    prm = W.Params(Cn=0.05, Pe=10.0, d1_cells=1.5, d2_cells=1.0)
    T = build_tables(g, [W.Shape(W.HALFPLANE, (0.0, 4 * h, 0.0, 0.0, 1.0, 0.0))], prm)
    y = (np.arange(16) + 0.5) * h
    x = (np.arange(32) + 0.5) * h
    P = 0.3 + 1.7 * y[:, None] - 0.4 * x[None, :]
    CM = mirror_value(P.reshape(-1), T)
    Mx, My = T.points["M"]
    assert np.max(np.abs(CM - (0.3 + 1.7 * My - 0.4 * Mx))) <= 1e-14


@pytest.mark.parametrize("theta", [30.0, 90.0, 150.0])
@pytest.mark.parametrize("value", [-1.0, 1.0])
def test_bulk_phases_stay_bulk_at_the_wall(theta, value):
    """A wall in a pure phase keeps it: no wetting film forms at any angle."""
    case = W.small_case(64, 32, kind="sin", theta_deg=theta)
    st, T = _state(case)
    CG = st.fill_C(np.full(case.grid.shape, value), initial=False)
    assert np.max(np.abs(CG - value)) <= 1e-14


def _wedge(p, p0, n, theta, Cn):
    """tanh profile of a straight interface through p0 meeting the wall (normal n) at theta."""
    t = np.array([n[1], -n[0]])
    q = p - p0[:, None]
    s = (t @ q) * math.sin(theta) - (n @ q) * math.cos(theta)
    return np.tanh(s / (SQ2 * Cn))


@pytest.mark.parametrize("kind,theta", [("flat", 60.0), ("flat", 150.0), ("tilted", 30.0), ("tilted", 120.0)])
def test_static_fill_reproduces_the_tanh_wedge_from_its_mirror_value(kind, theta):
    """Along the normal of a straight interface meeting the wall at theta, the equilibrium
    profile tanh(s/(sqrt2 Cn)) satisfies the static wall relation at every point.  Given the
    wedge's exact value at the mirror point (every averaging point set to it), the filled ghost
    puts the wedge's exact value at the intersect point.  Each ghost's wedge is taken against
    the plane through the contact point with that ghost's own normal (on the tilted wall the
    normals come from the volume fractions and differ slightly from the exact one)."""
    case = W.small_case(64, 32, kind=kind, theta_deg=theta)
    st, T = _state(case)
    shp = case.shapes[0].p
    p0 = np.array([1.0 if kind == "tilted" else 0.83, shp[1]])
    th = math.radians(theta)
    Cn = case.params.Cn
    g = T.gamma
    checked = 0
    for k in range(T.gidx.size):
        nk = T.normal[:, k]
        CMk = _wedge(T.points["M"][:, k:k + 1], p0, nk, th, Cn)[0]
        CIx = _wedge(T.points["I"][:, k:k + 1], p0, nk, th, Cn)[0]
        if abs(CMk) > 0.999:
            continue
        CG = st.fill_C(np.full(case.grid.shape, CMk), initial=False)[k]
        CI = (g[k] * CG + CMk) / (g[k] + 1)
        assert abs(CI - CIx) <= 1e-12, (k, CI, CIx)
        checked += 1
    assert checked >= 3


@pytest.mark.parametrize("theta", [50.0, 120.0])
def test_tanh_wedge_is_reproduced_under_refinement(theta):
    """C = tanh(s/(sqrt2 Cn)), s = (x - xc) sin(theta) - (y - yw) cos(theta), meets a flat wall at
    angle theta and satisfies the continuous static condition; the ghost values converge to it."""
    errs = []
    Cn = 0.06
    th = math.radians(theta)
    for n in (32, 64, 128):
        g = W.Grid((2 * n, n), (0.0, 0.0), (2.0, 1.0))
        h = g.h
        yw = (int(0.3 * n) + 0.37) * h          # same wall position relative to the cells
        prm = W.Params(Cn=Cn, Pe=10.0, theta_deg=theta, velocity_fill=False)
        T = build_tables(g, [W.Shape(W.HALFPLANE, (0.0, yw, 0.0, 0.0, 1.0, 0.0))], prm)
        x = (np.arange(2 * n) + 0.5) * h
        y = (np.arange(n) + 0.5) * h
        s = (x[None, :] - 1.0) * math.sin(th) - (y[:, None] - yw) * math.cos(th)
        Cex = np.tanh(s / (SQ2 * Cn))
        st = OracleState(g, prm, T, Cex)
        CG = st.fill_C(Cex.copy(), initial=False)
        near = np.abs(T.points["G"][0] - 1.0) < 4 * Cn
        errs.append(np.max(np.abs(CG - Cex.reshape(-1)[T.gidx])[near]))
    assert errs[1] < 0.75 * errs[0] and errs[2] < 0.75 * errs[1]
    assert errs[2] < 0.05


def test_dynamic_condition_relaxes_to_the_wall_balance():
    """With the fluid frozen, repeated dynamic updates converge to ghost values at which the
    wall equation holds with zero time derivative, g' taken at C_I (Eq. WallBCS_recast).

    The frozen-fluid iteration contracts when the diffusive part Cn/d1 of the linearised wall
    equation outweighs the wetting part sqrt2 cos(theta) |C_I|; d1 = 1.5 cells keeps this case
    in that regime."""
    case = W.small_case(64, 32, kind="sin", theta_deg=60.0, Vs=2000.0)   # Vs dt = 0.2
    case.params.d1_cells = 1.5
    st, T = _state(case)
    st.faces = [np.zeros(case.grid.shape) for _ in range(2)]   # no wall advection term
    P = st.C.copy()
    Pf = P.reshape(-1)
    CG_prev = Pf[T.gidx].copy()
    CG = CG_prev.copy()
    for _ in range(400):
        Pf[T.gidx] = 2 * CG - CG_prev
        new = st.fill_C(P, initial=False)
        CG_prev, CG = CG, new
    Pf[T.gidx] = CG
    CM = mirror_value(Pf, T)
    g = T.gamma
    CI = (g * CG + CM) / (g + 1)
    dCdn = (CM - CG) / ((1 + g) * T.dn)
    res = case.params.Cn * dCdn + math.cos(math.radians(60.0)) * (1 - CI * CI) / SQ2
    assert np.max(np.abs(CG - CG_prev)) <= 1e-12
    assert np.max(np.abs(res)) <= 1e-10
    assert np.max(np.abs(st.CI - CI)) <= 1e-10


def _random_faces(grid, seed, amp=0.05):
    rng = np.random.default_rng(seed)
    return [amp * rng.standard_normal(grid.shape) for _ in range(grid.ndim)]


@pytest.mark.parametrize("ls,kind", [(0.0, "sin"), (1e12, "sin"), (0.0, "circle"), (1e12, "tilted")])
def test_velocity_fill_limits(ls, kind):
    """No penetration at I always; no slip (ls = 0) gives zero tangential velocity at I;
    ls -> infinity gives zero normal derivative of the tangential velocity (the capillary
    bracket is zero under the static condition)."""
    case = W.small_case(64, 32, kind=kind, theta_deg=70.0, slip_length=ls)
    st, T = _state(case)
    st.faces = _random_faces(case.grid, 3)
    faces_before = [f.copy() for f in st.faces]
    st.fill_velocity(st.C)
    uG = st.last_uG
    n = T.normal
    g = T.gamma
    uc = centred_velocity(faces_before, case.grid)
    uM = np.stack([mirror_value(u.reshape(-1), T) for u in uc])
    uI = (g * uG + uM) / (g + 1)
    assert np.max(np.abs((uI * n).sum(0))) <= 1e-13
    VtM = uM - (uM * n).sum(0) * n
    VtG = uG - (uG * n).sum(0) * n
    if ls == 0.0:
        assert np.max(np.abs(g * VtG + VtM)) <= 1e-13
    else:
        assert np.max(np.abs(VtG - VtM)) <= 1e-12
    # faces touching a ghost hold the mean of the two adjacent centred values; others unchanged
    ghost = np.zeros(case.grid.cells, bool)
    ghost[T.gidx] = True
    ghost = ghost.reshape(case.grid.shape)
    ux_c = uc[0].reshape(-1).copy()
    ux_c[T.gidx] = uG[0]
    ux_c = ux_c.reshape(case.grid.shape)
    touch = ghost | np.roll(ghost, -1, axis=1)
    expect = np.where(touch, 0.5 * (ux_c + np.roll(ux_c, -1, axis=1)), faces_before[0])
    assert np.array_equal(st.faces[0], expect)


@pytest.mark.parametrize("kind", ["flat", "sin", "circle"])
def test_mass_identity_before_ghost_overwrite(kind):
    """sum C* = (4/3) sum C^n - (1/3) sum C^(n-1): the zero mode of the spectral solve,
    with the flux-form advection and the reflecting Laplacian summing to zero."""
    case = W.small_case(64, 32, kind=kind, theta_deg=60.0)
    st, T = _state(case)
    st.faces = _random_faces(case.grid, 5, 0.2)
    for _ in range(5):
        Cs = st.provisional()
        ref = (4.0 / 3.0) * st.C.sum() - (1.0 / 3.0) * st.Cp.sum()
        assert abs(Cs.sum() - ref) <= 1e-11 * np.abs(st.C).sum()
        st.step(1)


# ---- general mixed boundary condition for any scalar ----------------------------------------

def _flat_on_centre_tables():
    """Wall on a cell face with d1 = 1.5h, d2 = 1h: M, IP1 and IP2 fall on cell centres, so the
    mirror value of a linear field is exact (pinned above)."""
    g = W.Grid((32, 16), (0.0, 0.0), (2.0, 1.0))
    h = g.h
    prm = W.Params(Cn=0.05, Pe=10.0, d1_cells=1.5, d2_cells=1.0)
    T = build_tables(g, [W.Shape(W.HALFPLANE, (0.0, 4 * h, 0.0, 0.0, 1.0, 0.0))], prm)
    y = (np.arange(16) + 0.5) * h
    x = (np.arange(32) + 0.5) * h
    return g, T, x, y


@pytest.mark.parametrize("a,b", [(1.0, 0.0), (0.0, 1.0), (-2.5, 1.0), (0.7, -0.3)])
def test_mixed_condition_reproduces_a_linear_field(a, b):
    """For f = 0.3 + 1.7 y - 0.4 x the wall value and normal derivative are known in closed form;
    the ghost value that imposes a f_I + b df/dn = g with that g is the field's own value at G."""
    from oracle.solver import fill_scalar
    g_, T, x, y = _flat_on_centre_tables()
    f = 0.3 + 1.7 * y[:, None] - 0.4 * x[None, :]
    Ix, Iy = T.points["I"]
    Gx, Gy = T.points["G"]
    nx_, ny_ = T.normal
    fI = 0.3 + 1.7 * Iy - 0.4 * Ix
    dfdn = -0.4 * nx_ + 1.7 * ny_
    wrong = f.copy()
    wrong.reshape(-1)[T.gidx] = 99.0                    # the ghosts' previous values play no role
    out = fill_scalar(wrong, T, a, b, a * fI + b * dfdn)
    assert np.max(np.abs(out.reshape(-1)[T.gidx] - (0.3 + 1.7 * Gy - 0.4 * Gx))) <= 1e-12
    keep = np.ones(g_.cells, dtype=bool)
    keep[T.gidx] = False
    assert np.array_equal(out.reshape(-1)[keep], wrong.reshape(-1)[keep])


@pytest.mark.parametrize("kind", ["sin", "circle"])
def test_mixed_condition_holds_at_the_wall_on_curved_walls(kind):
    """On curved walls the filled ghost and the mirror value satisfy the condition at I exactly,
    with I's value and derivative formed from G and M by the two-point formulas."""
    from oracle.solver import fill_scalar
    case = W.small_case(64, 32, kind=kind)
    T = build_tables(case.grid, case.shapes, case.params)
    rng = np.random.default_rng(4)
    f = rng.standard_normal(case.grid.shape)
    gv = rng.standard_normal(T.n_ghost)
    for a, b in ((1.0, 0.0), (0.0, 1.0), (-3.0, 0.5)):
        out = fill_scalar(f, T, a, b, gv)
        fG = out.reshape(-1)[T.gidx]
        fM = mirror_value(f.reshape(-1), T)
        fI = (T.gamma * fG + fM) / (T.gamma + 1.0)
        dfdn = (fM - fG) / ((1.0 + T.gamma) * T.dn)
        assert np.max(np.abs(a * fI + b * dfdn - gv)) <= 1e-9 * (1.0 + np.max(np.abs(b / T.dn)))


def test_neumann_zero_is_the_mirror_value():
    from oracle.solver import fill_scalar
    case = W.small_case(64, 32, kind="sin")
    T = build_tables(case.grid, case.shapes, case.params)
    f = np.random.default_rng(2).standard_normal(case.grid.shape)
    out = fill_scalar(f, T, 0.0, 1.0, 0.0)
    assert np.max(np.abs(out.reshape(-1)[T.gidx] - mirror_value(f.reshape(-1), T))) <= 1e-14
