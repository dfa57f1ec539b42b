"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on identical seeded
inputs.  Tolerances: L-inf <= 1e-9 on C for the FP64 path after 200 steps (the project's
target); stage tests (one operation on the same input) are held to 1e-11 relative."""
import dataclasses
import sys

import numpy as np
import pytest

import workloads as W
from oracle.geometry import build_tables
from oracle.solver import OracleState, chemical_potential, diagnostics, spectral_solve

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print("[gpu]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def chib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2104_00350_amd import chib as m
    return m


def _geom_from_oracle(chib, case, T):
    g = case.grid
    return chib.Geometry.from_tables(g.n, g.lo, g.hi, T.gidx, T.normal, T.dn, T.gamma, T.ap, T.w, T.alpha)


def _pair(chib, case, faces=None, precision=64, own_geometry=False):
    T = build_tables(case.grid, case.shapes, case.params)
    if own_geometry:
        geo = chib.Geometry.build(case.grid.n, case.grid.lo, case.grid.hi, case.shapes, case.params)
    else:
        geo = _geom_from_oracle(chib, case, T)
    C0, f0 = case.initial_fields()
    if faces is not None:
        f0 = faces
    st = chib.State(geo, case.params, precision)
    st.set_initial(C0, f0)
    orc = OracleState(case.grid, case.params, T, C0, f0)
    return st, orc, T


def _linf(a, b):
    return float(np.max(np.abs(np.asarray(a, dtype=np.float64) - b)))


def _random_faces(grid, seed, amp):
    rng = np.random.default_rng(seed)
    return [amp * rng.standard_normal(grid.shape) for _ in range(grid.ndim)]


# ---- stages -----------------------------------------------------------------------------

@pytest.mark.parametrize("n", [(8, 8), (64, 32), (128, 64), (512, 256), (1024, 512), (16, 8, 8),
                               (32, 16, 64), (64, 64, 64)])
def test_spectral_solve_stage(chib, n):
    d = len(n)
    grid = W.Grid(n, (0.0,) * d, tuple(v / 64.0 for v in n))
    prm = W.Params(Cn=0.02, Pe=100.0, dt=1e-4)
    T = build_tables(grid, [], prm)
    geo = chib.Geometry.from_tables(grid.n, grid.lo, grid.hi, T.gidx, T.normal, T.dn, T.gamma, T.ap, T.w)
    st = chib.State(geo, prm)
    st.set_initial(np.zeros(grid.shape))
    rng = np.random.default_rng(sum(n))
    Q = rng.standard_normal(grid.shape) * 1e9
    _say("solve stage", n)
    out = st.stage(chib.STAGE_SOLVE, Q)
    ref = spectral_solve(Q, grid, st_alpha(prm)[0], st_alpha(prm)[1])
    assert _linf(out, ref) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("tile", [3, 4])
@pytest.mark.parametrize("radix", [8, 16])
@pytest.mark.parametrize("precision", [64, 32])
@pytest.mark.parametrize("n", [(256, 256, 8), (32, 8, 256), (256, 256)])
def test_fixed_size_transform_kernels(chib, n, precision, radix, tile):
    """256-point lines in the tile widths that have fixed-size instances (x pass 8 or 16 lines, y pass
    8 or 16 columns, bounded-axis solve a full 32 KB tile) give the same bits as the runtime-size
    kernels at narrower tiles, whose per-line arithmetic is the same, and match the oracle."""
    d = len(n)
    grid = W.Grid(n, (0.0,) * d, tuple(v / 64.0 for v in n))
    prm = W.Params(Cn=0.02, Pe=100.0, dt=1e-4)
    T = build_tables(grid, [], prm)
    geo = chib.Geometry.from_tables(grid.n, grid.lo, grid.hi, T.gidx, T.normal, T.dn, T.gamma, T.ap, T.w)
    st = chib.State(geo, prm, precision)
    st.set_initial(np.zeros(grid.shape))
    Q = np.random.default_rng(7).standard_normal(grid.shape) * 1e9
    full = 4 if precision == 64 else 5      # log2 of the columns of a full bounded-axis tile
    _say("fixed-size transforms", n, precision, radix, tile)
    st.set_shapes([[tile, radix, 1], [tile, radix, 1], [full, radix, 1], [tile, radix, 1]])
    fixed = st.stage(chib.STAGE_SOLVE, Q)
    st.set_shapes([[2, radix, 1], [2, radix, 1], [full - 1, radix, 1], [2, radix, 1]])
    runtime = st.stage(chib.STAGE_SOLVE, Q)
    assert np.array_equal(np.asarray(fixed), np.asarray(runtime))
    ref = spectral_solve(Q, grid, st_alpha(prm)[0], st_alpha(prm)[1])
    assert _linf(fixed, ref) <= (1e-12 if precision == 64 else 1e-4) * np.max(np.abs(ref))


def st_alpha(prm):
    from oracle.solver import derived_coefficients
    _, al, a = derived_coefficients(prm)
    return al, a


@pytest.mark.parametrize("maker", [lambda: W.config1(), lambda: W.small_case(64, 32, kind="sin"),
                                   lambda: W.small_case_3d(32)])
def test_rhs_stage_and_initial_fill(chib, maker):
    case = maker()
    faces = _random_faces(case.grid, 4, 0.3)
    st, orc, T = _pair(chib, case, faces)
    _say("rhs stage", case.name)
    q = st.stage(chib.STAGE_RHS)
    qref = orc.rhs()
    assert _linf(q, qref) <= 1e-11 * np.max(np.abs(qref))
    assert _linf(st.get(chib.FIELD_C), orc.C) <= 1e-13
    assert _linf(st.get(chib.FIELD_C_PREV), orc.Cp) <= 1e-13
    for a in range(case.grid.ndim):
        assert _linf(st.get(chib.FIELD_U + a), orc.faces[a]) <= 1e-13
    phi = st.stage(chib.STAGE_PHI)
    pref = chemical_potential(orc.C, case.grid, T, case.params.Cn)
    assert _linf(phi, pref) <= 1e-11 * np.max(np.abs(pref))


# ---- full steps ---------------------------------------------------------------------------

def test_config1_200_steps(chib):
    case = W.config1()
    st, orc, _ = _pair(chib, case)
    _say("config1 200 steps")
    st.step(200)
    orc.step(200)
    err = _linf(st.get(chib.FIELD_C), orc.C)
    _say("config1 Linf", err)
    assert err <= 1e-9
    for a in range(2):
        assert _linf(st.get(chib.FIELD_U + a), orc.faces[a]) <= 1e-9
    dg = st.diagnostics()
    dref = diagnostics(case.grid, case.params, orc.T.alpha, orc.C)
    for k in ("mass_box", "mass_fluid", "free_energy", "max_abs_C"):
        assert abs(dg[k] - dref[k]) <= 1e-9 * max(1.0, abs(dref[k])), k
    assert dg["step"] == 200 and dg["status"] == 0


def test_diagnostics_3d_grid_stride(chib):
    """A 3D grid of 4M cells, more than one sweep of the first reduction pass (8192 blocks of 256
    threads), so each thread folds several cells: the diagnostics match the oracle's, and a second
    call returns the same bits (fixed reduction order)."""
    g = W.Grid((256, 128, 128), (-4.0, -2.0, -2.0), (4.0, 2.0, 2.0))
    prm = W.Params(Cn=0.05, Pe=200.0, Re=5.0, Ca=0.05, theta_deg=70.0, slip_length=0.01, dt=1e-4,
                   subgrid=20)   # 20 subgrid points per direction: the oracle counts in seconds
    case = W.Case("diag_stride", g, [W.Shape(W.SPHERE, (0.0, 0.0, 0.0, 1.0))], prm, 0, (0.0, 0.0, 1.5),
                  0.5, 1e-2, 3)
    st, orc, T = _pair(chib, case)
    _say("diagnostics 256x128x128")
    dg = st.diagnostics()          # runs the pending initial ghost fill first
    assert _linf(st.get(chib.FIELD_C), orc.C) <= 1e-12
    dref = diagnostics(g, prm, T.alpha, orc.C)
    for k in ("mass_box", "mass_fluid", "free_energy", "max_abs_C"):
        assert abs(dg[k] - dref[k]) <= 1e-9 * max(1.0, abs(dref[k])), k
    assert dg == st.diagnostics()


def test_diagnostics_thick_z_chunks(chib):
    """512 x 512 x 256 (64M cells): 16-plane chunks would need 16384 reduction blocks, more than the
    partial buffer holds, so the z-march takes 32-plane chunks.  Random field, no wall; the oracle's
    diagnostics of the same field."""
    g = W.Grid((512, 512, 256), (0.0, 0.0, 0.0), (2.0, 2.0, 1.0))
    prm = W.Params(Cn=0.02, Pe=100.0, dt=1e-4)
    T = build_tables(g, [], prm)
    geo = _geom_from_oracle(chib, W.Case("thick", g, [], prm, 0, (1.0, 1.0, 0.5), 0.25, 0.0, None), T)
    rng = np.random.default_rng(21)
    C0 = 0.2 + 0.6 * rng.standard_normal(g.shape)
    st = chib.State(geo, prm)
    st.set_initial(C0)
    _say("diagnostics 512x512x256")
    dg = st.diagnostics()
    dref = diagnostics(g, prm, T.alpha, C0)
    for k in ("mass_box", "mass_fluid", "free_energy", "max_abs_C"):
        assert abs(dg[k] - dref[k]) <= 1e-9 * max(1.0, abs(dref[k])), k
    assert dg == st.diagnostics()


def test_diagnostics_fp32_state(chib):
    """FP32 state, 3D z-march: the reductions run in double on the stored floats.  No wall, so the
    initial fill leaves the field as set and the oracle sees the same float-rounded values."""
    g = W.Grid((256, 64, 64), (0.0, 0.0, 0.0), (4.0, 1.0, 1.0))
    prm = W.Params(Cn=0.05, Pe=100.0, dt=1e-4)
    T = build_tables(g, [], prm)
    geo = _geom_from_oracle(chib, W.Case("fp32", g, [], prm, 0, (2.0, 0.5, 0.5), 0.25, 0.0, None), T)
    rng = np.random.default_rng(33)
    C0 = (0.1 + 0.7 * rng.standard_normal(g.shape)).astype(np.float32).astype(np.float64)
    st = chib.State(geo, prm, 32)
    st.set_initial(C0)
    dg = st.diagnostics()
    dref = diagnostics(g, prm, T.alpha, C0)
    for k in ("mass_box", "mass_fluid", "free_energy", "max_abs_C"):
        assert abs(dg[k] - dref[k]) <= 1e-9 * max(1.0, abs(dref[k])), k


@pytest.mark.parametrize("n", [(64, 32), (16, 8, 8)])
def test_wall_free_box_full_steps(chib, n):
    """No immersed wall: zero ghosts and no face touching one, so the fills have empty lists; the
    steps (advection by a random flow included) still match the oracle."""
    d = len(n)
    grid = W.Grid(n, (0.0,) * d, tuple(v / 16.0 for v in n))
    prm = W.Params(Cn=0.1, Pe=50.0, dt=1e-3)
    centre = tuple(0.5 * v / 16.0 for v in n)
    case = W.Case("wall_free", grid, [], prm, 100, centre, 0.25 * min(n) / 16.0, 1e-2, 5)
    st, orc, T = _pair(chib, case, _random_faces(grid, 6, 0.2))
    assert len(T.gidx) == 0
    _say("wall-free box", n)
    st.step(100)
    orc.step(100)
    assert _linf(st.get(chib.FIELD_C), orc.C) <= 1e-9
    for a in range(d):
        assert _linf(st.get(chib.FIELD_U + a), orc.faces[a]) == 0.0


def test_config1_own_geometry(chib):
    case = W.config1()
    st, orc, _ = _pair(chib, case, own_geometry=True)
    st.step(200)
    orc.step(200)
    assert _linf(st.get(chib.FIELD_C), orc.C) <= 1e-9


@pytest.mark.parametrize("i", range(6))
def test_config2_cases_200_steps(chib, i):
    case = W.config2(i)
    st, orc, _ = _pair(chib, case)
    _say("config2 case", i, case.name)
    st.step(200)
    orc.step(200)
    err = _linf(st.get(chib.FIELD_C), orc.C)
    _say("config2 case", i, "Linf", err)
    assert err <= 1e-9


@pytest.mark.parametrize("kind,theta", [("sin", 45.0), ("circle", 120.0), ("tilted", 70.0)])
def test_velocity_fill_with_flow(chib, kind, theta):
    """Nonzero initial face velocities exercise the advection and the slip fill."""
    case = W.small_case(64, 32, kind=kind, theta_deg=theta, slip_length=0.02)
    faces = _random_faces(case.grid, 8, 0.5)
    st, orc, _ = _pair(chib, case, faces)
    _say("velocity fill", kind)
    st.step(100)
    orc.step(100)
    assert _linf(st.get(chib.FIELD_C), orc.C) <= 1e-9
    for a in range(2):
        assert _linf(st.get(chib.FIELD_U + a), orc.faces[a]) <= 1e-9


@pytest.mark.parametrize("kind", ["sin", "flat"])
def test_dynamic_condition(chib, kind):
    case = W.small_case(64, 32, kind=kind, theta_deg=60.0, Vs=200.0)
    st, orc, _ = _pair(chib, case)
    _say("dynamic", kind)
    st.step(100)
    orc.step(100)
    assert _linf(st.get(chib.FIELD_C), orc.C) <= 1e-9
    assert _linf(st.get(chib.FIELD_CI), orc.CI) <= 1e-9


def test_3d_sphere_50_steps(chib):
    case = W.small_case_3d(32)
    st, orc, _ = _pair(chib, case)
    _say("3d sphere 32^3")
    st.step(50)
    orc.step(50)
    assert _linf(st.get(chib.FIELD_C), orc.C) <= 1e-9
    for a in range(3):
        assert _linf(st.get(chib.FIELD_U + a), orc.faces[a]) <= 1e-9


class _Config3Run:
    """Config 3 at its full 256^3 size: the GPU path in FP64 and in FP32 and the oracle, all from the
    same inputs and the oracle's tables, advanced together and compared on every cell at
    checkpoints (one test per checkpoint, so each test takes a fraction of the oracle's run)."""

    def __init__(self, chib):
        case = W.config3(256)
        # the step is compared on the oracle's own tables; at 256^3 the oracle counts its volume
        # fractions with 20 subgrid points per direction (100 would take the CPU a quarter of an
        # hour), the count the builders' agreement at 100 is checked on smaller grids
        case.params = dataclasses.replace(case.params, subgrid=20)
        _say("config3 256^3: oracle tables")
        T = build_tables(case.grid, case.shapes, case.params)
        geo = _geom_from_oracle(chib, case, T)
        C0, f0 = case.initial_fields()
        self.chib = chib
        self.st = {}
        for prec in (64, 32):
            self.st[prec] = chib.State(geo, case.params, prec)
            self.st[prec].set_initial(C0, f0)
        self.orc = OracleState(case.grid, case.params, T, C0, f0)
        self.done = 0
        self.res = {}

    def at(self, n):
        if n not in self.res:
            assert n > self.done
            _say("config3 256^3: steps", self.done, "->", n)
            for st in self.st.values():
                st.step(n - self.done)
            self.orc.step(n - self.done)
            self.done = n
            C64 = self.st[64].get(self.chib.FIELD_C)
            d32 = np.asarray(self.st[32].get(self.chib.FIELD_C), dtype=np.float64) - self.orc.C
            self.res[n] = {"fp64_linf": _linf(C64, self.orc.C), "fp32_linf": float(np.max(np.abs(d32))),
                           "fp32_l2": float(np.sqrt(np.mean(d32 * d32)))}
            _say("config3 step", n, self.res[n])
        return self.res[n]


@pytest.fixture(scope="module")
def config3_run(chib):
    run = _Config3Run(chib)
    yield run
    run.st.clear()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("n", [50, 100, 150, 200])
def test_config3_full_size_fp64(config3_run, n):
    """The project's gate on the plain FP64 path: L-inf <= 1e-9 on every cell, through 200 steps."""
    assert config3_run.at(n)["fp64_linf"] <= 1e-9


@pytest.mark.xfail(strict=True, reason=(
    "measured L-inf 4.1e-4 and L2 1.8e-5 after 200 steps, against the gate of 1e-4 proposed before the "
    "run: the FP32 path misses it at full size"))
def test_config3_full_size_200_steps_fp32(config3_run):
    """The FP32 path against the FP64 oracle, held to the sanity gate L-inf <= 1e-4 proposed for it
    before it was run; its L2 is reported beside."""
    assert config3_run.at(200)["fp32_linf"] <= 1e-4


def test_fp32_path_tracks_fp64_oracle(chib):
    case = W.config1()
    st, orc, _ = _pair(chib, case, precision=32)
    st.step(200)
    orc.step(200)
    err = _linf(st.get(chib.FIELD_C), orc.C)
    _say("fp32 config1 Linf", err)
    assert err <= 1e-3


def test_bitwise_determinism_and_checkpoint(chib):
    case = W.small_case(64, 32, kind="sin", theta_deg=50.0)
    faces = _random_faces(case.grid, 2, 0.2)
    st1, _, T = _pair(chib, case, faces)
    st1.step(30)
    blob = st1.save()
    st1.step(30)
    a = st1.get(chib.FIELD_C)
    st2, _, _ = _pair(chib, case, faces)
    st2.step(60)
    assert np.array_equal(a, st2.get(chib.FIELD_C))
    st3, _, _ = _pair(chib, case, faces)
    st3.load(blob)
    st3.step(30)
    assert np.array_equal(a, st3.get(chib.FIELD_C))
    assert np.array_equal(st1.get(chib.FIELD_U), st3.get(chib.FIELD_U))
    assert st3.diagnostics()["step"] == 60


def test_nan_is_reported(chib):
    case = W.config1()
    st, _, _ = _pair(chib, case)
    C0, _ = case.initial_fields()
    C0[10, 10] = np.nan
    st.set(chib.FIELD_C, C0)
    dg = st.diagnostics()
    assert dg["status"] == chib.ENAN


def test_tuned_shapes_keep_parity(chib):
    """Launch shapes chosen by the autotuner change speed, not results (beyond FFT rounding)."""
    case = W.small_case_3d(32)
    st, orc, _ = _pair(chib, case)
    shapes = st.tune(2)
    _say("tuned shapes", shapes)
    assert shapes[0][1] in (4, 8, 16) and all(s[1] in (8, 16) for s in shapes[1:])
    st.step(20)
    orc.step(20)
    assert _linf(st.get(chib.FIELD_C), orc.C) <= 1e-9
    for radix in (8, 16):
        for lt in (1, 2, 3):
            st.set_shapes([[lt, radix, 1 + (lt & 1)]] * 4)
            out = st.stage(chib.STAGE_SOLVE, orc.rhs())
            ref = orc.provisional()
            assert _linf(out, ref) <= 1e-12 * np.max(np.abs(ref))
    with pytest.raises(chib.ChibError):
        st.set_shapes([[2, 4, 1]] * 4)


def test_full_size_launch_shapes_agree(chib):
    """At 256^3 the measured launch shapes (fixed-size y, bounded-axis and x passes at radix 16, 8
    and 8), the default shapes (the radix-16 fixed-size instances, the ones the 256^3 oracle
    comparison steps with) and shapes that take only runtime-size transform kernels give the same
    C after 5 steps up to FFT rounding."""
    case = W.config3(256)
    g = case.grid
    geo = chib.Geometry.build_device(g.n, g.lo, g.hi, case.shapes, case.params)
    C0, faces = case.initial_fields()
    out = {}
    for name, shapes in (("measured", [[2, 4, 5], [4, 16, 1], [4, 8, 1], [3, 8, 1]]), ("default", None),
                         ("runtime-size", [[2, 4, 5], [2, 8, 1], [3, 16, 1], [2, 16, 1]])):
        st = chib.State(geo, case.params)
        st.set_initial(C0, faces)
        if shapes:
            st.set_shapes(shapes)
        _say("256^3 shapes", name)
        st.step(5)
        out[name] = np.asarray(st.get(chib.FIELD_C))
        del st
    for name in ("default", "runtime-size"):
        err = float(np.max(np.abs(out["measured"] - out[name])))
        _say("256^3 shapes: measured vs", name, err)
        assert err <= 1e-11


def test_radix_4_outside_the_z_march_takes_radix_8(chib):
    """Pass-0 radix 4 exists for the z-marching kernel only; the 2D rhs kernels (line-tiled and
    y-marching) take radix 8 for it, bit for bit."""
    case = W.small_case(128, 64, kind="sin", theta_deg=70.0)
    faces = _random_faces(case.grid, 4, 0.3)
    st, _, _ = _pair(chib, case, faces)
    st.step(0)
    blob = st.save()
    for unroll in (1, 2, 3):
        out = []
        for radix in (4, 8):
            st.load(blob)
            st.set_shapes([[2, radix, unroll], [3, 8, 1], [3, 8, 1], [3, 8, 1]])
            assert st.shapes()[0] == [2, radix, unroll]
            st.step(5)
            out.append(st.get(chib.FIELD_C))
        assert np.array_equal(out[0], out[1]), unroll


@pytest.mark.parametrize("n", [(256, 16, 32), (512, 8, 32)])
def test_z_marching_rhs_variants(chib, n):
    """Every shape of the z-marching rhs kernel (3D, nx = 256 and 512: one and two columns per
    thread), fused with the x transform or split from it, matches the oracle step.  Chunks of 8 to
    256 planes cover chunks shorter than, equal to and (clamped) longer than the grid."""
    h = 4.0 / n[0]
    grid = W.Grid(n, (-2.0, -0.5 * h * n[1], -0.5 * h * n[2]), (2.0, 0.5 * h * n[1], 0.5 * h * n[2]))
    prm = W.Params(Cn=0.02, Pe=100.0, Ca=0.1, theta_deg=70.0, slip_length=0.01, dt=1e-4, subgrid=20)
    case = W.Case("slab3d", grid, [W.Shape(W.HALFPLANE, (0.0, 0.0, -0.1, 0.0, 0.0, 1.0))], prm, 10,
                  (0.0, 0.0, -0.1), 0.2, 1e-3, 5)
    faces = _random_faces(grid, 6, 0.3)
    st, orc, _ = _pair(chib, case, faces)
    st.step(0)
    blob = st.save()
    orc.step(6)
    for lt in (1, 2, 3):
        for radix in (4, 8, 16):
            for zc in (3, 4, 5, 6, 7, 8):      # 6..8: stencil-only z-march + separate x transform
                st.load(blob)
                st.set_shapes([[lt, radix, zc], [3, 8, 1], [4, 16, 1], [3, 8, 1]])
                st.step(6)
                err = _linf(st.get(chib.FIELD_C), orc.C)
                assert err <= 1e-11, (n, lt, radix, zc, err)


@pytest.mark.parametrize("maker,steps", [(lambda: W.small_case(128, 64, kind="sin", theta_deg=50.0), 60),
                                         (lambda: W.config2(1), 20), (lambda: W.config5(True, 120.0), 6)])
def test_y_marching_rhs_2d(chib, maker, steps):
    """The y-marching rhs kernel (2D, one, two and four columns per thread at nx = 128, 512 and
    1024) with both FFT radices and every tile height matches the oracle step with flow."""
    case = maker()
    faces = _random_faces(case.grid, 9, 0.3)
    st, orc, _ = _pair(chib, case, faces)
    st.step(0)
    blob = st.save()
    orc.step(steps)
    hi = {128: 5, 512: 3, 1024: 2}[case.grid.n[0]]
    for lt in range(1, hi + 1):
        for radix in (8, 16):
            st.load(blob)
            st.set_shapes([[lt, radix, 3], [3, 8, 1], [3, 8, 1], [3, 8, 1]])
            assert st.shapes()[0] == [lt, radix, 3]
            _say("y-march", case.name, lt, radix)
            st.step(steps)
            err = _linf(st.get(chib.FIELD_C), orc.C)
            assert err <= 1e-11, (lt, radix, err)


@pytest.mark.parametrize("i", range(6))
def test_config2_full_length_5000_steps(chib, i):
    """Config 2 at its full length: gated at 200 steps by the project's L-inf <= 1e-9 and held at
    1000, 2000 and 5000 steps to a bound fixed before these runs: rounding differences of a step
    map that does not expand them accumulate at most linearly, 1e-9 per 200 steps.  The values are
    printed at each checkpoint."""
    case = W.config2(i)
    st, orc, T = _pair(chib, case)
    done = 0
    for n in (200, 1000, 2000, 5000):
        st.step(n - done)
        orc.step(n - done)
        done = n
        C1 = st.get(chib.FIELD_C)
        err = _linf(C1, orc.C)
        _say("config2", case.name, "step", n, "Linf vs oracle", err)
        assert np.all(np.isfinite(C1))
        assert err <= 1e-9 * n / 200, (n, err)
