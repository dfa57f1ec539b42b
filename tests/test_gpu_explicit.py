"""GPU parity of the explicit Adams-Bashforth step (Eq. ExpCH, CH_IB_FLAG_EXPLICIT) against the
FP64 oracle on identical seeded inputs: L-inf <= 1e-9 on C (FP64) after the step counts below,
bit-exact checkpoint/resume of the rate history, and the scheme's restrictions."""
import dataclasses
import sys

import numpy as np
import pytest

import workloads as W
from oracle.geometry import build_tables
from oracle.solver import OracleState

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


def _explicit(case, dt):
    return dataclasses.replace(case, params=dataclasses.replace(case.params, explicit=True, dt=dt))


def _pair(chib, case, faces=None, precision=64):
    T = build_tables(case.grid, case.shapes, case.params)
    g = case.grid
    geo = chib.Geometry.from_tables(g.n, g.lo, g.hi, T.gidx, T.normal, T.dn, T.gamma, T.ap, T.w, T.alpha)
    C0, f0 = case.initial_fields()
    if faces is not None:
        f0 = faces
    st = chib.State(geo, case.params, precision)
    st.set_initial(C0, f0)
    return st, OracleState(case.grid, case.params, T, C0, f0)


def _linf(a, b):
    return float(np.max(np.abs(np.asarray(a, dtype=np.float64) - b)))


def _faces(grid, seed, amp):
    rng = np.random.default_rng(seed)
    return [amp * rng.standard_normal(grid.shape) for _ in range(grid.ndim)]


@pytest.mark.parametrize("maker,steps", [(lambda: W.config1(), 200),
                                         (lambda: W.small_case(64, 32, kind="sin", theta_deg=45.0), 200),
                                         (lambda: W.small_case(64, 32, kind="circle", theta_deg=120.0), 200)])
def test_explicit_steps_match_the_oracle(chib, maker, steps):
    case = _explicit(maker(), 2e-5)
    st, orc = _pair(chib, case)
    _say("explicit", case.name)
    st.step(steps)
    orc.step(steps)
    err = _linf(st.get(chib.FIELD_C), orc.C)
    _say("explicit", case.name, "Linf", err)
    assert err <= 1e-9
    assert st.diagnostics()["status"] == 0


def test_explicit_with_flow_and_velocity_fill(chib):
    case = _explicit(W.small_case(64, 32, kind="tilted", theta_deg=70.0, slip_length=0.02), 2e-5)
    st, orc = _pair(chib, case, _faces(case.grid, 8, 0.5))
    st.step(100)
    orc.step(100)
    assert _linf(st.get(chib.FIELD_C), orc.C) <= 1e-9
    for a in range(2):
        assert _linf(st.get(chib.FIELD_U + a), orc.faces[a]) <= 1e-9


def test_explicit_3d(chib):
    case = _explicit(W.small_case_3d(32), 1e-5)
    st, orc = _pair(chib, case, _faces(case.grid, 3, 0.2))
    _say("explicit 3d")
    st.step(40)
    orc.step(40)
    assert _linf(st.get(chib.FIELD_C), orc.C) <= 1e-9


def test_explicit_3d_z_marching_kernels(chib):
    """At nx a multiple of 64 the 3D phi and update kernels march in z over 64 x 4 tiles."""
    from oracle.solver import chemical_potential
    case = _explicit(W.small_case_3d(64), 1e-5)
    st, orc = _pair(chib, case, _faces(case.grid, 4, 0.2))
    phi = st.stage(chib.STAGE_PHI)
    ref = chemical_potential(orc.C, case.grid, orc.T, case.params.Cn)
    assert _linf(phi, ref) <= 1e-11 * np.max(np.abs(ref))
    _say("explicit 3d 64^3")
    st.step(20)
    orc.step(20)
    assert _linf(st.get(chib.FIELD_C), orc.C) <= 1e-9


@pytest.mark.parametrize("n", [(64, 32), (64, 8, 16)])
def test_explicit_wall_free_box(chib, n):
    """No immersed wall: zero ghosts, so the phi ghost pass and the fills have empty lists; (64, 8, 16)
    takes the z-marching phi and update kernels."""
    d = len(n)
    grid = W.Grid(n, (0.0,) * d, tuple(v / 16.0 for v in n))
    prm = W.Params(Cn=0.1, Pe=50.0, dt=1e-5, explicit=True)
    centre = tuple(0.5 * v / 16.0 for v in n)
    case = W.Case("explicit_wall_free", grid, [], prm, 60, centre, 0.25 * min(n) / 16.0, 1e-2, 4)
    st, orc = _pair(chib, case, _faces(grid, 12, 0.3))
    assert len(orc.T.gidx) == 0
    _say("explicit wall-free", n)
    st.step(60)
    orc.step(60)
    assert _linf(st.get(chib.FIELD_C), orc.C) <= 1e-9


def test_explicit_fp32_tracks_the_fp64_oracle(chib):
    case = _explicit(W.config1(), 2e-5)
    st, orc = _pair(chib, case, precision=32)
    st.step(200)
    orc.step(200)
    assert _linf(st.get(chib.FIELD_C), orc.C) <= 1e-3


def test_explicit_checkpoint_keeps_the_rate_history(chib):
    case = _explicit(W.small_case(64, 32, kind="sin", theta_deg=60.0), 2e-5)
    faces = _faces(case.grid, 2, 0.2)
    st1, _ = _pair(chib, case, faces)
    st1.step(15)
    blob = st1.save()
    st1.step(15)
    st2, _ = _pair(chib, case, faces)
    st2.load(blob)
    st2.step(15)
    assert np.array_equal(st1.get(chib.FIELD_C), st2.get(chib.FIELD_C))
    semi, _ = _pair(chib, W.small_case(64, 32, kind="sin", theta_deg=60.0), faces)
    with pytest.raises(chib.ChibError) as e:
        semi.load(blob)                       # a blob of the other time scheme
    assert e.value.code == chib.EINVAL


def test_batches_reject_explicit_states(chib):
    case = _explicit(W.small_case(64, 32, kind="flat"), 2e-5)
    st, _ = _pair(chib, case)
    with pytest.raises(chib.ChibError) as e:
        chib.Batch([st])
    assert e.value.code == chib.EUNSUPPORTED
