"""GPU: the batched sweep (grouped launches per phase, hipGraph replays) against stepping each
state alone (bit for bit with the same launch shapes) and against the oracle."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle.geometry import build_tables, face_fractions
from oracle.solver import OracleState

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def chib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2104_00350_amd import chib as m
    return m


def _cases():
    return [W.small_case(64, 32, kind="flat", theta_deg=50.0),
            W.small_case(128, 64, kind="sin", theta_deg=120.0, seed=3),
            W.small_case(256, 128, kind="circle", theta_deg=80.0, seed=4),
            W.small_case(64, 32, kind="tilted", theta_deg=100.0, seed=5),
            W.config4_cases(6)[5]]


def _make(chib, case, faces_seed):
    T = build_tables(case.grid, case.shapes, case.params)
    g = case.grid
    geo = chib.Geometry.from_tables(g.n, g.lo, g.hi, T.gidx, T.normal, T.dn, T.gamma, T.ap, T.w, T.alpha)
    if case.params.navier_stokes:   # the momentum step needs the staggered-cell fractions too
        geo.set_face_fractions(face_fractions(g, case.shapes, case.params))
    st = chib.State(geo, case.params)
    C0, _ = case.initial_fields()
    rng = np.random.default_rng(faces_seed)
    faces = [0.2 * rng.standard_normal(g.shape) for _ in range(2)]
    st.set_initial(C0, faces)
    return st, T, C0, faces


def _with_rhs_kernel(st, unroll):
    sh = st.shapes()
    sh[0][2] = unroll
    st.set_shapes(sh)
    return st


@pytest.mark.parametrize("unroll", [1, 3])      # line-tiled and y-marching rhs
def test_batched_steps_equal_single_steps(chib, unroll):
    cases = _cases()
    singles = [_with_rhs_kernel(_make(chib, c, 10 + i)[0], unroll) for i, c in enumerate(cases)]
    members = [_with_rhs_kernel(_make(chib, c, 10 + i)[0], unroll) for i, c in enumerate(cases)]
    b = chib.Batch(members)
    print("[gpu] batch of", len(members), file=sys.stderr, flush=True)
    b.step(21)            # ten graph replays of two steps plus one direct step
    b.sync()
    for s in singles:
        s.step(21)
    for s, m in zip(singles, members):
        assert np.array_equal(s.get(chib.FIELD_C), m.get(chib.FIELD_C))
        assert np.array_equal(s.get(chib.FIELD_C_PREV), m.get(chib.FIELD_C_PREV))
        assert np.array_equal(s.get(chib.FIELD_U), m.get(chib.FIELD_U))
        assert m.diagnostics()["step"] == 21
    b.step(4)
    b.sync()
    for s in singles:
        s.step(4)
    for s, m in zip(singles, members):
        assert np.array_equal(s.get(chib.FIELD_C), m.get(chib.FIELD_C))


def test_batch_against_oracle_after_tuning(chib):
    cases = _cases()[:3]
    made = [_make(chib, c, 20 + i) for i, c in enumerate(cases)]
    b = chib.Batch([m[0] for m in made])
    radix, unroll = b.tune(2)
    print("[gpu] batch tuned", radix, unroll, file=sys.stderr, flush=True)
    assert all(r in (8, 16) for r in radix) and unroll in (1, 2, 3)
    b.step(40)
    b.sync()
    for case, (st, T, C0, faces) in zip(cases, made):
        orc = OracleState(case.grid, case.params, T, C0, faces)
        orc.step(40)
        assert float(np.max(np.abs(st.get(chib.FIELD_C) - orc.C))) <= 1e-9
        assert float(np.max(np.abs(st.get(chib.FIELD_U) - orc.faces[0]))) <= 1e-9


def test_batch_rejects_3d_and_dynamic(chib):
    c3 = W.small_case_3d(16)
    g = c3.grid
    geo = chib.Geometry.build(g.n, g.lo, g.hi, c3.shapes, c3.params)
    s3 = chib.State(geo, c3.params)
    s3.set_initial(c3.initial_fields()[0])
    with pytest.raises(chib.ChibError) as e:
        chib.Batch([s3])
    assert e.value.code == chib.EUNSUPPORTED
    cd = W.small_case(64, 32, kind="flat", Vs=100.0)
    sd, _, _, _ = _make(chib, cd, 2)
    with pytest.raises(chib.ChibError) as e:
        chib.Batch([sd])
    assert e.value.code == chib.EUNSUPPORTED


def test_momentum_members_step_like_single_states(chib):
    """Members with the momentum step ride along in a batch (their own launches on the batch's
    stream) and end bit for bit where stepping them alone ends; the grouped member beside them
    too, through graph replays, a direct step and a tuning pass."""
    import dataclasses
    cases = [W.small_case(64, 32, kind="sin", theta_deg=70.0, seed=8),
             W.small_case(64, 32, kind="flat", theta_deg=50.0),
             W.small_case(128, 64, kind="circle", theta_deg=110.0, seed=9)]
    for i in (0, 2):
        cases[i] = dataclasses.replace(cases[i], params=dataclasses.replace(cases[i].params, navier_stokes=True))
    singles = [_make(chib, c, 30 + i)[0] for i, c in enumerate(cases)]
    members = [_make(chib, c, 30 + i)[0] for i, c in enumerate(cases)]
    b = chib.Batch(members)
    b.step(9)
    b.sync()
    for s in singles:
        s.step(9)
    fields = (chib.FIELD_C, chib.FIELD_C_PREV, chib.FIELD_U, chib.FIELD_V)
    for i, (s, m) in enumerate(zip(singles, members)):
        for f in fields + ((chib.FIELD_P,) if i != 1 else ()):
            assert np.array_equal(s.get(f), m.get(f)), (i, f)
        assert m.diagnostics()["step"] == 9
    b.tune(1)   # (the grouped member's shared FFT radices may now differ from its own shapes)
    for s, m in zip(singles, members):
        s.set_shapes(m.shapes())
    b.step(4)
    b.sync()
    for s in singles:
        s.step(4)
    for i, (s, m) in enumerate(zip(singles, members)):
        for f in fields:
            if i == 1:
                assert float(np.max(np.abs(s.get(f) - m.get(f)))) <= 1e-11, (i, f)
            else:
                assert np.array_equal(s.get(f), m.get(f)), (i, f)


def test_batch_of_momentum_members_only(chib):
    """A batch whose every member has the momentum step (no grouped launches at all)."""
    import dataclasses
    c = W.small_case(64, 32, kind="tilted", theta_deg=100.0, seed=5)
    c = dataclasses.replace(c, params=dataclasses.replace(c.params, navier_stokes=True))
    single, member = _make(chib, c, 41)[0], _make(chib, c, 41)[0]
    b = chib.Batch([member])
    b.step(3)
    b.sync()
    single.step(3)
    assert np.array_equal(single.get(chib.FIELD_C), member.get(chib.FIELD_C))
    assert np.array_equal(single.get(chib.FIELD_U), member.get(chib.FIELD_U))
