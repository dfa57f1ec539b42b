"""The allocation-free diagnostics entry point (ch_ib_diagnostics_noalloc) against ch_ib_diagnostics
through the C ABI: the same kernels in the same order, so every value must agree bit for bit; two
calls in a row, the second on a smaller grid, which reuses the same fixed device scratch."""
import ctypes
import sys

import numpy as np
import pytest

import workloads as W

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


def _state(chib, case, steps):
    geo = chib.Geometry.build(case.grid.n, case.grid.lo, case.grid.hi, case.shapes, case.params)
    st = chib.State(geo, case.params, 64)
    C0, faces = case.initial_fields()
    st.set_initial(C0, faces)
    st.step(steps)
    st.sync()
    return st


def _both(chib, st):
    lib = chib.lib
    a, b = chib.Diag(), chib.Diag()
    rc_a = lib.ch_ib_diagnostics(st.h, ctypes.byref(a))
    rc_b = lib.ch_ib_diagnostics_noalloc(st.h, ctypes.byref(b))
    assert rc_a == 0 and rc_b == 0, (rc_a, rc_b, lib.ch_ib_last_error())
    keys = ("mass_box", "mass_fluid", "free_energy", "max_abs_C", "step", "status")
    return {k: getattr(a, k) for k in keys}, {k: getattr(b, k) for k in keys}


def test_noalloc_diagnostics_match_twice_then_on_a_smaller_grid(chib):
    first = W.config1()                                # 128 x 64
    second = W.small_case(64, 32, kind="sin")          # smaller input, same scratch
    for case, steps in ((first, 30), (second, 10)):
        _say("noalloc diagnostics", case.name)
        st = _state(chib, case, steps)
        ref, got = _both(chib, st)
        assert ref == got, (case.name, ref, got)
        assert np.isfinite(got["free_energy"]) and got["step"] == steps
        st.close()
