#!/usr/bin/env python3
"""Benchmark of the CH + ghost-cell IB step on one MI355X.

Workload: the 3D solid sphere (radius 1 at the origin of [-2,2]^3) on a 256^3 grid with a
spherical droplet of radius 0.5 resting on its top, Cn = 0.015, Pe = 200, Ca = 0.05, static
90-degree contact angle, slip length 0.01, dt = 1e-4, FP64, velocity fill on.  Inputs are
synthetic (seeded tanh droplet, fluid at rest) and resident in HBM before timing starts.

Prints ONE JSON line: whole-job cell-updates/s, the roofline of the dominant kernel (its
algorithmic bytes per launch over its mean HIP-event duration during the timed steps) and
the FP64 CPU oracle timed on the host on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "CH+IB cell-updates/s at 256³; learned/plain speedup at ≤1° contact-angle err"


def algorithmic_bytes(name: str, cells: int, d: int, es: int, G: int, NF: int, dynamic: bool = False) -> float:
    """Bytes the method must move per launch of each kernel of a step.

    Field passes count each array they must read and write once; the ghost kernels count
    their table entries, gathers and writes per ghost (and per re-interpolated face).  The
    velocity fill gathers the centred velocity at every averaging point (2 face values per
    axis) and, with the dynamic condition only, the centred gradient of C as well."""
    K = 2 * d + 1
    if name in ("rhs_xdht", "rhs_stencil"):
        return cells * es * (2 + d + 1)              # C^n, C^(n-1), d face arrays in; Q (or its transform) out
    if name in ("xdht_fwd", "ydht_fwd", "ydht_inv", "neumann_solve", "xdht_out"):
        return cells * es * 2                        # one read, one write
    if name == "ghost_dphi":                         # per ghost: tables, C^n and C^(n-1) on the cells within
        U = 2 * d * d + 2 * d + 1                    # two steps of each interpolation point's centre cell
        return G * (4 + 2 * K * (4 + es) + (2 * U + 2 * d + 1) * 2 * es + es)   # (and the ghost's stencil), dg out
    if name == "ghost_fill_C":
        return G * (4 + 8 * K + es * (7 + 4 * K))
    if name == "ghost_fill_u":
        per_ghost = 4 + 8 * K + es * (3 * d + 4 + 2 * K + 2 * K * (4 if dynamic else 2) * d)
        per_face = 16 + es * 4 + 16 + es * 3
        return G * per_ghost + NF * per_face
    if name == "phi":                                # explicit step: phi on every cell, mirror value at ghosts
        return cells * es * 2 + G * (4 + 2 * K * (4 + es) + 2 * K * es + es)
    if name == "explicit_update":                    # C, phi, R, d faces in; C^(n+1), R out
        return cells * es * (5 + d)
    if name == "ghost_fills":                        # static: both fills, one launch plus the faces
        return (algorithmic_bytes("ghost_fill_C", cells, d, es, G, NF, dynamic)
                + algorithmic_bytes("ghost_fill_u", cells, d, es, G, NF, dynamic))
    # momentum step (Navier-Stokes coupling)
    if name == "ns_phi":
        return algorithmic_bytes("phi", cells, d, es, G, NF, dynamic)
    if name == "ns_predict":                         # u^n, N^(n-1), alpha_face (d each), C, phi in; u**, N^n out
        return cells * es * (5 * d + 2)
    if name == "ns_vel_fill":
        return algorithmic_bytes("ghost_fill_u", cells, d, es, G, NF, dynamic)
    if name == "ns_pressure_rhs":                    # u** (d), C, p^n, p^(n-1) in; rhs out
        return cells * es * (d + 4)
    if name == "ns_poisson":                         # d + (d - 1) passes, one read and one write each
        return cells * es * 2 * (2 * d - 1)
    if name == "ns_correct":                         # u^n, u** (d each), C, p^(n+1), p^n, p^(n-1) in; u^(n+1), 2u^(n+1) - u^n out
        return cells * es * (4 * d + 4)
    return 0.0


def kernel_template(name: str, shapes, es: int, n) -> list:
    """Device kernel instantiation(s) behind a step kernel name, for the launch shapes in use on a
    grid of n cells per axis."""
    t = "double" if es == 8 else "float"
    E = 32768 // es
    nx = n[0]
    lines = n[1] * (n[2] if len(n) == 3 else 1)

    def clamp(v, hi):
        return 1 if v < 1 else min(v, hi)

    def log2(v):
        return v.bit_length() - 1

    if name == "rhs_xdht":
        lt, r, u = shapes[0]
        if u >= 3 and nx in (256, 512):
            L = 2 ** min(max(lt, 1), 3 if nx == 256 else 2)
            return [f"k_rhs_xdht_zm<{t}, {L}, {nx // 256}, {8 if (r == 4 and L == 8) else r}, false>"]
        return [f"k_rhs_xdht<{t}, 3, {E}, {u}, {max(r, 8)}>"]
    if name == "rhs_stencil":
        lt = shapes[0][0]
        return [f"k_rhs_xdht_zm<{t}, {2 ** min(max(lt, 1), 3 if nx == 256 else 2)}, {nx // 256}, 8, true>"]
    if name in ("xdht_fwd", "xdht_out"):
        lt, r, _ = shapes[3]
        logL = clamp(lt, log2(max(min(E // nx, lines), 2)))
        fixed = (8, logL) if (nx == 256 and logL in (3, 4)) else (0, 0)
        return [f"k_xdht<{t}, {E}, {r if r == 8 else 16}, {fixed[0]}, {fixed[1]}>"]
    if name in ("ydht_fwd", "ydht_inv"):
        lt, r, _ = shapes[1]
        lb = clamp(lt, log2(max(min(E // n[1], nx), 2)))
        fixed = (8, lb) if (n[1] == 256 and lb in (3, 4) and nx * 256 * es < 2 ** 32) else (0, 0)
        return [f"k_strided_dht<{t}, {E}, {r if r == 8 else 16}, {fixed[0]}, {fixed[1]}>"]
    if name == "neumann_solve":
        lt, r, _ = shapes[2]
        lb = clamp(lt, log2(max(min(E // n[-1], nx), 2)))
        stride = nx * (n[1] if len(n) == 3 else 1)
        fixed = (8, lb) if (n[-1] == 256 and (256 << lb) == E and stride * 256 * es < 2 ** 32) else (0, 0)
        return [f"k_neumann_solve<{t}, {E}, {r if r == 8 else 16}, {fixed[0]}, {fixed[1]}>"]
    if name in ("ns_predict", "ns_pressure_rhs", "ns_correct"):
        return [f"k_{name}<{t}>"]
    if name == "ghost_dphi":
        return [f"k_point_phit<{t}>", f"k_ghost_dg<{t}>", f"k_patch_dq<{t}>"]
    if name == "ghost_fill_C":
        return [f"k_fill_static<{t}>"]
    if name == "ghost_fill_u":
        return [f"k_vel_ghosts<{t}>", f"k_vel_faces<{t}>"]
    if name == "ghost_fills":
        return [f"k_fill_static_vel<{t}>", f"k_vel_faces<{t}>"]
    return []


def code_digest(path: str) -> str:
    """sha256 of a source file with its comments and whitespace removed, so that the recorded counters
    stay valid across edits that change no code."""
    import hashlib
    import re
    src = open(path, encoding="utf-8").read()
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    return hashlib.sha256("".join(src.split()).encode()).hexdigest()


def measured_traffic(name: str, shapes, es: int, n):
    """HBM bytes per launch from the committed counter summary, or None when the kernel source has
    changed since the counters were taken (or the kernel was not profiled)."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic_sphere256_fp64.json")
    if es != 8 or not os.path.exists(path):
        return None
    rec = json.load(open(path))
    digests = rec.get("sources_code_sha256") or {}
    for f in ("kernels.hip", "ns.hip"):
        if code_digest(os.path.join(ROOT, "paper_2104_00350_amd", "csrc", f)) != digests.get(f):
            return None
    by_shape = rec.get("k_rhs_xdht_zm_by_pass0_shape") or {}
    key = ",".join(str(v) for v in shapes[0])
    total = 0
    for k in kernel_template(name, shapes, es, n):
        if k.startswith("k_rhs_xdht_zm"):
            # its z-chunk (a runtime launch argument) changes the halo re-reads: take the counters of
            # the same launch shape, or none
            if key not in by_shape:
                return None
            total += by_shape[key]["hbm_bytes"]
        elif k not in rec["per_dispatch"]:
            return None
        else:
            total += rec["per_dispatch"][k]["hbm_bytes"]
    return total


def sweep_benchmark(chib, torch, steps: int, count: int = 64) -> dict:
    """Config-4 sweep: `count` uneven 2D sinusoidal-wall cases, time-to-solution of `steps` steps
    each, stepped one case after another versus all together in one batch (grouped launches
    replayed as a hipGraph).  Launch shapes are tuned once per distinct grid size for both."""
    import workloads as W
    cases = W.config4_cases(count)
    geos = [chib.Geometry.build(c.grid.n, c.grid.lo, c.grid.hi, c.shapes, c.params) for c in cases]

    def make_states():
        out = []
        for c, g in zip(cases, geos):
            st = chib.State(g, c.params)
            C0, faces = c.initial_fields()
            st.set_initial(C0, faces)
            st.step(0)
            out.append(st)
        return out

    singles = make_states()
    tuned = {}
    for st in singles:
        key = st.n
        if key not in tuned:
            tuned[key] = st.tune(3)
        st.set_shapes(tuned[key])
    members = make_states()
    for st in members:
        st.set_shapes(tuned[st.n])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for st in singles:
        st.step(steps)
    torch.cuda.synchronize()
    t_single = time.perf_counter() - t0
    batch = chib.Batch(members)
    radix, unroll = batch.tune(3)
    batch.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.step(steps)
    batch.sync()
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    worst = max(float(abs(a.get(chib.FIELD_C) - b.get(chib.FIELD_C)).max()) for a, b in zip(singles, members))
    diags = [st.diagnostics() for st in members]
    nonfinite = [c.name for c, dg in zip(cases, diags) if dg["status"] != 0]
    cells = sum(c.grid.cells for c in cases)
    batch.close()
    return {"cases": count, "steps_each": steps, "cells_total": cells,
            "sizes": sorted({f"{c.grid.n[0]}x{c.grid.n[1]}" for c in cases}),
            "one_by_one_s": round(t_single, 4), "batched_s": round(t_batch, 4),
            "speedup": round(t_single / t_batch, 3),
            "batched_cell_updates_per_s": cells * steps / t_batch,
            "batch_radix_rhs_solve_out": radix, "batch_cells_in_flight": unroll,
            "max_abs_diff_batched_vs_single": worst,
            "max_abs_C_over_cases": max(dg["max_abs_C"] for dg in diags),
            "cases_not_finite": nonfinite}


def explicit_benchmark(chib, geo, case, steps: int, precision: int, NF: int, semi_ms: float) -> dict:
    """The explicit Adams-Bashforth step (Eq. ExpCH) on the same 256^3 workload at a tenth of the
    semi-implicit time step (the paper's factor between the two schemes' stable steps): kernel
    times, bytes, and the time to cover the same simulated time as one semi-implicit step."""
    import dataclasses
    prm = dataclasses.replace(case.params, explicit=True, dt=case.params.dt / 10)
    st = chib.State(geo, prm, precision)
    C0, faces = case.initial_fields()
    st.set_initial(C0, faces)
    st.step(5)
    st.sync()
    t0 = time.perf_counter()
    ms = st.step_timed(steps)
    wall = time.perf_counter() - t0
    dg = st.diagnostics()
    es = 8 if precision == 64 else 4
    cells = case.grid.cells
    kern = {}
    for name, t in ms.items():
        b = algorithmic_bytes(name, cells, 3, es, st.G, NF, False)
        kern[name] = {"ms": round(t, 5), "alg_bytes": int(b), "GB_s": round(b / (t * 1e-3) / 1e9, 1),
                      "frac_of_8TBs": round(b / (t * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    ms_step = 1e3 * wall / steps
    st.close()
    return {"workload": f"same 3D sphere workload, explicit scheme, dt = {prm.dt:g}",
            "steps": steps, "status": dg["status"], "max_abs_C": dg["max_abs_C"],
            "cell_updates_per_s": cells * steps / wall, "ms_per_step": round(ms_step, 5), "kernels": kern,
            "time_per_unit_sim_time_vs_semi_implicit": round(10 * ms_step / semi_ms, 3)}


def ns_benchmark(chib, case, steps: int, precision: int, semi_ms: float, NF: int, shapes) -> dict:
    """The coupled order-parameter + momentum step (Navier-Stokes coupling, sections 4.2.3, 4.3 and 4.4) on
    the same 256^3 workload, matched fluids (rho1 = rho2, mu1 = mu2: the explicit viscous term
    then allows the workload's dt), started from rest: kernel times, bytes and the cost over the
    order-parameter step alone."""
    import dataclasses
    prm = dataclasses.replace(case.params, navier_stokes=True)
    g = case.grid
    geo = chib.Geometry.build_device(g.n, g.lo, g.hi, case.shapes, prm)
    st = chib.State(geo, prm, precision)
    st.set_shapes(shapes)          # the order-parameter passes run with the main state's launch shapes
    C0, faces = case.initial_fields()
    st.set_initial(C0, faces)
    st.step(5)
    st.sync()
    t0 = time.perf_counter()
    ms = st.step_timed(steps)
    wall = time.perf_counter() - t0
    dg = st.diagnostics()
    es = 8 if precision == 64 else 4
    cells = g.cells
    kern = {}
    for name, t in ms.items():
        b = algorithmic_bytes(name, cells, 3, es, st.G, NF, False)
        kern[name] = {"ms": round(t, 5), "alg_bytes": int(b), "GB_s": round(b / (t * 1e-3) / 1e9, 1),
                      "frac_of_8TBs": round(b / (t * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    import numpy as np
    umax = max(float(np.max(np.abs(st.get(chib.FIELD_U + a)))) for a in range(3))
    ms_step = 1e3 * wall / steps
    st.close()
    return {"workload": "same 3D sphere workload with the momentum step (Re 5, Ca 0.05, matched fluids)",
            "steps": steps, "status": dg["status"], "max_abs_C": dg["max_abs_C"], "max_abs_u": umax,
            "cell_updates_per_s": cells * steps / wall, "ms_per_step": round(ms_step, 5),
            "vs_order_parameter_step": round(ms_step / semi_ms, 3), "kernels": kern}


def scalar_fill_benchmark(chib, st, case, reps: int = 50) -> dict:
    """Mixed-condition ghost fill of an arbitrary scalar (Robin, per-ghost g) on the 256^3 ghost set,
    timed with HIP events on the stream it is enqueued on."""
    import ctypes
    import numpy as np
    import torch
    f = torch.tensor(np.random.default_rng(1).standard_normal(case.grid.cells), dtype=torch.float64, device="cuda")
    gv = torch.zeros(st.G, dtype=torch.float64, device="cuda")
    lib = chib.lib
    call = lambda: chib.check(lib.ch_ib_scalar_fill(st.h, ctypes.c_void_p(f.data_ptr()), -2.5, 1.0, 0.0,
                                                    ctypes.c_void_p(gv.data_ptr())))
    call()
    st.sync()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        call()
    e1.record(stream)
    e1.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / reps
    K = 7
    per_ghost = 4 + 2 * K * (4 + 8) + 2 * K * 8 + 2 * 8 + 8 + 8   # tables, gathers, dn, gamma, g, write
    b = st.G * per_ghost
    return {"what": "ghost fill of a scalar under a f + b df/dn = g (Robin, per-ghost g), host checks included",
            "ghosts": st.G, "us_per_call": round(us, 2), "alg_bytes": b, "GB_s": round(b / (us * 1e-6) / 1e9, 1)}


def diagnostics_benchmark(st, case, es: int, reps: int = 20) -> dict:
    """Diagnostics (mass, free energy, max |C|) on the 256^3 state: wall time of the synchronous call,
    which holds both reduction kernels, the 64-byte copy to the host and the wait."""
    st.diagnostics()
    t0 = time.perf_counter()
    for _ in range(reps):
        st.diagnostics()
    us = (time.perf_counter() - t0) * 1e6 / reps
    b = 2 * es * case.grid.cells      # C and alpha, each read once (neighbours from cache)
    return {"what": "synchronous diagnostics call (two reduction kernels, copy to host, wait)",
            "us_per_call": round(us, 2), "alg_bytes": b, "GB_s": round(b / (us * 1e-6) / 1e9, 1),
            "frac_of_8TBs": round(b / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)}


def host_round_trip_benchmark(chib, st, case, ks=(1, 100)) -> dict:
    """Rate when the caller hands C over in host memory: set C from a pageable host array, K steps,
    C back to the host, wall time of the whole.  (Setting C restarts the history, so each K starts
    with the initial fill, as a host-side caller's first step would.)"""
    cells = case.grid.cells
    C_host = st.get(chib.FIELD_C)
    out = {"what": "set C from pageable host memory + K steps + get C to host (wall)"}
    for k in ks:
        st.set(chib.FIELD_C, C_host)
        st.step(1)
        st.sync()
        t0 = time.perf_counter()
        st.set(chib.FIELD_C, C_host)
        st.step(k)
        C_host = st.get(chib.FIELD_C)
        dt = time.perf_counter() - t0
        out[f"K{k}"] = {"ms": round(dt * 1e3, 3), "cell_updates_per_s": cells * k / dt}
    return out


def learned_benchmark(chib, n_angles: int) -> dict:
    """Learned wall-band correction (config 5 with the momentum step on): the first `n_angles` held-out
    contact angles, each on the plain 1024x512 grid (the reference), the plain 512x256 grid and the
    512x256 grid with the committed correction trained on momentum-step runs, 80000 steps of 2.5e-5
    (t = 2); states advance one after another; contact angles from the same cap fit."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2104_00350_amd import learned as LR
    _, eval_a = LR.study_angles()
    coarse = W.config5_flow(False)
    net = chib.Net(coarse.grid.cells, coarse.grid.cells // 256, 1, 1, 0.1, torch.cuda.current_stream())
    net.set_params(np.load(LR.WEIGHTS_FLOW))
    cps = [8000, 20000, 40000, 80000]
    ev = LR.evaluate(net, W.config5_flow, eval_a[:n_angles], 400, cps, 0.5, log=lambda m: None)
    net.close()
    sm = LR.summarize(ev, cps)
    return {"workload": "config 5 with the momentum step: 2D sinusoidal wall y = 0.3 + 0.1 sin(2 pi x / 0.5) in "
                        "[0,4]x[0,2], droplet R = 0.4, Cn = 0.01, Pe = 300, Re = 10, Ca = 0.05, l_s = 0.01, "
                        f"held-out angles {[round(a, 1) for a in eval_a[:n_angles]]}, 80000 steps of dt = 2.5e-5, "
                        "correction every 400 steps at weight 0.5",
            "study_file": "profiles/learned_study_cfg5flow.json (all 8 held-out angles)",
            "speedup_learned_vs_plain_fine": round(sm["speedup_learned_vs_fine"], 3),
            "speedup_plain_coarse_vs_plain_fine": round(sm["speedup_coarse_vs_fine"], 3),
            "seconds": {"fine": round(sm["fine_s"], 3), "coarse": round(sm["coarse_s"], 3),
                        "learned": round(sm["learned_s"], 3)},
            "angle_err_vs_fine_deg": [{"step": p["step"], "cases": p["cases"],
                                       "plain_coarse": p["mean_abs_err_coarse_deg"],
                                       "learned": p["mean_abs_err_learned_deg"],
                                       "fine_vs_prescribed": p["mean_abs_fine_minus_theta_deg"]}
                                      for p in sm["per_checkpoint"]],
            "within_1deg": {"cap_fit_vs_fine": sm["learned_within_1deg_cap_fit"],
                            "fine_at_equilibrium": sm["fine_at_equilibrium"],
                            "equilibrium_target_met": bool(sm["learned_within_1deg_cap_fit"]
                                                           and sm["fine_at_equilibrium"])},
            "fallbacks_to_fine": sm["fallbacks"]}


def geometry_benchmark(chib, torch, case, tabs100, t_dev100: float) -> dict:
    """Geometry preprocessing (one-time, not in the step metric).  The workload's tables use the
    paper's 100 subgrid points per direction (device builder).  The host builder is timed and
    compared bit for bit at 20 points per direction (at 100 it takes about a minute on the host),
    and the tables at 20 are compared with those at 100: how much the coarser count moves the
    volume fractions, normals and wall distances."""
    import dataclasses
    import numpy as np
    g = case.grid
    prm20 = dataclasses.replace(case.params, subgrid=20)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dev20 = chib.Geometry.build_device(g.n, g.lo, g.hi, case.shapes, prm20).export()
    t_dev20 = time.perf_counter() - t0
    t0 = time.perf_counter()
    host20 = chib.Geometry.build(g.n, g.lo, g.hi, case.shapes, prm20).export()
    t_host20 = time.perf_counter() - t0
    same = all(np.array_equal(dev20[k], host20[k]) for k in dev20)
    out = {"subgrid": 100, "device_builder_s": round(t_dev100, 4), "ghosts": int(tabs100["gidx"].size),
           "at_20_subgrid_points": {"device_builder_s": round(t_dev20, 4), "host_builder_s": round(t_host20, 4),
                                    "device_tables_equal_host": same, "ghosts": int(dev20["gidx"].size)}}
    a100, a20 = tabs100["alpha"], dev20["alpha"]
    cmp = {"max_abs_alpha_diff": float(np.max(np.abs(a100 - a20))),
           "cells_with_alpha_diff": int(np.count_nonzero(a100 != a20)),
           "same_ghost_list": bool(np.array_equal(tabs100["gidx"], dev20["gidx"]))}
    if cmp["same_ghost_list"]:
        n1, n2 = tabs100["normal"], dev20["normal"]
        cosang = np.clip(np.sum(n1 * n2, axis=0) / (np.linalg.norm(n1, axis=0) * np.linalg.norm(n2, axis=0)), -1, 1)
        cmp["max_normal_angle_diff_deg"] = float(np.degrees(np.max(np.arccos(cosang))))
        cmp["max_dn_diff_over_h"] = float(np.max(np.abs(tabs100["dn"] - dev20["dn"])) / g.h)
    out["tables_20_vs_100"] = cmp
    return out


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(case, steps: int, steps_one_core: int) -> dict:
    """The FP64 oracle on the host, on a bounded sample (a few steps) of the same workload: scipy's
    FFTs on every host thread, then on one thread (NumPy's stencils are single-threaded either way)."""
    import dataclasses
    import oracle.solver as OS
    from oracle.geometry import build_tables
    # the oracle's tables with 20 subgrid points per direction (at 100 the oracle's counting alone
    # takes a quarter of an hour; the timed steps do the same work either way)
    T = build_tables(case.grid, case.shapes, dataclasses.replace(case.params, subgrid=20))
    C0, faces = case.initial_fields()
    orc = OS.OracleState(case.grid, case.params, T, C0, faces)
    print("[bench] oracle tables built; timing its steps", file=sys.stderr, flush=True)
    orc.step(1)   # warm-up (FFT plans, page faults)
    threads = OS.WORKERS
    t0 = time.perf_counter()
    orc.step(steps)
    dt = time.perf_counter() - t0
    one = None
    if steps_one_core > 0:
        OS.WORKERS = 1
        try:
            t0 = time.perf_counter()
            orc.step(steps_one_core)
            dt1 = time.perf_counter() - t0
        finally:
            OS.WORKERS = threads
        one = {"value": case.grid.cells * steps_one_core / dt1, "cores": 1,
               "sample": f"{steps_one_core} further steps ({dt1:.1f} s)"}
    return {"value": case.grid.cells * steps / dt, "unit": "cell-updates/s", "cores": threads,
            "kind": "oracle", "cpu_model": cpu_model(), "host_threads": os.cpu_count(),
            "sample": f"{steps} steps of the same 256^3 workload after 1 warm-up step, tables counted with 20 "
                      "subgrid points per direction "
                      f"({dt:.1f} s; scipy FFTs on {threads} threads, NumPy stencils single-threaded)",
            "one_core": one}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precision", type=int, default=64, choices=(64, 32))
    ap.add_argument("--n", type=int, default=256, help="cells per axis of the sphere workload")
    ap.add_argument("--cpu-steps", type=int, default=12)
    ap.add_argument("--cpu-steps-one-core", type=int, default=6)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="keep the default launch shapes")
    ap.add_argument("--shapes", default="", help="fixed launch shapes 'a,b,c;d,e,f;g,h,i;j,k,l' instead of tuning")
    ap.add_argument("--sweep-steps", type=int, default=2000, help="steps per case of the batched sweep (0: skip)")
    ap.add_argument("--learned-angles", type=int, default=2,
                    help="held-out angles of the learned-correction comparison, 1..8 (0: skip)")
    ap.add_argument("--explicit-steps", type=int, default=100,
                    help="timed steps of the explicit scheme on the same workload (0: skip)")
    ap.add_argument("--ns-steps", type=int, default=50,
                    help="timed steps with the momentum step (Navier-Stokes coupling) on the same workload (0: skip)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run one plain device copy of this size (for counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(json.dumps({"error": "chib runs on one GPU; runs across several GPUs are not implemented"}))
        return 2

    import numpy as np
    import torch
    import workloads as W
    from paper_2104_00350_amd import chib

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        return 2
    case = W.config3(args.n)
    g = case.grid
    chib.Geometry.build_device(g.n, g.lo, g.hi, case.shapes, case.params)      # loads its kernels
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    geo = chib.Geometry.build_device(g.n, g.lo, g.hi, case.shapes, case.params)   # 100 subgrid points per direction
    t_geom = time.perf_counter() - t0
    st = chib.State(geo, case.params, args.precision)
    C0, faces = case.initial_fields()
    st.set_initial(C0, faces)
    st.step(1)
    if args.shapes:
        st.set_shapes([[int(v) for v in grp.split(",")] for grp in args.shapes.split(";")])
        shapes = st.shapes()
    else:
        shapes = st.shapes() if args.no_tune else st.tune(5)   # launch shapes, chosen before timing
    st.step(max(args.warmup, 1))
    st.sync()
    print(f"[bench] geometry {t_geom:.1f}s, ghosts {st.G}, shapes {shapes}, warmup done", file=sys.stderr,
          flush=True)

    if args.copy_calibration_mib:
        nel = args.copy_calibration_mib * (1 << 20) // 8
        a = torch.ones(nel, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    # the timed region: K plain steps (ch_ib_step) on the state's stream, bracketed by a device
    # synchronisation on both sides; HIP events on that stream give the device time alongside
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(st.stream)
    st.step(args.steps)
    ev1.record(st.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    event_ms = ev0.elapsed_time(ev1)
    # per-kernel breakdown from a separate call with HIP events between the kernels
    ms = st.step_timed(min(args.steps, 100))
    st.sync()
    dg = st.diagnostics()
    if dg["status"] != 0:
        print(json.dumps({"error": "non-finite state after the timed steps"}))
        return 1

    cells = g.cells
    es = 8 if args.precision == 64 else 4
    # faces touching ghosts (the velocity fill's second work list), from the exported tables
    tabs = geo.export()
    nx, ny = g.n[0], g.n[1]
    faces_set = set()
    for c in tabs["gidx"].tolist():
        i, j, k = c % nx, (c // nx) % ny, c // (nx * ny)
        for a_, (di, dj, dk) in enumerate(((1, 0, 0), (0, 1, 0), (0, 0, 1))):
            cm = ((i - di) % nx) + nx * (((j - dj) % ny) + ny * (k - dk))
            faces_set.add((a_, cm))
            faces_set.add((a_, c))
    NF = len(faces_set)

    kernels = {}
    for name, t in ms.items():
        b = algorithmic_bytes(name, cells, 3, es, st.G, NF, case.params.Vs > 0)
        kernels[name] = {"ms": round(t, 5), "alg_bytes": int(b), "GB_s": round(b / (t * 1e-3) / 1e9, 1)}
    dominant = max(ms, key=ms.get)
    dom = kernels[dominant]
    gpu_ms = sum(ms.values())
    value = cells * args.steps / wall
    achieved = dom["alg_bytes"] / (ms[dominant] * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == 64 else "f32",
        "data": "synthetic",
        "config": {"workload": f"3D sphere wall r=1 in [-2,2]^3, {args.n}^3 cells, droplet R=0.5 on top, "
                               "Cn=0.015 Pe=200 Ca=0.05 theta=90 ls=0.01 dt=1e-4, velocity fill on",
                   "grid": list(g.n), "ghosts": st.G, "faces_touching_ghosts": NF,
                   "launch_shapes": shapes},
        "roofline": {"bound": "hbm", "kernel": dominant, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(dominant, shapes, es, tuple(g.n)),
                     "alg_bytes_per_launch": dom["alg_bytes"]},
        "ms_per_step_hip_events": round(event_ms / args.steps, 5),
        "kernel_ms_per_step_sum": round(gpu_ms, 5),
        "kernel_breakdown": f"ch_ib_step_timed over {min(args.steps, 100)} further steps (events between kernels)",
        "path_GB_s": round(sum(k["alg_bytes"] for k in kernels.values()) / (gpu_ms * 1e-3) / 1e9, 1),
        "kernels": kernels,
    }
    out["scalar_fill"] = scalar_fill_benchmark(chib, st, case)
    out["diagnostics"] = diagnostics_benchmark(st, case, es)
    out["host_round_trip"] = host_round_trip_benchmark(chib, st, case)
    out["geometry"] = geometry_benchmark(chib, torch, case, tabs, t_geom)
    if args.explicit_steps > 0:
        print("[bench] explicit scheme", file=sys.stderr, flush=True)
        out["explicit"] = explicit_benchmark(chib, geo, case, args.explicit_steps, args.precision, NF,
                                             out["ms_per_step"])
    if args.ns_steps > 0:
        print("[bench] Navier-Stokes coupling", file=sys.stderr, flush=True)
        out["navier_stokes"] = ns_benchmark(chib, case, args.ns_steps, args.precision, out["ms_per_step"], NF,
                                            st.shapes())
    if args.sweep_steps > 0:
        print("[bench] batched sweep (64 cases)", file=sys.stderr, flush=True)
        out["batched_sweep"] = sweep_benchmark(chib, torch, args.sweep_steps)
    if args.learned_angles > 0:
        print("[bench] learned correction study (config 5 with the momentum step, held-out angles)", file=sys.stderr,
              flush=True)
        out["learned"] = learned_benchmark(chib, min(args.learned_angles, 8))
    if not args.no_cpu_baseline:
        print(f"[bench] GPU done ({value:.3e} cell-updates/s); timing the CPU oracle", file=sys.stderr,
              flush=True)
        out["cpu_baseline"] = cpu_baseline(case, args.cpu_steps, args.cpu_steps_one_core)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
