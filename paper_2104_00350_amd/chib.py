"""Thin ctypes binding of libchib.so (include/ch_ib.h): argument marshalling only.

Every step of the method runs in the HIP library; PyTorch only provides the device
workspace and the stream.  Importing works without a GPU (the library is a plain shared
object); creating a state needs one.  A missing library raises immediately.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libchib.so")

OK, EINVAL, EGEOM, EHIP, ENOMEM, ENAN, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
HALFPLANE, SINUSOID, SPHERE, BOX = 1, 2, 3, 4
FIELD_C, FIELD_C_PREV, FIELD_U, FIELD_V, FIELD_W, FIELD_CI, FIELD_ALPHA, FIELD_PHI, FIELD_P = range(9)
FLAG_VELOCITY_FILL = 1
FLAG_EXPLICIT = 2
FLAG_NAVIER_STOKES = 4
STAGE_RHS, STAGE_SOLVE, STAGE_PHI = 1, 2, 3


class ChibError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"ch_ib error {code}: {msg}")
        self.code = code


class Grid(C.Structure):
    _fields_ = [("ndim", C.c_int), ("n", C.c_int * 3), ("lo", C.c_double * 3), ("hi", C.c_double * 3)]


class Shape(C.Structure):
    _fields_ = [("kind", C.c_int), ("p", C.c_double * 10)]


class Params(C.Structure):
    _fields_ = [("Cn", C.c_double), ("Pe", C.c_double), ("Re", C.c_double), ("Ca", C.c_double),
                ("mu", C.c_double), ("theta_deg", C.c_double), ("Vs", C.c_double),
                ("slip_length", C.c_double), ("dt", C.c_double), ("S", C.c_double),
                ("d1_cells", C.c_double), ("d2_cells", C.c_double), ("subgrid", C.c_int),
                ("precision", C.c_int), ("flags", C.c_int),
                ("rho1", C.c_double), ("rho2", C.c_double), ("mu1", C.c_double), ("mu2", C.c_double),
                ("body_force", C.c_double * 3)]


class GhostTables(C.Structure):
    _fields_ = [("n_ghost", C.c_int64), ("ndim", C.c_int), ("n_ap", C.c_int),
                ("gidx", C.POINTER(C.c_int64)), ("normal", C.POINTER(C.c_double)),
                ("dn", C.POINTER(C.c_double)), ("gamma", C.POINTER(C.c_double)),
                ("ap", C.POINTER(C.c_int64)), ("w", C.POINTER(C.c_double)),
                ("alpha", C.POINTER(C.c_double))]


class Diag(C.Structure):
    _fields_ = [("mass_box", C.c_double), ("mass_fluid", C.c_double), ("free_energy", C.c_double),
                ("max_abs_C", C.c_double), ("step", C.c_int64), ("status", C.c_int), ("pad_", C.c_int)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2104_00350_amd.build.build()")
    # torch ships a HIP runtime with the same soname as the library's dependency: loading torch
    # first makes the library bind to that one runtime, so both share device memory and streams
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64p = C.c_void_p, C.c_int, C.POINTER(C.c_int64)
    sig = {
        "ch_ib_strerror": (C.c_char_p, [i32]),
        "ch_ib_last_error": (C.c_char_p, []),
        "ch_ib_version": (i32, []),
        "ch_ib_geometry_build": (i32, [C.POINTER(Grid), C.POINTER(Shape), i32, C.POINTER(Params), C.POINTER(vp)]),
        "ch_ib_geometry_import": (i32, [C.POINTER(Grid), C.POINTER(GhostTables), C.POINTER(vp)]),
        "ch_ib_geometry_export": (i32, [vp, C.POINTER(GhostTables)]),
        "ch_ib_geometry_count": (i32, [vp, i64p, C.POINTER(C.c_int)]),
        "ch_ib_geometry_free": (None, [vp]),
        "ch_ib_geometry_face_fractions": (i32, [vp, vp]),
        "ch_ib_geometry_set_face_fractions": (i32, [vp, vp]),
        "ch_ib_workspace_bytes": (C.c_size_t, [C.POINTER(Grid), vp, C.POINTER(Params)]),
        "ch_ib_state_create": (i32, [C.POINTER(Grid), vp, C.POINTER(Params), vp, C.c_size_t, vp, C.POINTER(vp)]),
        "ch_ib_state_set": (i32, [vp, i32, vp, i32]),
        "ch_ib_state_get": (i32, [vp, i32, vp, i32]),
        "ch_ib_step": (i32, [vp, i32]),
        "ch_ib_sync": (i32, [vp]),
        "ch_ib_step_timed": (i32, [vp, i32, i32, C.POINTER(C.c_double), C.POINTER(C.c_char_p),
                                   C.POINTER(C.c_int)]),
        "ch_ib_diagnostics": (i32, [vp, C.POINTER(Diag)]),
        "ch_ib_diagnostics_noalloc": (i32, [vp, C.POINTER(Diag)]),
        "ch_ib_tune": (i32, [vp, i32, C.POINTER(C.c_int)]),
        "ch_ib_get_shapes": (i32, [vp, C.POINTER(C.c_int)]),
        "ch_ib_set_shapes": (i32, [vp, C.POINTER(C.c_int)]),
        "ch_ib_stage": (i32, [vp, i32, vp, vp]),
        "ch_ib_geometry_device_bytes": (C.c_size_t, [vp]),
        "ch_ib_geometry_build_device": (i32, [vp, vp, i32, vp, vp, C.c_size_t, vp, C.POINTER(vp)]),
        "ch_ib_scalar_fill": (i32, [vp, vp, C.c_double, C.c_double, C.c_double, vp]),
        "ch_ib_state_save": (i32, [vp, vp, C.POINTER(C.c_size_t)]),
        "ch_ib_state_load": (i32, [vp, vp, C.c_size_t]),
        "ch_ib_state_free": (None, [vp]),
        "ch_ib_coefficients": (i32, [C.POINTER(Params), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                     C.POINTER(C.c_double)]),
        "ch_ib_batch_workspace_bytes": (C.c_size_t, [i32]),
        "ch_ib_batch_create": (i32, [C.POINTER(vp), i32, vp, C.c_size_t, vp, C.POINTER(vp)]),
        "ch_ib_batch_step": (i32, [vp, i32]),
        "ch_ib_batch_tune": (i32, [vp, i32, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
        "ch_ib_batch_sync": (i32, [vp]),
        "ch_ib_batch_free": (None, [vp]),
        "ch_ib_wall_field": (i32, [C.POINTER(Grid), C.POINTER(Shape), i32, vp, vp]),
        "ch_ib_net_workspace_bytes": (C.c_size_t, [C.c_int64, i32, C.c_int64, i32]),
        "ch_ib_net_create": (i32, [C.c_int64, i32, C.c_int64, i32, C.c_double, vp, C.c_size_t, vp, C.POINTER(vp)]),
        "ch_ib_net_set_params": (i32, [vp, vp]),
        "ch_ib_net_get_params": (i32, [vp, vp]),
        "ch_ib_net_bind": (i32, [vp, vp, vp, vp, C.c_double, C.POINTER(C.c_int)]),
        "ch_ib_net_forward": (i32, [vp, vp]),
        "ch_ib_net_apply": (i32, [vp, C.c_double]),
        "ch_ib_net_rebind": (i32, [vp, vp]),
        "ch_ib_net_extract": (i32, [vp, vp, C.c_int64, vp]),
        "ch_ib_net_store_get": (i32, [vp, C.c_int64, vp, vp, vp]),
        "ch_ib_net_train_step": (i32, [vp, vp, i32, C.c_double, C.c_double, C.POINTER(C.c_double)]),
        "ch_ib_net_gradient": (i32, [vp, vp, i32, C.c_double, vp, C.POINTER(C.c_double)]),
        "ch_ib_restrict2": (i32, [vp, vp, i32]),
        "ch_ib_net_free": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


def check(rc: int) -> None:
    if rc != OK:
        raise ChibError(rc, lib.ch_ib_last_error().decode() or lib.ch_ib_strerror(rc).decode())


def make_grid(n: Sequence[int], lo: Sequence[float], hi: Sequence[float]) -> Grid:
    g = Grid()
    g.ndim = len(n)
    for a in range(3):
        g.n[a] = int(n[a]) if a < len(n) else 1
        g.lo[a] = float(lo[a]) if a < len(n) else 0.0
        g.hi[a] = float(hi[a]) if a < len(n) else 1.0
    return g


def make_params(prm, precision: int = 64) -> Params:
    p = Params()
    for name in ("Cn", "Pe", "Re", "Ca", "mu", "theta_deg", "Vs", "slip_length", "dt", "S",
                 "d1_cells", "d2_cells"):
        setattr(p, name, float(getattr(prm, name)))
    p.subgrid = int(prm.subgrid)
    p.precision = int(precision)
    ns = bool(getattr(prm, "navier_stokes", False))
    p.flags = ((FLAG_VELOCITY_FILL if prm.velocity_fill else 0) | (FLAG_EXPLICIT if getattr(prm, "explicit", False) else 0)
               | (FLAG_NAVIER_STOKES if ns else 0))
    for name in ("rho1", "rho2", "mu1", "mu2"):
        setattr(p, name, float(getattr(prm, name, 1.0)))
    bf = tuple(getattr(prm, "body_force", (0.0, 0.0, 0.0))) + (0.0, 0.0, 0.0)
    for a in range(3):
        p.body_force[a] = float(bf[a])
    return p


def make_shapes(shapes) -> "C.Array":
    arr = (Shape * max(1, len(shapes)))()
    for i, s in enumerate(shapes):
        arr[i].kind = int(s.kind)
        for k, v in enumerate(s.padded()):
            arr[i].p[k] = float(v)
    return arr


def coefficients(prm) -> tuple:
    p = make_params(prm)
    S, al, a = C.c_double(), C.c_double(), C.c_double()
    check(lib.ch_ib_coefficients(C.byref(p), C.byref(S), C.byref(al), C.byref(a)))
    return S.value, al.value, a.value


class Geometry:
    """Host-side ghost tables (ch_ib_geometry)."""

    def __init__(self, handle: int, grid: Grid):
        self.h = C.c_void_p(handle)
        self.grid = grid

    @classmethod
    def build(cls, n, lo, hi, shapes, prm) -> "Geometry":
        g = make_grid(n, lo, hi)
        sh = make_shapes(shapes)
        p = make_params(prm)
        out = C.c_void_p()
        check(lib.ch_ib_geometry_build(C.byref(g), sh, len(shapes), C.byref(p), C.byref(out)))
        return cls(out.value, g)

    @classmethod
    def build_device(cls, n, lo, hi, shapes, prm, device: str = "cuda:0", stream=None) -> "Geometry":
        """The same tables computed on the GPU (ch_ib_geometry_build_device), in a torch-owned
        scratch buffer that is released afterwards."""
        import torch
        g = make_grid(n, lo, hi)
        sh = make_shapes(shapes)
        p = make_params(prm)
        nbytes = lib.ch_ib_geometry_device_bytes(C.byref(g))
        if not nbytes:      # a bad grid: the builder itself reports why
            check(lib.ch_ib_geometry_build_device(C.byref(g), sh, len(shapes), C.byref(p), None, 0, None,
                                                  C.byref(C.c_void_p())))
        buf = torch.empty(nbytes, dtype=torch.uint8, device=device)
        ptr = (buf.data_ptr() + 255) // 256 * 256
        st = stream if stream is not None else torch.cuda.current_stream(device)
        out = C.c_void_p()
        check(lib.ch_ib_geometry_build_device(C.byref(g), sh, len(shapes), C.byref(p), C.c_void_p(ptr),
                                              nbytes - (ptr - buf.data_ptr()), C.c_void_p(st.cuda_stream),
                                              C.byref(out)))
        del buf
        return cls(out.value, g)

    @classmethod
    def from_tables(cls, n, lo, hi, gidx, normal, dn, gamma, ap, w, alpha=None) -> "Geometry":
        g = make_grid(n, lo, hi)
        d = len(n)
        keep = [np.ascontiguousarray(gidx, dtype=np.int64), np.ascontiguousarray(normal, dtype=np.float64),
                np.ascontiguousarray(dn, dtype=np.float64), np.ascontiguousarray(gamma, dtype=np.float64),
                np.ascontiguousarray(ap, dtype=np.int64), np.ascontiguousarray(w, dtype=np.float64)]
        t = GhostTables()
        t.n_ghost = keep[0].size
        t.ndim = d
        t.n_ap = 2 * d + 1
        t.gidx = keep[0].ctypes.data_as(C.POINTER(C.c_int64))
        t.normal = keep[1].ctypes.data_as(C.POINTER(C.c_double))
        t.dn = keep[2].ctypes.data_as(C.POINTER(C.c_double))
        t.gamma = keep[3].ctypes.data_as(C.POINTER(C.c_double))
        t.ap = keep[4].ctypes.data_as(C.POINTER(C.c_int64))
        t.w = keep[5].ctypes.data_as(C.POINTER(C.c_double))
        if alpha is not None:
            al = np.ascontiguousarray(alpha, dtype=np.float64).reshape(-1)
            keep.append(al)
            t.alpha = al.ctypes.data_as(C.POINTER(C.c_double))
        out = C.c_void_p()
        check(lib.ch_ib_geometry_import(C.byref(g), C.byref(t), C.byref(out)))
        return cls(out.value, g)

    def count(self):
        G = C.c_int64()
        K = C.c_int()
        check(lib.ch_ib_geometry_count(self.h, C.byref(G), C.byref(K)))
        return G.value, K.value

    def face_fractions(self) -> np.ndarray:
        """Staggered-cell fluid fractions, shape (d,) + field shape (ch_ib_geometry_face_fractions)."""
        d = self.grid.ndim
        shape = tuple(self.grid.n[a] for a in reversed(range(d)))
        out = np.zeros((d,) + shape)
        check(lib.ch_ib_geometry_face_fractions(self.h, out.ctypes.data_as(C.c_void_p)))
        return out

    def set_face_fractions(self, fractions) -> None:
        """Attach staggered-cell fractions (d fields), e.g. to an imported geometry."""
        arr = np.ascontiguousarray(np.stack([np.asarray(f, dtype=np.float64) for f in fractions]))
        check(lib.ch_ib_geometry_set_face_fractions(self.h, arr.ctypes.data_as(C.c_void_p)))

    def export(self) -> dict:
        G, K = self.count()
        d = self.grid.ndim
        cells = int(np.prod([self.grid.n[a] for a in range(d)]))
        arrs = {"gidx": np.zeros(G, np.int64), "normal": np.zeros((d, G)), "dn": np.zeros(G),
                "gamma": np.zeros(G), "ap": np.zeros((2, K, G), np.int64), "w": np.zeros((2, K, G)),
                "alpha": np.zeros(cells)}
        t = GhostTables()
        t.n_ghost, t.ndim, t.n_ap = G, d, K
        t.gidx = arrs["gidx"].ctypes.data_as(C.POINTER(C.c_int64))
        t.normal = arrs["normal"].ctypes.data_as(C.POINTER(C.c_double))
        t.dn = arrs["dn"].ctypes.data_as(C.POINTER(C.c_double))
        t.gamma = arrs["gamma"].ctypes.data_as(C.POINTER(C.c_double))
        t.ap = arrs["ap"].ctypes.data_as(C.POINTER(C.c_int64))
        t.w = arrs["w"].ctypes.data_as(C.POINTER(C.c_double))
        t.alpha = arrs["alpha"].ctypes.data_as(C.POINTER(C.c_double))
        check(lib.ch_ib_geometry_export(self.h, C.byref(t)))
        return arrs

    def __del__(self):
        try:
            if self.h:
                lib.ch_ib_geometry_free(self.h)
                self.h = None
        except Exception:
            pass


class State:
    """One simulation state in a torch-owned device workspace, on torch's current stream."""

    def __init__(self, geom: Geometry, prm, precision: int = 64, device: str = "cuda:0", stream=None):
        import torch
        self.torch = torch
        self.geom = geom
        self.grid = geom.grid
        self.d = self.grid.ndim
        self.n = tuple(self.grid.n[a] for a in range(self.d))
        self.cells = int(np.prod(self.n))
        self.precision = precision
        self.np_dtype = np.float64 if precision == 64 else np.float32
        self.torch_dtype = torch.float64 if precision == 64 else torch.float32
        self.params = make_params(prm, precision)
        nbytes = lib.ch_ib_workspace_bytes(C.byref(self.grid), geom.h, C.byref(self.params))
        if nbytes == 0:
            raise ChibError(EINVAL, "workspace size query failed")
        self.device = torch.device(device)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        ptr = self.workspace.data_ptr()
        self._ws_ptr = ptr + ((-ptr) % 256)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        out = C.c_void_p()
        check(lib.ch_ib_state_create(C.byref(self.grid), geom.h, C.byref(self.params), C.c_void_p(self._ws_ptr),
                                     nbytes, C.c_void_p(self.stream.cuda_stream), C.byref(out)))
        self.h = out
        self.G = geom.count()[0]

    # fields -------------------------------------------------------------------------
    def _count(self, field):
        return self.G if field == FIELD_CI else self.cells

    def set(self, field: int, values) -> None:
        torch = self.torch
        if isinstance(values, torch.Tensor):
            t = values.to(device=self.device, dtype=self.torch_dtype).contiguous()
            if t.numel() != self._count(field):
                raise ValueError("wrong number of values")
            check(lib.ch_ib_state_set(self.h, field, C.c_void_p(t.data_ptr()), 1))
            return
        a = np.ascontiguousarray(values, dtype=self.np_dtype).reshape(-1)
        if a.size != self._count(field):
            raise ValueError("wrong number of values")
        check(lib.ch_ib_state_set(self.h, field, a.ctypes.data_as(C.c_void_p), 0))

    def get(self, field: int) -> np.ndarray:
        out = np.empty(self._count(field), dtype=self.np_dtype)
        check(lib.ch_ib_state_get(self.h, field, out.ctypes.data_as(C.c_void_p), 0))
        if field == FIELD_CI:
            return out
        return out.reshape(tuple(reversed(self.n)))

    def get_device(self, field: int):
        t = self.torch.empty(self._count(field), dtype=self.torch_dtype, device=self.device)
        check(lib.ch_ib_state_get(self.h, field, C.c_void_p(t.data_ptr()), 1))
        return t

    def set_initial(self, C0, faces: Optional[Sequence] = None) -> None:
        if faces is not None:
            for a, f in enumerate(faces):
                self.set(FIELD_U + a, f)
        self.set(FIELD_C, C0)

    # stepping -----------------------------------------------------------------------
    def step(self, n: int = 1) -> None:
        check(lib.ch_ib_step(self.h, int(n)))

    def sync(self) -> None:
        check(lib.ch_ib_sync(self.h))

    def tune(self, reps: int = 5) -> list:
        """Autotunes the launch shapes of the four field passes; returns them (4 x [log_tile, radix, unroll])."""
        out = (C.c_int * 12)()
        check(lib.ch_ib_tune(self.h, int(reps), out))
        return [list(out[3 * k:3 * k + 3]) for k in range(4)]

    def shapes(self) -> list:
        out = (C.c_int * 12)()
        check(lib.ch_ib_get_shapes(self.h, out))
        return [list(out[3 * k:3 * k + 3]) for k in range(4)]

    def set_shapes(self, shapes) -> None:
        flat = (C.c_int * 12)(*[int(v) for row in shapes for v in row])
        check(lib.ch_ib_set_shapes(self.h, flat))

    def step_timed(self, n: int) -> dict:
        """Runs n steps with HIP events between kernels; returns {kernel name: mean ms per step}."""
        ms = (C.c_double * 16)()
        names = (C.c_char_p * 16)()
        nk = C.c_int()
        check(lib.ch_ib_step_timed(self.h, int(n), 16, ms, names, C.byref(nk)))
        return {names[k].decode(): ms[k] for k in range(nk.value)}

    def diagnostics(self) -> dict:
        dg = Diag()
        rc = lib.ch_ib_diagnostics(self.h, C.byref(dg))
        if rc not in (OK, ENAN):
            check(rc)
        return {"mass_box": dg.mass_box, "mass_fluid": dg.mass_fluid, "free_energy": dg.free_energy,
                "max_abs_C": dg.max_abs_C, "step": dg.step, "status": dg.status}

    def diagnostics_noalloc(self) -> dict:
        """The same values through ch_ib_diagnostics_noalloc (the library's fixed device scratch)."""
        dg = Diag()
        rc = lib.ch_ib_diagnostics_noalloc(self.h, C.byref(dg))
        if rc not in (OK, ENAN):
            check(rc)
        return {"mass_box": dg.mass_box, "mass_fluid": dg.mass_fluid, "free_energy": dg.free_energy,
                "max_abs_C": dg.max_abs_C, "step": dg.step, "status": dg.status}

    def stage(self, stage: int, inp=None):
        torch = self.torch
        out = torch.empty(self.cells, dtype=self.torch_dtype, device=self.device)
        ip = None
        if inp is not None:
            t = torch.as_tensor(np.ascontiguousarray(inp).reshape(-1)) if not isinstance(inp, torch.Tensor) else inp
            t = t.to(device=self.device, dtype=self.torch_dtype).contiguous()
            ip = C.c_void_p(t.data_ptr())
        check(lib.ch_ib_stage(self.h, stage, ip, C.c_void_p(out.data_ptr())))
        return out.cpu().numpy().reshape(tuple(reversed(self.n)))

    def scalar_fill(self, field, a: float, b: float, g: float = 0.0, g_ghost=None):
        """Ghost values of `field` (one value per cell) under a f + b df/dn = g at the wall (uniform g,
        or one value per ghost in `g_ghost`).  A device tensor of the state's dtype is filled in place
        and returned; anything else is copied to the device, filled and returned as a numpy array."""
        torch = self.torch
        in_place = isinstance(field, torch.Tensor) and field.device.type == "cuda" and field.dtype == self.torch_dtype \
            and field.is_contiguous() and field.numel() == self.cells
        t = field if in_place else torch.as_tensor(np.ascontiguousarray(field, dtype=np.float64).reshape(-1)).to(
            device=self.device, dtype=self.torch_dtype).contiguous()
        gp = None
        if g_ghost is not None:
            gt = torch.as_tensor(np.ascontiguousarray(g_ghost, dtype=np.float64).reshape(-1)).to(
                device=self.device, dtype=self.torch_dtype).contiguous()
            if gt.numel() != self.G:
                raise ChibError(EINVAL, "g_ghost needs one value per ghost")
            gp = C.c_void_p(gt.data_ptr())
        check(lib.ch_ib_scalar_fill(self.h, C.c_void_p(t.data_ptr()), float(a), float(b), float(g), gp))
        check(lib.ch_ib_sync(self.h))
        if in_place:
            return field
        return t.cpu().numpy().astype(np.float64).reshape(tuple(reversed(self.n)))

    def save(self) -> bytes:
        n = C.c_size_t()
        check(lib.ch_ib_state_save(self.h, None, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        check(lib.ch_ib_state_save(self.h, buf, C.byref(n)))
        return buf.raw[: n.value]

    def load(self, blob: bytes) -> None:
        check(lib.ch_ib_state_load(self.h, blob, len(blob)))

    def close(self) -> None:
        if getattr(self, "h", None):
            lib.ch_ib_state_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def state_for_case(case, precision: int = 64, geom: Optional[Geometry] = None) -> State:
    """Builds the geometry with the library (unless given) and a state with the case's initial fields."""
    g = case.grid
    if geom is None:
        geom = Geometry.build(g.n, g.lo, g.hi, case.shapes, case.params)
    st = State(geom, case.params, precision)
    C0, faces = case.initial_fields()
    st.set_initial(C0, faces)
    return st


class Batch:
    """Independent 2D states advanced together: grouped launches per phase, replayed as a hipGraph."""

    def __init__(self, states, stream=None):
        import torch
        self.torch = torch
        self.states = list(states)
        n = len(self.states)
        nbytes = lib.ch_ib_batch_workspace_bytes(n)
        dev = self.states[0].device
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        ptr = self.workspace.data_ptr()
        ptr += (-ptr) % 256
        # a stream of its own (default priority): graphs cannot be captured on the NULL stream
        self.stream = stream if stream is not None else torch.cuda.Stream(device=dev)
        handles = (C.c_void_p * n)(*[s.h.value for s in self.states])
        out = C.c_void_p()
        check(lib.ch_ib_batch_create(handles, n, C.c_void_p(ptr), nbytes, C.c_void_p(self.stream.cuda_stream),
                                     C.byref(out)))
        self.h = out

    def step(self, n: int = 1) -> None:
        check(lib.ch_ib_batch_step(self.h, int(n)))

    def sync(self) -> None:
        check(lib.ch_ib_batch_sync(self.h))

    def tune(self, reps: int = 3):
        radix = (C.c_int * 3)()
        unroll = C.c_int()
        check(lib.ch_ib_batch_tune(self.h, int(reps), radix, C.byref(unroll)))
        return list(radix), unroll.value

    def close(self) -> None:
        if getattr(self, "h", None):
            lib.ch_ib_batch_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# -- learned wall-band correction (2D) ----------------------------------------------------------
NET_NPARAMS = 14177
NET_TILE = 16
NET_PATCH = 22 * 22 * 16


def wall_field(n, lo, hi, shapes):
    """Signed wall distance (ny, nx) and unit wall normal (2, ny, nx) of a 2D grid (host)."""
    g = make_grid(n, lo, hi)
    sh = make_shapes(shapes)
    cells = int(n[0]) * int(n[1])
    dist = np.empty(cells)
    nrm = np.empty(2 * cells)
    check(lib.ch_ib_wall_field(C.byref(g), sh, len(shapes), dist.ctypes.data_as(C.c_void_p),
                               nrm.ctypes.data_as(C.c_void_p)))
    return dist.reshape(n[1], n[0]), nrm.reshape(2, n[1], n[0])


class Net:
    """The correction network and its sample store in a torch-owned device workspace."""

    def __init__(self, max_cells: int, max_tiles: int, max_store_tiles: int, max_batch: int,
                 out_scale: float, stream, device: str = "cuda:0"):
        import torch
        self.torch = torch
        nbytes = lib.ch_ib_net_workspace_bytes(int(max_cells), int(max_tiles), int(max_store_tiles), int(max_batch))
        if nbytes == 0:
            raise ChibError(EINVAL, "network workspace size query failed")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=torch.device(device))
        ptr = self.workspace.data_ptr()
        ptr += (-ptr) % 256
        self.stream = stream
        out = C.c_void_p()
        check(lib.ch_ib_net_create(int(max_cells), int(max_tiles), int(max_store_tiles), int(max_batch),
                                   float(out_scale), C.c_void_p(ptr), nbytes, C.c_void_p(stream.cuda_stream),
                                   C.byref(out)))
        self.h = out
        self.n_tiles = 0
        self.out_scale = out_scale

    def set_params(self, params) -> None:
        a = np.ascontiguousarray(params, dtype=np.float32)
        if a.size != NET_NPARAMS:
            raise ValueError("wrong number of parameters")
        check(lib.ch_ib_net_set_params(self.h, a.ctypes.data_as(C.c_void_p)))

    def get_params(self) -> np.ndarray:
        a = np.empty(NET_NPARAMS, dtype=np.float32)
        check(lib.ch_ib_net_get_params(self.h, a.ctypes.data_as(C.c_void_p)))
        return a

    def bind(self, state: State, dist, normal, band_cells: float) -> int:
        d = np.ascontiguousarray(dist, dtype=np.float64)
        nn = np.ascontiguousarray(normal, dtype=np.float64)
        nt = C.c_int()
        check(lib.ch_ib_net_bind(self.h, state.h, d.ctypes.data_as(C.c_void_p), nn.ctypes.data_as(C.c_void_p),
                                 float(band_cells), C.byref(nt)))
        self.state = state
        self.n_tiles = nt.value
        return nt.value

    def forward(self) -> np.ndarray:
        """dC of the band tiles ([n_tiles, 16, 16], 0 outside the band) for the bound state."""
        t = self.torch.zeros(max(1, self.n_tiles) * NET_TILE * NET_TILE, dtype=self.torch.float32,
                             device=self.workspace.device)
        check(lib.ch_ib_net_forward(self.h, C.c_void_p(t.data_ptr())))
        self.stream.synchronize()
        return t.cpu().numpy()[: self.n_tiles * 256].reshape(self.n_tiles, NET_TILE, NET_TILE)

    def apply(self, weight: float = 1.0) -> None:
        check(lib.ch_ib_net_apply(self.h, float(weight)))

    def rebind(self, state: State) -> None:
        """Switches to another state on the same grid and wall (no copies)."""
        check(lib.ch_ib_net_rebind(self.h, state.h))
        self.state = state

    def extract(self, target_device, store_offset: int) -> np.ndarray:
        """One sample per band tile at store_offset..; returns the tiles' band-cell counts."""
        counts = np.zeros(max(1, self.n_tiles), dtype=np.float32)
        check(lib.ch_ib_net_extract(self.h, C.c_void_p(target_device.data_ptr()), int(store_offset),
                                    counts.ctypes.data_as(C.c_void_p)))
        return counts[: self.n_tiles]

    def store_get(self, slot: int):
        X = np.empty(NET_PATCH, dtype=np.uint16)
        Y = np.empty(256, dtype=np.float32)
        M = np.empty(256, dtype=np.float32)
        check(lib.ch_ib_net_store_get(self.h, int(slot), X.ctypes.data_as(C.c_void_p),
                                      Y.ctypes.data_as(C.c_void_p), M.ctypes.data_as(C.c_void_p)))
        Xf = (X.astype(np.uint32) << 16).view(np.float32).astype(np.float64).reshape(22, 22, 16)
        return np.transpose(Xf, (2, 0, 1)), Y.reshape(16, 16).astype(np.float64), M.reshape(16, 16).astype(np.float64)

    def train_step(self, ids, lr: float, inv_count: float, want_loss: bool = False):
        a = np.ascontiguousarray(ids, dtype=np.int64)
        loss = C.c_double()
        check(lib.ch_ib_net_train_step(self.h, a.ctypes.data_as(C.c_void_p), a.size, float(lr), float(inv_count),
                                       C.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def gradient(self, ids, inv_count: float):
        a = np.ascontiguousarray(ids, dtype=np.int64)
        g = np.empty(NET_NPARAMS, dtype=np.float32)
        loss = C.c_double()
        check(lib.ch_ib_net_gradient(self.h, a.ctypes.data_as(C.c_void_p), a.size, float(inv_count),
                                     g.ctypes.data_as(C.c_void_p), C.byref(loss)))
        return loss.value, g

    def close(self) -> None:
        if getattr(self, "h", None):
            lib.ch_ib_net_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def restrict2(fine: State, coarse: State, both_levels: bool = False) -> None:
    """Coarse C := 2x2 means of the fine C (and C_prev too with both_levels, keeping the history);
    otherwise the coarse state restarts from C at its next step."""
    check(lib.ch_ib_restrict2(fine.h, coarse.h, int(both_levels)))
