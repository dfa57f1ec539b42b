"""Seeded synthetic workloads: grids, wall shapes, parameters and initial fields.

This module is the only code shared by the oracle and the device library's
Python binding.  It holds no arithmetic of the method itself: it only states
the problem (box, wall shape parameters, dimensionless groups) and draws the
initial order-parameter field and face velocities from a seeded generator, so
that both sides start from bit-identical inputs.

Wall shapes are described by a kind code and up to ten numbers; the meaning of
the numbers is the one documented in ``include/ch_ib.h``:

* ``HALFPLANE``: p[0:3] a point on the wall, p[3:6] the wall normal pointing
  into the fluid.  Solid where (x - p) . n < 0.
* ``SINUSOID``: p[0] mean height, p[1] amplitude, p[2] wavelength, p[3] phase
  (radians).  Solid where the wall-normal (last) coordinate lies below
  mean + amplitude * sin(2 pi x / wavelength + phase).
* ``SPHERE``: p[0:3] centre, p[3] radius (a circle in 2D).  Solid inside.
* ``BOX``: p[0:3] centre, p[3] half edge, p[4] rotation angle (radians, in the
  x-y plane).  Fluid inside the rotated square/cube, solid outside.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

HALFPLANE = 1
SINUSOID = 2
SPHERE = 3
BOX = 4


@dataclasses.dataclass
class Shape:
    kind: int
    p: Tuple[float, ...]

    def padded(self) -> List[float]:
        v = list(self.p) + [0.0] * (10 - len(self.p))
        return v[:10]


@dataclasses.dataclass
class Grid:
    """Uniform Cartesian box; axis 0 (x) is stored fastest.

    All axes but the last are periodic; the last axis is bounded by two flat
    box walls (Neumann for the order parameter, no penetration for velocity).
    """

    n: Tuple[int, ...]
    lo: Tuple[float, ...]
    hi: Tuple[float, ...]

    @property
    def ndim(self) -> int:
        return len(self.n)

    @property
    def h(self) -> float:
        return (self.hi[0] - self.lo[0]) / self.n[0]

    @property
    def shape(self) -> Tuple[int, ...]:
        """NumPy array shape of a cell field (x last, i.e. fastest)."""
        return tuple(reversed(self.n))

    @property
    def cells(self) -> int:
        return int(np.prod(self.n))


@dataclasses.dataclass
class Params:
    """Dimensionless groups and method options of one run.

    ``Vs == 0`` selects the static contact-angle condition (no contact-line
    friction); ``S <= 0`` selects the smallest stabilisation parameter that
    keeps the two Helmholtz factors real.  ``d1_cells``/``d2_cells`` are the
    intersect-to-mirror and mirror-to-interpolation distances in cell widths
    (``d1_cells <= 0`` means 2 cells, ``d2_cells <= 0`` 1.5 cells).
    With ``navier_stokes`` the face velocities follow the momentum equation
    (Reynolds number ``Re``, capillary number ``Ca``, phase densities and
    viscosities ``rho1``/``mu1`` for C = -1 and ``rho2``/``mu2`` for C = +1
    relative to the reference fluid, ``body_force`` an acceleration).
    """

    Cn: float
    Pe: float
    Re: float = 10.0
    Ca: float = 0.1
    mu: float = 1.0
    theta_deg: float = 90.0
    Vs: float = 0.0
    slip_length: float = 0.0
    dt: float = 1e-4
    S: float = 0.0
    d1_cells: float = 0.0
    d2_cells: float = 0.0
    subgrid: int = 0           # 0: 100 per direction
    velocity_fill: bool = True
    explicit: bool = False     # explicit Adams-Bashforth step instead of the semi-implicit one
    navier_stokes: bool = False  # advance the face velocities with the momentum equation too
    rho1: float = 1.0          # density of the C = -1 phase over the reference density
    rho2: float = 1.0          # density of the C = +1 phase over the reference density
    mu1: float = 1.0           # viscosity of the C = -1 phase over the reference viscosity
    mu2: float = 1.0           # viscosity of the C = +1 phase over the reference viscosity
    body_force: Tuple[float, ...] = (0.0, 0.0, 0.0)   # acceleration per axis (e.g. gravity)


@dataclasses.dataclass
class Case:
    name: str
    grid: Grid
    shapes: List[Shape]
    params: Params
    steps: int
    droplet_centre: Tuple[float, ...]
    droplet_radius: float
    noise: float
    seed: Optional[int]

    def initial_fields(self) -> Tuple[np.ndarray, List[np.ndarray]]:
        """Initial order parameter on every cell (solid included) and face velocities.

        C0 = tanh((R - r) / (sqrt(2) Cn)) plus seeded uniform noise; the face
        velocities start at rest.
        """
        return droplet_field(self.grid, self.droplet_centre, self.droplet_radius,
                             self.params.Cn, self.noise, self.seed)


def cell_centres(grid: Grid) -> List[np.ndarray]:
    """Broadcastable cell-centre coordinates, one array per axis (x first)."""
    out = []
    h = grid.h
    for a in range(grid.ndim):
        c = grid.lo[a] + (np.arange(grid.n[a], dtype=np.float64) + 0.5) * h
        shp = [1] * grid.ndim
        shp[grid.ndim - 1 - a] = grid.n[a]
        out.append(c.reshape(shp))
    return out


def droplet_field(grid: Grid, centre: Sequence[float], radius: float, Cn: float,
                  noise: float, seed: Optional[int]):
    xs = cell_centres(grid)
    r2 = np.zeros(grid.shape)
    for a in range(grid.ndim):
        r2 = r2 + (xs[a] - centre[a]) ** 2
    r = np.sqrt(r2)
    C0 = np.tanh((radius - r) / (math.sqrt(2.0) * Cn))
    if noise > 0.0:
        rng = np.random.default_rng(seed)
        C0 = C0 + rng.uniform(-noise, noise, size=grid.shape)
    faces = [np.zeros(grid.shape) for _ in range(grid.ndim)]
    return np.ascontiguousarray(C0), faces


# ---------------------------------------------------------------------------
# The workloads named by the configurations of this project.

def config1() -> Case:
    """2D flat wall at y = 0.1, 128 x 64 on [0,2] x [0,1], 60 degrees, 200 steps."""
    g = Grid((128, 64), (0.0, 0.0), (2.0, 1.0))
    prm = Params(Cn=0.02, Pe=100.0, Re=10.0, Ca=0.1, theta_deg=60.0,
                 slip_length=0.01, dt=1e-4)
    return Case("cfg1_flat_128x64", g, [Shape(HALFPLANE, (0.0, 0.1, 0.0, 0.0, 1.0, 0.0))],
                prm, 200, (1.0, 0.1), 0.25, 1e-3, 1)


def config2(i: int = 0) -> Case:
    """2D sinusoidal wall, 512 x 256 on [0,4] x [0,2]; case i of the six (angle, slip) pairs."""
    angles = (45.0, 90.0, 135.0)
    slips = (0.005, 0.02)
    th = angles[i // 2]
    ls = slips[i % 2]
    g = Grid((512, 256), (0.0, 0.0), (4.0, 2.0))
    prm = Params(Cn=0.01, Pe=300.0, Re=10.0, Ca=0.05, theta_deg=th,
                 slip_length=ls, dt=1e-4)
    return Case(f"cfg2_sin_512x256_th{int(th)}_ls{ls}", g,
                [Shape(SINUSOID, (0.3, 0.1, 0.5, 0.0))], prm, 5000,
                (2.125, 0.4), 0.4, 1e-3, 2 + i)


def config3(n: int = 256) -> Case:
    """3D solid sphere r=1 at the origin of [-2,2]^3, droplet R=0.5 on its top."""
    g = Grid((n, n, n), (-2.0, -2.0, -2.0), (2.0, 2.0, 2.0))
    prm = Params(Cn=0.015, Pe=200.0, Re=5.0, Ca=0.05, theta_deg=90.0,
                 slip_length=0.01, dt=1e-4)
    return Case(f"cfg3_sphere_{n}cubed", g, [Shape(SPHERE, (0.0, 0.0, 0.0, 1.0))], prm, 2000,
                (0.0, 0.0, 1.5), 0.5, 0.0, None)


def config4_cases(count: int = 64, seed: int = 2021) -> List[Case]:
    """Uneven-size sinusoidal-wall parameter sweep (all parameters drawn from one seed)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        nx = int(rng.choice([128, 256, 512, 1024]))
        amp = float(rng.uniform(0.02, 0.15))
        lam = float(rng.uniform(0.25, 1.0))
        th = float(rng.uniform(30.0, 150.0))
        ls = float(10.0 ** rng.uniform(-3.0, -1.0))
        lam_p = 2.0 / round(2.0 / lam)
        g = Grid((nx, nx // 2), (0.0, 0.0), (2.0, 1.0))
        h = g.h
        prm = Params(Cn=2.5 * h, Pe=300.0, Re=10.0, Ca=0.05, theta_deg=th,
                     slip_length=ls, dt=1e-4)
        yw = 0.25 + amp * math.sin(2.0 * math.pi * 1.0 / lam_p)
        out.append(Case(f"cfg4_{i:02d}_{nx}", g,
                        [Shape(SINUSOID, (0.25, amp, lam_p, 0.0))], prm, 2000,
                        (1.0, yw), 0.4, 1e-3, seed * 1000 + i))
    return out


def config5(fine: bool, theta_deg: float = 60.0, seed: int = 2104) -> Case:
    """Coarse (512 x 256) or fine (1024 x 512) sinusoidal-wall run of the learned-correction study."""
    n = (1024, 512) if fine else (512, 256)
    g = Grid(n, (0.0, 0.0), (4.0, 2.0))
    prm = Params(Cn=0.01, Pe=300.0, Re=10.0, Ca=0.05, theta_deg=theta_deg,
                 slip_length=0.01, dt=1e-4)
    return Case(f"cfg5_{'fine' if fine else 'coarse'}_th{theta_deg:.1f}", g,
                [Shape(SINUSOID, (0.3, 0.1, 0.5, 0.0))], prm, 20000,
                (2.125, 0.4), 0.4, 1e-3, seed)


def config5_flow(fine: bool, theta_deg: float = 60.0, seed: int = 2104) -> Case:
    """The learned-correction study's case with the momentum step on (Re 10, Ca 0.05, matched fluids).

    The explicit viscous term limits the step on the fine grid to about Re h^2/4 = 3.8e-5, so the
    simulated time t = 2 of the frozen-flow runs (20000 steps of 1e-4) is covered by 80000 steps of
    2.5e-5 on both grids."""
    c = config5(fine, theta_deg, seed)
    c.params = dataclasses.replace(c.params, dt=2.5e-5, navier_stokes=True)
    c.name = c.name.replace("cfg5_", "cfg5flow_")
    c.steps = 80000
    return c


def small_case(nx: int = 64, ny: int = 32, theta_deg: float = 60.0, kind: str = "flat",
               Vs: float = 0.0, seed: int = 7, velocity_fill: bool = True,
               slip_length: float = 0.01) -> Case:
    """Small 2D cases for fast tests (a few tiles, seconds on the CPU)."""
    g = Grid((nx, ny), (0.0, 0.0), (2.0, 1.0))
    h = g.h
    prm = Params(Cn=max(0.02, 1.5 * h), Pe=100.0, Re=10.0, Ca=0.1, theta_deg=theta_deg,
                 Vs=Vs, slip_length=slip_length, dt=1e-4, velocity_fill=velocity_fill)
    if kind == "flat":
        shapes = [Shape(HALFPLANE, (0.0, 0.2, 0.0, 0.0, 1.0, 0.0))]
        yc = 0.2
    elif kind == "tilted":
        a = math.radians(15.0)
        shapes = [Shape(HALFPLANE, (1.0, 0.5, 0.0, -math.sin(a), math.cos(a), 0.0))]
        yc = 0.5
    elif kind == "sin":
        shapes = [Shape(SINUSOID, (0.25, 0.06, 0.5, 0.0))]
        yc = 0.25 + 0.06 * math.sin(2.0 * math.pi * 1.0 / 0.5)
    elif kind == "circle":
        shapes = [Shape(SPHERE, (1.0, 0.42, 0.0, 0.22))]
        yc = 0.64
    else:
        raise ValueError(kind)
    return Case(f"small_{kind}_{nx}x{ny}", g, shapes, prm, 50, (1.0, yc), 0.3, 1e-3, seed)


def small_case_3d(n: int = 32, theta_deg: float = 90.0, seed: int = 11) -> Case:
    """Small 3D sphere case (scaled-down config 3), with 20 subgrid points per direction so that
    the FP64 oracle counts its volume fractions in seconds."""
    g = Grid((n, n, n), (-2.0, -2.0, -2.0), (2.0, 2.0, 2.0))
    h = g.h
    prm = Params(Cn=max(0.015, 1.5 * h), Pe=200.0, Re=5.0, Ca=0.05, theta_deg=theta_deg,
                 slip_length=0.01, dt=1e-4, subgrid=20)
    return Case(f"small_sphere_{n}cubed", g, [Shape(SPHERE, (0.0, 0.0, 0.0, 1.0))], prm, 20,
                (0.0, 0.0, 1.5), 0.5, 1e-3, seed)
