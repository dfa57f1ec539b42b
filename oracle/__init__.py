"""FP64 CPU oracle of the hybrid ghost-cell immersed-boundary / Cahn-Hilliard step.

TEST INFRASTRUCTURE ONLY.  Nothing in the device library imports, calls or
links this package; only the tests, the smoke check and the CPU-baseline leg
of the benchmark use it.  It shares no code with the HIP path: the only module
both sides import is ``workloads`` (seeded inputs, no arithmetic of the method).

Every function follows a passage of Shahmardi, Rosti, Tammisola & Brandt,
"A fully Eulerian hybrid immersed boundary-phase field model for contact line
dynamics on complex geometries" (arXiv:2104.00350), cited by section and
equation label in its docstring.

Pins (what fixes each part independently of this code) are listed in
``tests/test_oracle_*.py``.  Parts with no independent pin say "parity
unpinned" in their docstring.
"""
from .geometry import GhostTables, build_tables, volume_fraction, GeometryError  # noqa: F401
from .solver import OracleState, derived_coefficients, spectral_solve  # noqa: F401
