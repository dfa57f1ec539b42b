"""MI355X (gfx950) library for the hybrid ghost-cell immersed-boundary / Cahn-Hilliard
wetting step (arXiv:2104.00350): HIP kernels behind a C ABI (include/ch_ib.h), bound here
with ctypes.  See chib.py for the binding and build.py for the in-tree build."""
