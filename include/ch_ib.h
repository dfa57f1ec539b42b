/*
 * ch_ib.h -- C ABI of the MI355X library for the hybrid ghost-cell immersed-boundary /
 * Cahn-Hilliard wetting step of Shahmardi, Rosti, Tammisola & Brandt,
 * "A fully Eulerian hybrid immersed boundary-phase field model for contact line dynamics
 * on complex geometries" (arXiv:2104.00350).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every function that can fail returns an int status: CH_IB_OK (0) or a negative code.
 *   Nothing aborts or throws.  ch_ib_last_error() returns a thread-local detail string.
 * - Grids are uniform Cartesian boxes, 2D or 3D, cell centred, axis 0 (x) stored fastest
 *   (linear cell index = i + n0*(j + n1*k)).  Every axis but the last is periodic; the last
 *   axis is bounded by two flat box walls (Neumann for the order parameter, no penetration
 *   for velocity).  This is the box of the end of Appendix A.1 of the paper.  Each n[a] must
 *   be a power of two between 8 and 2048 and all spacings equal.
 * - Fields are order parameter C (cell centred) and face velocities on the staggered grid:
 *   u_a[c] is the velocity normal to the face between cell c and cell c + e_a (section 3.1).
 *   The face of the last axis above the top cell row is a box wall and always reads as 0.
 * - Device memory is owned by the caller: the library never allocates or frees device
 *   memory.  A state lives inside one caller-provided workspace (ch_ib_workspace_bytes)
 *   and enqueues all its work on one caller-provided HIP stream.  Host objects
 *   (geometry, state handles) are owned by the library and released by the *_free calls.
 * - Nothing is re-entrant on the same state; distinct states may be used from distinct
 *   threads.
 */
#ifndef CH_IB_H
#define CH_IB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------------------- */
enum {
  CH_IB_OK = 0,
  CH_IB_EINVAL = -1,       /* invalid argument or parameter set */
  CH_IB_EGEOM = -2,        /* geometry preprocessing failed (e.g. ghost touching the box wall) */
  CH_IB_EHIP = -3,         /* a HIP runtime call failed */
  CH_IB_ENOMEM = -4,       /* workspace or caller buffer too small */
  CH_IB_ENAN = -5,         /* a non-finite value was found in the state */
  CH_IB_EUNSUPPORTED = -6  /* valid request the library does not implement (e.g. non power-of-two grid) */
};

/* ---- wall shapes (solid region; several shapes form a union) --------------------------
 * HALFPLANE: p[0..2] a point on the wall, p[3..5] wall normal pointing into the fluid;
 *            solid where (x - p).n < 0.
 * SINUSOID : p[0] mean height, p[1] amplitude, p[2] wavelength, p[3] phase (radians);
 *            solid where x_last < p0 + p1 sin(2 pi x_0 / p2 + p3).
 * SPHERE   : p[0..2] centre, p[3] radius (circle in 2D); solid inside.
 * BOX      : p[0..2] centre, p[3] half edge, p[4] rotation (radians) in the x-y plane;
 *            fluid inside the rotated square/cube, solid outside. */
enum { CH_IB_HALFPLANE = 1, CH_IB_SINUSOID = 2, CH_IB_SPHERE = 3, CH_IB_BOX = 4 };

/* ---- fields addressed by ch_ib_state_set / ch_ib_state_get ------------------------------ */
enum {
  CH_IB_FIELD_C = 0,       /* order parameter C^n, all cells (solid included) */
  CH_IB_FIELD_C_PREV = 1,  /* C^(n-1) (get only; set through ch_ib_state_load) */
  CH_IB_FIELD_U = 2,       /* face velocity along axis 0 */
  CH_IB_FIELD_V = 3,       /* face velocity along axis 1 */
  CH_IB_FIELD_W = 4,       /* face velocity along axis 2 (3D) */
  CH_IB_FIELD_CI = 5,      /* per-ghost wall value C_I of the dynamic condition (n_ghost values) */
  CH_IB_FIELD_ALPHA = 6,   /* fluid volume fraction (get only) */
  CH_IB_FIELD_PHI = 7,     /* chemical potential C^3 - C - Cn^2 lap C with mirror ghosts (get only) */
  CH_IB_FIELD_P = 8        /* pressure p^n of the momentum step, zero mean (get only) */
};

/* ---- params.flags ---------------------------------------------------------------------- */
enum {
  CH_IB_FLAG_VELOCITY_FILL = 1, /* refill faces touching ghosts every step (section 4.3) */
  CH_IB_FLAG_EXPLICIT = 2,       /* explicit Adams-Bashforth step (Eq. ExpCH) instead of the
                                    semi-implicit one; needs a time step about ten times smaller */
  CH_IB_FLAG_NAVIER_STOKES = 4   /* advance the face velocities with the momentum equation too
                                    (sections 2, 3.2, 4.2.3, 4.3 and 4.4); implies the velocity fill */
};

typedef struct {
  int ndim;        /* 2 or 3 */
  int n[3];        /* cells per axis */
  double lo[3];    /* box lower corner */
  double hi[3];    /* box upper corner */
} ch_ib_grid;

typedef struct {
  int kind;        /* CH_IB_HALFPLANE ... CH_IB_BOX */
  double p[10];
} ch_ib_shape;

/* Dimensionless groups and method options.  Non-dimensional form of the paper's system:
 * dC/dt + div(uC) = (1/Pe) lap(C^3 - C - Cn^2 lap C), wall condition
 * DC/Dt = Vs [Cn dC/dn + cos(theta)(1 - C^2)/sqrt2] (Vs = 0: static, Eq. WallBCS with mu_f = 0),
 * Navier slip with slip length ls and capillary bracket scaled by 1/Ca (Eq. SlipVelocity). */
typedef struct {
  double Cn, Pe, Re, Ca, mu;  /* Re is carried but not used by the order-parameter step */
  double theta_deg;           /* equilibrium contact angle, measured through the C = +1 phase */
  double Vs;                  /* contact-line relaxation coefficient; 0 selects the static condition */
  double slip_length;
  double dt;
  double S;                   /* stabilisation of Appendix A.1; <= 0 selects Cn sqrt(6 Pe/dt) */
  double d1_cells;            /* intersect-to-mirror distance in cells; <= 0 selects 2 */
  double d2_cells;            /* mirror-to-interpolation-point spacing in cells; <= 0 selects 1.5 */
  int subgrid;                /* subgrid points per direction for the volume fraction; 0: 100 */
  int precision;              /* 64 (FP64) or 32 (FP32) arithmetic on the device */
  int flags;                  /* CH_IB_FLAG_* */
  /* momentum step (CH_IB_FLAG_NAVIER_STOKES only; all four must then be positive): densities and
   * viscosities of the C = -1 (rho1, mu1) and C = +1 (rho2, mu2) phases relative to the reference
   * fluid of Re; body_force is an acceleration per axis (e.g. gravity) */
  double rho1, rho2, mu1, mu2;
  double body_force[3];
} ch_ib_params;

/* Per-ghost tables (structure of arrays, sorted by ghost cell index), section 4.1.
 * ap/w are laid out [2][n_ap][n_ghost]: averaging points and weights of IP1 then IP2.
 * Unused averaging slots carry weight 0 and repeat a used index. */
typedef struct {
  int64_t n_ghost;
  int ndim;
  int n_ap;          /* 2*ndim + 1 */
  int64_t *gidx;     /* [n_ghost] linear cell index of the ghost point */
  double *normal;    /* [ndim][n_ghost] unit wall normal, pointing into the fluid */
  double *dn;        /* [n_ghost] ghost-to-intersect distance */
  double *gamma;     /* [n_ghost] d1 / dn */
  int64_t *ap;       /* [2][n_ap][n_ghost] averaging-point cell indices */
  double *w;         /* [2][n_ap][n_ghost] normalised inverse-squared-distance weights */
  double *alpha;     /* [cells] fluid volume fraction, or NULL */
} ch_ib_ghost_tables;

typedef struct {
  double mass_box;     /* h^d sum C */
  double mass_fluid;   /* h^d sum alpha C */
  double free_energy;  /* bulk + gradient (alpha weighted) + diffuse wall term, u = 0 */
  double max_abs_C;
  int64_t step;
  int status;          /* CH_IB_OK or CH_IB_ENAN */
  int pad_;
} ch_ib_diag;

typedef struct ch_ib_geometry ch_ib_geometry;
typedef struct ch_ib_state ch_ib_state;

/* ---- errors ------------------------------------------------------------------------------ */
const char *ch_ib_strerror(int status);
const char *ch_ib_last_error(void);
int ch_ib_version(void);  /* major*10000 + minor*100 + patch */

/* ---- geometry (one-time host preprocessing, section 4.1) ----------------------------------
 * ch_ib_geometry_build: volume fraction by subgrid counting (4.1.1), normals from corner
 *   gradients of the volume fraction (Eqs. NormalVectors_part1/2), ghost points, intersect
 *   points by marching along the normal and bisecting, mirror points at d1 and interpolation
 *   points at d2 and 2*d2 beyond it (4.1.2), plus-stencil averaging points with normalised
 *   1/h^2 weights (Eq. "weright averaged").  Host arrays passed in are copied.
 *   Returns EGEOM if a ghost touches the bounded axis' box wall or an interpolation point has
 *   no fluid averaging point within 2h, EINVAL on a bad grid or shape.
 * ch_ib_geometry_import: tables from the caller (copied), e.g. produced by another
 *   implementation; alpha may be NULL (then mass_fluid and the free energy use alpha = 1).
 * ch_ib_geometry_export: copies the tables into caller-allocated arrays sized from
 *   ch_ib_geometry_count (alpha is copied if non-NULL).
 * ch_ib_geometry_free: releases the host object (NULL is accepted). */
int ch_ib_geometry_build(const ch_ib_grid *grid, const ch_ib_shape *shapes, int n_shapes,
                         const ch_ib_params *params, ch_ib_geometry **out);
int ch_ib_geometry_import(const ch_ib_grid *grid, const ch_ib_ghost_tables *tables,
                          ch_ib_geometry **out);

/* Fluid fractions of the staggered (face-centred) cells, section 4.1.1's other three volume
 * fractions: ndim fields of cells doubles, field a for the faces between cell c and c + e_a, each
 * control volume the cell shifted by h/2 along a, counted with the same subgrid points.
 * ch_ib_geometry_build and ch_ib_geometry_build_device compute them when params->flags has
 * CH_IB_FLAG_NAVIER_STOKES (the device builder bit for bit with the host builder).
 * ch_ib_geometry_face_fractions: copies them to dst (ndim * cells doubles, caller-allocated);
 *   EUNSUPPORTED if the geometry holds none (imported or built without the flag).
 * ch_ib_geometry_set_face_fractions: replaces them with a copy of src (same layout; every value
 *   in [0, 1], else EINVAL), e.g. for an imported geometry. */
int ch_ib_geometry_face_fractions(const ch_ib_geometry *geom, double *dst);
int ch_ib_geometry_set_face_fractions(ch_ib_geometry *geom, const double *src);

/* Geometry preprocessing on the GPU: the tables of ch_ib_geometry_build (same readings, same
 * sequence of operations, no contraction of multiplies and adds), computed with one thread per
 * cell for the volume fraction and the ghost list and one per ghost for the rest, returned as an
 * ordinary host geometry object.  Integer tables and the doubles match the host builder bit for bit
 * except where a sinusoid's sine from the device math library differs in its last bit.
 * ch_ib_geometry_device_bytes: device scratch the builder needs for this grid (0 on a bad grid);
 *   it holds per-ghost arrays for up to cells/8 + 1024 ghosts.
 * ch_ib_geometry_build_device: device_scratch (caller-owned, 256-byte aligned, >= that many
 *   bytes) is used on hip_stream (a hipStream_t; NULL = default stream) and free again on return;
 *   synchronous.  At most 8 shapes.  Same errors as ch_ib_geometry_build, plus ENOMEM for a small
 *   scratch or more ghosts than it holds and EHIP on a device error. */
size_t ch_ib_geometry_device_bytes(const ch_ib_grid *grid);
int ch_ib_geometry_build_device(const ch_ib_grid *grid, const ch_ib_shape *shapes, int n_shapes,
                                const ch_ib_params *params, void *device_scratch, size_t bytes, void *hip_stream,
                                ch_ib_geometry **out);
int ch_ib_geometry_export(const ch_ib_geometry *geom, ch_ib_ghost_tables *dst);
int ch_ib_geometry_count(const ch_ib_geometry *geom, int64_t *n_ghost, int *n_ap);
void ch_ib_geometry_free(ch_ib_geometry *geom);

/* ---- state ----------------------------------------------------------------------------------
 * ch_ib_workspace_bytes: device bytes one state needs (0 on invalid input).
 * ch_ib_state_create: carves the state out of device_workspace (>= that many bytes, 256-byte
 *   aligned, caller-owned, must outlive the state), uploads the tables and coefficient tables
 *   on hip_stream (a hipStream_t; NULL = default stream) and waits for the upload.
 *   EINVAL if S is below the bound of Appendix A.1 or a parameter is out of range.
 * ch_ib_state_set: copies a field in (host or device pointer, element type double for
 *   precision 64 and float for precision 32).  Setting C (or a velocity) marks the state as a
 *   fresh start: the next ch_ib_step first fills the ghosts of the current fields (initial
 *   fill) and sets C^(n-1) = C^n.
 * ch_ib_state_get: copies a field out (same element type rules); synchronous. */
size_t ch_ib_workspace_bytes(const ch_ib_grid *grid, const ch_ib_geometry *geom,
                             const ch_ib_params *params);
int ch_ib_state_create(const ch_ib_grid *grid, const ch_ib_geometry *geom,
                       const ch_ib_params *params, void *device_workspace, size_t bytes,
                       void *hip_stream, ch_ib_state **out);
int ch_ib_state_set(ch_ib_state *st, int field, const void *src, int src_on_device);
int ch_ib_state_get(ch_ib_state *st, int field, void *dst, int dst_on_device);

/* ---- time stepping (the hot path) -----------------------------------------------------------
 * ch_ib_step: enqueues n_steps steps on the state's stream and returns without waiting.  One
 *   step: right-hand side of Eq. Helmholtz1 (history, conservative advection, Laplacian of
 *   the explicit chemical-potential part), the two Helmholtz solves of Appendix A.1 as one
 *   spectral division (Hartley transforms on periodic axes, DCT-II on the bounded axis), the
 *   contact-angle ghost fill of C (section 4.2.2) and, with CH_IB_FLAG_VELOCITY_FILL, the
 *   no-penetration / Navier-slip fill of the faces touching ghosts (section 4.3).
 *   With CH_IB_FLAG_EXPLICIT the step is Eq. ExpCH instead: the chemical potential on every
 *   cell (ghosts take the mirror value, dphi/dn = 0), the rate R = -div(u C) + lap(phi)/Pe, and
 *   C^(n+1) = C^n + dt (3/2 R^n - 1/2 R^(n-1)) (second-order Adams-Bashforth; the first step
 *   after the fields are set or loaded without a rate is a forward Euler step), then the same
 *   fills.  The workspace then holds one more field for R.
 *   With CH_IB_FLAG_NAVIER_STOKES the faces follow the momentum equation: after the order-parameter
 *   step (semi-implicit: advected by 2u^n - u^(n-1), Appendix A.1; explicit: by u^n) comes the
 *   momentum step of sections 4.2.3, 4.3 and 4.4 on the staggered grid, with rho and mu linear in C^(n+1),
 *   phi the chemical potential above and the capillary force 3/(2 sqrt2 Re Ca Cn) phi grad C:
 *   Adams-Bashforth prediction (Eq. PredictionExp; the first step after the fields are set uses a
 *   forward Euler convective term and no pressure history, p^n = p^(n-1) = 0), penalisation
 *   u** = alpha_face u* (Eq. Penalization2), the
 *   velocity ghost fill on u**, the pressure of Eq. PressurePoisson (rho0 = min(rho1, rho2),
 *   p^ = 2p^n - p^(n-1), zero-mean, no flux through the box walls) by the same transforms, and
 *   the correction of Eq. correction.  The box walls of the bounded axis are no-slip.  Needs a
 *   geometry with staggered-cell fractions (EINVAL at state creation otherwise); not available to
 *   batches or the learned correction.
 * ch_ib_sync: waits for the stream; reports CH_IB_EHIP on a device error.
 * ch_ib_diagnostics: mass, free energy, max |C| (deterministic fixed-order reductions);
 *   synchronous; status CH_IB_ENAN (also returned) if any C is not finite. */
int ch_ib_step(ch_ib_state *st, int n_steps);
int ch_ib_sync(ch_ib_state *st);
int ch_ib_diagnostics(ch_ib_state *st, ch_ib_diag *out);

/* ch_ib_diagnostics_noalloc: for callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid allocation).  The same values as
 * ch_ib_diagnostics, from the same kernels, but the reduction's partial sums live in a fixed
 * device array of the library (8192 x 8 + 8 doubles, 512 KiB per GPU, held until the process
 * ends) instead of the state's workspace; nothing is allocated.  The state's device must be the
 * current device (CH_IB_EINVAL otherwise); a reduction needing more than 8192 partial sums is
 * rejected with CH_IB_ENOMEM.  Every call on one GPU uses that GPU's one array: calls that
 * overlap on the same GPU race.  Synchronous, like ch_ib_diagnostics. */
int ch_ib_diagnostics_noalloc(ch_ib_state *st, ch_ib_diag *out);

/* ---- stage entry points (each runs one part of the step on device buffers of the state's
 * element type, n cells each; used to check each stage on its own) ------------------------------
 * CH_IB_STAGE_RHS  : out = Q of Eq. Helmholtz1 from the current C^n, C^(n-1), faces (in unused).
 * CH_IB_STAGE_SOLVE: out = solution C of (lap_h - a)(lap_h + alpha_s) C = in (Eqs. Helmholtz1-2).
 * CH_IB_STAGE_PHI  : out = chemical potential of the current C (in unused). */
enum { CH_IB_STAGE_RHS = 1, CH_IB_STAGE_SOLVE = 2, CH_IB_STAGE_PHI = 3 };
int ch_ib_stage(ch_ib_state *st, int stage, const void *in_device, void *out_device);

/* ---- ghost fill of any scalar under a mixed wall condition ------------------------------------
 * The ghost-cell procedure of section 4.2.2 applied to a general boundary condition, as the
 * abstract and the conclusions propose (Dirichlet, Neumann or mixed conditions on any field):
 * for a field f on the state's grid, every ghost value is set so that
 *     a f_I + b (df/dn)_I = g     at the wall,
 * with f_I = (gamma f_G + f_M)/(gamma + 1) and (df/dn)_I = (f_M - f_G)/((1 + gamma) dn) formed from
 * the ghost and its mirror value (Eqs. extrapolation, interpolationAtWall, ProjectingToNT; n into
 * the fluid), i.e. f_G = ((gamma + 1) g - f_M (a + b/dn)) / (a gamma - b/dn).  b = 0: Dirichlet;
 * a = 0: Neumann (g = 0 gives the mirror value).
 * field_device: the state's element type, one value per cell, x fastest; only the ghost cells are
 *   written (the averaging points are fluid cells, never ghosts).  Caller-owned.
 * g_ghost_device: NULL for the uniform g, else one value of g per ghost in the ghost order of the
 *   geometry (ch_ib_geometry_export), the state's element type.
 * Enqueued on the state's stream; returns without waiting.  EINVAL if field_device is NULL, a, b or
 * g is not finite, a = b = 0, or a gamma - b/dn = (a d1 - b)/dn vanishes (b/a within the range of
 * d1 = gamma dn over the ghosts), where the condition does not fix the ghost value. */
int ch_ib_scalar_fill(ch_ib_state *st, void *field_device, double a, double b, double g,
                      const void *g_ghost_device);

/* ---- measurement ------------------------------------------------------------------------------
 * ch_ib_step_timed: enqueues n_steps (1..4096) steps exactly as ch_ib_step does, with a HIP event
 *   recorded on the state's stream between consecutive kernels, then waits once.  ms_out[k]
 *   receives the mean duration (ms per step) of the k-th kernel of a step and names_out[k] its
 *   name (static string); *n_kernels the number of kernels per step.  At most max_kernels entries
 *   are written (ENOMEM if a step has more).  Events are created and destroyed inside the call. */
int ch_ib_step_timed(ch_ib_state *st, int n_steps, int max_kernels, double *ms_out, const char **names_out,
                     int *n_kernels);

/* ---- launch-shape autotuning ------------------------------------------------------------------
 * The four field passes of a step (0 fused rhs + x transform, 1 strided y transform (3D only),
 * 2 bounded-axis solve, 3 x transform out) each have a launch shape of three ints:
 * {log2 lines or columns per tile, largest FFT radix (8 or 16; pass 0 also 4, which only the
 * z-marching kernel with up to 4 rows per tile uses, the others taking 8), third field}.  The third field is
 * 1 for passes 1-3; for pass 0 it is the cells in flight per thread (1 or 2) of the line-tiled
 * kernel; for 2D grids with nx <= 1024, 3 selects the y-marching kernel (rows y-1..y+1 held per
 * thread, each value loaded and combined once); for 3D grids, 3..5 select the z-marching kernel
 * (nx = 256 or 512 only) with 2^value planes per workgroup, or 6..8 split that kernel in two: a
 * stencil-only z-march over 2^(value-3) planes writing the right-hand side, then the x transform
 * in place with pass 3's shape (16 more bytes per cell, no FFT inside the stencil loop).  Shapes
 * change speed, never results, apart from rounding: every shape computes the same sums in the
 * same order per element except for the FFT radix and the y-marching kernel (which evaluates the
 * bulk-energy derivative once per value and scales it by 1/Cn^2 inside the Laplacian factor).
 * ch_ib_tune: times every candidate shape of each pass reps times with HIP events on the state's
 *   buffers (the fields are left unchanged), keeps the fastest and writes the 12 chosen ints to
 *   shapes_out (may be NULL).  Synchronous.
 * ch_ib_get_shapes / ch_ib_set_shapes: read or impose the 12 ints (e.g. from a cache); values
 *   are clamped to what the grid and the LDS tile allow; EINVAL on a radix other than 8 or 16
 *   (or 4 for pass 0). */
int ch_ib_tune(ch_ib_state *st, int reps, int *shapes_out);
int ch_ib_get_shapes(const ch_ib_state *st, int *shapes_out);
int ch_ib_set_shapes(ch_ib_state *st, const int *shapes);

/* ---- batched sweep ------------------------------------------------------------------------------
 * A batch advances many independent 2D states (uneven sizes allowed) together: every phase of
 * the step is one grouped launch over all member states (block -> state through per-state tile
 * offsets; per-state descriptors in device memory), and two consecutive steps are captured in
 * one hipGraph that ch_ib_batch_step replays.  Results are the same as stepping each state on
 * its own with the same launch shapes (bit for bit).
 * ch_ib_batch_workspace_bytes: device bytes for the descriptors and offsets of n_states states.
 * ch_ib_batch_create: states must be 2D, of one precision, with the static contact-angle
 *   condition (Vs = 0); their pending initial fills are done here.  The batch keeps pointers to
 *   the states: while it exists, the member states must not be stepped on their own or freed.
 *   device_workspace (caller-owned, 256-byte aligned) must outlive the batch.  EUNSUPPORTED for
 *   3D, dynamic or explicit-scheme states, EINVAL for mixed precisions.  Members with the
 *   momentum step (Navier-Stokes coupling, section 4.4) are accepted: the grouped launches cover
 *   the others, and each of these is advanced by its own launches (those of ch_ib_step, on the
 *   batch's stream, one member after another), with the same results as ch_ib_step.
 * ch_ib_batch_step: enqueues n_steps steps for every member on the batch's stream (graph replays
 *   plus at most one direct step; on the NULL stream, which cannot be captured, direct grouped
 *   launches only; then the momentum members' steps); the members' step counters and buffer
 *   roles are updated.
 * ch_ib_batch_tune: tunes the launch shapes of one member per distinct grid size
 *   (ch_ib_tune), applies them to all members of that size, then times full batched steps of the
 *   grouped members for the choices shared by the grouped kernels and the tile heights (greedy: rhs radix and rhs
 *   kernel, then per grid size the rhs, solve and output tile heights, written to the members'
 *   shapes, then the solve radix, then the output radix); radix_out[0..2] (rhs, solve, out) and
 *   *unroll_out (either may be NULL) receive the shared choices.  Leaves the fields unchanged.
 *   Synchronous.
 * ch_ib_batch_sync: waits for the batch's stream.  ch_ib_batch_free: releases the graphs and the
 *   host object (not the states). */
typedef struct ch_ib_batch ch_ib_batch;
size_t ch_ib_batch_workspace_bytes(int n_states);
int ch_ib_batch_create(ch_ib_state *const *states, int n_states, void *device_workspace, size_t bytes,
                       void *hip_stream, ch_ib_batch **out);
int ch_ib_batch_step(ch_ib_batch *b, int n_steps);
int ch_ib_batch_tune(ch_ib_batch *b, int reps, int *radix_out, int *unroll_out);
int ch_ib_batch_sync(ch_ib_batch *b);
void ch_ib_batch_free(ch_ib_batch *b);

/* ---- checkpoint / resume ---------------------------------------------------------------------
 * ch_ib_state_save: if buf is NULL, *len receives the size needed; otherwise writes a versioned
 *   blob (C^n, C^(n-1), faces, per-ghost history, step counter; with the explicit scheme also
 *   the previous step's rate) and sets *len.  Synchronous.
 * ch_ib_state_load: restores a blob saved from a state with the same grid, tables, precision and
 *   time scheme.
 * ch_ib_state_free: releases the host handle (the workspace stays the caller's). */
int ch_ib_state_save(ch_ib_state *st, void *buf, size_t *len);
int ch_ib_state_load(ch_ib_state *st, const void *buf, size_t len);
void ch_ib_state_free(ch_ib_state *st);

/* Derived coefficients of Appendix A.1 for a parameter set: S, alpha_s and a = alpha_s + S/Cn^2.
 * EINVAL if S is below Cn sqrt(6 Pe/dt). */
int ch_ib_coefficients(const ch_ib_params *params, double *S, double *alpha_s, double *a);

/* ---- learned wall-band correction (2D, FP64 states, static condition) ------------------------
 * An extension of the method, not part of the paper: a coarse run is corrected in the band of
 * fluid cells near the wall (0 < wall distance <= band cells, |C| < 0.9) by a three-layer 3x3
 * convolutional network on features [C, phi, wall distance / (band h) clipped to [-2, 2], n_x,
 * n_y]: 5 -> 32 -> 32 channels with tanh, then 32 -> 1 scaled by out_scale.  Layers 1-2 run as
 * BF16 matrix-core products with FP32 accumulation; weights are BF16 copies of FP32 master
 * weights, biases FP32.  Convolutions are periodic along x and see zeros outside the box along y.
 *
 * ch_ib_wall_field (host, no GPU): signed distance to the wall (positive in the fluid, the
 *   minimum over the shapes) and the unit normal into the fluid at the nearest wall point, per
 *   cell; dist[N], normal[2][N] caller-allocated (x fastest).  Half-plane, sinusoid and circle
 *   walls in 2D; EUNSUPPORTED otherwise.
 * ch_ib_net_workspace_bytes / ch_ib_net_create: one caller-owned device workspace (256-byte
 *   aligned) sized for grids of up to max_cells cells, max_tiles band tiles, a sample store of
 *   max_store_tiles tiles (17.5 KB each) and training batches of up to max_batch tiles; all work
 *   of the network is enqueued on hip_stream (use the bound state's stream).
 * ch_ib_net_set_params / get_params: CH_IB_NET_NPARAMS floats (layout: W1[9][32][16] (tap, out,
 *   in; inputs 5..15 must be zero), b1[32], W2[9][32][32], b2[32], W3[9][32], b3; tap = 3 ky + kx
 *   multiplies the input at (x + kx - 1, y + ky - 1)); set_params also resets the optimiser.
 * ch_ib_net_bind: attaches a 2D FP64 static-condition state (semi-implicit, with or without the
 *   momentum step) whose grid sizes are multiples of 16;
 *   wall_dist[N] and wall_normal[2][N] are host arrays (as ch_ib_wall_field returns), copied;
 *   the band tiles are the 16x16 tiles holding a cell with 0 < dist <= band_cells h.
 * ch_ib_net_rebind: attaches another state with the same grid and wall (same tiles and wall
 *   field; the caller guarantees the wall is the same), without copying anything.
 * ch_ib_net_forward: dC of the band tiles of the bound state's current C into dC_device
 *   ([n_tiles][16][16] floats, 0 outside the band), or into the network's own buffer if NULL;
 *   dC is limited so that C + dC stays in [-1, 1].
 * ch_ib_net_apply: C += weight dC (0 <= weight <= 1) in both time levels of the bound state, then
 *   the ghost values are filled again from the corrected field.
 * ch_ib_net_extract: stores one training sample per band tile at store_offset..: the feature
 *   patch, the target correction target_device[c] - C[c] (target: a device field of the bound
 *   grid) and the band mask; mask_counts (optional, host, n_tiles floats) gets each tile's count.
 * ch_ib_net_store_get: host copy of stored sample `slot` (X: 22*22*16 BF16 values, Y, M: 256).
 * ch_ib_net_train_step: forward and backward pass of the listed stored samples (count <= max_batch;
 *   the loss is sum over masked cells of (dC - Y)^2 times inv_count) and one Adam step (beta1
 *   0.9, beta2 0.999, eps 1e-8) with learning rate lr; loss_out (optional) gets the loss (syncs).
 * ch_ib_net_gradient: the same pass without the update; grad_host gets the summed gradient.
 * ch_ib_restrict2: sets the coarse state's C to the 2x2 means of the fine state's C (fine grid
 *   twice as many cells per axis, same box).  both_levels = 0: the coarse state restarts from it
 *   (C_prev := C, ghosts refilled) at its next step; both_levels = 1: C_prev is restricted from
 *   the fine C_prev as well and the ghosts of C are refilled at once (the two-level history is
 *   kept; static condition only).  With both_levels = 1 and the momentum step on both states
 *   (EINVAL if only one runs it) the momentum state is restricted too: every coarse face is the
 *   mean of the two fine faces that tile it (u^n, the advecting velocity and the previous
 *   convective term; a divergence-free fine field stays divergence-free), both pressure levels
 *   by 2x2 means, and the history flags follow the fine state.  Synchronous. */
#define CH_IB_NET_NPARAMS 14177
typedef struct ch_ib_net ch_ib_net;
int ch_ib_wall_field(const ch_ib_grid *grid, const ch_ib_shape *shapes, int n_shapes, double *dist, double *normal);
size_t ch_ib_net_workspace_bytes(int64_t max_cells, int max_tiles, int64_t max_store_tiles, int max_batch);
int ch_ib_net_create(int64_t max_cells, int max_tiles, int64_t max_store_tiles, int max_batch, double out_scale,
                     void *device_workspace, size_t bytes, void *hip_stream, ch_ib_net **out);
int ch_ib_net_set_params(ch_ib_net *net, const float *params);
int ch_ib_net_get_params(ch_ib_net *net, float *params);
int ch_ib_net_bind(ch_ib_net *net, ch_ib_state *st, const double *wall_dist, const double *wall_normal,
                   double band_cells, int *n_tiles);
int ch_ib_net_forward(ch_ib_net *net, float *dC_device);
int ch_ib_net_rebind(ch_ib_net *net, ch_ib_state *st);
int ch_ib_net_apply(ch_ib_net *net, double weight);
int ch_ib_net_extract(ch_ib_net *net, const double *target_device, int64_t store_offset, float *mask_counts);
int ch_ib_net_store_get(ch_ib_net *net, int64_t slot, unsigned short *X, float *Y, float *M);
int ch_ib_net_train_step(ch_ib_net *net, const int64_t *sample_ids, int count, double lr, double inv_count,
                         double *loss_out);
int ch_ib_net_gradient(ch_ib_net *net, const int64_t *sample_ids, int count, double inv_count, float *grad_host,
                       double *loss_out);
int ch_ib_restrict2(ch_ib_state *fine, ch_ib_state *coarse, int both_levels);
void ch_ib_net_free(ch_ib_net *net);

#ifdef __cplusplus
}
#endif
#endif /* CH_IB_H */
