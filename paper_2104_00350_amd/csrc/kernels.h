// Internal launch interface between the host driver and the device kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace chib {

// Everything one step needs, as plain values and device pointers (element type T chosen
// by the launcher: double for precision 64, float for precision 32).
constexpr int kGhostSlots = 16;   // lanes (and table slots) per ghost in the ghost kernels

struct Plan {
  int d = 2;
  int n[3] = {1, 1, 1};
  int logn[3] = {0, 0, 0};
  int64_t N = 0;       // cells
  double h = 0;

  // coefficients of the step (non-dimensional, see ch_ib.h)
  double Pe = 0, Cn = 0, dt = 0, S = 0, alpha_s = 0, a = 0;
  double cos_t = 0, Ca = 1, mu = 1, ls = 0, Vs = 0;
  int vel_fill = 0, dynamic = 0;
  int explicit_ab2 = 0;     // explicit Adams-Bashforth step (Eq. ExpCH) instead of the semi-implicit one

  // fields
  void *C[2] = {nullptr, nullptr};
  void *F[3] = {nullptr, nullptr, nullptr};
  void *W = nullptr;        // spectral workspace, N elements (explicit step: the chemical potential)
  void *R = nullptr;        // explicit step: rate of the previous step, N elements
  void *alpha = nullptr;    // N elements or nullptr (then alpha = 1)
  void *Fadv[3] = {nullptr, nullptr, nullptr};   // advecting faces of the rhs pass (nullptr: F)

  // momentum step (Navier-Stokes coupling): face fields of d components, N elements each
  int ns = 0;
  double Re = 1, rho1 = 1, rho2 = 1, mu1 = 1, mu2 = 1, g[3] = {0, 0, 0};
  void *Us[3] = {nullptr, nullptr, nullptr};   // u** (prediction after penalisation, then filled)
  void *Ut[3] = {nullptr, nullptr, nullptr};   // 2u^n - u^(n-1), the advecting velocity of the rhs pass
  void *Nh[3] = {nullptr, nullptr, nullptr};   // convective term of the previous momentum step
  void *Af[3] = {nullptr, nullptr, nullptr};   // staggered-cell fluid volume fractions
  void *P[2] = {nullptr, nullptr};             // pressure p^n, p^(n-1)
  int poisson = 0;          // bounded-axis pass divides by the Laplacian's eigenvalue (pressure)

  // ghost tables (SoA, sorted by cell)
  int64_t G = 0;
  int K = 0;
  const int *gidx = nullptr;       // [G]
  const void *normal = nullptr;    // [d][G]
  const void *dn = nullptr;        // [G]
  const void *gamma = nullptr;     // [G]
  const int *ap = nullptr;         // [2][K][G]
  const void *w = nullptr;         // [2][K][G]
  // the same two tables ghost-major, kGhostSlots slots per ghost (slots >= 2K: cell 0, weight 0), for
  // the kernels that give each ghost a lane group: one wave request then covers a few cache lines
  const int *apg = nullptr;        // [G][kGhostSlots]
  const void *wg = nullptr;        // [G][kGhostSlots]
  // the cells where dg needs phi~ (averaging points and ghosts, sorted), each slot's index into
  // them, and phi~ there
  int64_t NU = 0;
  const int *pt_cell = nullptr;    // [NU]
  const int *pt_idx = nullptr;     // [G][kGhostSlots]
  void *pt_phi = nullptr;          // [NU]
  void *CGn = nullptr, *CGnm1 = nullptr, *CMs = nullptr, *CI = nullptr, *CGnew = nullptr;
  void *UG = nullptr;              // [d][G]

  // wall condition dphi/dn = 0 of the semi-implicit step: per ghost the change of g,
  // dg = (phi~_M - phi~_G)/Cn^2, and the cells whose rhs it changes (ghosts and their face
  // neighbours, sorted by cell) with the change dq of each and the first of them on every x-row
  void *dg = nullptr;              // [G]
  int64_t NP = 0;
  const int *pl_cell = nullptr;    // [NP]
  const int *pl_ref = nullptr;     // [2d+1][NP]: own ghost index, then the ghost at +e_a and -e_a per axis, or -1
  const int *pl_row = nullptr;     // [rows + 1]
  void *pl_dq = nullptr;           // [NP]

  // faces touching ghosts (velocity fill)
  int64_t NF = 0;
  const int *f_cell = nullptr;     // left cell of the face
  const int *f_axis = nullptr;
  const int *f_gL = nullptr;       // ghost index of the left cell or -1
  const int *f_gR = nullptr;       // ghost index of the right cell or -1
  void *stashL = nullptr, *stashR = nullptr;

  // transform tables (element type T): FFT twiddles exp(-2 pi i m / n_a) per axis,
  // cos/sin(pi k / (2 n_last)) for the cosine transform, 1D eigenvalues per axis
  const void *twr[3] = {nullptr, nullptr, nullptr};
  const void *twi[3] = {nullptr, nullptr, nullptr};
  const void *dctc = nullptr, *dcts = nullptr;
  const void *lam[3] = {nullptr, nullptr, nullptr};

  // reduction scratch: partial[nred][8] and out[8] in double
  void *partial = nullptr;
  void *red_out = nullptr;
  int nred = 0;

  // launch shapes of the four field passes: 0 fused rhs + x transform, 1 strided y
  // transform (3D), 2 bounded-axis solve, 3 x transform out
  struct Shape {
    int log_tile;  // log2 lines (x passes) or columns (strided passes) per tile
    int radix;     // largest FFT radix: 8 or 16
    int unroll;    // cells in flight per thread (rhs pass)
  };
  Shape shape[4] = {{3, 8, 2}, {4, 16, 1}, {4, 16, 1}, {4, 16, 1}};

  hipStream_t stream = nullptr;
};

// Optional per-kernel event recorder for measured steps.
struct KernelTimer {
  static constexpr int kMax = 16;
  hipEvent_t ev[kMax + 1];
  const char *names[kMax];
  int n = 0;
  hipError_t mark(const char *name, hipStream_t s) {
    if (n >= kMax) return hipErrorInvalidValue;
    names[n] = name;
    return hipEventRecord(ev[n++], s);
  }
  hipError_t end(hipStream_t s) { return hipEventRecord(ev[n], s); }
};

template <typename T> hipError_t enqueue_step(const Plan &p, int cur, KernelTimer *tm = nullptr);
template <typename T> hipError_t enqueue_initial_fill(const Plan &p, int cur);
template <typename T> hipError_t tune_shapes(Plan &p, int cur, int reps);
// One explicit Adams-Bashforth step (first: no previous rate, forward Euler) from C[cur] into C[1-cur].
template <typename T> hipError_t enqueue_explicit_step(const Plan &p, int cur, int first, KernelTimer *tm = nullptr);
// Largest log2 tile height (passes 0 and 3: lines; 1 and 2: columns) a pass allows on this grid.
template <typename T> int max_log_tile(const Plan &p, int pass);
template <typename T> hipError_t enqueue_ghost_refresh(const Plan &p, int cur);   // static fill again, same step
template <typename T> hipError_t enqueue_rhs(const Plan &p, int cur, void *out);
template <typename T> hipError_t enqueue_solve(const Plan &p, const void *in, void *out);
template <typename T> hipError_t enqueue_phi(const Plan &p, int cur, void *out);
// Ghost values of the scalar field f (N elements) under a f + b df/dn = g (g_ghost: G values or null).
template <typename T>
hipError_t enqueue_scalar_fill(const Plan &p, void *f, double a, double b, double g, const void *g_ghost);
template <typename T> hipError_t enqueue_diag(const Plan &p, int cur);
// Pressure solve in place on W: W <- the zero-mean p with lap_h p = W (zero flux through the box walls).
template <typename T> hipError_t enqueue_poisson(const Plan &p);
// Velocity ghost fill (slip and no-penetration) on the faces p.F with the order parameter Cfin.
template <typename T> hipError_t enqueue_velocity_fill(const Plan &p, const void *Cfin);
// Momentum step on the new order parameter C[cur] (prediction, penalisation, velocity fill,
// pressure, correction); first: no previous convective term.  Leaves p^(n+1) in W.
template <typename T> hipError_t enqueue_momentum(const Plan &p, int cur, int first, KernelTimer *tm = nullptr);

// One grouped step over a batch of 2D cases (see the batched kernels).
struct BatchLaunch {
  const void *descs = nullptr;   // device array of per-case descriptors
  static constexpr int kPhases = 7;
  const int *off = nullptr;      // device [kPhases][n+1] per-phase tile offsets
  int n = 0;
  unsigned total[kPhases] = {0, 0, 0, 0, 0, 0, 0};
  size_t lds[4] = {0, 0, 0, 0};  // rhs, solve, out; y-marching rhs (0 unless every case allows it)
  int radix_rhs = 8, unroll = 2, radix_neu = 16, radix_out = 16;  // shared by all cases (unroll 3: y-march)
  hipStream_t stream = nullptr;
};
template <typename T> void fill_case_desc(const Plan &p, int cur, void *desc_host);
template <typename T> size_t case_desc_bytes();
template <typename T> void case_tiles(const Plan &p, int *tiles, size_t *lds);
template <typename T> hipError_t enqueue_batch_step(const BatchLaunch &bl, int parity);

// Logical tile of hardware block b of nb: blocks are dealt round-robin to the 8 XCDs, so this
// gives each XCD a run of consecutive tiles and neighbouring tiles (which read each other's halo
// lines) share its L2.  A permutation of [0, nb) when nb is a multiple of 8, else the identity.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  if ((nb & 7) == 0) {
    const int per = nb >> 3;
    return (b & 7) * per + (b >> 3);
  }
  return b;
}

// Launch-shape helpers shared with the host (elements per LDS tile).
template <typename T> constexpr int tile_elems() { return 32768 / (int)sizeof(T); }  // 32 KB of LDS

}  // namespace chib
