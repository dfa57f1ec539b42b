// C ABI of the library: state creation inside a caller-owned device workspace, field
// transfer, the step loop, diagnostics, stage entry points and checkpoints.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"
#include "kernels.h"

using chib::fail;

namespace {

constexpr int kVersion = 10000;  // 1.0.0
constexpr uint32_t kMagic = 0x42494843u;  // "CHIB"
constexpr int kNred = 8192;   // blocks of the first reduction pass (8 cells per thread at 256^3)

struct FaceList {
  std::vector<int> cell, axis, gL, gR;
};

// Faces with a ghost on either side (section 4.3: their velocity is re-interpolated).
FaceList build_faces(const ch_ib_geometry &g) {
  FaceList fl;
  const int d = g.ndim;
  const int64_t G = g.n_ghost;
  const int nx = g.n[0], ny = g.n[1];
  std::vector<std::pair<int, int64_t>> faces;  // (axis, left cell)
  faces.reserve((size_t)G * 2 * d);
  auto shift = [&](int64_t c, int a, int s) -> int64_t {
    int i = (int)(c % nx), j = (int)((c / nx) % ny), k = (int)(c / ((int64_t)nx * ny));
    int q[3] = {i, j, k};
    q[a] += s;
    if (a < d - 1) q[a] = (q[a] + g.n[a]) % g.n[a];
    return q[0] + (int64_t)nx * (q[1] + (int64_t)ny * q[2]);
  };
  for (int64_t gi = 0; gi < G; ++gi) {
    const int64_t c = g.gidx[gi];
    for (int a = 0; a < d; ++a) {
      faces.emplace_back(a, shift(c, a, -1));
      faces.emplace_back(a, c);
    }
  }
  std::sort(faces.begin(), faces.end());
  faces.erase(std::unique(faces.begin(), faces.end()), faces.end());
  auto ghost_of = [&](int64_t c) -> int {
    auto it = std::lower_bound(g.gidx.begin(), g.gidx.end(), c);
    return (it != g.gidx.end() && *it == c) ? (int)(it - g.gidx.begin()) : -1;
  };
  for (auto &f : faces) {
    fl.axis.push_back(f.first);
    fl.cell.push_back((int)f.second);
    fl.gL.push_back(ghost_of(f.second));
    fl.gR.push_back(ghost_of(shift(f.second, f.first, 1)));
  }
  return fl;
}

// Cells whose rhs the wall condition dphi/dn = 0 changes (section 4.2.2): every ghost and its face
// neighbours, sorted by cell, each with its own ghost index and those of its 2d face neighbours
// (-1 where the cell or the neighbour is no ghost), and the first entry of every x-row.
struct PatchList {
  std::vector<int> cell;   // [NP]
  std::vector<int> ref;    // [2d+1][NP]
  std::vector<int> row;    // [rows+1]
  // cells where dg needs phi~ (every ghost's averaging points and the ghost itself), sorted, and
  // for every slot of every ghost (ghost-major, kGhostSlots per ghost; slot 2K the ghost) its index
  std::vector<int> pt_cell;   // [NU]
  std::vector<int> pt_idx;    // [G][kGhostSlots]
};

PatchList build_patch(const ch_ib_geometry &g) {
  PatchList pl;
  const int d = g.ndim;
  const int64_t G = g.n_ghost;
  if (G == 0) return pl;
  const int nx = g.n[0], ny = g.n[1];
  auto shift = [&](int64_t c, int a, int s) -> int64_t {
    int q[3] = {(int)(c % nx), (int)((c / nx) % ny), (int)(c / ((int64_t)nx * ny))};
    q[a] += s;
    if (a < d - 1) q[a] = (q[a] + g.n[a]) % g.n[a];
    if (q[a] < 0 || q[a] >= g.n[a]) return -1;   // beyond a box wall (never for a ghost's neighbour)
    return q[0] + (int64_t)nx * (q[1] + (int64_t)ny * q[2]);
  };
  std::vector<int64_t> cells;
  cells.reserve((size_t)G * (2 * d + 1));
  for (int64_t gi = 0; gi < G; ++gi) {
    const int64_t c = g.gidx[gi];
    cells.push_back(c);
    for (int a = 0; a < d; ++a)
      for (int sgn : {1, -1}) {
        const int64_t q = shift(c, a, sgn);
        if (q >= 0) cells.push_back(q);
      }
  }
  std::sort(cells.begin(), cells.end());
  cells.erase(std::unique(cells.begin(), cells.end()), cells.end());
  const int64_t NP = (int64_t)cells.size();
  auto ghost_of = [&](int64_t c) -> int {
    if (c < 0) return -1;
    auto it = std::lower_bound(g.gidx.begin(), g.gidx.end(), c);
    return (it != g.gidx.end() && *it == c) ? (int)(it - g.gidx.begin()) : -1;
  };
  const int nref = 2 * d + 1;
  pl.cell.resize(NP);
  pl.ref.assign((size_t)nref * NP, -1);
  for (int64_t e = 0; e < NP; ++e) {
    const int64_t c = cells[e];
    pl.cell[e] = (int)c;
    pl.ref[e] = ghost_of(c);
    for (int a = 0; a < d; ++a) {
      pl.ref[(size_t)(1 + 2 * a) * NP + e] = ghost_of(shift(c, a, 1));
      pl.ref[(size_t)(2 + 2 * a) * NP + e] = ghost_of(shift(c, a, -1));
    }
  }
  const int64_t rows = g.cells / nx;
  pl.row.assign((size_t)rows + 1, 0);
  int64_t e = 0;
  for (int64_t r = 0; r <= rows; ++r) {
    while (e < NP && cells[e] / nx < r) ++e;
    pl.row[r] = (int)e;
  }
  const int KK = 2 * g.n_ap;
  std::vector<int64_t> pts(g.ap.begin(), g.ap.end());
  pts.insert(pts.end(), g.gidx.begin(), g.gidx.end());
  std::sort(pts.begin(), pts.end());
  pts.erase(std::unique(pts.begin(), pts.end()), pts.end());
  pl.pt_cell.assign(pts.begin(), pts.end());
  pl.pt_idx.assign((size_t)G * chib::kGhostSlots, 0);
  auto pt_of = [&](int64_t c) { return (int)(std::lower_bound(pts.begin(), pts.end(), c) - pts.begin()); };
  for (int64_t gi = 0; gi < G; ++gi) {
    for (int k = 0; k < KK; ++k) pl.pt_idx[(size_t)gi * chib::kGhostSlots + k] = pt_of(g.ap[(size_t)k * G + gi]);
    pl.pt_idx[(size_t)gi * chib::kGhostSlots + KK] = pt_of(g.gidx[gi]);
  }
  return pl;
}

struct Layout {
  size_t total = 0;
  size_t off(size_t bytes) {
    size_t o = total;
    total += (bytes + 255) & ~(size_t)255;
    return o;
  }
};

struct Offsets {
  size_t C[2], F[3], W, R, alpha, gidx, normal, dn, gamma, ap, w, apg, wg, CGn, CGnm1, CMs, CI, CGnew, UG;
  size_t dg, pl_cell, pl_ref, pl_row, pl_dq, pt_cell, pt_idx, pt_phi;
  size_t Us[3], Ut[3], Nh[3], Af[3], P[2];
  size_t f_cell, f_axis, f_gL, f_gR, stashL, stashR;
  size_t twr[3], twi[3], dctc, dcts, lam[3], partial, red_out;
  size_t total;
};

Offsets plan_layout(const ch_ib_geometry &g, int es, int64_t NF, const PatchList &pl, bool explicit_ab2, bool ns) {
  const int64_t NP = (int64_t)pl.cell.size(), NU = (int64_t)pl.pt_cell.size();
  Layout L;
  Offsets o{};
  const int64_t N = g.cells, G = g.n_ghost;
  const int d = g.ndim, K = g.n_ap;
  o.C[0] = L.off(N * es);
  o.C[1] = L.off(N * es);
  for (int a = 0; a < 3; ++a) o.F[a] = a < d ? L.off(N * es) : 0;
  o.W = L.off(N * es);
  o.R = explicit_ab2 ? L.off(N * es) : 0;
  // momentum step: u**, the advecting 2u^n - u^(n-1) (semi-implicit only), the previous
  // convective term, the staggered-cell fractions and two pressure levels
  for (int a = 0; a < 3; ++a) {
    o.Us[a] = ns && a < d ? L.off(N * es) : 0;
    o.Ut[a] = ns && !explicit_ab2 && a < d ? L.off(N * es) : 0;
    o.Nh[a] = ns && a < d ? L.off(N * es) : 0;
    o.Af[a] = ns && a < d ? L.off(N * es) : 0;
  }
  for (int k = 0; k < 2; ++k) o.P[k] = ns ? L.off(N * es) : 0;
  o.alpha = g.alpha.empty() ? 0 : L.off(N * es);
  o.gidx = L.off(G * 4);
  o.normal = L.off(d * G * es);
  o.dn = L.off(G * es);
  o.gamma = L.off(G * es);
  o.ap = L.off(2 * K * G * 4);
  o.w = L.off(2 * K * G * es);
  o.apg = L.off(chib::kGhostSlots * G * 4);
  o.wg = L.off(chib::kGhostSlots * G * es);
  o.CGn = L.off(G * es);
  o.CGnm1 = L.off(G * es);
  o.CMs = L.off(G * es);
  o.CI = L.off(G * es);
  o.CGnew = L.off(G * es);
  o.UG = L.off(d * G * es);
  o.dg = L.off(G * es);
  o.pl_cell = L.off(NP * 4);
  o.pl_ref = L.off((2 * d + 1) * NP * 4);
  o.pl_row = L.off((N / g.n[0] + 1) * 4);
  o.pl_dq = L.off(NP * es);
  o.pt_cell = L.off(NU * 4);
  o.pt_idx = L.off((int64_t)pl.pt_idx.size() * 4);
  o.pt_phi = L.off(NU * es);
  o.f_cell = L.off(NF * 4);
  o.f_axis = L.off(NF * 4);
  o.f_gL = L.off(NF * 4);
  o.f_gR = L.off(NF * 4);
  o.stashL = L.off(NF * es);
  o.stashR = L.off(NF * es);
  for (int a = 0; a < 3; ++a) {
    o.twr[a] = a < d ? L.off(g.n[a] * es) : 0;
    o.twi[a] = a < d ? L.off(g.n[a] * es) : 0;
    o.lam[a] = a < d ? L.off(g.n[a] * es) : 0;
  }
  o.dctc = L.off((g.n[d - 1] / 2 + 1) * es);
  o.dcts = L.off((g.n[d - 1] / 2 + 1) * es);
  o.partial = L.off(kNred * 8 * sizeof(double));
  o.red_out = L.off(8 * sizeof(double));
  o.total = L.total;
  return o;
}

int check_params(const ch_ib_params *p, double *S, double *alpha_s, double *a) {
  if (!p) return fail(CH_IB_EINVAL, "params is NULL");
  if (!(p->Cn > 0) || !(p->Pe > 0) || !(p->dt > 0)) return fail(CH_IB_EINVAL, "Cn, Pe and dt must be positive");
  if (p->precision != 64 && p->precision != 32) return fail(CH_IB_EINVAL, "precision must be 64 or 32");
  if (p->Vs < 0 || p->slip_length < 0) return fail(CH_IB_EINVAL, "Vs and slip_length must be >= 0");
  if ((p->flags & (CH_IB_FLAG_VELOCITY_FILL | CH_IB_FLAG_NAVIER_STOKES)) && (!(p->Ca > 0) || !(p->mu > 0)))
    return fail(CH_IB_EINVAL, "Ca and mu must be positive for the velocity fill");
  if ((p->flags & CH_IB_FLAG_NAVIER_STOKES) &&
      (!(p->Re > 0) || !(p->rho1 > 0) || !(p->rho2 > 0) || !(p->mu1 > 0) || !(p->mu2 > 0) ||
       !std::isfinite(p->body_force[0]) || !std::isfinite(p->body_force[1]) || !std::isfinite(p->body_force[2])))
    return fail(CH_IB_EINVAL, "the momentum step needs positive Re, rho1, rho2, mu1, mu2 and a finite body force");
  const double Cn = p->Cn, Pe = p->Pe, dt = p->dt;
  const double Smin = Cn * std::sqrt(6.0 * Pe / dt);
  const double Sv = p->S > 0 ? p->S : Smin;
  double disc = 1.0 - 6.0 * Cn * Cn * Pe / (dt * Sv * Sv);
  if (disc < -1e-12) return fail(CH_IB_EINVAL, "S is below the stability bound Cn sqrt(6 Pe/dt)");
  disc = std::max(disc, 0.0);
  const double al = -(Sv / (2.0 * Cn * Cn)) * (1.0 + std::sqrt(disc));
  if (S) *S = Sv;
  if (alpha_s) *alpha_s = al;
  if (a) *a = al + Sv / (Cn * Cn);
  return CH_IB_OK;
}

}  // namespace

struct ch_ib_state {
  ch_ib_geometry geom;  // copy of grid info and host tables (alpha kept only on device)
  ch_ib_params prm{};
  int es = 8;
  chib::Plan plan;
  char *ws = nullptr;
  Offsets off{};
  int cur = 0;
  int needs_init = 1;
  int64_t step = 0;
  int sticky = CH_IB_OK;
  int has_alpha = 0;
  int r_valid = 0;      // explicit step: R holds the previous step's rate
  int ns_first = 1;     // momentum step: no previous convective term yet
  int ut_valid = 0;     // momentum step: Ut holds 2u^n - u^(n-1)
  double d1_min = 0, d1_max = 0;   // range of gamma dn = d1 over the ghosts (mixed-condition checks)
};

static int hip_fail(ch_ib_state *st, hipError_t e, const char *where) {
  std::string m = std::string(where) + ": " + hipGetErrorString(e);
  if (st) st->sticky = CH_IB_EHIP;
  return fail(CH_IB_EHIP, m);
}

template <typename T>
static void upload(std::vector<T> &host_keep, const std::vector<double> &src, void *dst, hipStream_t s) {
  host_keep.assign(src.begin(), src.end());
  if (!host_keep.empty())
    (void)hipMemcpyAsync(dst, host_keep.data(), host_keep.size() * sizeof(T), hipMemcpyHostToDevice, s);
}

extern "C" const char *ch_ib_strerror(int status) {
  switch (status) {
    case CH_IB_OK: return "ok";
    case CH_IB_EINVAL: return "invalid argument";
    case CH_IB_EGEOM: return "geometry preprocessing failed";
    case CH_IB_EHIP: return "HIP runtime error";
    case CH_IB_ENOMEM: return "workspace or buffer too small";
    case CH_IB_ENAN: return "non-finite value in the state";
    case CH_IB_EUNSUPPORTED: return "unsupported request";
    default: return "unknown status";
  }
}

extern "C" int ch_ib_version(void) { return kVersion; }

extern "C" int ch_ib_coefficients(const ch_ib_params *params, double *S, double *alpha_s, double *a) {
  return check_params(params, S, alpha_s, a);
}

extern "C" size_t ch_ib_workspace_bytes(const ch_ib_grid *grid, const ch_ib_geometry *geom,
                                        const ch_ib_params *params) {
  if (!grid || !geom || !params) return 0;
  ch_ib_geometry tmp;
  if (chib::check_grid(grid, &tmp)) return 0;
  if (tmp.cells != geom->cells || tmp.ndim != geom->ndim) return 0;
  if (params->precision != 64 && params->precision != 32) return 0;
  const int es = params->precision == 64 ? 8 : 4;
  FaceList fl = build_faces(*geom);
  PatchList pl = build_patch(*geom);
  return plan_layout(*geom, es, (int64_t)fl.cell.size(), pl,
                     (params->flags & CH_IB_FLAG_EXPLICIT) != 0, (params->flags & CH_IB_FLAG_NAVIER_STOKES) != 0)
             .total +
         256;
}

extern "C" int ch_ib_state_create(const ch_ib_grid *grid, const ch_ib_geometry *geom, const ch_ib_params *params,
                                  void *device_workspace, size_t bytes, void *hip_stream, ch_ib_state **out) {
  if (!out) return fail(CH_IB_EINVAL, "out is NULL");
  *out = nullptr;
  if (!geom || !device_workspace) return fail(CH_IB_EINVAL, "NULL geometry or workspace");
  double S, al, a;
  int rc = check_params(params, &S, &al, &a);
  if (rc) return rc;
  ch_ib_geometry chk;
  if ((rc = chib::check_grid(grid, &chk))) return rc;
  if (chk.cells != geom->cells || chk.ndim != geom->ndim) return fail(CH_IB_EINVAL, "geometry built for another grid");
  const size_t need = ch_ib_workspace_bytes(grid, geom, params);
  if (bytes < need) return fail(CH_IB_ENOMEM, "workspace too small: need " + std::to_string(need) + " bytes");
  if (((uintptr_t)device_workspace) & 255) return fail(CH_IB_EINVAL, "workspace must be 256-byte aligned");

  if ((params->flags & CH_IB_FLAG_NAVIER_STOKES) &&
      geom->face_alpha.size() != (size_t)geom->ndim * (size_t)geom->cells)
    return fail(CH_IB_EINVAL, "the momentum step needs a geometry with staggered-cell fractions");
  if ((params->flags & CH_IB_FLAG_NAVIER_STOKES) && geom->cells >= ((int64_t)1 << 31))
    return fail(CH_IB_EUNSUPPORTED, "the momentum step indexes cells with 32-bit integers (fewer than 2^31 cells)");
  auto *st = new ch_ib_state();
  st->geom = *geom;
  st->prm = *params;
  st->es = params->precision == 64 ? 8 : 4;
  st->ws = (char *)device_workspace;
  st->has_alpha = !geom->alpha.empty();
  FaceList fl = build_faces(*geom);
  const int64_t NF = (int64_t)fl.cell.size();
  PatchList pl = build_patch(*geom);
  const int64_t NP = (int64_t)pl.cell.size();
  const bool ns = (params->flags & CH_IB_FLAG_NAVIER_STOKES) != 0;
  st->off = plan_layout(*geom, st->es, NF, pl, (params->flags & CH_IB_FLAG_EXPLICIT) != 0, ns);
  const Offsets &o = st->off;
  chib::Plan &p = st->plan;
  const int d = geom->ndim;
  p.d = d;
  for (int ax = 0; ax < 3; ++ax) {
    p.n[ax] = geom->n[ax];
    int l = 0;
    while ((1 << l) < geom->n[ax]) ++l;
    p.logn[ax] = l;
  }
  p.N = geom->cells;
  p.h = geom->h;
  p.Pe = params->Pe;
  p.Cn = params->Cn;
  p.dt = params->dt;
  p.S = S;
  p.alpha_s = al;
  p.a = a;
  p.cos_t = std::cos(params->theta_deg * M_PI / 180.0);
  p.Ca = params->Ca;
  p.mu = params->mu;
  p.ls = params->slip_length;
  p.Vs = params->Vs;
  p.vel_fill = (params->flags & CH_IB_FLAG_VELOCITY_FILL) ? 1 : 0;
  p.dynamic = params->Vs > 0 ? 1 : 0;
  p.explicit_ab2 = (params->flags & CH_IB_FLAG_EXPLICIT) ? 1 : 0;
  if (ns) {
    p.ns = 1;
    p.vel_fill = 1;
    p.Re = params->Re;
    p.rho1 = params->rho1;
    p.rho2 = params->rho2;
    p.mu1 = params->mu1;
    p.mu2 = params->mu2;
    for (int a = 0; a < 3; ++a) p.g[a] = a < geom->ndim ? params->body_force[a] : 0.0;
  }
  char *W0 = st->ws;
  p.C[0] = W0 + o.C[0];
  p.C[1] = W0 + o.C[1];
  for (int ax = 0; ax < 3; ++ax) p.F[ax] = ax < d ? W0 + o.F[ax] : nullptr;
  p.W = W0 + o.W;
  p.R = p.explicit_ab2 ? W0 + o.R : nullptr;
  for (int a = 0; a < 3; ++a) {
    p.Us[a] = ns && a < d ? W0 + o.Us[a] : nullptr;
    p.Ut[a] = ns && !p.explicit_ab2 && a < d ? W0 + o.Ut[a] : nullptr;
    p.Nh[a] = ns && a < d ? W0 + o.Nh[a] : nullptr;
    p.Af[a] = ns && a < d ? W0 + o.Af[a] : nullptr;
  }
  for (int k = 0; k < 2; ++k) p.P[k] = ns ? W0 + o.P[k] : nullptr;
  p.alpha = st->has_alpha ? W0 + o.alpha : nullptr;
  p.G = geom->n_ghost;
  p.K = geom->n_ap;
  p.gidx = (const int *)(W0 + o.gidx);
  p.normal = W0 + o.normal;
  p.dn = W0 + o.dn;
  p.gamma = W0 + o.gamma;
  p.ap = (const int *)(W0 + o.ap);
  p.w = W0 + o.w;
  p.apg = (const int *)(W0 + o.apg);
  p.wg = W0 + o.wg;
  p.CGn = W0 + o.CGn;
  p.CGnm1 = W0 + o.CGnm1;
  p.CMs = W0 + o.CMs;
  p.CI = W0 + o.CI;
  p.CGnew = W0 + o.CGnew;
  p.UG = W0 + o.UG;
  p.dg = W0 + o.dg;
  p.NP = NP;
  p.pl_cell = (const int *)(W0 + o.pl_cell);
  p.pl_ref = (const int *)(W0 + o.pl_ref);
  p.pl_row = (const int *)(W0 + o.pl_row);
  p.pl_dq = W0 + o.pl_dq;
  p.NU = (int64_t)pl.pt_cell.size();
  p.pt_cell = (const int *)(W0 + o.pt_cell);
  p.pt_idx = (const int *)(W0 + o.pt_idx);
  p.pt_phi = W0 + o.pt_phi;
  p.NF = NF;
  p.f_cell = (const int *)(W0 + o.f_cell);
  p.f_axis = (const int *)(W0 + o.f_axis);
  p.f_gL = (const int *)(W0 + o.f_gL);
  p.f_gR = (const int *)(W0 + o.f_gR);
  p.stashL = W0 + o.stashL;
  p.stashR = W0 + o.stashR;
  for (int ax = 0; ax < 3; ++ax) {
    p.twr[ax] = ax < d ? W0 + o.twr[ax] : nullptr;
    p.twi[ax] = ax < d ? W0 + o.twi[ax] : nullptr;
    p.lam[ax] = ax < d ? W0 + o.lam[ax] : nullptr;
  }
  p.dctc = W0 + o.dctc;
  p.dcts = W0 + o.dcts;
  p.partial = W0 + o.partial;
  p.red_out = W0 + o.red_out;
  p.nred = (int)std::min<int64_t>(kNred, (p.N + 255) / 256);
  p.stream = (hipStream_t)hip_stream;

  // host-side tables in double, converted to the element type on upload
  const int64_t G = geom->n_ghost;
  const double h = geom->h;
  std::vector<double> tw[3][2], lam[3], dctc, dcts;
  for (int ax = 0; ax < d; ++ax) {
    const int n = geom->n[ax];
    tw[ax][0].resize(n);
    tw[ax][1].resize(n);
    lam[ax].resize(n);
    for (int m = 0; m < n; ++m) {
      const double ang = 2.0 * M_PI * (double)m / (double)n;
      tw[ax][0][m] = std::cos(ang);
      tw[ax][1][m] = -std::sin(ang);
      const double sarg = ax < d - 1 ? M_PI * (double)m / (double)n : M_PI * (double)m / (2.0 * n);
      const double sv = std::sin(sarg);
      lam[ax][m] = -(4.0 / (h * h)) * sv * sv;
    }
  }
  {
    const int n = geom->n[d - 1];
    dctc.resize(n / 2 + 1);
    dcts.resize(n / 2 + 1);
    for (int k = 0; k <= n / 2; ++k) {
      dctc[k] = std::cos(M_PI * (double)k / (2.0 * n));
      dcts[k] = std::sin(M_PI * (double)k / (2.0 * n));
    }
  }
  std::vector<int> gidx32(G), ap32(geom->ap.size());
  for (int64_t i = 0; i < G; ++i) gidx32[i] = (int)geom->gidx[i];
  for (size_t i = 0; i < geom->ap.size(); ++i) ap32[i] = (int)geom->ap[i];
  // ghost-major copies: slot k of ghost g at g * kGhostSlots + k
  const int KK = 2 * geom->n_ap;
  std::vector<int> apg32((size_t)G * chib::kGhostSlots, 0);
  std::vector<double> wgv((size_t)G * chib::kGhostSlots, 0.0);
  for (int64_t g = 0; g < G; ++g)
    for (int k = 0; k < KK; ++k) {
      apg32[(size_t)g * chib::kGhostSlots + k] = ap32[(size_t)k * G + g];
      wgv[(size_t)g * chib::kGhostSlots + k] = geom->w[(size_t)k * G + g];
    }
  hipStream_t s = p.stream;
  std::vector<std::vector<double>> keep_d;
  std::vector<std::vector<float>> keep_f;
  keep_d.reserve(32);
  keep_f.reserve(32);
  auto up = [&](const std::vector<double> &src, void *dst) {
    if (st->es == 8) {
      keep_d.emplace_back();
      upload(keep_d.back(), src, dst, s);
    } else {
      keep_f.emplace_back();
      upload(keep_f.back(), src, dst, s);
    }
  };
  hipError_t e = hipSuccess;
  if (G) {
    e = hipMemcpyAsync((void *)p.gidx, gidx32.data(), G * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync((void *)p.ap, ap32.data(), ap32.size() * 4, hipMemcpyHostToDevice, s);
    up(geom->normal, (void *)p.normal);
    up(geom->dn, (void *)p.dn);
    up(geom->gamma, (void *)p.gamma);
    up(geom->w, (void *)p.w);
    if (e == hipSuccess) e = hipMemcpyAsync((void *)p.apg, apg32.data(), apg32.size() * 4, hipMemcpyHostToDevice, s);
    up(wgv, (void *)p.wg);
  }
  if (NP && e == hipSuccess) {
    e = hipMemcpyAsync((void *)p.pl_cell, pl.cell.data(), NP * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync((void *)p.pl_ref, pl.ref.data(), pl.ref.size() * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync((void *)p.pl_row, pl.row.data(), pl.row.size() * 4, hipMemcpyHostToDevice, s);
  }
  if (p.NU && e == hipSuccess) {
    e = hipMemcpyAsync((void *)p.pt_cell, pl.pt_cell.data(), pl.pt_cell.size() * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync((void *)p.pt_idx, pl.pt_idx.data(), pl.pt_idx.size() * 4, hipMemcpyHostToDevice, s);
  }
  if (NF && e == hipSuccess) {
    e = hipMemcpyAsync((void *)p.f_cell, fl.cell.data(), NF * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync((void *)p.f_axis, fl.axis.data(), NF * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync((void *)p.f_gL, fl.gL.data(), NF * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync((void *)p.f_gR, fl.gR.data(), NF * 4, hipMemcpyHostToDevice, s);
  }
  for (int ax = 0; ax < d; ++ax) {
    up(tw[ax][0], (void *)p.twr[ax]);
    up(tw[ax][1], (void *)p.twi[ax]);
    up(lam[ax], (void *)p.lam[ax]);
  }
  up(dctc, (void *)p.dctc);
  up(dcts, (void *)p.dcts);
  if (st->has_alpha) up(geom->alpha, p.alpha);
  if (ns) {
    std::vector<double> fa((size_t)p.N);
    for (int a = 0; a < d; ++a) {
      std::copy(geom->face_alpha.begin() + (size_t)a * p.N, geom->face_alpha.begin() + (size_t)(a + 1) * p.N,
                fa.begin());
      up(fa, p.Af[a]);
    }
  }
  // fields start at zero
  if (e == hipSuccess) e = hipMemsetAsync(p.C[0], 0, (size_t)p.N * st->es, s);
  if (e == hipSuccess) e = hipMemsetAsync(p.C[1], 0, (size_t)p.N * st->es, s);
  for (int ax = 0; ax < d && e == hipSuccess; ++ax) e = hipMemsetAsync(p.F[ax], 0, (size_t)p.N * st->es, s);
  for (int ax = 0; ns && ax < d && e == hipSuccess; ++ax) {
    e = hipMemsetAsync(p.Us[ax], 0, (size_t)p.N * st->es, s);
    if (e == hipSuccess) e = hipMemsetAsync(p.Nh[ax], 0, (size_t)p.N * st->es, s);
    if (e == hipSuccess && p.Ut[ax]) e = hipMemsetAsync(p.Ut[ax], 0, (size_t)p.N * st->es, s);
  }
  for (int k = 0; ns && k < 2 && e == hipSuccess; ++k) e = hipMemsetAsync(p.P[k], 0, (size_t)p.N * st->es, s);
  if (G && e == hipSuccess) e = hipMemsetAsync(p.CI, 0, (size_t)G * st->es, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) {
    delete st;
    return hip_fail(nullptr, e, "state upload");
  }
  st->geom.alpha.clear();
  st->geom.alpha.shrink_to_fit();
  st->geom.face_alpha.clear();
  st->geom.face_alpha.shrink_to_fit();
  if (G) {
    st->d1_min = st->d1_max = geom->gamma[0] * geom->dn[0];
    for (int64_t i = 1; i < G; ++i) {
      const double v = geom->gamma[i] * geom->dn[i];
      st->d1_min = std::min(st->d1_min, v);
      st->d1_max = std::max(st->d1_max, v);
    }
  }
  *out = st;
  return CH_IB_OK;
}

static int64_t field_count(const ch_ib_state *st, int field) {
  switch (field) {
    case CH_IB_FIELD_C:
    case CH_IB_FIELD_C_PREV:
    case CH_IB_FIELD_ALPHA:
    case CH_IB_FIELD_PHI: return st->plan.N;
    case CH_IB_FIELD_U:
    case CH_IB_FIELD_V: return st->plan.N;
    case CH_IB_FIELD_W: return st->plan.d == 3 ? st->plan.N : -1;
    case CH_IB_FIELD_CI: return st->plan.G;
    case CH_IB_FIELD_P: return st->plan.ns ? st->plan.N : -1;
    default: return -1;
  }
}

extern "C" int ch_ib_state_set(ch_ib_state *st, int field, const void *src, int src_on_device) {
  if (!st || !src) return fail(CH_IB_EINVAL, "NULL argument");
  const int64_t cnt = field_count(st, field);
  if (cnt < 0) return fail(CH_IB_EINVAL, "unknown field for this grid");
  void *dst = nullptr;
  chib::Plan &p = st->plan;
  switch (field) {
    case CH_IB_FIELD_C: dst = p.C[st->cur]; break;
    case CH_IB_FIELD_U: dst = p.F[0]; break;
    case CH_IB_FIELD_V: dst = p.F[1]; break;
    case CH_IB_FIELD_W: dst = p.F[2]; break;
    case CH_IB_FIELD_CI: dst = p.CI; break;
    default: return fail(CH_IB_EINVAL, "field is read-only");
  }
  if (cnt == 0) return CH_IB_OK;
  hipError_t e = hipMemcpyAsync(dst, src, (size_t)cnt * st->es,
                                src_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, p.stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p.stream);
  if (e != hipSuccess) return hip_fail(st, e, "state_set");
  if (field != CH_IB_FIELD_CI) {
    st->needs_init = 1;
    st->r_valid = 0;
    st->ns_first = 1;
    st->ut_valid = 0;
    // new fields restart the momentum history: no pressure yet (p^ = 0 in the first step)
    for (int k = 0; k < 2 && p.ns && e == hipSuccess; ++k)
      e = hipMemsetAsync(p.P[k], 0, (size_t)p.N * st->es, p.stream);
    if (p.ns && e == hipSuccess) e = hipStreamSynchronize(p.stream);
    if (e != hipSuccess) return hip_fail(st, e, "state_set");
  }
  return CH_IB_OK;
}

template <typename T>
static hipError_t run_init(ch_ib_state *st) {
  return chib::enqueue_initial_fill<T>(st->plan, st->cur);
}

static int ensure_init(ch_ib_state *st) {
  if (!st->needs_init) return CH_IB_OK;
  hipError_t e = st->es == 8 ? run_init<double>(st) : run_init<float>(st);
  if (e != hipSuccess) return hip_fail(st, e, "initial fill");
  st->needs_init = 0;
  return CH_IB_OK;
}

int chib::state_ref(ch_ib_state *st, chib::StateRef *out) {
  if (!st || !out) return fail(CH_IB_EINVAL, "NULL argument");
  if (st->sticky) return fail(st->sticky, "state is in an error state");
  int rc = ensure_init(st);
  if (rc) return rc;
  out->plan = &st->plan;
  out->cur = st->cur;
  out->es = st->es;
  return CH_IB_OK;
}

void chib::state_mark_reinit(ch_ib_state *st) {
  if (st) st->needs_init = 1;
}

void chib::state_copy_momentum_flags(const ch_ib_state *from, ch_ib_state *to) {
  if (!from || !to) return;
  to->ns_first = from->ns_first;
  to->ut_valid = from->ut_valid;
}

extern "C" int ch_ib_state_get(ch_ib_state *st, int field, void *dst, int dst_on_device) {
  if (!st || !dst) return fail(CH_IB_EINVAL, "NULL argument");
  const int64_t cnt = field_count(st, field);
  if (cnt < 0) return fail(CH_IB_EINVAL, "unknown field for this grid");
  chib::Plan &p = st->plan;
  const void *src = nullptr;
  hipError_t e = hipSuccess;
  switch (field) {
    case CH_IB_FIELD_C: src = p.C[st->cur]; break;
    case CH_IB_FIELD_C_PREV: src = p.C[1 - st->cur]; break;
    case CH_IB_FIELD_U: src = p.F[0]; break;
    case CH_IB_FIELD_V: src = p.F[1]; break;
    case CH_IB_FIELD_W: src = p.F[2]; break;
    case CH_IB_FIELD_CI: src = p.CI; break;
    case CH_IB_FIELD_P: src = p.P[0]; break;
    case CH_IB_FIELD_ALPHA:
      if (!st->has_alpha) {
        if (st->es == 8) {
          std::vector<double> ones(cnt, 1.0);
          e = hipMemcpyAsync(p.W, ones.data(), cnt * 8, hipMemcpyHostToDevice, p.stream);
          if (e == hipSuccess) e = hipStreamSynchronize(p.stream);
        } else {
          std::vector<float> ones(cnt, 1.0f);
          e = hipMemcpyAsync(p.W, ones.data(), cnt * 4, hipMemcpyHostToDevice, p.stream);
          if (e == hipSuccess) e = hipStreamSynchronize(p.stream);
        }
        src = p.W;
      } else {
        src = p.alpha;
      }
      break;
    case CH_IB_FIELD_PHI: {
      int rc = ensure_init(st);
      if (rc) return rc;
      e = st->es == 8 ? chib::enqueue_phi<double>(p, st->cur, p.W) : chib::enqueue_phi<float>(p, st->cur, p.W);
      src = p.W;
      break;
    }
    default: return fail(CH_IB_EINVAL, "bad field");
  }
  if (e != hipSuccess) return hip_fail(st, e, "state_get");
  if (cnt == 0) return CH_IB_OK;
  e = hipMemcpyAsync(dst, src, (size_t)cnt * st->es, dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                     p.stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p.stream);
  if (e != hipSuccess) return hip_fail(st, e, "state_get");
  return CH_IB_OK;
}

// One step of the state's scheme; the explicit scheme's first step after (re)initialisation has no
// previous rate.
static hipError_t enqueue_one_step(ch_ib_state *st, chib::KernelTimer *tm) {
  chib::Plan &p = st->plan;
  hipError_t e = hipSuccess;
  chib::Plan q = p;   // the order-parameter part
  if (p.ns) {
    // the momentum step does the velocity fill; the semi-implicit rhs advects with 2u^n - u^(n-1)
    q.vel_fill = 0;
    if (!p.explicit_ab2) {
      for (int a = 0; a < p.d && !st->ut_valid && e == hipSuccess; ++a)
        e = hipMemcpyAsync(p.Ut[a], p.F[a], (size_t)p.N * st->es, hipMemcpyDeviceToDevice, p.stream);
      if (e != hipSuccess) return e;
      st->ut_valid = 1;
      for (int a = 0; a < 3; ++a) q.Fadv[a] = p.Ut[a];
    }
  }
  if (p.explicit_ab2) {
    e = st->es == 8 ? chib::enqueue_explicit_step<double>(q, st->cur, !st->r_valid, tm)
                    : chib::enqueue_explicit_step<float>(q, st->cur, !st->r_valid, tm);
    if (e == hipSuccess) st->r_valid = 1;
  } else {
    e = st->es == 8 ? chib::enqueue_step<double>(q, st->cur, tm) : chib::enqueue_step<float>(q, st->cur, tm);
  }
  if (e != hipSuccess || !p.ns) return e;
  e = st->es == 8 ? chib::enqueue_momentum<double>(p, 1 - st->cur, st->ns_first, tm)
                  : chib::enqueue_momentum<float>(p, 1 - st->cur, st->ns_first, tm);
  if (e != hipSuccess) return e;
  st->ns_first = 0;
  // p^(n+1) is in W: it becomes p^n, p^n becomes p^(n-1), and p^(n-1)'s buffer the workspace
  void *w = p.W;
  p.W = p.P[1];
  p.P[1] = p.P[0];
  p.P[0] = w;
  return e;
}

extern "C" int ch_ib_step(ch_ib_state *st, int n_steps) {
  if (!st) return fail(CH_IB_EINVAL, "NULL state");
  if (n_steps < 0) return fail(CH_IB_EINVAL, "n_steps must be >= 0");
  if (st->sticky) return fail(st->sticky, "state is in an error state");
  int rc = ensure_init(st);
  if (rc) return rc;
  for (int i = 0; i < n_steps; ++i) {
    hipError_t e = enqueue_one_step(st, nullptr);
    if (e != hipSuccess) return hip_fail(st, e, "step");
    st->cur = 1 - st->cur;
    st->step++;
  }
  return CH_IB_OK;
}

extern "C" int ch_ib_step_timed(ch_ib_state *st, int n_steps, int max_kernels, double *ms_out,
                                const char **names_out, int *n_kernels) {
  if (!st || !ms_out || !names_out || !n_kernels) return fail(CH_IB_EINVAL, "NULL argument");
  if (n_steps < 1 || n_steps > 4096) return fail(CH_IB_EINVAL, "n_steps must be in 1..4096");
  if (st->sticky) return fail(st->sticky, "state is in an error state");
  int rc = ensure_init(st);
  if (rc) return rc;
  constexpr int ne = chib::KernelTimer::kMax + 1;
  std::vector<chib::KernelTimer> tms((size_t)n_steps);
  hipError_t e = hipSuccess;
  size_t created = 0;
  for (auto &tm : tms)
    for (int k = 0; k < ne && e == hipSuccess; ++k) {
      e = hipEventCreate(&tm.ev[k]);
      if (e == hipSuccess) ++created;   // only events that exist are destroyed below
    }
  // all steps are enqueued back to back; one wait at the end
  for (int s = 0; s < n_steps && e == hipSuccess; ++s) {
    tms[s].n = 0;
    e = enqueue_one_step(st, &tms[s]);
    if (e != hipSuccess) break;
    st->cur = 1 - st->cur;
    st->step++;
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st->plan.stream);
  std::vector<double> acc(chib::KernelTimer::kMax, 0.0);
  const int nk = tms[0].n;
  for (int s = 0; s < n_steps && e == hipSuccess; ++s)
    for (int k = 0; k < nk && e == hipSuccess; ++k) {
      float ms = 0.f;
      e = hipEventElapsedTime(&ms, tms[s].ev[k], tms[s].ev[k + 1]);
      acc[k] += ms;
    }
  size_t destroyed = 0;
  for (auto &tm : tms)
    for (int k = 0; k < ne && destroyed < created; ++k, ++destroyed) (void)hipEventDestroy(tm.ev[k]);
  if (e != hipSuccess) return hip_fail(st, e, "step_timed");
  if (nk > max_kernels) return fail(CH_IB_ENOMEM, "more kernels per step than max_kernels");
  for (int k = 0; k < nk; ++k) {
    ms_out[k] = acc[k] / n_steps;
    names_out[k] = tms[0].names[k];
  }
  *n_kernels = nk;
  return CH_IB_OK;
}

extern "C" int ch_ib_get_shapes(const ch_ib_state *st, int *out) {
  if (!st || !out) return fail(CH_IB_EINVAL, "NULL argument");
  for (int k = 0; k < 4; ++k) {
    out[3 * k] = st->plan.shape[k].log_tile;
    out[3 * k + 1] = st->plan.shape[k].radix;
    out[3 * k + 2] = st->plan.shape[k].unroll;
  }
  return CH_IB_OK;
}

extern "C" int ch_ib_set_shapes(ch_ib_state *st, const int *in) {
  if (!st || !in) return fail(CH_IB_EINVAL, "NULL argument");
  for (int k = 0; k < 4; ++k)
    if ((in[3 * k + 1] != 8 && in[3 * k + 1] != 16 && (k != 0 || in[3 * k + 1] != 4)) || in[3 * k] < 1 || in[3 * k] > 11 || in[3 * k + 2] < 1 ||
        in[3 * k + 2] > (k == 0 ? 8 : 2))
      return fail(CH_IB_EINVAL, "shape out of range");
  for (int k = 0; k < 4; ++k) st->plan.shape[k] = {in[3 * k], in[3 * k + 1], in[3 * k + 2]};
  return CH_IB_OK;
}

extern "C" int ch_ib_tune(ch_ib_state *st, int reps, int *out) {
  if (!st) return fail(CH_IB_EINVAL, "NULL state");
  if (reps < 1 || reps > 100) return fail(CH_IB_EINVAL, "reps must be in 1..100");
  if (st->sticky) return fail(st->sticky, "state is in an error state");
  int rc = ensure_init(st);
  if (rc) return rc;
  hipError_t e = st->es == 8 ? chib::tune_shapes<double>(st->plan, st->cur, reps)
                             : chib::tune_shapes<float>(st->plan, st->cur, reps);
  if (e == hipSuccess) e = hipStreamSynchronize(st->plan.stream);
  if (e != hipSuccess) return hip_fail(st, e, "tune");
  return out ? ch_ib_get_shapes(st, out) : CH_IB_OK;
}

extern "C" int ch_ib_sync(ch_ib_state *st) {
  if (!st) return fail(CH_IB_EINVAL, "NULL state");
  hipError_t e = hipStreamSynchronize(st->plan.stream);
  if (e != hipSuccess) return hip_fail(st, e, "sync");
  return st->sticky;
}

extern "C" int ch_ib_diagnostics(ch_ib_state *st, ch_ib_diag *out) {
  if (!st || !out) return fail(CH_IB_EINVAL, "NULL argument");
  int rc = ensure_init(st);
  if (rc) return rc;
  chib::Plan &p = st->plan;
  hipError_t e = st->es == 8 ? chib::enqueue_diag<double>(p, st->cur) : chib::enqueue_diag<float>(p, st->cur);
  double r[8];
  if (e == hipSuccess) e = hipMemcpyAsync(r, p.red_out, sizeof(r), hipMemcpyDeviceToHost, p.stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p.stream);
  if (e != hipSuccess) return hip_fail(st, e, "diagnostics");
  const double vol = std::pow(p.h, p.d);
  out->mass_box = vol * r[0];
  out->mass_fluid = vol * r[1];
  out->free_energy = vol * (r[2] - (2.0 * std::sqrt(2.0) / 3.0) * p.cos_t * r[3]);
  out->max_abs_C = r[4];
  out->step = st->step;
  out->status = r[5] > 0 ? CH_IB_ENAN : CH_IB_OK;
  out->pad_ = 0;
  if (out->status) return fail(CH_IB_ENAN, "non-finite value in C");
  return CH_IB_OK;
}

// ---------------------------------------------------------------------------------------------
// Diagnostics without any allocation: the reduction's partial sums (kNred blocks of 8) and its
// final 8 values live in a file-scope device array instead of the state's workspace.  Each GPU
// holds its own copy; its address is looked up once per device (with that device current) and
// only that address is used on the host.  Calls that overlap on one GPU share the array and race.
constexpr size_t kScratchPartials = kNred;
static __device__ __align__(256) double scratch[kScratchPartials * 8 + 8];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first call per device).
int scratch_address(void **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(CH_IB_EHIP, std::string("scratch: hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(CH_IB_EUNSUPPORTED, "scratch: device index beyond 63");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(CH_IB_EHIP, std::string("scratch: hipGetSymbolAddress: ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return CH_IB_OK;
}
}  // namespace

extern "C" int ch_ib_diagnostics_noalloc(ch_ib_state *st, ch_ib_diag *out) {
  if (!st || !out) return fail(CH_IB_EINVAL, "NULL argument");
  chib::Plan &p = st->plan;
  if ((size_t)p.nred > kScratchPartials)
    return fail(CH_IB_ENOMEM, "reduction needs " + std::to_string(p.nred) + " partial sums, the static scratch holds " +
                                  std::to_string(kScratchPartials));
  // the state's workspace must sit on the current device, whose copy of the array is used
  hipPointerAttribute_t attr{};
  hipError_t e = hipPointerGetAttributes(&attr, st->ws);
  int dev = -1;
  if (e == hipSuccess) e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(st, e, "diagnostics_noalloc");
  if (attr.device != dev) return fail(CH_IB_EINVAL, "the state's device is not the current device");
  void *base = nullptr;
  int rc = scratch_address(&base);
  if (rc) return rc;
  rc = ensure_init(st);
  if (rc) return rc;
  chib::Plan q = p;
  q.partial = base;
  q.red_out = (double *)base + kScratchPartials * 8;
  e = st->es == 8 ? chib::enqueue_diag<double>(q, st->cur) : chib::enqueue_diag<float>(q, st->cur);
  double r[8];
  if (e == hipSuccess) e = hipMemcpyAsync(r, q.red_out, sizeof(r), hipMemcpyDeviceToHost, p.stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p.stream);
  if (e != hipSuccess) return hip_fail(st, e, "diagnostics_noalloc");
  const double vol = std::pow(p.h, p.d);
  out->mass_box = vol * r[0];
  out->mass_fluid = vol * r[1];
  out->free_energy = vol * (r[2] - (2.0 * std::sqrt(2.0) / 3.0) * p.cos_t * r[3]);
  out->max_abs_C = r[4];
  out->step = st->step;
  out->status = r[5] > 0 ? CH_IB_ENAN : CH_IB_OK;
  out->pad_ = 0;
  if (out->status) return fail(CH_IB_ENAN, "non-finite value in C");
  return CH_IB_OK;
}

extern "C" int ch_ib_stage(ch_ib_state *st, int stage, const void *in_device, void *out_device) {
  if (!st || !out_device) return fail(CH_IB_EINVAL, "NULL argument");
  chib::Plan &p = st->plan;
  hipError_t e = hipSuccess;
  int rc = ensure_init(st);
  if (rc) return rc;
  switch (stage) {
    case CH_IB_STAGE_RHS:
      e = st->es == 8 ? chib::enqueue_rhs<double>(p, st->cur, out_device) : chib::enqueue_rhs<float>(p, st->cur, out_device);
      break;
    case CH_IB_STAGE_SOLVE:
      if (!in_device) return fail(CH_IB_EINVAL, "SOLVE needs an input");
      e = st->es == 8 ? chib::enqueue_solve<double>(p, in_device, out_device)
                      : chib::enqueue_solve<float>(p, in_device, out_device);
      break;
    case CH_IB_STAGE_PHI:
      e = st->es == 8 ? chib::enqueue_phi<double>(p, st->cur, out_device) : chib::enqueue_phi<float>(p, st->cur, out_device);
      break;
    default: return fail(CH_IB_EINVAL, "unknown stage");
  }
  if (e == hipSuccess) e = hipStreamSynchronize(p.stream);
  if (e != hipSuccess) return hip_fail(st, e, "stage");
  return CH_IB_OK;
}

extern "C" int ch_ib_scalar_fill(ch_ib_state *st, void *field_device, double a, double b, double g,
                                 const void *g_ghost_device) {
  if (!st || !field_device) return fail(CH_IB_EINVAL, "NULL state or field");
  if (!std::isfinite(a) || !std::isfinite(b) || !std::isfinite(g)) return fail(CH_IB_EINVAL, "non-finite a, b or g");
  const chib::Plan &p = st->plan;
  // the condition fixes f_G only where a gamma - b/dn = (a d1 - b)/dn does not vanish, with
  // d1 = gamma dn the intersect-to-mirror distance (one value per geometry up to rounding)
  if (a == 0.0 && b == 0.0) return fail(CH_IB_EINVAL, "a and b are both zero: the condition fixes nothing");
  if (p.G && a != 0.0) {
    const double r = b / a;
    if (r >= st->d1_min * (1.0 - 1e-9) && r <= st->d1_max * (1.0 + 1e-9))
      return fail(CH_IB_EINVAL, "a d1 = b: the condition does not fix the ghost values");
  }
  hipError_t e = st->es == 8 ? chib::enqueue_scalar_fill<double>(p, field_device, a, b, g, g_ghost_device)
                             : chib::enqueue_scalar_fill<float>(p, field_device, a, b, g, g_ghost_device);
  if (e != hipSuccess) return hip_fail(st, e, "scalar_fill");
  return CH_IB_OK;
}

namespace {
struct BlobHeader {
  uint32_t magic, version;
  int32_t es, d, n[3], needs_init;
  int64_t G, NF, step;
};
}  // namespace

static unsigned blob_version(const chib::Plan &p) { return (p.explicit_ab2 ? 2u : 1u) + (p.ns ? 2u : 0u); }

// Device fields of the momentum step kept in a blob, in order.
static std::vector<const void *> ns_fields(const chib::Plan &p) {
  std::vector<const void *> f;
  if (!p.ns) return f;
  f.push_back(p.P[0]);
  f.push_back(p.P[1]);
  for (int a = 0; a < p.d; ++a) f.push_back(p.Nh[a]);
  for (int a = 0; a < p.d && p.Ut[0]; ++a) f.push_back(p.Ut[a]);
  return f;
}

static size_t ns_extra(const chib::Plan &p, int es) {
  return p.ns ? 2 * sizeof(int64_t) + ns_fields(p).size() * (size_t)p.N * es : 0;
}

extern "C" int ch_ib_state_save(ch_ib_state *st, void *buf, size_t *len) {
  if (!st || !len) return fail(CH_IB_EINVAL, "NULL argument");
  const chib::Plan &p = st->plan;
  const size_t fb = (size_t)p.N * st->es, gb = (size_t)p.G * st->es;
  // version 2 (explicit scheme) appends the history flag and the previous step's rate; versions 3
  // and 4 (momentum step, semi-implicit / explicit) then append two flags, p^n, p^(n-1), the
  // previous convective term and, semi-implicit, the advecting velocity
  const size_t extra = (p.explicit_ab2 ? sizeof(int64_t) + fb : 0) + ns_extra(p, st->es);
  const size_t need = sizeof(BlobHeader) + (2 + p.d) * fb + 3 * gb + extra;
  if (!buf) {
    *len = need;
    return CH_IB_OK;
  }
  if (*len < need) return fail(CH_IB_ENOMEM, "buffer too small");
  BlobHeader hd{kMagic, blob_version(p), st->es, p.d, {p.n[0], p.n[1], p.n[2]}, st->needs_init,
                p.G, p.NF, st->step};
  char *b = (char *)buf;
  std::memcpy(b, &hd, sizeof(hd));
  b += sizeof(hd);
  const void *srcs[8];
  size_t sz[8];
  int ns = 0;
  srcs[ns] = p.C[st->cur], sz[ns++] = fb;
  srcs[ns] = p.C[1 - st->cur], sz[ns++] = fb;
  for (int a = 0; a < p.d; ++a) srcs[ns] = p.F[a], sz[ns++] = fb;
  srcs[ns] = p.CGn, sz[ns++] = gb;
  srcs[ns] = p.CGnm1, sz[ns++] = gb;
  srcs[ns] = p.CI, sz[ns++] = gb;
  hipError_t e = hipSuccess;
  for (int i = 0; i < ns && e == hipSuccess; ++i) {
    if (sz[i]) e = hipMemcpyAsync(b, srcs[i], sz[i], hipMemcpyDeviceToHost, p.stream);
    b += sz[i];
  }
  if (p.explicit_ab2 && e == hipSuccess) {
    const int64_t rv = st->r_valid;
    std::memcpy(b, &rv, sizeof(rv));
    b += sizeof(rv);
    e = hipMemcpyAsync(b, p.R, fb, hipMemcpyDeviceToHost, p.stream);
    b += fb;
  }
  if (p.ns && e == hipSuccess) {
    const int64_t fl[2] = {st->ns_first, st->ut_valid};
    std::memcpy(b, fl, sizeof(fl));
    b += sizeof(fl);
    for (const void *src : ns_fields(p)) {
      if (e == hipSuccess) e = hipMemcpyAsync(b, src, fb, hipMemcpyDeviceToHost, p.stream);
      b += fb;
    }
  }
  if (e == hipSuccess) e = hipStreamSynchronize(p.stream);
  if (e != hipSuccess) return hip_fail(st, e, "save");
  *len = need;
  return CH_IB_OK;
}

extern "C" int ch_ib_state_load(ch_ib_state *st, const void *buf, size_t len) {
  if (!st || !buf) return fail(CH_IB_EINVAL, "NULL argument");
  chib::Plan &p = st->plan;
  BlobHeader hd;
  if (len < sizeof(hd)) return fail(CH_IB_EINVAL, "blob too short");
  std::memcpy(&hd, buf, sizeof(hd));
  if (hd.magic != kMagic || hd.version < 1 || hd.version > 4) return fail(CH_IB_EINVAL, "not a state blob");
  if (hd.version != blob_version(p)) return fail(CH_IB_EINVAL, "blob saved with another time scheme");
  if (hd.es != st->es || hd.d != p.d || hd.n[0] != p.n[0] || hd.n[1] != p.n[1] || hd.n[2] != p.n[2] ||
      hd.G != p.G || hd.NF != p.NF)
    return fail(CH_IB_EINVAL, "blob saved from a different grid, geometry or precision");
  const size_t fb = (size_t)p.N * st->es, gb = (size_t)p.G * st->es;
  const size_t extra = (p.explicit_ab2 ? sizeof(int64_t) + fb : 0) + ns_extra(p, st->es);
  const size_t need = sizeof(BlobHeader) + (2 + p.d) * fb + 3 * gb + extra;
  if (len < need) return fail(CH_IB_EINVAL, "blob too short");
  const char *b = (const char *)buf + sizeof(hd);
  st->cur = 0;
  void *dsts[8];
  size_t sz[8];
  int ns = 0;
  dsts[ns] = p.C[0], sz[ns++] = fb;
  dsts[ns] = p.C[1], sz[ns++] = fb;
  for (int a = 0; a < p.d; ++a) dsts[ns] = p.F[a], sz[ns++] = fb;
  dsts[ns] = p.CGn, sz[ns++] = gb;
  dsts[ns] = p.CGnm1, sz[ns++] = gb;
  dsts[ns] = p.CI, sz[ns++] = gb;
  hipError_t e = hipSuccess;
  for (int i = 0; i < ns && e == hipSuccess; ++i) {
    if (sz[i]) e = hipMemcpyAsync(dsts[i], b, sz[i], hipMemcpyHostToDevice, p.stream);
    b += sz[i];
  }
  int64_t rv = 0;
  if (p.explicit_ab2 && e == hipSuccess) {
    std::memcpy(&rv, b, sizeof(rv));
    b += sizeof(rv);
    e = hipMemcpyAsync(p.R, b, fb, hipMemcpyHostToDevice, p.stream);
    b += fb;
  }
  int64_t fl[2] = {1, 0};
  if (p.ns && e == hipSuccess) {
    std::memcpy(fl, b, sizeof(fl));
    b += sizeof(fl);
    for (const void *dst : ns_fields(p)) {
      if (e == hipSuccess) e = hipMemcpyAsync((void *)dst, b, fb, hipMemcpyHostToDevice, p.stream);
      b += fb;
    }
  }
  if (e == hipSuccess) e = hipStreamSynchronize(p.stream);
  if (e != hipSuccess) return hip_fail(st, e, "load");
  st->r_valid = rv ? 1 : 0;
  st->ns_first = fl[0] ? 1 : 0;
  st->ut_valid = fl[1] ? 1 : 0;
  st->step = hd.step;
  st->needs_init = hd.needs_init;
  st->sticky = CH_IB_OK;
  return CH_IB_OK;
}

extern "C" void ch_ib_state_free(ch_ib_state *st) { delete st; }


// ---------------------------------------------------------------------------------------------
// Batched sweep.

struct ch_ib_batch {
  std::vector<ch_ib_state *> st;
  std::vector<ch_ib_state *> grp;   // members advanced by the grouped launches
  std::vector<ch_ib_state *> seq;   // members with the momentum step: their own launches, in turn
  int es = 8;
  char *ws = nullptr;
  size_t ws_bytes = 0;
  hipStream_t stream = nullptr;
  chib::BatchLaunch bl;
  int parity = 0;               // launch parity relative to the uploaded descriptors
  hipGraphExec_t graph[2] = {nullptr, nullptr};  // two steps starting at parity 0 / 1
  hipGraph_t graph_def[2] = {nullptr, nullptr};
};

static size_t batch_desc_bytes(int es) {
  return es == 8 ? chib::case_desc_bytes<double>() : chib::case_desc_bytes<float>();
}

extern "C" size_t ch_ib_batch_workspace_bytes(int n) {
  if (n < 1) return 0;
  const size_t d = std::max(batch_desc_bytes(8), batch_desc_bytes(4));
  return ((d * n + 255) & ~(size_t)255) +
         ((chib::BatchLaunch::kPhases * (size_t)(n + 1) * sizeof(int) + 255) & ~(size_t)255) + 256;
}

static void batch_drop_graphs(ch_ib_batch *b) {
  for (int k = 0; k < 2; ++k) {
    if (b->graph[k]) (void)hipGraphExecDestroy(b->graph[k]);
    if (b->graph_def[k]) (void)hipGraphDestroy(b->graph_def[k]);
    b->graph[k] = nullptr;
    b->graph_def[k] = nullptr;
  }
}

// Uploads descriptors (from each member's current buffer roles) and tile offsets.
static int batch_upload(ch_ib_batch *b) {
  const int n = (int)b->grp.size();
  const size_t db = batch_desc_bytes(b->es);
  std::vector<unsigned char> descs(db * n);
  constexpr int NPH = chib::BatchLaunch::kPhases;
  std::vector<int> off(NPH * (size_t)(n + 1), 0);
  size_t lds[4] = {0, 0, 0, 0};
  bool ym_all = true;
  for (int c = 0; c < n; ++c) {
    ch_ib_state *s = b->grp[c];
    int tiles[NPH];
    size_t l[4];
    if (b->es == 8) {
      chib::fill_case_desc<double>(s->plan, s->cur, descs.data() + db * c);
      chib::case_tiles<double>(s->plan, tiles, l);
    } else {
      chib::fill_case_desc<float>(s->plan, s->cur, descs.data() + db * c);
      chib::case_tiles<float>(s->plan, tiles, l);
    }
    for (int ph = 0; ph < NPH; ++ph) off[ph * (n + 1) + c + 1] = off[ph * (n + 1) + c] + tiles[ph];
    for (int k = 0; k < 4; ++k) lds[k] = std::max(lds[k], l[k]);
    ym_all = ym_all && l[3] > 0;
  }
  if (!ym_all) lds[3] = 0;
  const size_t doff = (db * n + 255) & ~(size_t)255;
  hipError_t e = hipSuccess;
  if (n > 0) {
    e = hipMemcpyAsync(b->ws, descs.data(), descs.size(), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(b->ws + doff, off.data(), off.size() * sizeof(int), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  }
  if (e != hipSuccess) return hip_fail(nullptr, e, "batch upload");
  b->bl.descs = b->ws;
  b->bl.off = (const int *)(b->ws + doff);
  b->bl.n = n;
  for (int ph = 0; ph < NPH; ++ph) b->bl.total[ph] = (unsigned)off[ph * (n + 1) + n];
  for (int k = 0; k < 4; ++k) b->bl.lds[k] = lds[k];
  b->bl.stream = b->stream;
  b->parity = 0;
  batch_drop_graphs(b);
  return CH_IB_OK;
}

static hipError_t batch_direct_step(ch_ib_batch *b, int parity) {
  if (b->bl.n == 0) return hipSuccess;   // no member for the grouped launches
  return b->es == 8 ? chib::enqueue_batch_step<double>(b->bl, parity) : chib::enqueue_batch_step<float>(b->bl, parity);
}

extern "C" int ch_ib_batch_create(ch_ib_state *const *states, int n, void *ws, size_t bytes, void *stream,
                                  ch_ib_batch **out) {
  if (!out) return fail(CH_IB_EINVAL, "out is NULL");
  *out = nullptr;
  if (!states || n < 1 || !ws) return fail(CH_IB_EINVAL, "bad state list or workspace");
  if (bytes < ch_ib_batch_workspace_bytes(n)) return fail(CH_IB_ENOMEM, "batch workspace too small");
  if (((uintptr_t)ws) & 255) return fail(CH_IB_EINVAL, "workspace must be 256-byte aligned");
  const int es = states[0] ? states[0]->es : 0;
  for (int c = 0; c < n; ++c) {
    ch_ib_state *s = states[c];
    if (!s) return fail(CH_IB_EINVAL, "NULL state");
    if (s->es != es) return fail(CH_IB_EINVAL, "mixed precisions in one batch");
    if (s->plan.d != 2) return fail(CH_IB_EUNSUPPORTED, "batches hold 2D states only");
    if (s->plan.dynamic) return fail(CH_IB_EUNSUPPORTED, "batches hold static contact-angle states only");
    if (s->plan.explicit_ab2) return fail(CH_IB_EUNSUPPORTED, "batches hold semi-implicit states only");
    if (s->sticky) return fail(s->sticky, "a member state is in an error state");
  }
  for (int c = 0; c < n; ++c) {
    int rc = ensure_init(states[c]);
    if (rc) return rc;
    hipError_t e = hipStreamSynchronize(states[c]->plan.stream);
    if (e != hipSuccess) return hip_fail(states[c], e, "batch create");
  }
  auto *b = new ch_ib_batch();
  b->st.assign(states, states + n);
  for (ch_ib_state *s : b->st) (s->plan.ns ? b->seq : b->grp).push_back(s);
  b->es = es;
  b->ws = (char *)ws;
  b->ws_bytes = bytes;
  b->stream = (hipStream_t)stream;
  // shared kernel choices follow the first grouped member's shapes (so that a batched step is the
  // same computation as stepping each member with those shapes)
  const ch_ib_state *s0 = b->grp.empty() ? states[0] : b->grp[0];
  b->bl.radix_rhs = s0->plan.shape[0].radix;
  {
    const int u = s0->plan.shape[0].unroll;   // 3: y-march where every case allows it
    b->bl.unroll = u == 3 ? 3 : std::min(u, 2);
  }
  b->bl.radix_neu = s0->plan.shape[2].radix;
  b->bl.radix_out = s0->plan.shape[3].radix;
  int rc = batch_upload(b);
  if (rc) {
    delete b;
    return rc;
  }
  *out = b;
  return CH_IB_OK;
}

extern "C" int ch_ib_batch_step(ch_ib_batch *b, int n_steps) {
  if (!b) return fail(CH_IB_EINVAL, "NULL batch");
  if (n_steps < 0) return fail(CH_IB_EINVAL, "n_steps must be >= 0");
  hipError_t e = hipSuccess;
  int left = b->grp.empty() ? 0 : n_steps;
  if (!b->stream) {  // the legacy NULL stream cannot be captured: direct grouped launches
    for (; left > 0 && e == hipSuccess; --left) {
      e = batch_direct_step(b, b->parity);
      b->parity ^= 1;
    }
  }
  while (left >= 2 && e == hipSuccess) {
    const int p = b->parity;
    if (!b->graph[p]) {
      e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) e = batch_direct_step(b, p);
      if (e == hipSuccess) e = batch_direct_step(b, 1 - p);
      hipGraph_t g = nullptr;
      hipError_t e2 = hipStreamEndCapture(b->stream, &g);
      if (e == hipSuccess) e = e2;
      if (e == hipSuccess) {
        b->graph_def[p] = g;
        e = hipGraphInstantiate(&b->graph[p], g, nullptr, nullptr, 0);
      } else if (g) {
        (void)hipGraphDestroy(g);
      }
      if (e != hipSuccess) break;
    }
    e = hipGraphLaunch(b->graph[p], b->stream);
    left -= 2;
  }
  if (left == 1 && e == hipSuccess) {
    e = batch_direct_step(b, b->parity);
    if (e == hipSuccess) b->parity ^= 1;
  }
  if (e != hipSuccess) return hip_fail(nullptr, e, "batch step");
  for (ch_ib_state *s : b->grp) {
    s->step += n_steps;
    if (n_steps & 1) s->cur = 1 - s->cur;
  }
  // members with the momentum step: the same launches as ch_ib_step, on the batch's stream
  for (ch_ib_state *s : b->seq) {
    const hipStream_t own = s->plan.stream;
    s->plan.stream = b->stream;
    for (int i = 0; i < n_steps && e == hipSuccess; ++i) {
      e = enqueue_one_step(s, nullptr);
      if (e == hipSuccess) {
        s->cur = 1 - s->cur;
        s->step++;
      }
    }
    s->plan.stream = own;
    if (e != hipSuccess) return hip_fail(s, e, "batch step");
  }
  return CH_IB_OK;
}

extern "C" int ch_ib_batch_sync(ch_ib_batch *b) {
  if (!b) return fail(CH_IB_EINVAL, "NULL batch");
  hipError_t e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return hip_fail(nullptr, e, "batch sync");
  return CH_IB_OK;
}

extern "C" int ch_ib_batch_tune(ch_ib_batch *b, int reps, int *radix_out, int *unroll_out) {
  if (!b) return fail(CH_IB_EINVAL, "NULL batch");
  if (reps < 1 || reps > 100) return fail(CH_IB_EINVAL, "reps must be in 1..100");
  hipError_t e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return hip_fail(nullptr, e, "batch tune");
  // 1. per distinct grid size, tune one member and copy its shapes to the others
  std::vector<std::pair<int, int>> sizes;
  for (ch_ib_state *s : b->st) {
    std::pair<int, int> key{s->plan.n[0], s->plan.n[1]};
    if (std::find(sizes.begin(), sizes.end(), key) != sizes.end()) continue;
    sizes.push_back(key);
    int rc = ch_ib_tune(s, reps, nullptr);
    if (rc) return rc;
    for (ch_ib_state *o : b->st)
      if (o->plan.n[0] == key.first && o->plan.n[1] == key.second)
        for (int k = 0; k < 4; ++k) o->plan.shape[k] = s->plan.shape[k];
  }
  // 2. the shared radix / cells in flight: time full batched steps of the grouped members (an even
  // number, so that every member's buffer roles end where they started; the fields advance, so
  // restore them after).  Members with the momentum step keep the shapes of step 1.
  if (b->grp.empty()) {
    if (radix_out) {
      radix_out[0] = b->bl.radix_rhs;
      radix_out[1] = b->bl.radix_neu;
      radix_out[2] = b->bl.radix_out;
    }
    if (unroll_out) *unroll_out = b->bl.unroll;
    return CH_IB_OK;
  }
  sizes.clear();
  for (ch_ib_state *s : b->grp) {
    std::pair<int, int> key{s->plan.n[0], s->plan.n[1]};
    if (std::find(sizes.begin(), sizes.end(), key) == sizes.end()) sizes.push_back(key);
  }
  std::vector<std::vector<unsigned char>> saved(b->grp.size());
  for (size_t c = 0; c < b->grp.size(); ++c) {
    size_t len = 0;
    int rc = ch_ib_state_save(b->grp[c], nullptr, &len);
    if (rc) return rc;
    saved[c].resize(len);
    rc = ch_ib_state_save(b->grp[c], saved[c].data(), &len);
    if (rc) return rc;
  }
  int rc = batch_upload(b);
  if (rc) return rc;
  hipEvent_t e0, e1;
  e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  auto time_pair = [&]() -> float {
    e = batch_direct_step(b, 0);
    if (e == hipSuccess) e = batch_direct_step(b, 1);
    float tmin = 1e30f;
    for (int r = 0; r < reps && e == hipSuccess; ++r) {
      e = hipEventRecord(e0, b->stream);
      if (e == hipSuccess) e = batch_direct_step(b, 0);
      if (e == hipSuccess) e = batch_direct_step(b, 1);
      if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      tmin = std::min(tmin, ms);
    }
    return tmin;
  };
  // greedy over the shared choices: rhs radix x cells in flight, then the solve radix, then the out radix
  {
    float best = 1e30f;
    int br = b->bl.radix_rhs, bu = b->bl.unroll;
    for (int radix : {8, 16})
      for (int un : {1, 2, 3}) {
        if (e != hipSuccess) break;
        if (un == 3 && !b->bl.lds[3]) continue;
        b->bl.radix_rhs = radix;
        b->bl.unroll = un;
        const float t = time_pair();
        if (t < best) {
          best = t;
          br = radix;
          bu = un;
        }
      }
    b->bl.radix_rhs = br;
    b->bl.unroll = bu;
  }
  // tile heights per distinct grid size (rhs lines, solve columns, out lines), timed on the whole
  // batch: a case that runs alone wants small tiles to fill the GPU, a batch has parallelism to spare
  for (int pass : {0, 2, 3}) {
    for (const auto &key : sizes) {
      if (e != hipSuccess) break;
      std::vector<ch_ib_state *> grp;
      for (ch_ib_state *s : b->grp)
        if (s->plan.n[0] == key.first && s->plan.n[1] == key.second) grp.push_back(s);
      const int hi = b->es == 8 ? chib::max_log_tile<double>(grp[0]->plan, pass)
                                : chib::max_log_tile<float>(grp[0]->plan, pass);
      int best_lt = grp[0]->plan.shape[pass].log_tile;
      float best = 1e30f;
      for (int lt = 1; lt <= hi && e == hipSuccess; ++lt) {
        for (ch_ib_state *s : grp) s->plan.shape[pass].log_tile = lt;
        rc = batch_upload(b);
        if (rc) return rc;
        const float t = time_pair();
        if (t < best) {
          best = t;
          best_lt = lt;
        }
      }
      for (ch_ib_state *s : grp) s->plan.shape[pass].log_tile = best_lt;
      rc = batch_upload(b);
      if (rc) return rc;
    }
  }
  for (int which = 0; which < 2 && e == hipSuccess; ++which) {
    int &slot = which == 0 ? b->bl.radix_neu : b->bl.radix_out;
    float best = 1e30f;
    int bv = slot;
    for (int radix : {8, 16}) {
      if (e != hipSuccess) break;
      slot = radix;
      const float t = time_pair();
      if (t < best) {
        best = t;
        bv = radix;
      }
    }
    slot = bv;
  }
  const int br = b->bl.radix_rhs, bu = b->bl.unroll, bn = b->bl.radix_neu, bo = b->bl.radix_out;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return hip_fail(nullptr, e, "batch tune");
  for (size_t c = 0; c < b->grp.size(); ++c) {
    rc = ch_ib_state_load(b->grp[c], saved[c].data(), saved[c].size());
    if (rc) return rc;
  }
  rc = batch_upload(b);
  if (rc) return rc;
  b->bl.radix_rhs = br;
  b->bl.unroll = bu;
  b->bl.radix_neu = bn;
  b->bl.radix_out = bo;
  if (radix_out) {
    radix_out[0] = br;
    radix_out[1] = bn;
    radix_out[2] = bo;
  }
  if (unroll_out) *unroll_out = bu;
  return CH_IB_OK;
}

extern "C" void ch_ib_batch_free(ch_ib_batch *b) {
  if (!b) return;
  batch_drop_graphs(b);
  delete b;
}
