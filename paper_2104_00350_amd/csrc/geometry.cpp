// Host geometry preprocessing (section 4.1 of the paper): volume fraction by subgrid
// counting, wall normals from corner gradients of the volume fraction, ghost / intersect /
// mirror / interpolation points along the normal, plus-stencil averaging points with
// normalised inverse-squared-distance weights.  Runs once per geometry; the per-step work
// only reads the resulting compact per-ghost tables.
//
// Readings of passages the paper leaves open (kept identical in every implementation of
// the method in this project):
//  - unit normal n = m / sqrt(m.m + 1e-30), m the mean of the 2^d corner gradients, each
//    corner gradient the mean one-cell difference of alpha across the corner divided by h;
//  - subgrid points at sub-cell centres, 100 per direction by default (the paper's count);
//  - ghost: solid cell centre with a face neighbour whose centre is fluid; a ghost in the
//    first or last cell layer of the bounded axis is rejected;
//  - intersect point: march from the ghost along n in steps of h/100 to the first fluid
//    point, then 60 bisections keeping the fluid end;
//  - mirror point d1 beyond the intersect point (default 2h: near one cell diagonal the
//    averaging stencil of the first interpolation point reaches the ghost's own fluid
//    neighbours and near-wall modes grow for strongly wetting angles), interpolation
//    points d2 and 2*d2 beyond the mirror point (default d2 = 1.5h);
//  - averaging points: the cell containing the interpolation point and its 2d face
//    neighbours; solid ones are dropped and the weights renormalised; with none left, the
//    nearest fluid centre within 2h takes the whole weight.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>

#include "internal.h"

namespace {

constexpr double kTwoPi = 6.283185307179586;

struct Shapes {
  std::vector<ch_ib_shape> s;
  int d = 2;
  int n[3] = {1, 1, 1};
  double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};

  bool solid_one(const ch_ib_shape &sh, const double *x) const {
    const double *p = sh.p;
    switch (sh.kind) {
      case CH_IB_HALFPLANE: {
        double v = (x[0] - p[0]) * p[3] + (x[1] - p[1]) * p[4];
        if (d == 3) v = v + (x[2] - p[2]) * p[5];
        return v < 0.0;
      }
      case CH_IB_SINUSOID: {
        double yw = p[0] + p[1] * std::sin(kTwoPi * x[0] / p[2] + p[3]);
        return x[d - 1] < yw;
      }
      case CH_IB_SPHERE: {
        double dx = x[0] - p[0], dy = x[1] - p[1];
        double r2 = dx * dx + dy * dy;
        if (d == 3) {
          double dz = x[2] - p[2];
          r2 = r2 + dz * dz;
        }
        return r2 < p[3] * p[3];
      }
      case CH_IB_BOX: {
        double c = std::cos(p[4]), s_ = std::sin(p[4]);
        double dx = x[0] - p[0], dy = x[1] - p[1];
        double q0 = c * dx + s_ * dy;
        double q1 = -s_ * dx + c * dy;
        bool out = std::fabs(q0) > p[3] || std::fabs(q1) > p[3];
        if (d == 3) out = out || std::fabs(x[2] - p[2]) > p[3];
        return out;
      }
      default:
        return false;
    }
  }

  // Union of the solid regions at a point, periodic axes shifted by one period when outside.
  bool solid(const double *xin) const {
    double x[3] = {xin[0], xin[1], d == 3 ? xin[2] : 0.0};
    for (int a = 0; a < d - 1; ++a) {
      double L = hi[a] - lo[a];
      if (x[a] >= hi[a]) x[a] = x[a] - L;
      else if (x[a] < lo[a]) x[a] = x[a] + L;
    }
    for (const auto &sh : s)
      if (solid_one(sh, x)) return true;
    return false;
  }

  // Conservative: false only if every point of the cell is on the centre's side of this shape.
  bool may_cut(const ch_ib_shape &sh, const double *xc, double h) const {
    const double hd = 0.5 * h * std::sqrt((double)d);
    const double m = 1e-9 * h;
    const double *p = sh.p;
    switch (sh.kind) {
      case CH_IB_HALFPLANE: {
        double nn = 0.0, v = 0.0;
        for (int a = 0; a < d; ++a) {
          nn += p[3 + a] * p[3 + a];
          v += (xc[a] - p[a]) * p[3 + a];
        }
        return std::fabs(v / std::sqrt(nn)) <= hd + m;
      }
      case CH_IB_SPHERE: {
        double r2 = 0.0;
        for (int a = 0; a < d; ++a) r2 += (xc[a] - p[a]) * (xc[a] - p[a]);
        return std::fabs(std::sqrt(r2) - p[3]) <= hd + m;
      }
      case CH_IB_SINUSOID: {
        double lip = kTwoPi * std::fabs(p[1]) / p[2];
        double yw = p[0] + p[1] * std::sin(kTwoPi * xc[0] / p[2] + p[3]);
        return std::fabs(xc[d - 1] - yw) <= 0.5 * h + 0.5 * lip * h + m;
      }
      case CH_IB_BOX: {
        double c = std::cos(p[4]), s_ = std::sin(p[4]);
        double dx = xc[0] - p[0], dy = xc[1] - p[1];
        double q[3] = {std::fabs(c * dx + s_ * dy) - p[3], std::fabs(-s_ * dx + c * dy) - p[3],
                       d == 3 ? std::fabs(xc[2] - p[2]) - p[3] : -1e300};
        double out2 = 0.0, qmax = -1e300;
        for (int a = 0; a < d; ++a) {
          double qq = std::max(q[a], 0.0);
          out2 += qq * qq;
          qmax = std::max(qmax, q[a]);
        }
        double sd = std::sqrt(out2) + std::min(qmax, 0.0);
        return std::fabs(sd) <= hd + m;
      }
      default:
        return true;
    }
  }
};

template <typename F>
void parallel_for(int64_t n, F f) {
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (n < 4096 || nt == 1) {
    for (int64_t i = 0; i < n; ++i) f(i);
    return;
  }
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nt; ++t)
    th.emplace_back([&, t]() {
      for (int64_t i = t; i < n; i += nt) f(i);
    });
  for (auto &x : th) x.join();
}

}  // namespace

namespace chib {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }
const char *last_error() { return g_last_error.c_str(); }
int fail(int code, const std::string &msg) {
  set_error(msg);
  return code;
}

int check_grid(const ch_ib_grid *grid, ch_ib_geometry *g) {
  if (!grid) return fail(CH_IB_EINVAL, "grid is NULL");
  if (grid->ndim != 2 && grid->ndim != 3) return fail(CH_IB_EINVAL, "ndim must be 2 or 3");
  g->grid = *grid;
  g->ndim = grid->ndim;
  g->cells = 1;
  for (int a = 0; a < 3; ++a) {
    g->n[a] = a < grid->ndim ? grid->n[a] : 1;
    g->lo[a] = a < grid->ndim ? grid->lo[a] : 0.0;
  }
  for (int a = 0; a < grid->ndim; ++a) {
    int n = grid->n[a];
    if (n < 8 || n > 2048) return fail(CH_IB_EUNSUPPORTED, "each axis needs 8..2048 cells");
    if (n & (n - 1)) return fail(CH_IB_EUNSUPPORTED, "cells per axis must be a power of two");
    if (!(grid->hi[a] > grid->lo[a])) return fail(CH_IB_EINVAL, "empty box");
    g->cells *= n;
  }
  g->h = (grid->hi[0] - grid->lo[0]) / grid->n[0];
  for (int a = 1; a < grid->ndim; ++a) {
    double ha = (grid->hi[a] - grid->lo[a]) / grid->n[a];
    if (std::fabs(ha - g->h) > 1e-12 * g->h) return fail(CH_IB_EINVAL, "grid spacing must be uniform");
  }
  if (g->cells >= (int64_t(1) << 31)) return fail(CH_IB_EUNSUPPORTED, "grids above 2^31 cells");
  return CH_IB_OK;
}

}  // namespace chib

extern "C" const char *ch_ib_last_error(void) { return chib::last_error(); }

extern "C" int ch_ib_geometry_build(const ch_ib_grid *grid, const ch_ib_shape *shapes, int n_shapes,
                                    const ch_ib_params *params, ch_ib_geometry **out) {
  using chib::fail;
  if (!out || !params) return fail(CH_IB_EINVAL, "NULL argument");
  *out = nullptr;
  if (n_shapes < 0 || (n_shapes > 0 && !shapes)) return fail(CH_IB_EINVAL, "bad shape list");
  auto *g = new ch_ib_geometry();
  int rc = chib::check_grid(grid, g);
  if (rc) {
    delete g;
    return rc;
  }
  const int d = g->ndim;
  const double h = g->h;
  Shapes S;
  S.d = d;
  for (int a = 0; a < d; ++a) {
    S.n[a] = g->n[a];
    S.lo[a] = grid->lo[a];
    S.hi[a] = grid->hi[a];
  }
  for (int i = 0; i < n_shapes; ++i) {
    if (shapes[i].kind < CH_IB_HALFPLANE || shapes[i].kind > CH_IB_BOX) {
      delete g;
      return fail(CH_IB_EINVAL, "unknown shape kind");
    }
    if (shapes[i].kind == CH_IB_SINUSOID && !(shapes[i].p[2] > 0)) {
      delete g;
      return fail(CH_IB_EINVAL, "sinusoid wavelength must be positive");
    }
    S.s.push_back(shapes[i]);
  }
  const int sub = params->subgrid > 0 ? params->subgrid : 100;
  const int64_t N = g->cells;
  const int nx = g->n[0], ny = g->n[1], nz = g->n[2];

  auto coords = [&](int64_t lin, int *ijk) {
    ijk[0] = (int)(lin % nx);
    ijk[1] = (int)((lin / nx) % ny);
    ijk[2] = (int)(lin / ((int64_t)nx * ny));
  };
  auto centre = [&](const int *ijk, double *x) {
    for (int a = 0; a < d; ++a) x[a] = g->lo[a] + ((double)ijk[a] + 0.5) * h;
  };

  // P1-P2: centre solid mask and volume fraction; with fa >= 0 the control volumes are the
  // staggered cells of the faces normal to axis fa (shifted by h/2 along fa), the three further
  // fractions of the staggered grid
  std::vector<uint8_t> csolid(N);
  const double hs = h / sub;
  const int64_t per_cell = (int64_t)sub * sub * (d == 3 ? sub : 1);
  auto fractions = [&](int fa, std::vector<double> &out, uint8_t *mask) {
    out.assign(N, 0.0);
    double off[3] = {0.0, 0.0, 0.0};
    if (fa >= 0) off[fa] = 0.5 * h;
    parallel_for(N, [&](int64_t c) {
      int ijk[3];
      coords(c, ijk);
      double xc[3] = {0, 0, 0};
      centre(ijk, xc);
      for (int a = 0; a < d; ++a) xc[a] = xc[a] + off[a];
      bool cs = S.solid(xc);
      if (mask) mask[c] = cs;
      bool cut = false;
      for (const auto &sh : S.s) cut = cut || S.may_cut(sh, xc, h);
      if (!cut) {
        out[c] = cs ? 0.0 : 1.0;
        return;
      }
      double base[3];
      for (int a = 0; a < d; ++a) base[a] = g->lo[a] + (double)ijk[a] * h + off[a];
      int64_t fluid = 0;
      double x[3];
      const int s2 = d == 3 ? sub : 1;
      for (int k = 0; k < s2; ++k) {
        if (d == 3) x[2] = base[2] + ((double)k + 0.5) * hs;
        for (int j = 0; j < sub; ++j) {
          x[1] = base[1] + ((double)j + 0.5) * hs;
          for (int i = 0; i < sub; ++i) {
            x[0] = base[0] + ((double)i + 0.5) * hs;
            if (!S.solid(x)) ++fluid;
          }
        }
      }
      out[c] = (double)fluid / (double)per_cell;
    });
  };
  fractions(-1, g->alpha, csolid.data());
  if (params->flags & CH_IB_FLAG_NAVIER_STOKES) {
    std::vector<double> fr;
    g->face_alpha.resize((size_t)d * N);
    for (int a = 0; a < d; ++a) {
      fractions(a, fr, nullptr);
      std::copy(fr.begin(), fr.end(), g->face_alpha.begin() + (size_t)a * N);
    }
  }

  // ghosts
  auto lin_of = [&](const int *ijk) -> int64_t {
    return ijk[0] + (int64_t)nx * (ijk[1] + (int64_t)ny * ijk[2]);
  };
  for (int64_t c = 0; c < N; ++c) {
    if (!csolid[c]) continue;
    int ijk[3];
    coords(c, ijk);
    bool nb_fluid = false;
    for (int a = 0; a < d && !nb_fluid; ++a) {
      for (int sgn = -1; sgn <= 1; sgn += 2) {
        int q[3] = {ijk[0], ijk[1], ijk[2]};
        q[a] += sgn;
        if (a < d - 1) q[a] = (q[a] + g->n[a]) % g->n[a];
        else if (q[a] < 0 || q[a] >= g->n[a]) continue;
        if (!csolid[lin_of(q)]) {
          nb_fluid = true;
          break;
        }
      }
    }
    if (!nb_fluid) continue;
    if (ijk[d - 1] == 0 || ijk[d - 1] == g->n[d - 1] - 1) {
      delete g;
      return fail(CH_IB_EGEOM, "a ghost point touches the box wall of the bounded axis");
    }
    g->gidx.push_back(c);
  }
  const int64_t G = (int64_t)g->gidx.size();
  const int K = 2 * d + 1;
  g->n_ghost = G;
  g->n_ap = K;
  g->normal.assign((size_t)d * G, 0.0);
  g->dn.assign(G, 0.0);
  g->gamma.assign(G, 0.0);
  g->ap.assign((size_t)2 * K * G, 0);
  g->w.assign((size_t)2 * K * G, 0.0);

  const double d1 = (params->d1_cells > 0 ? params->d1_cells : 2.0) * h;
  const double d2 = (params->d2_cells > 0 ? params->d2_cells : 1.5) * h;
  std::vector<int> err(G, 0);

  parallel_for(G, [&](int64_t gi) {
    const int64_t c = g->gidx[gi];
    int ijk[3];
    coords(c, ijk);
    // P3: normal from corner gradients of alpha
    auto alpha_at = [&](int i, int j, int k) {
      int q[3] = {i, j, k};
      for (int a = 0; a < d - 1; ++a) q[a] = (q[a] + g->n[a]) % g->n[a];
      if (d == 2) q[2] = 0;
      return g->alpha[lin_of(q)];
    };
    double m[3] = {0, 0, 0};
    const int nc = 1 << d;
    for (int corner = 0; corner < nc; ++corner) {
      int s[3] = {corner & 1, (corner >> 1) & 1, (corner >> 2) & 1};
      double mc[3] = {0, 0, 0};
      for (int t = 0; t < nc; ++t) {
        int tt[3] = {t & 1, (t >> 1) & 1, (t >> 2) & 1};
        int q[3] = {ijk[0] + s[0] - 1 + tt[0], ijk[1] + s[1] - 1 + tt[1], d == 3 ? ijk[2] + s[2] - 1 + tt[2] : 0};
        double av = alpha_at(q[0], q[1], q[2]);
        for (int a = 0; a < d; ++a) mc[a] += tt[a] ? av : -av;
      }
      for (int a = 0; a < d; ++a) m[a] += mc[a] / ((double)(nc / 2) * h);
    }
    double mm = 0.0;
    for (int a = 0; a < d; ++a) {
      m[a] /= (double)nc;
      mm += m[a] * m[a];
    }
    const double inv = 1.0 / std::sqrt(mm + 1e-30);
    double n[3] = {0, 0, 0};
    for (int a = 0; a < d; ++a) n[a] = m[a] * inv;
    double Gp[3] = {0, 0, 0};
    centre(ijk, Gp);
    // P5: intersect point
    const double delta = h / 100.0;
    int kf = 0;
    for (int k = 1; k <= 1000; ++k) {
      double P[3];
      for (int a = 0; a < d; ++a) P[a] = Gp[a] + ((double)k * delta) * n[a];
      if (!S.solid(P)) {
        kf = k;
        break;
      }
    }
    if (!kf) {
      err[gi] = 1;
      return;
    }
    double tlo = (double)(kf - 1) * delta, thi = (double)kf * delta;
    for (int it = 0; it < 60; ++it) {
      double tm = 0.5 * (tlo + thi);
      double P[3];
      for (int a = 0; a < d; ++a) P[a] = Gp[a] + tm * n[a];
      if (S.solid(P)) tlo = tm;
      else thi = tm;
    }
    double I[3], dn2 = 0.0;
    for (int a = 0; a < d; ++a) {
      I[a] = Gp[a] + thi * n[a];
      dn2 += (I[a] - Gp[a]) * (I[a] - Gp[a]);
    }
    const double dn = std::sqrt(dn2);
    // P6: mirror and interpolation points
    double M[3], IP[2][3];
    for (int a = 0; a < d; ++a) {
      M[a] = I[a] + d1 * n[a];
      IP[0][a] = M[a] + d2 * n[a];
      IP[1][a] = M[a] + (2.0 * d2) * n[a];
    }
    for (int a = 0; a < d; ++a) g->normal[(size_t)a * G + gi] = n[a];
    g->dn[gi] = dn;
    g->gamma[gi] = d1 / dn;
    // P7-P8: averaging points and weights
    for (int jp = 0; jp < 2; ++jp) {
      int cs[3] = {0, 0, 0};
      for (int a = 0; a < d; ++a) cs[a] = (int)std::floor((IP[jp][a] - g->lo[a]) / h);
      int64_t idx[7];
      double hk[7];
      bool valid[7];
      for (int sl = 0; sl < K; ++sl) {
        int u[3] = {cs[0], cs[1], cs[2]};
        if (sl > 0) u[(sl - 1) / 2] += ((sl - 1) % 2 == 0) ? -1 : 1;
        bool ok = true;
        int wq[3] = {0, 0, 0};
        for (int a = 0; a < d; ++a) {
          if (a < d - 1) wq[a] = ((u[a] % g->n[a]) + g->n[a]) % g->n[a];
          else {
            ok = ok && u[a] >= 0 && u[a] < g->n[a];
            wq[a] = std::min(std::max(u[a], 0), g->n[a] - 1);
          }
        }
        int64_t lin = lin_of(wq);
        ok = ok && !csolid[lin];
        double dist2 = 0.0;
        for (int a = 0; a < d; ++a) {
          double dd = IP[jp][a] - (g->lo[a] + ((double)u[a] + 0.5) * h);
          dist2 = dist2 + dd * dd;
        }
        idx[sl] = lin;
        hk[sl] = std::sqrt(dist2);
        valid[sl] = ok;
      }
      double wv[7] = {0, 0, 0, 0, 0, 0, 0};
      int first = -1;
      for (int sl = 0; sl < K; ++sl)
        if (valid[sl]) {
          first = sl;
          break;
        }
      if (first < 0) {
        // fallback: nearest fluid centre within 2h
        double best = 1e300;
        int64_t bl = -1;
        for (int oz = (d == 3 ? -2 : 0); oz <= (d == 3 ? 2 : 0); ++oz)
          for (int oy = -2; oy <= 2; ++oy)
            for (int ox = -2; ox <= 2; ++ox) {
              int u[3] = {cs[0] + ox, cs[1] + oy, cs[2] + oz};
              if (u[d - 1] < 0 || u[d - 1] >= g->n[d - 1]) continue;
              int wq[3] = {0, 0, 0};
              for (int a = 0; a < d; ++a) wq[a] = a < d - 1 ? ((u[a] % g->n[a]) + g->n[a]) % g->n[a] : u[a];
              int64_t lin = lin_of(wq);
              if (csolid[lin]) continue;
              double dist2 = 0.0;
              for (int a = 0; a < d; ++a) {
                double dd = IP[jp][a] - (g->lo[a] + ((double)u[a] + 0.5) * h);
                dist2 += dd * dd;
              }
              double dist = std::sqrt(dist2);
              if (dist <= 2.0 * h && dist < best) {
                best = dist;
                bl = lin;
              }
            }
        if (bl < 0) {
          err[gi] = 2;
          return;
        }
        for (int sl = 0; sl < K; ++sl) {
          idx[sl] = bl;
          wv[sl] = sl == 0 ? 1.0 : 0.0;
        }
      } else {
        int near = -1;
        for (int sl = 0; sl < K; ++sl)
          if (valid[sl] && hk[sl] < 1e-12 * h) {
            near = sl;
            break;
          }
        if (near >= 0) {
          wv[near] = 1.0;
        } else {
          double invs[7], q = 0.0;
          for (int sl = 0; sl < K; ++sl)
            if (valid[sl]) {
              invs[sl] = 1.0 / (hk[sl] * hk[sl]);
              q += invs[sl];
            }
          for (int sl = 0; sl < K; ++sl)
            if (valid[sl]) wv[sl] = invs[sl] / q;
        }
        for (int sl = 0; sl < K; ++sl)
          if (!valid[sl]) idx[sl] = idx[first];
      }
      for (int sl = 0; sl < K; ++sl) {
        g->ap[((size_t)jp * K + sl) * G + gi] = idx[sl];
        g->w[((size_t)jp * K + sl) * G + gi] = wv[sl];
      }
    }
  });
  for (int64_t gi = 0; gi < G; ++gi) {
    if (err[gi] == 1) {
      delete g;
      return fail(CH_IB_EGEOM, "marching along the normal found no fluid within 10 cells");
    }
    if (err[gi] == 2) {
      delete g;
      return fail(CH_IB_EGEOM, "an interpolation point has no fluid averaging point within 2h");
    }
  }
  (void)nz;
  *out = g;
  return CH_IB_OK;
}

extern "C" int ch_ib_geometry_import(const ch_ib_grid *grid, const ch_ib_ghost_tables *t,
                                     ch_ib_geometry **out) {
  using chib::fail;
  if (!out || !t) return fail(CH_IB_EINVAL, "NULL argument");
  *out = nullptr;
  auto *g = new ch_ib_geometry();
  int rc = chib::check_grid(grid, g);
  if (rc) {
    delete g;
    return rc;
  }
  const int d = g->ndim;
  const int K = 2 * d + 1;
  if (t->ndim != d || t->n_ap != K || t->n_ghost < 0) {
    delete g;
    return fail(CH_IB_EINVAL, "table dimensions do not match the grid");
  }
  const int64_t G = t->n_ghost;
  if (G > 0 && (!t->gidx || !t->normal || !t->dn || !t->gamma || !t->ap || !t->w)) {
    delete g;
    return fail(CH_IB_EINVAL, "NULL table array");
  }
  g->n_ghost = G;
  g->n_ap = K;
  g->gidx.assign(t->gidx, t->gidx + G);
  g->normal.assign(t->normal, t->normal + (size_t)d * G);
  g->dn.assign(t->dn, t->dn + G);
  g->gamma.assign(t->gamma, t->gamma + G);
  g->ap.assign(t->ap, t->ap + (size_t)2 * K * G);
  g->w.assign(t->w, t->w + (size_t)2 * K * G);
  if (t->alpha) g->alpha.assign(t->alpha, t->alpha + g->cells);
  for (int64_t i = 0; i < G; ++i) {
    if (g->gidx[i] < 0 || g->gidx[i] >= g->cells || (i && g->gidx[i] <= g->gidx[i - 1])) {
      delete g;
      return fail(CH_IB_EINVAL, "ghost indices must be in range and strictly increasing");
    }
    if (!(g->dn[i] > 0) || !(g->gamma[i] > 0)) {
      delete g;
      return fail(CH_IB_EINVAL, "dn and gamma must be positive");
    }
    int last = (int)((d == 2) ? (g->gidx[i] / g->n[0]) : (g->gidx[i] / ((int64_t)g->n[0] * g->n[1])));
    if (last == 0 || last == g->n[d - 1] - 1) {
      delete g;
      return fail(CH_IB_EGEOM, "a ghost point touches the box wall of the bounded axis");
    }
  }
  for (size_t i = 0; i < g->ap.size(); ++i)
    if (g->ap[i] < 0 || g->ap[i] >= g->cells) {
      delete g;
      return fail(CH_IB_EINVAL, "averaging point index out of range");
    }
  *out = g;
  return CH_IB_OK;
}

extern "C" int ch_ib_geometry_export(const ch_ib_geometry *g, ch_ib_ghost_tables *t) {
  using chib::fail;
  if (!g || !t) return fail(CH_IB_EINVAL, "NULL argument");
  if (t->n_ghost != g->n_ghost || t->n_ap != g->n_ap || t->ndim != g->ndim)
    return fail(CH_IB_ENOMEM, "destination sized for a different table");
  const int64_t G = g->n_ghost;
  const int d = g->ndim, K = g->n_ap;
  if (G > 0 && (!t->gidx || !t->normal || !t->dn || !t->gamma || !t->ap || !t->w))
    return fail(CH_IB_EINVAL, "NULL destination array");
  std::copy(g->gidx.begin(), g->gidx.end(), t->gidx);
  std::copy(g->normal.begin(), g->normal.end(), t->normal);
  std::copy(g->dn.begin(), g->dn.end(), t->dn);
  std::copy(g->gamma.begin(), g->gamma.end(), t->gamma);
  std::copy(g->ap.begin(), g->ap.end(), t->ap);
  std::copy(g->w.begin(), g->w.end(), t->w);
  if (t->alpha) {
    if (g->alpha.empty()) std::fill(t->alpha, t->alpha + g->cells, 1.0);
    else std::copy(g->alpha.begin(), g->alpha.end(), t->alpha);
  }
  (void)d;
  (void)K;
  return CH_IB_OK;
}

extern "C" int ch_ib_geometry_count(const ch_ib_geometry *g, int64_t *n_ghost, int *n_ap) {
  if (!g) return chib::fail(CH_IB_EINVAL, "NULL geometry");
  if (n_ghost) *n_ghost = g->n_ghost;
  if (n_ap) *n_ap = g->n_ap;
  return CH_IB_OK;
}

extern "C" void ch_ib_geometry_free(ch_ib_geometry *g) { delete g; }

// Signed distance to the wall (positive in the fluid) and the unit wall normal (into the fluid)
// of the nearest wall point, per cell of a 2D grid: the minimum of the shapes' own signed
// distances (union of solids).  Half-plane and circle in closed form; sinusoid by the nearest
// point of the curve (16 seeds over one wavelength around the cell, then Newton on the squared
// distance).  Used for the features of the learned wall-band correction.
extern "C" int ch_ib_wall_field(const ch_ib_grid *grid, const ch_ib_shape *shapes, int n_shapes, double *dist,
                                double *normal) {
  ch_ib_geometry g;
  int rc = chib::check_grid(grid, &g);
  if (rc) return rc;
  if (g.ndim != 2) return chib::fail(CH_IB_EUNSUPPORTED, "wall field: 2D grids only");
  if (!dist || !normal || (n_shapes > 0 && !shapes)) return chib::fail(CH_IB_EINVAL, "NULL argument");
  for (int s = 0; s < n_shapes; ++s)
    if (shapes[s].kind != CH_IB_HALFPLANE && shapes[s].kind != CH_IB_SINUSOID && shapes[s].kind != CH_IB_SPHERE)
      return chib::fail(CH_IB_EUNSUPPORTED, "wall field: half-plane, sinusoid and circle walls only");
  const int nx = g.n[0], ny = g.n[1];
  const double h = g.h;
  parallel_for((int64_t)nx * ny, [&](int64_t c) {
    const int i = (int)(c % nx), j = (int)(c / nx);
    const double x = g.lo[0] + (i + 0.5) * h, y = g.lo[1] + (j + 0.5) * h;
    double best = 1e300, bn0 = 0.0, bn1 = 1.0;
    for (int s = 0; s < n_shapes; ++s) {
      const double *p = shapes[s].p;
      double sd = 0.0, n0 = 0.0, n1 = 1.0;
      if (shapes[s].kind == CH_IB_HALFPLANE) {
        const double nn = std::sqrt(p[3] * p[3] + p[4] * p[4]);
        n0 = p[3] / nn;
        n1 = p[4] / nn;
        sd = (x - p[0]) * n0 + (y - p[1]) * n1;
      } else if (shapes[s].kind == CH_IB_SPHERE) {
        const double dx = x - p[0], dy = y - p[1];
        const double r = std::sqrt(dx * dx + dy * dy);
        sd = r - p[3];
        n0 = r > 0 ? dx / r : 0.0;
        n1 = r > 0 ? dy / r : 1.0;
      } else {
        const double A = p[1], lam = p[2], k = kTwoPi / lam, ph = p[3];
        auto D = [&](double t) {
          const double yw = p[0] + A * std::sin(k * t + ph);
          return (t - x) * (t - x) + (yw - y) * (yw - y);
        };
        double tb = x, db = D(x);
        for (int q = 0; q < 16; ++q) {
          const double t = x + lam * ((q + 0.5) / 16.0 - 0.5);
          const double v = D(t);
          if (v < db) { db = v; tb = t; }
        }
        for (int it = 0; it < 50; ++it) {   // Newton on D'(t) = 0
          const double sn = std::sin(k * tb + ph), cs = std::cos(k * tb + ph);
          const double yw = p[0] + A * sn, y1 = A * k * cs, y2 = -A * k * k * sn;
          const double g1 = 2.0 * ((tb - x) + (yw - y) * y1);
          const double g2 = 2.0 * (1.0 + y1 * y1 + (yw - y) * y2);
          if (g2 <= 0.0) break;
          const double step = g1 / g2;
          tb -= step;
          if (std::fabs(step) < 1e-15 * (1.0 + std::fabs(tb))) break;
        }
        const double yw = p[0] + A * std::sin(k * tb + ph), y1 = A * k * std::cos(k * tb + ph);
        const double dd = std::sqrt((tb - x) * (tb - x) + (yw - y) * (yw - y));
        const double yx = p[0] + A * std::sin(k * x + ph);
        sd = y >= yx ? dd : -dd;
        const double nn = std::sqrt(1.0 + y1 * y1);
        n0 = -y1 / nn;
        n1 = 1.0 / nn;
      }
      if (sd < best) { best = sd; bn0 = n0; bn1 = n1; }
    }
    dist[c] = n_shapes > 0 ? best : 1e300;
    normal[c] = bn0;
    normal[(int64_t)nx * ny + c] = bn1;
  });
  return CH_IB_OK;
}

extern "C" int ch_ib_geometry_face_fractions(const ch_ib_geometry *g, double *dst) {
  using chib::fail;
  if (!g || !dst) return fail(CH_IB_EINVAL, "NULL argument");
  if (g->face_alpha.empty())
    return fail(CH_IB_EUNSUPPORTED, "the geometry holds no staggered-cell fractions");
  std::copy(g->face_alpha.begin(), g->face_alpha.end(), dst);
  return CH_IB_OK;
}

extern "C" int ch_ib_geometry_set_face_fractions(ch_ib_geometry *g, const double *src) {
  using chib::fail;
  if (!g || !src) return fail(CH_IB_EINVAL, "NULL argument");
  const size_t n = (size_t)g->ndim * (size_t)g->cells;
  for (size_t i = 0; i < n; ++i)
    if (!(src[i] >= 0.0 && src[i] <= 1.0)) return fail(CH_IB_EINVAL, "fractions must lie in [0, 1]");
  g->face_alpha.assign(src, src + n);
  return CH_IB_OK;
}
