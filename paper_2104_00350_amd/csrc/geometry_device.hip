// Geometry preprocessing on the GPU (section 4.1): the same tables as the host builder
// (ch_ib_geometry_build), computed with one thread per cell for the volume fraction and the
// ghost list and one thread per ghost for normals, intersect, mirror and interpolation points,
// averaging points and weights.  The readings of the passages the paper leaves open are those
// of the host builder (see geometry.cpp) and the arithmetic is the same sequence of operations,
// compiled without contraction of multiplies and adds, so integer tables and most doubles match
// the host builder bit for bit.  The one exception is the sinusoid, whose sine comes from the
// device math library: a subgrid point within an ulp of the wall may count on the other side.
//
// The caller owns the device scratch (ch_ib_geometry_device_bytes); the result is an ordinary
// host geometry object.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"

namespace {

constexpr int kGeomThreads = 256;
constexpr int kMaxShapes = 8;
constexpr double kTwoPiD = 6.283185307179586;

struct DevShapes {
  int n_shapes;
  int d;
  int n[3];
  double lo[3], hi[3];
  int kind[kMaxShapes];
  double p[kMaxShapes][10];
  double bc[kMaxShapes], bs[kMaxShapes];   // cos and sin of a box's angle (host-computed)
};

struct GeomArgs {
  DevShapes S;
  double h, hs, d1, d2;
  int sub;
  int64_t N;
  double off[3];   // control-volume shift: 0 for the cells, h/2 along one axis for staggered cells
};

__device__ bool solid_one(const DevShapes &S, int i, const double *x) {
  const double *p = S.p[i];
  const int d = S.d;
  switch (S.kind[i]) {
    case CH_IB_HALFPLANE: {
      double v = (x[0] - p[0]) * p[3] + (x[1] - p[1]) * p[4];
      if (d == 3) v = v + (x[2] - p[2]) * p[5];
      return v < 0.0;
    }
    case CH_IB_SINUSOID: {
      double yw = p[0] + p[1] * sin(kTwoPiD * x[0] / p[2] + p[3]);
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
      double c = S.bc[i], s_ = S.bs[i];
      double dx = x[0] - p[0], dy = x[1] - p[1];
      double q0 = c * dx + s_ * dy;
      double q1 = -s_ * dx + c * dy;
      bool out = fabs(q0) > p[3] || fabs(q1) > p[3];
      if (d == 3) out = out || fabs(x[2] - p[2]) > p[3];
      return out;
    }
    default:
      return false;
  }
}

__device__ bool solid(const DevShapes &S, const double *xin) {
  const int d = S.d;
  double x[3] = {xin[0], xin[1], d == 3 ? xin[2] : 0.0};
  for (int a = 0; a < d - 1; ++a) {
    double L = S.hi[a] - S.lo[a];
    if (x[a] >= S.hi[a]) x[a] = x[a] - L;
    else if (x[a] < S.lo[a]) x[a] = x[a] + L;
  }
  for (int i = 0; i < S.n_shapes; ++i)
    if (solid_one(S, i, x)) return true;
  return false;
}

__device__ bool may_cut(const DevShapes &S, int i, const double *xc, double h) {
  const int d = S.d;
  const double hd = 0.5 * h * sqrt((double)d);
  const double m = 1e-9 * h;
  const double *p = S.p[i];
  switch (S.kind[i]) {
    case CH_IB_HALFPLANE: {
      double nn = 0.0, v = 0.0;
      for (int a = 0; a < d; ++a) {
        nn += p[3 + a] * p[3 + a];
        v += (xc[a] - p[a]) * p[3 + a];
      }
      return fabs(v / sqrt(nn)) <= hd + m;
    }
    case CH_IB_SPHERE: {
      double r2 = 0.0;
      for (int a = 0; a < d; ++a) r2 += (xc[a] - p[a]) * (xc[a] - p[a]);
      return fabs(sqrt(r2) - p[3]) <= hd + m;
    }
    case CH_IB_SINUSOID: {
      double lip = kTwoPiD * fabs(p[1]) / p[2];
      double yw = p[0] + p[1] * sin(kTwoPiD * xc[0] / p[2] + p[3]);
      return fabs(xc[d - 1] - yw) <= 0.5 * h + 0.5 * lip * h + m;
    }
    case CH_IB_BOX: {
      double c = S.bc[i], s_ = S.bs[i];
      double dx = xc[0] - p[0], dy = xc[1] - p[1];
      double q[3] = {fabs(c * dx + s_ * dy) - p[3], fabs(-s_ * dx + c * dy) - p[3],
                     d == 3 ? fabs(xc[2] - p[2]) - p[3] : -1e300};
      double out2 = 0.0, qmax = -1e300;
      for (int a = 0; a < d; ++a) {
        double qq = fmax(q[a], 0.0);
        out2 += qq * qq;
        qmax = fmax(qmax, q[a]);
      }
      double sd = sqrt(out2) + fmin(qmax, 0.0);
      return fabs(sd) <= hd + m;
    }
    default:
      return true;
  }
}

__device__ void coords(const DevShapes &S, int64_t lin, int *ijk) {
  ijk[0] = (int)(lin % S.n[0]);
  ijk[1] = (int)((lin / S.n[0]) % S.n[1]);
  ijk[2] = (int)(lin / ((int64_t)S.n[0] * S.n[1]));
}

__device__ int64_t lin_of(const DevShapes &S, const int *ijk) {
  return ijk[0] + (int64_t)S.n[0] * (ijk[1] + (int64_t)S.n[1] * ijk[2]);
}

// P1: centre solid mask; a cell no shape can cut gets its volume fraction (0 or 1) here, a cut
// cell is flagged for the subgrid count.
__global__ __launch_bounds__(kGeomThreads) void k_gd_classify(GeomArgs A, double *__restrict__ alpha,
                                                              unsigned char *__restrict__ csolid,
                                                              unsigned char *__restrict__ cutf) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= A.N) return;
  const DevShapes &S = A.S;
  const int d = S.d;
  int ijk[3];
  coords(S, c, ijk);
  double xc[3] = {0, 0, 0};
  for (int a = 0; a < d; ++a) xc[a] = S.lo[a] + ((double)ijk[a] + 0.5) * A.h;
  for (int a = 0; a < d; ++a) xc[a] = xc[a] + A.off[a];
  const bool cs = solid(S, xc);
  if (csolid) csolid[c] = cs ? 1 : 0;
  bool cut = false;
  for (int i = 0; i < S.n_shapes; ++i) cut = cut || may_cut(S, i, xc, A.h);
  cutf[c] = cut ? 1 : 0;
  if (!cut) alpha[c] = cs ? 0.0 : 1.0;
}

// P2: volume fraction of the cut cells by counting subgrid points, one 64-lane wave per cut cell
// (the lanes share its sub^d points; the count is an integer, so its order does not matter).
__global__ __launch_bounds__(kGeomThreads) void k_gd_subgrid(GeomArgs A, const int *__restrict__ cutlist,
                                                             int64_t n_cut, double *__restrict__ alpha) {
  const int lane = threadIdx.x & 63;
  const int64_t item = (int64_t)blockIdx.x * (kGeomThreads / 64) + (threadIdx.x >> 6);
  if (item >= n_cut) return;   // whole waves leave together
  const DevShapes &S = A.S;
  const int d = S.d;
  const int64_t c = cutlist[item];
  int ijk[3];
  coords(S, c, ijk);
  double base[3] = {0, 0, 0};
  for (int a = 0; a < d; ++a) base[a] = S.lo[a] + (double)ijk[a] * A.h + A.off[a];
  const int sub = A.sub;
  const int per_cell = sub * sub * (d == 3 ? sub : 1);   // sub <= 1000 (checked on the host)
  // point q = i + sub (j + sub k); lane starts at q = lane and strides by 64, carried digit-wise
  int i = lane % sub, j = (lane / sub) % sub, k = lane / (sub * sub);
  const int di = 64 % sub, dj = (64 / sub) % sub, dk = 64 / (sub * sub);
  int fluid = 0;
  for (int q = lane; q < per_cell; q += 64) {
    double x[3] = {0, 0, 0};
    x[0] = base[0] + ((double)i + 0.5) * A.hs;
    x[1] = base[1] + ((double)j + 0.5) * A.hs;
    if (d == 3) x[2] = base[2] + ((double)k + 0.5) * A.hs;
    if (!solid(S, x)) ++fluid;
    i += di;
    if (i >= sub) {
      i -= sub;
      ++j;
    }
    j += dj;
    if (j >= sub) {
      j -= sub;
      ++k;
    }
    k += dk;
  }
  for (int off = 32; off > 0; off >>= 1) fluid += __shfl_down(fluid, off, 64);
  if (lane == 0) alpha[c] = (double)fluid / (double)per_cell;
}

// Ghost: solid centre with a face neighbour whose centre is fluid.  Flags a ghost in the first
// or last layer of the bounded axis (*bad = 1).
__device__ bool is_ghost(const DevShapes &S, const unsigned char *__restrict__ csolid, int64_t c, int *bad) {
  if (!csolid[c]) return false;
  const int d = S.d;
  int ijk[3];
  coords(S, c, ijk);
  bool nb_fluid = false;
  for (int a = 0; a < d && !nb_fluid; ++a) {
    for (int sgn = -1; sgn <= 1; sgn += 2) {
      int q[3] = {ijk[0], ijk[1], ijk[2]};
      q[a] += sgn;
      if (a < d - 1) q[a] = (q[a] + S.n[a]) % S.n[a];
      else if (q[a] < 0 || q[a] >= S.n[a]) continue;
      if (!csolid[lin_of(S, q)]) {
        nb_fluid = true;
        break;
      }
    }
  }
  if (nb_fluid && (ijk[d - 1] == 0 || ijk[d - 1] == S.n[d - 1] - 1)) *bad = 1;
  return nb_fluid;
}

// Per-block counts (phase 1) or the list in cell order (phase 2, block offsets given) of the
// ghosts (MODE 0, mask = centre solid mask) or of the cut cells (MODE 1, mask = cut flags): a
// block-wide scan of the flags ranks them inside the block.
template <int MODE>
__global__ __launch_bounds__(kGeomThreads) void k_gd_list(GeomArgs A, const unsigned char *__restrict__ mask,
                                                          int *__restrict__ bcount, const int *__restrict__ boff,
                                                          int *__restrict__ list, int *__restrict__ bad) {
  __shared__ int s[kGeomThreads];
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int b = 0;
  int flag = 0;
  if (c < A.N) flag = MODE == 0 ? (is_ghost(A.S, mask, c, &b) ? 1 : 0) : (mask[c] ? 1 : 0);
  if (b) *bad = 1;   // every writer stores the same value
  s[threadIdx.x] = flag;
  __syncthreads();
  for (int off = 1; off < kGeomThreads; off <<= 1) {   // inclusive Hillis-Steele scan
    const int v = threadIdx.x >= (unsigned)off ? s[threadIdx.x - off] : 0;
    __syncthreads();
    s[threadIdx.x] += v;
    __syncthreads();
  }
  if (!boff) {
    if (threadIdx.x == kGeomThreads - 1) bcount[blockIdx.x] = s[kGeomThreads - 1];
    return;
  }
  if (flag) list[boff[blockIdx.x] + s[threadIdx.x] - 1] = (int)c;
}

// P3-P8 per ghost: normal from corner gradients of alpha, intersect point by marching along the
// normal and bisecting, mirror and interpolation points, averaging points and weights.
__global__ __launch_bounds__(kGeomThreads) void k_gd_tables(GeomArgs A, const double *__restrict__ alpha,
                                                            const unsigned char *__restrict__ csolid,
                                                            const int *__restrict__ gidx, int64_t G,
                                                            double *__restrict__ normal, double *__restrict__ dn_out,
                                                            double *__restrict__ gam_out, int *__restrict__ ap,
                                                            double *__restrict__ w, int *__restrict__ err) {
  const int64_t gi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gi >= G) return;
  const DevShapes &S = A.S;
  const int d = S.d;
  const double h = A.h;
  const int K = 2 * d + 1;
  const int64_t c = gidx[gi];
  int ijk[3];
  coords(S, c, ijk);
  auto alpha_at = [&](int i, int j, int k) {
    int q[3] = {i, j, k};
    for (int a = 0; a < d - 1; ++a) q[a] = (q[a] + S.n[a]) % S.n[a];
    if (d == 2) q[2] = 0;
    return alpha[lin_of(S, q)];
  };
  double m[3] = {0, 0, 0};
  const int nc = 1 << d;
  for (int corner = 0; corner < nc; ++corner) {
    int sc[3] = {corner & 1, (corner >> 1) & 1, (corner >> 2) & 1};
    double mc[3] = {0, 0, 0};
    for (int t = 0; t < nc; ++t) {
      int tt[3] = {t & 1, (t >> 1) & 1, (t >> 2) & 1};
      int q[3] = {ijk[0] + sc[0] - 1 + tt[0], ijk[1] + sc[1] - 1 + tt[1], d == 3 ? ijk[2] + sc[2] - 1 + tt[2] : 0};
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
  const double inv = 1.0 / sqrt(mm + 1e-30);
  double n[3] = {0, 0, 0};
  for (int a = 0; a < d; ++a) n[a] = m[a] * inv;
  double Gp[3] = {0, 0, 0};
  for (int a = 0; a < d; ++a) Gp[a] = S.lo[a] + ((double)ijk[a] + 0.5) * h;
  const double delta = h / 100.0;
  int kf = 0;
  for (int k = 1; k <= 1000; ++k) {
    double P[3] = {0, 0, 0};
    for (int a = 0; a < d; ++a) P[a] = Gp[a] + ((double)k * delta) * n[a];
    if (!solid(S, P)) {
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
    double P[3] = {0, 0, 0};
    for (int a = 0; a < d; ++a) P[a] = Gp[a] + tm * n[a];
    if (solid(S, P)) tlo = tm;
    else thi = tm;
  }
  double I[3] = {0, 0, 0}, dn2 = 0.0;
  for (int a = 0; a < d; ++a) {
    I[a] = Gp[a] + thi * n[a];
    dn2 += (I[a] - Gp[a]) * (I[a] - Gp[a]);
  }
  const double dn = sqrt(dn2);
  double M[3] = {0, 0, 0}, IP[2][3] = {{0, 0, 0}, {0, 0, 0}};
  for (int a = 0; a < d; ++a) {
    M[a] = I[a] + A.d1 * n[a];
    IP[0][a] = M[a] + A.d2 * n[a];
    IP[1][a] = M[a] + (2.0 * A.d2) * n[a];
  }
  for (int a = 0; a < d; ++a) normal[(int64_t)a * G + gi] = n[a];
  dn_out[gi] = dn;
  gam_out[gi] = A.d1 / dn;
  for (int jp = 0; jp < 2; ++jp) {
    int cs[3] = {0, 0, 0};
    for (int a = 0; a < d; ++a) cs[a] = (int)floor((IP[jp][a] - S.lo[a]) / h);
    int64_t idx[7] = {0, 0, 0, 0, 0, 0, 0};
    double hk[7] = {0, 0, 0, 0, 0, 0, 0};
    bool valid[7] = {false, false, false, false, false, false, false};
    for (int sl = 0; sl < K; ++sl) {
      int u[3] = {cs[0], cs[1], cs[2]};
      if (sl > 0) u[(sl - 1) / 2] += ((sl - 1) % 2 == 0) ? -1 : 1;
      bool ok = true;
      int wq[3] = {0, 0, 0};
      for (int a = 0; a < d; ++a) {
        if (a < d - 1) {
          wq[a] = ((u[a] % S.n[a]) + S.n[a]) % S.n[a];
        } else {
          ok = ok && u[a] >= 0 && u[a] < S.n[a];
          wq[a] = min(max(u[a], 0), S.n[a] - 1);
        }
      }
      const int64_t lin = lin_of(S, wq);
      ok = ok && !csolid[lin];
      double dist2 = 0.0;
      for (int a = 0; a < d; ++a) {
        double dd = IP[jp][a] - (S.lo[a] + ((double)u[a] + 0.5) * h);
        dist2 = dist2 + dd * dd;
      }
      idx[sl] = lin;
      hk[sl] = sqrt(dist2);
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
            if (u[d - 1] < 0 || u[d - 1] >= S.n[d - 1]) continue;
            int wq[3] = {0, 0, 0};
            for (int a = 0; a < d; ++a) wq[a] = a < d - 1 ? ((u[a] % S.n[a]) + S.n[a]) % S.n[a] : u[a];
            const int64_t lin = lin_of(S, wq);
            if (csolid[lin]) continue;
            double dist2 = 0.0;
            for (int a = 0; a < d; ++a) {
              double dd = IP[jp][a] - (S.lo[a] + ((double)u[a] + 0.5) * h);
              dist2 += dd * dd;
            }
            const double dist = sqrt(dist2);
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
      int nearest = -1;
      for (int sl = 0; sl < K; ++sl)
        if (valid[sl] && hk[sl] < 1e-12 * h) {
          nearest = sl;
          break;
        }
      if (nearest >= 0) {
        wv[nearest] = 1.0;
      } else {
        double invs[7] = {0, 0, 0, 0, 0, 0, 0}, q = 0.0;
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
      ap[((int64_t)jp * K + sl) * G + gi] = (int)idx[sl];
      w[((int64_t)jp * K + sl) * G + gi] = wv[sl];
    }
  }
  err[gi] = 0;
}

// Scratch layout (bytes, 256-aligned pieces): alpha N doubles, solid and cut masks N bytes each,
// the cut-cell list N ints, block counts and offsets, the bad flag, then per-ghost arrays sized
// for gmax ghosts.
struct DevLayout {
  size_t alpha, csolid, cutf, cutlist, bcount, boff, bad, gidx, normal, dn, gam, ap, w, err, total;
  int64_t gmax;
  int64_t nblocks;
};

size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

DevLayout dev_layout(int64_t N, int d) {
  DevLayout L{};
  const int K = 2 * d + 1;
  L.nblocks = (N + kGeomThreads - 1) / kGeomThreads;
  L.gmax = N / 8 + 1024;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += up256(bytes);
    return at;
  };
  L.alpha = take(N * 8);
  L.csolid = take(N);
  L.cutf = take(N);
  L.cutlist = take(N * 4);
  L.bcount = take(L.nblocks * 4);
  L.boff = take(L.nblocks * 4);
  L.bad = take(4);
  L.gidx = take(L.gmax * 4);
  L.normal = take((size_t)d * L.gmax * 8);
  L.dn = take(L.gmax * 8);
  L.gam = take(L.gmax * 8);
  L.ap = take((size_t)2 * K * L.gmax * 4);
  L.w = take((size_t)2 * K * L.gmax * 8);
  L.err = take(L.gmax * 4);
  L.total = o;
  return L;
}

int hip_error(hipError_t e, const char *where) {
  return chib::fail(CH_IB_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

}  // namespace

extern "C" size_t ch_ib_geometry_device_bytes(const ch_ib_grid *grid) {
  ch_ib_geometry g;
  if (chib::check_grid(grid, &g)) return 0;
  return dev_layout(g.cells, g.ndim).total + 256;
}

extern "C" int ch_ib_geometry_build_device(const ch_ib_grid *grid, const ch_ib_shape *shapes, int n_shapes,
                                           const ch_ib_params *params, void *device_scratch, size_t bytes,
                                           void *hip_stream, ch_ib_geometry **out) {
  using chib::fail;
  if (!out || !params) return fail(CH_IB_EINVAL, "NULL argument");
  *out = nullptr;
  ch_ib_geometry tmp;
  int rc = chib::check_grid(grid, &tmp);
  if (rc) return rc;
  if (n_shapes < 0 || (n_shapes > 0 && !shapes)) return fail(CH_IB_EINVAL, "bad shape list");
  if (n_shapes > kMaxShapes) return fail(CH_IB_EUNSUPPORTED, "at most 8 shapes on the device builder");
  if (!device_scratch) return fail(CH_IB_EINVAL, "NULL device scratch");
  if (((uintptr_t)device_scratch) & 255) return fail(CH_IB_EINVAL, "device scratch must be 256-byte aligned");
  const int d = tmp.ndim;
  const int64_t N = tmp.cells;
  const DevLayout L = dev_layout(N, d);
  if (bytes < L.total) return fail(CH_IB_ENOMEM, "device scratch too small: need " + std::to_string(L.total) + " bytes");
  GeomArgs A{};
  A.S.n_shapes = n_shapes;
  A.S.d = d;
  for (int a = 0; a < 3; ++a) {
    A.S.n[a] = tmp.n[a];
    A.S.lo[a] = a < d ? grid->lo[a] : 0.0;
    A.S.hi[a] = a < d ? grid->hi[a] : 0.0;
  }
  for (int i = 0; i < n_shapes; ++i) {
    if (shapes[i].kind < CH_IB_HALFPLANE || shapes[i].kind > CH_IB_BOX) return fail(CH_IB_EINVAL, "unknown shape kind");
    if (shapes[i].kind == CH_IB_SINUSOID && !(shapes[i].p[2] > 0))
      return fail(CH_IB_EINVAL, "sinusoid wavelength must be positive");
    A.S.kind[i] = shapes[i].kind;
    std::memcpy(A.S.p[i], shapes[i].p, sizeof(A.S.p[i]));
    A.S.bc[i] = std::cos(shapes[i].p[4]);
    A.S.bs[i] = std::sin(shapes[i].p[4]);
  }
  A.h = tmp.h;
  A.sub = params->subgrid > 0 ? params->subgrid : 100;
  if (A.sub > 1000) return fail(CH_IB_EUNSUPPORTED, "at most 1000 subgrid points per direction on the device builder");
  A.hs = tmp.h / A.sub;
  A.d1 = (params->d1_cells > 0 ? params->d1_cells : 2.0) * tmp.h;
  A.d2 = (params->d2_cells > 0 ? params->d2_cells : 1.5) * tmp.h;
  A.N = N;
  char *ws = (char *)device_scratch;
  double *alpha = (double *)(ws + L.alpha);
  unsigned char *csolid = (unsigned char *)(ws + L.csolid);
  int *bcount = (int *)(ws + L.bcount), *boff = (int *)(ws + L.boff), *bad = (int *)(ws + L.bad);
  int *gidx = (int *)(ws + L.gidx), *ap = (int *)(ws + L.ap), *err = (int *)(ws + L.err);
  double *normal = (double *)(ws + L.normal), *dn = (double *)(ws + L.dn), *gam = (double *)(ws + L.gam);
  double *w = (double *)(ws + L.w);
  hipStream_t s = (hipStream_t)hip_stream;
  const unsigned nb = (unsigned)L.nblocks;

  unsigned char *cutf = (unsigned char *)(ws + L.cutf);
  int *cutlist = (int *)(ws + L.cutlist);
  std::vector<int> counts(nb), offs(nb);
  // block counts -> exclusive block offsets (host prefix sum, uploaded); *total = sum of counts
  auto offsets = [&](int64_t *total) {
    hipError_t e2 = hipMemcpyAsync(counts.data(), bcount, (size_t)nb * 4, hipMemcpyDeviceToHost, s);
    if (e2 == hipSuccess) e2 = hipStreamSynchronize(s);
    if (e2 != hipSuccess) return e2;
    int64_t t = 0;
    for (unsigned b = 0; b < nb; ++b) {
      offs[b] = (int)t;
      t += counts[b];
    }
    *total = t;
    return hipMemcpyAsync(boff, offs.data(), (size_t)nb * 4, hipMemcpyHostToDevice, s);
  };
  int zero = 0;
  int64_t n_cut = 0, G = 0;
  hipError_t e = hipMemcpyAsync(bad, &zero, 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_gd_classify, dim3(nb), dim3(kGeomThreads), 0, s, A, alpha, csolid, cutf);
    hipLaunchKernelGGL(k_gd_list<1>, dim3(nb), dim3(kGeomThreads), 0, s, A, (const unsigned char *)cutf, bcount,
                       (const int *)nullptr, (int *)nullptr, bad);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = offsets(&n_cut);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_gd_list<1>, dim3(nb), dim3(kGeomThreads), 0, s, A, (const unsigned char *)cutf, bcount,
                       (const int *)boff, cutlist, bad);
    if (n_cut)
      hipLaunchKernelGGL(k_gd_subgrid, dim3((unsigned)((n_cut + 3) / 4)), dim3(kGeomThreads), 0, s, A,
                         (const int *)cutlist, n_cut, alpha);
    hipLaunchKernelGGL(k_gd_list<0>, dim3(nb), dim3(kGeomThreads), 0, s, A, (const unsigned char *)csolid, bcount,
                       (const int *)nullptr, (int *)nullptr, bad);
    e = hipGetLastError();
  }
  int hbad = 0;
  if (e == hipSuccess) e = offsets(&G);
  if (e == hipSuccess) e = hipMemcpyAsync(&hbad, bad, 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_error(e, "device geometry (volume fraction, ghosts)");
  if (hbad) return fail(CH_IB_EGEOM, "a ghost point touches the box wall of the bounded axis");
  if (G > L.gmax) return fail(CH_IB_ENOMEM, "more ghosts than the device builder holds (cells/8 + 1024)");
  {
    hipLaunchKernelGGL(k_gd_list<0>, dim3(nb), dim3(kGeomThreads), 0, s, A, (const unsigned char *)csolid, bcount,
                       (const int *)boff, gidx, bad);
    if (G)
      hipLaunchKernelGGL(k_gd_tables, dim3((unsigned)((G + kGeomThreads - 1) / kGeomThreads)), dim3(kGeomThreads), 0,
                         s, A, (const double *)alpha, (const unsigned char *)csolid, (const int *)gidx, G, normal, dn,
                         gam, ap, w, err);
    e = hipGetLastError();
  }
  auto *g = new ch_ib_geometry(tmp);
  const int K = 2 * d + 1;
  g->n_ghost = G;
  g->n_ap = K;
  g->alpha.resize(N);
  std::vector<int> gidx32(G), ap32((size_t)2 * K * G), err32(G);
  g->normal.resize((size_t)d * G);
  g->dn.resize(G);
  g->gamma.resize(G);
  g->w.resize((size_t)2 * K * G);
  auto get = [&](void *dst, const void *src, size_t nbytes) {
    if (e == hipSuccess && nbytes) e = hipMemcpyAsync(dst, src, nbytes, hipMemcpyDeviceToHost, s);
  };
  get(g->alpha.data(), alpha, (size_t)N * 8);
  get(gidx32.data(), gidx, (size_t)G * 4);
  get(err32.data(), err, (size_t)G * 4);
  get(g->normal.data(), normal, (size_t)d * G * 8);
  get(g->dn.data(), dn, (size_t)G * 8);
  get(g->gamma.data(), gam, (size_t)G * 8);
  get(ap32.data(), ap, (size_t)2 * K * G * 4);
  get(g->w.data(), w, (size_t)2 * K * G * 8);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    delete g;
    return hip_error(e, "device geometry (tables)");
  }
  for (int64_t i = 0; i < G; ++i) {
    if (err32[i] == 1) {
      delete g;
      return fail(CH_IB_EGEOM, "marching along the normal found no fluid within 10 cells");
    }
    if (err32[i] == 2) {
      delete g;
      return fail(CH_IB_EGEOM, "an interpolation point has no fluid averaging point within 2h");
    }
  }
  g->gidx.assign(gidx32.begin(), gidx32.end());
  g->ap.assign(ap32.begin(), ap32.end());
  // staggered-cell fractions for the momentum step: the same counting in cells shifted by h/2 along
  // each axis (the cell fractions are on the host already, so their device buffer is reused)
  if (params->flags & CH_IB_FLAG_NAVIER_STOKES) {
    g->face_alpha.resize((size_t)d * N);
    for (int a = 0; a < d && e == hipSuccess; ++a) {
      GeomArgs B = A;
      B.off[a] = 0.5 * tmp.h;
      int64_t nc = 0;
      hipLaunchKernelGGL(k_gd_classify, dim3(nb), dim3(kGeomThreads), 0, s, B, alpha, (unsigned char *)nullptr, cutf);
      hipLaunchKernelGGL(k_gd_list<1>, dim3(nb), dim3(kGeomThreads), 0, s, B, (const unsigned char *)cutf, bcount,
                         (const int *)nullptr, (int *)nullptr, bad);
      e = hipGetLastError();
      if (e == hipSuccess) e = offsets(&nc);
      if (e == hipSuccess) {
        hipLaunchKernelGGL(k_gd_list<1>, dim3(nb), dim3(kGeomThreads), 0, s, B, (const unsigned char *)cutf, bcount,
                           (const int *)boff, cutlist, bad);
        if (nc)
          hipLaunchKernelGGL(k_gd_subgrid, dim3((unsigned)((nc + 3) / 4)), dim3(kGeomThreads), 0, s, B,
                             (const int *)cutlist, nc, alpha);
        e = hipGetLastError();
      }
      if (e == hipSuccess)
        e = hipMemcpyAsync(g->face_alpha.data() + (size_t)a * N, alpha, (size_t)N * 8, hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    if (e != hipSuccess) {
      delete g;
      return hip_error(e, "device geometry (staggered fractions)");
    }
  }
  *out = g;
  return CH_IB_OK;
}
