// Momentum step of the Navier-Stokes coupling on the staggered grid (sections 2, 3.2, 4.2.3, 4.3 and 4.4):
// explicit Adams-Bashforth prediction (Eq. PredictionExp), volume penalisation with the
// staggered-cell fluid fractions (Eq. Penalization2), the slip / no-penetration velocity ghost
// fill, the variable-density pressure equation (Eq. PressurePoisson, rho0 = min(rho1, rho2),
// p^ = 2p^n - p^(n-1)) solved by the spectral pipeline, and the correction (Eq. correction).
//
// Non-dimensional momentum equation (lengths in domain units, density and viscosity relative to
// the reference fluid of Re):
//   du/dt + div(u u) = (1/rho) [-grad p + (1/Re) div(mu (grad u + grad u^T)) + kappa phi grad C] + g
// with rho = ((C+1) rho2 - (C-1) rho1)/2, mu likewise, phi = C^3 - C - Cn^2 lap C and
// kappa = 3/(2 sqrt2 Re Ca Cn), the factor that gives the planar profile the surface tension of
// the wall condition.
//
// Face field a holds u_a on the face between cell c and c + e_a.  Periodic axes wrap; the bounded
// (last) axis has no-slip box walls: the normal velocity on both walls is zero (the top wall face
// is stored and kept at zero), the tangential velocity has the image -u across a wall, no
// pressure gradient acts through a wall, and cell scalars are reflected.
//
// Every kernel takes one thread per cell and handles the d faces c + e_a/2 of that cell; the
// face and cell neighbours come from global memory through the caches.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace chib {

namespace {

constexpr int kNsThreads = 256;   // the tiled walk below assumes 2^8 threads

struct NsGrid {
  int n[3];       // cells per axis (1 beyond d); powers of two
  int ln[3];      // log2 of n
  int d;
  int64_t N;
};

template <typename T>
struct NsCoef {
  T inv_h, dt, inv_re, kappa;
  T rho1, rho2, mu1, mu2;
  T g[3];
  T rho0, inv_rho0, rho0_dt;
};

template <typename T>
struct FaceSet {
  T *f[3];
};

template <typename T>
__device__ __forceinline__ T rho_of(const NsCoef<T> &k, T C) {
  return T(0.5) * ((C + T(1)) * k.rho2 - (C - T(1)) * k.rho1);
}

template <typename T>
__device__ __forceinline__ T mu_of(const NsCoef<T> &k, T C) {
  return T(0.5) * ((C + T(1)) * k.mu2 - (C - T(1)) * k.mu1);
}

__device__ __forceinline__ void coords(const NsGrid &g, int64_t c, int *q) {
  q[0] = (int)(c & (g.n[0] - 1));
  q[1] = (int)((c >> g.ln[0]) & (g.n[1] - 1));
  q[2] = (int)(c >> (g.ln[0] + g.ln[1]));
}

// Cells a launch visits: one per thread (flat), or, on 3D grids, a tile of 2^ltx x 2^lty columns
// per workgroup marched through zc consecutive planes, so that the planes above and below a cell
// are still in the caches when its stencil reads them.
struct NsWalk {
  int flat;
  int ltx, lty;         // tile: 2^ltx cells along x by 2^lty along y (ltx + lty = log2 of the workgroup)
  int lbx, lby;         // log2 of the tile counts along x and y
  int zc;               // planes per workgroup
};

template <typename F>
__device__ __forceinline__ void for_each_cell(const NsWalk &wk, const NsGrid &g, F f) {
  if (wk.flat) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < g.N) f(c);
    return;
  }
  const int b = (int)blockIdx.x;
  const int bx = b & ((1 << wk.lbx) - 1);
  const int by = (b >> wk.lbx) & ((1 << wk.lby) - 1);
  const int bz = b >> (wk.lbx + wk.lby);
  const int i = (bx << wk.ltx) + (int)(threadIdx.x & ((1u << wk.ltx) - 1));
  const int j = (by << wk.lty) + (int)(threadIdx.x >> wk.ltx);
  const int64_t row = (int64_t)i + ((int64_t)j << g.ln[0]);
  for (int k = bz * wk.zc; k < (bz + 1) * wk.zc; ++k) f(row + ((int64_t)k << (g.ln[0] + g.ln[1])));
}

// Prediction (Eq. PredictionExp) and penalisation (Eq. Penalization2) on the d faces of each cell:
//   u** = alpha_f (u^n + dt (-(3/2 N^n - 1/2 N^(n-1)) + ((1/Re) V + kappa phi_f dC/dx_a) / rho_f + g_a))
// N: conservative central convective term; V: viscous term with mu from C^(n+1); phi = W.
// Writes N^n over N^(n-1).  first: forward Euler for the convective term.
// Neighbour offsets of a cell: op[b] / om[b] move one cell up / down along axis b (periodic axes
// wrap, the bounded axis steps a plane; validity along it is checked by the caller).
template <int D>
__device__ __forceinline__ void nbr_offsets(const NsGrid &g, const int *q, int *op, int *om) {
#pragma unroll
  for (int b = 0; b < D; ++b) {
    const int sh = b == 0 ? 0 : (b == 1 ? g.ln[0] : g.ln[0] + g.ln[1]);
    if (b < D - 1) {
      op[b] = (((q[b] + 1) & (g.n[b] - 1)) - q[b]) << sh;
      om[b] = (((q[b] - 1) & (g.n[b] - 1)) - q[b]) << sh;
    } else {
      op[b] = 1 << sh;
      om[b] = -(1 << sh);
    }
  }
}

template <typename T, int D>
__device__ __forceinline__ void ns_predict_cell(FaceSet<T> U, const T *__restrict__ C,
                                                const T *__restrict__ phi, FaceSet<T> Nh,
                                                FaceSet<T> Af, FaceSet<T> Us, NsGrid g, NsCoef<T> k,
                                                int first, int64_t c64) {
  constexpr int d = D, bw = D - 1;
  const int c = (int)c64;
  const int nw = g.n[bw];
  int q[3];
  coords(g, c64, q);
  const int w = q[bw];
  int op[3], om[3];
  nbr_offsets<D>(g, q, op, om);
  auto step = [&](int ax, int sgn) { return sgn > 0 ? op[ax] : om[ax]; };
  // face value of component a at index i whose bounded coordinate is wq (zero outside the box and
  // on the top wall face); the load always happens, from the cell itself when i is not valid, so
  // that every load of the stencil can be in flight at once
  auto fv = [&](const T *f, int a, int i, int wq) -> T {
    const bool ok = wq >= 0 && wq < nw && !(a == bw && wq == nw - 1);
    const T v = f[ok ? i : c];
    return ok ? v : T(0);
  };
  auto F1 = [&](const T *f, int a, int ax, int sgn) -> T {
    return fv(f, a, c + step(ax, sgn), w + (ax == bw ? sgn : 0));
  };
  auto F2 = [&](const T *f, int a, int ax1, int s1, int ax2, int s2) -> T {
    return fv(f, a, c + step(ax1, s1) + step(ax2, s2), w + (ax1 == bw ? s1 : 0) + (ax2 == bw ? s2 : 0));
  };
  // cell scalar one cell away (reflected on the bounded axis)
  auto roff = [&](int ax, int sgn) {
    if (ax == bw && (w + sgn < 0 || w + sgn >= nw)) return 0;
    return step(ax, sgn);
  };
#pragma unroll
  for (int a = 0; a < d; ++a) {
    if (a == bw && w == nw - 1) {   // top wall face: no penetration
      Us.f[a][c] = T(0);
      Nh.f[a][c] = T(0);
      continue;
    }
    const T *ua = U.f[a];
    const T u0 = ua[c];
    // convective term
    T N = T(0);
#pragma unroll
    for (int b = 0; b < d; ++b) {
      if (b == a) {
        const T uc0 = T(0.5) * (F1(ua, a, a, -1) + u0);
        const T uc1 = T(0.5) * (u0 + F1(ua, a, a, 1));
        N += (uc1 * uc1 - uc0 * uc0) * k.inv_h;
      } else {
        const T *ub = U.f[b];
        const T e1 = T(0.5) * (u0 + F1(ua, a, b, 1)) * T(0.5) * (fv(ub, b, c, w) + F1(ub, b, a, 1));
        const T e0 = T(0.5) * (F1(ua, a, b, -1) + u0) * T(0.5) * (F1(ub, b, b, -1) + F2(ub, b, b, -1, a, 1));
        const T E1 = (b == bw && w == nw - 1) ? T(0) : e1;
        const T E0 = (b == bw && w == 0) ? T(0) : e0;
        N += (E1 - E0) * k.inv_h;
      }
    }
    // viscous term
    const T mu_c = mu_of(k, C[c]);
    const T mu_a = mu_of(k, C[c + roff(a, 1)]);
    const T tn0 = T(2) * mu_c * (u0 - F1(ua, a, a, -1)) * k.inv_h;
    const T tn1 = T(2) * mu_a * (F1(ua, a, a, 1) - u0) * k.inv_h;
    T V = (tn1 - tn0) * k.inv_h;
#pragma unroll
    for (int b = 0; b < d; ++b) {
      if (b == a) continue;
      const T *ub = U.f[b];
      // edge c + e_a/2 + e_b/2
      const T me1 = T(0.25) * (mu_c + mu_a + mu_of(k, C[c + roff(b, 1)]) + mu_of(k, C[c + roff(a, 1) + roff(b, 1)]));
      const T ub_up = (b == bw && w == nw - 1) ? -u0 : F1(ua, a, b, 1);
      const T tau1 = me1 * ((ub_up - u0) * k.inv_h + (F1(ub, b, a, 1) - fv(ub, b, c, w)) * k.inv_h);
      // edge c + e_a/2 - e_b/2; on the bottom wall the no-slip image and u_b = 0 along the wall
      const T mu_b = mu_of(k, C[c + roff(b, -1)]);
      const T mu_ab = mu_of(k, C[c + roff(b, -1) + roff(a, 1)]);
      const T me0 = T(0.25) * (mu_b + mu_ab + mu_c + mu_a);
      const T ua_m = F1(ua, a, b, -1);
      const T tin = me0 * ((u0 - ua_m) * k.inv_h + (F2(ub, b, b, -1, a, 1) - F1(ub, b, b, -1)) * k.inv_h);
      const T twall = T(0.5) * (mu_c + mu_a) * (u0 - (-u0)) * k.inv_h;
      const T tau0 = (b == bw && w == 0) ? twall : tin;
      V += (tau1 - tau0) * k.inv_h;
    }
    // capillary force and density on the face
    const int ia = c + roff(a, 1);
    const T C0 = C[c], C1 = C[ia];
    const T F = k.kappa * (T(0.5) * (phi[c] + phi[ia])) * (C1 - C0) * k.inv_h;
    const T rf = T(0.5) * (rho_of(k, C0) + rho_of(k, C1));
    const T Np = first ? N : Nh.f[a][c];
    const T us = u0 + k.dt * (-(T(1.5) * N - T(0.5) * Np) + (V * k.inv_re + F) / rf + k.g[a]);
    Us.f[a][c] = Af.f[a][c] * us;
    Nh.f[a][c] = N;
  }
}

template <typename T, int D>
__global__ __launch_bounds__(kNsThreads) void k_ns_predict(FaceSet<T> U, const T *__restrict__ C,
                                                           const T *__restrict__ phi, FaceSet<T> Nh,
                                                           FaceSet<T> Af, FaceSet<T> Us, NsGrid g, NsCoef<T> k,
                                                           int first, NsWalk wk) {
  for_each_cell(wk, g, [&](int64_t c) { ns_predict_cell<T, D>(U, C, phi, Nh, Af, Us, g, k, first, c); });
}

// 3D prediction with each edge formed once.  The convective flux E_ab = (u_a mean along b)(u_b mean
// along a) and the shear stress tau_ab = mu_e (du_a/dx_b + du_b/dx_a) of an edge are symmetric in a and
// b and are used by four faces; the per-cell kernel forms them four times.  Here a workgroup owns a
// 64 x 8 tile of columns and marches it through zc planes: per plane it forms the xy, xz and yz edges
// of the tile and of the halo column and row below it into LDS, every face takes its two edge
// differences from there, and the xz and yz edges of the plane below come from registers.  Same
// formulas and wall rules as ns_predict_cell (the four-cell mean viscosity of an edge is summed in the
// order of its lower-axis face, so the other face's value may differ in the last bit).
constexpr int kEx = 64, kEy = 8, kEhx = kEx + 1, kEhy = kEy + 1;
constexpr int kEThreads = kEx * kEy;   // one thread per column of the tile

// E and tau of the xy (0), xz (1) and yz (2) edges at cell (qx, qy, qz): edge o lies at the cell
// centre plus half a cell along each of its two axes.
template <typename T>
__device__ __forceinline__ void ns_edges(const FaceSet<T> &U, const T *__restrict__ C, const NsGrid &g,
                                         const NsCoef<T> &k, int qx, int qy, int qz, T *E, T *Tau) {
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
  const int cq = qx + (qy << g.ln[0]) + (qz << (g.ln[0] + g.ln[1]));
  const int ox = ((qx + 1) & (nx - 1)) - qx;
  const int oy = (((qy + 1) & (ny - 1)) - qy) << g.ln[0];
  const bool top = qz == nz - 1;
  const int oz = top ? 0 : (1 << (g.ln[0] + g.ln[1]));   // (unused at the top, kept in the box)
  const T ux0 = U.f[0][cq], uy0 = U.f[1][cq];
  const T uzr = U.f[2][cq];
  const T uz0 = top ? T(0) : uzr;
  const T ux_y = U.f[0][cq + oy], uy_x = U.f[1][cq + ox];
  const T ux_z = U.f[0][cq + oz], uy_z = U.f[1][cq + oz];
  const T uzx = U.f[2][cq + ox], uzy = U.f[2][cq + oy];
  const T uz_x = top ? T(0) : uzx, uz_y = top ? T(0) : uzy;
  const T mu_c = mu_of(k, C[cq]), mu_x = mu_of(k, C[cq + ox]), mu_y = mu_of(k, C[cq + oy]);
  const T mu_xy = mu_of(k, C[cq + ox + oy]);
  const T mu_z = mu_of(k, C[cq + oz]), mu_xz = mu_of(k, C[cq + ox + oz]), mu_yz = mu_of(k, C[cq + oy + oz]);
  // xy
  E[0] = T(0.5) * (ux0 + ux_y) * T(0.5) * (uy0 + uy_x);
  Tau[0] = T(0.25) * (mu_c + mu_x + mu_y + mu_xy) * ((ux_y - ux0) * k.inv_h + (uy_x - uy0) * k.inv_h);
  // xz and yz: on the top wall E = 0, the tangential velocity has the image -u, u_z = 0 along the wall
  const T e1 = T(0.5) * (ux0 + ux_z) * T(0.5) * (uz0 + uz_x);
  const T e2 = T(0.5) * (uy0 + uy_z) * T(0.5) * (uz0 + uz_y);
  E[1] = top ? T(0) : e1;
  E[2] = top ? T(0) : e2;
  const T ux_up = top ? -ux0 : ux_z, uy_up = top ? -uy0 : uy_z;
  Tau[1] = T(0.25) * (mu_c + mu_x + mu_z + mu_xz) * ((ux_up - ux0) * k.inv_h + (uz_x - uz0) * k.inv_h);
  Tau[2] = T(0.25) * (mu_c + mu_y + mu_z + mu_yz) * ((uy_up - uy0) * k.inv_h + (uz_y - uz0) * k.inv_h);
}

template <typename T>
__global__ __launch_bounds__(kEThreads) void k_ns_predict_edges(FaceSet<T> U, const T *__restrict__ C,
                                                                const T *__restrict__ phi, FaceSet<T> Nh,
                                                                FaceSet<T> Af, FaceSet<T> Us, NsGrid g,
                                                                NsCoef<T> k, int first, int zc) {
  __shared__ T sE[3][kEhy][kEhx];
  __shared__ T sT[3][kEhy][kEhx];
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
  const int tiles_x = nx / kEx, tiles_y = ny / kEy;
  int bidx = (int)blockIdx.x;
  const int bx = bidx % tiles_x;
  bidx /= tiles_x;
  const int by = bidx % tiles_y;
  const int bz = bidx / tiles_y;
  const int x0 = bx * kEx, y0 = by * kEy, z0 = bz * zc;
  const int tid = (int)threadIdx.x;
  const int tx = tid & (kEx - 1), ty = tid >> 6;
  const int x = x0 + tx, y = y0 + ty;
  const int X = tx + 1, Y = ty + 1;
  const int plane_sh = g.ln[0] + g.ln[1];
  const int oxp = ((x + 1) & (nx - 1)) - x, oxm = ((x - 1) & (nx - 1)) - x;
  const int oyp = (((y + 1) & (ny - 1)) - y) << g.ln[0], oym = (((y - 1) & (ny - 1)) - y) << g.ln[0];
  // xz and yz edges of the plane below this thread's cell
  T Ezx, Tzx, Ezy, Tzy;
  if (z0 == 0) {   // the bottom wall: no flux, shear from the no-slip image
    const int c = x + (y << g.ln[0]);
    const T mu_c = mu_of(k, C[c]);
    const T ux = U.f[0][c], uy = U.f[1][c];
    Ezx = T(0);
    Ezy = T(0);
    Tzx = T(0.5) * (mu_c + mu_of(k, C[c + oxp])) * (ux - (-ux)) * k.inv_h;
    Tzy = T(0.5) * (mu_c + mu_of(k, C[c + oyp])) * (uy - (-uy)) * k.inv_h;
  } else {
    T E[3], Tau[3];
    ns_edges(U, C, g, k, x, y, z0 - 1, E, Tau);
    Ezx = E[1];
    Tzx = Tau[1];
    Ezy = E[2];
    Tzy = Tau[2];
  }
  for (int kz = z0; kz < z0 + zc; ++kz) {
    for (int e = tid; e < kEhx * kEhy; e += kEThreads) {
      const int yy = e / kEhx, xx = e - yy * kEhx;
      T E[3], Tau[3];
      ns_edges(U, C, g, k, (x0 - 1 + xx) & (nx - 1), (y0 - 1 + yy) & (ny - 1), kz, E, Tau);
#pragma unroll
      for (int o = 0; o < 3; ++o) {
        sE[o][yy][xx] = E[o];
        sT[o][yy][xx] = Tau[o];
      }
    }
    __syncthreads();
    const int c = x + (y << g.ln[0]) + (kz << plane_sh);
    const int ozp = kz < nz - 1 ? (1 << plane_sh) : 0, ozm = kz > 0 ? -(1 << plane_sh) : 0;
    const int op[3] = {oxp, oyp, ozp}, om[3] = {oxm, oym, ozm};
    const T C0 = C[c];
    const T mu_c = mu_of(k, C0);
    const T phc = phi[c];
    const T rc = rho_of(k, C0);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (a == 2 && kz == nz - 1) {   // top wall face
        Us.f[a][c] = T(0);
        Nh.f[a][c] = T(0);
        continue;
      }
      const T *ua = U.f[a];
      const T u0 = ua[c];
      const T umr = ua[c + om[a]], upr = ua[c + op[a]];
      // the face below the bottom wall and the top wall face are zero
      const T um = (a == 2 && kz == 0) ? T(0) : umr;
      const T up = (a == 2 && kz + 1 == nz - 1) ? T(0) : upr;
      T N = T(0), V;
      const T uc0 = T(0.5) * (um + u0), uc1 = T(0.5) * (u0 + up);
      const T Ca = C[c + op[a]];
      const T mu_a = mu_of(k, Ca);
      const T tn0 = T(2) * mu_c * (u0 - um) * k.inv_h;
      const T tn1 = T(2) * mu_a * (up - u0) * k.inv_h;
      V = (tn1 - tn0) * k.inv_h;
      if (a == 0) {
        N += (uc1 * uc1 - uc0 * uc0) * k.inv_h;
        N += (sE[0][Y][X] - sE[0][Y - 1][X]) * k.inv_h;
        N += (sE[1][Y][X] - Ezx) * k.inv_h;
        V += (sT[0][Y][X] - sT[0][Y - 1][X]) * k.inv_h;
        V += (sT[1][Y][X] - Tzx) * k.inv_h;
      } else if (a == 1) {
        N += (sE[0][Y][X] - sE[0][Y][X - 1]) * k.inv_h;
        N += (uc1 * uc1 - uc0 * uc0) * k.inv_h;
        N += (sE[2][Y][X] - Ezy) * k.inv_h;
        V += (sT[0][Y][X] - sT[0][Y][X - 1]) * k.inv_h;
        V += (sT[2][Y][X] - Tzy) * k.inv_h;
      } else {
        N += (sE[1][Y][X] - sE[1][Y][X - 1]) * k.inv_h;
        N += (sE[2][Y][X] - sE[2][Y - 1][X]) * k.inv_h;
        N += (uc1 * uc1 - uc0 * uc0) * k.inv_h;
        V += (sT[1][Y][X] - sT[1][Y][X - 1]) * k.inv_h;
        V += (sT[2][Y][X] - sT[2][Y - 1][X]) * k.inv_h;
      }
      const T F = k.kappa * (T(0.5) * (phc + phi[c + op[a]])) * (Ca - C0) * k.inv_h;
      const T rf = T(0.5) * (rc + rho_of(k, Ca));
      const T Np = first ? N : Nh.f[a][c];
      const T us = u0 + k.dt * (-(T(1.5) * N - T(0.5) * Np) + (V * k.inv_re + F) / rf + k.g[a]);
      Us.f[a][c] = Af.f[a][c] * us;
      Nh.f[a][c] = N;
    }
    Ezx = sE[1][Y][X];
    Tzx = sT[1][Y][X];
    Ezy = sE[2][Y][X];
    Tzy = sT[2][Y][X];
    __syncthreads();   // the next plane's edges overwrite the buffers
  }
}

// Right-hand side of Eq. PressurePoisson at the cell centres:
//   div((1 - rho0/rho_f) grad p^) + (rho0/dt) div u**,  p^ = 2 P0 - P1; no flux through the walls.
template <typename T, int D>
__device__ __forceinline__ void ns_prhs_cell(FaceSet<T> Us, const T *__restrict__ C,
                                             const T *__restrict__ P0, const T *__restrict__ P1,
                                             T *__restrict__ R, NsGrid g, NsCoef<T> k, int64_t c64) {
  constexpr int d = D, bw = D - 1;
  const int c = (int)c64;
  const int nw = g.n[bw];
  int q[3];
  coords(g, c64, q);
  const int w = q[bw];
  int op[3], om[3];
  nbr_offsets<D>(g, q, op, om);
  auto ph = [&](int i) { return T(2) * P0[i] - P1[i]; };
  const T phc = ph(c);
  const T rc = rho_of(k, C[c]);
  T acc1 = T(0), acc2 = T(0);
#pragma unroll
  for (int a = 0; a < d; ++a) {
    // flux (1 - rho0/rho_f) dp^/dx_a through the upper and the lower face of the cell along a
    // (every load happens, from the cell itself where a face lies on a box wall)
    const bool top = a == bw && w == nw - 1, bottom = a == bw && w == 0;
    const int i1 = c + (top ? 0 : op[a]);
    const int i0 = c + (bottom ? 0 : om[a]);
    const T rf1 = T(0.5) * (rc + rho_of(k, C[i1]));
    const T rf0 = T(0.5) * (rho_of(k, C[i0]) + rc);
    const T fu1 = (T(1) - k.rho0 / rf1) * ((ph(i1) - phc) * k.inv_h);
    const T fl0 = (T(1) - k.rho0 / rf0) * ((phc - ph(i0)) * k.inv_h);
    const T uu1 = Us.f[a][c], ul0 = Us.f[a][i0];
    const T fu = top ? T(0) : fu1, uu = top ? T(0) : uu1;
    const T fl = bottom ? T(0) : fl0, ul = bottom ? T(0) : ul0;
    acc1 += fu - fl;
    acc2 += uu - ul;
  }
  R[c] = acc1 * k.inv_h + k.rho0_dt * (acc2 * k.inv_h);
}

template <typename T, int D>
__global__ __launch_bounds__(kNsThreads) void k_ns_pressure_rhs(FaceSet<T> Us, const T *__restrict__ C,
                                                                const T *__restrict__ P0, const T *__restrict__ P1,
                                                                T *__restrict__ R, NsGrid g, NsCoef<T> k, NsWalk wk) {
  for_each_cell(wk, g, [&](int64_t c) { ns_prhs_cell<T, D>(Us, C, P0, P1, R, g, k, c); });
}

// Correction (Eq. correction): u^(n+1) = u** - dt (grad p^(n+1) / rho0 + (1/rho_f - 1/rho0) grad p^)
// on every face but the top wall face; also writes the advecting velocity 2u^(n+1) - u^n of the
// next order-parameter step (Ut, may be absent).
template <typename T, int D>
__device__ __forceinline__ void ns_correct_cell(FaceSet<T> U, FaceSet<T> Ut, FaceSet<T> Us,
                                                const T *__restrict__ C, const T *__restrict__ Pn,
                                                const T *__restrict__ P0, const T *__restrict__ P1,
                                                NsGrid g, NsCoef<T> k, int with_ut, int64_t c64) {
  constexpr int d = D, bw = D - 1;
  const int c = (int)c64;
  const int nw = g.n[bw];
  int q[3];
  coords(g, c64, q);
  const int w = q[bw];
  int op[3], om[3];
  nbr_offsets<D>(g, q, op, om);
  const T phc = T(2) * P0[c] - P1[c];
  const T rc = rho_of(k, C[c]);
  const T pc = Pn[c];
#pragma unroll
  for (int a = 0; a < d; ++a) {
    const bool top = a == bw && w == nw - 1;
    const int ca = c + (top ? 0 : op[a]);
    const T Gn = (Pn[ca] - pc) * k.inv_h;
    const T Gh = ((T(2) * P0[ca] - P1[ca]) - phc) * k.inv_h;
    const T rf = T(0.5) * (rc + rho_of(k, C[ca]));
    const T u1 = Us.f[a][c] - k.dt * (Gn * k.inv_rho0 + (T(1) / rf - k.inv_rho0) * Gh);
    const T un = top ? T(0) : u1;
    const T uo = U.f[a][c];
    U.f[a][c] = un;
    if (with_ut) Ut.f[a][c] = T(2) * un - uo;
  }
}

template <typename T, int D>
__global__ __launch_bounds__(kNsThreads) void k_ns_correct(FaceSet<T> U, FaceSet<T> Ut, FaceSet<T> Us,
                                                           const T *__restrict__ C, const T *__restrict__ Pn,
                                                           const T *__restrict__ P0, const T *__restrict__ P1,
                                                           NsGrid g, NsCoef<T> k, int with_ut, NsWalk wk) {
  for_each_cell(wk, g, [&](int64_t c) { ns_correct_cell<T, D>(U, Ut, Us, C, Pn, P0, P1, g, k, with_ut, c); });
}

// 3D z-marching forms of the pressure rhs and the correction (tiled walk only): a thread carries its
// column's values of the planes below and above from one plane to the next instead of fetching them
// again; x and y neighbours come through the caches.  Same expressions as the per-cell forms.
struct ZCol {
  int c0;          // linear index of the column's first plane
  int oxp, oxm, oyp, oym;
  int k0, k1;      // planes [k0, k1)
  int psh;         // log2 of the plane size
};

__device__ __forceinline__ ZCol zcol(const NsWalk &wk, const NsGrid &g, int b) {
  ZCol z;
  const int bx = b & ((1 << wk.lbx) - 1);
  const int by = (b >> wk.lbx) & ((1 << wk.lby) - 1);
  const int bz = b >> (wk.lbx + wk.lby);
  const int i = (bx << wk.ltx) + (int)(threadIdx.x & ((1u << wk.ltx) - 1));
  const int j = (by << wk.lty) + (int)(threadIdx.x >> wk.ltx);
  z.psh = g.ln[0] + g.ln[1];
  z.k0 = bz * wk.zc;
  z.k1 = z.k0 + wk.zc;
  z.c0 = i + (j << g.ln[0]) + (z.k0 << z.psh);
  z.oxp = ((i + 1) & (g.n[0] - 1)) - i;
  z.oxm = ((i - 1) & (g.n[0] - 1)) - i;
  z.oyp = (((j + 1) & (g.n[1] - 1)) - j) << g.ln[0];
  z.oym = (((j - 1) & (g.n[1] - 1)) - j) << g.ln[0];
  return z;
}

template <typename T>
__global__ __launch_bounds__(kNsThreads) void k_ns_pressure_rhs_zm(FaceSet<T> Us, const T *__restrict__ C,
                                                                   const T *__restrict__ P0,
                                                                   const T *__restrict__ P1, T *__restrict__ R,
                                                                   NsGrid g, NsCoef<T> k, NsWalk wk) {
  // XCD-aware tile order: the y-neighbour tiles whose rows this pass re-reads run on the same L2
  // (0.298 -> 0.280 ms at 256^3; the correction and the prediction ran slower with it)
  const ZCol z = zcol(wk, g, xcd_tile(blockIdx.x, gridDim.x));
  const int nz = g.n[2], pl = 1 << z.psh;
  auto ph = [&](int i) { return T(2) * P0[i] - P1[i]; };
  int c = z.c0;
  const int cb = z.k0 > 0 ? c - pl : c;     // the plane below (the first plane itself at the bottom)
  T ph_m = ph(cb), r_m = rho_of(k, C[cb]), uz_m = Us.f[2][cb];
  T phc = ph(c), rc = rho_of(k, C[c]);
  for (int kz = z.k0; kz < z.k1; ++kz, c += pl) {
    const bool top = kz == nz - 1, bottom = kz == 0;
    const int cp = top ? c : c + pl;
    const T ph_p = ph(cp), r_p = rho_of(k, C[cp]);
    T acc1 = T(0), acc2 = T(0);
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const int i1 = c + (a == 0 ? z.oxp : z.oyp), i0 = c + (a == 0 ? z.oxm : z.oym);
      const T rf1 = T(0.5) * (rc + rho_of(k, C[i1]));
      const T rf0 = T(0.5) * (rho_of(k, C[i0]) + rc);
      const T fu = (T(1) - k.rho0 / rf1) * ((ph(i1) - phc) * k.inv_h);
      const T fl = (T(1) - k.rho0 / rf0) * ((phc - ph(i0)) * k.inv_h);
      acc1 += fu - fl;
      acc2 += Us.f[a][c] - Us.f[a][i0];
    }
    const T uzc = Us.f[2][c];
    const T fu1 = (T(1) - k.rho0 / (T(0.5) * (rc + r_p))) * ((ph_p - phc) * k.inv_h);
    const T fl0 = (T(1) - k.rho0 / (T(0.5) * (r_m + rc))) * ((phc - ph_m) * k.inv_h);
    const T fu = top ? T(0) : fu1, uu = top ? T(0) : uzc;
    const T fl = bottom ? T(0) : fl0, ul = bottom ? T(0) : uz_m;
    acc1 += fu - fl;
    acc2 += uu - ul;
    R[c] = acc1 * k.inv_h + k.rho0_dt * (acc2 * k.inv_h);
    ph_m = phc;
    r_m = rc;
    uz_m = uzc;
    phc = ph_p;
    rc = r_p;
  }
}

template <typename T>
__global__ __launch_bounds__(kNsThreads) void k_ns_correct_zm(FaceSet<T> U, FaceSet<T> Ut, FaceSet<T> Us,
                                                              const T *__restrict__ C, const T *__restrict__ Pn,
                                                              const T *__restrict__ P0, const T *__restrict__ P1,
                                                              NsGrid g, NsCoef<T> k, int with_ut, NsWalk wk) {
  const ZCol z = zcol(wk, g, (int)blockIdx.x);
  const int nz = g.n[2], pl = 1 << z.psh;
  int c = z.c0;
  T pc = Pn[c], phc = T(2) * P0[c] - P1[c], rc = rho_of(k, C[c]);
  for (int kz = z.k0; kz < z.k1; ++kz, c += pl) {
    const bool top = kz == nz - 1;
    const int cp = top ? c : c + pl;
    const T p_p = Pn[cp], ph_p = T(2) * P0[cp] - P1[cp], r_p = rho_of(k, C[cp]);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      T Gn, Gh, rf;
      if (a < 2) {
        const int ca = c + (a == 0 ? z.oxp : z.oyp);
        Gn = (Pn[ca] - pc) * k.inv_h;
        Gh = ((T(2) * P0[ca] - P1[ca]) - phc) * k.inv_h;
        rf = T(0.5) * (rc + rho_of(k, C[ca]));
      } else {
        Gn = (p_p - pc) * k.inv_h;
        Gh = (ph_p - phc) * k.inv_h;
        rf = T(0.5) * (rc + r_p);
      }
      const T u1 = Us.f[a][c] - k.dt * (Gn * k.inv_rho0 + (T(1) / rf - k.inv_rho0) * Gh);
      const T un = (a == 2 && top) ? T(0) : u1;
      const T uo = U.f[a][c];
      U.f[a][c] = un;
      if (with_ut) Ut.f[a][c] = T(2) * un - uo;
    }
    pc = p_p;
    phc = ph_p;
    rc = r_p;
  }
}

template <typename T>
NsCoef<T> ns_coef(const Plan &p) {
  NsCoef<T> k;
  k.inv_h = (T)(1.0 / p.h);
  k.dt = (T)p.dt;
  k.inv_re = (T)(1.0 / p.Re);
  k.kappa = (T)(3.0 / (2.0 * 1.4142135623730951 * p.Re * p.Ca * p.Cn));
  k.rho1 = (T)p.rho1;
  k.rho2 = (T)p.rho2;
  k.mu1 = (T)p.mu1;
  k.mu2 = (T)p.mu2;
  for (int a = 0; a < 3; ++a) k.g[a] = (T)p.g[a];
  const double rho0 = p.rho1 < p.rho2 ? p.rho1 : p.rho2;
  k.rho0 = (T)rho0;
  k.inv_rho0 = (T)(1.0 / rho0);
  k.rho0_dt = (T)(rho0 / p.dt);
  return k;
}

NsGrid ns_grid(const Plan &p) {
  NsGrid g;
  g.n[0] = p.n[0];
  g.n[1] = p.n[1];
  g.n[2] = p.d == 3 ? p.n[2] : 1;
  g.ln[0] = p.logn[0];
  g.ln[1] = p.logn[1];
  g.ln[2] = p.d == 3 ? p.logn[2] : 0;
  g.d = p.d;
  g.N = p.N;
  return g;
}

// 3D: tiles of 64 x 4 columns (fewer along x on narrower grids) marched through 16 planes; 2D: flat.
NsWalk ns_walk(const Plan &p, unsigned *nb) {
  NsWalk w{};
  w.flat = 1;
  *nb = (unsigned)((p.N + kNsThreads - 1) / kNsThreads);
  if (p.d != 3) return w;
  const int ltx = p.logn[0] < 6 ? p.logn[0] : 6;
  const int lty = 8 - ltx;   // 256 threads
  if (lty > p.logn[1]) return w;
  w.flat = 0;
  w.ltx = ltx;
  w.lty = lty;
  w.lbx = p.logn[0] - ltx;
  w.lby = p.logn[1] - lty;
  w.zc = p.n[2] < 16 ? p.n[2] : 16;
  *nb = (unsigned)((1u << (w.lbx + w.lby)) * (unsigned)(p.n[2] / w.zc));
  return w;
}

template <typename T>
FaceSet<T> faces(void *const *f, int d) {
  FaceSet<T> s;
  for (int a = 0; a < 3; ++a) s.f[a] = (T *)(a < d ? f[a] : f[0]);
  return s;
}

}  // namespace

template <typename T>
hipError_t enqueue_momentum(const Plan &p, int cur, int first, KernelTimer *tm) {
  hipError_t e = hipSuccess;
  auto mark = [&](const char *name) {
    if (tm && e == hipSuccess) e = tm->mark(name, p.stream);
  };
  if (!p.ns || !p.P[0] || !p.P[1]) return hipErrorInvalidValue;
  const NsGrid g = ns_grid(p);
  const NsCoef<T> k = ns_coef<T>(p);
  unsigned nb = 0;
  const NsWalk wk = ns_walk(p, &nb);
  const T *C = (const T *)p.C[cur];
  const FaceSet<T> U = faces<T>(p.F, p.d), Us = faces<T>(p.Us, p.d), Nh = faces<T>(p.Nh, p.d);
  const FaceSet<T> Af = faces<T>(p.Af, p.d);
  const bool with_ut = p.Ut[0] != nullptr;
  const FaceSet<T> Ut = with_ut ? faces<T>(p.Ut, p.d) : U;
  mark("ns_phi");
  if (e == hipSuccess) e = enqueue_phi<T>(p, cur, p.W);
  mark("ns_predict");
  if (e == hipSuccess) {
    if (p.d == 2)
      hipLaunchKernelGGL((k_ns_predict<T, 2>), dim3(nb), dim3(kNsThreads), 0, p.stream, U, C, (const T *)p.W, Nh, Af,
                         Us, g, k, first, wk);
    else if (p.n[0] % kEx == 0 && p.n[1] % kEy == 0) {
      const int zc = p.n[2] < 16 ? p.n[2] : 16;
      const unsigned nbe = (unsigned)((p.n[0] / kEx) * (p.n[1] / kEy) * (p.n[2] / zc));
      hipLaunchKernelGGL((k_ns_predict_edges<T>), dim3(nbe), dim3(kEThreads), 0, p.stream, U, C, (const T *)p.W, Nh,
                         Af, Us, g, k, first, zc);
    } else
      hipLaunchKernelGGL((k_ns_predict<T, 3>), dim3(nb), dim3(kNsThreads), 0, p.stream, U, C, (const T *)p.W, Nh, Af,
                         Us, g, k, first, wk);
    e = hipGetLastError();
  }
  mark("ns_vel_fill");
  if (e == hipSuccess && p.G) {
    Plan q = p;
    for (int a = 0; a < 3; ++a) q.F[a] = p.Us[a];
    q.vel_fill = 1;
    e = enqueue_velocity_fill<T>(q, C);
  }
  mark("ns_pressure_rhs");
  if (e == hipSuccess) {
    if (p.d == 2)
      hipLaunchKernelGGL((k_ns_pressure_rhs<T, 2>), dim3(nb), dim3(kNsThreads), 0, p.stream, Us, C,
                         (const T *)p.P[0], (const T *)p.P[1], (T *)p.W, g, k, wk);
    else if (!wk.flat)
      hipLaunchKernelGGL((k_ns_pressure_rhs_zm<T>), dim3(nb), dim3(kNsThreads), 0, p.stream, Us, C,
                         (const T *)p.P[0], (const T *)p.P[1], (T *)p.W, g, k, wk);
    else
      hipLaunchKernelGGL((k_ns_pressure_rhs<T, 3>), dim3(nb), dim3(kNsThreads), 0, p.stream, Us, C,
                         (const T *)p.P[0], (const T *)p.P[1], (T *)p.W, g, k, wk);
    e = hipGetLastError();
  }
  mark("ns_poisson");
  if (e == hipSuccess) e = enqueue_poisson<T>(p);
  mark("ns_correct");
  if (e == hipSuccess) {
    if (p.d == 2)
      hipLaunchKernelGGL((k_ns_correct<T, 2>), dim3(nb), dim3(kNsThreads), 0, p.stream, U, Ut, Us, C,
                         (const T *)p.W, (const T *)p.P[0], (const T *)p.P[1], g, k, with_ut ? 1 : 0, wk);
    else if (!wk.flat)
      hipLaunchKernelGGL((k_ns_correct_zm<T>), dim3(nb), dim3(kNsThreads), 0, p.stream, U, Ut, Us, C,
                         (const T *)p.W, (const T *)p.P[0], (const T *)p.P[1], g, k, with_ut ? 1 : 0, wk);
    else
      hipLaunchKernelGGL((k_ns_correct<T, 3>), dim3(nb), dim3(kNsThreads), 0, p.stream, U, Ut, Us, C,
                         (const T *)p.W, (const T *)p.P[0], (const T *)p.P[1], g, k, with_ut ? 1 : 0, wk);
    e = hipGetLastError();
  }
  if (tm && e == hipSuccess) e = tm->end(p.stream);
  return e;
}

template hipError_t enqueue_momentum<double>(const Plan &, int, int, KernelTimer *);
template hipError_t enqueue_momentum<float>(const Plan &, int, int, KernelTimer *);

}  // namespace chib
