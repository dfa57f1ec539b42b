// Momentum step of the Navier-Stokes coupling on the staggered grid (sections 2 and 3.3-3.5):
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

constexpr int kNsThreads = 256;

struct NsGrid {
  int n[3];       // cells per axis (1 beyond d)
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

__device__ __forceinline__ int64_t lin3(const NsGrid &g, const int *q) {
  return (int64_t)q[0] + (int64_t)g.n[0] * ((int64_t)q[1] + (int64_t)g.n[1] * q[2]);
}

// q + s e_b with periodic wrap on the periodic axes (the bounded axis is left as is).
__device__ __forceinline__ void step_to(const NsGrid &g, const int *q, int b, int s, int *r) {
  r[0] = q[0];
  r[1] = q[1];
  r[2] = q[2];
  r[b] += s;
  if (b < g.d - 1) r[b] = (r[b] + g.n[b]) % g.n[b];
}

// Face value u_a at cell q: zero outside the box along the bounded axis and on the top wall face.
template <typename T>
__device__ __forceinline__ T face_at(const NsGrid &g, const T *__restrict__ F, int a, const int *q) {
  const int w = q[g.d - 1], nw = g.n[g.d - 1];
  if (w < 0 || w >= nw) return T(0);
  if (a == g.d - 1 && w == nw - 1) return T(0);
  return F[lin3(g, q)];
}

// Cell scalar at q, reflected across the bounded axis' walls.
template <typename T>
__device__ __forceinline__ T cell_at(const NsGrid &g, const T *__restrict__ f, const int *q) {
  int r[3] = {q[0], q[1], q[2]};
  const int bw = g.d - 1;
  if (r[bw] < 0) r[bw] = 0;
  if (r[bw] >= g.n[bw]) r[bw] = g.n[bw] - 1;
  return f[lin3(g, r)];
}

template <typename T>
__device__ __forceinline__ T rho_of(const NsCoef<T> &k, T C) {
  return T(0.5) * ((C + T(1)) * k.rho2 - (C - T(1)) * k.rho1);
}

template <typename T>
__device__ __forceinline__ T mu_of(const NsCoef<T> &k, T C) {
  return T(0.5) * ((C + T(1)) * k.mu2 - (C - T(1)) * k.mu1);
}

__device__ __forceinline__ void coords(const NsGrid &g, int64_t c, int *q) {
  q[0] = (int)(c % g.n[0]);
  const int64_t r = c / g.n[0];
  q[1] = (int)(r % g.n[1]);
  q[2] = (int)(r / g.n[1]);
}

// Prediction (Eq. PredictionExp) and penalisation (Eq. Penalization2) on the d faces of each cell:
//   u** = alpha_f (u^n + dt (-(3/2 N^n - 1/2 N^(n-1)) + ((1/Re) V + kappa phi_f dC/dx_a) / rho_f + g_a))
// N: conservative central convective term; V: viscous term with mu from C^(n+1); phi = W.
// Writes N^n over N^(n-1).  first: forward Euler for the convective term.
template <typename T>
__global__ __launch_bounds__(kNsThreads) void k_ns_predict(FaceSet<T> U, const T *__restrict__ C,
                                                           const T *__restrict__ phi, FaceSet<T> Nh,
                                                           FaceSet<T> Af, FaceSet<T> Us, NsGrid g, NsCoef<T> k,
                                                           int first) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.N) return;
  const int d = g.d, bw = d - 1, nw = g.n[bw];
  int q[3];
  coords(g, c, q);
  const int w = q[bw];
  for (int a = 0; a < d; ++a) {
    if (a == bw && w == nw - 1) {   // top wall face: no penetration
      Us.f[a][c] = T(0);
      Nh.f[a][c] = T(0);
      continue;
    }
    const T *ua = U.f[a];
    int qa[3], qm[3];
    step_to(g, q, a, 1, qa);
    step_to(g, q, a, -1, qm);
    const T u0 = face_at(g, ua, a, q);
    // convective term
    T N = T(0);
    for (int b = 0; b < d; ++b) {
      if (b == a) {
        const T uc0 = T(0.5) * (face_at(g, ua, a, qm) + u0);
        const T uc1 = T(0.5) * (u0 + face_at(g, ua, a, qa));
        N += (uc1 * uc1 - uc0 * uc0) * k.inv_h;
      } else {
        const T *ub = U.f[b];
        int qb[3], qbm[3], qab[3], qbma[3];
        step_to(g, q, b, 1, qb);
        step_to(g, q, b, -1, qbm);
        step_to(g, qbm, a, 1, qbma);
        (void)qab;
        T E1 = T(0.5) * (u0 + face_at(g, ua, a, qb)) * T(0.5) * (face_at(g, ub, b, q) + face_at(g, ub, b, qa));
        if (b == bw && w == nw - 1) E1 = T(0);
        T E0 = T(0);
        if (!(b == bw && w == 0))
          E0 = T(0.5) * (face_at(g, ua, a, qbm) + u0) * T(0.5) * (face_at(g, ub, b, qbm) + face_at(g, ub, b, qbma));
        N += (E1 - E0) * k.inv_h;
      }
    }
    // viscous term
    const T mu_c = mu_of(k, C[c]);
    const T mu_a = mu_of(k, cell_at(g, C, qa));
    const T tn0 = T(2) * mu_c * (u0 - face_at(g, ua, a, qm)) * k.inv_h;
    const T tn1 = T(2) * mu_a * (face_at(g, ua, a, qa) - u0) * k.inv_h;
    T V = (tn1 - tn0) * k.inv_h;
    for (int b = 0; b < d; ++b) {
      if (b == a) continue;
      const T *ub = U.f[b];
      int qb[3], qab[3], qbm[3], qabm[3], qbma[3];
      step_to(g, q, b, 1, qb);
      step_to(g, qa, b, 1, qab);
      step_to(g, q, b, -1, qbm);
      step_to(g, qa, b, -1, qabm);
      step_to(g, qbm, a, 1, qbma);
      (void)qabm;
      // edge c + e_a/2 + e_b/2
      const T me1 = T(0.25) * (mu_c + mu_a + mu_of(k, cell_at(g, C, qb)) + mu_of(k, cell_at(g, C, qab)));
      const T ub_up = (b == bw && w == nw - 1) ? -u0 : face_at(g, ua, a, qb);
      const T tau1 = me1 * ((ub_up - u0) * k.inv_h + (face_at(g, ub, b, qa) - face_at(g, ub, b, q)) * k.inv_h);
      T tau0;
      if (b == bw && w == 0) {   // edge on the bottom wall: no-slip image, u_b = 0 along the wall
        tau0 = T(0.5) * (mu_c + mu_a) * (u0 - (-u0)) * k.inv_h;
      } else {
        const T mu_b = mu_of(k, cell_at(g, C, qbm));
        const T mu_ab = mu_of(k, cell_at(g, C, qbma));
        const T me0 = T(0.25) * (mu_b + mu_ab + mu_c + mu_a);
        const T ua_m = face_at(g, ua, a, qbm);
        tau0 = me0 * ((u0 - ua_m) * k.inv_h + (face_at(g, ub, b, qbma) - face_at(g, ub, b, qbm)) * k.inv_h);
      }
      V += (tau1 - tau0) * k.inv_h;
    }
    // capillary force and density on the face
    const T C0 = C[c], C1 = cell_at(g, C, qa);
    const T F = k.kappa * (T(0.5) * (phi[c] + cell_at(g, phi, qa))) * (C1 - C0) * k.inv_h;
    const T rf = T(0.5) * (rho_of(k, C0) + rho_of(k, C1));
    const T Np = first ? N : Nh.f[a][c];
    const T us = u0 + k.dt * (-(T(1.5) * N - T(0.5) * Np) + (V * k.inv_re + F) / rf + k.g[a]);
    Us.f[a][c] = Af.f[a][c] * us;
    Nh.f[a][c] = N;
  }
}

// Right-hand side of Eq. PressurePoisson at the cell centres:
//   div((1 - rho0/rho_f) grad p^) + (rho0/dt) div u**,  p^ = 2 P0 - P1; no flux through the walls.
template <typename T>
__global__ __launch_bounds__(kNsThreads) void k_ns_pressure_rhs(FaceSet<T> Us, const T *__restrict__ C,
                                                                const T *__restrict__ P0, const T *__restrict__ P1,
                                                                T *__restrict__ R, NsGrid g, NsCoef<T> k) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.N) return;
  const int d = g.d, bw = d - 1, nw = g.n[bw];
  int q[3];
  coords(g, c, q);
  const int w = q[bw];
  auto ph = [&](const int *r) { return T(2) * cell_at(g, P0, r) - cell_at(g, P1, r); };
  // flux (1 - rho0/rho_f) dp^/dx_a on the face of cell r along a (zero on the top wall face)
  auto flux = [&](const int *r, int a) {
    if (a == bw && r[bw] == nw - 1) return T(0);
    int ra[3];
    step_to(g, r, a, 1, ra);
    const T rf = T(0.5) * (rho_of(k, cell_at(g, C, r)) + rho_of(k, cell_at(g, C, ra)));
    return (T(1) - k.rho0 / rf) * ((ph(ra) - ph(r)) * k.inv_h);
  };
  T acc1 = T(0), acc2 = T(0);
  for (int a = 0; a < d; ++a) {
    int qm[3];
    step_to(g, q, a, -1, qm);
    const bool below_wall = (a == bw && w == 0);
    const T fu = flux(q, a);
    const T fl = below_wall ? T(0) : flux(qm, a);
    acc1 += fu - fl;
    acc2 += face_at(g, Us.f[a], a, q) - face_at(g, Us.f[a], a, qm);
  }
  R[c] = acc1 * k.inv_h + k.rho0_dt * (acc2 * k.inv_h);
}

// Correction (Eq. correction): u^(n+1) = u** - dt (grad p^(n+1) / rho0 + (1/rho_f - 1/rho0) grad p^)
// on every face but the top wall face; also writes the advecting velocity 2u^(n+1) - u^n of the
// next order-parameter step (Ut, may be absent).
template <typename T>
__global__ __launch_bounds__(kNsThreads) void k_ns_correct(FaceSet<T> U, FaceSet<T> Ut, FaceSet<T> Us,
                                                           const T *__restrict__ C, const T *__restrict__ Pn,
                                                           const T *__restrict__ P0, const T *__restrict__ P1,
                                                           NsGrid g, NsCoef<T> k, int with_ut) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.N) return;
  const int d = g.d, bw = d - 1, nw = g.n[bw];
  int q[3];
  coords(g, c, q);
  const int w = q[bw];
  const T phc = T(2) * P0[c] - P1[c];
  const T rc = rho_of(k, C[c]);
  for (int a = 0; a < d; ++a) {
    T un = T(0);
    if (!(a == bw && w == nw - 1)) {
      int qa[3];
      step_to(g, q, a, 1, qa);
      const int64_t ca = lin3(g, qa);
      const T Gn = (Pn[ca] - Pn[c]) * k.inv_h;
      const T Gh = ((T(2) * P0[ca] - P1[ca]) - phc) * k.inv_h;
      const T rf = T(0.5) * (rc + rho_of(k, C[ca]));
      un = Us.f[a][c] - k.dt * (Gn * k.inv_rho0 + (T(1) / rf - k.inv_rho0) * Gh);
    }
    const T uo = U.f[a][c];
    U.f[a][c] = un;
    if (with_ut) Ut.f[a][c] = T(2) * un - uo;
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
  g.d = p.d;
  g.N = p.N;
  return g;
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
  const unsigned nb = (unsigned)((p.N + kNsThreads - 1) / kNsThreads);
  const T *C = (const T *)p.C[cur];
  const FaceSet<T> U = faces<T>(p.F, p.d), Us = faces<T>(p.Us, p.d), Nh = faces<T>(p.Nh, p.d);
  const FaceSet<T> Af = faces<T>(p.Af, p.d);
  const bool with_ut = p.Ut[0] != nullptr;
  const FaceSet<T> Ut = with_ut ? faces<T>(p.Ut, p.d) : U;
  mark("ns_phi");
  if (e == hipSuccess) e = enqueue_phi<T>(p, cur, p.W);
  mark("ns_predict");
  if (e == hipSuccess) {
    hipLaunchKernelGGL((k_ns_predict<T>), dim3(nb), dim3(kNsThreads), 0, p.stream, U, C, (const T *)p.W, Nh, Af, Us,
                       g, k, first);
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
    hipLaunchKernelGGL((k_ns_pressure_rhs<T>), dim3(nb), dim3(kNsThreads), 0, p.stream, Us, C, (const T *)p.P[0],
                       (const T *)p.P[1], (T *)p.W, g, k);
    e = hipGetLastError();
  }
  mark("ns_poisson");
  if (e == hipSuccess) e = enqueue_poisson<T>(p);
  mark("ns_correct");
  if (e == hipSuccess) {
    hipLaunchKernelGGL((k_ns_correct<T>), dim3(nb), dim3(kNsThreads), 0, p.stream, U, Ut, Us, C, (const T *)p.W,
                       (const T *)p.P[0], (const T *)p.P[1], g, k, with_ut ? 1 : 0);
    e = hipGetLastError();
  }
  if (tm && e == hipSuccess) e = tm->end(p.stream);
  return e;
}

template hipError_t enqueue_momentum<double>(const Plan &, int, int, KernelTimer *);
template hipError_t enqueue_momentum<float>(const Plan &, int, int, KernelTimer *);

}  // namespace chib
