// Device kernels of one time step of the hybrid ghost-cell IB / Cahn-Hilliard method
// (Appendix A.1 and sections 4.2.2 and 4.3 of the paper), written for gfx950 (CDNA4):
// 64-wide wavefronts, 256-thread workgroups, 32 KB LDS tiles, XCD-aware tile order.
//
// Step pipeline (C^n in C[cur], C^(n-1) in C[1-cur]; the step overwrites C[1-cur]):
//   K1  rhs + Hartley transform along x     C^n, C^(n-1), faces -> W       (contiguous lines)
//   K2  Hartley transform along y (3D)      W -> W                          (strided columns)
//   K3  cosine transform along the bounded axis, division by (lam-a)(lam+alpha_s),
//       inverse cosine transform            W -> W                          (strided columns)
//   K4  Hartley transform along y (3D)      W -> W
//   K5  Hartley transform along x           W -> C[1-cur]  (= C* on every cell)
//   K6  contact-angle ghost fill of C       C[1-cur] at ghost cells
//   K7  no-penetration / Navier-slip fill of faces touching ghosts
//
// The Hartley transform H[k] = sum x[n] cas(2 pi k n / N) diagonalises the periodic second
// difference exactly as the Fourier transform does (modes k and N-k share an eigenvalue) and
// keeps every array real: N values per line, no half-spectrum padding.  Two real lines are
// transformed at once as the real and imaginary parts of one complex FFT.  The cosine
// transform (type II) diagonalises the second difference with reflecting box walls; it is
// computed from one complex FFT of the even/odd reordered sequence, again two lines at once.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <type_traits>

#include "kernels.h"

namespace chib {

namespace {

constexpr int kThreads = 256;

struct Dims {
  int nx, ny, nz;
  int lnx, lny, lnz;
  int64_t plane;
};

template <typename T>
struct RhsCoef {
  T pe_cn2;   // Pe / Cn^2
  T inv_dt;
  T S;
  T inv_cn2;  // 1 / Cn^2
  T inv_h;
  T inv_h2;
};

// The wall condition dphi/dn = 0 in the rhs (end of section 4.2.2, Eq. WallBCS): g at every ghost
// G becomes g_G + dg_G, dg_G = (phi~_M - phi~_G)/Cn^2 with phi~ = C~^3 - C~ - Cn^2 lap_h C~ the
// explicit chemical potential of the step (k_ghost_dphi).  Through lap_h(g) that changes Q by
// -2d dg_G/h^2 at the ghost and by +dg_G/h^2 at each face neighbour: a sparse patch over the
// ghosts and their neighbours, listed sorted by cell with the first entry of every x-row, and its
// value dq per entry (k_patch_dq).  The rhs kernels add it in LDS before their x transform.
// dq == nullptr: no patch.
template <typename T>
struct RhsPatch {
  const int *row;    // [rows + 1]
  const int *cell;   // [np]
  const T *dq;       // [np]
};

// Adds the patch entries [e0, e1) of the x-rows line0 .. line0 + L - 1 to a line tile in LDS
// (row l at l * pitch, element i at i + i/16); one entry per thread, no two entries share a cell.
template <typename T>
__device__ __forceinline__ void patch_tile(T *__restrict__ s, const RhsPatch<T> &rp, int64_t line0, int lnx,
                                           int pitch, int e0, int e1) {
  for (int e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
    const int c = rp.cell[e];
    const int l = (int)((c >> lnx) - line0);
    const int i = c & ((1 << lnx) - 1);
    s[l * pitch + i + (i >> 4)] += rp.dq[e];
  }
}


// ---------------------------------------------------------------------------------------
// Register DFTs of length R in {2, 4, 8, 16}, natural order in and out.  Forward uses
// exp(-2 pi i / R); INV the conjugate.  Twiddles are powers of w16 = exp(-2 pi i / 16).
constexpr double kC16[16] = {1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
                             0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
                             -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173,
                             0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613};
constexpr double kS16[16] = {0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613,
                             1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
                             0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
                             -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173};

// x <- x * w16^e (forward) or x * conj(w16^e) (INV); e is a compile-time constant after unrolling.
template <typename T, bool INV>
__device__ __forceinline__ void rot16(T &re, T &im, int e) {
  e &= 15;
  if (e == 0) return;
  if (e == 8) {
    re = -re;
    im = -im;
    return;
  }
  if (e == 4 || e == 12) {  // -i (forward, e=4) / +i
    const bool minus_i = (e == 4) != INV;
    const T r = re;
    if (minus_i) {
      re = im;
      im = -r;
    } else {
      re = -im;
      im = r;
    }
    return;
  }
  const T c = (T)kC16[e];
  const T sn = INV ? (T)kS16[e] : -(T)kS16[e];
  const T r = re;
  re = r * c - im * sn;
  im = r * sn + im * c;
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void dft_reg(T *xr, T *xi);

template <typename T, int R1, int R2, bool INV>
__device__ __forceinline__ void dft_split(T *xr, T *xi) {
  constexpr int R = R1 * R2;
  T yr[R], yi[R];
#pragma unroll
  for (int n1 = 0; n1 < R1; ++n1) {
    T ar[R2], ai[R2];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) {
      ar[n2] = xr[n1 + R1 * n2];
      ai[n2] = xi[n1 + R1 * n2];
    }
    dft_reg<T, R2, INV>(ar, ai);
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) {
      rot16<T, INV>(ar[k2], ai[k2], n1 * k2 * (16 / R));
      yr[n1 * R2 + k2] = ar[k2];
      yi[n1 * R2 + k2] = ai[k2];
    }
  }
#pragma unroll
  for (int k2 = 0; k2 < R2; ++k2) {
    T ar[R1], ai[R1];
#pragma unroll
    for (int n1 = 0; n1 < R1; ++n1) {
      ar[n1] = yr[n1 * R2 + k2];
      ai[n1] = yi[n1 * R2 + k2];
    }
    dft_reg<T, R1, INV>(ar, ai);
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
      xr[k2 + R2 * k1] = ar[k1];
      xi[k2 + R2 * k1] = ai[k1];
    }
  }
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void dft_reg(T *xr, T *xi) {
  if constexpr (R == 2) {
    const T ar = xr[0], ai = xi[0];
    xr[0] = ar + xr[1];
    xi[0] = ai + xi[1];
    xr[1] = ar - xr[1];
    xi[1] = ai - xi[1];
  } else if constexpr (R == 4) {
    const T ar = xr[0] + xr[2], ai = xi[0] + xi[2];
    const T br = xr[0] - xr[2], bi = xi[0] - xi[2];
    const T cr = xr[1] + xr[3], ci = xi[1] + xi[3];
    const T dr = xr[1] - xr[3], di = xi[1] - xi[3];
    xr[0] = ar + cr;
    xi[0] = ai + ci;
    xr[2] = ar - cr;
    xi[2] = ai - ci;
    if (!INV) {  // y1 = b - i d, y3 = b + i d
      xr[1] = br + di;
      xi[1] = bi - dr;
      xr[3] = br - di;
      xi[3] = bi + dr;
    } else {
      xr[1] = br - di;
      xi[1] = bi + dr;
      xr[3] = br + di;
      xi[3] = bi - dr;
    }
  } else if constexpr (R == 8) {
    dft_split<T, 2, 4, INV>(xr, xi);
  } else {
    static_assert(R == 16, "radix");
    dft_split<T, 4, 4, INV>(xr, xi);
  }
}

constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v >> 1); }

// LDS address of element n of sequence b: b*ps + n*ns, plus padw extra elements after every
// 16 positions (keeps the stride-16 accesses of the radix-16 stages off a single bank).
__device__ __forceinline__ int lds_at(int b, int n, int ps, int ns, int padw) {
  return b * ps + n * ns + (n >> 4) * padw;
}

// Stages `tot` elements from global memory into LDS, element e read from src(e) and written to
// LDS slot dst(e): every thread issues kBatch independent loads before its LDS stores, so a tile
// costs one memory round trip per batch rather than one per element.
constexpr int kBatch = 8;
template <typename T, typename Src, typename Dst>
__device__ __forceinline__ void stage_tile(T *__restrict__ s, int tot, Src src, Dst dst) {
  for (int e0 = threadIdx.x; e0 < tot; e0 += kBatch * blockDim.x) {
    T v[kBatch];
#pragma unroll
    for (int k = 0; k < kBatch; ++k) {
      const int e = e0 + k * blockDim.x;
      v[k] = e < tot ? src(e) : T(0);
    }
#pragma unroll
    for (int k = 0; k < kBatch; ++k) {
      const int e = e0 + k * blockDim.x;
      if (e < tot) s[dst(e)] = v[k];
    }
  }
}

// w^r for r = 1..R-1 from w = w^1 by products of at most four factors.
template <typename T, int R>
__device__ __forceinline__ void twiddle_powers(T w1r, T w1i, T *wr, T *wi) {
  wr[1] = w1r;
  wi[1] = w1i;
#pragma unroll
  for (int r = 2; r < R; ++r) {
    const int a = (r & 1) ? r - 1 : r / 2;   // r = a + (r - a)
    const int c = r - a;
    wr[r] = wr[a] * wr[c] - wi[a] * wi[c];
    wi[r] = wr[a] * wi[c] + wi[a] * wr[c];
  }
}

// One Stockham stage of radix R over `np` sequences of length N in LDS.  p = 2^lp is the
// product of the radices of the previous stages.  Inputs are staged in registers.
template <typename T> struct Pair2;
template <> struct Pair2<double> { using type = double2; };
template <> struct Pair2<float> { using type = float2; };

// 16 bytes of a padded LDS tile at an element offset that is only a multiple of 2: the tiles put a
// 2-element gap after every 16 positions, so a 4-float group need not be 16-byte aligned.  One
// 16-byte access for double2, two 8-byte ones for float4.
template <typename T, typename V>
__device__ __forceinline__ void lds_put16(T *a, const V &v) {
  if constexpr (sizeof(T) == 8) {
    *reinterpret_cast<V *>(a) = v;
  } else {
    using H = typename Pair2<T>::type;
    const H *h = reinterpret_cast<const H *>(&v);
    *reinterpret_cast<H *>(a) = h[0];
    *reinterpret_cast<H *>(a + 2) = h[1];
  }
}
template <typename V, typename T>
__device__ __forceinline__ V lds_get16(const T *a) {
  if constexpr (sizeof(T) == 8) {
    return *reinterpret_cast<const V *>(a);
  } else {
    using H = typename Pair2<T>::type;
    V v;
    H *h = reinterpret_cast<H *>(&v);
    h[0] = *reinterpret_cast<const H *>(a);
    h[1] = *reinterpret_cast<const H *>(a + 2);
    return v;
  }
}

// PAIRED: the imaginary part sits right after the real part (io == 1), and both move as one
// 2-element LDS access; with the sequence index fastest across lanes (bfast) the lanes served
// together then touch distinct bank groups, where two separate accesses would collide.
template <typename T, int R, int IT, bool INV, bool PAIRED = false>
__device__ __forceinline__ void fft_stage(T *__restrict__ s, int logN, int lognp, int ps, int ns, int io, int padw,
                                          bool bfast, int lp, const T *__restrict__ twr, const T *__restrict__ twi) {
  using P2 = typename Pair2<T>::type;
  constexpr int LR = ilog2c(R);
  const int nt = blockDim.x;
  const int tid = threadIdx.x;
  const int lq = logN - LR;
  const int total = 1 << (lognp + lq);
  const int p = 1 << lp;
  const int sh = logN - LR - lp;
  const int npm = (1 << lognp) - 1;
  // lds_at(b, n + r d) = lds_at(b, n) + r (d ns + (d / 16) padw) when d is a multiple of 16, and
  // lds_at(b, n) + r d ns when n + (R - 1) d stays in n's group of 16 (d = 1, n a multiple of R)
  // (radix 16 keeps the general form: the linear one would cost it 25 VGPRs and a wave per SIMD)
  const bool rlin = R <= 8 && lq >= 4, wlin = R <= 8 && (lp >= 4 || lp == 0);
  const int rst = rlin ? (ns << lq) + (padw << (lq - 4)) : 0;
  const int wst = lp >= 4 ? (ns << lp) + (padw << (lp - 4)) : ns;
  T xr[IT][R], xi[IT][R];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int item = tid + it * nt;
    if (item < total) {
      int b, i;
      if (bfast) {
        b = item & npm;
        i = item >> lognp;
      } else {
        i = item & ((1 << lq) - 1);
        b = item >> lq;
      }
      auto rd = [&](int r, int a) {
        if constexpr (PAIRED) {
          const P2 v = *reinterpret_cast<const P2 *>(s + a);
          xr[it][r] = v.x;
          xi[it][r] = v.y;
        } else {
          xr[it][r] = s[a];
          xi[it][r] = s[a + io];
        }
      };
      if (rlin) {   // inputs 2^lq >= 16 apart: the padded address is linear in r
        const int a0 = lds_at(b, i, ps, ns, padw);
#pragma unroll
        for (int r = 0; r < R; ++r) rd(r, a0 + r * rst);
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) rd(r, lds_at(b, i + (r << lq), ps, ns, padw));
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int item = tid + it * nt;
    if (item < total) {
      int b, i;
      if (bfast) {
        b = item & npm;
        i = item >> lognp;
      } else {
        i = item & ((1 << lq) - 1);
        b = item >> lq;
      }
      const int k = i & (p - 1);
      if (lp > 0) {
        const int m = k << sh;
        T wr[R], wi[R];
        twiddle_powers<T, R>(twr[m], INV ? -twi[m] : twi[m], wr, wi);
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const T ur = xr[it][r];
          xr[it][r] = ur * wr[r] - xi[it][r] * wi[r];
          xi[it][r] = ur * wi[r] + xi[it][r] * wr[r];
        }
      }
      dft_reg<T, R, INV>(xr[it], xi[it]);
      const int j = ((i - k) << LR) + k;
      auto wr_ = [&](int r, int a) {
        if constexpr (PAIRED) {
          P2 v;
          v.x = xr[it][r];
          v.y = xi[it][r];
          *reinterpret_cast<P2 *>(s + a) = v;
        } else {
          s[a] = xr[it][r];
          s[a + io] = xi[it][r];
        }
      };
      if (wlin) {   // outputs p apart with p >= 16, or p = 1 (then all R in one padding group)
        const int a0 = lds_at(b, j, ps, ns, padw);
#pragma unroll
        for (int r = 0; r < R; ++r) wr_(r, a0 + r * wst);
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) wr_(r, lds_at(b, j + r * p, ps, ns, padw));
      }
    }
  }
  __syncthreads();
}

// Complex FFT of 2^lognp independent length-2^logN sequences held in LDS: mixed-radix
// Stockham autosort with register-resident radix-16 butterflies (then 8, 4 or 2 for the
// remaining factor).  E bounds the tile (elements of T) so that every thread holds at most
// 16 complex values per stage.  No 1/N scaling.
template <typename T, int E, bool INV, int MAXR = 16, int NT = 256, bool PAIRED = false>
__device__ __forceinline__ void lds_fft(T *__restrict__ s, int logN, int lognp, int ps, int ns, int io, int padw,
                                        bool bfast, const T *__restrict__ twr, const T *__restrict__ twi) {
  constexpr int IT16 = (E / 2 / 16 + NT - 1) / NT;
  constexpr int IT8 = (E / 2 / 8 + NT - 1) / NT;
  constexpr int IT4 = (E / 2 / 4 + NT - 1) / NT;
  constexpr int IT2 = (E / 2 / 2 + NT - 1) / NT;
  int lp = 0;
  int rem = logN;
  if constexpr (MAXR >= 16) {
    while (rem >= 4) {
      fft_stage<T, 16, IT16, INV, PAIRED>(s, logN, lognp, ps, ns, io, padw, bfast, lp, twr, twi);
      lp += 4;
      rem -= 4;
    }
  } else if constexpr (MAXR == 4) {
    while (rem >= 2) {
      fft_stage<T, 4, IT4, INV, PAIRED>(s, logN, lognp, ps, ns, io, padw, bfast, lp, twr, twi);
      lp += 2;
      rem -= 2;
    }
  } else {
    while (rem >= 3) {
      fft_stage<T, 8, IT8, INV, PAIRED>(s, logN, lognp, ps, ns, io, padw, bfast, lp, twr, twi);
      lp += 3;
      rem -= 3;
    }
  }
  if (rem == 3) fft_stage<T, 8, IT8, INV, PAIRED>(s, logN, lognp, ps, ns, io, padw, bfast, lp, twr, twi);
  else if (rem == 2) fft_stage<T, 4, IT4, INV, PAIRED>(s, logN, lognp, ps, ns, io, padw, bfast, lp, twr, twi);
  else if (rem == 1) fft_stage<T, 2, IT2, INV, PAIRED>(s, logN, lognp, ps, ns, io, padw, bfast, lp, twr, twi);
}

// Padded LDS pitch of a contiguous line of n elements (one pad element per 16).
__host__ __device__ __forceinline__ int line_pitch(int n) { return n + (n >> 4); }
// Padded LDS size (elements) of a tile of B interleaved columns by N positions.
__host__ __device__ __forceinline__ int col_tile(int N, int B) { return N * B + (N >> 4) * 2; }

// ---------------------------------------------------------------------------------------
// Right-hand side Q of the first Helmholtz equation at one cell:
//   Q = (Pe/Cn^2)(C^/dt - div_h(u C~)) + lap_h((C~^3 - C~ - S C~)/Cn^2)
// with C~ = 2C^n - C^(n-1), C^ = 2C^n - C^(n-1)/2; periodic axes wrap, the bounded (last)
// axis reflects for the Laplacian and has zero normal velocity on its box walls.
template <typename T, int D>
__device__ __forceinline__ T rhs_at(const T *__restrict__ Cn, const T *__restrict__ Cp, const T *__restrict__ F0,
                                    const T *__restrict__ F1, const T *__restrict__ F2, int i, int j, int k,
                                    const Dims &dm, const RhsCoef<T> &cf) {
  const int nx = dm.nx;
  const int64_t c = (int64_t)i + (int64_t)nx * ((int64_t)j + (int64_t)dm.ny * k);
  auto ct = [&](int64_t q) { return T(2) * Cn[q] - Cp[q]; };
  auto gf = [&](T v) { return (v * v * v - v - cf.S * v) * cf.inv_cn2; };
  const int64_t rowb = c - i;
  const int ip = (i + 1) & (nx - 1), im = (i - 1) & (nx - 1);
  const T c0 = ct(c);
  const T cxp = ct(rowb + ip), cxm = ct(rowb + im);
  T flux = F0[c] * (c0 + cxp) - F0[rowb + im] * (cxm + c0);
  T gsum = gf(cxp) + gf(cxm);
  if (D == 2) {
    const bool top = (j == dm.ny - 1), bot = (j == 0);
    const T cyp = top ? c0 : ct(c + nx);
    const T cym = bot ? c0 : ct(c - nx);
    flux += (top ? T(0) : F1[c] * (c0 + cyp)) - (bot ? T(0) : F1[c - nx] * (cym + c0));
    gsum += gf(cyp) + gf(cym);
  } else {
    const int jp = (j + 1) & (dm.ny - 1), jm = (j - 1) & (dm.ny - 1);
    const int64_t cyp_i = c + (int64_t)(jp - j) * nx, cym_i = c + (int64_t)(jm - j) * nx;
    const T cyp = ct(cyp_i), cym = ct(cym_i);
    flux += F1[c] * (c0 + cyp) - F1[cym_i] * (cym + c0);
    gsum += gf(cyp) + gf(cym);
    const bool top = (k == dm.nz - 1), bot = (k == 0);
    const T czp = top ? c0 : ct(c + dm.plane);
    const T czm = bot ? c0 : ct(c - dm.plane);
    flux += (top ? T(0) : F2[c] * (c0 + czp)) - (bot ? T(0) : F2[c - dm.plane] * (czm + c0));
    gsum += gf(czp) + gf(czm);
  }
  const T A = flux * T(0.5) * cf.inv_h;
  const T lap = (gsum - T(2 * D) * gf(c0)) * cf.inv_h2;
  const T cc = T(2) * Cn[c] - T(0.5) * Cp[c];
  return cf.pe_cn2 * (cc * cf.inv_dt - A) + lap;
}

// Untangles the complex FFT of the pair (a + i b) into the Hartley transforms of a and b:
// with Z[k] = p + iq and Z[N-k] = r + is, H_a[k] = (p - q + r + s)/2, H_b[k] = (p + q - r + s)/2.
template <typename T>
__device__ __forceinline__ T hartley_of_pair(T p, T q, T r, T s, int par) {
  return par ? (p + q - r + s) * T(0.5) : (p - q + r + s) * T(0.5);
}

// ---------------------------------------------------------------------------------------
// K1: rhs of L consecutive x-lines into LDS, Hartley transform along x, store to W.
template <typename T, int D, int E, int U = 1, int MAXR = 16>
__device__ __forceinline__ void rhs_xdht_body(unsigned char *smem_raw, const T *__restrict__ Cn, const T *__restrict__ Cp,
                                                       const T *__restrict__ F0, const T *__restrict__ F1,
                                                       const T *__restrict__ F2, T *__restrict__ W, Dims dm,
                                                       RhsCoef<T> cf, int logL, const T *__restrict__ twr,
                                                       const T *__restrict__ twi, int tile, const RhsPatch<T> &rp) {
  T *s = reinterpret_cast<T *>(smem_raw);
  const int L = 1 << logL;
  const int nx = dm.nx;
  const int line0 = tile * L;
  const int tot = L << dm.lnx;
  const int pitch = line_pitch(nx);
  // U cells per iteration so that their loads are in flight together
  for (int e0 = threadIdx.x; e0 < tot; e0 += U * blockDim.x) {
    T q[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * blockDim.x;
      if (e < tot) {
        const int l = e >> dm.lnx;
        const int i = e & (nx - 1);
        const int line = line0 + l;
        int j, k;
        if (D == 2) {
          j = line;
          k = 0;
        } else {
          j = line & (dm.ny - 1);
          k = line >> dm.lny;
        }
        q[u] = rhs_at<T, D>(Cn, Cp, F0, F1, F2, i, j, k, dm, cf);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * blockDim.x;
      if (e < tot) {
        const int l = e >> dm.lnx;
        const int i = e & (nx - 1);
        s[l * pitch + i + (i >> 4)] = q[u];
      }
    }
  }
  if (rp.dq) {   // the ghost patch of the tile's lines
    __syncthreads();
    patch_tile(s, rp, line0, dm.lnx, pitch, rp.row[line0], rp.row[line0 + L]);
  }
  __syncthreads();
  lds_fft<T, E, false, MAXR>(s, dm.lnx, logL - 1, 2 * pitch, 1, pitch, 1, false, twr, twi);
  const int half = tot >> 1;
  for (int e = threadIdx.x; e < half; e += blockDim.x) {
    const int b = e >> dm.lnx;
    const int kx = e & (nx - 1);
    const int kk = (nx - kx) & (nx - 1);
    const T *pb = s + b * 2 * pitch;
    const int ak = kx + (kx >> 4), an = kk + (kk >> 4);
    const T p = pb[ak], q = pb[pitch + ak], r = pb[an], sv = pb[pitch + an];
    T *o = W + (int64_t)(line0 + 2 * b) * nx + kx;
    o[0] = (p - q + r + sv) * T(0.5);
    o[nx] = (p + q - r + sv) * T(0.5);
  }
}

template <typename T, int D, int E, int U = 1, int MAXR = 16>
__global__ __launch_bounds__(kThreads) void k_rhs_xdht(const T *__restrict__ Cn, const T *__restrict__ Cp,
                                                       const T *__restrict__ F0, const T *__restrict__ F1,
                                                       const T *__restrict__ F2, T *__restrict__ W, Dims dm,
                                                       RhsCoef<T> cf, int logL, const T *__restrict__ twr,
                                                       const T *__restrict__ twi, RhsPatch<T> rp) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  rhs_xdht_body<T, D, E, U, MAXR>(smem_raw, Cn, Cp, F0, F1, F2, W, dm, cf, logL, twr, twi, xcd_tile(blockIdx.x, gridDim.x),
                                  rp);
}

// Extra LDS of the y-marching K1 (two rows of C~ for the x neighbours) over the line tile.
__host__ __device__ __forceinline__ int ym_extra(int nx) { return 2 * nx; }

// K1 for 2D grids, marching in y: the workgroup owns the L rows of its tile across the whole x
// range, thread t the columns x = t + 256 m (m < XM, nx <= 256 XM).  C~ = 2C^n - C^(n-1) of row
// y-1 and the raw C^n, C^(n-1) of rows y and y+1 stay in registers, so every value is loaded
// once and y neighbours never leave the thread (C~, C^ = 2C^n - C^(n-1)/2 and g(C~) =
// C~^3 - (1 + S) C~ are formed from them as needed); the raw values of row y+2 are requested
// while row y is computed.  x neighbours come from a two-row
// ring of C~ in LDS (one barrier per row); each Q row goes straight into the line tile, which
// then goes through the same x transform as the line-tiled K1.  1/Cn^2 scales the Laplacian.
template <typename T, int XM, int R>
__device__ __forceinline__ void rhs_ym_body(unsigned char *smem_raw, const T *__restrict__ Cn,
                                            const T *__restrict__ Cp, const T *__restrict__ F0,
                                            const T *__restrict__ F1, T *__restrict__ W, Dims dm, RhsCoef<T> cf,
                                            int logL, const T *__restrict__ twr, const T *__restrict__ twi,
                                            int tile, const RhsPatch<T> &rp) {
  const int nx = dm.nx, ny = dm.ny;
  const int L = 1 << logL;
  const int pitch = line_pitch(nx);
  T *fb = reinterpret_cast<T *>(smem_raw);           // L rows x pitch: Q, then its transform
  T *xr = fb + L * pitch;                             // 2 rows x nx: C~ of the current row
  const int y0 = tile * L;
  const int tid = threadIdx.x;
  const T s1 = T(1) + cf.S;
  const T klap = cf.inv_h2 * cf.inv_cn2;
  auto g = [&](T v) { return v * (v * v - s1); };
  auto rowp = [&](const T *__restrict__ a, int y) { return a + (int64_t)(y < 0 ? 0 : (y >= ny ? ny - 1 : y)) * nx; };
  // per column: C~ of row y-1, the raw C^n, C^(n-1) of rows y, y+1 and y+2 (in flight), F1 of row y-1
  T cm[XM], a0[XM], b0[XM], a1[XM], b1[XM], an[XM], bn[XM], f1m[XM];
#pragma unroll
  for (int m = 0; m < XM; ++m) {
    const int i = tid + 256 * m;
    if (i < nx) {
      const T a_m = rowp(Cn, y0 - 1)[i], b_m = rowp(Cp, y0 - 1)[i];
      a0[m] = rowp(Cn, y0)[i];
      b0[m] = rowp(Cp, y0)[i];
      a1[m] = rowp(Cn, y0 + 1)[i];
      b1[m] = rowp(Cp, y0 + 1)[i];
      f1m[m] = rowp(F1, y0 - 1)[i];
      an[m] = rowp(Cn, y0 + 2)[i];
      bn[m] = rowp(Cp, y0 + 2)[i];
      cm[m] = T(2) * a_m - b_m;
    }
  }
  for (int r = 0; r < L; ++r) {
    const int y = y0 + r;
    const bool top = y == ny - 1, bot = y == 0;
    T *xb = xr + (r & 1) * nx;
    T f0[XM], f0m[XM], f1[XM];
#pragma unroll
    for (int m = 0; m < XM; ++m) {
      const int i = tid + 256 * m;
      if (i < nx) {
        const T *r0 = rowp(F0, y), *r1 = rowp(F1, y);
        f0[m] = r0[i];
        f0m[m] = r0[(i - 1) & (nx - 1)];
        f1[m] = r1[i];
        xb[i] = T(2) * a0[m] - b0[m];
      }
    }
    __syncthreads();   // the row is in LDS; the ring slot written next row was last read two rows ago
#pragma unroll
    for (int m = 0; m < XM; ++m) {
      const int i = tid + 256 * m;
      if (i < nx) {
        const T v0 = T(2) * a0[m] - b0[m];
        const T cxp = xb[(i + 1) & (nx - 1)], cxm = xb[(i - 1) & (nx - 1)];
        const T cyp = top ? v0 : T(2) * a1[m] - b1[m], cym = bot ? v0 : cm[m];
        T flux = f0[m] * (v0 + cxp) - f0m[m] * (cxm + v0);
        flux += (top ? T(0) : f1[m] * (v0 + cyp)) - (bot ? T(0) : f1m[m] * (cym + v0));
        const T g0 = g(v0);
        const T gsum = g(cxp) + g(cxm) + (top ? g0 : g(cyp)) + (bot ? g0 : g(cym));
        const T A = flux * T(0.5) * cf.inv_h;
        const T lap = (gsum - T(4) * g0) * klap;
        const T h0 = T(2) * a0[m] - T(0.5) * b0[m];
        fb[r * pitch + i + (i >> 4)] = cf.pe_cn2 * (h0 * cf.inv_dt - A) + lap;
        // slide the window down one row and request the row after next
        cm[m] = v0;
        a0[m] = a1[m];
        b0[m] = b1[m];
        a1[m] = an[m];
        b1[m] = bn[m];
        f1m[m] = f1[m];
        if (r + 1 < L) {
          an[m] = rowp(Cn, y + 3)[i];
          bn[m] = rowp(Cp, y + 3)[i];
        }
      }
    }
  }
  if (rp.dq) {   // the ghost patch of the tile's rows
    __syncthreads();
    patch_tile(fb, rp, y0, dm.lnx, pitch, rp.row[y0], rp.row[y0 + L]);
  }
  __syncthreads();
  lds_fft<T, tile_elems<T>(), false, R>(fb, dm.lnx, logL - 1, 2 * pitch, 1, pitch, 1, false, twr, twi);
  const int half = (L * nx) >> 1;
  for (int e = tid; e < half; e += blockDim.x) {
    const int b = e >> dm.lnx;
    const int kx = e & (nx - 1);
    const int kk = (nx - kx) & (nx - 1);
    const T *pb = fb + b * 2 * pitch;
    const int ak = kx + (kx >> 4), a2 = kk + (kk >> 4);
    const T p = pb[ak], q = pb[pitch + ak], rr = pb[a2], sv = pb[pitch + a2];
    T *o = W + (int64_t)(y0 + 2 * b) * nx + kx;
    o[0] = (p - q + rr + sv) * T(0.5);
    o[nx] = (p + q - rr + sv) * T(0.5);
  }
}

template <typename T, int XM, int R>
__global__ __launch_bounds__(kThreads, R == 8 ? 4 : 3) void k_rhs_xdht_ym(const T *__restrict__ Cn, const T *__restrict__ Cp,
                                                          const T *__restrict__ F0, const T *__restrict__ F1,
                                                          T *__restrict__ W, Dims dm, RhsCoef<T> cf, int logL,
                                                          const T *__restrict__ twr, const T *__restrict__ twi,
                                                          RhsPatch<T> rp) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  rhs_ym_body<T, XM, R>(smem_raw, Cn, Cp, F0, F1, W, dm, cf, logL, twr, twi, xcd_tile(blockIdx.x, gridDim.x), rp);
}

// K1 for 3D grids, marching in z (2.5D blocking): a workgroup owns L consecutive y rows and
// a chunk of ZC planes.  Thread t owns the x positions x = t + 256 m (m < nx/256, nx >= 256)
// of rows -1..L of the tile, i.e. whole column segments including the two halo rows, and
// keeps C~ of planes z-1, z, z+1 in registers, so y and z neighbours never leave the thread;
// x neighbours (of C~ and of the x faces) come from LDS.  Each plane's L rows of Q go through
// the same Hartley transform as K1 and are stored to W.  Requires nx a multiple of 256.
// Software pipeline: while plane z is transformed and stored, the loads of C^n, C^(n-1) for
// plane z+2 and of the faces and patch entries for plane z+1 are in flight, so a plane only
// ever waits for data requested one plane earlier.  The FFT twiddles are read from LDS: vector
// memory counters retire in order, so a global twiddle load inside the FFT would also wait for
// every request in flight.
template <typename T, int L, int XM, int R, bool SPLIT = false>
__global__ __launch_bounds__(kThreads, (L == 2 && XM == 1 && R == 4) ? 3 : 1) void k_rhs_xdht_zm(const T *__restrict__ Cn, const T *__restrict__ Cp,
                                                          const T *__restrict__ F0, const T *__restrict__ F1,
                                                          const T *__restrict__ F2, T *__restrict__ W, Dims dm,
                                                          RhsCoef<T> cf, int zc_log, const T *__restrict__ twr,
                                                          const T *__restrict__ twi, RhsPatch<T> rp) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  constexpr int nx = 256 * XM, lnx = ilog2c(nx);   // the launcher takes this kernel only for nx = 256 XM
  T *plane = reinterpret_cast<T *>(smem_raw);        // L rows x nx: C~ of plane z
  T *fxp = plane + L * nx;                             // L rows x nx: x faces of plane z
  const int pitch = line_pitch(nx);
  T *fb = fxp + L * nx;                                // L rows x pitch: FFT tile
  T *tw = fb + L * pitch;                              // 2 x nx: the x twiddles (read from LDS, so that
                                                       // the FFT never waits on the global requests in flight)
  const int nyt = dm.ny / L;
  const int t = xcd_tile(blockIdx.x, gridDim.x);
  const int yt = t % nyt;
  const int zc = t / nyt;
  const int y0 = yt * L;
  const int ZC = 1 << zc_log;
  const int z0 = zc * ZC;
  const int tid = threadIdx.x;
  auto gf = [&](T v) { return (v * v * v - v - cf.S * v) * cf.inv_cn2; };
  auto row_of = [&](int r) { return (y0 + r + dm.ny) & (dm.ny - 1); };  // r in -1..L
  auto zbase = [&](int z) { return (int64_t)(z < 0 ? 0 : (z >= dm.nz ? dm.nz - 1 : z)) * dm.plane; };
  // C~ at rows -1..L of planes z-1 (rows 0..L-1 kept), z, z+1; C^ = 2C^n - C^(n-1)/2 of the own
  // rows of planes z, z+1; raw C^n, C^(n-1) of plane z+2 in flight
  T cm[XM][L], c0[XM][L + 2], cp[XM][L + 2], h0[XM][L], hp[XM][L], na[XM][L + 2], nb[XM][L + 2];
  // faces of plane z (F1 at rows -1..L-1, z faces of plane z-1 below) and of plane z+1 in flight
  T f0[XM][L], f1[XM][L + 1], f2[XM][L], uzm[XM][L], nf0[XM][L], nf1[XM][L + 1], nf2[XM][L];
  // Cache policy: C^n, C^(n-1) and the x and z faces are read here for the last time in the step and
  // W is read next by another pass over the whole grid, so all of them go as non-temporal (streaming)
  // accesses that leave the L2 and the Infinity Cache to the y faces (rows shared by neighbouring
  // tiles) and to the next passes; measured 181 -> 168 us together with the x pass out's streaming reads
  auto load_c = [&](int z) {   // planes beyond the box reflect onto the boundary plane
    const int64_t zb = zbase(z);
#pragma unroll
    for (int m = 0; m < XM; ++m)
#pragma unroll
      for (int r = 0; r < L + 2; ++r) {
        const int64_t q = zb + (int64_t)row_of(r - 1) * nx + tid + 256 * m;
        na[m][r] = __builtin_nontemporal_load(Cn + q);
        nb[m][r] = __builtin_nontemporal_load(Cp + q);
      }
  };
  auto load_f = [&](int z) {
    const int64_t zb = zbase(z);
#pragma unroll
    for (int m = 0; m < XM; ++m) {
#pragma unroll
      for (int r = 0; r < L; ++r) {
        const int64_t q = zb + (int64_t)row_of(r) * nx + tid + 256 * m;
        nf0[m][r] = __builtin_nontemporal_load(F0 + q);
        nf2[m][r] = __builtin_nontemporal_load(F2 + q);
      }
#pragma unroll
      for (int r = 0; r < L + 1; ++r) nf1[m][r] = F1[zb + (int64_t)row_of(r - 1) * nx + tid + 256 * m];
    }
  };
  auto take_c = [&](T (&dst)[XM][L + 2], T (&hat)[XM][L]) {
#pragma unroll
    for (int m = 0; m < XM; ++m)
#pragma unroll
      for (int r = 0; r < L + 2; ++r) {
        dst[m][r] = T(2) * na[m][r] - nb[m][r];
        if (r >= 1 && r <= L) hat[m][r - 1] = T(2) * na[m][r] - T(0.5) * nb[m][r];
      }
  };
  auto take_f = [&]() {
#pragma unroll
    for (int m = 0; m < XM; ++m) {
#pragma unroll
      for (int r = 0; r < L; ++r) {
        uzm[m][r] = f2[m][r];
        f0[m][r] = nf0[m][r];
        f2[m][r] = nf2[m][r];
      }
#pragma unroll
      for (int r = 0; r < L + 1; ++r) f1[m][r] = nf1[m][r];
    }
  };
  if constexpr (!SPLIT)
    for (int e = tid; e < nx; e += blockDim.x) {   // ordered before the first FFT by the plane barrier
      tw[e] = twr[e];
      tw[nx + e] = twi[e];
    }
  // prologue: C~ of planes z0-1, z0, z0+1 and the faces of plane z0 (and the z faces below it)
  {
    T th[XM][L];
    load_c(z0 - 1);   // the reflecting wall below plane 0 is plane 0 itself
    take_c(cp, th);
#pragma unroll
    for (int m = 0; m < XM; ++m)
#pragma unroll
      for (int r = 0; r < L; ++r) {
        cm[m][r] = cp[m][r + 1];
        f2[m][r] = z0 > 0 ? F2[zbase(z0 - 1) + (int64_t)row_of(r) * nx + tid + 256 * m] : T(0);
      }
  }
  load_c(z0);
  take_c(c0, h0);
  load_c(z0 + 1);
  take_c(cp, hp);
  load_f(z0);
  take_f();
  // ghost patch (SPLIT: added by the caller afterwards): the entries of the tile's rows of a plane
  // are requested one plane ahead and added to its Q tile after the stencil
  constexpr int PF = 2;
  const bool patch = !SPLIT && rp.dq != nullptr;
  int e_lo = 0, e_hi = 0, n_lo = 0, n_hi = 0, pc[PF], npc[PF];
  T pd[PF], npd[PF];
  auto range_of = [&](int z, int &lo, int &hi) {
    const int64_t R0 = (int64_t)z * dm.ny + y0;
    lo = rp.row[R0];
    hi = rp.row[R0 + L];
  };
  // every request is unconditional (indices clamped into the list, which is not empty when the
  // patch is on): a register with a default on one path would have to wait for the load in flight
  auto load_p = [&](int lo, int hi) {
    const int last = hi > 0 ? hi - 1 : 0;
#pragma unroll
    for (int k = 0; k < PF; ++k) {
      const int e = min(lo + tid + 256 * k, last);
      npc[k] = rp.cell[e];
      npd[k] = rp.dq[e];
    }
  };
  const int zlast = z0 + ZC - 1;
  if (patch) {
    range_of(z0, e_lo, e_hi);
    load_p(e_lo, e_hi);
#pragma unroll
    for (int k = 0; k < PF; ++k) {
      pc[k] = npc[k];
      pd[k] = npd[k];
    }
    range_of(min(z0 + 1, zlast), n_lo, n_hi);
  }
  // plane z+1 becomes current: the first use of the requests made at the top of plane z, placed
  // before the stores of W so that the wait does not include their completion
  int nn_lo = 0, nn_hi = 0;
  auto rotate = [&]() {
#pragma unroll
    for (int m = 0; m < XM; ++m) {
#pragma unroll
      for (int r = 0; r < L; ++r) cm[m][r] = c0[m][r + 1];
#pragma unroll
      for (int r = 0; r < L + 2; ++r) c0[m][r] = cp[m][r];
#pragma unroll
      for (int r = 0; r < L; ++r) h0[m][r] = hp[m][r];
    }
    take_c(cp, hp);
    take_f();
    if (patch) {
#pragma unroll
      for (int k = 0; k < PF; ++k) {
        pc[k] = npc[k];
        pd[k] = npd[k];
      }
      e_lo = n_lo;
      e_hi = n_hi;
      n_lo = nn_lo;
      n_hi = nn_hi;
    }
  };
  for (int zi = 0; zi < ZC; ++zi) {
    const int z = z0 + zi;
    const int64_t zb = (int64_t)z * dm.plane;
    const bool more = zi + 1 < ZC;
    const bool top = z == dm.nz - 1, bot = z == 0;
#pragma unroll
    for (int m = 0; m < XM; ++m)
#pragma unroll
      for (int r = 0; r < L; ++r) {
        plane[r * nx + tid + 256 * m] = c0[m][r + 1];
        fxp[r * nx + tid + 256 * m] = f0[m][r];
      }
    __syncthreads();
    T q[XM][L];
#pragma unroll
    for (int m = 0; m < XM; ++m) {
      const int i = tid + 256 * m;
      const int ip = (i + 1) & (nx - 1), im = (i - 1) & (nx - 1);
#pragma unroll
      for (int r = 0; r < L; ++r) {
        const T v0 = c0[m][r + 1];
        const T cxp = plane[r * nx + ip], cxm = plane[r * nx + im];
        const T cyp = c0[m][r + 2], cym = c0[m][r];
        const T czp = top ? v0 : cp[m][r + 1];
        const T czm = bot ? v0 : cm[m][r];
        T flux = f0[m][r] * (v0 + cxp) - fxp[r * nx + im] * (cxm + v0);
        flux += f1[m][r + 1] * (v0 + cyp) - f1[m][r] * (cym + v0);
        flux += (top ? T(0) : f2[m][r] * (v0 + czp)) - (bot ? T(0) : uzm[m][r] * (czm + v0));
        const T gsum = gf(cxp) + gf(cxm) + gf(cyp) + gf(cym) + gf(czp) + gf(czm);
        const T A = flux * T(0.5) * cf.inv_h;
        const T lap = (gsum - T(6) * gf(v0)) * cf.inv_h2;
        q[m][r] = cf.pe_cn2 * (h0[m][r] * cf.inv_dt - A) + lap;
        if constexpr (SPLIT) W[zb + (int64_t)row_of(r) * nx + i] = q[m][r];
      }
    }
    // plane z+1 follows in this chunk: request what it needs beyond what is held, after the stencil
    // (measured: 6 % faster than before it, with the same registers)
    if (more) {
      load_c(z + 2);
      load_f(z + 1);
      if (patch) {
        load_p(n_lo, n_hi);
        range_of(min(z + 2, zlast), nn_lo, nn_hi);   // (not used past the chunk's last plane)
      }
    }
    if constexpr (SPLIT) {
      __syncthreads();   // every x-neighbour read of this plane is done before the next write
      if (more) rotate();
    } else {
#pragma unroll
    for (int m = 0; m < XM; ++m)
#pragma unroll
      for (int r = 0; r < L; ++r) {
        const int i = tid + 256 * m;
        fb[r * pitch + i + (i >> 4)] = q[m][r];
      }
    __syncthreads();
    const int64_t line0 = (int64_t)z * dm.ny + y0;
    if (patch && e_hi > e_lo) {
#pragma unroll
      for (int k = 0; k < PF; ++k)
        if (e_lo + tid + 256 * k < e_hi) {
          const int l = (int)((pc[k] >> lnx) - line0);
          const int i = pc[k] & (nx - 1);
          fb[l * pitch + i + (i >> 4)] += pd[k];
        }
      if (e_hi - e_lo > PF * 256) patch_tile(fb, rp, line0, lnx, pitch, e_lo + PF * 256, e_hi);
      __syncthreads();
    }
    lds_fft<T, L * 256 * XM, false, R>(fb, lnx, ilog2c(L) - 1, 2 * pitch, 1, pitch, 1, false, tw, tw + nx);
    // (the FFT's final barrier also protects the LDS plane buffers for the next plane's writes)
    if (more) rotate();
    const int half = (L * nx) >> 1;
    for (int e = tid; e < half; e += blockDim.x) {
      const int b = e >> lnx;
      const int kx = e & (nx - 1);
      const int kk = (nx - kx) & (nx - 1);
      const T *pb = fb + b * 2 * pitch;
      const int ak = kx + (kx >> 4), an = kk + (kk >> 4);
      const T p = pb[ak], qq = pb[pitch + ak], rr = pb[an], sv = pb[pitch + an];
      T *o = W + (line0 + 2 * b) * nx + kx;
      __builtin_nontemporal_store((p - qq + rr + sv) * T(0.5), o);
      __builtin_nontemporal_store((p + qq - rr + sv) * T(0.5), o + nx);
    }
    }
  }
}

// K5 (and the forward x pass of the SOLVE stage): Hartley transform of L consecutive
// contiguous lines of length nx from `in` to `out`.
template <typename T, int E, int MAXR = 16, int CLN = 0, int CLB = 0>
__device__ __forceinline__ void xdht_body(unsigned char *smem_raw, const T *__restrict__ in, T *__restrict__ out, int lnx,
                                                   int logL, const T *__restrict__ twr, const T *__restrict__ twi, int tile) {
  if constexpr (CLN != 0) lnx = CLN;   // compile-time line length and tile height (see neumann_body)
  if constexpr (CLB != 0) logL = CLB;
  T *s = reinterpret_cast<T *>(smem_raw);
  const int L = 1 << logL;
  const int nx = 1 << lnx;
  const int line0 = tile * L;
  const int tot = L << lnx;
  const int pitch = line_pitch(nx);
  const T *src = in + (int64_t)line0 * nx;
  // (streaming reads: the input is not read again by this pass or the next one)
  constexpr int CP = 16 / (int)sizeof(T);
  typedef T FV __attribute__((ext_vector_type(CP)));
  if constexpr (CLN != 0 && CLB != 0) {
    // fixed size: 16 bytes per thread and every RS-th line, so that offsets step by constants
    constexpr int RS = (CP * kThreads) >> CLN, KR = (1 << CLB) / RS;
    static_assert(RS >= 1 && KR * RS == (1 << CLB), "fixed-size tile");
    const int i = (threadIdx.x & ((1 << CLN) / CP - 1)) * CP, l0 = threadIdx.x / ((1 << CLN) / CP);
    FV v[KR];
#pragma unroll
    for (int k = 0; k < KR; ++k)
      v[k] = __builtin_nontemporal_load(reinterpret_cast<const FV *>(src + (l0 + k * RS) * (1 << CLN) + i));
#pragma unroll
    for (int k = 0; k < KR; ++k) {
      T *d = s + (l0 + k * RS) * pitch + i + (i >> 4);   // CP elements of one padding group
      const T *e = reinterpret_cast<const T *>(&v[k]);
#pragma unroll
      for (int c = 0; c < CP; ++c) d[c] = e[c];
    }
  } else {
    stage_tile(s, tot, [&](int e) { return __builtin_nontemporal_load(src + e); }, [&](int e) {
      const int l = e >> lnx, i = e & (nx - 1);
      return l * pitch + i + (i >> 4);
    });
  }
  __syncthreads();
  lds_fft<T, E, false, MAXR>(s, lnx, logL - 1, 2 * pitch, 1, pitch, 1, false, twr, twi);
  T *dst = out + (int64_t)line0 * nx;
  const int half = tot >> 1;
  for (int e = threadIdx.x; e < half; e += blockDim.x) {
    const int b = e >> lnx;
    const int kx = e & (nx - 1);
    const int kk = (nx - kx) & (nx - 1);
    const T *pb = s + b * 2 * pitch;
    const int ak = kx + (kx >> 4), an = kk + (kk >> 4);
    const T p = pb[ak], q = pb[pitch + ak], r = pb[an], sv = pb[pitch + an];
    T *o = dst + (int64_t)(2 * b) * nx + kx;
    o[0] = (p - q + r + sv) * T(0.5);
    o[nx] = (p + q - r + sv) * T(0.5);
  }
}

template <typename T, int E, int MAXR = 16, int CLN = 0, int CLB = 0>
__global__ __launch_bounds__(kThreads) void k_xdht(const T *__restrict__ in, T *__restrict__ out, int lnx,
                                                   int logL, const T *__restrict__ twr, const T *__restrict__ twi) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  xdht_body<T, E, MAXR, CLN, CLB>(smem_raw, in, out, lnx, logL, twr, twi, xcd_tile(blockIdx.x, gridDim.x));
}

template <typename T> struct Vec2;
template <> struct Vec2<double> { using type = double2; };
template <> struct Vec2<float> { using type = float2; };

// K2/K4: in-place Hartley transform along a strided axis of length N = 2^logN.  A tile is
// B = 2^logB adjacent x-columns (contiguous in memory) times N positions; tile t covers
// base = (t >> lognxb) * outer + (t & (nxb-1)) * B, element n at base + n*stride.  Columns
// 2b and 2b+1 form the pair b (real and imaginary parts of one complex line).
template <typename T, int E, int MAXR = 16, int CLN = 0, int CLB = 0>
__global__ __launch_bounds__(kThreads) void k_strided_dht(T *__restrict__ W, int logN, int64_t stride, int logB,
                                                          int lognxb, int64_t outer, const T *__restrict__ twr,
                                                          const T *__restrict__ twi) {
  if constexpr (CLN != 0) logN = CLN;   // compile-time line length and tile width (see neumann_body)
  if constexpr (CLB != 0) logB = CLB;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *s = reinterpret_cast<T *>(smem_raw);
  using V2 = typename Vec2<T>::type;
  const int N = 1 << logN, B = 1 << logB;
  const int t = xcd_tile(blockIdx.x, gridDim.x);
  const int64_t base = (int64_t)(t >> lognxb) * outer + (int64_t)(t & ((1 << lognxb) - 1)) * B;
  const int tot = N << logB;
  // fixed size (as in neumann_body): 16 bytes of adjacent columns per thread, every RS-th position,
  // unsigned 32-bit byte offsets from a uniform base (the caller bounds N * stride * sizeof(T))
  using FV = std::conditional_t<sizeof(T) == 8, double2, float4>;
  constexpr int CP = 16 / (int)sizeof(T);
  constexpr int RS = CLB ? (CP * kThreads) >> CLB : 16, KR = CLN ? (1 << CLN) / RS : 1;
  char *const gb = reinterpret_cast<char *>(W + base);
  if constexpr (CLN != 0 && CLB != 0) {
    static_assert(RS % 16 == 0 && KR * RS == (1 << CLN), "fixed-size tile");
    const int fcol = (threadIdx.x & ((B / CP) - 1)) * CP, fn0 = threadIdx.x / (B / CP);
    const unsigned foff = ((unsigned)fn0 * (unsigned)stride + (unsigned)fcol) * (unsigned)sizeof(T);
    const unsigned fstep = (unsigned)RS * (unsigned)stride * (unsigned)sizeof(T);
    const int fa0 = fn0 * B + (fn0 >> 4) * 2 + fcol, fda = RS * B + (RS >> 4) * 2;
    FV v[KR];
#pragma unroll
    for (int k = 0; k < KR; ++k) v[k] = *reinterpret_cast<const FV *>(gb + (foff + k * fstep));
#pragma unroll
    for (int k = 0; k < KR; ++k) lds_put16(s + fa0 + k * fda, v[k]);
  } else {
    stage_tile(s, tot, [&](int e) { return W[base + (e >> logB) * stride + (e & (B - 1))]; }, [&](int e) {
      const int n = e >> logB, col = e & (B - 1);
      return n * B + (n >> 4) * 2 + col;
    });
  }
  __syncthreads();
  lds_fft<T, E, false, MAXR, 256, true>(s, logN, logB - 1, 2, B, 1, 2, true, twr, twi);
  const int lp = logB - 1;
  const int half = tot >> 1;
  if constexpr (CLN != 0 && CLB != 0) {
    // one column pair per thread, every RO-th position; the offset is made opaque so that the
    // compiler forms these addresses here rather than holding them from the staging loads
    constexpr int RO = (2 * kThreads) >> CLB, KO = (1 << CLN) / RO;
    const int b = threadIdx.x & ((B >> 1) - 1), n0 = threadIdx.x >> (logB - 1);
    unsigned ooff = ((unsigned)n0 * (unsigned)stride + 2u * b) * (unsigned)sizeof(T);
    const unsigned ostep = (unsigned)RO * (unsigned)stride * (unsigned)sizeof(T);
    asm volatile("" : "+v"(ooff));
#pragma unroll
    for (int j = 0; j < KO; ++j) {
      const int n = n0 + j * RO;
      const int nn = (N - n) & (N - 1);
      const V2 u0 = *reinterpret_cast<const V2 *>(s + n * B + (n >> 4) * 2 + 2 * b);
      const V2 u1 = *reinterpret_cast<const V2 *>(s + nn * B + (nn >> 4) * 2 + 2 * b);
      V2 v;
      v.x = (u0.x - u0.y + u1.x + u1.y) * T(0.5);
      v.y = (u0.x + u0.y - u1.x + u1.y) * T(0.5);
      *reinterpret_cast<V2 *>(gb + (ooff + j * ostep)) = v;
    }
    return;
  }
  for (int e = threadIdx.x; e < half; e += blockDim.x) {
    const int b = e & ((1 << lp) - 1), n = e >> lp;
    const int nn = (N - n) & (N - 1);
    const int a0 = n * B + (n >> 4) * 2 + 2 * b, a1 = nn * B + (nn >> 4) * 2 + 2 * b;
    const V2 u0 = *reinterpret_cast<const V2 *>(s + a0), u1 = *reinterpret_cast<const V2 *>(s + a1);
    const T p = u0.x, q = u0.y;
    const T r = u1.x, sv = u1.y;
    V2 v;
    v.x = (p - q + r + sv) * T(0.5);
    v.y = (p + q - r + sv) * T(0.5);
    *reinterpret_cast<V2 *>(W + base + n * stride + 2 * b) = v;
  }
}

// K3: along the bounded axis, per column: DCT-II (even/odd reorder + FFT + post-twiddle),
// division by (lam - a)(lam + alpha_s) times the inverse normalisation, inverse DCT-II
// (pre-twiddle + inverse FFT + reorder).  lam = lamx[kx] (+ lamy[ky]) + lamz[kz].
template <typename T, int E, int MAXR = 16, int CLN = 0, int CLB = 0>
__device__ __forceinline__ void neumann_body(unsigned char *smem_raw, T *__restrict__ W, int logN, int64_t stride, int logB,
                                                            int lognxb, int64_t outer, const T *__restrict__ lamx,
                                                            const T *__restrict__ lamy, const T *__restrict__ lamz,
                                                            T a, T alpha_s, T inv_norm, const T *__restrict__ twr,
                                                            const T *__restrict__ twi, const T *__restrict__ dctc,
                                                            const T *__restrict__ dcts, int tile, int poisson) {
  // CLN/CLB != 0 fix the line length and the tile width at compile time, so that the FFT's
  // LDS addresses fold into instruction offsets
  if constexpr (CLN != 0) logN = CLN;
  if constexpr (CLB != 0) logB = CLB;
  T *s = reinterpret_cast<T *>(smem_raw);
  const int N = 1 << logN, B = 1 << logB;
  const int t = tile;
  const int xb = t & ((1 << lognxb) - 1);
  const int oy = t >> lognxb;
  const int64_t base = (int64_t)oy * outer + (int64_t)xb * B;
  const int tot = N << logB;
  // fixed size: a thread keeps 16 bytes of adjacent columns and every (CP kThreads / B)-th
  // position, so its global offsets step by a constant (unsigned 32-bit bytes from a uniform base:
  // the caller bounds N * stride * sizeof(T)) and, the step being even, all its positions share one parity and
  // land on reordered slots a constant LDS distance apart (16 positions, one padding group)
  using FV = std::conditional_t<sizeof(T) == 8, double2, float4>;
  constexpr int CP = 16 / (int)sizeof(T);
  constexpr int RS = CLB ? (CP * kThreads) >> CLB : 2, KR = CLN ? (1 << CLN) / RS : 1;
  const int fcol = (threadIdx.x & ((B / CP) - 1)) * CP, fn0 = threadIdx.x / (B / CP);
  const int fp0 = (fn0 & 1) ? N - 1 - (fn0 >> 1) : fn0 >> 1;
  const int fa0 = fp0 * B + (fp0 >> 4) * 2 + fcol;
  const int fda = (fn0 & 1) ? -((RS / 2) * B + 2) : (RS / 2) * B + 2;
  unsigned foff = ((unsigned)fn0 * (unsigned)stride + (unsigned)fcol) * (unsigned)sizeof(T);   // bytes
  const unsigned fstep = (unsigned)RS * (unsigned)stride * (unsigned)sizeof(T);
  char *const gb = reinterpret_cast<char *>(W + base);
  if constexpr (CLN != 0 && CLB != 0) {
    static_assert(RS == 32 && KR * RS == (1 << CLN), "fixed-size tile");
    FV v[KR];
#pragma unroll
    for (int k = 0; k < KR; ++k) v[k] = *reinterpret_cast<const FV *>(gb + (foff + k * fstep));
#pragma unroll
    for (int k = 0; k < KR; ++k) lds_put16(s + fa0 + k * fda, v[k]);
  } else {
    stage_tile(s, tot, [&](int e) { return W[base + (e >> logB) * stride + (e & (B - 1))]; }, [&](int e) {
      const int n = e >> logB, col = e & (B - 1);
      const int pos = (n & 1) ? (N - 1 - (n >> 1)) : (n >> 1);
      return pos * B + (pos >> 4) * 2 + col;
    });
  }
  __syncthreads();
  lds_fft<T, E, false, MAXR, 256, true>(s, logN, logB - 1, 2, B, 1, 2, true, twr, twi);
  const int half = N >> 1;
  const int lpairs = logB - 1;   // B / 2 column pairs per position
  const int items = (half + 1) << lpairs;
  const T lam_y = lamy ? lamy[oy] : T(0);
  const T hnorm = inv_norm * T(0.5);
  // the pressure (POIS) divides by lam itself and drops the mean mode (lam = 0); the order
  // parameter divides by (lam - a)(lam + alpha_s), which is never zero, so the four divisors of
  // an item share divisions: 1/d1 = d2 / (d1 d2) and so on, in FP64 even 1/(d1 d2) = d3 d4 / (d1 d2 d3 d4)
  auto solve = [&](auto pois) {
    constexpr bool POIS = decltype(pois)::value;
    for (int e = threadIdx.x; e < items; e += blockDim.x) {
      const int b = e & ((1 << lpairs) - 1);
      const int k = e >> lpairs;
      const int kk = (N - k) & (N - 1);
      using V2 = typename Pair2<T>::type;
      T *zk = s + k * B + (k >> 4) * 2 + 2 * b;
      T *zn = s + kk * B + (kk >> 4) * 2 + 2 * b;
      const V2 uk = *reinterpret_cast<const V2 *>(zk), un = *reinterpret_cast<const V2 *>(zn);
      const T p = uk.x, q = uk.y, r = un.x, sv = un.y;
      // (the spectra of the two columns are (p + r, q - sv)/2 and (q + sv, r - p)/2; the halves,
      // the doubling below and the final halving are exact powers of two and fold into hnorm)
      const T var = p + r, vai = q - sv;
      const T vbr = q + sv, vbi = r - p;
      const T c = dctc[k], sn = dcts[k];
      const int kxa = xb * B + 2 * b;
      const T la = lamx[kxa] + lam_y, lb = lamx[kxa + 1] + lam_y;
      const T lk = lamz[k];
      const T lnk = k ? lamz[N - k] : T(0);
      // cosine-transform coefficients X[k], X[N-k] of both columns
      T xa1 = c * var + sn * vai, xa2 = sn * var - c * vai;
      T xb1 = c * vbr + sn * vbi, xb2 = sn * vbr - c * vbi;
      if constexpr (POIS) {
        auto fac = [&](T l) { return l != T(0) ? hnorm / l : T(0); };
        xa1 *= fac(la + lk);
        xb1 *= fac(lb + lk);
        xa2 = k ? xa2 * fac(la + lnk) : T(0);
        xb2 = k ? xb2 * fac(lb + lnk) : T(0);
      } else {
        auto den = [&](T l) { return (l - a) * (l + alpha_s); };
        const T d1 = den(la + lk), d2 = den(lb + lk), d3 = den(la + lnk), d4 = den(lb + lnk);
        const T p12 = d1 * d2, p34 = d3 * d4;
        T r12, r34;
        if constexpr (sizeof(T) == 8) {   // one division (the product of four stays far inside FP64)
          const T rr = hnorm / (p12 * p34);
          r12 = rr * p34;
          r34 = rr * p12;
        } else {                          // two (in FP32 the product of four can underflow the quotient)
          r12 = hnorm / p12;
          r34 = hnorm / p34;
        }
        xa1 *= r12 * d2;
        xb1 *= r12 * d1;
        xa2 = k ? xa2 * (r34 * d4) : T(0);
        xb2 = k ? xb2 * (r34 * d3) : T(0);
      }
      // back to the reordered-sequence spectrum: V'[k] = e^{i pi k/2N} (X[k] - i X[N-k]) / 2
      const T a1 = c * xa1 + sn * xa2, a2 = sn * xa1 - c * xa2;
      const T b1 = c * xb1 + sn * xb2, b2 = sn * xb1 - c * xb2;
      V2 ok;
      ok.x = a1 - b2;
      ok.y = a2 + b1;
      *reinterpret_cast<V2 *>(zk) = ok;
      if (k != 0 && k != half) {
        V2 on;
        on.x = a1 + b2;
        on.y = b1 - a2;
        *reinterpret_cast<V2 *>(zn) = on;
      }
    }
  };
  if (poisson) solve(std::true_type{});
  else solve(std::false_type{});
  __syncthreads();
  lds_fft<T, E, true, MAXR, 256, true>(s, logN, logB - 1, 2, B, 1, 2, true, twr, twi);
  if constexpr (CLN != 0 && CLB != 0) {
    // (an empty asm makes the offset opaque here, so the compiler forms these addresses now
    // instead of holding the staging loads' addresses in registers through the whole solve)
    asm volatile("" : "+v"(foff));
#pragma unroll
    for (int k = 0; k < KR; ++k)
      *reinterpret_cast<FV *>(gb + (foff + k * fstep)) = lds_get16<FV>(s + fa0 + k * fda);
  } else {
    for (int e = threadIdx.x; e < tot; e += blockDim.x) {
      const int n = e >> logB, col = e & (B - 1);
      const int pos = (n & 1) ? (N - 1 - (n >> 1)) : (n >> 1);
      W[base + n * stride + col] = s[pos * B + (pos >> 4) * 2 + col];
    }
  }
}

// The fixed-size instance is held to 128 VGPRs (4 waves per SIMD, as the LDS tile allows): the
// constant addresses free the compiler to hoist more, and at 3 waves it runs no faster.
template <typename T, int E, int MAXR = 16, int CLN = 0, int CLB = 0>
__global__ __launch_bounds__(kThreads, CLN ? 4 : 1) void k_neumann_solve(T *__restrict__ W, int logN, int64_t stride, int logB,
                                                            int lognxb, int64_t outer, const T *__restrict__ lamx,
                                                            const T *__restrict__ lamy, const T *__restrict__ lamz,
                                                            T a, T alpha_s, T inv_norm, const T *__restrict__ twr,
                                                            const T *__restrict__ twi, const T *__restrict__ dctc,
                                                            const T *__restrict__ dcts, int poisson) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  neumann_body<T, E, MAXR, CLN, CLB>(smem_raw, W, logN, stride, logB, lognxb, outer, lamx, lamy, lamz, a, alpha_s, inv_norm, twr, twi, dctc, dcts, xcd_tile(blockIdx.x, gridDim.x), poisson);
}

// ---------------------------------------------------------------------------------------
// Ghost-cell helpers.

template <typename T>
__device__ __forceinline__ T mirror_gather(const T *__restrict__ f, const int *__restrict__ ap,
                                           const T *__restrict__ w, int64_t g, int64_t G, int K) {
  T o1 = T(0), o2 = T(0);
  for (int k = 0; k < K; ++k) o1 += w[(int64_t)k * G + g] * f[ap[(int64_t)k * G + g]];
  for (int k = 0; k < K; ++k) o2 += w[(int64_t)(K + k) * G + g] * f[ap[(int64_t)(K + k) * G + g]];
  return T(2) * o1 - o2;
}

// Central-difference gradient at a cell (periodic axes wrap, the bounded axis reflects).
template <typename T>
__device__ __forceinline__ void grad_at(const T *__restrict__ f, int64_t c, const Dims &dm, int d, T inv2h, T *g) {
  const int i = (int)(c & (dm.nx - 1));
  const int64_t r = c >> dm.lnx;
  const int j = (int)(r & (dm.ny - 1));
  const int k = (int)(r >> dm.lny);
  const int64_t rowb = c - i;
  g[0] = (f[rowb + ((i + 1) & (dm.nx - 1))] - f[rowb + ((i - 1) & (dm.nx - 1))]) * inv2h;
  if (d == 2) {
    const int64_t up = j < dm.ny - 1 ? c + dm.nx : c;
    const int64_t dnn = j > 0 ? c - dm.nx : c;
    g[1] = (f[up] - f[dnn]) * inv2h;
  } else {
    const int jp = (j + 1) & (dm.ny - 1), jm = (j - 1) & (dm.ny - 1);
    g[1] = (f[c + (int64_t)(jp - j) * dm.nx] - f[c + (int64_t)(jm - j) * dm.nx]) * inv2h;
    const int64_t up = k < dm.nz - 1 ? c + dm.plane : c;
    const int64_t dnn = k > 0 ? c - dm.plane : c;
    g[2] = (f[up] - f[dnn]) * inv2h;
  }
}

// Cell-centred velocity component a: mean of the two faces along a (box-wall faces read 0).
template <typename T>
__device__ __forceinline__ T centred_u(const T *__restrict__ Fa, int64_t c, int a, const Dims &dm, int d) {
  int64_t step;
  int idx, n;
  const int i = (int)(c & (dm.nx - 1));
  const int64_t r = c >> dm.lnx;
  const int j = (int)(r & (dm.ny - 1));
  const int k = (int)(r >> dm.lny);
  if (a == 0) {
    const int64_t rowb = c - i;
    return T(0.5) * (Fa[rowb + ((i - 1) & (dm.nx - 1))] + Fa[c]);
  }
  if (a == 1) {
    step = dm.nx;
    idx = j;
    n = dm.ny;
  } else {
    step = dm.plane;
    idx = k;
    n = dm.nz;
  }
  if (a < d - 1) {  // periodic y in 3D
    const int jm = (j - 1) & (dm.ny - 1);
    return T(0.5) * (Fa[c + (int64_t)(jm - j) * dm.nx] + Fa[c]);
  }
  const T lo = idx > 0 ? Fa[c - step] : T(0);
  const T hi = idx < n - 1 ? Fa[c] : T(0);
  return T(0.5) * (lo + hi);
}

// Sum over the 16 lanes of an aligned lane group (fixed order: deterministic).
template <typename T>
__device__ __forceinline__ T group16_sum(T v) {
  v += __shfl_xor(v, 8);
  v += __shfl_xor(v, 4);
  v += __shfl_xor(v, 2);
  v += __shfl_xor(v, 1);
  return v;
}

// K6 (static condition, no contact-line friction): per ghost, C_M = 2 IDW(IP1) - IDW(IP2),
// then the wall relation of Eq. WallBCS with mu_f = 0, dC/dn = -cos(theta)(1 - C^2)/(sqrt2 Cn),
// integrated exactly from M back to I: C_I = (C_M + t)/(1 + t C_M), t = tanh(b),
// b = gamma dn cos(theta)/(sqrt2 Cn), C_M taken inside [-1, 1]; C_G = ((gamma+1) C_I - C_M)/gamma
// (Eq. UpdateC).
// Sixteen lanes per ghost: lane s < 2K gathers one weighted averaging point.
template <typename T>
__device__ __forceinline__ void fill_static_body(T *__restrict__ C, const int *__restrict__ gidx,
                                                          const T *__restrict__ dn, const T *__restrict__ gam,
                                                          const int *__restrict__ ap, const T *__restrict__ w,
                                                          T *__restrict__ CGn, T *__restrict__ CGnm1,
                                                          T *__restrict__ CMs, int64_t G, int K, T cb, int init, int64_t tile) {
  const int64_t g = ((int64_t)tile * blockDim.x + threadIdx.x) >> 4;
  const int sl = threadIdx.x & 15;
  // the ghost's own table entries are requested with the gather, not after the lane sum
  const int64_t gs = g < G ? g : G - 1;
  const T ga = gam[gs], dng = dn[gs];
  const int cgi = gidx[gs];
  T v = T(0);
  if (g < G && sl < 2 * K) {
    const int64_t i = g * kGhostSlots + sl;
    v = (sl < K ? T(2) : T(-1)) * w[i] * C[ap[i]];
  }
  const T CM = group16_sum(v);
  if (g >= G || sl != 0) return;
  const T t = tanh(ga * dng * cb);
  const T Mc = CM > T(1) ? T(1) : (CM < T(-1) ? T(-1) : CM);
  const T CI = (Mc + t) / (T(1) + t * Mc);
  const T CG = ((ga + T(1)) * CI - CM) / ga;
  C[cgi] = CG;
  CMs[g] = CM;
  if (init != 2) CGnm1[g] = init ? CG : CGn[g];   // 2: refresh within a step, history kept
  CGn[g] = CG;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_fill_static(T *__restrict__ C, const int *__restrict__ gidx,
                                                          const T *__restrict__ dn, const T *__restrict__ gam,
                                                          const int *__restrict__ ap, const T *__restrict__ w,
                                                          T *__restrict__ CGn, T *__restrict__ CGnm1,
                                                          T *__restrict__ CMs, int64_t G, int K, T cb, int init) {
  fill_static_body<T>(C, gidx, dn, gam, ap, w, CGn, CGnm1, CMs, G, K, cb, init, blockIdx.x);
}

// Dynamic condition, part 1: provisional ghost values C^_G = 2 C^n_G - C^(n-1)_G.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_scatter_pg(T *__restrict__ C, const int *__restrict__ gidx,
                                                         const T *__restrict__ CGn, const T *__restrict__ CGnm1,
                                                         int64_t G) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= G) return;
  C[gidx[g]] = T(2) * CGn[g] - CGnm1[g];
}

// Dynamic condition, part 2 (Eqs. interpolationAtWall, ProjectingToNT, WallBCS_recast):
// C_I <- C_I + dt [ -u_I . grad_t C_I + Vs (Cn dC/dn + cos(theta)(1 - C_I*^2)/sqrt2) ],
// C_I* = (gamma C^_G + C_M)/(gamma+1), dC/dn = (C_M - C^_G)/((1+gamma) dn); then
// C_G = ((gamma+1) C_I - C_M)/gamma.  All reads from the provisional field (Jacobi).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_fill_dynamic(
    const T *__restrict__ C, const T *__restrict__ F0, const T *__restrict__ F1, const T *__restrict__ F2,
    const int *__restrict__ gidx, const T *__restrict__ nrm, const T *__restrict__ dn, const T *__restrict__ gam,
    const int *__restrict__ ap, const T *__restrict__ w, T *__restrict__ CI, T *__restrict__ CGnew,
    T *__restrict__ CMs, int64_t G, int K, Dims dm, int d, T inv2h, T Cn, T Vs, T cos_t, T dt, int init) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= G) return;
  const int64_t cg = gidx[g];
  const T PG = C[cg];
  const T CM = mirror_gather(C, ap, w, g, G, K);
  const T ga = gam[g];
  const T CIs = (ga * PG + CM) / (ga + T(1));
  CMs[g] = CM;
  if (init) {
    CI[g] = CIs;
    CGnew[g] = PG;
    return;
  }
  T gG[3] = {0, 0, 0}, gM[3] = {0, 0, 0}, n[3] = {0, 0, 0}, uG[3] = {0, 0, 0}, uM[3] = {0, 0, 0};
  grad_at(C, cg, dm, d, inv2h, gG);
  const T *Fs[3] = {F0, F1, F2};
  for (int jp = 0; jp < 2; ++jp) {
    const T coef = jp == 0 ? T(2) : T(-1);
    for (int k = 0; k < K; ++k) {
      const int64_t sl = (int64_t)(jp * K + k) * G + g;
      const T wk = w[sl];
      const int64_t c = ap[sl];
      T gk[3];
      grad_at(C, c, dm, d, inv2h, gk);
      for (int a = 0; a < d; ++a) {
        gM[a] += coef * wk * gk[a];
        uM[a] += coef * wk * centred_u(Fs[a], c, a, dm, d);
      }
    }
  }
  T gn = T(0), un = T(0);
  for (int a = 0; a < d; ++a) {
    n[a] = nrm[(int64_t)a * G + g];
    uG[a] = centred_u(Fs[a], cg, a, dm, d);
  }
  T gI[3], uI[3];
  for (int a = 0; a < d; ++a) {
    gI[a] = (ga * gG[a] + gM[a]) / (ga + T(1));
    uI[a] = (ga * uG[a] + uM[a]) / (ga + T(1));
    gn += gI[a] * n[a];
  }
  T adv = T(0);
  for (int a = 0; a < d; ++a) adv += uI[a] * (gI[a] - gn * n[a]);
  (void)un;
  const T dCdn = (CM - PG) / ((T(1) + ga) * dn[g]);
  const T rhs = -adv + Vs * (Cn * dCdn + cos_t * (T(1) - CIs * CIs) * T(0.70710678118654752440));
  const T ci = CI[g] + dt * rhs;
  CI[g] = ci;
  CGnew[g] = ((ga + T(1)) * ci - CM) / ga;
}

// Dynamic condition, part 3: write the new ghost values and rotate the per-ghost history.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_commit_ghosts(T *__restrict__ C, const int *__restrict__ gidx,
                                                            const T *__restrict__ CGnew, T *__restrict__ CGn,
                                                            T *__restrict__ CGnm1, int64_t G, int init) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= G) return;
  const T v = CGnew[g];
  C[gidx[g]] = v;
  CGnm1[g] = init ? v : CGn[g];
  CGn[g] = v;
}

// Explicit chemical potential phi~ = C~^3 - C~ - Cn^2 lap_h C~ of the semi-implicit step at one cell,
// C~ = 2C^n - C^(n-1); periodic axes wrap, the bounded axis reflects (the Laplacian of the solve).
template <typename T>
__device__ __forceinline__ T phit_at(const T *__restrict__ Cn, const T *__restrict__ Cp, int64_t c, const Dims &dm,
                                     int d, T cn2, T inv_h2) {
  auto ct = [&](int64_t q) { return T(2) * Cn[q] - Cp[q]; };
  const int i = (int)(c & (dm.nx - 1));
  const int64_t r = c >> dm.lnx;
  const int j = (int)(r & (dm.ny - 1));
  const int k = (int)(r >> dm.lny);
  const int64_t rowb = c - i;
  const T v = ct(c);
  T acc = ct(rowb + ((i + 1) & (dm.nx - 1))) + ct(rowb + ((i - 1) & (dm.nx - 1)));
  if (d == 2) {
    acc = acc + (j < dm.ny - 1 ? ct(c + dm.nx) : v);
    acc = acc + (j > 0 ? ct(c - dm.nx) : v);
  } else {
    const int jp = (j + 1) & (dm.ny - 1), jm = (j - 1) & (dm.ny - 1);
    acc = acc + ct(c + (int64_t)(jp - j) * dm.nx);
    acc = acc + ct(c + (int64_t)(jm - j) * dm.nx);
    acc = acc + (k < dm.nz - 1 ? ct(c + dm.plane) : v);
    acc = acc + (k > 0 ? ct(c - dm.plane) : v);
  }
  const T lap = (acc - T(2 * d) * v) * inv_h2;
  return v * v * v - v - cn2 * lap;
}

// The wall condition dphi/dn = 0 of the semi-implicit step (end of section 4.2.2, Eq. WallBCS):
// per ghost, dg = (phi~_M - phi~_G)/Cn^2 with phi~_M = 2 IDW(IP1) - IDW(IP2) of phi~ (Eq.
// extrapolation).  Sixteen lanes per ghost: lane s < 2K one weighted averaging point, lane 2K
// the ghost itself; fixed-order lane-group sum.
template <typename T>
__device__ __forceinline__ void ghost_dphi_body(const T *__restrict__ Cn, const T *__restrict__ Cp,
                                                const int *__restrict__ gidx, const int *__restrict__ ap,
                                                const T *__restrict__ w, T *__restrict__ dg, int64_t G, int K,
                                                const Dims &dm, int d, T cn2, T inv_h2, T inv_cn2, int64_t tile) {
  const int64_t g = ((int64_t)tile * blockDim.x + threadIdx.x) >> 4;
  const int sl = threadIdx.x & 15;
  T v = T(0);
  if (g < G && sl <= 2 * K) {
    int64_t c;
    T coef;
    if (sl < 2 * K) {
      const int64_t i = g * kGhostSlots + sl;
      c = ap[i];
      coef = (sl < K ? T(2) : T(-1)) * w[i];
    } else {
      c = gidx[g];
      coef = T(-1);
    }
    v = coef * phit_at(Cn, Cp, c, dm, d, cn2, inv_h2);
  }
  const T sum = group16_sum(v);
  if (g < G && sl == 0) dg[g] = sum * inv_cn2;
}

// The same dg from phi~ evaluated once per listed point (many ghosts share averaging points):
// k_point_phit takes one point per thread (the list is sorted by cell, so neighbouring threads read
// neighbouring cells), k_ghost_dg gathers those values per ghost.  Each product and the lane sum are
// those of ghost_dphi_body, in the same order, so both give the same bits.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_point_phit(const T *__restrict__ Cn, const T *__restrict__ Cp,
                                                         const int *__restrict__ pt_cell, T *__restrict__ pt_phi,
                                                         int64_t nu, Dims dm, int d, T cn2, T inv_h2) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u < nu) pt_phi[u] = phit_at(Cn, Cp, (int64_t)pt_cell[u], dm, d, cn2, inv_h2);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_ghost_dg(const T *__restrict__ pt_phi, const int *__restrict__ pt_idx,
                                                       const T *__restrict__ w, T *__restrict__ dg, int64_t G, int K,
                                                       T inv_cn2) {
  const int64_t g = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4;
  const int sl = threadIdx.x & 15;
  T v = T(0);
  if (g < G && sl <= 2 * K) {
    const int64_t i = g * kGhostSlots + sl;
    const T coef = sl < 2 * K ? (sl < K ? T(2) : T(-1)) * w[i] : T(-1);
    v = coef * pt_phi[pt_idx[i]];
  }
  const T sum = group16_sum(v);
  if (g < G && sl == 0) dg[g] = sum * inv_cn2;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_ghost_dphi(const T *__restrict__ Cn, const T *__restrict__ Cp,
                                                         const int *__restrict__ gidx, const int *__restrict__ ap,
                                                         const T *__restrict__ w, T *__restrict__ dg, int64_t G,
                                                         int K, Dims dm, int d, T cn2, T inv_h2, T inv_cn2) {
  ghost_dphi_body<T>(Cn, Cp, gidx, ap, w, dg, G, K, dm, d, cn2, inv_h2, inv_cn2, blockIdx.x);
}

// The rhs patch of every listed cell: dq = (sum of the neighbouring ghosts' dg - 2d dg_own)/h^2,
// the neighbours in a fixed order (+e_a, -e_a per axis).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_patch_dq(const int *__restrict__ ref, const T *__restrict__ dg,
                                                       T *__restrict__ dq, int64_t np, int nref, T twod, T inv_h2) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= np) return;
  T acc = T(0);
  for (int j = 1; j < nref; ++j) {
    const int id = ref[(int64_t)j * np + e];
    if (id >= 0) acc += dg[id];
  }
  const int own = ref[e];
  if (own >= 0) acc -= twod * dg[own];
  dq[e] = acc * inv_h2;
}

// The patch added to a rhs stored cell by cell (stage entry point, stencil-only z-march).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_rhs_patch(T *__restrict__ Q, const int *__restrict__ cell,
                                                        const T *__restrict__ dq, int64_t np) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < np) Q[cell[e]] += dq[e];
}

// K7a: ghost velocities (Eqs. NoPenetration, UpdateVtan, UpdateVandW in vector form) and,
// for the faces touching ghosts, the cell-centred velocity of their non-ghost side, all
// from the faces as they are before this fill.  Blocks [0, nbg) take sixteen lanes per
// ghost (lane s < 2K: one averaging point's gradient and centred velocity, lane 2K: the
// ghost's own gradient); the remaining blocks take one face per thread.  With the static
// condition (capillary = 0) the wall equation makes the bracket Kc of Eq. UpdateVtan zero,
// and no gradient of C is gathered.
template <typename T>
__device__ __forceinline__ void vel_ghosts_body(
    const T *__restrict__ C, const T *__restrict__ F0, const T *__restrict__ F1, const T *__restrict__ F2,
    const int *__restrict__ gidx, const T *__restrict__ nrm, const T *__restrict__ dn, const T *__restrict__ gam,
    const int *__restrict__ ap, const T *__restrict__ w, const T *__restrict__ CMs, T *__restrict__ UG, int64_t G,
    int K, const int *__restrict__ f_cell, const int *__restrict__ f_axis, const int *__restrict__ f_gL,
    const int *__restrict__ f_gR, T *__restrict__ stashL, T *__restrict__ stashR, int64_t NF, Dims dm, int d,
    T inv2h, T Cn, T cos_t, T inv_Ca, T inv_mu, T ls, int capillary, unsigned nbg, int64_t tile) {
  const T *Fs[3] = {F0, F1, F2};
  if (tile >= nbg) {
    const int64_t f = (int64_t)(tile - nbg) * blockDim.x + threadIdx.x;
    if (f >= NF) return;
    const int a = f_axis[f];
    const int64_t cL = f_cell[f];
    int64_t cR;
    {
      const int i = (int)(cL & (dm.nx - 1));
      const int64_t r = cL >> dm.lnx;
      const int j = (int)(r & (dm.ny - 1));
      if (a == 0) cR = cL - i + ((i + 1) & (dm.nx - 1));
      else if (a == 1) cR = (d == 3) ? cL + (int64_t)(((j + 1) & (dm.ny - 1)) - j) * dm.nx : cL + dm.nx;
      else cR = cL + dm.plane;
    }
    stashL[f] = f_gL[f] < 0 ? centred_u(Fs[a], cL, a, dm, d) : T(0);
    stashR[f] = f_gR[f] < 0 ? centred_u(Fs[a], cR, a, dm, d) : T(0);
    return;
  }
  const int64_t g = ((int64_t)tile * blockDim.x + threadIdx.x) >> 4;
  const int sl = threadIdx.x & 15;
  // the ghost's own table entries are requested with the gathers, not after the lane sums
  const int64_t gs = g < G ? g : G - 1;
  const T ga = gam[gs], dng = dn[gs];
  T n[3] = {0, 0, 0};
  for (int a = 0; a < d; ++a) n[a] = nrm[(int64_t)a * G + gs];
  T gm[3] = {0, 0, 0}, um[3] = {0, 0, 0}, gg[3] = {0, 0, 0};
  if (g < G) {
    if (sl < 2 * K) {
      const int64_t i = g * kGhostSlots + sl;
      const T cw = (sl < K ? T(2) : T(-1)) * w[i];
      const int64_t c = ap[i];
      T gk[3] = {0, 0, 0};
      if (capillary) grad_at(C, c, dm, d, inv2h, gk);
      for (int a = 0; a < d; ++a) {
        gm[a] = cw * gk[a];
        um[a] = cw * centred_u(Fs[a], c, a, dm, d);
      }
    } else if (sl == 2 * K && capillary) {
      grad_at(C, (int64_t)gidx[g], dm, d, inv2h, gg);
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    gm[a] = group16_sum(gm[a]);
    um[a] = group16_sum(um[a]);
    gg[a] = group16_sum(gg[a]);
  }
  if (g >= G || sl != 0) return;
  T VnM = T(0), gIn = T(0), gI[3];
  for (int a = 0; a < d; ++a) {
    VnM += um[a] * n[a];
    gI[a] = (ga * gg[a] + gm[a]) / (ga + T(1));
    gIn += gI[a] * n[a];
  }
  const T VnG = -VnM / ga;
  T Kc = T(0);
  if (capillary) {   // only then are C and C_M read (the static fill may be writing them meanwhile)
    const T CG = C[gidx[g]], CM = CMs[g];
    const T CIv = (ga * CG + CM) / (ga + T(1));
    const T dCdn = (CM - CG) / ((T(1) + ga) * dng);
    Kc = (T(1.06066017177982128660) * Cn * dCdn + T(0.75) * cos_t * (T(1) - CIv * CIv)) * inv_Ca;
  }
  const T den = ls + ga * dng;
  const T fM = (ls - dng) / den;
  const T fK = ls * (ga + T(1)) * dng * inv_mu / den;
  for (int a = 0; a < d; ++a) {
    const T VtM = um[a] - VnM * n[a];
    const T gt = gI[a] - gIn * n[a];
    const T VtG = VtM * fM - Kc * gt * fK;
    UG[(int64_t)a * G + g] = VnG * n[a] + VtG;
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_vel_ghosts(
    const T *__restrict__ C, const T *__restrict__ F0, const T *__restrict__ F1, const T *__restrict__ F2,
    const int *__restrict__ gidx, const T *__restrict__ nrm, const T *__restrict__ dn, const T *__restrict__ gam,
    const int *__restrict__ ap, const T *__restrict__ w, const T *__restrict__ CMs, T *__restrict__ UG, int64_t G,
    int K, const int *__restrict__ f_cell, const int *__restrict__ f_axis, const int *__restrict__ f_gL,
    const int *__restrict__ f_gR, T *__restrict__ stashL, T *__restrict__ stashR, int64_t NF, Dims dm, int d,
    T inv2h, T Cn, T cos_t, T inv_Ca, T inv_mu, T ls, int capillary, unsigned nbg) {
  vel_ghosts_body<T>(C, F0, F1, F2, gidx, nrm, dn, gam, ap, w, CMs, UG, G, K, f_cell, f_axis, f_gL, f_gR, stashL, stashR, NF, dm, d, inv2h, Cn, cos_t, inv_Ca, inv_mu, ls, capillary, nbg, blockIdx.x);
}

// K6 + K7a in one launch for the static condition, where the velocity fill does not read C:
// blocks [0, nbc) fill the C ghosts, the others compute the ghost velocities and face stashes.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_fill_static_vel(
    T *__restrict__ C, const int *__restrict__ gidx, const T *__restrict__ dn, const T *__restrict__ gam,
    const int *__restrict__ ap, const T *__restrict__ w, T *__restrict__ CGn, T *__restrict__ CGnm1,
    T *__restrict__ CMs, int64_t G, int K, T cb, const T *__restrict__ F0, const T *__restrict__ F1,
    const T *__restrict__ F2, const T *__restrict__ nrm, T *__restrict__ UG, const int *__restrict__ f_cell,
    const int *__restrict__ f_axis, const int *__restrict__ f_gL, const int *__restrict__ f_gR, T *__restrict__ stashL,
    T *__restrict__ stashR, int64_t NF, Dims dm, int d, T inv2h, T Cn, T cos_t, T inv_Ca, T inv_mu, T ls,
    unsigned nbc, unsigned nbg) {
  if (blockIdx.x < nbc) {
    fill_static_body<T>(C, gidx, dn, gam, ap, w, CGn, CGnm1, CMs, G, K, cb, 0, blockIdx.x);
    return;
  }
  vel_ghosts_body<T>(C, F0, F1, F2, gidx, nrm, dn, gam, ap, w, CMs, UG, G, K, f_cell, f_axis, f_gL, f_gR, stashL,
                     stashR, NF, dm, d, inv2h, Cn, cos_t, inv_Ca, inv_mu, ls, 0, nbg, blockIdx.x - nbc);
}

// K7b: every face touching a ghost becomes the mean of its two cell-centred values.
template <typename T>
__device__ __forceinline__ void vel_faces_body(T *__restrict__ F0, T *__restrict__ F1, T *__restrict__ F2,
                                                        const T *__restrict__ UG, int64_t G,
                                                        const int *__restrict__ f_cell, const int *__restrict__ f_axis,
                                                        const int *__restrict__ f_gL, const int *__restrict__ f_gR,
                                                        const T *__restrict__ stashL, const T *__restrict__ stashR,
                                                        int64_t NF, int64_t tile) {
  const int64_t f = (int64_t)tile * blockDim.x + threadIdx.x;
  if (f >= NF) return;
  const int a = f_axis[f];
  const int gL = f_gL[f], gR = f_gR[f];
  const T vL = gL >= 0 ? UG[(int64_t)a * G + gL] : stashL[f];
  const T vR = gR >= 0 ? UG[(int64_t)a * G + gR] : stashR[f];
  T *Fa = a == 0 ? F0 : (a == 1 ? F1 : F2);
  Fa[f_cell[f]] = T(0.5) * (vL + vR);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_vel_faces(T *__restrict__ F0, T *__restrict__ F1, T *__restrict__ F2,
                                                        const T *__restrict__ UG, int64_t G,
                                                        const int *__restrict__ f_cell, const int *__restrict__ f_axis,
                                                        const int *__restrict__ f_gL, const int *__restrict__ f_gR,
                                                        const T *__restrict__ stashL, const T *__restrict__ stashR,
                                                        int64_t NF) {
  vel_faces_body<T>(F0, F1, F2, UG, G, f_cell, f_axis, f_gL, f_gR, stashL, stashR, NF, blockIdx.x);
}

// ---------------------------------------------------------------------------------------
// Chemical potential phi = C^3 - C - Cn^2 lap_h C on every cell, then the mirror value at
// the ghosts (dphi/dn = 0).
template <typename T, int D>
__global__ __launch_bounds__(kThreads) void k_phi(const T *__restrict__ C, T *__restrict__ phi, Dims dm, T cn2,
                                                  T inv_h2, int64_t N) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  const int i = (int)(c & (dm.nx - 1));
  const int64_t r = c >> dm.lnx;
  const int j = (int)(r & (dm.ny - 1));
  const int k = (int)(r >> dm.lny);
  const int64_t rowb = c - i;
  const T c0 = C[c];
  T sum = C[rowb + ((i + 1) & (dm.nx - 1))] + C[rowb + ((i - 1) & (dm.nx - 1))];
  if (D == 2) {
    sum += (j < dm.ny - 1 ? C[c + dm.nx] : c0) + (j > 0 ? C[c - dm.nx] : c0);
  } else {
    const int jp = (j + 1) & (dm.ny - 1), jm = (j - 1) & (dm.ny - 1);
    sum += C[c + (int64_t)(jp - j) * dm.nx] + C[c + (int64_t)(jm - j) * dm.nx];
    sum += (k < dm.nz - 1 ? C[c + dm.plane] : c0) + (k > 0 ? C[c - dm.plane] : c0);
  }
  const T lap = (sum - T(2 * D) * c0) * inv_h2;
  phi[c] = c0 * c0 * c0 - c0 - cn2 * lap;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_phi_ghost(T *__restrict__ phi, const int *__restrict__ gidx,
                                                        const int *__restrict__ ap, const T *__restrict__ w,
                                                        int64_t G, int K) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= G) return;
  phi[gidx[g]] = mirror_gather(phi, ap, w, g, G, K);
}

// Ghost fill of any scalar under the mixed condition a f + b df/dn = g at the wall: the ghost-cell
// procedure of section 4.2.2 with a general boundary condition.  With f_I and (df/dn)_I formed
// from the ghost and the mirror value as for C, f_G = ((gamma+1) g - f_M (a + b/dn)) / (a gamma - b/dn).
// The averaging points are fluid cells, never ghosts, so reads and writes do not overlap.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_scalar_fill(T *__restrict__ f, const int *__restrict__ gidx,
                                                          const int *__restrict__ ap, const T *__restrict__ w,
                                                          const T *__restrict__ dn, const T *__restrict__ gam,
                                                          const T *__restrict__ gv, T g0, T a, T b, int64_t G,
                                                          int K) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= G) return;
  const T fM = mirror_gather(f, ap, w, g, G, K);
  const T gg = gv ? gv[g] : g0;
  const T d = dn[g], gm = gam[g];
  f[gidx[g]] = ((gm + T(1)) * gg - fM * (a + b / d)) / (a * gm - b / d);
}

// Explicit step (Eq. ExpCH, non-dimensional) on every cell: the rate
//   R = -div_h(u C^n) + (1/Pe) lap_h phi^n
// (conservative central advection, zero normal velocity on the bounded axis' box walls, where
// the Laplacian reflects), then C^(n+1) = C^n + dt (3/2 R - 1/2 R_prev) with R_prev = R on the
// first step (forward Euler).  R replaces R_prev in place; the ghosts are refilled afterwards.
template <typename T, int D>
__global__ __launch_bounds__(kThreads) void k_explicit(const T *__restrict__ C, const T *__restrict__ phi,
                                                       const T *__restrict__ F0, const T *__restrict__ F1,
                                                       const T *__restrict__ F2, T *__restrict__ R,
                                                       T *__restrict__ Cnext, Dims dm, T half_inv_h, T inv_h2,
                                                       T inv_pe, T dt, int first, int64_t N) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  const int nx = dm.nx;
  const int i = (int)(c & (nx - 1));
  const int64_t rowb = c - i;
  const int ip = (i + 1) & (nx - 1), im = (i - 1) & (nx - 1);
  const T c0 = C[c], p0 = phi[c];
  T flux = F0[c] * (c0 + C[rowb + ip]) - F0[rowb + im] * (C[rowb + im] + c0);
  T lsum = phi[rowb + ip] + phi[rowb + im];
  if (D == 2) {
    const int j = (int)(c >> dm.lnx);
    const bool top = j == dm.ny - 1, bot = j == 0;
    flux += (top ? T(0) : F1[c] * (c0 + C[c + nx])) - (bot ? T(0) : F1[c - nx] * (C[c - nx] + c0));
    lsum += (top ? p0 : phi[c + nx]) + (bot ? p0 : phi[c - nx]);
  } else {
    const int j = (int)((c >> dm.lnx) & (dm.ny - 1));
    const int k = (int)(c >> (dm.lnx + dm.lny));
    const int64_t cyp = c + (int64_t)(((j + 1) & (dm.ny - 1)) - j) * nx;
    const int64_t cym = c + (int64_t)(((j - 1) & (dm.ny - 1)) - j) * nx;
    flux += F1[c] * (c0 + C[cyp]) - F1[cym] * (C[cym] + c0);
    lsum += phi[cyp] + phi[cym];
    const bool top = k == dm.nz - 1, bot = k == 0;
    flux += (top ? T(0) : F2[c] * (c0 + C[c + dm.plane])) - (bot ? T(0) : F2[c - dm.plane] * (C[c - dm.plane] + c0));
    lsum += (top ? p0 : phi[c + dm.plane]) + (bot ? p0 : phi[c - dm.plane]);
  }
  const T r = -flux * half_inv_h + inv_pe * (lsum - T(2 * D) * p0) * inv_h2;
  const T rp = first ? r : R[c];
  R[c] = r;
  Cnext[c] = c0 + dt * (T(1.5) * r - T(0.5) * rp);
}

// 3D z-marching forms of k_phi and k_explicit (2.5D blocking): a workgroup owns a 64 x 4 tile of
// (x, y) columns and a chunk of 2^zc_log planes; each thread keeps the values of planes z-1, z,
// z+1 of its own column in registers and the tile's plane z (with its one-cell x/y halo) sits in
// LDS, so every plane is read from memory once instead of three times.  Same sums in the same
// order as the one-cell-per-thread kernels.  Requires nx % 64 == 0 and ny % 4 == 0.
constexpr int kZmTx = 64, kZmTy = 4;

// Halo value of plane base zb that thread (tx, ty) supplies to the tile (x, then y neighbours);
// threads inside the tile supply none (returns their own cell, unused).
template <typename T>
__device__ __forceinline__ T zm_halo(const T *__restrict__ f, int64_t zb, int x, int y, int tx, int ty,
                                     const Dims &dm) {
  const int nx = dm.nx, ny = dm.ny;
  if (tx == 0) return f[zb + ((x - 1) & (nx - 1)) + (int64_t)nx * y];
  if (tx == kZmTx - 1) return f[zb + ((x + 1) & (nx - 1)) + (int64_t)nx * y];
  return T(0);
}
template <typename T>
__device__ __forceinline__ T zm_halo_y(const T *__restrict__ f, int64_t zb, int x, int y, int ty, const Dims &dm) {
  const int nx = dm.nx, ny = dm.ny;
  if (ty == 0) return f[zb + x + (int64_t)nx * ((y - 1) & (ny - 1))];
  if (ty == kZmTy - 1) return f[zb + x + (int64_t)nx * ((y + 1) & (ny - 1))];
  return T(0);
}
template <typename T>
__device__ __forceinline__ void zm_tile_store(T (*s)[kZmTx + 2], int tx, int ty, T own, T hx, T hy) {
  s[ty + 1][tx + 1] = own;
  if (tx == 0) s[ty + 1][0] = hx;
  if (tx == kZmTx - 1) s[ty + 1][kZmTx + 1] = hx;
  if (ty == 0) s[0][tx + 1] = hy;
  if (ty == kZmTy - 1) s[kZmTy + 1][tx + 1] = hy;
}

// Planes are taken kZmU at a time: their loads (own column and halo) are issued together, so a
// thread has kZmU requests in flight per field instead of one.
constexpr int kZmU = 4;

template <typename T>
__global__ __launch_bounds__(kThreads) void k_phi_zm(const T *__restrict__ C, T *__restrict__ phi, Dims dm, T cn2,
                                                     T inv_h2, int zc_log) {
  __shared__ T s[2][kZmTy + 2][kZmTx + 2];
  const int nbx = dm.nx / kZmTx, nby = dm.ny / kZmTy;
  const int t = blockIdx.x;
  const int bx = t % nbx, by = (t / nbx) % nby, bz = t / (nbx * nby);
  const int tx = threadIdx.x & (kZmTx - 1), ty = threadIdx.x / kZmTx;
  const int x = bx * kZmTx + tx, y = by * kZmTy + ty;
  const int z0 = bz << zc_log;
  const int64_t col = x + (int64_t)dm.nx * y;
  auto zb = [&](int z) { return (int64_t)(z < 0 ? 0 : (z >= dm.nz ? dm.nz - 1 : z)) * dm.plane; };
  T cm = C[zb(z0 - 1) + col], c0 = C[zb(z0) + col];
  for (int zg = 0; zg < (1 << zc_log); zg += kZmU) {
    const int zs = z0 + zg;
    T cz[kZmU], hx[kZmU], hy[kZmU];
#pragma unroll
    for (int u = 0; u < kZmU; ++u) {
      cz[u] = C[zb(zs + u + 1) + col];
      hx[u] = zm_halo(C, zb(zs + u), x, y, tx, ty, dm);
      hy[u] = zm_halo_y(C, zb(zs + u), x, y, ty, dm);
    }
#pragma unroll
    for (int u = 0; u < kZmU; ++u) {
      const int z = zs + u;
      const T cp = cz[u];
      T (*sb)[kZmTx + 2] = s[u & 1];
      zm_tile_store(sb, tx, ty, c0, hx[u], hy[u]);
      __syncthreads();   // this slot was last read two planes ago, before the previous barrier
      T sum = sb[ty + 1][tx + 2] + sb[ty + 1][tx];
      sum += sb[ty + 2][tx + 1] + sb[ty][tx + 1];
      sum += (z < dm.nz - 1 ? cp : c0) + (z > 0 ? cm : c0);
      const T lap = (sum - T(6) * c0) * inv_h2;
      phi[zb(z) + col] = c0 * c0 * c0 - c0 - cn2 * lap;
      cm = c0;
      c0 = cp;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_explicit_zm(const T *__restrict__ C, const T *__restrict__ phi,
                                                          const T *__restrict__ F0, const T *__restrict__ F1,
                                                          const T *__restrict__ F2, T *__restrict__ R,
                                                          T *__restrict__ Cnext, Dims dm, T half_inv_h, T inv_h2,
                                                          T inv_pe, T dt, int first, int zc_log) {
  __shared__ T sc[2][kZmTy + 2][kZmTx + 2], sp[2][kZmTy + 2][kZmTx + 2];
  const int nx = dm.nx, ny = dm.ny;
  const int nbx = nx / kZmTx, nby = ny / kZmTy;
  const int t = blockIdx.x;
  const int bx = t % nbx, by = (t / nbx) % nby, bz = t / (nbx * nby);
  const int tx = threadIdx.x & (kZmTx - 1), ty = threadIdx.x / kZmTx;
  const int x = bx * kZmTx + tx, y = by * kZmTy + ty;
  const int z0 = bz << zc_log;
  const int64_t col = x + (int64_t)nx * y;
  const int64_t colxm = ((x - 1) & (nx - 1)) + (int64_t)nx * y;
  const int64_t colym = x + (int64_t)nx * ((y - 1) & (ny - 1));
  auto zb = [&](int z) { return (int64_t)(z < 0 ? 0 : (z >= dm.nz ? dm.nz - 1 : z)) * dm.plane; };
  T cm = C[zb(z0 - 1) + col], c0 = C[zb(z0) + col];
  T pm = phi[zb(z0 - 1) + col], p0 = phi[zb(z0) + col];
  T f2m = F2[zb(z0 - 1) + col];   // the face below plane z0 (unused at the bottom wall)
  for (int zg = 0; zg < (1 << zc_log); zg += kZmU) {
    const int zs = z0 + zg;
    T cz[kZmU], pz[kZmU], hcx[kZmU], hcy[kZmU], hpx[kZmU], hpy[kZmU];
    T f0z[kZmU], f0mz[kZmU], f1z[kZmU], f1mz[kZmU], f2z[kZmU], rz[kZmU];
#pragma unroll
    for (int u = 0; u < kZmU; ++u) {
      const int64_t b = zb(zs + u), b1 = zb(zs + u + 1);
      cz[u] = C[b1 + col];
      pz[u] = phi[b1 + col];
      f0z[u] = F0[b + col];
      f0mz[u] = F0[b + colxm];
      f1z[u] = F1[b + col];
      f1mz[u] = F1[b + colym];
      f2z[u] = F2[b + col];
      rz[u] = R[b + col];
      hcx[u] = zm_halo(C, b, x, y, tx, ty, dm);
      hcy[u] = zm_halo_y(C, b, x, y, ty, dm);
      hpx[u] = zm_halo(phi, b, x, y, tx, ty, dm);
      hpy[u] = zm_halo_y(phi, b, x, y, ty, dm);
    }
#pragma unroll
    for (int u = 0; u < kZmU; ++u) {
      const int z = zs + u;
      const int64_t c = zb(z) + col;
      const T cp = cz[u], pp = pz[u];
      const T f0 = f0z[u], f0m = f0mz[u], f1 = f1z[u], f1m = f1mz[u], f2 = f2z[u];
      const T rprev = rz[u];
      T (*sbc)[kZmTx + 2] = sc[u & 1];
      T (*sbp)[kZmTx + 2] = sp[u & 1];
      zm_tile_store(sbc, tx, ty, c0, hcx[u], hcy[u]);
      zm_tile_store(sbp, tx, ty, p0, hpx[u], hpy[u]);
      __syncthreads();   // these slots were last read two planes ago, before the previous barrier
      const bool top = z == dm.nz - 1, bot = z == 0;
      T flux = f0 * (c0 + sbc[ty + 1][tx + 2]) - f0m * (sbc[ty + 1][tx] + c0);
      T lsum = sbp[ty + 1][tx + 2] + sbp[ty + 1][tx];
      flux += f1 * (c0 + sbc[ty + 2][tx + 1]) - f1m * (sbc[ty][tx + 1] + c0);
      lsum += sbp[ty + 2][tx + 1] + sbp[ty][tx + 1];
      flux += (top ? T(0) : f2 * (c0 + cp)) - (bot ? T(0) : f2m * (cm + c0));
      lsum += (top ? p0 : pp) + (bot ? p0 : pm);
      const T r = -flux * half_inv_h + inv_pe * (lsum - T(6) * p0) * inv_h2;
      const T rp = first ? r : rprev;
      R[c] = r;
      Cnext[c] = c0 + dt * (T(1.5) * r - T(0.5) * rp);
      cm = c0;
      c0 = cp;
      pm = p0;
      p0 = pp;
      f2m = f2;
    }
  }
}

inline bool stencil_zm_ok(const Plan &p) {
  return p.d == 3 && p.n[0] % kZmTx == 0 && p.n[1] % kZmTy == 0 && p.n[2] >= 16;   // chunks of 16 planes
}
inline int stencil_zm_log(const Plan &p) { return p.logn[2] < 4 ? p.logn[2] : 4; }   // >= log2(kZmU) below
inline unsigned stencil_zm_blocks(const Plan &p) {
  return (unsigned)((p.n[0] / kZmTx) * (p.n[1] / kZmTy) * (p.n[2] >> stencil_zm_log(p)));
}

template <typename T, int D>
__global__ __launch_bounds__(kThreads) void k_rhs_only(const T *__restrict__ Cn, const T *__restrict__ Cp,
                                                       const T *__restrict__ F0, const T *__restrict__ F1,
                                                       const T *__restrict__ F2, T *__restrict__ Q, Dims dm,
                                                       RhsCoef<T> cf, int64_t N) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  const int i = (int)(c & (dm.nx - 1));
  const int64_t r = c >> dm.lnx;
  const int j = (int)(r & (dm.ny - 1));
  const int k = (int)(r >> dm.lny);
  Q[c] = rhs_at<T, D>(Cn, Cp, F0, F1, F2, i, j, k, dm, cf);
}

// ---------------------------------------------------------------------------------------
// Diagnostics: fixed-order two-pass reductions (deterministic).  Slots: 0 sum C, 1 sum
// alpha C, 2 sum alpha (bulk + gradient energy density), 3 sum |grad alpha| g(C),
// 4 max |C|, 5 count of non-finite C.
// Sum (max for slot 4) of the six slots over a wave by a butterfly of lane exchanges: a fixed
// pairing, so the result does not depend on timing.
__device__ inline void wave_reduce6(double acc[6]) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) {
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      const double o = __shfl_xor(acc[s], m, 64);
      acc[s] = s == 4 ? fmax(acc[s], o) : acc[s] + o;
    }
  }
}

// Per block: each wave reduces its lanes, then the first lanes combine the waves in index order.
template <typename T, int D>
__global__ __launch_bounds__(kThreads) void k_diag_partial(const T *__restrict__ C, const T *__restrict__ alpha,
                                                           double *__restrict__ partial, Dims dm, double Cn,
                                                           double inv_h, double inv4cn, int64_t N) {
  __shared__ double red[kThreads / 64][6];
  double acc[6] = {0, 0, 0, 0, 0, 0};
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += stride) {
    const double v = (double)C[c];
    const double al = alpha ? (double)alpha[c] : 1.0;
    if (!(v == v) || v - v != 0.0) {
      acc[5] += 1.0;
      continue;
    }
    const int i = (int)(c & (dm.nx - 1));
    const int64_t r = c >> dm.lnx;
    const int j = (int)(r & (dm.ny - 1));
    const int k = (int)(r >> dm.lny);
    const int64_t rowb = c - i;
    double g2 = 0.0;
    double ga2 = 0.0;
    {
      const double dx = ((double)C[rowb + ((i + 1) & (dm.nx - 1))] - v) * inv_h;
      g2 += dx * dx;
      if (alpha) {
        const double da = ((double)alpha[rowb + ((i + 1) & (dm.nx - 1))] -
                           (double)alpha[rowb + ((i - 1) & (dm.nx - 1))]) * 0.5 * inv_h;
        ga2 += da * da;
      }
    }
    if (D == 2) {
      const double up = j < dm.ny - 1 ? (double)C[c + dm.nx] : v;
      const double dy = (up - v) * inv_h;
      g2 += dy * dy;
      if (alpha) {
        const double au = j < dm.ny - 1 ? (double)alpha[c + dm.nx] : al;
        const double ad = j > 0 ? (double)alpha[c - dm.nx] : al;
        const double da = (au - ad) * 0.5 * inv_h;
        ga2 += da * da;
      }
    } else {
      const int jp = (j + 1) & (dm.ny - 1), jm = (j - 1) & (dm.ny - 1);
      const double dy = ((double)C[c + (int64_t)(jp - j) * dm.nx] - v) * inv_h;
      g2 += dy * dy;
      const double up = k < dm.nz - 1 ? (double)C[c + dm.plane] : v;
      const double dz = (up - v) * inv_h;
      g2 += dz * dz;
      if (alpha) {
        const double day = ((double)alpha[c + (int64_t)(jp - j) * dm.nx] -
                            (double)alpha[c + (int64_t)(jm - j) * dm.nx]) * 0.5 * inv_h;
        const double au = k < dm.nz - 1 ? (double)alpha[c + dm.plane] : al;
        const double ad = k > 0 ? (double)alpha[c - dm.plane] : al;
        const double daz = (au - ad) * 0.5 * inv_h;
        ga2 += day * day + daz * daz;
      }
    }
    const double bulk = (v * v - 1.0) * (v * v - 1.0) * inv4cn;
    acc[0] += v;
    acc[1] += al * v;
    acc[2] += al * (bulk + 0.5 * Cn * g2);
    acc[3] += sqrt(ga2) * (2.0 + 3.0 * v - v * v * v) * 0.25;
    acc[4] = fmax(acc[4], fabs(v));
  }
  wave_reduce6(acc);
  const int lane = (int)threadIdx.x & 63, wv = (int)threadIdx.x >> 6;
  if (lane == 0)
    for (int s = 0; s < 6; ++s) red[wv][s] = acc[s];
  __syncthreads();
  if (threadIdx.x < 6) {
    const int s = (int)threadIdx.x;
    double r = red[0][s];
    for (int w = 1; w < kThreads / 64; ++w) r = s == 4 ? fmax(r, red[w][s]) : r + red[w][s];
    partial[(int64_t)blockIdx.x * 8 + s] = r;
  }
}

// 3D diagnostics marching in z: a block owns a 64 x 4 tile of (x, y) columns over zc planes, each
// thread keeps C and alpha of planes z and z+1 (alpha also z-1) of its column in registers, so C and
// alpha come from HBM once; the x and y neighbours are in the same plane as the tile's own loads.
// Tiles go in XCD-aware order, so the neighbouring tiles whose halo rows a tile reads share its L2
// (116 -> 99 us per call at 256^3).  Same per-cell terms as k_diag_partial<T, 3>.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_diag_partial_zm(const T *__restrict__ C, const T *__restrict__ alpha,
                                                              double *__restrict__ partial, Dims dm, double Cn,
                                                              double inv_h, double inv4cn, int zc) {
  __shared__ double red[kThreads / 64][6];
  double acc[6] = {0, 0, 0, 0, 0, 0};
  const int tiles_x = dm.nx >> 6, tiles_y = dm.ny >> 2;
  int b = xcd_tile(blockIdx.x, gridDim.x);
  const int bx = b % tiles_x;
  b /= tiles_x;
  const int by = b % tiles_y;
  const int bz = b / tiles_y;
  const int x = (bx << 6) + ((int)threadIdx.x & 63), y = (by << 2) + ((int)threadIdx.x >> 6);
  const int z0 = bz * zc, z1 = min(z0 + zc, dm.nz);
  const int oxp = ((x + 1) & (dm.nx - 1)) - x, oxm = ((x - 1) & (dm.nx - 1)) - x;
  const int64_t oyp = (int64_t)((((y + 1) & (dm.ny - 1)) - y) << dm.lnx);
  const int64_t oym = (int64_t)((((y - 1) & (dm.ny - 1)) - y) << dm.lnx);
  int64_t c = ((int64_t)y << dm.lnx) + x + (int64_t)z0 * dm.plane;
  double v = (double)C[c];
  double al = alpha ? (double)alpha[c] : 1.0;
  double ad = alpha && z0 > 0 ? (double)alpha[c - dm.plane] : al;
  for (int k = z0; k < z1; ++k, c += dm.plane) {
    double vu = v, au = al;
    if (k < dm.nz - 1) {
      vu = (double)C[c + dm.plane];
      if (alpha) au = (double)alpha[c + dm.plane];
    }
    if (!(v == v) || v - v != 0.0) {
      acc[5] += 1.0;
    } else {
      const double dx = ((double)C[c + oxp] - v) * inv_h;
      const double dy = ((double)C[c + oyp] - v) * inv_h;
      const double dz = (vu - v) * inv_h;
      double g2 = dx * dx;
      g2 += dy * dy;
      g2 += dz * dz;
      double ga2 = 0.0;
      if (alpha) {
        const double da = ((double)alpha[c + oxp] - (double)alpha[c + oxm]) * 0.5 * inv_h;
        const double day = ((double)alpha[c + oyp] - (double)alpha[c + oym]) * 0.5 * inv_h;
        const double daz = (au - ad) * 0.5 * inv_h;
        ga2 += da * da;
        ga2 += day * day + daz * daz;
      }
      const double bulk = (v * v - 1.0) * (v * v - 1.0) * inv4cn;
      acc[0] += v;
      acc[1] += al * v;
      acc[2] += al * (bulk + 0.5 * Cn * g2);
      acc[3] += sqrt(ga2) * (2.0 + 3.0 * v - v * v * v) * 0.25;
      acc[4] = fmax(acc[4], fabs(v));
    }
    ad = al;
    al = au;
    v = vu;
  }
  wave_reduce6(acc);
  const int lane = (int)threadIdx.x & 63, wv = (int)threadIdx.x >> 6;
  if (lane == 0)
    for (int s = 0; s < 6; ++s) red[wv][s] = acc[s];
  __syncthreads();
  if (threadIdx.x < 6) {
    const int s = (int)threadIdx.x;
    double r = red[0][s];
    for (int w = 1; w < kThreads / 64; ++w) r = s == 4 ? fmax(r, red[w][s]) : r + red[w][s];
    partial[(int64_t)blockIdx.x * 8 + s] = r;
  }
}

__global__ __launch_bounds__(kThreads) void k_diag_final(const double *__restrict__ partial, int nred,
                                                         double *__restrict__ out) {
  __shared__ double red[6][kThreads];
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < nred; b += blockDim.x)
    for (int s = 0; s < 6; ++s) {
      const double v = partial[(int64_t)b * 8 + s];
      if (s == 4) acc[s] = fmax(acc[s], v);
      else acc[s] += v;
    }
  for (int s = 0; s < 6; ++s) red[s][threadIdx.x] = acc[s];
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int s = 0; s < 6; ++s) {
        if (s == 4) red[s][threadIdx.x] = fmax(red[s][threadIdx.x], red[s][threadIdx.x + w]);
        else red[s][threadIdx.x] += red[s][threadIdx.x + w];
      }
    __syncthreads();
  }
  if (threadIdx.x < 6) out[threadIdx.x] = red[threadIdx.x][0];
}

// ---------------------------------------------------------------------------------------
// Host-side launch shapes.

inline int ilog2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

inline Dims make_dims(const Plan &p) {
  Dims dm;
  dm.nx = p.n[0];
  dm.ny = p.n[1];
  dm.nz = p.d == 3 ? p.n[2] : 1;
  dm.lnx = p.logn[0];
  dm.lny = p.logn[1];
  dm.lnz = p.d == 3 ? p.logn[2] : 0;
  dm.plane = (int64_t)dm.nx * dm.ny;
  return dm;
}

template <typename T>
inline RhsCoef<T> make_coef(const Plan &p) {
  RhsCoef<T> cf;
  cf.pe_cn2 = (T)(p.Pe / (p.Cn * p.Cn));
  cf.inv_dt = (T)(1.0 / p.dt);
  cf.S = (T)p.S;
  cf.inv_cn2 = (T)(1.0 / (p.Cn * p.Cn));
  cf.inv_h = (T)(1.0 / p.h);
  cf.inv_h2 = (T)(1.0 / (p.h * p.h));
  return cf;
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

// The rhs' ghost patch (none without ghosts).
template <typename T>
inline RhsPatch<T> make_patch(const Plan &p) {
  RhsPatch<T> rp{};
  if (p.G > 0 && p.NP > 0 && p.pl_dq) {
    rp.row = p.pl_row;
    rp.cell = p.pl_cell;
    rp.dq = (const T *)p.pl_dq;
  }
  return rp;
}

// dg of every ghost from C^n, C^(n-1), then dq of every patched cell (before the rhs pass of a
// semi-implicit step).
template <typename T>
hipError_t launch_ghost_patch(const Plan &p, const T *Cn, const T *Cp) {
  if (p.G == 0 || p.NP == 0 || !p.dg) return hipSuccess;
  const Dims dm = make_dims(p);
  if (p.NU && p.pt_phi) {
    hipLaunchKernelGGL((k_point_phit<T>), dim3(blocks_for(p.NU)), dim3(kThreads), 0, p.stream, Cn, Cp, p.pt_cell,
                       (T *)p.pt_phi, p.NU, dm, p.d, (T)(p.Cn * p.Cn), (T)(1.0 / (p.h * p.h)));
    hipLaunchKernelGGL((k_ghost_dg<T>), dim3(blocks_for(p.G * 16)), dim3(kThreads), 0, p.stream,
                       (const T *)p.pt_phi, p.pt_idx, (const T *)p.wg, (T *)p.dg, p.G, p.K, (T)(1.0 / (p.Cn * p.Cn)));
  } else {
    hipLaunchKernelGGL((k_ghost_dphi<T>), dim3(blocks_for(p.G * 16)), dim3(kThreads), 0, p.stream, Cn, Cp, p.gidx,
                       p.apg, (const T *)p.wg, (T *)p.dg, p.G, p.K, dm, p.d, (T)(p.Cn * p.Cn), (T)(1.0 / (p.h * p.h)),
                       (T)(1.0 / (p.Cn * p.Cn)));
  }
  hipLaunchKernelGGL((k_patch_dq<T>), dim3(blocks_for(p.NP)), dim3(kThreads), 0, p.stream, p.pl_ref,
                     (const T *)p.dg, (T *)p.pl_dq, p.NP, 2 * p.d + 1, (T)(2 * p.d), (T)(1.0 / (p.h * p.h)));
  return hipGetLastError();
}

// The patch added to a rhs field stored cell by cell.
template <typename T>
hipError_t launch_rhs_patch(const Plan &p, T *Q) {
  const RhsPatch<T> rp = make_patch<T>(p);
  if (!rp.dq) return hipSuccess;
  hipLaunchKernelGGL((k_rhs_patch<T>), dim3(blocks_for(p.NP)), dim3(kThreads), 0, p.stream, Q, rp.cell, rp.dq, p.NP);
  return hipGetLastError();
}

// Faces that advect C in the rhs pass: the extrapolated velocity when the momentum equation is
// solved too, else the faces themselves.
inline const void *adv_face(const Plan &p, int a) { return p.Fadv[a] ? p.Fadv[a] : p.F[a]; }

// Launch shapes.  Each pass has a runtime-selected variant (see Plan::Shape): the log2 of
// its lines (x passes) or columns (strided passes) per tile, the largest FFT radix (8 or
// 16: fewer LDS passes against fewer registers) and, for the fused rhs pass, how many cells
// each thread keeps in flight.
inline int max_log_lines(const Plan &p, int E) {
  const int lines = p.d == 3 ? p.n[1] * p.n[2] : p.n[1];
  int L = E / p.n[0];
  if (L > lines) L = lines;
  if (L < 2) L = 2;
  return ilog2(L);
}

inline int max_log_cols(const Plan &p, int N, int E) {
  int B = E / N;
  if (B > p.n[0]) B = p.n[0];
  if (B < 2) B = 2;
  return ilog2(B);
}

inline int clamp_log(int v, int hi) { return v < 1 ? 1 : (v > hi ? hi : v); }

// The fixed-size instances (256-point lines, template constants for the line length and tile width)
// serve the tile widths and radices below; other shapes take the runtime-size kernels.
template <typename T>
hipError_t launch_xdht(const Plan &p, const T *in, T *out, const Plan::Shape &sh) {
  constexpr int E = tile_elems<T>();
  const int logL = clamp_log(sh.log_tile, max_log_lines(p, E));
  const int lines = p.d == 3 ? p.n[1] * p.n[2] : p.n[1];
  const unsigned nb = (unsigned)(lines >> logL);
  const size_t lds = (size_t)(1 << logL) * line_pitch(p.n[0]) * sizeof(T);
#define CHIB_XDHT(...)                                                                                         \
  hipLaunchKernelGGL((k_xdht<__VA_ARGS__>), dim3(nb), dim3(kThreads), lds, p.stream, in, out, p.logn[0], logL, \
                     (const T *)p.twr[0], (const T *)p.twi[0])
  const bool r8 = sh.radix == 8, fixed = p.logn[0] == 8;
  if (fixed && logL == 3) {
    if (r8) CHIB_XDHT(T, E, 8, 8, 3);
    else CHIB_XDHT(T, E, 16, 8, 3);
  } else if (fixed && logL == 4) {
    if (r8) CHIB_XDHT(T, E, 8, 8, 4);
    else CHIB_XDHT(T, E, 16, 8, 4);
  } else if (r8) {
    CHIB_XDHT(T, E, 8);
  } else {
    CHIB_XDHT(T, E, 16);
  }
#undef CHIB_XDHT
  return hipGetLastError();
}

template <typename T>
hipError_t launch_ydht(const Plan &p, const Plan::Shape &sh) {
  constexpr int E = tile_elems<T>();
  const int nx = p.n[0];
  const int lb = clamp_log(sh.log_tile, max_log_cols(p, p.n[1], E));
  const int lxb = p.logn[0] - lb;
  const unsigned nb = (unsigned)((nx >> lb) * p.n[2]);
  const size_t lds = (size_t)col_tile(p.n[1], 1 << lb) * sizeof(T);
#define CHIB_YDHT(...)                                                                                          \
  hipLaunchKernelGGL((k_strided_dht<__VA_ARGS__>), dim3(nb), dim3(kThreads), lds, p.stream, (T *)p.W, p.logn[1], \
                     (int64_t)nx, lb, lxb, (int64_t)nx * p.n[1], (const T *)p.twr[1], (const T *)p.twi[1])
  const bool r8 = sh.radix == 8;
  const bool fixed = p.logn[1] == 8 && (int64_t)nx * 256 * (int64_t)sizeof(T) < (int64_t(1) << 32);
  if (fixed && lb == 3) {
    if (r8) CHIB_YDHT(T, E, 8, 8, 3);
    else CHIB_YDHT(T, E, 16, 8, 3);
  } else if (fixed && lb == 4) {
    if (r8) CHIB_YDHT(T, E, 8, 8, 4);
    else CHIB_YDHT(T, E, 16, 8, 4);
  } else if (r8) {
    CHIB_YDHT(T, E, 8);
  } else {
    CHIB_YDHT(T, E, 16);
  }
#undef CHIB_YDHT
  return hipGetLastError();
}

template <typename T>
hipError_t launch_neumann(const Plan &p, const Plan::Shape &sh) {
  constexpr int E = tile_elems<T>();
  const int nx = p.n[0];
  const int ax = p.d - 1;
  const int Nn = p.n[ax];
  const int lb = clamp_log(sh.log_tile, max_log_cols(p, Nn, E));
  const int lxb = p.logn[0] - lb;
  const int64_t stride = p.d == 3 ? (int64_t)nx * p.n[1] : (int64_t)nx;
  const int64_t outer = p.d == 3 ? (int64_t)nx : 0;
  const unsigned nb = (unsigned)((nx >> lb) * (p.d == 3 ? p.n[1] : 1));
  const size_t lds = (size_t)col_tile(Nn, 1 << lb) * sizeof(T);
  const double norm = (double)p.N;  // 1/(nx [ny] n_last): inverse Hartley scales and the inverse FFT
  const T *lamy = p.d == 3 ? (const T *)p.lam[1] : (const T *)nullptr;
#define CHIB_NEUMANN(...)                                                                                        \
  hipLaunchKernelGGL((k_neumann_solve<__VA_ARGS__>), dim3(nb), dim3(kThreads), lds, p.stream, (T *)p.W,          \
                     p.logn[ax], stride, lb, lxb, outer, (const T *)p.lam[0], lamy, (const T *)p.lam[ax], (T)p.a, \
                     (T)p.alpha_s, (T)(1.0 / norm), (const T *)p.twr[ax], (const T *)p.twi[ax],               \
                     (const T *)p.dctc, (const T *)p.dcts, p.poisson)
  // 256-point lines in a full tile
  constexpr int FB = ilog2c(E / 256);
  const bool fixed = p.logn[ax] == 8 && lb == FB && stride * 256 * (int64_t)sizeof(T) < (int64_t(1) << 32);
  if (fixed) {
    if (sh.radix == 8) CHIB_NEUMANN(T, E, 8, 8, FB);
    else CHIB_NEUMANN(T, E, 16, 8, FB);
  } else if (sh.radix == 8) {
    CHIB_NEUMANN(T, E, 8);
  } else {
    CHIB_NEUMANN(T, E, 16);
  }
#undef CHIB_NEUMANN
  return hipGetLastError();
}

template <typename T, int D, int U, int R>
void launch_rhs_variant(const Plan &p, const T *Cn, const T *Cp, int logL, unsigned nb, size_t lds) {
  const Dims dm = make_dims(p);
  const RhsCoef<T> cf = make_coef<T>(p);
  hipLaunchKernelGGL((k_rhs_xdht<T, D, tile_elems<T>(), U, R>), dim3(nb), dim3(kThreads), lds, p.stream, Cn, Cp,
                     (const T *)adv_face(p, 0), (const T *)adv_face(p, 1), (const T *)(D == 3 ? adv_face(p, 2) : adv_face(p, 1)), (T *)p.W, dm, cf,
                     logL, (const T *)p.twr[0], (const T *)p.twi[0], make_patch<T>(p));
}

// y-marching variant (2D, nx up to 1024): unroll = 3.
inline bool ym_ok(const Plan &p) { return p.d == 2 && p.n[0] <= 1024; }

template <typename T, int XM, int R>
void launch_ym_variant(const Plan &p, const T *Cn, const T *Cp, int logL) {
  const Dims dm = make_dims(p);
  const RhsCoef<T> cf = make_coef<T>(p);
  const unsigned nb = (unsigned)(p.n[1] >> logL);
  const size_t lds = ((size_t)(1 << logL) * line_pitch(p.n[0]) + ym_extra(p.n[0])) * sizeof(T);
  hipLaunchKernelGGL((k_rhs_xdht_ym<T, XM, R>), dim3(nb), dim3(kThreads), lds, p.stream, Cn, Cp,
                     (const T *)adv_face(p, 0), (const T *)adv_face(p, 1), (T *)p.W, dm, cf, logL, (const T *)p.twr[0],
                     (const T *)p.twi[0], make_patch<T>(p));
}

template <typename T, int R>
void launch_ym(const Plan &p, const T *Cn, const T *Cp, int logL) {
  if (p.n[0] <= 256) launch_ym_variant<T, 1, R>(p, Cn, Cp, logL);
  else if (p.n[0] <= 512) launch_ym_variant<T, 2, R>(p, Cn, Cp, logL);
  else launch_ym_variant<T, 4, R>(p, Cn, Cp, logL);
}

// z-marching variant (3D, nx a multiple of 256 up to 512): unroll = log2 of the planes per chunk.
inline bool zm_ok(const Plan &p) { return p.d == 3 && (p.n[0] == 256 || p.n[0] == 512) && p.n[1] >= 2; }

template <typename T, int L, int XM, int R, bool SPLIT = false>
void launch_zm_variant(const Plan &p, const T *Cn, const T *Cp, int zc_log) {
  const Dims dm = make_dims(p);
  const RhsCoef<T> cf = make_coef<T>(p);
  const unsigned nb = (unsigned)((p.n[1] / L) * (p.n[2] >> zc_log));
  const size_t lds = ((size_t)2 * L * p.n[0] + (SPLIT ? 0 : (size_t)L * line_pitch(p.n[0]) + 2 * p.n[0])) * sizeof(T);
  hipLaunchKernelGGL((k_rhs_xdht_zm<T, L, XM, R, SPLIT>), dim3(nb), dim3(kThreads), lds, p.stream, Cn, Cp,
                     (const T *)adv_face(p, 0), (const T *)adv_face(p, 1), (const T *)adv_face(p, 2), (T *)p.W, dm, cf, zc_log,
                     (const T *)p.twr[0], (const T *)p.twi[0], make_patch<T>(p));
}

// Stencil-only z-march (the rhs Q into W, no transform) with L rows per tile.
template <typename T, int XM>
void launch_zm_split(const Plan &p, const T *Cn, const T *Cp, int logL, int zc_log) {
  if (logL <= 1) launch_zm_variant<T, 2, XM, 8, true>(p, Cn, Cp, zc_log);
  else if (logL == 2) launch_zm_variant<T, 4, XM, 8, true>(p, Cn, Cp, zc_log);
  else if constexpr (XM == 1) launch_zm_variant<T, 8, XM, 8, true>(p, Cn, Cp, zc_log);
}

template <typename T, int XM>
void launch_zm_xm(const Plan &p, const T *Cn, const T *Cp, int logL, int radix, int zc_log) {
  if (logL <= 1) {
    if (radix == 4) launch_zm_variant<T, 2, XM, 4>(p, Cn, Cp, zc_log);
    else if (radix == 8) launch_zm_variant<T, 2, XM, 8>(p, Cn, Cp, zc_log);
    else launch_zm_variant<T, 2, XM, 16>(p, Cn, Cp, zc_log);
  } else if (logL == 2) {
    if (radix == 4) launch_zm_variant<T, 4, XM, 4>(p, Cn, Cp, zc_log);
    else if (radix == 8) launch_zm_variant<T, 4, XM, 8>(p, Cn, Cp, zc_log);
    else launch_zm_variant<T, 4, XM, 16>(p, Cn, Cp, zc_log);
  } else if constexpr (XM == 1) {   // (512-wide grids take at most 4 rows per tile)
    if (radix <= 8) launch_zm_variant<T, 8, XM, 8>(p, Cn, Cp, zc_log);
    else launch_zm_variant<T, 8, XM, 16>(p, Cn, Cp, zc_log);
  }
}

// Pass 0.  unroll 1-2: one fused rhs + x-transform kernel per line tile; 2D, 3: the y-marching
// form of it (nx up to 1024); 3D, 3-5: the same fused
// work z-marching over 2^unroll planes (3D, nx 256 or 512); 6-8: a stencil-only z-march over
// 2^(unroll-3) planes writing Q, then the x transform of W in place (with split_only, the
// caller launches that transform itself).
template <typename T, int D>
hipError_t launch_rhs(const Plan &p, const T *Cn, const T *Cp, const Plan::Shape &sh, bool split_only = false) {
  constexpr int E = tile_elems<T>();
  if (D == 3 && sh.unroll >= 3 && zm_ok(p)) {
    int logL = sh.log_tile < 1 ? 1 : (sh.log_tile > 3 ? 3 : sh.log_tile);
    if (p.n[0] == 512 && logL > 2) logL = 2;   // two 512-wide planes of C~ and x faces plus the tile stay in LDS
    while ((1 << logL) > p.n[1]) --logL;
    const bool split = sh.unroll >= 6;
    int zc_log = split ? sh.unroll - 3 : sh.unroll;
    while ((1 << zc_log) > p.n[2]) --zc_log;
    if (split) {
      if (p.n[0] == 256) launch_zm_split<T, 1>(p, Cn, Cp, logL, zc_log);
      else launch_zm_split<T, 2>(p, Cn, Cp, logL, zc_log);
      hipError_t e = hipGetLastError();
      if (e == hipSuccess) e = launch_rhs_patch<T>(p, (T *)p.W);
      if (e != hipSuccess || split_only) return e;
      return launch_xdht<T>(p, (const T *)p.W, (T *)p.W, p.shape[3]);
    }
    if (p.n[0] == 256) launch_zm_xm<T, 1>(p, Cn, Cp, logL, sh.radix, zc_log);
    else launch_zm_xm<T, 2>(p, Cn, Cp, logL, sh.radix, zc_log);
    return hipGetLastError();
  }
  const int logL = clamp_log(sh.log_tile, max_log_lines(p, E));
  if (D == 2 && sh.unroll == 3 && ym_ok(p)) {
    if (sh.radix <= 8) launch_ym<T, 8>(p, Cn, Cp, logL);
    else launch_ym<T, 16>(p, Cn, Cp, logL);
    return hipGetLastError();
  }
  const int lines = p.d == 3 ? p.n[1] * p.n[2] : p.n[1];
  const unsigned nb = (unsigned)(lines >> logL);
  const size_t lds = (size_t)(1 << logL) * line_pitch(p.n[0]) * sizeof(T);
  const bool r8 = sh.radix <= 8, u2 = sh.unroll >= 2;
  if (r8 && u2) launch_rhs_variant<T, D, 2, 8>(p, Cn, Cp, logL, nb, lds);
  else if (r8) launch_rhs_variant<T, D, 1, 8>(p, Cn, Cp, logL, nb, lds);
  else if (u2) launch_rhs_variant<T, D, 2, 16>(p, Cn, Cp, logL, nb, lds);
  else launch_rhs_variant<T, D, 1, 16>(p, Cn, Cp, logL, nb, lds);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_spectral_tail(const Plan &p, KernelTimer *tm = nullptr) {
  hipError_t e = hipSuccess;
  auto mark = [&](const char *name) {
    if (tm && e == hipSuccess) e = tm->mark(name, p.stream);
  };
  if (p.d == 3) {
    mark("ydht_fwd");
    if (e == hipSuccess) e = launch_ydht<T>(p, p.shape[1]);
  }
  mark("neumann_solve");
  if (e == hipSuccess) e = launch_neumann<T>(p, p.shape[2]);
  if (p.d == 3) {
    mark("ydht_inv");
    if (e == hipSuccess) e = launch_ydht<T>(p, p.shape[1]);
  }
  return e;
}

template <typename T>
hipError_t launch_ghost_fill(const Plan &p, T *Cout, int init) {
  if (p.G == 0) return hipSuccess;
  const unsigned nb = blocks_for(p.G);
  const Dims dm = make_dims(p);
  if (!p.dynamic) {
    const T cb = (T)(p.cos_t / (1.4142135623730951 * p.Cn));
    hipLaunchKernelGGL((k_fill_static<T>), dim3(blocks_for(p.G * 16)), dim3(kThreads), 0, p.stream, Cout, p.gidx,
                       (const T *)p.dn,
                       (const T *)p.gamma, p.apg, (const T *)p.wg, (T *)p.CGn, (T *)p.CGnm1, (T *)p.CMs, p.G, p.K, cb,
                       init);
  } else {
    if (!init)
      hipLaunchKernelGGL((k_scatter_pg<T>), dim3(nb), dim3(kThreads), 0, p.stream, Cout, p.gidx,
                         (const T *)p.CGn, (const T *)p.CGnm1, p.G);
    hipLaunchKernelGGL((k_fill_dynamic<T>), dim3(nb), dim3(kThreads), 0, p.stream, (const T *)Cout,
                       (const T *)p.F[0], (const T *)p.F[1], (const T *)p.F[2], p.gidx, (const T *)p.normal,
                       (const T *)p.dn, (const T *)p.gamma, p.ap, (const T *)p.w, (T *)p.CI, (T *)p.CGnew,
                       (T *)p.CMs, p.G, p.K, dm, p.d, (T)(0.5 / p.h), (T)p.Cn, (T)p.Vs, (T)p.cos_t, (T)p.dt, init);
    hipLaunchKernelGGL((k_commit_ghosts<T>), dim3(nb), dim3(kThreads), 0, p.stream, Cout, p.gidx,
                       (const T *)p.CGnew, (T *)p.CGn, (T *)p.CGnm1, p.G, init);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_velocity_faces(const Plan &p) {
  if (p.NF)
    hipLaunchKernelGGL((k_vel_faces<T>), dim3(blocks_for(p.NF)), dim3(kThreads), 0, p.stream, (T *)p.F[0],
                       (T *)p.F[1], (T *)p.F[2], (const T *)p.UG, p.G, p.f_cell, p.f_axis, p.f_gL, p.f_gR,
                       (const T *)p.stashL, (const T *)p.stashR, p.NF);
  return hipGetLastError();
}

// Static condition with the velocity fill: C ghosts and ghost velocities in one launch, then the faces.
template <typename T>
hipError_t launch_static_fills(const Plan &p, T *Cout) {
  const Dims dm = make_dims(p);
  const unsigned nbc = blocks_for(p.G * 16), nbg = blocks_for(p.G * 16);
  const T cb = (T)(p.cos_t / (1.4142135623730951 * p.Cn));
  hipLaunchKernelGGL((k_fill_static_vel<T>), dim3(nbc + nbg + blocks_for(p.NF)), dim3(kThreads), 0, p.stream, Cout,
                     p.gidx, (const T *)p.dn, (const T *)p.gamma, p.apg, (const T *)p.wg, (T *)p.CGn, (T *)p.CGnm1,
                     (T *)p.CMs, p.G, p.K, cb, (const T *)p.F[0], (const T *)p.F[1], (const T *)p.F[2],
                     (const T *)p.normal, (T *)p.UG, p.f_cell, p.f_axis, p.f_gL, p.f_gR, (T *)p.stashL,
                     (T *)p.stashR, p.NF, dm, p.d, (T)(0.5 / p.h), (T)p.Cn, (T)p.cos_t, (T)(1.0 / p.Ca),
                     (T)(1.0 / p.mu), (T)p.ls, nbc, nbg);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? launch_velocity_faces<T>(p) : e;
}

template <typename T>
hipError_t launch_velocity_fill(const Plan &p, const T *Cfin) {
  if (!p.vel_fill || p.G == 0) return hipSuccess;
  const Dims dm = make_dims(p);
  const unsigned nbg = blocks_for(p.G * 16);
  hipLaunchKernelGGL((k_vel_ghosts<T>), dim3(nbg + blocks_for(p.NF)), dim3(kThreads), 0, p.stream, Cfin,
                     (const T *)p.F[0], (const T *)p.F[1], (const T *)p.F[2], p.gidx, (const T *)p.normal,
                     (const T *)p.dn, (const T *)p.gamma, p.apg, (const T *)p.wg, (const T *)p.CMs, (T *)p.UG, p.G,
                     p.K, p.f_cell, p.f_axis, p.f_gL, p.f_gR, (T *)p.stashL, (T *)p.stashR, p.NF, dm, p.d,
                     (T)(0.5 / p.h), (T)p.Cn, (T)p.cos_t, (T)(1.0 / p.Ca), (T)(1.0 / p.mu), (T)p.ls,
                     p.dynamic ? 1 : 0, nbg);
  if (p.NF)
    hipLaunchKernelGGL((k_vel_faces<T>), dim3(blocks_for(p.NF)), dim3(kThreads), 0, p.stream, (T *)p.F[0],
                       (T *)p.F[1], (T *)p.F[2], (const T *)p.UG, p.G, p.f_cell, p.f_axis, p.f_gL, p.f_gR,
                       (const T *)p.stashL, (const T *)p.stashR, p.NF);
  return hipGetLastError();
}

}  // namespace

// The fills that end a step, on the new field C: ghost values of C, then the velocity fill
// (with the static condition both in one launch plus the face pass).
template <typename T>
hipError_t launch_step_fills(const Plan &p, T *C, KernelTimer *tm) {
  hipError_t e = hipSuccess;
  auto mark = [&](const char *name) {
    if (tm && e == hipSuccess) e = tm->mark(name, p.stream);
  };
  if (!p.dynamic && p.vel_fill && p.G) {
    mark("ghost_fills");
    if (e == hipSuccess) e = launch_static_fills<T>(p, C);
  } else {
    mark("ghost_fill_C");
    if (e == hipSuccess) e = launch_ghost_fill<T>(p, C, 0);
    if (p.vel_fill && p.G) mark("ghost_fill_u");
    if (e == hipSuccess) e = launch_velocity_fill<T>(p, C);
  }
  return e;
}

template <typename T>
hipError_t enqueue_step(const Plan &p, int cur, KernelTimer *tm) {
  const T *Cn = (const T *)p.C[cur];
  T *Cp = (T *)p.C[1 - cur];
  hipError_t e = hipSuccess;
  auto mark = [&](const char *name) {
    if (tm && e == hipSuccess) e = tm->mark(name, p.stream);
  };
  const bool split = p.d == 3 && p.shape[0].unroll >= 6 && zm_ok(p);
  if (p.G) {
    mark("ghost_dphi");
    if (e == hipSuccess) e = launch_ghost_patch<T>(p, Cn, Cp);
  }
  mark(split ? "rhs_stencil" : "rhs_xdht");
  if (e == hipSuccess)
    e = p.d == 2 ? launch_rhs<T, 2>(p, Cn, Cp, p.shape[0], true) : launch_rhs<T, 3>(p, Cn, Cp, p.shape[0], true);
  if (split) {
    mark("xdht_fwd");
    if (e == hipSuccess) e = launch_xdht<T>(p, (const T *)p.W, (T *)p.W, p.shape[3]);
  }
  if (e == hipSuccess) e = launch_spectral_tail<T>(p, tm);
  mark("xdht_out");
  if (e == hipSuccess) e = launch_xdht<T>(p, (const T *)p.W, Cp, p.shape[3]);
  if (e == hipSuccess) e = launch_step_fills<T>(p, Cp, tm);
  if (tm && e == hipSuccess) e = tm->end(p.stream);
  return e;
}

// Times every candidate shape of each pass on the state's buffers (the spectral workspace
// only; the fields are not modified) and keeps the fastest.  `out` receives the chosen
// shapes.  The candidates: lines/columns per tile from 2 to the 32 KB LDS limit, radix 8 or
// 16, and 1 or 2 cells in flight per thread in the fused rhs pass.
template <typename T>
hipError_t tune_shapes(Plan &p, int cur, int reps) {
  constexpr int E = tile_elems<T>();
  hipEvent_t e0, e1;
  hipError_t e = hipEventCreate(&e0);
  if (e != hipSuccess) return e;
  e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    (void)hipEventDestroy(e0);
    return e;
  }
  auto time_it = [&](auto &&launch) -> float {
    float best = 1e30f;
    for (int w = 0; w < 2 && e == hipSuccess; ++w) e = launch();
    for (int r = 0; r < reps && e == hipSuccess; ++r) {
      e = hipEventRecord(e0, p.stream);
      if (e == hipSuccess) e = launch();
      if (e == hipSuccess) e = hipEventRecord(e1, p.stream);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (ms < best) best = ms;
    }
    return best;
  };
  // the transform passes are timed where the step runs them, right after the passes before them
  // (untimed): repeated on their own, W stays in the 256 MB Infinity Cache, which the fused rhs
  // pass's streaming traffic flushes in a real step, and the tuner would favour other shapes
  auto time_after = [&](auto &&pre, auto &&launch) -> float {
    float best = 1e30f;
    for (int w = 0; w < 2 && e == hipSuccess; ++w) {
      e = pre();
      if (e == hipSuccess) e = launch();
    }
    for (int r = 0; r < reps && e == hipSuccess; ++r) {
      e = pre();
      if (e == hipSuccess) e = hipEventRecord(e0, p.stream);
      if (e == hipSuccess) e = launch();
      if (e == hipSuccess) e = hipEventRecord(e1, p.stream);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (ms < best) best = ms;
    }
    return best;
  };
  const T *Cn = (const T *)p.C[cur];
  const T *Cp = (const T *)p.C[1 - cur];
  e = launch_ghost_patch<T>(p, Cn, Cp);   // the rhs candidates read the ghost patch
  auto rhs = [&]() { return p.d == 2 ? launch_rhs<T, 2>(p, Cn, Cp, p.shape[0]) : launch_rhs<T, 3>(p, Cn, Cp, p.shape[0]); };
  // pass 0: fused rhs
  if (e == hipSuccess) {
    const int hi = max_log_lines(p, E);
    float best = 1e30f;
    Plan::Shape bs = p.shape[0];
    for (int lt = 1; lt <= hi; ++lt)
      for (int radix : {4, 8, 16})
        for (int un : {1, 2, 3, 4, 5, 6, 7, 8}) {
          const int zl = un >= 6 ? un - 3 : un;
          if (radix == 4 && (p.d != 3 || un < 3 || un > 5 || lt > 2)) continue;   // z-march only
          if (un >= 3 && p.d == 2 && (un != 3 || !ym_ok(p))) continue;
          if (un >= 3 && p.d == 3 && (!zm_ok(p) || lt > 3 || (1 << lt) > p.n[1] || (1 << zl) > p.n[2])) continue;
          if (un >= 6 && radix == 16) continue;   // the stencil-only kernel has no transform
          Plan::Shape sh{lt, radix, un};
          const float t = time_it([&]() {
            return p.d == 2 ? launch_rhs<T, 2>(p, Cn, Cp, sh) : launch_rhs<T, 3>(p, Cn, Cp, sh);
          });
          if (e != hipSuccess) break;
          if (t < best) {
            best = t;
            bs = sh;
          }
        }
    p.shape[0] = bs;
  }
  // pass 1: strided Hartley (3D); pass 2: bounded-axis solve (in place on W)
  if (p.d == 3 && e == hipSuccess) {
    const int hi = max_log_cols(p, p.n[1], E);
    float best = 1e30f;
    Plan::Shape bs = p.shape[1];
    for (int lt = 1; lt <= hi; ++lt)
      for (int radix : {8, 16}) {
        Plan::Shape sh{lt, radix, 1};
        // the shape serves the forward pass (after the rhs) and the inverse one (after the solve)
        const float t = time_after(rhs, [&]() { return launch_ydht<T>(p, sh); }) +
                        time_after([&]() {
                          hipError_t r = rhs();
                          if (r == hipSuccess) r = launch_ydht<T>(p, sh);
                          return r == hipSuccess ? launch_neumann<T>(p, p.shape[2]) : r;
                        }, [&]() { return launch_ydht<T>(p, sh); });
        if (e != hipSuccess) break;
        if (t < best) {
          best = t;
          bs = sh;
        }
      }
    p.shape[1] = bs;
  }
  if (e == hipSuccess) {
    const int hi = max_log_cols(p, p.n[p.d - 1], E);
    float best = 1e30f;
    Plan::Shape bs = p.shape[2];
    for (int lt = 1; lt <= hi; ++lt)
      for (int radix : {8, 16}) {
        Plan::Shape sh{lt, radix, 1};
        const float t = time_after([&]() {
          hipError_t r = rhs();
          return (r == hipSuccess && p.d == 3) ? launch_ydht<T>(p, p.shape[1]) : r;
        }, [&]() { return launch_neumann<T>(p, sh); });
        if (e != hipSuccess) break;
        if (t < best) {
          best = t;
          bs = sh;
        }
      }
    p.shape[2] = bs;
  }
  // pass 3: x Hartley, W -> W (in place: each tile is read whole before it is written)
  if (e == hipSuccess) {
    const int hi = max_log_lines(p, E);
    float best = 1e30f;
    Plan::Shape bs = p.shape[3];
    for (int lt = 1; lt <= hi; ++lt)
      for (int radix : {8, 16}) {
        Plan::Shape sh{lt, radix, 1};
        const float t = time_after([&]() {
          hipError_t r = rhs();
          if (r == hipSuccess) r = launch_spectral_tail<T>(p);
          return r;
        }, [&]() { return launch_xdht<T>(p, (const T *)p.W, (T *)p.W, sh); });
        if (e != hipSuccess) break;
        if (t < best) {
          best = t;
          bs = sh;
        }
      }
    p.shape[3] = bs;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return e;
}

template <typename T>
hipError_t enqueue_initial_fill(const Plan &p, int cur) {
  T *C = (T *)p.C[cur];
  hipError_t e = launch_ghost_fill<T>(p, C, 1);
  if (e != hipSuccess) return e;
  e = launch_velocity_fill<T>(p, C);
  if (e != hipSuccess) return e;
  return hipMemcpyAsync(p.C[1 - cur], p.C[cur], (size_t)p.N * sizeof(T), hipMemcpyDeviceToDevice, p.stream);
}

template <typename T>
hipError_t enqueue_ghost_refresh(const Plan &p, int cur) {
  if (p.dynamic) return hipErrorInvalidValue;   // the dynamic fill advances C_I: not repeatable
  return launch_ghost_fill<T>(p, (T *)p.C[cur], 2);
}

template <typename T>
hipError_t enqueue_rhs(const Plan &p, int cur, void *out) {
  const Dims dm = make_dims(p);
  const RhsCoef<T> cf = make_coef<T>(p);
  const T *F2 = (const T *)(p.d == 3 ? adv_face(p, 2) : adv_face(p, 1));
  hipError_t e = launch_ghost_patch<T>(p, (const T *)p.C[cur], (const T *)p.C[1 - cur]);
  if (e != hipSuccess) return e;
  if (p.d == 2)
    hipLaunchKernelGGL((k_rhs_only<T, 2>), dim3(blocks_for(p.N)), dim3(kThreads), 0, p.stream, (const T *)p.C[cur],
                       (const T *)p.C[1 - cur], (const T *)adv_face(p, 0), (const T *)adv_face(p, 1), F2, (T *)out, dm, cf, p.N);
  else
    hipLaunchKernelGGL((k_rhs_only<T, 3>), dim3(blocks_for(p.N)), dim3(kThreads), 0, p.stream, (const T *)p.C[cur],
                       (const T *)p.C[1 - cur], (const T *)adv_face(p, 0), (const T *)adv_face(p, 1), F2, (T *)out, dm, cf, p.N);
  e = hipGetLastError();
  return e == hipSuccess ? launch_rhs_patch<T>(p, (T *)out) : e;
}

template <typename T>
hipError_t enqueue_solve(const Plan &p, const void *in, void *out) {
  hipError_t e = launch_xdht<T>(p, (const T *)in, (T *)p.W, p.shape[3]);
  if (e != hipSuccess) return e;
  if ((e = launch_spectral_tail<T>(p)) != hipSuccess) return e;
  return launch_xdht<T>(p, (const T *)p.W, (T *)out, p.shape[3]);
}

template <typename T>
hipError_t enqueue_poisson(const Plan &p) {
  Plan q = p;
  q.poisson = 1;
  hipError_t e = launch_xdht<T>(q, (const T *)q.W, (T *)q.W, q.shape[3]);
  if (e != hipSuccess) return e;
  if ((e = launch_spectral_tail<T>(q)) != hipSuccess) return e;
  return launch_xdht<T>(q, (const T *)q.W, (T *)q.W, q.shape[3]);
}

template <typename T>
hipError_t enqueue_velocity_fill(const Plan &p, const void *Cfin) {
  return launch_velocity_fill<T>(p, (const T *)Cfin);
}

template <typename T>
hipError_t enqueue_phi(const Plan &p, int cur, void *out) {
  const Dims dm = make_dims(p);
  const T cn2 = (T)(p.Cn * p.Cn), ih2 = (T)(1.0 / (p.h * p.h));
  if (p.d == 2)
    hipLaunchKernelGGL((k_phi<T, 2>), dim3(blocks_for(p.N)), dim3(kThreads), 0, p.stream, (const T *)p.C[cur],
                       (T *)out, dm, cn2, ih2, p.N);
  else if (stencil_zm_ok(p))
    hipLaunchKernelGGL((k_phi_zm<T>), dim3(stencil_zm_blocks(p)), dim3(kThreads), 0, p.stream, (const T *)p.C[cur],
                       (T *)out, dm, cn2, ih2, stencil_zm_log(p));
  else
    hipLaunchKernelGGL((k_phi<T, 3>), dim3(blocks_for(p.N)), dim3(kThreads), 0, p.stream, (const T *)p.C[cur],
                       (T *)out, dm, cn2, ih2, p.N);
  if (p.G)
    hipLaunchKernelGGL((k_phi_ghost<T>), dim3(blocks_for(p.G)), dim3(kThreads), 0, p.stream, (T *)out, p.gidx, p.ap,
                       (const T *)p.w, p.G, p.K);
  return hipGetLastError();
}

template <typename T>
hipError_t enqueue_diag(const Plan &p, int cur) {
  const Dims dm = make_dims(p);
  if (p.d == 2)
    hipLaunchKernelGGL((k_diag_partial<T, 2>), dim3(p.nred), dim3(kThreads), 0, p.stream, (const T *)p.C[cur],
                       (const T *)p.alpha, (double *)p.partial, dm, p.Cn, 1.0 / p.h, 0.25 / p.Cn, p.N);
  int nred = p.nred;
  if (p.d == 3) {
    // z-march when whole 64 x 4 column tiles fit and the block count fits the partial buffer
    // (p.nred blocks); thicker z-chunks until it does
    int64_t blocks = -1;
    int zc = 16;
    if (p.n[0] % 64 == 0 && p.n[1] % 4 == 0) {
      const int64_t cols = (int64_t)(p.n[0] / 64) * (p.n[1] / 4);
      for (;; zc *= 2) {
        blocks = cols * ((p.n[2] + zc - 1) / zc);
        if (blocks <= p.nred || zc >= p.n[2]) break;
      }
    }
    if (blocks > 0 && blocks <= p.nred) {
      nred = (int)blocks;
      hipLaunchKernelGGL((k_diag_partial_zm<T>), dim3((unsigned)blocks), dim3(kThreads), 0, p.stream,
                         (const T *)p.C[cur], (const T *)p.alpha, (double *)p.partial, dm, p.Cn, 1.0 / p.h,
                         0.25 / p.Cn, zc);
    } else {
      hipLaunchKernelGGL((k_diag_partial<T, 3>), dim3(p.nred), dim3(kThreads), 0, p.stream, (const T *)p.C[cur],
                         (const T *)p.alpha, (double *)p.partial, dm, p.Cn, 1.0 / p.h, 0.25 / p.Cn, p.N);
    }
  }
  hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(kThreads), 0, p.stream, (const double *)p.partial, nred,
                     (double *)p.red_out);
  return hipGetLastError();
}

template <typename T>
int max_log_tile(const Plan &p, int pass) {
  constexpr int E = tile_elems<T>();
  if (pass == 0 || pass == 3) return max_log_lines(p, E);
  return max_log_cols(p, p.n[pass == 1 ? 1 : p.d - 1], E);
}

template int max_log_tile<double>(const Plan &, int);
template int max_log_tile<float>(const Plan &, int);
template hipError_t tune_shapes<double>(Plan &, int, int);
template hipError_t tune_shapes<float>(Plan &, int, int);
template hipError_t enqueue_step<double>(const Plan &, int, KernelTimer *);
template hipError_t enqueue_step<float>(const Plan &, int, KernelTimer *);
template hipError_t enqueue_initial_fill<double>(const Plan &, int);
template hipError_t enqueue_initial_fill<float>(const Plan &, int);
template hipError_t enqueue_ghost_refresh<double>(const Plan &, int);
template hipError_t enqueue_ghost_refresh<float>(const Plan &, int);
template hipError_t enqueue_rhs<double>(const Plan &, int, void *);
template hipError_t enqueue_rhs<float>(const Plan &, int, void *);
template hipError_t enqueue_solve<double>(const Plan &, const void *, void *);
template hipError_t enqueue_solve<float>(const Plan &, const void *, void *);
template hipError_t enqueue_poisson<double>(const Plan &);
template hipError_t enqueue_poisson<float>(const Plan &);
template hipError_t enqueue_velocity_fill<double>(const Plan &, const void *);
template hipError_t enqueue_velocity_fill<float>(const Plan &, const void *);
template <typename T>
hipError_t enqueue_explicit_step(const Plan &p, int cur, int first, KernelTimer *tm) {
  if (!p.R) return hipErrorInvalidValue;
  const T *Cn = (const T *)p.C[cur];
  T *Cnext = (T *)p.C[1 - cur];
  hipError_t e = hipSuccess;
  auto mark = [&](const char *name) {
    if (tm && e == hipSuccess) e = tm->mark(name, p.stream);
  };
  mark("phi");
  if (e == hipSuccess) e = enqueue_phi<T>(p, cur, p.W);
  mark("explicit_update");
  if (e == hipSuccess) {
    const Dims dm = make_dims(p);
    const T hih = (T)(0.5 / p.h), ih2 = (T)(1.0 / (p.h * p.h)), ipe = (T)(1.0 / p.Pe), dt = (T)p.dt;
    const T *F2 = (const T *)(p.d == 3 ? p.F[2] : p.F[1]);
    if (p.d == 2)
      hipLaunchKernelGGL((k_explicit<T, 2>), dim3(blocks_for(p.N)), dim3(kThreads), 0, p.stream, Cn,
                         (const T *)p.W, (const T *)p.F[0], (const T *)p.F[1], F2, (T *)p.R, Cnext, dm, hih, ih2,
                         ipe, dt, first, p.N);
    else if (stencil_zm_ok(p))
      hipLaunchKernelGGL((k_explicit_zm<T>), dim3(stencil_zm_blocks(p)), dim3(kThreads), 0, p.stream, Cn,
                         (const T *)p.W, (const T *)p.F[0], (const T *)p.F[1], F2, (T *)p.R, Cnext, dm, hih, ih2,
                         ipe, dt, first, stencil_zm_log(p));
    else
      hipLaunchKernelGGL((k_explicit<T, 3>), dim3(blocks_for(p.N)), dim3(kThreads), 0, p.stream, Cn,
                         (const T *)p.W, (const T *)p.F[0], (const T *)p.F[1], F2, (T *)p.R, Cnext, dm, hih, ih2,
                         ipe, dt, first, p.N);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = launch_step_fills<T>(p, Cnext, tm);
  if (tm && e == hipSuccess) e = tm->end(p.stream);
  return e;
}

template <typename T>
hipError_t enqueue_scalar_fill(const Plan &p, void *f, double a, double b, double g, const void *g_ghost) {
  if (!p.G) return hipSuccess;
  hipLaunchKernelGGL((k_scalar_fill<T>), dim3(blocks_for(p.G)), dim3(kThreads), 0, p.stream, (T *)f, p.gidx, p.ap,
                     (const T *)p.w, (const T *)p.dn, (const T *)p.gamma, (const T *)g_ghost, (T)g, (T)a, (T)b, p.G,
                     p.K);
  return hipGetLastError();
}

template hipError_t enqueue_scalar_fill<double>(const Plan &, void *, double, double, double, const void *);
template hipError_t enqueue_scalar_fill<float>(const Plan &, void *, double, double, double, const void *);
template hipError_t enqueue_explicit_step<double>(const Plan &, int, int, KernelTimer *);
template hipError_t enqueue_explicit_step<float>(const Plan &, int, int, KernelTimer *);
template hipError_t enqueue_phi<double>(const Plan &, int, void *);
template hipError_t enqueue_phi<float>(const Plan &, int, void *);
template hipError_t enqueue_diag<double>(const Plan &, int);
template hipError_t enqueue_diag<float>(const Plan &, int);

}  // namespace chib

// =======================================================================================
// Batched sweep: many independent 2D cases advanced together.  Each phase of the step is
// one grouped launch over all cases: block b belongs to the case c with
// off[c] <= b < off[c+1] (per-case tile counts, prefix-summed), whose pointers, sizes,
// coefficients and tile shapes are read from a descriptor in device memory.  No block ever
// waits for another; the order between phases is the stream order (or the graph's edges).
namespace chib {

template <typename T>
struct CaseDesc {
  T *C[2];                 // C[p] = C^n and C[1-p] = C^(n-1) (then C^(n+1)) for launch parity p
  T *F0, *F1, *W;
  Dims dm;
  RhsCoef<T> cf;
  const T *twr0, *twi0, *twr1, *twi1, *lamx, *lamy, *dctc, *dcts;
  T a, alpha_s, inv_norm;
  int logL_rhs, logL_out, logB, lognxb;
  const int *gidx, *ap;
  const T *dn, *gam, *normal, *w;
  T *CGn, *CGnm1, *CMs, *UG;
  int64_t G, NF;
  int K, vel_fill;
  T cb, inv2h, Cn, cos_t, inv_Ca, inv_mu, ls;
  const int *f_cell, *f_axis, *f_gL, *f_gR;
  T *stashL, *stashR;
  unsigned nbg;
  RhsPatch<T> rp;          // dphi/dn = 0 at the ghosts: the rhs patch
  T *dg, *pl_dq;           // [G], [NP]: written by kb_dphi, kb_dq
  const int *pl_ref;       // [5][NP]
  int64_t NP;
  T cn2, inv_h2, inv_cn2;
};

namespace {

__device__ __forceinline__ int find_case(const int *__restrict__ off, int n, int b) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= b) lo = mid;
    else hi = mid;
  }
  return lo;
}

template <typename T, int E, int U, int R>
__global__ __launch_bounds__(kThreads) void kb_rhs(const CaseDesc<T> *__restrict__ cs, const int *__restrict__ off,
                                                   int n, int parity) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int c = find_case(off, n, blockIdx.x);
  const CaseDesc<T> &d = cs[c];
  rhs_xdht_body<T, 2, E, U, R>(smem_raw, d.C[parity], d.C[1 - parity], d.F0, d.F1, d.F1, d.W, d.dm, d.cf,
                               d.logL_rhs, d.twr0, d.twi0, (int)(blockIdx.x - off[c]), d.rp);
}

// dg of every ghost of every case, then dq of every patched cell, before the rhs pass.
template <typename T>
__global__ __launch_bounds__(kThreads) void kb_dphi(const CaseDesc<T> *__restrict__ cs, const int *__restrict__ off,
                                                    int n, int parity) {
  const int c = find_case(off, n, blockIdx.x);
  const CaseDesc<T> &d = cs[c];
  ghost_dphi_body<T>(d.C[parity], d.C[1 - parity], d.gidx, d.ap, d.w, d.dg, d.G, d.K, d.dm, 2, d.cn2, d.inv_h2,
                     d.inv_cn2, (int64_t)(blockIdx.x - off[c]));
}

template <typename T>
__global__ __launch_bounds__(kThreads) void kb_dq(const CaseDesc<T> *__restrict__ cs, const int *__restrict__ off,
                                                  int n) {
  const int c = find_case(off, n, blockIdx.x);
  const CaseDesc<T> &d = cs[c];
  const int64_t e = (int64_t)(blockIdx.x - off[c]) * blockDim.x + threadIdx.x;
  if (e >= d.NP) return;
  T acc = T(0);
  for (int j = 1; j < 5; ++j) {
    const int id = d.pl_ref[(int64_t)j * d.NP + e];
    if (id >= 0) acc += d.dg[id];
  }
  const int own = d.pl_ref[e];
  if (own >= 0) acc -= T(4) * d.dg[own];
  d.pl_dq[e] = acc * d.inv_h2;
}

template <typename T, int R>
__global__ __launch_bounds__(kThreads, R == 8 ? 4 : 3) void kb_rhs_ym(const CaseDesc<T> *__restrict__ cs,
                                                      const int *__restrict__ off, int n, int parity) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int c = find_case(off, n, blockIdx.x);
  const CaseDesc<T> &d = cs[c];
  const int t = (int)(blockIdx.x - off[c]);
  // the same instantiation as the single-state launch for this width, so results match bit for bit
  if (d.dm.nx <= 256)
    rhs_ym_body<T, 1, R>(smem_raw, d.C[parity], d.C[1 - parity], d.F0, d.F1, d.W, d.dm, d.cf, d.logL_rhs, d.twr0, d.twi0, t, d.rp);
  else if (d.dm.nx <= 512)
    rhs_ym_body<T, 2, R>(smem_raw, d.C[parity], d.C[1 - parity], d.F0, d.F1, d.W, d.dm, d.cf, d.logL_rhs, d.twr0, d.twi0, t, d.rp);
  else
    rhs_ym_body<T, 4, R>(smem_raw, d.C[parity], d.C[1 - parity], d.F0, d.F1, d.W, d.dm, d.cf, d.logL_rhs, d.twr0, d.twi0, t, d.rp);
}

template <typename T, int E, int R>
__global__ __launch_bounds__(kThreads) void kb_neumann(const CaseDesc<T> *__restrict__ cs, const int *__restrict__ off,
                                                       int n) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int c = find_case(off, n, blockIdx.x);
  const CaseDesc<T> &d = cs[c];
  neumann_body<T, E, R>(smem_raw, d.W, d.dm.lny, (int64_t)d.dm.nx, d.logB, d.lognxb, (int64_t)0, d.lamx,
                        (const T *)nullptr, d.lamy, d.a, d.alpha_s, d.inv_norm, d.twr1, d.twi1, d.dctc, d.dcts,
                        (int)(blockIdx.x - off[c]), 0);
}

template <typename T, int E, int R>
__global__ __launch_bounds__(kThreads) void kb_out(const CaseDesc<T> *__restrict__ cs, const int *__restrict__ off,
                                                   int n, int parity) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int c = find_case(off, n, blockIdx.x);
  const CaseDesc<T> &d = cs[c];
  xdht_body<T, E, R>(smem_raw, d.W, d.C[1 - parity], d.dm.lnx, d.logL_out, d.twr0, d.twi0,
                     (int)(blockIdx.x - off[c]));
}

// Static C fill and (with the velocity fill) the ghost velocities of every case in one launch:
// per case, the first blocks fill C, the following ones compute ghost velocities and face stashes.
template <typename T>
__global__ __launch_bounds__(kThreads) void kb_fill(const CaseDesc<T> *__restrict__ cs, const int *__restrict__ off,
                                                    int n, int parity) {
  const int c = find_case(off, n, blockIdx.x);
  const CaseDesc<T> &d = cs[c];
  const int64_t t = (int64_t)(blockIdx.x - off[c]);
  const int64_t nbc = (d.G * 16 + kThreads - 1) / kThreads;
  if (t < nbc) {
    fill_static_body<T>(d.C[1 - parity], d.gidx, d.dn, d.gam, d.ap, d.w, d.CGn, d.CGnm1, d.CMs, d.G, d.K, d.cb, 0, t);
    return;
  }
  vel_ghosts_body<T>(d.C[1 - parity], d.F0, d.F1, d.F1, d.gidx, d.normal, d.dn, d.gam, d.ap, d.w, d.CMs, d.UG, d.G,
                     d.K, d.f_cell, d.f_axis, d.f_gL, d.f_gR, d.stashL, d.stashR, d.NF, d.dm, 2, d.inv2h, d.Cn,
                     d.cos_t, d.inv_Ca, d.inv_mu, d.ls, 0, d.nbg, t - nbc);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void kb_velf(const CaseDesc<T> *__restrict__ cs, const int *__restrict__ off,
                                                    int n) {
  const int c = find_case(off, n, blockIdx.x);
  const CaseDesc<T> &d = cs[c];
  vel_faces_body<T>(d.F0, d.F1, d.F1, d.UG, d.G, d.f_cell, d.f_axis, d.f_gL, d.f_gR, d.stashL, d.stashR, d.NF,
                    (int64_t)(blockIdx.x - off[c]));
}

}  // namespace

// Host side: descriptors from the member plans, per-phase tile offsets, one batched step.
template <typename T>
void fill_case_desc(const Plan &p, int cur, void *desc_host) {
  CaseDesc<T> d{};
  d.C[0] = (T *)p.C[cur];
  d.C[1] = (T *)p.C[1 - cur];
  d.F0 = (T *)p.F[0];
  d.F1 = (T *)p.F[1];
  d.W = (T *)p.W;
  d.dm = make_dims(p);
  d.cf = make_coef<T>(p);
  d.twr0 = (const T *)p.twr[0];
  d.twi0 = (const T *)p.twi[0];
  d.twr1 = (const T *)p.twr[1];
  d.twi1 = (const T *)p.twi[1];
  d.lamx = (const T *)p.lam[0];
  d.lamy = (const T *)p.lam[1];
  d.dctc = (const T *)p.dctc;
  d.dcts = (const T *)p.dcts;
  d.a = (T)p.a;
  d.alpha_s = (T)p.alpha_s;
  d.inv_norm = (T)(1.0 / (double)p.N);
  constexpr int E = tile_elems<T>();
  d.logL_rhs = clamp_log(p.shape[0].log_tile, max_log_lines(p, E));
  d.logL_out = clamp_log(p.shape[3].log_tile, max_log_lines(p, E));
  d.logB = clamp_log(p.shape[2].log_tile, max_log_cols(p, p.n[1], E));
  d.lognxb = p.logn[0] - d.logB;
  d.gidx = p.gidx;
  d.ap = p.apg;   // the batch's ghost kernels take the ghost-major tables
  d.dn = (const T *)p.dn;
  d.gam = (const T *)p.gamma;
  d.normal = (const T *)p.normal;
  d.w = (const T *)p.wg;
  d.CGn = (T *)p.CGn;
  d.CGnm1 = (T *)p.CGnm1;
  d.CMs = (T *)p.CMs;
  d.UG = (T *)p.UG;
  d.G = p.G;
  d.NF = p.NF;
  d.K = p.K;
  d.vel_fill = p.vel_fill && p.G > 0;
  d.cb = (T)(p.cos_t / (1.4142135623730951 * p.Cn));
  d.inv2h = (T)(0.5 / p.h);
  d.Cn = (T)p.Cn;
  d.cos_t = (T)p.cos_t;
  d.inv_Ca = (T)(1.0 / p.Ca);
  d.inv_mu = (T)(1.0 / p.mu);
  d.ls = (T)p.ls;
  d.f_cell = p.f_cell;
  d.f_axis = p.f_axis;
  d.f_gL = p.f_gL;
  d.f_gR = p.f_gR;
  d.stashL = (T *)p.stashL;
  d.stashR = (T *)p.stashR;
  d.nbg = blocks_for(p.G * 16);
  d.rp = make_patch<T>(p);
  d.dg = (T *)p.dg;
  d.pl_dq = (T *)p.pl_dq;
  d.pl_ref = p.pl_ref;
  d.NP = p.NP;
  d.cn2 = (T)(p.Cn * p.Cn);
  d.inv_h2 = (T)(1.0 / (p.h * p.h));
  d.inv_cn2 = (T)(1.0 / (p.Cn * p.Cn));
  std::memcpy(desc_host, &d, sizeof(d));
}

template <typename T>
size_t case_desc_bytes() {
  return sizeof(CaseDesc<T>);
}

// Per-phase tile counts of one case (0 rhs, 1 neumann, 2 out, 3 fill, 4 dphi, 5 velf, 6 dq) and the
// LDS bytes of its tiles (0 rhs, 1 neumann, 2 out).
template <typename T>
void case_tiles(const Plan &p, int *tiles, size_t *lds) {
  constexpr int E = tile_elems<T>();
  const int lr = clamp_log(p.shape[0].log_tile, max_log_lines(p, E));
  const int lo = clamp_log(p.shape[3].log_tile, max_log_lines(p, E));
  const int lb = clamp_log(p.shape[2].log_tile, max_log_cols(p, p.n[1], E));
  tiles[0] = p.n[1] >> lr;
  tiles[1] = p.n[0] >> lb;
  tiles[2] = p.n[1] >> lo;
  const bool vf = p.vel_fill && p.G > 0;
  tiles[3] = (int)blocks_for(p.G * 16) + (vf ? (int)(blocks_for(p.G * 16) + blocks_for(p.NF)) : 0);
  const bool pt = make_patch<T>(p).dq != nullptr;
  tiles[4] = pt ? (int)blocks_for(p.G * 16) : 0;   // (the ghost velocities run inside phase 3)
  tiles[5] = vf ? (int)blocks_for(p.NF) : 0;
  tiles[6] = pt ? (int)blocks_for(p.NP) : 0;
  lds[0] = (size_t)(1 << lr) * line_pitch(p.n[0]) * sizeof(T);
  lds[1] = (size_t)col_tile(p.n[1], 1 << lb) * sizeof(T);
  lds[2] = (size_t)(1 << lo) * line_pitch(p.n[0]) * sizeof(T);
  lds[3] = ym_ok(p) ? lds[0] + (size_t)ym_extra(p.n[0]) * sizeof(T) : 0;   // 0: no y-march
}

template <typename T>
hipError_t enqueue_batch_step(const BatchLaunch &bl, int parity) {
  constexpr int E = tile_elems<T>();
  const CaseDesc<T> *cs = (const CaseDesc<T> *)bl.descs;
  const int n = bl.n;
  const int *off = bl.off;
  auto O = [&](int ph) { return off + ph * (n + 1); };
  const unsigned nb0 = bl.total[0], nb1 = bl.total[1], nb2 = bl.total[2];
  const unsigned nb3 = bl.total[3], nb4 = bl.total[4], nb5 = bl.total[5], nb6 = bl.total[6];
  const bool r8 = bl.radix_rhs <= 8, u2 = bl.unroll >= 2;
  if (nb4) hipLaunchKernelGGL((kb_dphi<T>), dim3(nb4), dim3(kThreads), 0, bl.stream, cs, O(4), n, parity);
  if (nb6) hipLaunchKernelGGL((kb_dq<T>), dim3(nb6), dim3(kThreads), 0, bl.stream, cs, O(6), n);
  if (bl.unroll == 3 && bl.lds[3]) {
    if (r8) hipLaunchKernelGGL((kb_rhs_ym<T, 8>), dim3(nb0), dim3(kThreads), bl.lds[3], bl.stream, cs, O(0), n, parity);
    else hipLaunchKernelGGL((kb_rhs_ym<T, 16>), dim3(nb0), dim3(kThreads), bl.lds[3], bl.stream, cs, O(0), n, parity);
  } else if (r8 && u2) hipLaunchKernelGGL((kb_rhs<T, E, 2, 8>), dim3(nb0), dim3(kThreads), bl.lds[0], bl.stream, cs, O(0), n, parity);
  else if (r8) hipLaunchKernelGGL((kb_rhs<T, E, 1, 8>), dim3(nb0), dim3(kThreads), bl.lds[0], bl.stream, cs, O(0), n, parity);
  else if (u2) hipLaunchKernelGGL((kb_rhs<T, E, 2, 16>), dim3(nb0), dim3(kThreads), bl.lds[0], bl.stream, cs, O(0), n, parity);
  else hipLaunchKernelGGL((kb_rhs<T, E, 1, 16>), dim3(nb0), dim3(kThreads), bl.lds[0], bl.stream, cs, O(0), n, parity);
  if (bl.radix_neu == 8) hipLaunchKernelGGL((kb_neumann<T, E, 8>), dim3(nb1), dim3(kThreads), bl.lds[1], bl.stream, cs, O(1), n);
  else hipLaunchKernelGGL((kb_neumann<T, E, 16>), dim3(nb1), dim3(kThreads), bl.lds[1], bl.stream, cs, O(1), n);
  if (bl.radix_out == 8) hipLaunchKernelGGL((kb_out<T, E, 8>), dim3(nb2), dim3(kThreads), bl.lds[2], bl.stream, cs, O(2), n, parity);
  else hipLaunchKernelGGL((kb_out<T, E, 16>), dim3(nb2), dim3(kThreads), bl.lds[2], bl.stream, cs, O(2), n, parity);
  if (nb3) hipLaunchKernelGGL((kb_fill<T>), dim3(nb3), dim3(kThreads), 0, bl.stream, cs, O(3), n, parity);
  if (nb5) hipLaunchKernelGGL((kb_velf<T>), dim3(nb5), dim3(kThreads), 0, bl.stream, cs, O(5), n);
  return hipGetLastError();
}

template void fill_case_desc<double>(const Plan &, int, void *);
template void fill_case_desc<float>(const Plan &, int, void *);
template size_t case_desc_bytes<double>();
template size_t case_desc_bytes<float>();
template void case_tiles<double>(const Plan &, int *, size_t *);
template void case_tiles<float>(const Plan &, int *, size_t *);
template hipError_t enqueue_batch_step<double>(const BatchLaunch &, int);
template hipError_t enqueue_batch_step<float>(const BatchLaunch &, int);

}  // namespace chib
