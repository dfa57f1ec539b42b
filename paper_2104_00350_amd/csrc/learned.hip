// Learned wall-band correction of a coarse 2D run (an extension of the method, not part of the
// paper): a three-layer 3x3 convolutional network maps per-cell features of the coarse state
// [C, phi, wall distance / (band h) clipped to [-2, 2], n_x, n_y] to a correction dC that is added
// to C in the wall band (0 < wall distance <= band cells, |C| < 0.9), after which the ghost
// values are filled again from the corrected field.
//
//   z1 = W1 * X + b1,  h1 = tanh(z1)        5 (padded to 16) -> 32 channels, BF16 MFMA, FP32 acc
//   z2 = W2 * h1 + b2, h2 = tanh(z2)        32 -> 32 channels, BF16 MFMA, FP32 acc
//   dC = s_out (W3 * h2 + b3)               32 -> 1 channel, FP32 FMA on BF16 inputs
//
// "*" is a 3x3 cross-correlation over the full grid, periodic along x and with zero values
// outside the box along y for every layer's input.  The network runs on 16x16 output tiles
// that touch the band: a workgroup stages the 22x22 feature patch in LDS and computes h1 on
// 20x20, h2 on 18x18 and dC on 16x16 cells, so tiles never exchange data.  Weights are BF16
// copies of FP32 master weights, biases FP32; X, h1, h2 and the backward signals that feed
// an MFMA are rounded to BF16 (round to nearest even) where they are stored in LDS.
//
// Training (k_net_train) runs the forward and the whole backward pass of one stored sample
// tile per workgroup and writes that tile's gradient; k_net_adam sums the tiles' gradients in
// a fixed order (deterministic) and takes one Adam step on the FP32 master weights.
//
// MFMA: v_mfma_f32_16x16x16_bf16 with one 64-lane wave per 16x16 output block; lane l holds
// A[l % 16][4 (l / 16) + r], B[4 (l / 16) + r][l % 16] and D[4 (l / 16) + r][l % 16], r = 0..3.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "ch_ib.h"
#include "internal.h"
#include "kernels.h"

namespace chib {
namespace net {

constexpr int TS = 16;            // output tile edge
constexpr int HX = TS + 6;        // feature patch edge
constexpr int E1 = TS + 4;        // h1 region edge
constexpr int E2 = TS + 2;        // h2 region edge
constexpr int CIN = 16;           // stored input channels (NFEAT used, the rest zero)
constexpr int NFEAT = 5;
constexpr int CH = 32;
constexpr int OFF_W1 = 0;                       // [9][CH][CIN]  (tap, out, in)
constexpr int OFF_B1 = OFF_W1 + 9 * CH * CIN;
constexpr int OFF_W2 = OFF_B1 + CH;             // [9][CH][CH]   (tap, out, in)
constexpr int OFF_B2 = OFF_W2 + 9 * CH * CH;
constexpr int OFF_W3 = OFF_B2 + CH;             // [9][CH]       (tap, in)
constexpr int OFF_B3 = OFF_W3 + 9 * CH;
constexpr int NPARAM = OFF_B3 + 1;
constexpr int PSTRIDE = (NPARAM + 63) / 64 * 64;
constexpr int XTILE = HX * HX * CIN;            // BF16 values per stored feature patch
constexpr int kT = 256;
static_assert(NPARAM == CH_IB_NET_NPARAMS, "parameter count of the ABI");

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__host__ __device__ inline unsigned short f2bf(float f) {
  unsigned u;
  std::memcpy(&u, &f, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short b) { return __uint_as_float(((unsigned)b) << 16); }

struct Fields {
  const double *C;
  const double *phi;
  const float *dist;      // [N]
  const float *nrm;       // [2][N]
  int nx, ny, lnx;
  float inv_band;         // 1 / (band cells * h)
  double band;            // band cells * h
};

// Stages the 22x22 feature patch of tile (tx0, ty0) in LDS, X[(y * HX + x) * CIN + k].
__device__ void load_features(unsigned short *X, int tx0, int ty0, const Fields &f) {
  const int64_t N = (int64_t)f.nx * f.ny;
  for (int idx = threadIdx.x; idx < HX * HX; idx += blockDim.x) {
    const int px = idx % HX, py = idx / HX;
    const int gy = ty0 - 3 + py;
    const int gx = (tx0 - 3 + px + f.nx) & (f.nx - 1);
    float v[NFEAT] = {0.f, 0.f, 0.f, 0.f, 0.f};
    if (gy >= 0 && gy < f.ny) {
      const int64_t c = ((int64_t)gy << f.lnx) + gx;
      v[0] = (float)f.C[c];
      v[1] = (float)f.phi[c];
      v[2] = fminf(fmaxf(f.dist[c] * f.inv_band, -2.f), 2.f);
      v[3] = f.nrm[c];
      v[4] = f.nrm[N + c];
    }
    unsigned short *xp = X + idx * CIN;
#pragma unroll
    for (int k = 0; k < CIN; ++k) xp[k] = k < NFEAT ? f2bf(v[k]) : (unsigned short)0;
  }
}

struct Lds {
  unsigned short X[HX * HX * CIN];
  unsigned short H1[E1 * E1 * CH];
  unsigned short H2[E2 * E2 * CH];
  unsigned short W1[9 * CH * CIN];
  unsigned short W2[9 * CH * CH];
  float W3[9 * CH];
  float b1[CH], b2[CH];
  float out[TS * TS];
  float b3;
};

struct LdsTrain {
  Lds f;
  unsigned short G2[E2 * E2 * CH];   // BF16 backward signal at h2 (pre-activation)
  float g3[TS * TS];
  float red[kT];
};

__device__ void load_params(Lds &s, const float *master, const unsigned short *wbf) {
  for (int i = threadIdx.x; i < 9 * CH * CIN; i += blockDim.x) s.W1[i] = wbf[OFF_W1 + i];
  for (int i = threadIdx.x; i < 9 * CH * CH; i += blockDim.x) s.W2[i] = wbf[OFF_W2 + i];
  for (int i = threadIdx.x; i < 9 * CH; i += blockDim.x) s.W3[i] = bf2f(wbf[OFF_W3 + i]);
  if (threadIdx.x < CH) {
    s.b1[threadIdx.x] = master[OFF_B1 + threadIdx.x];
    s.b2[threadIdx.x] = master[OFF_B2 + threadIdx.x];
  }
  if (threadIdx.x == 0) s.b3 = master[OFF_B3];
}

// Forward pass on one tile; s.X and the parameters are staged.  Leaves h1, h2 (BF16) and
// s.out = dC (FP32) of the 16x16 cells.
__device__ void forward(Lds &s, int ty0, int ny, float out_scale) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int i = lane & 15, kg = lane >> 4;
  // layer 1: M = 400 h1 cells (25 blocks), N = 32 channels (2 blocks), K = 9 taps x 16 inputs
  for (int job = wave; job < 25 * 2; job += nw) {
    const int mb = job >> 1, nb = job & 1;
    const int P = mb * 16 + i;
    const int Pc = P < E1 * E1 ? P : 0;
    const int x1 = Pc % E1, y1 = Pc / E1;
    v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int q = (y1 + t / 3) * HX + (x1 + t % 3);
      const v4s a = *(const v4s *)&s.X[q * CIN + 4 * kg];
      const v4s b = *(const v4s *)&s.W1[(t * CH + nb * 16 + i) * CIN + 4 * kg];
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
    }
    const int co = nb * 16 + i;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int Po = mb * 16 + 4 * kg + r;
      if (Po < E1 * E1) {
        const int gy = ty0 - 2 + Po / E1;
        const float hv = (gy >= 0 && gy < ny) ? tanhf(acc[r] + s.b1[co]) : 0.f;
        s.H1[Po * CH + co] = f2bf(hv);
      }
    }
  }
  __syncthreads();
  // layer 2: M = 324 h2 cells (21 blocks), N = 32, K = 9 taps x 32 inputs
  for (int job = wave; job < 21 * 2; job += nw) {
    const int mb = job >> 1, nb = job & 1;
    const int P = mb * 16 + i;
    const int Pc = P < E2 * E2 ? P : 0;
    const int x2 = Pc % E2, y2 = Pc / E2;
    v4f acc = {0.f, 0.f, 0.f, 0.f};
    for (int t = 0; t < 9; ++t) {
      const int q = (y2 + t / 3) * E1 + (x2 + t % 3);
#pragma unroll
      for (int kb = 0; kb < 2; ++kb) {
        const v4s a = *(const v4s *)&s.H1[q * CH + kb * 16 + 4 * kg];
        const v4s b = *(const v4s *)&s.W2[(t * CH + nb * 16 + i) * CH + kb * 16 + 4 * kg];
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
      }
    }
    const int co = nb * 16 + i;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int Po = mb * 16 + 4 * kg + r;
      if (Po < E2 * E2) {
        const int gy = ty0 - 1 + Po / E2;
        const float hv = (gy >= 0 && gy < ny) ? tanhf(acc[r] + s.b2[co]) : 0.f;
        s.H2[Po * CH + co] = f2bf(hv);
      }
    }
  }
  __syncthreads();
  // layer 3: one cell per thread
  if (threadIdx.x < TS * TS) {
    const int x3 = threadIdx.x % TS, y3 = threadIdx.x / TS;
    float acc = 0.f;
    for (int t = 0; t < 9; ++t) {
      const unsigned short *hp = &s.H2[((y3 + t / 3) * E2 + (x3 + t % 3)) * CH];
      const float *wp = &s.W3[t * CH];
#pragma unroll
      for (int c = 0; c < CH; ++c) acc += bf2f(hp[c]) * wp[c];
    }
    s.out[threadIdx.x] = out_scale * (acc + s.b3);
  }
  __syncthreads();
}

__device__ __forceinline__ bool in_band(const Fields &f, int64_t c) {
  const double d = (double)f.dist[c];
  return d > 0.0 && d <= f.band && fabs(f.C[c]) < 0.9;
}

// dC of the band tiles (0 outside the band), written per tile as [tile][16 * 16].
__global__ __launch_bounds__(kT) void k_net_forward(const int2 *tiles, Fields f, const float *master,
                                                    const unsigned short *wbf, float out_scale, float *dC) {
  __shared__ Lds s;
  const int2 tl = tiles[blockIdx.x];
  load_params(s, master, wbf);
  load_features(s.X, tl.x, tl.y, f);
  __syncthreads();
  forward(s, tl.y, f.ny, out_scale);
  const int x = tl.x + threadIdx.x % TS, y = tl.y + threadIdx.x / TS;
  const int64_t c = ((int64_t)y << f.lnx) + x;
  float v = 0.f;
  if (in_band(f, c)) {   // the corrected value stays in the physical range [-1, 1]
    const double Cc = f.C[c];
    const double Cn = fmin(fmax(Cc + (double)s.out[threadIdx.x], -1.0), 1.0);
    v = (float)(Cn - Cc);
  }
  dC[(int64_t)blockIdx.x * TS * TS + threadIdx.x] = v;
}

// C += dC on the tiles' own cells, in both time levels (the correction shifts the state).
__global__ __launch_bounds__(kT) void k_net_add(const int2 *tiles, const float *dC, double *C0, double *C1, int lnx,
                                                double weight) {
  const int2 tl = tiles[blockIdx.x];
  const int x = tl.x + threadIdx.x % TS, y = tl.y + threadIdx.x / TS;
  const int64_t c = ((int64_t)y << lnx) + x;
  const double v = weight * (double)dC[(int64_t)blockIdx.x * TS * TS + threadIdx.x];
  C0[c] += v;
  C1[c] += v;
}

// One training sample per band tile: the feature patch, the target correction (target - C)
// and the band mask of the 16x16 cells.
__global__ __launch_bounds__(kT) void k_net_extract(const int2 *tiles, Fields f, const double *target,
                                                    unsigned short *sX, float *sY, float *sM, int64_t off) {
  __shared__ unsigned short X[HX * HX * CIN];
  const int2 tl = tiles[blockIdx.x];
  load_features(X, tl.x, tl.y, f);
  __syncthreads();
  const int64_t slot = off + blockIdx.x;
  unsigned short *dst = sX + slot * XTILE;
  for (int i = threadIdx.x; i < XTILE; i += blockDim.x) dst[i] = X[i];
  const int x = tl.x + threadIdx.x % TS, y = tl.y + threadIdx.x / TS;
  const int64_t c = ((int64_t)y << f.lnx) + x;
  sY[slot * TS * TS + threadIdx.x] = (float)(target[c] - f.C[c]);
  sM[slot * TS * TS + threadIdx.x] = in_band(f, c) ? 1.f : 0.f;
}

// Forward and backward pass of one stored tile; writes the tile's gradient (PSTRIDE floats) and
// its share of the loss  sum_cells M (dC - Y)^2 * inv_count.
__global__ __launch_bounds__(kT) void k_net_train(const int64_t *ids, const unsigned short *sX, const float *sY,
                                                  const float *sM, const int *tile_y, int ny, const float *master,
                                                  const unsigned short *wbf, float out_scale, float inv_count,
                                                  float *grad, float *tile_loss) {
  __shared__ LdsTrain S;
  Lds &s = S.f;
  const int64_t id = ids[blockIdx.x];
  const int ty0 = tile_y[id];
  load_params(s, master, wbf);
  const unsigned short *src = sX + id * XTILE;
  for (int k = threadIdx.x; k < XTILE; k += blockDim.x) s.X[k] = src[k];
  __syncthreads();
  forward(s, ty0, ny, out_scale);
  float *gout = grad + (int64_t)blockIdx.x * PSTRIDE;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
  const int i = lane & 15, kg = lane >> 4;

  // output layer: g3 = dLoss/d(W3 * h2 + b3)
  {
    const float m = sM[id * TS * TS + tid];
    const float diff = s.out[tid] - sY[id * TS * TS + tid];
    S.red[tid] = m * diff * diff * inv_count;
    S.g3[tid] = 2.f * inv_count * m * diff * out_scale;
  }
  __syncthreads();
  if (tid == 0) {
    float l = 0.f, gb = 0.f;
    for (int k = 0; k < TS * TS; ++k) {
      l += S.red[k];
      gb += S.g3[k];
    }
    tile_loss[blockIdx.x] = l;
    gout[OFF_B3] = gb;
  }
  for (int o = tid; o < 9 * CH; o += blockDim.x) {          // dW3[t][c]
    const int t = o / CH, c = o % CH;
    float acc = 0.f;
    for (int p = 0; p < TS * TS; ++p)
      acc += S.g3[p] * bf2f(s.H2[(((p / TS) + t / 3) * E2 + (p % TS) + t % 3) * CH + c]);
    gout[OFF_W3 + o] = acc;
  }
  for (int o = tid; o < E2 * E2 * CH; o += blockDim.x) {     // signal at z2
    const int q = o / CH, c = o % CH;
    const int x2 = q % E2, y2 = q / E2;
    float acc = 0.f;
    for (int t = 0; t < 9; ++t) {
      const int px = x2 - t % 3, py = y2 - t / 3;
      if (px >= 0 && px < TS && py >= 0 && py < TS) acc += S.g3[py * TS + px] * s.W3[t * CH + c];
    }
    const float hv = bf2f(s.H2[o]);
    const int gy = ty0 - 1 + y2;
    S.G2[o] = f2bf((gy >= 0 && gy < ny) ? acc * (1.f - hv * hv) : 0.f);
  }
  __syncthreads();
  if (tid < CH) {                                            // db2
    float acc = 0.f;
    for (int q = 0; q < E2 * E2; ++q) acc += bf2f(S.G2[q * CH + tid]);
    gout[OFF_B2 + tid] = acc;
  }
  // dW2[t][co][ci] = sum_q G2[q][co] h1[q + tap][ci]: M = ci, N = co, K = 324 cells (21 blocks)
  for (int job = wave; job < 9 * 4; job += nw) {
    const int t = job >> 2, mbk = (job >> 1) & 1, nb = job & 1;
    const int ci = mbk * 16 + i, co = nb * 16 + i;
    v4f acc = {0.f, 0.f, 0.f, 0.f};
    for (int kb = 0; kb < 21; ++kb) {
      v4s a, b;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int q = kb * 16 + 4 * kg + r;
        if (q < E2 * E2) {
          const int x2 = q % E2, y2 = q / E2;
          a[r] = (short)s.H1[((y2 + t / 3) * E1 + x2 + t % 3) * CH + ci];
          b[r] = (short)S.G2[q * CH + co];
        } else {
          a[r] = 0;
          b[r] = 0;
        }
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) gout[OFF_W2 + (t * CH + co) * CH + mbk * 16 + 4 * kg + r] = acc[r];
  }
  __syncthreads();
  // signal at z1, in place of h1: M = 400 h1 cells, N = ci, K = 9 taps x 32 co
  for (int job = wave; job < 25 * 2; job += nw) {
    const int mb = job >> 1, nb = job & 1;
    const int P = mb * 16 + i;
    const int Pc = P < E1 * E1 ? P : 0;
    const int x1 = Pc % E1, y1 = Pc / E1;
    const int ci = nb * 16 + i;
    v4f acc = {0.f, 0.f, 0.f, 0.f};
    for (int t = 0; t < 9; ++t) {
      const int x2 = x1 - t % 3, y2 = y1 - t / 3;
      const bool ok = P < E1 * E1 && x2 >= 0 && x2 < E2 && y2 >= 0 && y2 < E2;
#pragma unroll
      for (int kb = 0; kb < 2; ++kb) {
        v4s a = {0, 0, 0, 0};
        if (ok) a = *(const v4s *)&S.G2[(y2 * E2 + x2) * CH + kb * 16 + 4 * kg];
        v4s b;
#pragma unroll
        for (int r = 0; r < 4; ++r) b[r] = (short)s.W2[(t * CH + kb * 16 + 4 * kg + r) * CH + ci];
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int Po = mb * 16 + 4 * kg + r;
      if (Po < E1 * E1) {
        const float hv = bf2f(s.H1[Po * CH + ci]);
        const int gy = ty0 - 2 + Po / E1;
        s.H1[Po * CH + ci] = f2bf((gy >= 0 && gy < ny) ? acc[r] * (1.f - hv * hv) : 0.f);
      }
    }
  }
  __syncthreads();
  if (tid < CH) {                                            // db1
    float acc = 0.f;
    for (int q = 0; q < E1 * E1; ++q) acc += bf2f(s.H1[q * CH + tid]);
    gout[OFF_B1 + tid] = acc;
  }
  // dW1[t][co][ci] = sum_r G1[r][co] X[r + tap][ci]: M = ci (16), N = co, K = 400 cells (25 blocks)
  for (int job = wave; job < 9 * 2; job += nw) {
    const int t = job >> 1, nb = job & 1;
    const int co = nb * 16 + i;
    v4f acc = {0.f, 0.f, 0.f, 0.f};
    for (int kb = 0; kb < 25; ++kb) {
      v4s a, b;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int q = kb * 16 + 4 * kg + r;                 // < 400 always
        const int x1 = q % E1, y1 = q / E1;
        a[r] = (short)s.X[((y1 + t / 3) * HX + x1 + t % 3) * CIN + i];
        b[r] = (short)s.H1[q * CH + co];
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) gout[OFF_W1 + (t * CH + co) * CIN + 4 * kg + r] = acc[r];
  }
}

// Sums the tiles' gradients in tile order; with lr >= 0 takes one Adam step (beta1 0.9,
// beta2 0.999, eps 1e-8, bias-corrected) and refreshes the BF16 weight copies; always writes
// the summed gradient to gsum (if non-null) and the summed loss to loss[0].
__global__ __launch_bounds__(kT) void k_net_adam(const float *grad, int n, const float *tile_loss, float *master,
                                                 unsigned short *wbf, float *m, float *v, float *gsum, float lr,
                                                 float c1, float c2, float *loss) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    float l = 0.f;
    for (int b = 0; b < n; ++b) l += tile_loss[b];
    loss[0] = l;
  }
  if (j >= NPARAM) return;
  float g = 0.f;
  for (int b = 0; b < n; ++b) g += grad[(int64_t)b * PSTRIDE + j];
  if (gsum) gsum[j] = g;
  if (lr < 0.f) return;
  const float mj = 0.9f * m[j] + 0.1f * g;
  const float vj = 0.999f * v[j] + 0.001f * g * g;
  m[j] = mj;
  v[j] = vj;
  const float p = master[j] - lr * (mj * c1) / (sqrtf(vj * c2) + 1e-8f);
  master[j] = p;
  wbf[j] = f2bf(p);
}

// Coarse C = mean of the 2x2 fine cells it covers.
__global__ __launch_bounds__(kT) void k_restrict2(const double *Cf, int lnxf, double *Cc, int lnxc, int64_t Nc) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= Nc) return;
  const int64_t i = c & ((1 << lnxc) - 1), j = c >> lnxc;
  const int64_t f0 = ((2 * j) << lnxf) + 2 * i, f1 = ((2 * j + 1) << lnxf) + 2 * i;
  Cc[c] = 0.25 * ((Cf[f0] + Cf[f0 + 1]) + (Cf[f1] + Cf[f1 + 1]));
}

// Staggered faces of a 2x finer grid onto the coarse faces: each coarse face is the mean of the two
// fine faces that tile it (x faces: the right faces of fine column 2i+1, rows 2j and 2j+1; y faces:
// the top faces of fine row 2j+1, columns 2i and 2i+1), so the flux through every coarse cell's
// boundary is the fine flux through it and a discretely divergence-free fine field restricts to
// a divergence-free coarse one.
__global__ __launch_bounds__(kT) void k_restrict2_faces(const double *Uf, const double *Vf, int lnxf, double *Uc,
                                                        double *Vc, int lnxc, int64_t Nc) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= Nc) return;
  const int64_t i = c & ((1 << lnxc) - 1), j = c >> lnxc;
  Uc[c] = 0.5 * (Uf[((2 * j) << lnxf) + 2 * i + 1] + Uf[((2 * j + 1) << lnxf) + 2 * i + 1]);
  Vc[c] = 0.5 * (Vf[((2 * j + 1) << lnxf) + 2 * i] + Vf[((2 * j + 1) << lnxf) + 2 * i + 1]);
}

}  // namespace net
}  // namespace chib

using namespace chib::net;

namespace {
struct NetLayout {
  size_t master, wbf, m, v, grad, tile_loss, loss, gsum, phi, dist, nrm, tiles, tile_y, dC, ids, sX, sY, sM, total;
};
size_t al(size_t x) { return (x + 255) & ~(size_t)255; }
NetLayout net_layout(int64_t max_cells, int max_tiles, int64_t max_store, int max_batch) {
  NetLayout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = al(o + bytes); return r; };
  L.master = take(NPARAM * 4);
  L.wbf = take(NPARAM * 2);
  L.m = take(NPARAM * 4);
  L.v = take(NPARAM * 4);
  L.grad = take((size_t)max_batch * PSTRIDE * 4);
  L.tile_loss = take((size_t)max_batch * 4);
  L.loss = take(16);
  L.gsum = take(NPARAM * 4);
  L.phi = take((size_t)max_cells * 8);
  L.dist = take((size_t)max_cells * 4);
  L.nrm = take((size_t)max_cells * 8);
  L.tiles = take((size_t)max_tiles * 8);
  L.tile_y = take((size_t)max_store * 4);
  L.dC = take((size_t)max_tiles * TS * TS * 4);
  L.ids = take((size_t)max_batch * 8);
  L.sX = take((size_t)max_store * XTILE * 2);
  L.sY = take((size_t)max_store * TS * TS * 4);
  L.sM = take((size_t)max_store * TS * TS * 4);
  L.total = o;
  return L;
}
}  // namespace

struct ch_ib_net {
  int64_t max_cells = 0, max_store = 0;
  int max_tiles = 0, max_batch = 0;
  float out_scale = 1.f;
  char *ws = nullptr;
  NetLayout L{};
  hipStream_t stream = nullptr;
  int64_t adam_t = 0;
  // binding
  ch_ib_state *st = nullptr;
  int nx = 0, ny = 0, lnx = 0;
  double h = 0, band = 0;
  std::vector<int2> tiles;
  std::vector<float> host_dist, host_nrm;
  std::vector<int> store_ty;
  template <typename T>
  T *at(size_t off) const { return (T *)(ws + off); }
};

static int net_hip(hipError_t e, const char *where) {
  return chib::fail(CH_IB_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

extern "C" size_t ch_ib_net_workspace_bytes(int64_t max_cells, int max_tiles, int64_t max_store_tiles, int max_batch) {
  if (max_cells <= 0 || max_tiles <= 0 || max_store_tiles < 0 || max_batch <= 0) return 0;
  return net_layout(max_cells, max_tiles, max_store_tiles, max_batch).total;
}

extern "C" int ch_ib_net_create(int64_t max_cells, int max_tiles, int64_t max_store_tiles, int max_batch,
                                double out_scale, void *device_workspace, size_t bytes, void *hip_stream,
                                ch_ib_net **out) {
  if (!out || !device_workspace) return chib::fail(CH_IB_EINVAL, "NULL argument");
  *out = nullptr;
  if (max_cells <= 0 || max_tiles <= 0 || max_store_tiles < 0 || max_batch <= 0 || !(out_scale > 0))
    return chib::fail(CH_IB_EINVAL, "sizes must be positive and out_scale > 0");
  NetLayout L = net_layout(max_cells, max_tiles, max_store_tiles, max_batch);
  if (bytes < L.total) return chib::fail(CH_IB_ENOMEM, "network workspace too small");
  if (((uintptr_t)device_workspace & 255) != 0) return chib::fail(CH_IB_EINVAL, "workspace must be 256-byte aligned");
  ch_ib_net *n = new ch_ib_net;
  n->max_cells = max_cells;
  n->max_tiles = max_tiles;
  n->max_store = max_store_tiles;
  n->max_batch = max_batch;
  n->out_scale = (float)out_scale;
  n->ws = (char *)device_workspace;
  n->L = L;
  n->stream = (hipStream_t)hip_stream;
  n->store_ty.assign((size_t)max_store_tiles, 0);
  hipError_t e = hipMemsetAsync(n->ws, 0, L.total < L.sX ? L.total : L.sX, n->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
  if (e != hipSuccess) {
    delete n;
    return net_hip(e, "net_create");
  }
  *out = n;
  return CH_IB_OK;
}

extern "C" void ch_ib_net_free(ch_ib_net *n) { delete n; }

extern "C" int ch_ib_net_set_params(ch_ib_net *n, const float *params) {
  if (!n || !params) return chib::fail(CH_IB_EINVAL, "NULL argument");
  std::vector<unsigned short> bf(NPARAM);
  for (int j = 0; j < NPARAM; ++j) bf[j] = f2bf(params[j]);
  hipError_t e = hipMemcpyAsync(n->at<float>(n->L.master), params, NPARAM * 4, hipMemcpyHostToDevice, n->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(n->at<unsigned short>(n->L.wbf), bf.data(), NPARAM * 2, hipMemcpyHostToDevice, n->stream);
  if (e == hipSuccess) e = hipMemsetAsync(n->at<float>(n->L.m), 0, NPARAM * 4, n->stream);
  if (e == hipSuccess) e = hipMemsetAsync(n->at<float>(n->L.v), 0, NPARAM * 4, n->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
  if (e != hipSuccess) return net_hip(e, "net_set_params");
  n->adam_t = 0;
  return CH_IB_OK;
}

extern "C" int ch_ib_net_get_params(ch_ib_net *n, float *params) {
  if (!n || !params) return chib::fail(CH_IB_EINVAL, "NULL argument");
  hipError_t e = hipMemcpyAsync(params, n->at<float>(n->L.master), NPARAM * 4, hipMemcpyDeviceToHost, n->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
  return e == hipSuccess ? CH_IB_OK : net_hip(e, "net_get_params");
}

extern "C" int ch_ib_net_bind(ch_ib_net *n, ch_ib_state *st, const double *wall_dist, const double *wall_normal,
                              double band_cells, int *n_tiles) {
  if (!n || !st || !wall_dist || !wall_normal) return chib::fail(CH_IB_EINVAL, "NULL argument");
  chib::StateRef r;
  int rc = chib::state_ref(st, &r);
  if (rc) return rc;
  const chib::Plan &p = *r.plan;
  if (p.d != 2 || r.es != 8) return chib::fail(CH_IB_EUNSUPPORTED, "the learned correction needs a 2D FP64 state");
  if (p.dynamic) return chib::fail(CH_IB_EUNSUPPORTED, "the learned correction needs the static condition");
  if (p.explicit_ab2) return chib::fail(CH_IB_EUNSUPPORTED, "the learned correction needs the semi-implicit scheme");
  if ((p.n[0] % TS) || (p.n[1] % TS)) return chib::fail(CH_IB_EUNSUPPORTED, "grid sizes must be multiples of 16");
  if (p.N > n->max_cells) return chib::fail(CH_IB_EINVAL, "grid larger than max_cells");
  if (!(band_cells > 0)) return chib::fail(CH_IB_EINVAL, "band_cells must be > 0");
  const int nx = p.n[0], ny = p.n[1];
  const double band = band_cells * p.h;
  std::vector<int2> tl;
  for (int ty = 0; ty < ny; ty += TS)
    for (int tx = 0; tx < nx; tx += TS) {
      bool any = false;
      for (int y = ty; y < ty + TS && !any; ++y)
        for (int x = tx; x < tx + TS; ++x) {
          const double d = wall_dist[(int64_t)y * nx + x];
          if (d > 0.0 && d <= band) {
            any = true;
            break;
          }
        }
      if (any) tl.push_back(make_int2(tx, ty));
    }
  if ((int)tl.size() > n->max_tiles) return chib::fail(CH_IB_EINVAL, "more band tiles than max_tiles");
  n->host_dist.assign(wall_dist, wall_dist + p.N);
  n->host_nrm.assign(wall_normal, wall_normal + 2 * p.N);
  std::vector<float> df(n->host_dist.begin(), n->host_dist.end()), nf(n->host_nrm.begin(), n->host_nrm.end());
  hipError_t e = hipMemcpyAsync(n->at<float>(n->L.dist), df.data(), df.size() * 4, hipMemcpyHostToDevice, n->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(n->at<float>(n->L.nrm), nf.data(), nf.size() * 4, hipMemcpyHostToDevice, n->stream);
  if (e == hipSuccess && !tl.empty())
    e = hipMemcpyAsync(n->at<int2>(n->L.tiles), tl.data(), tl.size() * 8, hipMemcpyHostToDevice, n->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
  if (e != hipSuccess) return net_hip(e, "net_bind");
  n->st = st;
  n->nx = nx;
  n->ny = ny;
  n->lnx = p.logn[0];
  n->h = p.h;
  n->band = band;
  n->tiles = tl;
  if (n_tiles) *n_tiles = (int)tl.size();
  return CH_IB_OK;
}

extern "C" int ch_ib_net_rebind(ch_ib_net *n, ch_ib_state *st) {
  if (!n || !st) return chib::fail(CH_IB_EINVAL, "NULL argument");
  if (!n->st) return chib::fail(CH_IB_EINVAL, "network was never bound");
  chib::StateRef r;
  int rc = chib::state_ref(st, &r);
  if (rc) return rc;
  const chib::Plan &p = *r.plan;
  if (p.d != 2 || r.es != 8 || p.dynamic || p.explicit_ab2 || p.n[0] != n->nx || p.n[1] != n->ny || p.h != n->h)
    return chib::fail(CH_IB_EINVAL, "rebind needs a 2D FP64 static state on the bound grid");
  n->st = st;
  return CH_IB_OK;
}

static int net_fields(ch_ib_net *n, chib::StateRef &r, chib::net::Fields &f) {
  if (!n || !n->st) return chib::fail(CH_IB_EINVAL, "network is not bound to a state");
  int rc = chib::state_ref(n->st, &r);
  if (rc) return rc;
  hipError_t e = chib::enqueue_phi<double>(*r.plan, r.cur, n->at<double>(n->L.phi));
  if (e != hipSuccess) return net_hip(e, "phi");
  f.C = (const double *)r.plan->C[r.cur];
  f.phi = n->at<double>(n->L.phi);
  f.dist = n->at<float>(n->L.dist);
  f.nrm = n->at<float>(n->L.nrm);
  f.nx = n->nx;
  f.ny = n->ny;
  f.lnx = n->lnx;
  f.inv_band = (float)(1.0 / n->band);
  f.band = n->band;
  return CH_IB_OK;
}

extern "C" int ch_ib_net_forward(ch_ib_net *n, float *dC_device) {
  chib::StateRef r;
  chib::net::Fields f;
  int rc = net_fields(n, r, f);
  if (rc) return rc;
  if (n->tiles.empty()) return CH_IB_OK;
  float *out = dC_device ? dC_device : n->at<float>(n->L.dC);
  hipLaunchKernelGGL(k_net_forward, dim3((unsigned)n->tiles.size()), dim3(kT), 0, r.plan->stream,
                     n->at<int2>(n->L.tiles), f, n->at<float>(n->L.master), n->at<unsigned short>(n->L.wbf),
                     n->out_scale, out);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? CH_IB_OK : net_hip(e, "net_forward");
}

extern "C" int ch_ib_net_apply(ch_ib_net *n, double weight) {
  if (!(weight >= 0.0 && weight <= 1.0)) return chib::fail(CH_IB_EINVAL, "weight must lie in [0, 1]");
  int rc = ch_ib_net_forward(n, nullptr);
  if (rc) return rc;
  if (n->tiles.empty()) return CH_IB_OK;
  chib::StateRef r;
  rc = chib::state_ref(n->st, &r);
  if (rc) return rc;
  const chib::Plan &p = *r.plan;
  hipLaunchKernelGGL(k_net_add, dim3((unsigned)n->tiles.size()), dim3(kT), 0, p.stream, n->at<int2>(n->L.tiles),
                     n->at<float>(n->L.dC), (double *)p.C[r.cur], (double *)p.C[1 - r.cur], n->lnx, weight);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = chib::enqueue_ghost_refresh<double>(p, r.cur);
  return e == hipSuccess ? CH_IB_OK : net_hip(e, "net_apply");
}

extern "C" int ch_ib_net_extract(ch_ib_net *n, const double *target_device, int64_t store_offset,
                                 float *mask_counts) {
  if (!target_device) return chib::fail(CH_IB_EINVAL, "NULL target");
  chib::StateRef r;
  chib::net::Fields f;
  int rc = net_fields(n, r, f);
  if (rc) return rc;
  const int nt = (int)n->tiles.size();
  if (store_offset < 0 || store_offset + nt > n->max_store) return chib::fail(CH_IB_EINVAL, "sample store is full");
  if (nt == 0) return CH_IB_OK;
  hipLaunchKernelGGL(k_net_extract, dim3((unsigned)nt), dim3(kT), 0, r.plan->stream, n->at<int2>(n->L.tiles), f,
                     target_device, n->at<unsigned short>(n->L.sX), n->at<float>(n->L.sY), n->at<float>(n->L.sM),
                     store_offset);
  for (int b = 0; b < nt; ++b) n->store_ty[(size_t)(store_offset + b)] = n->tiles[b].y;
  hipError_t e = hipGetLastError();
  if (e == hipSuccess)
    e = hipMemcpyAsync(n->at<int>(n->L.tile_y) + store_offset, n->store_ty.data() + store_offset, (size_t)nt * 4,
                       hipMemcpyHostToDevice, r.plan->stream);
  if (e == hipSuccess && mask_counts) {
    std::vector<float> M((size_t)nt * TS * TS);
    e = hipMemcpyAsync(M.data(), n->at<float>(n->L.sM) + store_offset * TS * TS, M.size() * 4, hipMemcpyDeviceToHost,
                       r.plan->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(r.plan->stream);
    if (e == hipSuccess)
      for (int b = 0; b < nt; ++b) {
        float c = 0.f;
        for (int k = 0; k < TS * TS; ++k) c += M[(size_t)b * TS * TS + k];
        mask_counts[b] = c;
      }
  }
  if (e == hipSuccess) e = hipStreamSynchronize(r.plan->stream);
  return e == hipSuccess ? CH_IB_OK : net_hip(e, "net_extract");
}

extern "C" int ch_ib_net_store_get(ch_ib_net *n, int64_t slot, unsigned short *X, float *Y, float *M) {
  if (!n) return chib::fail(CH_IB_EINVAL, "NULL network");
  if (slot < 0 || slot >= n->max_store) return chib::fail(CH_IB_EINVAL, "slot out of range");
  hipError_t e = hipSuccess;
  if (X) e = hipMemcpyAsync(X, n->at<unsigned short>(n->L.sX) + slot * XTILE, XTILE * 2, hipMemcpyDeviceToHost, n->stream);
  if (e == hipSuccess && Y)
    e = hipMemcpyAsync(Y, n->at<float>(n->L.sY) + slot * TS * TS, TS * TS * 4, hipMemcpyDeviceToHost, n->stream);
  if (e == hipSuccess && M)
    e = hipMemcpyAsync(M, n->at<float>(n->L.sM) + slot * TS * TS, TS * TS * 4, hipMemcpyDeviceToHost, n->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
  return e == hipSuccess ? CH_IB_OK : net_hip(e, "net_store_get");
}

static int net_train(ch_ib_net *n, const int64_t *ids, int count, double lr, double inv_count, float *grad_host,
                     double *loss_out) {
  if (!n || !ids) return chib::fail(CH_IB_EINVAL, "NULL argument");
  if (!n->st) return chib::fail(CH_IB_EINVAL, "network is not bound to a state");
  if (count <= 0 || count > n->max_batch) return chib::fail(CH_IB_EINVAL, "batch size out of range");
  for (int b = 0; b < count; ++b)
    if (ids[b] < 0 || ids[b] >= n->max_store) return chib::fail(CH_IB_EINVAL, "sample id out of range");
  hipError_t e = hipMemcpyAsync(n->at<int64_t>(n->L.ids), ids, (size_t)count * 8, hipMemcpyHostToDevice, n->stream);
  if (e != hipSuccess) return net_hip(e, "net_train");
  hipLaunchKernelGGL(k_net_train, dim3((unsigned)count), dim3(kT), 0, n->stream, n->at<int64_t>(n->L.ids),
                     n->at<unsigned short>(n->L.sX), n->at<float>(n->L.sY), n->at<float>(n->L.sM),
                     n->at<int>(n->L.tile_y), n->ny, n->at<float>(n->L.master), n->at<unsigned short>(n->L.wbf),
                     n->out_scale, (float)inv_count, n->at<float>(n->L.grad), n->at<float>(n->L.tile_loss));
  float c1 = 1.f, c2 = 1.f;
  if (lr >= 0) {
    n->adam_t++;
    c1 = (float)(1.0 / (1.0 - std::pow(0.9, (double)n->adam_t)));
    c2 = (float)(1.0 / (1.0 - std::pow(0.999, (double)n->adam_t)));
  }
  hipLaunchKernelGGL(k_net_adam, dim3((NPARAM + kT - 1) / kT), dim3(kT), 0, n->stream, n->at<float>(n->L.grad), count,
                     n->at<float>(n->L.tile_loss), n->at<float>(n->L.master), n->at<unsigned short>(n->L.wbf),
                     n->at<float>(n->L.m), n->at<float>(n->L.v), grad_host ? n->at<float>(n->L.gsum) : nullptr,
                     (float)lr, c1, c2, n->at<float>(n->L.loss));
  e = hipGetLastError();
  if (e == hipSuccess && grad_host)
    e = hipMemcpyAsync(grad_host, n->at<float>(n->L.gsum), NPARAM * 4, hipMemcpyDeviceToHost, n->stream);
  if (e == hipSuccess && loss_out) {
    float l = 0.f;
    e = hipMemcpyAsync(&l, n->at<float>(n->L.loss), 4, hipMemcpyDeviceToHost, n->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
    *loss_out = l;
  }
  if (e == hipSuccess && grad_host) e = hipStreamSynchronize(n->stream);
  return e == hipSuccess ? CH_IB_OK : net_hip(e, "net_train");
}

extern "C" int ch_ib_net_train_step(ch_ib_net *n, const int64_t *sample_ids, int count, double lr, double inv_count,
                                    double *loss_out) {
  if (!(lr >= 0)) return chib::fail(CH_IB_EINVAL, "lr must be >= 0");
  return net_train(n, sample_ids, count, lr, inv_count, nullptr, loss_out);
}

extern "C" int ch_ib_net_gradient(ch_ib_net *n, const int64_t *sample_ids, int count, double inv_count,
                                  float *grad_host, double *loss_out) {
  if (!grad_host) return chib::fail(CH_IB_EINVAL, "NULL gradient buffer");
  return net_train(n, sample_ids, count, -1.0, inv_count, grad_host, loss_out);
}

extern "C" int ch_ib_restrict2(ch_ib_state *fine, ch_ib_state *coarse, int both_levels) {
  chib::StateRef rf, rc_;
  int rc = chib::state_ref(fine, &rf);
  if (rc) return rc;
  rc = chib::state_ref(coarse, &rc_);
  if (rc) return rc;
  const chib::Plan &pf = *rf.plan, &pc = *rc_.plan;
  if (pf.d != 2 || pc.d != 2 || rf.es != 8 || rc_.es != 8)
    return chib::fail(CH_IB_EUNSUPPORTED, "restriction: 2D FP64 states only");
  if (pf.n[0] != 2 * pc.n[0] || pf.n[1] != 2 * pc.n[1])
    return chib::fail(CH_IB_EINVAL, "restriction: the fine grid must have twice the cells per axis");
  if (both_levels && pf.ns != pc.ns)
    return chib::fail(CH_IB_EINVAL, "restriction: both states run the momentum step or neither does");
  // both states on one stream order: the fine state's work is finished before the copy
  hipError_t e = hipStreamSynchronize(pf.stream);
  if (e == hipSuccess) {
    for (int lev = 0; lev < (both_levels ? 2 : 1) && e == hipSuccess; ++lev) {
      const int cf = lev ? 1 - rf.cur : rf.cur, cc = lev ? 1 - rc_.cur : rc_.cur;
      hipLaunchKernelGGL(k_restrict2, dim3((unsigned)((pc.N + kT - 1) / kT)), dim3(kT), 0, pc.stream,
                         (const double *)pf.C[cf], pf.logn[0], (double *)pc.C[cc], pc.logn[0], pc.N);
      e = hipGetLastError();
    }
    if (e == hipSuccess && both_levels && pc.ns) {
      // the momentum state: faces u^n, the advecting 2u^n - u^(n-1) and the previous convective
      // term by face means, both pressure levels by cell means; the history flags follow
      const unsigned nb = (unsigned)((pc.N + kT - 1) / kT);
      hipLaunchKernelGGL(k_restrict2_faces, dim3(nb), dim3(kT), 0, pc.stream, (const double *)pf.F[0],
                         (const double *)pf.F[1], pf.logn[0], (double *)pc.F[0], (double *)pc.F[1], pc.logn[0], pc.N);
      if (pf.Ut[0] && pc.Ut[0])
        hipLaunchKernelGGL(k_restrict2_faces, dim3(nb), dim3(kT), 0, pc.stream, (const double *)pf.Ut[0],
                           (const double *)pf.Ut[1], pf.logn[0], (double *)pc.Ut[0], (double *)pc.Ut[1], pc.logn[0],
                           pc.N);
      hipLaunchKernelGGL(k_restrict2_faces, dim3(nb), dim3(kT), 0, pc.stream, (const double *)pf.Nh[0],
                         (const double *)pf.Nh[1], pf.logn[0], (double *)pc.Nh[0], (double *)pc.Nh[1], pc.logn[0],
                         pc.N);
      for (int k = 0; k < 2; ++k)
        hipLaunchKernelGGL(k_restrict2, dim3(nb), dim3(kT), 0, pc.stream, (const double *)pf.P[k], pf.logn[0],
                           (double *)pc.P[k], pc.logn[0], pc.N);
      e = hipGetLastError();
    }
    if (e == hipSuccess && both_levels) e = chib::enqueue_ghost_refresh<double>(pc, rc_.cur);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(pc.stream);
  if (e != hipSuccess) return net_hip(e, "restrict2");
  if (!both_levels) chib::state_mark_reinit(coarse);
  else if (pc.ns) chib::state_copy_momentum_flags(fine, coarse);
  return CH_IB_OK;
}
