// Fused Krylov pass on 2-D lattices (hot loop of the probing estimator).
//
// One workgroup owns a TX x TY tile of one probe.  With alpha = alpha_k and
// beta = beta_{k-1} of that probe it performs, in FP64 arithmetic on stored
// FP32 (LDQ_MIXED) or FP64 vectors:
//   p_k     = r_k + beta p_{k-1}              (tile + 2R halo, LDS)
//   s       = Q p_k                           (tile + R halo, never stored)
//   omega_i = sum_{c(s) = j} (dQ_i p_k)_s      (gradient dots, tile)
//   r_{k+1} = r_k - alpha s                   (tile + R halo, LDS)
//   gamma' = r'.r', delta' = r'.Q r', rho' = sum_{c(s) = j} r'_s   (tile)
// and writes r_{k+1}, p_k for the tile (16 B per site in FP32: the algorithmic
// minimum of reading and writing r and p once).  The scalars alpha_{k+1},
// beta_k and the per-shift recurrences are then advanced by the last workgroup
// of the probe (tail.h).  R is the stencil radius: 1 for the 5-point M,
// 2 for the 13-point M @ M (plus the 9-point observation term A^T A).
#include "ldq_internal.h"
#include "tail.h"

namespace ldq {

constexpr int T2X = 64, T2Y = 16;

template <typename T>
__device__ inline int colour2(const Pass2D<T> &a, int x, int y) {
  return a.colC > 0 ? (x + a.cola * y) % a.colC : a.colours[(size_t)y * a.nx + x];
}

// 9-point observation term (A^T A v)(x, y) from an LDS array with zero halo.
template <typename T, int W>
__device__ inline double obs9(const T *obs, size_t n, size_t s, const T (*X)[W], int px, int py) {
  double acc = 0.0;
#pragma unroll
  for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
    for (int dx = -1; dx <= 1; ++dx)
      acc += (double)obs[(size_t)((dy + 1) * 3 + (dx + 1)) * n + s] * (double)X[py + dy][px + dx];
  return acc;
}

// (kappa2 + 4) v - (4 axis neighbours): the 5-point M applied at (px, py).
template <typename T, int W>
__device__ inline double m5(double k2, const T (*X)[W], int px, int py) {
  return (k2 + 4.0) * (double)X[py][px] -
         ((double)X[py][px - 1] + (double)X[py][px + 1] + (double)X[py - 1][px] + (double)X[py + 1][px]);
}

// M @ M with constant kappa2 applied at (px, py); deg = in-box axis neighbours
// of the site (the diagonal of M @ M is (kappa2 + 4)^2 + deg).
template <typename T, int W>
__device__ inline double m13(double c, int deg, const T (*X)[W], int px, int py) {
  const double v = X[py][px];
  const double ax = (double)X[py][px - 1] + (double)X[py][px + 1] + (double)X[py - 1][px] + (double)X[py + 1][px];
  const double dg = (double)X[py - 1][px - 1] + (double)X[py - 1][px + 1] + (double)X[py + 1][px - 1] +
                    (double)X[py + 1][px + 1];
  const double fr = (double)X[py][px - 2] + (double)X[py][px + 2] + (double)X[py - 2][px] + (double)X[py + 2][px];
  return (c * c + (double)deg) * v - 2.0 * c * ax + 2.0 * dg + fr;
}

template <typename T, bool SQ, bool OBS, int W>
__device__ inline double applyQ2(const Pass2D<T> &a, const T (*X)[W], int px, int py, int gx, int gy, size_t s,
                                 size_t n) {
  double q;
  if constexpr (SQ) {
    const int deg = (gx > 0) + (gx < a.nx - 1) + (gy > 0) + (gy < a.ny - 1);
    q = a.scale * m13<T, W>(a.kappa2 + 4.0, deg, X, px, py);
  } else {
    const double k2 = a.kappa2_field ? (double)a.kappa2_field[s] : a.kappa2;
    q = a.scale * m5<T, W>(k2, X, px, py);
  }
  if constexpr (OBS) q += a.tau * obs9<T, W>(a.obs, n, s, X, px, py);
  return q;
}

template <typename T, int W>
__device__ inline double applyD2(const GradTerm<T> &g, const T (*X)[W], int px, int py, size_t s, size_t n) {
  if (g.kind == GK_DIAG) return g.scale * (double)g.field[s] * (double)X[py][px];
  if (g.kind == GK_SHIFTED) {
    const double k2 = g.field ? (double)g.field[s] : g.kappa2;
    return g.scale * m5<T, W>(k2, X, px, py);
  }
  return g.scale * obs9<T, W>(g.obs, n, s, X, px, py);
}

template <typename T, bool SQ, bool OBS>
__global__ __launch_bounds__(LDQ_BLOCK) void pass2d_kernel(Pass2D<T> a) {
  constexpr int R = SQ ? 2 : 1, H = 2 * R;
  constexpr int PW = T2X + 2 * H, PH = T2Y + 2 * H;
  constexpr int RW = T2X + 2 * R, RH = T2Y + 2 * R;
  __shared__ T sP[PH][PW];
  __shared__ T sR[RH][RW];
  __shared__ T sRN[RH][RW];

  const int L = xcd_remap(blockIdx.x, gridDim.x);
  const int probe = L / a.ntiles, tile = L - probe * a.ntiles;
  const ProbeState *st = a.tail.st + probe;
  if (!st->active) return;
  const int colour = st->colour;
  const double alpha = st->alpha, beta = st->beta_prev;
  const int tx0 = (tile % a.tiles_x) * T2X, ty0 = (tile / a.tiles_x) * T2Y;
  const size_t n = (size_t)a.nx * a.ny;
  const size_t off = (size_t)probe * n;
  const int tid = threadIdx.x;
  const int nq = LDQ_NQ_BASE + a.tail.ngrad;
  double q[LDQ_NQ_MAX];
#pragma unroll
  for (int i = 0; i < LDQ_NQ_MAX; ++i) q[i] = 0.0;

  if (a.mode == MODE_INIT) {
    // r_0 = v_j on the tile + R halo; no vector is written
    for (int e = tid; e < RW * RH; e += LDQ_BLOCK) {
      const int ry = e / RW, rx = e - ry * RW;
      const int gx = tx0 - R + rx, gy = ty0 - R + ry;
      T v = 0;
      if (gx >= 0 && gx < a.nx && gy >= 0 && gy < a.ny) v = (colour2(a, gx, gy) == colour) ? T(1) : T(0);
      sRN[ry][rx] = v;
    }
    __syncthreads();
  } else {
    // stage 1: p_k = r_k + beta p_{k-1} on tile + H, r_k on tile + R
    for (int e = tid; e < PW * PH; e += LDQ_BLOCK) {
      const int ey = e / PW, ex = e - ey * PW;
      const int gx = tx0 - H + ex, gy = ty0 - H + ey;
      T r = 0, p = 0;
      if (gx >= 0 && gx < a.nx && gy >= 0 && gy < a.ny) {
        const size_t s = (size_t)gy * a.nx + gx;
        if (a.mode == MODE_FIRST) {
          r = (colour2(a, gx, gy) == colour) ? T(1) : T(0);
          p = r;
        } else {
          r = a.r_in[off + s];
          p = (T)((double)r + beta * (double)a.p_in[off + s]);
        }
      }
      sP[ey][ex] = p;
      const int rx = ex - (H - R), ry = ey - (H - R);
      if (rx >= 0 && rx < RW && ry >= 0 && ry < RH) sR[ry][rx] = r;
    }
    __syncthreads();
    // stage 2: s = Q p_k, r_{k+1} = r_k - alpha s on tile + R; store the tile
    for (int e = tid; e < RW * RH; e += LDQ_BLOCK) {
      const int ry = e / RW, rx = e - ry * RW;
      const int gx = tx0 - R + rx, gy = ty0 - R + ry;
      const int px = rx + (H - R), py = ry + (H - R);
      T rn = 0;
      if (gx >= 0 && gx < a.nx && gy >= 0 && gy < a.ny) {
        const size_t s = (size_t)gy * a.nx + gx;
        const double sv = applyQ2<T, SQ, OBS, PW>(a, sP, px, py, gx, gy, s, n);
        rn = (T)((double)sR[ry][rx] - alpha * sv);
        if (rx >= R && rx < R + T2X && ry >= R && ry < R + T2Y) {
          a.r_out[off + s] = rn;
          a.p_out[off + s] = sP[py][px];
          if (colour2(a, gx, gy) == colour)
#pragma unroll
            for (int i = 0; i < LDQ_MAXP; ++i)
              if (i < a.tail.ngrad) q[LDQ_NQ_BASE + i] += applyD2<T, PW>(a.grad[i], sP, px, py, s, n);
        }
      }
      sRN[ry][rx] = rn;
    }
    __syncthreads();
  }
  // stage 3: dots of r_{k+1} on the tile
  for (int e = tid; e < T2X * T2Y; e += LDQ_BLOCK) {
    const int ty = e / T2X, tx = e - ty * T2X;
    const int gx = tx0 + tx, gy = ty0 + ty;
    if (gx < a.nx && gy < a.ny) {
      const size_t s = (size_t)gy * a.nx + gx;
      const double r = (double)sRN[ty + R][tx + R];
      const double qr = applyQ2<T, SQ, OBS, RW>(a, sRN, tx + R, ty + R, gx, gy, s, n);
      q[0] += r * r;
      q[1] += r * qr;
      if (colour2(a, gx, gy) == colour) q[2] += r;
    }
  }
  finish_pass(a.tail, probe, tile, a.ntiles, nq, a.mode, q);
}

template <typename T>
hipError_t launch_pass2d(const Pass2D<T> &a, bool squared, bool obs, hipStream_t stream) {
  const int nblocks = a.ntiles * a.nprobes;
  if (squared && obs)
    hipLaunchKernelGGL((pass2d_kernel<T, true, true>), dim3(nblocks), dim3(LDQ_BLOCK), 0, stream, a);
  else if (squared)
    hipLaunchKernelGGL((pass2d_kernel<T, true, false>), dim3(nblocks), dim3(LDQ_BLOCK), 0, stream, a);
  else
    hipLaunchKernelGGL((pass2d_kernel<T, false, false>), dim3(nblocks), dim3(LDQ_BLOCK), 0, stream, a);
  return hipGetLastError();
}

template hipError_t launch_pass2d<float>(const Pass2D<float> &, bool, bool, hipStream_t);
template hipError_t launch_pass2d<double>(const Pass2D<double> &, bool, bool, hipStream_t);

void pass2d_tiles(int nx, int ny, int *tiles_x, int *ntiles) {
  *tiles_x = (nx + T2X - 1) / T2X;
  *ntiles = *tiles_x * ((ny + T2Y - 1) / T2Y);
}

}  // namespace ldq
