// Fused Krylov pass on 2-D lattices (hot loop of the probing estimator).
//
// Per probe j and pass, with alpha = alpha_k and beta = beta_{k-1}:
//   p_k     = r_k + beta p_{k-1}
//   s       = Q p_k                              (never stored)
//   omega_i = sum_{c(x) = j} (dQ_i p_k)(x)        (gradient dots)
//   r_{k+1} = r_k - alpha s
//   gamma' = r'.r', delta' = r'.Q r', rho' = sum_{c(x) = j} r'(x)
// storing r_{k+1} and p_k: with FP32 storage, 16 B per site, the minimum for
// reading and writing r and p once.  Arithmetic is FP64 throughout.
//
// Work decomposition ("wave march"): one wave64 owns a strip of W = 64 - 4R
// lattice columns (R = stencil radius: 1 for the 5-point M, 2 for M @ M) and
// `rows` rows.  Lane l holds column x0 - 2R + l; the wave walks down the rows
// y0 - 2R .. y0 + rows + 2R - 1, loading one row of r and p per step
// (prefetched five rows ahead), and assembles Q p row by row: the contribution
// of an arriving row to the stencil sums of the rows within distance R is
// added to a ring of per-row accumulators held in registers; horizontal
// neighbours come from lane shuffles.  A row of s is complete R steps after it
// arrives, a row of Q r' another R steps later.  Waves are independent: no LDS
// arrays and no workgroup barriers.  Dot products are reduced per wave and
// written as one partial per (probe, quantity, wave tile); the next launch
// reduces them (tail.h).
#include "ldq_internal.h"
#include "tail.h"

namespace ldq {

__device__ inline double shfl_d(float v, int src) { return (double)__shfl(v, src, 64); }
__device__ inline double shfl_d(double v, int src) { return __shfl(v, src, 64); }

// (A^T A v)(x, yo) from the 9 coefficient planes at site so and the values of
// v at columns x - 1, x, x + 1 of rows yo - 1 (m), yo (c), yo + 1 (p).
template <typename T>
__device__ inline double obs_apply(const T *o, size_t n, size_t so, T lm, T cm, T rm, T lc, T cc, T rc, T lp, T cp,
                                   T rp) {
  return (double)o[0 * n + so] * (double)lm + (double)o[1 * n + so] * (double)cm + (double)o[2 * n + so] * (double)rm +
         (double)o[3 * n + so] * (double)lc + (double)o[4 * n + so] * (double)cc + (double)o[5 * n + so] * (double)rc +
         (double)o[6 * n + so] * (double)lp + (double)o[7 * n + so] * (double)cp + (double)o[8 * n + so] * (double)rp;
}

template <typename T, int R, bool OBS, int NG>
__global__ __launch_bounds__(64) void pass2d_kernel(Pass2D<T> a) {
  constexpr int W = 64 - 4 * R;
  const int lane = threadIdx.x;
  const int L = xcd_remap(blockIdx.x, gridDim.x);
  const int probe = L / a.ntiles, tile = L - probe * a.ntiles;
  const Step step = pass_prologue<1>(a.tail, probe, tile, a.ntiles, a.mode);
  if (!step.run) return;
  const int colour = step.colour;
  const double alpha = a.mode == MODE_INIT ? 0.0 : step.alpha;
  const double beta = step.beta;
  const bool gen = a.mode != MODE_STEP;          // r_k = p_k = v_j, generated from the colouring
  const bool store = a.mode != MODE_INIT;

  const int nx = a.nx, ny = a.ny;
  const size_t n = (size_t)nx * ny;
  const size_t off = (size_t)probe * n;
  const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
  const int x0 = tx * W, y0 = ty * a.rows;
  const int yb = min(y0 + a.rows, ny);
  const int x = x0 - 2 * R + lane;
  const bool xin = x >= 0 && x < nx;
  const bool xout = lane >= 2 * R && lane < 64 - 2 * R && x < nx;   // output column of this strip
  const int nrows = (yb - y0) + 4 * R;
  const int ylo = y0 - 2 * R;                      // lattice row of step 0
  const int degx = (x > 0) + (x < nx - 1);
  const double c = a.kappa2 + 4.0;                 // M = (kappa2 + 4) I - (axis neighbours)
  const int srcL1 = max(lane - 1, 0), srcR1 = min(lane + 1, 63);
  const int srcL2 = max(lane - 2, 0), srcR2 = min(lane + 2, 63);

  // Modular colouring c(x, y) = (x + a y) mod C, tracked as (x mod C) + (a y mod C).
  const int C = a.colC;
  const int cx = (C > 0 && xin) ? x % C : 0;
  const int astep = C > 0 ? a.cola % C : 0;
  int ay = 0;
  if (C > 0) {
    const long t = ((long)a.cola * (long)ylo) % C;
    ay = (int)(t < 0 ? t + C : t);
  }

  // prefetch queue (five rows ahead): r_k and p_{k-1}, or the generated probe
  T qr[5], qp[5];
  unsigned qmine = 0;   // bit u: site of prefetch slot u belongs to the probe
  auto fetch = [&](int slot, int i) {
    const int y = ylo + i;
    const bool in = xin && y >= 0 && y < ny && i < nrows;
    bool mine = false;
    if (in) {
      if (C > 0) {
        int v = cx + ay;
        v -= (v >= C) ? C : 0;
        mine = (v == colour);
      } else {
        mine = a.colours[(size_t)y * nx + x] == colour;
      }
    }
    if (C > 0) {
      ay += astep;
      ay -= (ay >= C) ? C : 0;
    }
    if (gen) {
      qr[slot] = mine ? T(1) : T(0);
      qp[slot] = T(0);
    } else {
      const size_t s = off + (size_t)y * nx + x;
      qr[slot] = in ? a.r_in[s] : T(0);
      qp[slot] = in ? a.p_in[s] : T(0);
    }
    qmine = (qmine & ~(1u << slot)) | ((mine ? 1u : 0u) << slot);
  };
#pragma unroll
  for (int u = 0; u < 5; ++u) fetch(u, u);

  // rings indexed by lattice row mod 5 (indices are compile-time after unrolling)
  double acc[5], acc2[5], obs_s[5], obs_r[5];
  double macc[NG > 0 ? NG : 1][5];
  T rq[5], pq[5], rnq[5], pl[5], pr[5], rl[5], rr[5];
  double k2q[5];
  unsigned mine = 0;    // bit (row mod 5): site (x, row) belongs to the probe
#pragma unroll
  for (int u = 0; u < 5; ++u) {
    acc[u] = acc2[u] = obs_s[u] = obs_r[u] = 0.0;
    rq[u] = pq[u] = rnq[u] = pl[u] = pr[u] = rl[u] = rr[u] = T(0);
    k2q[u] = 0.0;
#pragma unroll
    for (int g = 0; g < (NG > 0 ? NG : 1); ++g) macc[g][u] = 0.0;
  }
  constexpr int NQ = LDQ_NQ_BASE + NG;
  double q[NQ];
#pragma unroll
  for (int i = 0; i < NQ; ++i) q[i] = 0.0;

  for (int i0 = 0; i0 < nrows; i0 += 5) {
#pragma unroll
    for (int u = 0; u < 5; ++u) {
      const int i = i0 + u;
      if (i < nrows) {
        const int y = ylo + i;
        const bool in = xin && y >= 0 && y < ny;
        // ---- row y arrives: p_k = r_k + beta p_{k-1}, rounded to the storage precision
        const T r_y = qr[u];
        const T p_y = gen ? r_y : (T)((double)r_y + beta * (double)qp[u]);
        mine = (mine & ~(1u << u)) | (qmine & (1u << u));
        fetch(u, i + 5);
        rq[u] = r_y;
        pq[u] = p_y;
        const double p = p_y;
        const double h1 = shfl_d(p_y, srcL1) + shfl_d(p_y, srcR1);
        double k2 = a.kappa2;
        if constexpr (R == 1) {
          if (a.kappa2_field) k2 = in ? (double)a.kappa2_field[(size_t)y * nx + x] : 0.0;
        }
        k2q[u] = k2;
        if constexpr (OBS) {
          pl[u] = __shfl(p_y, srcL1, 64);
          pr[u] = __shfl(p_y, srcR1, 64);
        }
        if constexpr (R == 2) {
          // M @ M: row y adds p to rows y -+ 2, 2 h1 - 2c p to rows y -+ 1 and
          // (c^2 + deg) p - 2c h1 + h2 to row y
          const double h2 = shfl_d(p_y, srcL2) + shfl_d(p_y, srcR2);
          const int deg = degx + (y > 0) + (y < ny - 1);
          const double t1 = 2.0 * h1 - 2.0 * c * p;
          acc[(u + 3) % 5] += p;                                      // row y - 2 complete
          acc[(u + 4) % 5] += t1;
          acc[u] += (c * c + (double)deg) * p - 2.0 * c * h1 + h2;
          acc[(u + 1) % 5] += t1;
          acc[(u + 2) % 5] = p;                                       // row y + 2 starts
        } else {
          // M: row y adds -p to rows y -+ 1 and (kappa2 + 4) p - h1 to row y
          acc[(u + 4) % 5] -= p;                                      // row y - 1 complete
          acc[u] += (k2 + 4.0) * p - h1;
          acc[(u + 1) % 5] = -p;                                      // row y + 1 starts
        }
        if constexpr (OBS) {
          // tau (A^T A p) of row y - 1, from rows y - 2 .. y
          const int yo = y - 1;
          double v = 0.0;
          if (xin && yo >= 0 && yo < ny) {
            const int um = (u + 3) % 5, uc = (u + 4) % 5;
            v = obs_apply(a.obs, n, (size_t)yo * nx + x, pl[um], pq[um], pr[um], pl[uc], pq[uc], pr[uc], pl[u], pq[u],
                          pr[u]);
          }
          obs_s[(u + 4) % 5] = a.tau * v;
        }
        // ---- gradient dots w_g . p_k over the probe's sites of row y - 1
        {
          const int yg = y - 1;
          const int ug = (u + 4) % 5;
          const bool gout = xout && yg >= y0 && yg < yb && ((mine >> ug) & 1u);
#pragma unroll
          for (int g = 0; g < NG; ++g) {
            {
              const GradTerm<T> &gt = a.grad[g];
              if (gt.kind == GK_SHIFTED) {
                const double kd = gt.field ? (in ? (double)gt.field[(size_t)y * nx + x] : 0.0) : gt.kappa2;
                macc[g][ug] -= p;                                     // row y - 1 complete
                if (gout) q[LDQ_NQ_BASE + g] += gt.scale * macc[g][ug];
                macc[g][u] += (kd + 4.0) * p - h1;
                macc[g][(u + 1) % 5] = -p;
              } else if (gt.kind == GK_DIAG) {
                if (gout) q[LDQ_NQ_BASE + g] += gt.scale * (double)gt.field[(size_t)yg * nx + x] * (double)pq[ug];
              } else if constexpr (OBS) {
                // GK_OBS (the host allows it only when Q has an observation term)
                if (gout) {
                  const int um = (u + 3) % 5;
                  q[LDQ_NQ_BASE + g] += gt.scale * obs_apply(gt.obs, n, (size_t)yg * nx + x, pl[um], pq[um], pr[um],
                                                             pl[ug], pq[ug], pr[ug], pl[u], pq[u], pr[u]);
                }
              }
            }
          }
        }
        // ---- row ys = y - R of s = Q p_k is complete: r_{k+1} = r_k - alpha s
        const int ys = y - R;
        const int us = (u + 5 - R) % 5;
        const bool sin = xin && ys >= 0 && ys < ny;
        double sv = a.scale * acc[us];
        if constexpr (OBS) sv += obs_s[us];
        const T rn = sin ? (T)((double)rq[us] - alpha * sv) : T(0);
        rnq[us] = rn;
        if (store && xout && ys >= y0 && ys < yb) {
          const size_t so = off + (size_t)ys * nx + x;
          a.r_out[so] = rn;
          a.p_out[so] = pq[us];
        }
        // ---- row ys of r_{k+1} enters the Q r' accumulators
        const double rv = rn;
        const double g1 = shfl_d(rn, srcL1) + shfl_d(rn, srcR1);
        if constexpr (OBS) {
          rl[us] = __shfl(rn, srcL1, 64);
          rr[us] = __shfl(rn, srcR1, 64);
        }
        if constexpr (R == 2) {
          const double g2 = shfl_d(rn, srcL2) + shfl_d(rn, srcR2);
          const int deg = degx + (ys > 0) + (ys < ny - 1);
          const double t1 = 2.0 * g1 - 2.0 * c * rv;
          acc2[(us + 3) % 5] += rv;                                   // row ys - 2 complete
          acc2[(us + 4) % 5] += t1;
          acc2[us] += (c * c + (double)deg) * rv - 2.0 * c * g1 + g2;
          acc2[(us + 1) % 5] += t1;
          acc2[(us + 2) % 5] = rv;
        } else {
          acc2[(us + 4) % 5] -= rv;                                   // row ys - 1 complete
          acc2[us] += (k2q[us] + 4.0) * rv - g1;
          acc2[(us + 1) % 5] = -rv;
        }
        if constexpr (OBS) {
          const int yo = ys - 1;
          double v = 0.0;
          if (xin && yo >= 0 && yo < ny) {
            const int um = (us + 3) % 5, uc = (us + 4) % 5;
            v = obs_apply(a.obs, n, (size_t)yo * nx + x, rl[um], rnq[um], rr[um], rl[uc], rnq[uc], rr[uc], rl[us],
                          rnq[us], rr[us]);
          }
          obs_r[(us + 4) % 5] = a.tau * v;
        }
        // ---- row yd = ys - R of Q r_{k+1} is complete: dot products
        const int yd = ys - R;
        const int ud = (us + 5 - R) % 5;
        if (xout && yd >= y0 && yd < yb) {
          double qv = a.scale * acc2[ud];
          if constexpr (OBS) qv += obs_r[ud];
          const double r2 = rnq[ud];
          q[0] += r2 * r2;
          q[1] += r2 * qv;
          if ((mine >> ud) & 1u) q[2] += r2;
        }
      }
    }
  }
  pass_epilogue_n<NQ>(a.tail, probe, tile, a.ntiles, q);
}

template <typename T, int R, bool OBS>
static void launch_ng(const Pass2D<T> &a, int nblocks, hipStream_t stream) {
  switch (a.tail.ngrad) {
    case 0: hipLaunchKernelGGL((pass2d_kernel<T, R, OBS, 0>), dim3(nblocks), dim3(64), 0, stream, a); break;
    case 1: hipLaunchKernelGGL((pass2d_kernel<T, R, OBS, 1>), dim3(nblocks), dim3(64), 0, stream, a); break;
    default: hipLaunchKernelGGL((pass2d_kernel<T, R, OBS, 2>), dim3(nblocks), dim3(64), 0, stream, a); break;
  }
}

// ngrad <= 2 (checked by the host driver for 2-D lattices)
template <typename T>
hipError_t launch_pass2d(const Pass2D<T> &a, bool squared, bool obs, hipStream_t stream) {
  const int nblocks = a.ntiles * a.nprobes;
  if (squared && obs)
    launch_ng<T, 2, true>(a, nblocks, stream);
  else if (squared)
    launch_ng<T, 2, false>(a, nblocks, stream);
  else
    launch_ng<T, 1, false>(a, nblocks, stream);
  return hipGetLastError();
}

template hipError_t launch_pass2d<float>(const Pass2D<float> &, bool, bool, hipStream_t);
template hipError_t launch_pass2d<double>(const Pass2D<double> &, bool, bool, hipStream_t);

// Wave tiles: 64 - 4R columns by `rows` rows.
void pass2d_tiles(int nx, int ny, bool squared, int rows, int *tiles_x, int *ntiles) {
  const int W = squared ? 56 : 60;
  *tiles_x = (nx + W - 1) / W;
  *ntiles = *tiles_x * ((ny + rows - 1) / rows);
}

}  // namespace ldq
