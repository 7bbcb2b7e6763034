// Fused Krylov pass on 2-D lattices (hot loop of the probing estimator).
//
// Per probe j and pass, with alpha = alpha_k and beta = beta_{k-1}:
//   p_k     = r_k + beta p_{k-1}
//   s       = Q p_k                              (never stored)
//   omega_i = sum_{c(x) = j} (dQ_i p_k)(x)        (gradient dots)
//   r_{k+1} = r_k - alpha s
//   gamma' = r'.r', delta' = r'.Q r', rho' = sum_{c(x) = j} r'(x)
// storing r_{k+1} and p_k: with FP32 storage, 16 B per site, the minimum for
// reading and writing r and p once.
//
// Q is scale * M (5-point, R = 1) or scale * M @ M (13-point, R = 2), M =
// kappa2 I + L symmetric, plus optionally tau A^T A.  delta' needs M r' on the
// tile's own sites only: r'.M r' for R = 1 and |M r'|^2 for R = 2 (M
// symmetric), so the halo around a tile is H = R + 1 sites (r' on the own
// sites +- 1, hence s there, hence p on +- (R + 1)).
//
// Work decomposition ("wave march"): one wave64 owns a strip of W = 64 - 2H
// lattice columns and `rows` rows.  Lane l holds column x0 - H + l; the wave
// walks down the rows y0 - H .. y0 + rows + H - 1, loading one row of r and p
// per step (prefetched five rows ahead), and assembles Q p row by row: the
// contribution of an arriving row to the stencil sums of the rows within
// distance R is added to a ring of per-row accumulators held in registers;
// horizontal neighbours come from DPP lane shifts.  A row of s is complete R
// steps after it arrives, a row of M r' one step later.  Waves are
// independent: no LDS and no workgroup barriers.  Dot products are reduced per
// wave and written as one partial per (probe, quantity, wave tile); the next
// launch reduces them (tail.h).  rows + 2H is a multiple of 5 (the ring
// length), so the unrolled row loop needs no bounds check.
#include <type_traits>

#include "ldq_internal.h"
#include "tail.h"
#include "bufio.h"


namespace ldq {

// Lane i receives lane i - 1 (left neighbour column) / lane i + 1 (right)
// through a DPP wave shift; lanes without a source read 0 (bound_ctrl), and
// the strip edges never use them.
__device__ inline float from_left(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x138, 0xF, 0xF, true));
}
__device__ inline float from_right(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x130, 0xF, 0xF, true));
}
__device__ inline double from_left(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), 0x138, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x138, 0xF, 0xF, true);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}
__device__ inline double from_right(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), 0x130, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x130, 0xF, 0xF, true);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

// Buffer accesses: uniform resource and row offset (SGPRs) plus a per-lane
// byte offset, so no per-lane address arithmetic is needed; accesses outside
// num_records read 0 / are dropped by the hardware range check.
__device__ inline float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ inline double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

// (A^T A v)(x, yo) from the 9 coefficient planes at site so and the values of
// v at columns x - 1, x, x + 1 of rows yo - 1 (m), yo (c), yo + 1 (p).
template <typename T>
__device__ inline double obs_apply(const T *o, size_t n, size_t so, T lm, T cm, T rm, T lc, T cc, T rc, T lp, T cp,
                                   T rp) {
  return (double)o[0 * n + so] * (double)lm + (double)o[1 * n + so] * (double)cm + (double)o[2 * n + so] * (double)rm +
         (double)o[3 * n + so] * (double)lc + (double)o[4 * n + so] * (double)cc + (double)o[5 * n + so] * (double)rc +
         (double)o[6 * n + so] * (double)lp + (double)o[7 * n + so] * (double)cp + (double)o[8 * n + so] * (double)rp;
}

template <typename T, int R, bool OBS, int NG, bool GEN>
__global__ __launch_bounds__(64) void pass2d_kernel(Pass2D<T> a) {
  constexpr int H = R + 1;
  constexpr int W = 64 - 2 * H;
  constexpr int NQ = LDQ_NQ_BASE + NG;
  const int lane = threadIdx.x;
  const int L = xcd_remap(blockIdx.x, gridDim.x);
  const int probe = L / a.ntiles, tile = L - probe * a.ntiles;
  const ProbeRef pref = probe_ref(a.tail, probe, a.ntiles);
  const Step step = pass_prologue<1>(a.tail, pref, tile, a.ntiles, a.mode);
  if (!step.run) return;
  const int colour = step.colour;
  // GEN: r_k = p_k = v_j generated from the colouring (INIT: alpha = 0, nothing stored)
  const bool store = !GEN || a.mode != MODE_INIT;
  const double alpha = (GEN && a.mode == MODE_INIT) ? 0.0 : step.alpha;
  const double beta = step.beta;

  const int nx = a.nx, ny = a.ny;
  const size_t n = (size_t)nx * ny;
  const size_t off = (size_t)probe * n;
  const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
  const int x0 = tx * W, y0 = ty * a.rows;
  const int yb = min(y0 + a.rows, ny);
  const int x = x0 - H + lane;
  const int xc = min(max(x, 0), nx - 1);           // clamped column: every load address is valid
  const bool xin = x >= 0 && x < nx;
  const bool xout = lane >= H && lane < 64 - H && x < nx;   // output column of this strip
  const int nrows = a.rows + 2 * H;                // multiple of 5
  const int ylo = y0 - H;                          // lattice row of step 0
  const int degx = (x > 0) + (x < nx - 1);
  const double c = a.kappa2 + 4.0;                 // M = (kappa2 + 4) I - (axis neighbours)

  // Modular colouring c(x, y) = (x + a y) mod C = (x mod C + a y mod C) mod C.
  // The row parts are uniform across the wave and advance by a mod C per row.
  const int C = a.colC;
  const int cx = (C > 0 && xin) ? x % C : -1 - 2 * C;   // never matches when outside
  const int astep = C > 0 ? a.cola % C : 0;
  auto row_part = [&](int y) -> int {
    if (C <= 0) return 0;
    const long t = ((long)a.cola * (long)y) % C;
    return (int)(t < 0 ? t + C : t);
  };
  auto advance = [&](int v) -> int {
    v += astep;
    return v >= C ? v - C : v;
  };
  // entry of the probe vector at (x, y) of this lane: 0 / 1 for a colour
  // class, -1 / +1 for random signs (0 outside the lattice)
  auto mine_at = [&](int y, int ay) -> double {
    if (a.rad) return (xin && y >= 0 && y < ny) ? rad_sign(a.seed, colour, (int64_t)y * nx + x) : 0.0;
    if (a.uvec) return (xin && y >= 0 && y < ny) ? a.uvec[(size_t)colour * n + (size_t)y * nx + x] : 0.0;
    if (C > 0) {
      int v = cx + ay;
      v -= (v >= C) ? C : 0;
      return v == colour ? 1.0 : 0.0;
    }
    return (xin && y >= 0 && y < ny && a.colours[(size_t)y * nx + xc] == colour) ? 1.0 : 0.0;
  };
  int ay_in = row_part(ylo);                       // row part of the arriving row
  int ay_g = row_part(ylo - 1);                    // ... of the gradient row y - 1
  int ay_d = row_part(ylo - R - 1);                // ... of the dot-product row y - R - 1

  const T *rin = a.r_in + off + xc;
  const T *pin = a.p_in + off + xc;
  T *rout = a.r_out + off + xc;
  T *pout = a.p_out + off + xc;

  // prefetch queue of the next five rows (r_k, p_{k-1})
  T qr[5], qp[5];
  auto fetch = [&](int slot, int i) {
    const int y = ylo + i;
    T r = T(0), p = T(0);
    if (!GEN && y >= 0 && y < ny) {
      const size_t o = (size_t)y * nx;
      r = rin[o];
      p = pin[o];
    }
    qr[slot] = r;
    qp[slot] = p;
  };
  if constexpr (!GEN) {
#pragma unroll
    for (int u = 0; u < 5; ++u) fetch(u, u);
  }

  // rings indexed by lattice row mod 5 (indices are compile-time after unrolling)
  double acc[5], acc2[5], obs_s[5], obs_r[5];
  double macc[NG > 0 ? NG : 1][5];
  T rq[5], pq[5], rnq[5], pl[5], pr[5], rl[5], rr[5];
  double k2q[5];
#pragma unroll
  for (int u = 0; u < 5; ++u) {
    acc[u] = acc2[u] = obs_s[u] = obs_r[u] = 0.0;
    rq[u] = pq[u] = rnq[u] = pl[u] = pr[u] = rl[u] = rr[u] = T(0);
    k2q[u] = 0.0;
#pragma unroll
    for (int g = 0; g < (NG > 0 ? NG : 1); ++g) macc[g][u] = 0.0;
  }
  double q[NQ];
#pragma unroll
  for (int i = 0; i < NQ; ++i) q[i] = 0.0;

  for (int i0 = 0; i0 < nrows; i0 += 5) {
#pragma unroll
    for (int u = 0; u < 5; ++u) {
      const int i = i0 + u;
      const int y = ylo + i;
      const bool yin = y >= 0 && y < ny;
      // ---- row y arrives: p_k = r_k + beta p_{k-1}, rounded to the storage precision
      T r_y, p_y;
      if constexpr (GEN) {
        r_y = yin ? (T)mine_at(y, ay_in) : T(0);
        p_y = r_y;
      } else {
        r_y = xin ? qr[u] : T(0);
        p_y = xin ? (T)((double)qr[u] + beta * (double)qp[u]) : T(0);
        fetch(u, i + 5);
      }
      ay_in = advance(ay_in);
      rq[u] = r_y;
      pq[u] = p_y;
      const double p = p_y;
      const T pL = from_left(p_y), pR = from_right(p_y);
      const double h1 = (double)pL + (double)pR;
      double k2 = a.kappa2;
      if constexpr (R == 1) {
        if (a.kappa2_field) k2 = yin ? (double)a.kappa2_field[(size_t)y * nx + xc] : 0.0;
      }
      k2q[u] = k2;
      if constexpr (OBS) {
        pl[u] = pL;
        pr[u] = pR;
      }
      if constexpr (R == 2) {
        // M @ M: row y adds p to rows y -+ 2, 2 h1 - 2c p to rows y -+ 1 and
        // (c^2 + deg) p - 2c h1 + h2 to row y
        const double h2 = (double)from_left(pL) + (double)from_right(pR);
        const double c0 = c * c + (double)(degx + (y > 0) + (y < ny - 1));
        const double t1 = 2.0 * h1 - 2.0 * c * p;
        acc[(u + 3) % 5] += p;                                      // row y - 2 complete
        acc[(u + 4) % 5] += t1;
        acc[u] += c0 * p - 2.0 * c * h1 + h2;
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
        if (yo >= 0 && yo < ny) {
          const int um = (u + 3) % 5, uc = (u + 4) % 5;
          v = obs_apply(a.obs, n, (size_t)yo * nx + xc, pl[um], pq[um], pr[um], pl[uc], pq[uc], pr[uc], pl[u], pq[u],
                        pr[u]);
        }
        obs_s[(u + 4) % 5] = a.tau * v;
      }
      // ---- gradient dots w_g . p_k over the probe's sites of row y - 1
      if constexpr (NG > 0) {
        const int yg = y - 1;
        const int ug = (u + 4) % 5;
        const double gw = (xout && yg >= y0 && yg < yb) ? mine_at(yg, ay_g) : 0.0;
#pragma unroll
        for (int g = 0; g < NG; ++g) {
          const GradTerm<T> &gt = a.grad[g];
          if (gt.kind == GK_SHIFTED) {
            const double kd = gt.field ? (yin ? (double)gt.field[(size_t)y * nx + xc] : 0.0) : gt.kappa2;
            macc[g][ug] -= p;                                       // row y - 1 complete
            q[LDQ_NQ_BASE + g] += gw * gt.scale * macc[g][ug];
            macc[g][u] += (kd + 4.0) * p - h1;
            macc[g][(u + 1) % 5] = -p;
          } else if (gt.kind == GK_DIAG) {
            if (gw != 0.0) q[LDQ_NQ_BASE + g] += gw * gt.scale * (double)gt.field[(size_t)yg * nx + xc] * (double)pq[ug];
          } else if constexpr (OBS) {
            // GK_OBS (the host allows it only when Q has an observation term)
            if (gw != 0.0) {
              const int um = (u + 3) % 5;
              q[LDQ_NQ_BASE + g] += gw * gt.scale * obs_apply(gt.obs, n, (size_t)yg * nx + xc, pl[um], pq[um], pr[um],
                                                              pl[ug], pq[ug], pr[ug], pl[u], pq[u], pr[u]);
            }
          }
        }
      }
      ay_g = advance(ay_g);
      // ---- row ys = y - R of s = Q p_k is complete: r_{k+1} = r_k - alpha s
      const int ys = y - R;
      const int us = (u + 5 - R) % 5;
      const bool sin = xin && ys >= 0 && ys < ny;
      double sv = a.scale * acc[us];
      if constexpr (OBS) sv += obs_s[us];
      const T rn = sin ? (T)((double)rq[us] - alpha * sv) : T(0);
      rnq[us] = rn;
      if (store && xout && ys >= y0 && ys < yb) {
        const size_t o = (size_t)ys * nx;
        rout[o] = rn;
        pout[o] = pq[us];
      }
      // ---- row ys of r_{k+1} enters the M r' ring: row ys - 1 of M r' is complete
      const double rv = rn;
      const T rL = from_left(rn), rR = from_right(rn);
      const double g1 = (double)rL + (double)rR;
      if constexpr (OBS) {
        rl[us] = rL;
        rr[us] = rR;
      }
      acc2[(us + 4) % 5] -= rv;
      acc2[us] += ((R == 1 ? k2q[us] : a.kappa2) + 4.0) * rv - g1;
      acc2[(us + 1) % 5] = -rv;
      if constexpr (OBS) {
        const int yo = ys - 1;
        double v = 0.0;
        if (yo >= 0 && yo < ny) {
          const int um = (us + 3) % 5, uc = (us + 4) % 5;
          v = obs_apply(a.obs, n, (size_t)yo * nx + xc, rl[um], rnq[um], rr[um], rl[uc], rnq[uc], rr[uc], rl[us],
                        rnq[us], rr[us]);
        }
        obs_r[(us + 4) % 5] = a.tau * v;
      }
      // ---- dot products on row yd = ys - 1: r'.Q r' = scale r'.M r' (R = 1)
      // or scale |M r'|^2 (R = 2), plus r'.tau A^T A r'
      const int yd = ys - 1;
      const int ud = (us + 4) % 5;
      {
        const bool dout = xout && yd >= y0 && yd < yb;
        const double r2 = dout ? (double)rnq[ud] : 0.0;
        const double mr = dout ? acc2[ud] : 0.0;
        double qv = a.scale * mr * (R == 2 ? mr : r2);
        if constexpr (OBS) qv += r2 * obs_r[ud];
        q[0] += r2 * r2;
        q[1] += qv;
        q[2] += dout ? mine_at(yd, ay_d) * r2 : 0.0;
      }
      ay_d = advance(ay_d);
    }
  }
  pass_epilogue_n<NQ>(pref, tile, a.ntiles, q);
}

// Specialised STEP pass for the common case: modular colouring, constant
// kappa2, derivative operators fixed at compile time (NG >= 1: g0 is a
// shifted Laplacian with a constant shift; NG = 2 with OBS: g1 is A^T A with
// the same planes as Q's observation term).  Every load in the row loop is
// unconditional (clamped addresses, values selected afterwards), so the
// compiler can keep the five-row prefetch in flight instead of waiting for all
// outstanding loads at every conditional.
// Geometry and coefficients of one probe's tile for fast_tile.
template <typename T>
struct FastTile {
  int nx, ny, tiles_x, rows;
  int colC, cola;
  double kappa2;       // Q's constant shift
  double kd;           // gradient 0: shift of the derivative Laplacian
  double gs0, gs1;     // gradient scales
  double tau;          // observation weight
  const T *obs;        // observation planes (9 x n)
  const T *r_in, *p_in;
  T *r_out, *p_out;    // the probe's vectors
  const uint64_t *rmask;   // random-sign probes: the probe's strip masks [ny][tiles_x]
};

template <typename T, int R, bool OBS, int NG, int TR, bool RAD, typename Prologue>
__device__ inline bool fast_tile(const FastTile<T> &a, int tile, Prologue prologue, double *q);

// In the FP32 fast pass, workgroups 0 .. owner_blocks(nprobes) - 1 advance
// the probes' states (one probe each, no tile) and the rest run the tiles, so
// the per-shift recurrences run beside the tiles instead of delaying tile 0
// (one microsecond off a 512 x 512 launch of 41 probes).  They come first so
// that they are dispatched first; a multiple of 8 keeps the tiles' XCD
// mapping.  The FP64 pass keeps the owner role in tile 0: its occupancy is
// register-bound and it measured slower with the extra workgroups.
template <typename T>
__host__ __device__ constexpr bool sep_owner() { return sizeof(T) == 4; }
template <typename T>
__host__ __device__ inline int owner_blocks(int nprobes) { return sep_owner<T>() ? (nprobes + 7) & ~7 : 0; }

// FP32 without observations: held to 80 VGPRs, so that 6 waves per SIMD fit
// the 41 x 144 tiles of a 512 x 512 launch at once (the owner branch, which
// runs once per probe, may spill a few bytes for it).  RAD: random-sign
// probes, whose entries come from a.rmask instead of the modular colouring.
template <typename T, int R, bool OBS, int NG, int TR, bool RAD>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 && !OBS && TR < LDQ_ROWS2D_TALL ? 6 : 1))) void pass2d_fast(Pass2D<T> a) {
  constexpr int NQ = LDQ_NQ_BASE + NG;
  const int nown = owner_blocks<T>(a.nprobes);
  if ((int)blockIdx.x < nown) {
    if ((int)blockIdx.x < a.nprobes)
      (void)pass_prologue<1>(a.tail, probe_ref(a.tail, blockIdx.x, a.ntiles), 0, a.ntiles, MODE_STEP, ROLE_OWNER);
    return;
  }
  const int L = xcd_remap(blockIdx.x - nown, gridDim.x - nown);
  const int probe = L / a.ntiles, tile = L - probe * a.ntiles;
  const ProbeRef pref = probe_ref(a.tail, probe, a.ntiles);
  const size_t off = (size_t)probe * a.nx * a.ny;
  FastTile<T> ft;
  ft.nx = a.nx;
  ft.ny = a.ny;
  ft.tiles_x = a.tiles_x;
  ft.rows = a.rows;
  ft.colC = a.colC;
  ft.cola = a.cola;
  ft.kappa2 = a.kappa2;
  ft.kd = NG > 0 ? a.grad[0].kappa2 : 0.0;
  ft.gs0 = NG > 0 ? a.grad[0].scale : 0.0;
  ft.gs1 = NG > 1 ? a.grad[1].scale : 0.0;
  ft.tau = a.tau;
  ft.obs = a.obs;
  ft.r_in = a.r_in + off;
  ft.p_in = a.p_in + off;
  ft.r_out = a.r_out + off;
  ft.p_out = a.p_out + off;
  ft.rmask = RAD ? a.rmask + (size_t)probe * a.ny * a.tiles_x : nullptr;
  double q[NQ];
  auto prologue = [&]() {
    return pass_prologue<1>(a.tail, pref, tile, a.ntiles, MODE_STEP, sep_owner<T>() ? ROLE_TILE : ROLE_TILE0);
  };
  if (!fast_tile<T, R, OBS, NG, TR, RAD>(ft, tile, prologue, q)) return;
  pass_epilogue_n<NQ>(pref, tile, a.ntiles, q);
}

// Rows of a standard wave tile for stencil radius R: LDQ_ROWS2D rounded up to
// a multiple of the five-row ring after the 2H = 2R + 2 halo rows.
template <int R>
constexpr int rows_full() {
  int r = LDQ_ROWS2D;
  while ((r + 2 * R + 2) % 5 != 0) ++r;
  return r;
}
// Rows of the tall tile of the FP32 fast passes (64 rounded up the same way):
// fewer halo rows re-read per row of output (6 per 64 instead of 6 per 34),
// which pays where the vectors stream from HBM.
template <int R>
constexpr int rows_tall() {
  int r = LDQ_ROWS2D_TALL;
  while ((r + 2 * R + 2) % 5 != 0) ++r;
  return r;
}
// Rows of r and p requested ahead of the march: one five-row ring, or two for
// the tall tile (its waves are half as many, so registers allow the deeper
// prefetch, which halves the dependent round trips of a wave's 70 rows).
#ifndef LDQ_PF_TALL
#define LDQ_PF_TALL 10
#endif
template <int R, int TR>
constexpr int prefetch_rows() {
  return TR == rows_tall<R>() ? LDQ_PF_TALL : 5;
}

// One tile of one probe: the march of the fused pass; q[] receives this
// wave's sums of the pass's dot products.  The first rows of r and p are
// requested before prologue() (the reduction of the previous launch's
// partials, which yields alpha, beta and the probe's colour) so that its
// memory round trips overlap; returns false when the probe is not active.
// RAD: the probe's entries are the random signs of a.rmask (every site is the
// probe's; the masks need a tile of at most 64 rows with its halo).
template <typename T, int R, bool OBS, int NG, int TR, bool RAD, typename Prologue>
__device__ inline bool fast_tile(const FastTile<T> &a, int tile, Prologue prologue, double *q) {
  constexpr int H = R + 1;
  constexpr int W = 64 - 2 * H;
  constexpr int NQ = LDQ_NQ_BASE + NG;
  const int lane = threadIdx.x & 63;

  const int nx = a.nx, ny = a.ny;
  const size_t n = (size_t)nx * ny;
  const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
  const int x0 = tx * W, y0 = ty * a.rows;
  const int yb = min(y0 + a.rows, ny);
  const int x = x0 - H + lane;
  const int xc = min(max(x, 0), nx - 1);
  const bool xin = x >= 0 && x < nx;
  const bool xout = lane >= H && lane < 64 - H && x < nx;
  const int nrows = a.rows + 2 * H;
  const int ylo = y0 - H;
  const double gs0 = a.gs0;
  const double gs1 = a.gs1;
  // A tile is interior when every column and row it loads lies inside the
  // lattice: no masking there.
  const bool interior = x0 - H >= 0 && x0 - H + 63 <= nx - 1 && ylo >= 0 && ylo + nrows - 1 <= ny - 1;

  // Colour test.  (x + a y) mod C == colour  <=>  x mod C == (colour - a y)
  // mod C; the right side is uniform across the wave and steps by -a mod C
  // per row (kept in a scalar register), so each row costs one compare.
  const int C = __builtin_amdgcn_readfirstlane(a.colC);
  const int cx = xin ? x % C : -1 - 2 * C;
  const int astep = __builtin_amdgcn_readfirstlane(a.cola % C);

  // buffer resources over this probe's vectors and the observation planes
  const unsigned vbytes = (unsigned)(n * sizeof(T));
  const __amdgpu_buffer_rsrc_t rs_rin = make_rsrc(a.r_in, vbytes);
  const __amdgpu_buffer_rsrc_t rs_pin = make_rsrc(a.p_in, vbytes);
  const __amdgpu_buffer_rsrc_t rs_rout = make_rsrc(a.r_out, vbytes);
  const __amdgpu_buffer_rsrc_t rs_pout = make_rsrc(a.p_out, vbytes);
  const __amdgpu_buffer_rsrc_t rs_obs = make_rsrc(OBS ? a.obs : a.r_in, OBS ? 9u * vbytes : vbytes);
  const unsigned lx = (unsigned)xc * (unsigned)sizeof(T);           // lane byte offset
  // store offset: lanes outside the strip's output columns address past the
  // end of the buffer, where the hardware range check drops the store
  const unsigned lst = xout ? lx : 0xFFFFFFF0u;
  const unsigned rowb = (unsigned)nx * (unsigned)sizeof(T);         // row stride in bytes

  // rows ylo .. ylo + PF - 1 (clamped into the lattice), requested now
  constexpr int PF = prefetch_rows<R, TR>();
  static_assert(PF == 5 || PF == 10, "the prefetch ring is one or two stencil rings");
  static_assert((TR + 2 * H) % PF == 0, "the march is whole prefetch rings");
  T qr0[PF], qp0[PF];
#pragma unroll
  for (int u = 0; u < PF; ++u) {
    const unsigned so = (unsigned)min(max(ylo + u, 0), ny - 1) * rowb;
    qr0[u] = buf_ld((T *)nullptr, rs_rin, lx, so);
    qp0[u] = buf_ld((T *)nullptr, rs_pin, lx, so);
  }
  // Random signs: lane i holds the strip's mask of row ylo - 1 + i (the
  // gradient row of step i): bit l is set when the probe's entry at column
  // x0 - H + l is -1.  Masks are indexed by probe, not colour, so they are
  // requested with the first rows, before the prologue.
  unsigned mlo = 0u, mhi = 0u;
  if constexpr (RAD) {
    static_assert(TR + 2 * H <= 64, "one mask per lane and row of the march");
    const int ym = ylo - 1 + lane;
    if (lane < TR + 2 * H && ym >= 0 && ym < ny) {
      const uint64_t m = a.rmask[(size_t)ym * a.tiles_x + tx];
      mlo = (unsigned)m;
      mhi = (unsigned)(m >> 32);
    }
  }
  const Step step = prologue();
  if (!step.run) return false;
  const int colour = __builtin_amdgcn_readfirstlane(step.colour);
  const double alpha = step.alpha, beta = step.beta;
  const T beta_t = (T)beta;

#pragma unroll
  for (int i = 0; i < NQ; ++i) q[i] = 0.0;

  // The operator is applied in the storage type T (FP32 in the mixed form,
  // FP64 in the plain form) as M v = kappa2 v + (4 v - neighbours): the
  // Laplacian's coefficients are exact in either type and only kappa2 is
  // rounded, so the rows of M and M @ M keep their exact sums.  The squared
  // operator runs two such stages, s = M (M p).  Per-lane sums run in T over
  // groups of five rows and are then added in FP64.
  const T k2_t = (T)a.kappa2, dk_t = (T)(a.kd - a.kappa2), tau_t = (T)a.tau, alpha_t = (T)alpha;

  auto march = [&](auto interior_tag) {
    constexpr bool IN = decltype(interior_tag)::value;
    constexpr int RF = TR;   // the tile's rows (a.rows == TR: checked by the launchers)
    constexpr int NFULL = RF + 2 * H;
    // (colour - a (y - 1)) mod C for the gradient row y - 1 of step 0
    int tg;
    {
      const int yg = ylo - 1;
      const int ay = (int)((((long)astep * (long)(((yg % C) + C) % C)) % C));
      tg = colour - ay;
      tg += tg < 0 ? C : 0;
      tg = __builtin_amdgcn_readfirstlane(tg);
    }
    // byte offset of the arriving row y (interior tiles: ylo >= 0).  tg and yo
    // pass through an empty asm statement once per step, so that the compiler
    // derives each step's scalars in that step: in the straight-line interior
    // code it would otherwise compute them all up front and run out of
    // scalar registers.
    unsigned yo = IN ? (unsigned)ylo * rowb : 0u;
    const unsigned rowbPF = (unsigned)PF * rowb, rowbR = (unsigned)R * rowb;
    T qr[PF], qp[PF];
    auto fetch = [&](int slot, int i) {
      const int yy = ylo + min(i, NFULL - 1);
      const int yc = IN ? yy : min(max(yy, 0), ny - 1);
      qr[slot] = buf_ld((T *)nullptr, rs_rin, lx, (unsigned)yc * rowb);
      qp[slot] = buf_ld((T *)nullptr, rs_pin, lx, (unsigned)yc * rowb);
    };
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      qr[u] = qr0[u];
      qp[u] = qp0[u];
    }
    // rings indexed by lattice row mod 5: t = M p and s = M t (or s = M p for
    // the 5-point operator), tr = M r'
    T tacc[5], acc[5], tracc[5], obs_s[5];
    // per-lane sums over the probe's sites (at most ceil(rows / C) terms):
    // rho' and the gradient dots; gamma' and delta' over the current group of
    // five rows
    T racc = T(0), gacc0 = T(0), gacc1 = T(0), g0 = T(0), g1 = T(0);
    T rq[5], pq[5], rnq[5], pl[5], pr[5], rl[5], rr[5];
    bool mg[5];   // the lane's site of gradient row y - 1 is the probe's (ring by step)
#pragma unroll
    for (int u = 0; u < 5; ++u) {
      tacc[u] = acc[u] = tracc[u] = obs_s[u] = T(0);
      rq[u] = pq[u] = rnq[u] = pl[u] = pr[u] = rl[u] = rr[u] = T(0);
      mg[u] = false;
    }
    // one 5-point stage: value v of row y arrives in slot u of ring m; row
    // y - 1 of M v is complete afterwards and is returned
    auto mstage = [&](T *m, int u, T v) -> T {
      const T h = from_left(v) + from_right(v);
      m[(u + 4) % 5] -= v;
      m[u] += fma_t(k2_t, v, fma_t(T(4), v, -h));
      const T done = m[(u + 4) % 5];
      m[(u + 1) % 5] = -v;
      return done;
    };
    // A^T A is symmetric: its coefficient from site s to s + d equals the one
    // from s + d to s, so planes 5..8 of a row are planes 3..0 of the next
    // site or row (equal bit for bit: both entries accumulate the same
    // products in the same order).  Only planes 0..4 are loaded, those of row
    // y + 1 at step y into slot (u + 1) mod 5: at step y the planes of rows
    // y - 1 and y serve p's row y - 1, those of rows yd and yd + 1 r' row yd.
    T opl[5][5];
#pragma unroll
    for (int u = 0; u < 5; ++u)
#pragma unroll
      for (int d = 0; d < 5; ++d) opl[u][d] = T(0);
    auto load_planes = [&](int slot, int yo) {
      const int yoc = min(max(yo, 0), ny - 1);
      const unsigned so = (unsigned)yoc * rowb;
#pragma unroll
      for (int d = 0; d < 5; ++d) opl[slot][d] = buf_ld((T *)nullptr, rs_obs, lx, so + (unsigned)d * vbytes);
    };
    // (A^T A v) of row yo from the planes of rows yo (slot sc) and yo + 1
    // (slot sn) and the v rows held in the (l, c, r) rings at slots um, uc, up
    // (lanes 0 and 63 read 0 for the shifted terms: halo columns whose sums
    // are not used)
    auto obs_row = [&](int sc, int sn, int yo, const T *lm, const T *cm, const T *rm, int um, int uc, int up) -> T {
      const T *o = opl[sc];
      const T *on = opl[sn];
      T v = o[0] * lm[um];
      v = fma_t(o[1], cm[um], v);
      v = fma_t(o[2], rm[um], v);
      v = fma_t(o[3], lm[uc], v);
      v = fma_t(o[4], cm[uc], v);
      v = fma_t(from_right(o[3]), rm[uc], v);     // plane 5 = plane 3 at x + 1
      v = fma_t(from_left(on[2]), lm[up], v);     // plane 6 = plane 2 at (x - 1, y + 1)
      v = fma_t(on[1], cm[up], v);                // plane 7 = plane 1 at (x, y + 1)
      v = fma_t(from_right(on[0]), rm[up], v);    // plane 8 = plane 0 at (x + 1, y + 1)
      return (IN || (yo >= 0 && yo < ny)) ? v : T(0);
    };
    if constexpr (OBS) load_planes(0, ylo);
    // Interior tiles run the row loop fully unrolled (tiles have the standard
    // height): every prefetched value is then consumed in straight-line code
    // and the compiler keeps the loads in flight (a loop back edge would force
    // it to wait for them), and every row test below is a compile-time
    // constant.  Boundary tiles keep the loop and run-time row tests:
    // unrolled, their masking exhausts the registers.
    // five row steps starting at step i0 (ring slots are compile-time; the
    // rows arriving are in prefetch slots sb .. sb + 4)
    auto group = [&](int i0, int sb) {
#pragma unroll
      for (int u = 0; u < 5; ++u) {
        const int i = i0 + u;
        const int y = ylo + i;
        // rows of this step: gradient yg = y - 1, r' and stores ys = y - R,
        // dot products yd = y - R - 1; each is one of the tile's own rows
        // [y0, yb) for a contiguous range of steps
        const bool g_row = IN ? (i >= H + 1 && i < H + 1 + RF) : (y - 1 >= y0 && y - 1 < yb);
        const bool s_row = IN ? (i >= H + R && i < H + R + RF) : (y - R >= y0 && y - R < yb);
        const bool d_row = IN ? (i >= H + R + 1 && i < H + R + 1 + RF) : (y - R - 1 >= y0 && y - R - 1 < yb);
        // ---- row y arrives: p_k = r_k + beta p_{k-1}
        T r_y = qr[sb + u];
        T p_y = fma_t(beta_t, qp[sb + u], qr[sb + u]);
        if constexpr (!IN) {
          const bool in = xin && y >= 0 && y < ny;
          r_y = in ? r_y : T(0);
          p_y = in ? p_y : T(0);
        }
        if constexpr (IN) {
          __asm__ volatile("" : "+s"(yo), "+s"(tg));
          // the last PF steps prefetch nothing (no rows follow)
          if (i + PF < NFULL) {
            qr[sb + u] = buf_ld((T *)nullptr, rs_rin, lx, yo + rowbPF);
            qp[sb + u] = buf_ld((T *)nullptr, rs_pin, lx, yo + rowbPF);
          }
        } else {
          fetch(sb + u, i + PF);
        }
        rq[u] = r_y;
        pq[u] = p_y;
        if constexpr (OBS) {
          pl[u] = from_left(p_y);
          pr[u] = from_right(p_y);
        }
        // colour masks: row y - 1 now, row yd = y - R - 1 from R steps ago
        // (RAD: the sign masks, true where the probe's entry is -1)
        bool mine_g = cx == tg;
        if constexpr (RAD) {
          const uint64_t m = ((uint64_t)(unsigned)__builtin_amdgcn_readlane((int)mhi, i) << 32) |
                             (unsigned)__builtin_amdgcn_readlane((int)mlo, i);
          mine_g = __builtin_amdgcn_inverse_ballot_w64(m);
        }
        const bool mine_d = mg[(u + 5 - R) % 5];
        mg[u] = mine_g;
        tg -= astep;
        tg += tg < 0 ? C : 0;
        tg = __builtin_amdgcn_readfirstlane(tg);
        // t = M p: row y - 1 complete; for the squared operator it enters the
        // second stage, which completes row y - 2 of s = M t
        T tv = mstage(tacc, u, p_y);
        if constexpr (!IN) tv = (xin && y - 1 >= 0 && y - 1 < ny) ? tv : T(0);
        T sv = tv;                                                    // the fast path has scale 1
        if constexpr (R == 2) sv = mstage(acc, (u + 4) % 5, tv);
        T ov = T(0);                                                  // (A^T A p) of row y - 1
        if constexpr (OBS) {
          load_planes((u + 1) % 5, y + 1);
          ov = obs_row((u + 4) % 5, u, y - 1, pl, pq, pr, (u + 3) % 5, (u + 4) % 5, u);
          obs_s[(u + 4) % 5] = tau_t * ov;
        }
        if constexpr (NG > 0) {
          // (kd I + L) p = t + (kd - kappa2) p on row y - 1 over the probe's
          // sites (scaled at the end)
          if (g_row) {
            const T gv = fma_t(dk_t, pq[(u + 4) % 5], tv);
            if constexpr (RAD)
              gacc0 += mine_g ? -gv : gv;
            else
              gacc0 += mine_g ? gv : T(0);
            if constexpr (NG > 1 && OBS) gacc1 += mine_g ? ov : T(0);
          }
        }
        // ---- row ys = y - R of s = Q p_k is complete: r_{k+1} = r_k - alpha s
        const int ys = y - R;
        const int us = (u + 5 - R) % 5;
        if constexpr (OBS) sv += obs_s[us];
        T rn = fma_t(-alpha_t, sv, rq[us]);
        if constexpr (!IN) rn = (xin && ys >= 0 && ys < ny) ? rn : T(0);
        rnq[us] = rn;
        if (s_row) {
          const unsigned so = IN ? yo - rowbR : (unsigned)ys * rowb;
          buf_st(rn, rs_rout, lst, so);
          buf_st(pq[us], rs_pout, lst, so);
        }
        // ---- row ys of r_{k+1} enters the M r' stage: row yd = ys - 1 of
        // M r' is complete
        if constexpr (OBS) {
          rl[us] = from_left(rn);
          rr[us] = from_right(rn);
        }
        const T trv = mstage(tracc, us, rn);
        const int ud = (us + 4) % 5;
        // ---- dot products on row yd: r'.Q r' = r'.M r' (R = 1) or
        // |M r'|^2 (R = 2), plus r'.tau A^T A r'
        if (d_row) {
          const T rd = rnq[ud];
          T qv = R == 2 ? trv * trv : rd * trv;
          if constexpr (OBS)
            qv = fma_t(rd, tau_t * obs_row((u + 4 - R) % 5, (u + 5 - R) % 5, ys - 1, rl, rnq, rr, (us + 3) % 5, ud, us),
                       qv);
          g0 = fma_t(rd, rd, g0);
          g1 += qv;
          if constexpr (RAD)
            racc += mine_d ? -rd : rd;
          else
            racc += mine_d ? rd : T(0);
        }
        // keep the scheduler from interleaving row steps (it would stretch
        // live ranges across the straight-line code)
        if constexpr (IN) {
          yo += rowb;
          // the step's sums are complete here (the compiler would otherwise
          // sink the masked additions to the end, holding every step's
          // values and colour masks)
          __asm__ volatile("" : "+v"(racc), "+v"(gacc0), "+v"(gacc1), "+v"(g0), "+v"(g1));
          __builtin_amdgcn_sched_barrier(0);
        }
      }
      q[0] += (double)g0;
      q[1] += (double)g1;
      g0 = g1 = T(0);
    };
    if constexpr (IN) {
#pragma unroll
      for (int i0 = 0; i0 < NFULL; i0 += 5) group(i0, i0 % PF);
    } else {
#pragma nounroll
      for (int i0 = 0; i0 < nrows; i0 += PF) {
        group(i0, 0);
        if constexpr (PF == 10) group(i0 + 5, 5);
      }
    }
    q[2] = (double)racc;
    if constexpr (NG > 0) q[LDQ_NQ_BASE] = gs0 * (double)gacc0;
    if constexpr (NG > 1) q[LDQ_NQ_BASE + 1] = gs1 * (double)gacc1;
    return true;
  };
  if (interior)
    march(std::true_type{});
  else
    march(std::false_type{});
  // lanes outside the strip's output columns computed halo values only
#pragma unroll
  for (int i = 0; i < NQ; ++i) q[i] = xout ? q[i] : 0.0;
  return true;
}

// Batched STEP pass: one wave per work-list entry (field, probe, tile).
template <typename T, int R, int NG, int TR>
__global__ __launch_bounds__(64) void batch2d_fast(Batch2D<T> b) {
  constexpr int NQ = LDQ_NQ_BASE + NG;
  // the grid was sized for a work list at least this long (a replayed graph
  // keeps its grid while the list shrinks); workgroups beyond it leave, the
  // rest are spread over the XCDs as for a grid of exactly `cnt`
  const int cnt = *b.count;
  if ((int)blockIdx.x >= cnt) return;
  const WorkItem wk = b.work[xcd_remap(blockIdx.x, cnt)];
  const FieldDesc fd = b.fields[wk.field];
  const size_t po = (size_t)fd.part_off + (size_t)wk.probe * NQ * fd.ntiles;
  const ProbeRef pref{fd.item_base + wk.probe, b.tail.part_in + po, b.tail.part_out + po,
                      b.sigma + (size_t)wk.field * LDQ_MAXN};
  const size_t off = (size_t)fd.vec_off + (size_t)wk.probe * fd.nx * fd.ny;
  FastTile<T> ft;
  ft.nx = fd.nx;
  ft.ny = fd.ny;
  ft.tiles_x = fd.tiles_x;
  ft.rows = b.rows;
  ft.colC = b.colC;
  ft.cola = b.cola;
  ft.kappa2 = fd.kappa2;
  ft.kd = fd.kd;
  ft.gs0 = b.gscale;
  ft.gs1 = 0.0;
  ft.tau = 0.0;
  ft.obs = nullptr;
  ft.r_in = b.r_in + off;
  ft.p_in = b.p_in + off;
  ft.r_out = b.r_out + off;
  ft.p_out = b.p_out + off;
  double q[NQ];
  auto prologue = [&]() { return pass_prologue<1>(b.tail, pref, wk.tile, fd.ntiles, MODE_STEP); };
  ft.rmask = nullptr;
  if (!fast_tile<T, R, false, NG, TR, false>(ft, wk.tile, prologue, q)) return;
  pass_epilogue_n<NQ>(pref, wk.tile, fd.ntiles, q);
}

template <typename T, int R, int TR>
static void launch_batch_ng(const Batch2D<T> &b, int ngrad, int grid, hipStream_t stream) {
  if (ngrad == 0) hipLaunchKernelGGL((batch2d_fast<T, R, 0, TR>), dim3(grid), dim3(64), 0, stream, b);
  else hipLaunchKernelGGL((batch2d_fast<T, R, 1, TR>), dim3(grid), dim3(64), 0, stream, b);
}

// b.rows is the standard tile height or (FP32) the tall one.
template <typename T>
hipError_t launch_batch2d(const Batch2D<T> &b, int nwork, bool squared, int ngrad, hipStream_t stream) {
  if (nwork <= 0) return hipSuccess;
  if constexpr (sizeof(T) == 4) {
    if (squared && b.rows == rows_tall<2>()) {
      launch_batch_ng<T, 2, rows_tall<2>()>(b, ngrad, nwork, stream);
      return hipGetLastError();
    }
    if (!squared && b.rows == rows_tall<1>()) {
      launch_batch_ng<T, 1, rows_tall<1>()>(b, ngrad, nwork, stream);
      return hipGetLastError();
    }
  }
  if (squared) launch_batch_ng<T, 2, rows_full<2>()>(b, ngrad, nwork, stream);
  else launch_batch_ng<T, 1, rows_full<1>()>(b, ngrad, nwork, stream);
  return hipGetLastError();
}
template hipError_t launch_batch2d<float>(const Batch2D<float> &, int, bool, int, hipStream_t);
template hipError_t launch_batch2d<double>(const Batch2D<double> &, int, bool, int, hipStream_t);

// Work list of the probes still iterating: each active item appends its
// tiles (the order of items in the list varies from run to run; every tile
// writes fixed slots, so results do not).  An item that has stopped gets its
// final state copied into the other state buffer, since no later launch
// carries it forward.
__global__ void batch_compact_kernel(const FieldDesc *fields, const int32_t *item_field, int nitems,
                                     const ProbeState *st_cur, ProbeState *st_other, WorkItem *work, int *count) {
  const int item = blockIdx.x * blockDim.x + threadIdx.x;
  if (item >= nitems) return;
  const ProbeState ps = st_cur[item];
  if (!ps.active) {
    st_other[item] = ps;
    return;
  }
  const int f = item_field[item];
  const FieldDesc fd = fields[f];
  const int base = atomicAdd(count, fd.ntiles);
  for (int t = 0; t < fd.ntiles; ++t) work[base + t] = WorkItem{f, item - fd.item_base, t, 0};
}

hipError_t launch_batch_compact(const FieldDesc *fields, const int32_t *item_field, int nitems,
                                const ProbeState *st_cur, ProbeState *st_other, WorkItem *work, int *count,
                                hipStream_t stream) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(batch_compact_kernel, dim3((nitems + 255) / 256), dim3(256), 0, stream, fields, item_field,
                     nitems, st_cur, st_other, work, count);
  return hipGetLastError();
}

template <typename T, int R, bool OBS, bool GEN>
static void launch_ng(const Pass2D<T> &a, int nblocks, hipStream_t stream) {
  switch (a.tail.ngrad) {
    case 0: hipLaunchKernelGGL((pass2d_kernel<T, R, OBS, 0, GEN>), dim3(nblocks), dim3(64), 0, stream, a); break;
    case 1: hipLaunchKernelGGL((pass2d_kernel<T, R, OBS, 1, GEN>), dim3(nblocks), dim3(64), 0, stream, a); break;
    default: hipLaunchKernelGGL((pass2d_kernel<T, R, OBS, 2, GEN>), dim3(nblocks), dim3(64), 0, stream, a); break;
  }
}

template <typename T, bool GEN>
static void launch_gen(const Pass2D<T> &a, bool squared, bool obs, int nblocks, hipStream_t stream) {
  if (squared && obs)
    launch_ng<T, 2, true, GEN>(a, nblocks, stream);
  else if (squared)
    launch_ng<T, 2, false, GEN>(a, nblocks, stream);
  else
    launch_ng<T, 1, false, GEN>(a, nblocks, stream);
}

// ngrad <= 2 (checked by the host driver for 2-D lattices); a.rows + 2H must
// be a multiple of 5 (pass2d_rows).
template <typename T, int R, bool OBS, int TR>
static void launch_fast_ng(const Pass2D<T> &a, int ng, hipStream_t stream) {
  const dim3 g(a.ntiles * a.nprobes + owner_blocks<T>(a.nprobes));
  // random signs: without observations, standard tiles (launch_pass2d)
  if constexpr (!OBS && TR == rows_full<R>()) {
    if (a.rmask) {
      if (ng == 0) hipLaunchKernelGGL((pass2d_fast<T, R, false, 0, TR, true>), g, dim3(64), 0, stream, a);
      else hipLaunchKernelGGL((pass2d_fast<T, R, false, 1, TR, true>), g, dim3(64), 0, stream, a);
      return;
    }
  }
  if (ng == 0) hipLaunchKernelGGL((pass2d_fast<T, R, OBS, 0, TR, false>), g, dim3(64), 0, stream, a);
  else if (ng == 1 || !OBS) hipLaunchKernelGGL((pass2d_fast<T, R, OBS, 1, TR, false>), g, dim3(64), 0, stream, a);
  else hipLaunchKernelGGL((pass2d_fast<T, R, OBS, OBS ? 2 : 1, TR, false>), g, dim3(64), 0, stream, a);
}

template <typename T, int TR2, int TR1>
static void launch_fast(const Pass2D<T> &a, bool squared, bool obs, hipStream_t stream) {
  const int ng = a.tail.ngrad;
  if (squared && obs) launch_fast_ng<T, 2, true, TR2>(a, ng, stream);
  else if (squared) launch_fast_ng<T, 2, false, TR2>(a, ng, stream);
  else launch_fast_ng<T, 1, false, TR1>(a, ng, stream);
}

// ngrad <= 2 (checked by the host driver for 2-D lattices); a.rows + 2H must
// be a multiple of 5 (pass2d_rows).  The fast pass runs tiles of the standard
// height, and in FP32 also of the tall height; with random signs (a.rmask),
// standard tiles without observations only.
template <typename T>
hipError_t launch_pass2d(const Pass2D<T> &a, bool squared, bool obs, bool fast, hipStream_t stream) {
  const int nblocks = a.ntiles * a.nprobes;
  const bool std_rows = a.rows == (squared ? rows_full<2>() : rows_full<1>());
  const bool tall_rows =
      sizeof(T) == 4 && !a.rmask && a.rows == (squared ? rows_tall<2>() : rows_tall<1>());
  if (a.rmask && obs) fast = false;
  if (a.mode == MODE_STEP && fast && std_rows) {
    launch_fast<T, rows_full<2>(), rows_full<1>()>(a, squared, obs, stream);
  } else if (a.mode == MODE_STEP && fast && tall_rows) {
    if constexpr (sizeof(T) == 4) launch_fast<T, rows_tall<2>(), rows_tall<1>()>(a, squared, obs, stream);
  } else if (a.mode == MODE_STEP) {
    launch_gen<T, false>(a, squared, obs, nblocks, stream);
  } else {
    launch_gen<T, true>(a, squared, obs, nblocks, stream);
  }
  return hipGetLastError();
}

template hipError_t launch_pass2d<float>(const Pass2D<float> &, bool, bool, bool, hipStream_t);
template hipError_t launch_pass2d<double>(const Pass2D<double> &, bool, bool, bool, hipStream_t);

// Sign masks of random-sign probes for the specialised pass: word
// (j, y, tx) of out has bit l set when entry (x, y) of probe first + j is -1,
// x = tx W - H + l the column of lane l in strip tx (0 outside the lattice).
__global__ void rad_mask_kernel(uint64_t *out, uint64_t seed, int first, int nprobes, int nx, int ny, int tiles_x,
                                int W, int H) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)nprobes * ny * tiles_x) return;
  const int tx = (int)(idx % tiles_x);
  const int64_t jy = idx / tiles_x;
  const int y = (int)(jy % ny), j = (int)(jy / ny);
  uint64_t m = 0;
  for (int l = 0; l < 64; ++l) {
    const int x = tx * W - H + l;
    if (x >= 0 && x < nx && rad_sign(seed, first + j, (int64_t)y * nx + x) < 0.0) m |= 1ull << l;
  }
  out[idx] = m;
}

hipError_t launch_rad_masks(uint64_t *out, uint64_t seed, int first, int nprobes, int nx, int ny, bool squared,
                            hipStream_t stream) {
  const int H = squared ? 3 : 2, W = 64 - 2 * H;
  const int tiles_x = (nx + W - 1) / W;
  const int64_t words = (int64_t)nprobes * ny * tiles_x;
  if (words <= 0) return hipSuccess;
  hipLaunchKernelGGL(rad_mask_kernel, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, stream, out, seed, first,
                     nprobes, nx, ny, tiles_x, W, H);
  return hipGetLastError();
}

// Rows per wave tile near `want` with rows + 2H a multiple of 5 (halo H = R + 1).
int pass2d_rows(bool squared, int want) {
  const int H = squared ? 3 : 2;
  int rows = want < 1 ? 1 : want;
  while ((rows + 2 * H) % 5 != 0) ++rows;
  return rows;
}

// Wave tiles: 64 - 2H columns by `rows` rows.
void pass2d_tiles(int nx, int ny, bool squared, int rows, int *tiles_x, int *ntiles) {
  const int W = squared ? 58 : 60;
  *tiles_x = (nx + W - 1) / W;
  *ntiles = *tiles_x * ((ny + rows - 1) / rows);
}

}  // namespace ldq
