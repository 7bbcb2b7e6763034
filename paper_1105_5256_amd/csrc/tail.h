// Device code shared by the pass kernels: deterministic workgroup reduction,
// last-workgroup detection and the per-probe scalar tail (base CG scalars and
// the multi-shift CG-M recurrences, Sec. 2.1 last paragraph).
#pragma once

#include "ldq_internal.h"

namespace ldq {

#define LDQ_NQ_MAX (LDQ_NQ_BASE + LDQ_MAXP)

__device__ inline double wave_sum(double v) {
  // fixed butterfly order: every lane ends with the same, deterministic sum
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum q[0..nq) over the workgroup; the result is valid in red_out[] after the call
// (all threads).  Order of additions is fixed, so the result is reproducible.
__device__ inline void block_sum(double *q, int nq, double (*red)[LDQ_NQ_MAX], double *red_out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < LDQ_NQ_MAX; ++i) {
    if (i < nq) {
      double s = wave_sum(q[i]);
      if (lane == 0) red[wave][i] = s;
    }
  }
  __syncthreads();
  if (threadIdx.x < nq) {
    int i = threadIdx.x;
    double s = red[0][i];
    for (int w = 1; w < LDQ_BLOCK / 64; ++w) s += red[w][i];
    red_out[i] = s;
  }
  __syncthreads();
}

// Multi-shift and base-CG update of one probe after a pass.  Runs on wave 0 of
// the workgroup that finished the probe's pass last; lane l owns shift l.
//   MODE_INIT: dots of r_0 = v (gamma_0, delta_0 = v^T Q v, rho_0 = v^T v).
//   otherwise: dots of r_{k+1} (gamma', delta', rho') and omega_i = w_i^T p_k of
//              the pass that used alpha_k, beta_{k-1}.
__device__ inline void probe_tail(const TailArgs &ta, int probe, int mode, const double *tot) {
  const int lane = threadIdx.x & 63;
  ProbeState ps = ta.st[probe];
  const int N = ta.nshifts;
  ShiftState *shp = ta.sh + (size_t)probe * N;
  bool done = false;
  int status = 0;
  if (mode == MODE_INIT) {
    const double g0 = tot[0], d0 = tot[1], rho0 = tot[2];
    ps.vnorm2 = g0;
    ps.gamma = g0;
    ps.alpha_prev = 1.0;
    ps.beta_prev = 0.0;
    ps.iter = 0;
    for (int i = 0; i < LDQ_MAXP; ++i) ps.grad[i] = 0.0;
    if (g0 == 0.0) {
      done = true;                                   // empty colour class: contributes nothing
    } else if (!(d0 > 0.0) || !isfinite(d0)) {
      done = true;
      status = 2;
    } else {
      ps.alpha = g0 / d0;                           // alpha_0 = gamma_0 / (p_0^T Q p_0), p_0 = v
    }
    if (lane < N) {
      ShiftState s;
      s.zeta = cmk(1.0, 0.0);
      s.zeta_prev = cmk(1.0, 0.0);
      s.phi = cmk(rho0, 0.0);                        // phi_0 = v^T p^sigma_0 = v^T v
      s.psi = cmk(0.0, 0.0);
      s.frozen = done ? 1 : 0;
      s.pad = 0;
      shp[lane] = s;
    }
  } else {
    const double gn = tot[0], dn = tot[1], rhon = tot[2];
    const double ak = ps.alpha, akm1 = ps.alpha_prev, bkm1 = ps.beta_prev;
#pragma unroll
    for (int i = 0; i < LDQ_MAXP; ++i)
      if (i < ta.ngrad) ps.grad[i] += ak * tot[LDQ_NQ_BASE + i];   // x_{k+1} = x_k + alpha_k p_k
    const double bk = gn / ps.gamma;                 // beta_k
    bool frozen = true;
    if (lane < N) {
      ShiftState s = shp[lane];
      if (!s.frozen) {
        const cplx sig = ta.sigma[lane];
        // zeta_{k+1} = zeta_k zeta_{k-1} alpha_{k-1} /
        //   (alpha_k beta_{k-1} (zeta_{k-1} - zeta_k) + zeta_{k-1} alpha_{k-1} (1 - sigma alpha_k))
        cplx one_m = cmk(1.0 - sig.re * ak, -sig.im * ak);
        cplx den = cadd(cscale(csub(s.zeta_prev, s.zeta), ak * bkm1),
                        cmul(cscale(s.zeta_prev, akm1), one_m));
        cplx znext = cdiv(cscale(cmul(s.zeta, s.zeta_prev), akm1), den);
        cplx ratio = cdiv(znext, s.zeta);            // zeta_{k+1} / zeta_k
        s.psi = cadd(s.psi, cmul(cscale(ratio, ak), s.phi));          // psi += alpha^sigma_k phi
        s.phi = cadd(cscale(znext, rhon), cmul(cscale(cmul(ratio, ratio), bk), s.phi));
        s.zeta_prev = s.zeta;
        s.zeta = znext;
        const bool bad = !(isfinite(s.psi.re) && isfinite(s.psi.im));
        if (bad) status = 2;
        if (cabs2(znext) * gn <= ta.tol2 * ps.vnorm2 || bad) s.frozen = 1;
        shp[lane] = s;
      }
      frozen = s.frozen != 0;
    }
    const bool all_frozen = __all(frozen);
    const bool any_bad = __any(status != 0);
    ps.iter += 1;
    const bool base_ok = (ta.ngrad == 0) || (gn <= ta.grad_tol2 * ps.vnorm2);
    if (any_bad) {
      done = true;
      status = 2;
    } else if (gn == 0.0 || (all_frozen && base_ok)) {
      done = true;
    } else {
      const double pap = dn - bk * gn / ak;          // p_{k+1}^T Q p_{k+1}
      if (!(pap > 0.0) || !isfinite(pap)) {
        done = true;
        status = 2;
      } else {
        ps.alpha_prev = ak;
        ps.alpha = gn / pap;                         // alpha_{k+1}
        ps.beta_prev = bk;
      }
      if (!done && ps.iter >= ta.max_iter) {
        done = true;
        status = 3;
      }
    }
    ps.gamma = gn;
  }
  if (lane == 0) {
    if (done) {
      ps.active = 0;
      ps.status = status;
      atomicSub(ta.active_count, 1);
    }
    ta.st[probe] = ps;
  }
}

// Write this workgroup's partial sums, and if it is the last workgroup of the
// probe for this pass, reduce all partials in a fixed order and run the tail.
__device__ inline void finish_pass(const TailArgs &ta, int probe, int tile, int ntiles, int nq, int mode,
                                   double *q) {
  __shared__ double red[LDQ_BLOCK / 64][LDQ_NQ_MAX];
  __shared__ double tot[LDQ_NQ_MAX];
  __shared__ int is_last;
  block_sum(q, nq, red, tot);
  if (threadIdx.x == 0) {
    double *dst = ta.partials + ((size_t)probe * ntiles + tile) * nq;
    for (int i = 0; i < nq; ++i) dst[i] = tot[i];
    __threadfence();
    unsigned old = atomicAdd(ta.counters + probe, 1u);
    is_last = (old == (unsigned)(ntiles - 1));
  }
  __syncthreads();
  if (!is_last) return;
  __threadfence();
  double acc[LDQ_NQ_MAX];
#pragma unroll
  for (int i = 0; i < LDQ_NQ_MAX; ++i) acc[i] = 0.0;
  const double *src = ta.partials + (size_t)probe * ntiles * nq;
  for (int t = threadIdx.x; t < ntiles; t += LDQ_BLOCK) {
#pragma unroll
    for (int i = 0; i < LDQ_NQ_MAX; ++i)
      if (i < nq) acc[i] += src[(size_t)t * nq + i];
  }
  block_sum(acc, nq, red, tot);
  if (threadIdx.x == 0) ta.counters[probe] = 0u;
  if (threadIdx.x < 64) probe_tail(ta, probe, mode, tot);
}

// Logical (probe, tile) of a workgroup.  Consecutive workgroup ids are spread
// round-robin over the 8 XCDs; this remap gives each XCD a contiguous range of
// tiles of the same probe, so halo rows shared by neighbouring tiles are
// found in that XCD's L2.
__device__ inline int xcd_remap(int bid, int nblocks) {
  const int nx = 8;
  const int base = nblocks / nx, rem = nblocks % nx;
  const int xcd = bid % nx, slot = bid / nx;
  const int start = xcd < rem ? xcd * (base + 1) : rem * (base + 1) + (xcd - rem) * base;
  return start + slot;
}

}  // namespace ldq
