// Device code shared by the pass kernels: deterministic workgroup reductions,
// the per-probe scalar tail (base CG scalars and the multi-shift CG-M
// recurrences, Sec. 2.1 last paragraph) and the dot-product partials.
//
// Cross-workgroup reduction without fences: launch g writes one partial sum
// per (probe, quantity, tile); at the start of launch g + 1 every workgroup of
// a probe reduces those partials itself, in one fixed order, and so derives
// the same alpha_{k+1}, beta_k bit for bit.  Tile 0 of each probe additionally
// advances the per-shift recurrences and the gradient sums and writes the new
// probe state (state and partials are double-buffered across launches).
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

// Sum q[0..nq) over the workgroup of NW waves; every thread receives the
// totals in out[].  The order of additions is fixed.
template <int NW>
__device__ inline void block_sum(const double *q, int nq, double *out) {
  if constexpr (NW == 1) {
#pragma unroll
    for (int i = 0; i < LDQ_NQ_MAX; ++i) out[i] = (i < nq) ? wave_sum(q[i]) : 0.0;
  } else {
    __shared__ double red[NW][LDQ_NQ_MAX];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < LDQ_NQ_MAX; ++i) {
      if (i < nq) {
        double v = wave_sum(q[i]);
        if (lane == 0) red[wave][i] = v;
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < LDQ_NQ_MAX; ++i) {
      double v = 0.0;
      if (i < nq) {
        v = red[0][i];
        for (int w = 1; w < NW; ++w) v += red[w][i];
      }
      out[i] = v;
    }
    __syncthreads();
  }
}

// Where one probe's data lives: its index into the probe states, shift states
// and Lanczos history, its partial sums ([quantity][tile]) in the input and
// output partial buffers, and the shifts of its operator.
struct ProbeRef {
  int st;
  const double *pin;
  double *pout;
  const cplx *sigma;
};

// The layout of a single-operator launch: probe j's partials at j * nq * ntiles.
__device__ inline ProbeRef probe_ref(const TailArgs &ta, int probe, int ntiles) {
  const size_t o = (size_t)probe * (LDQ_NQ_BASE + ta.ngrad) * ntiles;
  return ProbeRef{probe, ta.part_in + o, ta.part_out + o, ta.sigma};
}

struct Step {
  bool run;       // this workgroup performs the pass
  int colour;     // colour class of the probe
  double alpha;   // alpha_k of the pass
  double beta;    // beta_{k-1} of the pass (p_k = r_k + beta p_{k-1})
};

// Per-shift update for the dots of r_{k+1} (wave 0 of tile 0; lane l owns shift l).
//   zeta_{k+1} = zeta_k zeta_{k-1} alpha_{k-1} /
//                (alpha_k beta_{k-1} (zeta_{k-1} - zeta_k) + zeta_{k-1} alpha_{k-1} (1 - sigma alpha_k))
//   psi += alpha_k (zeta_{k+1} / zeta_k) phi
//   phi  = zeta_{k+1} rho' + (zeta_{k+1} / zeta_k)^2 beta_k phi
// psi accumulates v^T x^sigma and phi tracks v^T p^sigma (scalar-only CG-M).
__device__ inline bool shifts_update(const TailArgs &ta, const ProbeRef &pr, double ak, double akm1, double bkm1,
                                     double bk, double gn, double rhon, double vnorm2, bool *bad_out) {
  const int lane = threadIdx.x & 63;
  bool frozen = true, bad = false;
  if (lane < ta.nshifts) {
    ShiftState *sp = ta.sh + (size_t)pr.st * ta.nshifts + lane;
    ShiftState s = *sp;
    if (!s.frozen) {
      const cplx sig = pr.sigma[lane];
      const cplx one_m = cmk(1.0 - sig.re * ak, -sig.im * ak);
      const cplx den = cadd(cscale(csub(s.zeta_prev, s.zeta), ak * bkm1), cmul(cscale(s.zeta_prev, akm1), one_m));
      const cplx znext = cdiv(cscale(cmul(s.zeta, s.zeta_prev), akm1), den);
      const cplx ratio = cdiv(znext, s.zeta);
      s.psi = cadd(s.psi, cmul(cscale(ratio, ak), s.phi));
      s.phi = cadd(cscale(znext, rhon), cmul(cscale(cmul(ratio, ratio), bk), s.phi));
      s.zeta_prev = s.zeta;
      s.zeta = znext;
      bad = !(isfinite(s.psi.re) && isfinite(s.psi.im) && isfinite(s.phi.re) && isfinite(s.phi.im));
      if (bad || cabs2(znext) * gn <= ta.tol2 * vnorm2) s.frozen = 1;
      *sp = s;
    }
    frozen = s.frozen != 0;
  }
  *bad_out = __any(bad);
  return __all(frozen);
}

// Who advances the probe's state in a pass: the workgroup of tile 0
// (ROLE_TILE0), or a separate workgroup that runs no tile (ROLE_OWNER, paired
// with ROLE_TILE for every tile workgroup, so that the per-shift recurrences
// run beside the tiles instead of delaying tile 0).
enum TailRole { ROLE_TILE0 = 0, ROLE_TILE = 1, ROLE_OWNER = 2 };

// Whether this workgroup advances the probe's state, and how many of the
// partial quantities it therefore reduces (the others need gamma', delta').
__device__ inline bool tail_owner(int role, int tile) { return role == ROLE_OWNER || (role == ROLE_TILE0 && tile == 0); }
__device__ inline int tail_nred(const TailArgs &ta, bool owner) { return owner ? LDQ_NQ_BASE + ta.ngrad : 2; }

// The memory reads of a prologue: this thread's share of the previous
// launch's partials and the probe's state.  The partials are read together
// with the state, before the state is inspected (one memory round trip
// instead of two; the partial buffers are allocated for every probe, and
// their values are used only when the probe is active and past its first
// pass).  A pass can issue these before its own first loads.
struct PrologueIn {
  double acc[LDQ_NQ_MAX];
  ProbeState in;
};

template <int NW>
__device__ inline PrologueIn prologue_load(const TailArgs &ta, const ProbeRef &pr, int ntiles, int nred) {
  PrologueIn li;
#pragma unroll
  for (int i = 0; i < LDQ_NQ_MAX; ++i) li.acc[i] = 0.0;
  const double *src = pr.pin;
  // NW = 1: one wave reduces on its own (it may be any wave of a larger
  // workgroup); tid is then the lane
  const int tid = NW == 1 ? (int)(threadIdx.x & 63) : (int)threadIdx.x;
  for (int t = tid; t < ntiles; t += NW * 64) {
#pragma unroll
    for (int i = 0; i < LDQ_NQ_MAX; ++i)
      if (i < nred) li.acc[i] += src[(size_t)i * ntiles + t];
  }
  li.in = ta.st_in[pr.st];
  return li;
}

// The rest of a prologue, on the values prologue_load() read.
template <int NW>
__device__ inline Step prologue_finish(const TailArgs &ta, const ProbeRef &pr, int mode, bool owner, int nred,
                                       const PrologueIn &li) {
  double tot[LDQ_NQ_MAX];
  const int tid = NW == 1 ? (int)(threadIdx.x & 63) : (int)threadIdx.x;
  const ProbeState in = li.in;
  Step step{false, in.colour, 0.0, 0.0};
  if (!in.active) {
    if (owner && tid == 0) ta.st_out[pr.st] = in;    // carry the final state forward
    return step;
  }
  if (mode == MODE_INIT) {
    step.run = true;
    return step;
  }
  block_sum<NW>(li.acc, nred, tot);

  ProbeState ps = in;
  bool done = false;
  int status = 0;
  if (mode == MODE_FIRST) {
    // dots of r_0 = v: gamma_0 = v.v, delta_0 = v^T Q v, rho_0 = v.v
    const double g0 = tot[0], d0 = tot[1];
    ps.vnorm2 = g0;
    ps.gamma = g0;
    ps.alpha_prev = 1.0;
    ps.beta_prev = 0.0;
    ps.iter = 0;
#pragma unroll
    for (int i = 0; i < LDQ_MAXP; ++i) ps.grad[i] = 0.0;
    if (g0 == 0.0) {
      done = true;                                 // empty colour class
    } else if (!(d0 > 0.0) || !isfinite(d0)) {
      done = true;
      status = 2;
    } else {
      ps.alpha = g0 / d0;                          // alpha_0 = gamma_0 / p_0^T Q p_0 with p_0 = v
    }
    if (owner && tid < 64 && tid < ta.nshifts) {
      ShiftState s;
      s.zeta = cmk(1.0, 0.0);
      s.zeta_prev = cmk(1.0, 0.0);
      s.phi = cmk(tot[2], 0.0);                    // phi_0 = v^T p_0 = v.v
      s.psi = cmk(0.0, 0.0);
      s.frozen = done ? 1 : 0;
      s.pad = 0;
      ta.sh[(size_t)pr.st * ta.nshifts + tid] = s;
    }
    step.alpha = ps.alpha;
    step.beta = 0.0;                               // beta_{-1} = 0: p_0 = r_0
  } else {
    // dots of r_{k+1} (gamma', delta', rho') and omega_i = w_i . p_k of the last pass
    const double gn = tot[0], dn = tot[1];
    const double ak = ps.alpha, akm1 = ps.alpha_prev, bkm1 = ps.beta_prev;
    const double bk = gn / ps.gamma;               // beta_k
    bool all_frozen = false;
    if (owner) {
      bool bad = false;
      if constexpr (NW == 1) {
        all_frozen = shifts_update(ta, pr, ak, akm1, bkm1, bk, gn, tot[2], ps.vnorm2, &bad);
      } else {
        __shared__ int sh_flags[2];
        if (threadIdx.x < 64) {
          const bool f = shifts_update(ta, pr, ak, akm1, bkm1, bk, gn, tot[2], ps.vnorm2, &bad);
          if (threadIdx.x == 0) {
            sh_flags[0] = f;
            sh_flags[1] = bad;
          }
        }
        __syncthreads();
        all_frozen = sh_flags[0] != 0;
        bad = sh_flags[1] != 0;
      }
      if (bad) {
        done = true;
        status = 2;
      }
#pragma unroll
      for (int i = 0; i < LDQ_MAXP; ++i)
        if (i < ta.ngrad) ps.grad[i] += ak * tot[LDQ_NQ_BASE + i];   // w.x_{k+1} = w.x_k + alpha_k w.p_k
    }
    ps.iter += 1;
    const bool base_ok = !ta.need_base || (gn <= ta.grad_tol2 * ps.vnorm2);
    if (!done) {
      if (gn == 0.0 || (all_frozen && base_ok)) {
        done = true;
      } else {
        const double pap = dn - bk * gn / ak;      // p_{k+1}^T Q p_{k+1}
        if (!(pap > 0.0) || !isfinite(pap)) {
          done = true;
          status = 2;
        } else {
          ps.alpha_prev = ak;
          ps.alpha = gn / pap;                     // alpha_{k+1}
          ps.beta_prev = bk;
        }
        if (!done && ps.iter >= ta.max_iter) {
          done = true;
          status = 3;
        }
      }
    }
    ps.gamma = gn;
    step.alpha = ps.alpha;
    step.beta = ps.beta_prev;
  }
  if (owner && tid == 0) {
    if (done) {
      ps.active = 0;
      ps.status = status;
      atomicSub(ta.active_count, 1);
    } else if (ps.iter < ta.hist_cap) {
      // the CG coefficients define the Lanczos tridiagonal matrix of the probe
      // (diagonal 1/alpha_i + beta_{i-1}/alpha_{i-1}, off-diagonal
      // sqrt(beta_{i-1})/alpha_{i-1}); its eigenvalues lie in the spectrum of Q
      double *h = ta.hist + ((size_t)pr.st * ta.hist_cap + ps.iter) * 2;
      h[0] = ps.alpha;
      h[1] = mode == MODE_FIRST ? 0.0 : ps.beta_prev;
    }
    ta.st_out[pr.st] = ps;
  }
  step.run = !done;
  return step;
}

// Start of a pass: reduce the previous launch's partials, advance the probe's
// scalars, decide whether it is finished.  Called by every thread of the
// workgroup (NW waves; one tile per workgroup).
template <int NW>
__device__ inline Step pass_prologue(const TailArgs &ta, const ProbeRef &pr, int tile, int ntiles, int mode,
                                     int role = ROLE_TILE0) {
  const bool owner = tail_owner(role, tile);
  const int nred = tail_nred(ta, owner);
  const PrologueIn li = prologue_load<NW>(ta, pr, ntiles, nred);
  return prologue_finish<NW>(ta, pr, mode, owner, nred, li);
}

// End of a pass: the workgroup's sums of the nq quantities go to part_out.
template <int NW>
__device__ inline void pass_epilogue(const TailArgs &ta, const ProbeRef &pr, int tile, int ntiles, const double *q) {
  double tot[LDQ_NQ_MAX];
  const int nq = LDQ_NQ_BASE + ta.ngrad;
  block_sum<NW>(q, nq, tot);
  if (threadIdx.x == 0) {
    for (int i = 0; i < nq; ++i) pr.pout[(size_t)i * ntiles + tile] = tot[i];
  }
}

// Single-wave epilogue with a compile-time number of quantities (the wave
// may be any wave of its workgroup).
template <int NQ>
__device__ inline void pass_epilogue_n(const ProbeRef &pr, int tile, int ntiles, const double *q) {
  double tot[NQ];
#pragma unroll
  for (int i = 0; i < NQ; ++i) tot[i] = wave_sum(q[i]);
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int i = 0; i < NQ; ++i) pr.pout[(size_t)i * ntiles + tile] = tot[i];
  }
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
