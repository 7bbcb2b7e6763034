// Fused Krylov pass on 3-D lattices: Q = scale (diag(kappa2) + L), 7-point.
//
// Same per-probe step as the 2-D pass (p_k = r_k + beta p_{k-1}; s = Q p_k;
// r_{k+1} = r_k - alpha s; gamma', delta', rho' and the gradient dots), with a
// TX x TY column of the lattice owned by one workgroup that marches along z
// over a segment of planes.  Three planes of p (xy halo 2), two of r and three
// of r_{k+1} (xy halo 1) live in LDS as a rolling window, so every stored
// vector element is read from HBM once per pass; only the xy halo and two
// planes per segment are re-read (from L2).
#include "bufio.h"
#include "ldq_internal.h"
#include "tail.h"

namespace ldq {

// Tile of one workgroup: T3X x T3Y output columns of the lattice (the fast
// pass below puts one wave on each of the T3Y + 4 rows of the tile and its
// halo, 64 = T3X + 4 lanes across), marched along z over zseg planes.
constexpr int T3X = 60, T3Y = 12;
constexpr int T3W = T3Y + 4;          // waves of the fast pass

template <typename T>
__device__ inline int colour3(const Pass3D<T> &a, int x, int y, int z) {
  return a.colC > 0 ? (x + a.cola * y + a.colb * z) % a.colC
                    : a.colours[((size_t)z * a.ny + y) * a.nx + x];
}
// Entry of probe `colour` at a site inside the lattice: 0 / 1 for a colour
// class, -1 / +1 for random signs.
template <typename T>
__device__ inline double probe3(const Pass3D<T> &a, int colour, int x, int y, int z) {
  if (a.rad) return rad_sign(a.seed, colour, ((int64_t)z * a.ny + y) * a.nx + x);
  if (a.uvec) return a.uvec[((size_t)colour * a.nz + z) * a.ny * a.nx + (size_t)y * a.nx + x];
  return colour3(a, x, y, z) == colour ? 1.0 : 0.0;
}

template <typename T>
__global__ __launch_bounds__(LDQ_BLOCK) void pass3d_kernel(Pass3D<T> a) {
  constexpr int PW = T3X + 4, PH = T3Y + 4, RW = T3X + 2, RH = T3Y + 2;
  __shared__ T sP[3][PH][PW];
  __shared__ T sR[2][RH][RW];
  __shared__ T sRN[3][RH][RW];

  const int L = xcd_remap(blockIdx.x, gridDim.x);
  const int probe = L / a.ntiles, tile = L - probe * a.ntiles;
  const ProbeRef pref = probe_ref(a.tail, probe, a.ntiles);
  const Step step = pass_prologue<LDQ_BLOCK / 64>(a.tail, pref, tile, a.ntiles, a.mode);
  if (!step.run) return;
  const int colour = step.colour;
  const double alpha = step.alpha, beta = step.beta;
  const int txi = tile % a.tiles_x, rest = tile / a.tiles_x;
  const int tyi = rest % a.tiles_y, tzi = rest / a.tiles_y;
  const int x0 = txi * T3X, y0 = tyi * T3Y, z0 = tzi * a.zseg;
  const int z1 = min(z0 + a.zseg, a.nz);
  const size_t n = (size_t)a.nx * a.ny * a.nz;
  const size_t off = (size_t)probe * n;
  const int tid = threadIdx.x;
  double q[LDQ_NQ_MAX];
#pragma unroll
  for (int i = 0; i < LDQ_NQ_MAX; ++i) q[i] = 0.0;

  auto inbox = [&](int x, int y, int z) {
    return x >= 0 && x < a.nx && y >= 0 && y < a.ny && z >= 0 && z < a.nz;
  };
  auto site = [&](int x, int y, int z) { return ((size_t)z * a.ny + y) * a.nx + x; };
  auto k2at = [&](size_t s) { return a.kappa2_field ? (double)a.kappa2_field[s] : a.kappa2; };

  // Q r_{k+1} at plane z on the tile, accumulated into the dots
  auto dots_plane = [&](int z) {
    const T(*cm)[RW] = sRN[(z + 3) % 3];
    const T(*dn)[RW] = sRN[(z + 2) % 3];
    const T(*up)[RW] = sRN[(z + 4) % 3];
    for (int e = tid; e < T3X * T3Y; e += LDQ_BLOCK) {
      const int ty = e / T3X, tx = e - ty * T3X;
      const int gx = x0 + tx, gy = y0 + ty;
      if (gx < a.nx && gy < a.ny) {
        const size_t s = site(gx, gy, z);
        const int px = tx + 1, py = ty + 1;
        const double r = (double)cm[py][px];
        const double lap = 6.0 * r - ((double)cm[py][px - 1] + (double)cm[py][px + 1] + (double)cm[py - 1][px] +
                                      (double)cm[py + 1][px] + (double)dn[py][px] + (double)up[py][px]);
        const double qr = a.scale * (k2at(s) * r + lap);
        q[0] += r * r;
        q[1] += r * qr;
        q[2] += probe3(a, colour, gx, gy, z) * r;
      }
    }
  };

  if (a.mode == MODE_INIT) {
    for (int t = z0 - 1; t <= z1; ++t) {
      __syncthreads();
      T(*dst)[RW] = sRN[(t + 3) % 3];
      for (int e = tid; e < RW * RH; e += LDQ_BLOCK) {
        const int ry = e / RW, rx = e - ry * RW;
        const int gx = x0 - 1 + rx, gy = y0 - 1 + ry;
        dst[ry][rx] = inbox(gx, gy, t) ? (T)probe3(a, colour, gx, gy, t) : T(0);
      }
      __syncthreads();
      if (t - 1 >= z0) dots_plane(t - 1);
    }
  } else {
    auto load_plane = [&](int z) {
      T(*dp)[PW] = sP[(z + 3) % 3];
      T(*dr)[RW] = sR[(z + 2) & 1];
      for (int e = tid; e < PW * PH; e += LDQ_BLOCK) {
        const int ey = e / PW, ex = e - ey * PW;
        const int gx = x0 - 2 + ex, gy = y0 - 2 + ey;
        T r = 0, p = 0;
        if (inbox(gx, gy, z)) {
          const size_t s = site(gx, gy, z);
          if (a.mode == MODE_FIRST) {
            r = (T)probe3(a, colour, gx, gy, z);
            p = r;
          } else {
            r = a.r_in[off + s];
            p = (T)((double)r + beta * (double)a.p_in[off + s]);
          }
        }
        dp[ey][ex] = p;
        const int rx = ex - 1, ry = ey - 1;
        if (rx >= 0 && rx < RW && ry >= 0 && ry < RH) dr[ry][rx] = r;
      }
    };
    load_plane(z0 - 2);
    load_plane(z0 - 1);
    for (int t = z0 - 1; t <= z1; ++t) {
      load_plane(t + 1);
      __syncthreads();
      // r_{k+1} at plane t on the tile + 1 halo
      {
        const T(*pc)[PW] = sP[(t + 3) % 3];
        const T(*pd)[PW] = sP[(t + 2) % 3];
        const T(*pu)[PW] = sP[(t + 4) % 3];
        const T(*rc)[RW] = sR[(t + 2) & 1];
        T(*dst)[RW] = sRN[(t + 3) % 3];
        const bool own = (t >= z0 && t < z1);
        for (int e = tid; e < RW * RH; e += LDQ_BLOCK) {
          const int ry = e / RW, rx = e - ry * RW;
          const int gx = x0 - 1 + rx, gy = y0 - 1 + ry;
          const int px = rx + 1, py = ry + 1;
          T rn = 0;
          if (inbox(gx, gy, t)) {
            const size_t s = site(gx, gy, t);
            const double pv = (double)pc[py][px];
            const double nb = (double)pc[py][px - 1] + (double)pc[py][px + 1] + (double)pc[py - 1][px] +
                              (double)pc[py + 1][px] + (double)pd[py][px] + (double)pu[py][px];
            const double sv = a.scale * (k2at(s) * pv + 6.0 * pv - nb);
            rn = (T)((double)rc[ry][rx] - alpha * sv);
            if (own && rx >= 1 && rx <= T3X && ry >= 1 && ry <= T3Y) {
              a.r_out[off + s] = rn;
              a.p_out[off + s] = pc[py][px];
              const double vw = probe3(a, colour, gx, gy, t);
              if (vw != 0.0) {
#pragma unroll
                for (int i = 0; i < LDQ_MAXP; ++i) {
                  if (i >= a.tail.ngrad) break;
                  const GradTerm<T> &g = a.grad[i];
                  double d;
                  if (g.kind == GK_DIAG) {
                    d = (double)g.field[s] * pv;
                  } else {
                    const double k2 = g.field ? (double)g.field[s] : g.kappa2;
                    d = k2 * pv + 6.0 * pv - nb;
                  }
                  q[LDQ_NQ_BASE + i] += vw * g.scale * d;
                }
              }
            }
          }
          dst[ry][rx] = rn;
        }
      }
      __syncthreads();
      if (t - 1 >= z0) dots_plane(t - 1);
    }
  }
  pass_epilogue<LDQ_BLOCK / 64>(a.tail, pref, tile, a.ntiles, q);
}


// Lane i receives lane i - 1 / i + 1 through a DPP wave shift (0 past the ends).
__device__ inline float lane_left(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x138, 0xF, 0xF, true));
}
__device__ inline float lane_right(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x130, 0xF, 0xF, true));
}
__device__ inline double lane_left(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), 0x138, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x138, 0xF, 0xF, true);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}
__device__ inline double lane_right(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), 0x130, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x130, 0xF, 0xF, true);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}
// Workgroup barrier for LDS traffic only: this wave's LDS accesses complete
// (lgkmcnt 0; vmcnt and expcnt left at their maxima in the gfx9 encoding)
// before it arrives, while its global loads stay in flight -- a full
// __syncthreads would drain the prefetch at every step.  The empty asm
// statements keep the compiler from moving memory accesses across.
__device__ inline void lds_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0xC07F);
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

__device__ inline float fma3(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ inline double fma3(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Specialised STEP pass for modular colourings, Q = diag(kappa2) + L (a field
// when FIELD, else a constant; scale 1) and NG diagonal derivative operators.
// Wave w of the workgroup owns lattice row y0 - 2 + w, lane l column x0 - 2 +
// l; z-neighbours are kept in registers (p at planes t - 1, t, t + 1; r' at
// t - 2, t - 1, t), x-neighbours come from DPP lane shifts and y-neighbours
// from one LDS row buffer per quantity, written once per z-step.  Step t forms
// s = Q p_k and r_{k+1} = r_k - alpha s on plane t (waves 1 .. T3W - 2, so the
// r' rows the next stencil needs exist) and Q r_{k+1} on plane t - 1 (the
// output waves 2 .. T3W - 3); one barrier per step.  Loads run PF planes
// ahead.  Arithmetic is in T with the Laplacian's exact coefficients; dot
// products in FP64.
template <typename T, int NG, bool FIELD>
__global__ __launch_bounds__(64 * T3W) void pass3d_fast(Pass3D<T> a) {
  constexpr int NQ = LDQ_NQ_BASE + NG;
  constexpr int PF = 4;                       // prefetch distance in planes
  // row buffers of p and r' per step parity; rows 0 and T3W + 1 stay 0 (the
  // missing neighbours of the outer waves), so every read is unconditional
  __shared__ T sp[2][T3W + 2][64];
  __shared__ T srn[2][T3W + 2][64];
  for (int k = threadIdx.x; k < 2 * (T3W + 2) * 64; k += blockDim.x) {
    (&sp[0][0][0])[k] = T(0);
    (&srn[0][0][0])[k] = T(0);
  }

  const int L = xcd_remap(blockIdx.x, gridDim.x);
  const int probe = L / a.ntiles, tile = L - probe * a.ntiles;
  const ProbeRef pref = probe_ref(a.tail, probe, a.ntiles);
  const Step step = pass_prologue<T3W>(a.tail, pref, tile, a.ntiles, MODE_STEP);
  if (!step.run) return;
  const int colour = __builtin_amdgcn_readfirstlane(step.colour);
  const T alpha_t = (T)step.alpha, beta_t = (T)step.beta;

  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const int txi = tile % a.tiles_x, rest = tile / a.tiles_x;
  const int tyi = rest % a.tiles_y, tzi = rest / a.tiles_y;
  const int x0 = txi * T3X, y0 = tyi * T3Y, z0 = tzi * a.zseg;
  const int z1 = min(z0 + a.zseg, nz);
  const int x = x0 - 2 + lane, y = y0 - 2 + w;
  const bool xin = x >= 0 && x < nx, yin = y >= 0 && y < ny;
  const bool in = xin && yin;
  const bool own = lane >= 2 && lane < 62 && x < nx && w >= 2 && w < T3W - 2 && y < ny;
  const int xc = min(max(x, 0), nx - 1), yc = min(max(y, 0), ny - 1);

  const size_t n = (size_t)nx * ny * nz;
  const size_t off = (size_t)probe * n;
  const unsigned vbytes = (unsigned)(n * sizeof(T));
  const __amdgpu_buffer_rsrc_t rs_rin = make_rsrc(a.r_in + off, vbytes);
  const __amdgpu_buffer_rsrc_t rs_pin = make_rsrc(a.p_in + off, vbytes);
  const __amdgpu_buffer_rsrc_t rs_rout = make_rsrc(a.r_out + off, vbytes);
  const __amdgpu_buffer_rsrc_t rs_pout = make_rsrc(a.p_out + off, vbytes);
  const __amdgpu_buffer_rsrc_t rs_k2 = make_rsrc(FIELD ? a.kappa2_field : a.r_in, vbytes);
  const __amdgpu_buffer_rsrc_t rs_g0 = make_rsrc(NG > 0 ? a.grad[0].field : a.r_in, vbytes);
  const __amdgpu_buffer_rsrc_t rs_g1 = make_rsrc(NG > 1 ? a.grad[1].field : a.r_in, vbytes);
  const unsigned lo = ((unsigned)yc * (unsigned)nx + (unsigned)xc) * (unsigned)sizeof(T);   // lane offset in a plane
  const unsigned planeb = (unsigned)nx * (unsigned)ny * (unsigned)sizeof(T);
  const T k2c = (T)a.kappa2;
  const T g0s = NG > 0 ? (T)a.grad[0].scale : T(0), g1s = NG > 1 ? (T)a.grad[1].scale : T(0);

  // colour (x + a y + b z) mod C == j  <=>  x mod C == (j - a y - b z) mod C
  const int C = __builtin_amdgcn_readfirstlane(a.colC);
  const int cx = xin ? x % C : -1;
  const int ay = __builtin_amdgcn_readfirstlane((int)(((long)a.cola * ((y % C + C) % C)) % C));
  const int bstep = __builtin_amdgcn_readfirstlane(a.colb % C);
  auto bz_of = [&](int z) -> int {
    return __builtin_amdgcn_readfirstlane((int)(((long)bstep * ((z % C + C) % C)) % C));
  };
  auto bz_next = [&](int bz) -> int {
    bz += bstep;
    return __builtin_amdgcn_readfirstlane(bz >= C ? bz - C : bz);
  };
  auto mine = [&](int bz) -> bool {
    int t = colour - ay - bz;
    t += (t < 0) ? C : 0;
    t += (t < 0) ? C : 0;
    return cx == t;
  };

  // prefetch ring: the raw r and p_{k-1} loads of plane z sit in slot
  // (z - zs) mod (PF + 1), zs = z0 - 2 the first plane of the march
  // together with kappa2 and, on the probe's own sites, the derivative
  // diagonals (every load of a step is issued PF planes ahead: waits are in
  // issue order, so one late load would drain the whole prefetch)
  T fr[PF + 1], fp[PF + 1], fk[PF + 1], fg0[PF + 1], fg1[PF + 1];
  auto load_into = [&](int k, int z, int bz) {
    const int zc = min(max(z, 0), nz - 1);
    const unsigned so = (unsigned)zc * planeb;
    fr[k] = buf_ld((T *)nullptr, rs_rin, lo, so);
    fp[k] = buf_ld((T *)nullptr, rs_pin, lo, so);
    if constexpr (FIELD) fk[k] = buf_ld((T *)nullptr, rs_k2, lo, so);
    if constexpr (NG > 0) {
      // only the probe's own sites read memory: the other lanes address past
      // the end of the buffer, which the hardware range check answers with 0
      // (an unconditional load keeps the wait counting in issue order)
      const bool use = own && z >= z0 && z < z1 && mine(bz);
      const unsigned go = use ? lo + so : 0xFFFFFFF0u;
      fg0[k] = buf_ld((T *)nullptr, rs_g0, go, 0u);
      if constexpr (NG > 1) fg1[k] = buf_ld((T *)nullptr, rs_g1, go, 0u);
    }
  };

  // p_k of plane z from its raw loads (0 outside the lattice)
  auto form_p = [&](T r, T pv, int z) -> T {
    const bool ok = in && z >= 0 && z < nz;
    return ok ? fma3(beta_t, pv, r) : T(0);
  };

  double q0 = 0.0, q1 = 0.0;
  T racc = T(0), g0acc = T(0), g1acc = T(0);

  // start: planes zs .. zs + PF in the ring; slots 0 and 1 are consumed at
  // once and refilled with planes zs + PF + 1 and zs + PF + 2
  const int zs = z0 - 2;
  // colour part of the planes: bz_l of the next plane to load
  int bz_l = bz_of(zs);
#pragma unroll
  for (int k = 0; k <= PF; ++k) {
    load_into(k, zs + k, bz_l);
    bz_l = bz_next(bz_l);
  }
  // rings: p at t - 1, t, t + 1; r at t; r' at t - 2, t - 1; kappa2 at t - 1, t
  T pm = form_p(fr[0], fp[0], zs), pc = form_p(fr[1], fp[1], zs + 1);
  T rc = (in && zs + 1 >= 0 && zs + 1 < nz) ? fr[1] : T(0);
  T kc = FIELD ? fk[1] : k2c, km = T(0);
  T g0c = fg0[1], g1c = fg1[1];
  load_into(0, zs + PF + 1, bz_l);
  bz_l = bz_next(bz_l);
  load_into(1, zs + PF + 2, bz_l);
  bz_l = bz_next(bz_l);
  T rnm2 = T(0), rnm1 = T(0);
  int bz_m = bz_of(zs);          // colour part of plane t - 1 (t = zs + 1 at the first step)

  // the ring slot of plane z is (z - zs) mod (PF + 1); the loop is unrolled by
  // PF + 1 so slots are compile-time
  // steps t = zs + 1 .. z1, padded to whole pairs of rings: the extra steps store
  // nothing and add no dot products (their planes fail the z0 <= t < z1
  // tests), and with no exit inside the unrolled ring the compiler does not
  // wait for every load in flight at the exit's join
  constexpr int RING2 = 2 * (PF + 1);   // two rings per loop iteration
  const int nsteps = (z1 - zs + RING2 - 1) / RING2 * RING2;
  for (int b = 0; b < nsteps; b += RING2) {
#pragma unroll
    for (int u = 0; u < RING2; ++u) {
      const int i = b + u;
      const int t = zs + 1 + i;
      // plane t + 1 of p from the ring, then refill its slot with plane t + 1 + PF
      const int sn = (u + 2) % (PF + 1);
      const T rn1 = fr[sn], pn1raw = fp[sn];
      const T pp = form_p(rn1, pn1raw, t + 1);
      const T kn = FIELD ? ((in && t + 1 >= 0 && t + 1 < nz) ? fk[sn] : T(0)) : k2c;
      const T g0n = fg0[sn], g1n = fg1[sn];
      load_into(sn, t + PF + 2, bz_l);
      bz_l = bz_next(bz_l);
      const bool tin = t >= 0 && t < nz;
      // y-neighbours of p_k on plane t
      sp[t & 1][w + 1][lane] = pc;
      lds_barrier();
      T s = T(0);
      const T ks = FIELD ? kc : k2c;
      {
        const T up = sp[t & 1][w][lane];
        const T dn = sp[t & 1][w + 2][lane];
        const T nb = (lane_left(pc) + lane_right(pc)) + (up + dn) + (pm + pp);
        s = fma3(ks, pc, fma3(T(6), pc, -nb));
      }
      const T rnew = (in && tin) ? fma3(-alpha_t, s, rc) : T(0);
      const int bz_c = bz_next(bz_m);
      if (own && t >= z0 && t < z1) {
        const unsigned so = (unsigned)t * planeb;
        buf_st(rnew, rs_rout, lo, so);
        buf_st(pc, rs_pout, lo, so);
        if constexpr (NG > 0) {
          // the diagonals were loaded (PF planes ago) on the probe's sites only
          g0acc = fma3(g0c, pc, g0acc);
          if constexpr (NG > 1) g1acc = fma3(g1c, pc, g1acc);
        }
      }
      srn[t & 1][w + 1][lane] = rnew;
      // Q r_{k+1} on plane t - 1 (its y-neighbours were written last step)
      if (t - 1 >= z0 && t - 1 < z1) {
        const T up = srn[(t - 1) & 1][w][lane];
        const T dn = srn[(t - 1) & 1][w + 2][lane];
        const T nb = (lane_left(rnm1) + lane_right(rnm1)) + (up + dn) + (rnm2 + rnew);
        const T km_t = FIELD ? km : k2c;
        const T qr = fma3(km_t, rnm1, fma3(T(6), rnm1, -nb));
        const double r2 = (double)rnm1;
        q0 = __builtin_fma(r2, r2, q0);
        q1 = __builtin_fma(r2, (double)qr, q1);
        racc += mine(bz_m) ? rnm1 : T(0);
      }
      // rotate
      pm = pc;
      pc = pp;
      rc = (in && t + 1 >= 0 && t + 1 < nz) ? rn1 : T(0);
      rnm2 = rnm1;
      rnm1 = rnew;
      km = kc;
      kc = kn;
      g0c = g0n;
      g1c = g1n;
      bz_m = bz_c;
    }
  }
  double qv[NQ];
  qv[0] = own ? q0 : 0.0;
  qv[1] = own ? q1 : 0.0;
  qv[2] = own ? (double)racc : 0.0;
  if constexpr (NG > 0) qv[LDQ_NQ_BASE] = own ? (double)g0s * (double)g0acc : 0.0;
  if constexpr (NG > 1) qv[LDQ_NQ_BASE + 1] = own ? (double)g1s * (double)g1acc : 0.0;
  double tot[LDQ_NQ_MAX];
#pragma unroll
  for (int i = 0; i < LDQ_NQ_MAX; ++i) tot[i] = i < NQ ? qv[i] : 0.0;
  pass_epilogue<T3W>(a.tail, pref, tile, a.ntiles, tot);
}

// Wide STEP pass for lattices at most 128 sites wide (an even number): lane
// l owns the two consecutive columns 2l, 2l + 1 of a whole lattice row, so a
// wave covers its row without an x-halo and with aligned 8-byte (FP64:
// 16-byte) loads and stores; x-neighbours are the lane's other column or one
// DPP shift away.  Otherwise as pass3d_fast (16 waves on the rows of a
// T3Y-row tile and its y-halo, z marched with one LDS barrier per plane).
// Its partial sums go to the slot of strip tile (0, ty, tz) of the strip
// numbering shared with the other 3-D passes; the other strip slots of
// (ty, tz) receive zeros.
template <typename T, int NG, bool FIELD>
__global__ __launch_bounds__(64 * T3W) void pass3d_wide(Pass3D<T> a) {
  using P2 = Pair<T>;
  constexpr int NQ = LDQ_NQ_BASE + NG;
  constexpr int PF = 4;
  // row buffers as in pass3d_fast (rows 0 and T3W + 1 stay 0)
  __shared__ P2 sp[2][T3W + 2][64];
  __shared__ P2 srn[2][T3W + 2][64];
  for (int k = threadIdx.x; k < 2 * (T3W + 2) * 64; k += blockDim.x) {
    (&sp[0][0][0])[k] = P2{T(0), T(0)};
    (&srn[0][0][0])[k] = P2{T(0), T(0)};
  }

  const int tyz = a.tiles_y * a.nzseg;
  const int L = xcd_remap(blockIdx.x, gridDim.x);
  const int probe = L / tyz, rest = L - probe * tyz;
  const int tyi = rest % a.tiles_y, tzi = rest / a.tiles_y;
  const int tile = a.tiles_x * rest;            // strip tile (0, tyi, tzi)
  const ProbeRef pref = probe_ref(a.tail, probe, a.ntiles);
  const Step step = pass_prologue<T3W>(a.tail, pref, tile, a.ntiles, MODE_STEP);
  if (!step.run) return;
  const int colour = __builtin_amdgcn_readfirstlane(step.colour);
  const T alpha_t = (T)step.alpha, beta_t = (T)step.beta;

  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const int y0 = tyi * T3Y, z0 = tzi * a.zseg;
  const int z1 = min(z0 + a.zseg, nz);
  const int xa = 2 * lane, y = y0 - 2 + w;
  const bool xin = xa < nx, yin = y >= 0 && y < ny;
  const bool in = xin && yin;
  const bool own = xin && w >= 2 && w < T3W - 2 && y < ny;
  const int yc = min(max(y, 0), ny - 1);

  const size_t n = (size_t)nx * ny * nz;
  const size_t off = (size_t)probe * n;
  const unsigned vbytes = (unsigned)(n * sizeof(T));
  const __amdgpu_buffer_rsrc_t rs_rin = make_rsrc(a.r_in + off, vbytes);
  const __amdgpu_buffer_rsrc_t rs_pin = make_rsrc(a.p_in + off, vbytes);
  const __amdgpu_buffer_rsrc_t rs_rout = make_rsrc(a.r_out + off, vbytes);
  const __amdgpu_buffer_rsrc_t rs_pout = make_rsrc(a.p_out + off, vbytes);
  const __amdgpu_buffer_rsrc_t rs_k2 = make_rsrc(FIELD ? a.kappa2_field : a.r_in, vbytes);
  const __amdgpu_buffer_rsrc_t rs_g0 = make_rsrc(NG > 0 ? a.grad[0].field : a.r_in, vbytes);
  const __amdgpu_buffer_rsrc_t rs_g1 = make_rsrc(NG > 1 ? a.grad[1].field : a.r_in, vbytes);
  // lane offset in a plane; lanes past the lattice's width address past the
  // end of the buffers (loads read 0, stores are dropped)
  const unsigned lo = xin ? ((unsigned)yc * (unsigned)nx + (unsigned)xa) * (unsigned)sizeof(T) : 0xFFFFFFF0u;
  const unsigned planeb = (unsigned)nx * (unsigned)ny * (unsigned)sizeof(T);
  const T k2c = (T)a.kappa2;
  const T g0s = NG > 0 ? (T)a.grad[0].scale : T(0), g1s = NG > 1 ? (T)a.grad[1].scale : T(0);

  const int C = __builtin_amdgcn_readfirstlane(a.colC);
  const int cxa = xin ? xa % C : -1, cxb = xin ? (xa + 1) % C : -1;
  const int ay = __builtin_amdgcn_readfirstlane((int)(((long)a.cola * ((y % C + C) % C)) % C));
  const int bstep = __builtin_amdgcn_readfirstlane(a.colb % C);
  auto bz_of = [&](int z) -> int {
    return __builtin_amdgcn_readfirstlane((int)(((long)bstep * ((z % C + C) % C)) % C));
  };
  auto bz_next = [&](int bz) -> int {
    bz += bstep;
    return __builtin_amdgcn_readfirstlane(bz >= C ? bz - C : bz);
  };
  // x mod C that is the probe's colour on this row and the plane of bz
  auto target = [&](int bz) -> int {
    int t = colour - ay - bz;
    t += (t < 0) ? C : 0;
    t += (t < 0) ? C : 0;
    return t;
  };

  P2 fr[PF + 1], fp[PF + 1], fk[PF + 1], fg0[PF + 1], fg1[PF + 1];
  auto load_into = [&](int k, int z, int bz) {
    const int zc = min(max(z, 0), nz - 1);
    const unsigned so = (unsigned)zc * planeb;
    fr[k] = buf_ld2((T *)nullptr, rs_rin, lo, so);
    fp[k] = buf_ld2((T *)nullptr, rs_pin, lo, so);
    if constexpr (FIELD) fk[k] = buf_ld2((T *)nullptr, rs_k2, lo, so);
    if constexpr (NG > 0) {
      // only pairs holding one of the probe's sites read memory (the other
      // element is masked where the values are used)
      const int tg = target(bz);
      const bool use = own && z >= z0 && z < z1 && (cxa == tg || cxb == tg);
      const unsigned go = use ? lo + so : 0xFFFFFFF0u;
      fg0[k] = buf_ld2((T *)nullptr, rs_g0, go, 0u);
      if constexpr (NG > 1) fg1[k] = buf_ld2((T *)nullptr, rs_g1, go, 0u);
    }
  };
  auto form_p = [&](P2 r, P2 pv, int z) -> P2 {
    const bool ok = in && z >= 0 && z < nz;
    return P2{ok ? fma3(beta_t, pv.a, r.a) : T(0), ok ? fma3(beta_t, pv.b, r.b) : T(0)};
  };
  // 7-point stencil of Q on one plane: centre c, x-pair neighbours from the
  // lane's own pair and the DPP shifts, y from LDS, z from the ring
  auto apply = [&](P2 c, P2 up, P2 dn, P2 zm, P2 zp, P2 kk) -> P2 {
    const T nba = (lane_left(c.b) + c.b) + (up.a + dn.a) + (zm.a + zp.a);
    const T nbb = (c.a + lane_right(c.a)) + (up.b + dn.b) + (zm.b + zp.b);
    return P2{fma3(kk.a, c.a, fma3(T(6), c.a, -nba)), fma3(kk.b, c.b, fma3(T(6), c.b, -nbb))};
  };
  const P2 zero{T(0), T(0)};
  const P2 k2p{k2c, k2c};

  double q0 = 0.0, q1 = 0.0;
  T racc = T(0), g0acc = T(0), g1acc = T(0);

  const int zs = z0 - 2;
  int bz_l = bz_of(zs);
#pragma unroll
  for (int k = 0; k <= PF; ++k) {
    load_into(k, zs + k, bz_l);
    bz_l = bz_next(bz_l);
  }
  P2 pm = form_p(fr[0], fp[0], zs), pc = form_p(fr[1], fp[1], zs + 1);
  const bool in1 = in && zs + 1 >= 0 && zs + 1 < nz;
  P2 rc{in1 ? fr[1].a : T(0), in1 ? fr[1].b : T(0)};
  P2 kc = FIELD ? fk[1] : k2p, km = zero;
  P2 g0c = fg0[1], g1c = fg1[1];
  load_into(0, zs + PF + 1, bz_l);
  bz_l = bz_next(bz_l);
  load_into(1, zs + PF + 2, bz_l);
  bz_l = bz_next(bz_l);
  P2 rnm2 = zero, rnm1 = zero;
  int bz_m = bz_of(zs);

  // steps t = zs + 1 .. z1, padded to whole pairs of rings: the extra steps store
  // nothing and add no dot products (their planes fail the z0 <= t < z1
  // tests), and with no exit inside the unrolled ring the compiler does not
  // wait for every load in flight at the exit's join
  constexpr int RING2 = 2 * (PF + 1);   // two rings per loop iteration
  const int nsteps = (z1 - zs + RING2 - 1) / RING2 * RING2;
  for (int b = 0; b < nsteps; b += RING2) {
#pragma unroll
    for (int u = 0; u < RING2; ++u) {
      const int i = b + u;
      const int t = zs + 1 + i;
      const int sn = (u + 2) % (PF + 1);
      const P2 rn1 = fr[sn], pn1raw = fp[sn];
      const P2 pp = form_p(rn1, pn1raw, t + 1);
      const bool inn = in && t + 1 >= 0 && t + 1 < nz;
      const P2 kn = FIELD ? P2{inn ? fk[sn].a : T(0), inn ? fk[sn].b : T(0)} : k2p;
      const P2 g0n = fg0[sn], g1n = fg1[sn];
      load_into(sn, t + PF + 2, bz_l);
      bz_l = bz_next(bz_l);
      const bool tin = t >= 0 && t < nz;
      sp[t & 1][w + 1][lane] = pc;
      lds_barrier();
      const P2 up = sp[t & 1][w][lane];
      const P2 dn = sp[t & 1][w + 2][lane];
      const P2 s = apply(pc, up, dn, pm, pp, FIELD ? kc : k2p);
      const bool rin = in && tin;
      const P2 rnew{rin ? fma3(-alpha_t, s.a, rc.a) : T(0), rin ? fma3(-alpha_t, s.b, rc.b) : T(0)};
      const int bz_c = bz_next(bz_m);
      if (own && t >= z0 && t < z1) {
        const unsigned so = (unsigned)t * planeb;
        buf_st2(rnew, rs_rout, lo, so);
        buf_st2(pc, rs_pout, lo, so);
        if constexpr (NG > 0) {
          const int tg = target(bz_c);
          const T ma = cxa == tg ? T(1) : T(0), mb = cxb == tg ? T(1) : T(0);
          g0acc = fma3(ma * g0c.a, pc.a, fma3(mb * g0c.b, pc.b, g0acc));
          if constexpr (NG > 1) g1acc = fma3(ma * g1c.a, pc.a, fma3(mb * g1c.b, pc.b, g1acc));
        }
      }
      srn[t & 1][w + 1][lane] = rnew;
      if (t - 1 >= z0 && t - 1 < z1) {
        const P2 upr = srn[(t - 1) & 1][w][lane];
        const P2 dnr = srn[(t - 1) & 1][w + 2][lane];
        const P2 qr = apply(rnm1, upr, dnr, rnm2, rnew, FIELD ? km : k2p);
        const double ra = (double)rnm1.a, rb = (double)rnm1.b;
        q0 = __builtin_fma(ra, ra, q0);
        q0 = __builtin_fma(rb, rb, q0);
        q1 = __builtin_fma(ra, (double)qr.a, q1);
        q1 = __builtin_fma(rb, (double)qr.b, q1);
        const int tm = target(bz_m);
        racc += (cxa == tm ? rnm1.a : T(0)) + (cxb == tm ? rnm1.b : T(0));
      }
      pm = pc;
      pc = pp;
      rc = P2{inn ? rn1.a : T(0), inn ? rn1.b : T(0)};
      rnm2 = rnm1;
      rnm1 = rnew;
      km = kc;
      kc = kn;
      g0c = g0n;
      g1c = g1n;
      bz_m = bz_c;
    }
  }
  double qv[NQ];
  qv[0] = own ? q0 : 0.0;
  qv[1] = own ? q1 : 0.0;
  qv[2] = own ? (double)racc : 0.0;
  if constexpr (NG > 0) qv[LDQ_NQ_BASE] = own ? (double)g0s * (double)g0acc : 0.0;
  if constexpr (NG > 1) qv[LDQ_NQ_BASE + 1] = own ? (double)g1s * (double)g1acc : 0.0;
  double tot[LDQ_NQ_MAX];
#pragma unroll
  for (int i = 0; i < LDQ_NQ_MAX; ++i) tot[i] = i < NQ ? qv[i] : 0.0;
  pass_epilogue<T3W>(a.tail, pref, tile, a.ntiles, tot);
  if (threadIdx.x == 0)
    for (int tx = 1; tx < a.tiles_x; ++tx)
      for (int i = 0; i < NQ; ++i) pref.pout[(size_t)i * a.ntiles + tile + tx] = 0.0;
}

// fast: STEP pass with a modular colouring, scale 1 and at most two diagonal
// derivative operators (checked by the host driver)
template <typename T>
hipError_t launch_pass3d(const Pass3D<T> &a, bool fast, hipStream_t stream) {
  const int nblocks = a.ntiles * a.nprobes;
  // the wide pass in FP32 only (its FP64 form needs more registers than a
  // 16-wave workgroup leaves)
  if (sizeof(T) == 4 && fast && a.mode == MODE_STEP && a.nx <= 128 && a.nx % 2 == 0) {
    if constexpr (sizeof(T) == 4) {
      const bool field = a.kappa2_field != nullptr;
      const dim3 g(a.tiles_y * a.nzseg * a.nprobes), b(64 * T3W);
      switch (a.tail.ngrad * 2 + (field ? 1 : 0)) {
        case 0: hipLaunchKernelGGL((pass3d_wide<T, 0, false>), g, b, 0, stream, a); break;
        case 1: hipLaunchKernelGGL((pass3d_wide<T, 0, true>), g, b, 0, stream, a); break;
        case 2: hipLaunchKernelGGL((pass3d_wide<T, 1, false>), g, b, 0, stream, a); break;
        case 3: hipLaunchKernelGGL((pass3d_wide<T, 1, true>), g, b, 0, stream, a); break;
        case 4: hipLaunchKernelGGL((pass3d_wide<T, 2, false>), g, b, 0, stream, a); break;
        default: hipLaunchKernelGGL((pass3d_wide<T, 2, true>), g, b, 0, stream, a); break;
      }
    }
  } else if (fast && a.mode == MODE_STEP) {
    const bool field = a.kappa2_field != nullptr;
    const dim3 g(nblocks), b(64 * T3W);
    switch (a.tail.ngrad * 2 + (field ? 1 : 0)) {
      case 0: hipLaunchKernelGGL((pass3d_fast<T, 0, false>), g, b, 0, stream, a); break;
      case 1: hipLaunchKernelGGL((pass3d_fast<T, 0, true>), g, b, 0, stream, a); break;
      case 2: hipLaunchKernelGGL((pass3d_fast<T, 1, false>), g, b, 0, stream, a); break;
      case 3: hipLaunchKernelGGL((pass3d_fast<T, 1, true>), g, b, 0, stream, a); break;
      case 4: hipLaunchKernelGGL((pass3d_fast<T, 2, false>), g, b, 0, stream, a); break;
      default: hipLaunchKernelGGL((pass3d_fast<T, 2, true>), g, b, 0, stream, a); break;
    }
  } else {
    hipLaunchKernelGGL((pass3d_kernel<T>), dim3(nblocks), dim3(LDQ_BLOCK), 0, stream, a);
  }
  return hipGetLastError();
}

template hipError_t launch_pass3d<float>(const Pass3D<float> &, bool, hipStream_t);
template hipError_t launch_pass3d<double>(const Pass3D<double> &, bool, hipStream_t);

void pass3d_tiles(int nx, int ny, int nz, int zseg, int *tiles_x, int *tiles_y, int *nzseg, int *ntiles) {
  *tiles_x = (nx + T3X - 1) / T3X;
  *tiles_y = (ny + T3Y - 1) / T3Y;
  *nzseg = (nz + zseg - 1) / zseg;
  *ntiles = *tiles_x * *tiles_y * *nzseg;
}

}  // namespace ldq
