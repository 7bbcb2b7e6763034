// Fused Krylov pass on 3-D lattices: Q = scale (diag(kappa2) + L), 7-point.
//
// Same per-probe step as the 2-D pass (p_k = r_k + beta p_{k-1}; s = Q p_k;
// r_{k+1} = r_k - alpha s; gamma', delta', rho' and the gradient dots), with a
// TX x TY column of the lattice owned by one workgroup that marches along z
// over a segment of planes.  Three planes of p (xy halo 2), two of r and three
// of r_{k+1} (xy halo 1) live in LDS as a rolling window, so every stored
// vector element is read from HBM once per pass; only the xy halo and two
// planes per segment are re-read (from L2).
#include "ldq_internal.h"
#include "tail.h"

namespace ldq {

constexpr int T3X = 32, T3Y = 8;

template <typename T>
__device__ inline int colour3(const Pass3D<T> &a, int x, int y, int z) {
  return a.colC > 0 ? (x + a.cola * y + a.colb * z) % a.colC
                    : a.colours[((size_t)z * a.ny + y) * a.nx + x];
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
        if (colour3(a, gx, gy, z) == colour) q[2] += r;
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
        dst[ry][rx] = (inbox(gx, gy, t) && colour3(a, gx, gy, t) == colour) ? T(1) : T(0);
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
            r = (colour3(a, gx, gy, z) == colour) ? T(1) : T(0);
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
              if (colour3(a, gx, gy, t) == colour) {
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
                  q[LDQ_NQ_BASE + i] += g.scale * d;
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

template <typename T>
hipError_t launch_pass3d(const Pass3D<T> &a, hipStream_t stream) {
  const int nblocks = a.ntiles * a.nprobes;
  hipLaunchKernelGGL((pass3d_kernel<T>), dim3(nblocks), dim3(LDQ_BLOCK), 0, stream, a);
  return hipGetLastError();
}

template hipError_t launch_pass3d<float>(const Pass3D<float> &, hipStream_t);
template hipError_t launch_pass3d<double>(const Pass3D<double> &, hipStream_t);

void pass3d_tiles(int nx, int ny, int nz, int zseg, int *tiles_x, int *tiles_y, int *nzseg, int *ntiles) {
  *tiles_x = (nx + T3X - 1) / T3X;
  *tiles_y = (ny + T3Y - 1) / T3Y;
  *nzseg = (nz + zseg - 1) / zseg;
  *ntiles = *tiles_x * *tiles_y * *nzseg;
}

}  // namespace ldq
