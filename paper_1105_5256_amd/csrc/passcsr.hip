// Krylov passes for a general sparse symmetric operator (Sec. 2.1: the
// multi-shift CG whose only operator access is the product Q p).
//
// Layout: the rows are cut into slices of 64, one wave per slice.  A slice
// keeps its entries column-major (entry k of lane l at sptr[s] + 64 k + l), so
// the wave loads them coalesced once per launch and keeps them in registers
// while it walks every active probe: the operator is read from memory once per
// pass, not once per probe.  Vectors are probe-major, [probe][row].
//
// One iteration k of a probe:
//   pass A: p_k = r_k + beta_{k-1} p_{k-1} (formed on the fly at every column
//           a row touches), r_{k+1} = r_k - alpha_k Q p_k, stores r_{k+1}, p_k,
//           partial sums of gamma' = |r_{k+1}|^2, rho' = v^T r_{k+1} and
//           omega_i = (dQ_i v)^T p_k;
//   pass B: partial sums of delta' = r_{k+1}^T Q r_{k+1};
//   tail:   one wave per probe reduces the partials in a fixed order and runs
//           the scalar recurrences (base CG and every shift).
// The product Q r_{k+1} needs r_{k+1} at the neighbours' neighbours, which a
// single pass over a general graph cannot form; hence the second pass.
#include "tail.h"
#include "bufio.h"

namespace ldq {

// ------------------------------------------------------------ slab build

struct CsrSrc {
  const int32_t *rowptr, *colind;   // CSR operator, or nullptr
  const double *val;
  const double *diag;               // diagonal operator, or nullptr
};

struct CsrSrcs {
  int nsrc;                         // Q first, then the derivative operators
  CsrSrc src[1 + LDQ_MAXP];
};

// Walk the union of the row patterns of all sources in increasing column
// order; f(column, values[]) is called once per distinct column.
template <typename F>
__device__ inline int union_row(const CsrSrcs &S, int64_t row, F f) {
  int32_t pos[1 + LDQ_MAXP], end[1 + LDQ_MAXP];
  bool diag_done[1 + LDQ_MAXP];
  for (int i = 0; i < S.nsrc; ++i) {
    if (S.src[i].rowptr) {
      pos[i] = S.src[i].rowptr[row];
      end[i] = S.src[i].rowptr[row + 1];
    } else {
      pos[i] = end[i] = 0;
    }
    diag_done[i] = S.src[i].diag == nullptr;
  }
  int count = 0;
  for (;;) {
    int64_t cmin = INT64_MAX;
    for (int i = 0; i < S.nsrc; ++i) {
      if (pos[i] < end[i]) cmin = min(cmin, (int64_t)S.src[i].colind[pos[i]]);
      if (!diag_done[i]) cmin = min(cmin, row);
    }
    if (cmin == INT64_MAX) break;
    double v[1 + LDQ_MAXP];
    for (int i = 0; i < S.nsrc; ++i) {
      v[i] = 0.0;
      if (pos[i] < end[i] && S.src[i].colind[pos[i]] == cmin) {
        v[i] = S.src[i].val[pos[i]];
        ++pos[i];
      } else if (!diag_done[i] && cmin == row) {
        v[i] = S.src[i].diag[row];
        diag_done[i] = true;
      }
    }
    f((int32_t)cmin, v);
    ++count;
  }
  return count;
}

__global__ void csr_slice_width_kernel(CsrSrcs S, int64_t n, int nslices, int32_t *width) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int len = 0;
  if (row < n) len = union_row(S, row, [](int32_t, const double *) {});
  // slices are aligned to waves: blockDim is a multiple of 64
  for (int off = 32; off >= 1; off >>= 1) len = max(len, __shfl_xor(len, off, 64));
  const int64_t s = row >> 6;
  if ((threadIdx.x & 63) == 0 && s < nslices) width[s] = len;
}

__global__ void csr_slab_fill_kernel(CsrSrcs S, int64_t n, int nslices, const int64_t *sptr, int32_t *col,
                                     double *val, double *g0, double *g1, double *g2, double *g3) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t s = row >> 6;
  if (s >= nslices) return;
  const int lane = (int)(row & 63);
  const int64_t base = sptr[s];
  const int w = (int)((sptr[s + 1] - base) >> 6);
  double *g[LDQ_MAXP] = {g0, g1, g2, g3};
  int k = 0;
  if (row < n) {
    union_row(S, row, [&](int32_t c, const double *v) {
      const int64_t e = base + (int64_t)k * 64 + lane;
      col[e] = c;
      val[e] = v[0];
      for (int i = 1; i < S.nsrc; ++i) g[i - 1][e] = v[i];
      ++k;
    });
  }
  // padding: the row's own index (or row 0 past the end) with zero values
  const int32_t self = row < n ? (int32_t)row : 0;
  for (; k < w; ++k) {
    const int64_t e = base + (int64_t)k * 64 + lane;
    col[e] = self;
    val[e] = 0.0;
    for (int i = 1; i < S.nsrc; ++i) g[i - 1][e] = 0.0;
  }
}

hipError_t launch_csr_slice_width(const CsrSrcs &S, int64_t n, int nslices, int32_t *width, hipStream_t st) {
  const int64_t threads = (int64_t)nslices * 64;
  csr_slice_width_kernel<<<dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st>>>(S, n, nslices, width);
  return hipGetLastError();
}

hipError_t launch_csr_slab_fill(const CsrSrcs &S, int64_t n, int nslices, const int64_t *sptr, int32_t *col,
                                double *val, double *const g[LDQ_MAXP], hipStream_t st) {
  const int64_t threads = (int64_t)nslices * 64;
  csr_slab_fill_kernel<<<dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st>>>(
      S, n, nslices, sptr, col, val, g[0], g[1], g[2], g[3]);
  return hipGetLastError();
}

// ---------------------------------------------------------------- passes

// The wave's slice, kept in registers when W > 0: the byte offset of each
// column in a vector (a gather is a buffer load at that offset from the
// probe's vector), the values of Q and of the derivative operators.  W is the
// slot count rounded up; the slots past the slice width gather element 0
// (one address for the whole wave) and weigh it by 0, so every gather is
// unconditional.  W == 0 re-reads the slice from memory for every probe (any
// width, 64-bit indexing).
template <typename T, int W, int NG>
struct SliceRegs {
  uint32_t off[W > 0 ? W : 1];
  double val[W > 0 ? W : 1];
  double gv[NG > 0 ? NG : 1][W > 0 ? W : 1];
};

struct WaveSlice {
  int s;            // slice
  int lane;
  int64_t row;      // the lane's row (clamped to n - 1 past the end)
  bool valid;
  int64_t off;      // first entry
  int w;            // width
};

template <typename T>
__device__ inline bool wave_slice(const PassCsr<T> &a, WaveSlice *ws) {
  // the wave index is uniform across the wave; say so, so that the slice
  // bounds live in scalar registers and the width tests are scalar branches
  const int wid = __builtin_amdgcn_readfirstlane(xcd_remap(blockIdx.x, gridDim.x) * 4 + (int)(threadIdx.x >> 6));
  if (wid >= a.nslices) return false;
  ws->s = wid;
  ws->lane = threadIdx.x & 63;
  const int64_t row = (int64_t)wid * 64 + ws->lane;
  ws->valid = row < a.n;
  ws->row = ws->valid ? row : a.n - 1;
  ws->off = a.sptr[wid];
  ws->w = (int)((a.sptr[wid + 1] - ws->off) >> 6);
  return true;
}

template <typename T, int W, int NG>
__device__ inline void load_slice(const PassCsr<T> &a, const WaveSlice &ws, SliceRegs<T, W, NG> &R) {
#pragma unroll
  for (int k = 0; k < W; ++k) {
    if (k < ws.w) {
      const int64_t e = ws.off + (int64_t)k * 64 + ws.lane;
      R.off[k] = (uint32_t)a.col[e] * (uint32_t)sizeof(T);
      R.val[k] = a.val[e];
#pragma unroll
      for (int i = 0; i < NG; ++i) R.gv[i][k] = a.gval[i][e];
    } else {
      R.off[k] = 0;
      R.val[k] = 0.0;
#pragma unroll
      for (int i = 0; i < NG; ++i) R.gv[i][k] = 0.0;
    }
  }
}



// Probe scalars of a chunk of 64 probes: lane l loads those of probe c0 + l
// once; the probe loop takes probe c0 + u from lane u into scalar registers.
struct ProbeChunk {
  int active, colour;
  double alpha, beta;
};

__device__ inline ProbeChunk load_chunk(const ProbeState *st, int c0, int nprobes) {
  ProbeChunk c{0, 0, 0.0, 0.0};
  const int j = c0 + (int)(threadIdx.x & 63);
  if (j < nprobes) {
    c.active = st[j].active;
    c.colour = st[j].colour;
    c.alpha = st[j].alpha;
    c.beta = st[j].beta_prev;
  }
  return c;
}

__device__ inline int lane_int(int v, int u) { return __builtin_amdgcn_readlane(v, u); }
__device__ inline double lane_double(double v, int u) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), u);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), u);
  return __builtin_bit_cast(double, (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Write the wave's sums of q[0..NQ) for probe j to the partials (lane 0).
template <int NQ>
__device__ inline void put_partials(double *part, int nq, int ntiles, int j, int tile, const int *slot,
                                    const double *q) {
  double t[NQ];
#pragma unroll
  for (int i = 0; i < NQ; ++i) t[i] = wave_sum(q[i]);
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int i = 0; i < NQ; ++i) part[((size_t)j * nq + slot[i]) * ntiles + tile] = t[i];
  }
}

// Pass A.  omega_i = (dQ_i v_j)^T p_k is summed as v_j^T (dQ_i p_k): the rows
// of colour j add (dQ_i p_k)_row, formed from the same gathered p_k values as
// (Q p_k)_row.
template <typename T, int W, int NG, bool FIRST>
__global__ __launch_bounds__(256) void csr_pass_a_kernel(PassCsr<T> a) {
  WaveSlice ws;
  if (!wave_slice(a, &ws)) return;
  const int64_t n = a.n;
  SliceRegs<T, W, NG> R;
  int32_t ccol[(FIRST && W > 0) ? W : 1];
  if constexpr (W > 0) {
    load_slice<T, W, NG>(a, ws, R);
    if constexpr (FIRST) {
#pragma unroll
      for (int k = 0; k < W; ++k) ccol[k] = (a.rad || a.uvec) ? 0 : a.colours[R.off[k] / (uint32_t)sizeof(T)];
    }
  }
  const int mycol = (a.rad || a.uvec) ? 0 : a.colours[ws.row];
  // entry of probe j (colour cj) at a row: 0 / 1 for a colour class, -1 / +1
  // for random signs
  auto probe_at = [&](int cj, int64_t row, int colour_of_row) -> double {
    if (a.uvec) return a.uvec[(size_t)cj * a.n + row];
    return a.rad ? rad_sign(a.seed, cj, row) : (colour_of_row == cj ? 1.0 : 0.0);
  };
  constexpr int NQ = 2 + NG;
  int slot[NQ];
  slot[0] = 0;   // gamma'
  slot[1] = 2;   // rho'
#pragma unroll
  for (int i = 0; i < NG; ++i) slot[2 + i] = LDQ_NQ_BASE + i;

  for (int c0 = 0; c0 < a.nprobes; c0 += 64) {
  const ProbeChunk pc = load_chunk(a.st, c0, a.nprobes);
  const int cnt = min(64, a.nprobes - c0);
  for (int u = 0; u < cnt; ++u) {
    if (!lane_int(pc.active, u)) continue;
    const int j = c0 + u;
    const int cj = lane_int(pc.colour, u);
    const double alpha = lane_double(pc.alpha, u);
    const double beta = FIRST ? 0.0 : lane_double(pc.beta, u);
    const size_t base = (size_t)j * n;
    const T *rb = a.r_in + base;
    const T *pb = a.p_in + base;
    double q = 0.0;
    double dq[NG > 0 ? NG : 1];
#pragma unroll
    for (int i = 0; i < NG; ++i) dq[i] = 0.0;
    if constexpr (W > 0) {
      if constexpr (FIRST) {
#pragma unroll
        for (int k = 0; k < W; ++k) {
          const double w = probe_at(cj, R.off[k] / (uint32_t)sizeof(T), ccol[k]);
          if (w != 0.0) {
            q = fma(R.val[k], w, q);
#pragma unroll
            for (int i = 0; i < NG; ++i) dq[i] = fma(R.gv[i][k], w, dq[i]);
          }
        }
      } else {
        const unsigned vbytes = (unsigned)(n * (int64_t)sizeof(T));
        const __amdgpu_buffer_rsrc_t rr = make_rsrc(rb, vbytes), rp = make_rsrc(pb, vbytes);
        T rv[W], pv[W];
#pragma unroll
        for (int k = 0; k < W; ++k) {
          rv[k] = buf_ld((T *)nullptr, rr, R.off[k], 0u);
          pv[k] = buf_ld((T *)nullptr, rp, R.off[k], 0u);
        }
#pragma unroll
        for (int k = 0; k < W; ++k) {
          const double x = fma(beta, (double)pv[k], (double)rv[k]);
          q = fma(R.val[k], x, q);
#pragma unroll
          for (int i = 0; i < NG; ++i) dq[i] = fma(R.gv[i][k], x, dq[i]);
        }
      }
    } else {
      for (int k = 0; k < ws.w; ++k) {
        const int64_t e = ws.off + (int64_t)k * 64 + ws.lane;
        const int32_t c = a.col[e];
        double x;
        if constexpr (FIRST)
          x = probe_at(cj, c, (a.rad || a.uvec) ? 0 : a.colours[c]);
        else
          x = fma(beta, (double)pb[c], (double)rb[c]);
        q = fma(a.val[e], x, q);
#pragma unroll
        for (int i = 0; i < NG; ++i) dq[i] = fma(a.gval[i][e], x, dq[i]);
      }
    }
    const double vown = probe_at(cj, ws.row, mycol);
    const double mine = ws.valid ? vown : 0.0;
    double rown, pown;
    if constexpr (FIRST) {
      rown = vown;
      pown = rown;
    } else {
      rown = (double)rb[ws.row];
      pown = fma(beta, (double)pb[ws.row], rown);
    }
    const double rnew = fma(-alpha, q, rown);
    if (ws.valid) {
      a.r_out[base + ws.row] = (T)rnew;
      a.p_out[base + ws.row] = (T)pown;
    }
    double qs[NQ];
    qs[0] = ws.valid ? rnew * rnew : 0.0;
    qs[1] = mine * rnew;
#pragma unroll
    for (int i = 0; i < NG; ++i) qs[2 + i] = mine * dq[i];
    put_partials<NQ>(a.part, a.nq, a.nslices, j, ws.s, slot, qs);
  }
  }
}

template <typename T, int W, bool INIT>
__global__ __launch_bounds__(256) void csr_pass_b_kernel(PassCsr<T> a) {
  WaveSlice ws;
  if (!wave_slice(a, &ws)) return;
  const int64_t n = a.n;
  SliceRegs<T, W, 0> R;
  int32_t ccol[(INIT && W > 0) ? W : 1];
  if constexpr (W > 0) {
    load_slice<T, W, 0>(a, ws, R);
    if constexpr (INIT) {
#pragma unroll
      for (int k = 0; k < W; ++k) ccol[k] = (a.rad || a.uvec) ? 0 : a.colours[R.off[k] / (uint32_t)sizeof(T)];
    }
  }
  const int mycol = (a.rad || a.uvec) ? 0 : a.colours[ws.row];
  auto probe_at = [&](int cj, int64_t row, int colour_of_row) -> double {
    if (a.uvec) return a.uvec[(size_t)cj * a.n + row];
    return a.rad ? rad_sign(a.seed, cj, row) : (colour_of_row == cj ? 1.0 : 0.0);
  };
  for (int c0 = 0; c0 < a.nprobes; c0 += 64) {
  const ProbeChunk pc = load_chunk(a.st, c0, a.nprobes);
  const int cnt = min(64, a.nprobes - c0);
  for (int u = 0; u < cnt; ++u) {
    if (!lane_int(pc.active, u)) continue;
    const int j = c0 + u;
    const int cj = lane_int(pc.colour, u);
    const size_t base = (size_t)j * n;
    const T *xb = a.r_in + base;
    double s = 0.0;
    if constexpr (W > 0) {
      if constexpr (INIT) {
#pragma unroll
        for (int k = 0; k < W; ++k) s = fma(R.val[k], probe_at(cj, R.off[k] / (uint32_t)sizeof(T), ccol[k]), s);
      } else {
        const __amdgpu_buffer_rsrc_t rx = make_rsrc(xb, (unsigned)(n * (int64_t)sizeof(T)));
        T xv[W];
#pragma unroll
        for (int k = 0; k < W; ++k) xv[k] = buf_ld((T *)nullptr, rx, R.off[k], 0u);
#pragma unroll
        for (int k = 0; k < W; ++k) s = fma(R.val[k], (double)xv[k], s);
      }
    } else {
      for (int k = 0; k < ws.w; ++k) {
        const int64_t e = ws.off + (int64_t)k * 64 + ws.lane;
        const int32_t c = a.col[e];
        const double x = INIT ? probe_at(cj, c, (a.rad || a.uvec) ? 0 : a.colours[c]) : (double)xb[c];
        s = fma(a.val[e], x, s);
      }
    }
    const double xo = INIT ? probe_at(cj, ws.row, mycol) : (double)xb[ws.row];
    if constexpr (INIT) {
      // dots of r_0 = v: |v|^2, v^T Q v, v^T v
      const int slot[3] = {0, 1, 2};
      double qs[3] = {ws.valid ? xo * xo : 0.0, ws.valid ? xo * s : 0.0, ws.valid ? xo * xo : 0.0};
      put_partials<3>(a.part, a.nq, a.nslices, j, ws.s, slot, qs);
    } else {
      const int slot[1] = {1};
      double qs[1] = {ws.valid ? xo * s : 0.0};
      put_partials<1>(a.part, a.nq, a.nslices, j, ws.s, slot, qs);
    }
  }
  }
}

// One workgroup of CSR_TAIL_W waves per probe: reduce the partials of passes
// A and B (one per 64-row slice: thousands per probe, so the reduction is
// spread over the workgroup, in a fixed order), advance the base CG scalars,
// every shift and the gradient sums (state updated in place).
constexpr int CSR_TAIL_W = 16;
__global__ __launch_bounds__(64 * CSR_TAIL_W) void csr_tail_kernel(TailArgs ta, int ntiles, int mode) {
  (void)pass_prologue<CSR_TAIL_W>(ta, probe_ref(ta, blockIdx.x, ntiles), 0, ntiles, mode);
}

static unsigned csr_grid(int nslices) { return (unsigned)((nslices + 3) / 4); }

template <typename T, int W, int NG>
static void pass_a_ng(const PassCsr<T> &a, bool first, dim3 g, dim3 b, hipStream_t st) {
  // 32 register slots leave no room for more than one derivative operator
  constexpr int WW = (W == 32 && NG > 1) ? 0 : W;
  if (first)
    csr_pass_a_kernel<T, WW, NG, true><<<g, b, 0, st>>>(a);
  else
    csr_pass_a_kernel<T, WW, NG, false><<<g, b, 0, st>>>(a);
}

template <typename T, int W>
static hipError_t pass_a_w(const PassCsr<T> &a, bool first, hipStream_t st) {
  const dim3 g(csr_grid(a.nslices)), b(256);
  switch (a.ngrad) {
    case 0: pass_a_ng<T, W, 0>(a, first, g, b, st); break;
    case 1: pass_a_ng<T, W, 1>(a, first, g, b, st); break;
    case 2: pass_a_ng<T, W, 2>(a, first, g, b, st); break;
    case 3: pass_a_ng<T, W, 3>(a, first, g, b, st); break;
    case 4: pass_a_ng<T, W, 4>(a, first, g, b, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, int W>
static hipError_t pass_b_w(const PassCsr<T> &a, bool init, hipStream_t st) {
  const dim3 g(csr_grid(a.nslices)), b(256);
  if (init)
    csr_pass_b_kernel<T, W, true><<<g, b, 0, st>>>(a);
  else
    csr_pass_b_kernel<T, W, false><<<g, b, 0, st>>>(a);
  return hipGetLastError();
}

// Register width for a slab whose widest slice has `maxw` slots (0: re-read
// from memory; also when byte offsets into a vector overflow 32 bits).
int csr_register_width(int maxw, int64_t n, int elem) {
  if ((double)n * elem >= 4294967296.0) return 0;
  if (maxw <= 8) return 8;
  if (maxw <= 16) return 16;
  if (maxw <= 32) return 32;
  return 0;
}

template <typename T>
hipError_t launch_csr_pass_a(const PassCsr<T> &a, int W, bool first, hipStream_t st) {
  switch (W) {
    case 8: return pass_a_w<T, 8>(a, first, st);
    case 16: return pass_a_w<T, 16>(a, first, st);
    case 32: return pass_a_w<T, 32>(a, first, st);
    default: return pass_a_w<T, 0>(a, first, st);
  }
}

template <typename T>
hipError_t launch_csr_pass_b(const PassCsr<T> &a, int W, bool init, hipStream_t st) {
  switch (W) {
    case 8: return pass_b_w<T, 8>(a, init, st);
    case 16: return pass_b_w<T, 16>(a, init, st);
    case 32: return pass_b_w<T, 32>(a, init, st);
    default: return pass_b_w<T, 0>(a, init, st);
  }
}

hipError_t launch_csr_tail(const TailArgs &ta, int nprobes, int ntiles, int mode, hipStream_t st) {
  if (nprobes <= 0) return hipSuccess;
  csr_tail_kernel<<<dim3(nprobes), dim3(64 * CSR_TAIL_W), 0, st>>>(ta, ntiles, mode);
  return hipGetLastError();
}

template hipError_t launch_csr_pass_a<float>(const PassCsr<float> &, int, bool, hipStream_t);
template hipError_t launch_csr_pass_a<double>(const PassCsr<double> &, int, bool, hipStream_t);
template hipError_t launch_csr_pass_b<float>(const PassCsr<float> &, int, bool, hipStream_t);
template hipError_t launch_csr_pass_b<double>(const PassCsr<double> &, int, bool, hipStream_t);

}  // namespace ldq
