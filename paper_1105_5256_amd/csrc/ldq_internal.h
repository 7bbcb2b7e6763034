// Internal types shared by the host driver and the HIP kernels of libldq.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define LDQ_MAXP 4          // derivative operators per call
#define LDQ_MAXN 64         // shifts per call (one wave64 lane per shift)
#define LDQ_BLOCK 256       // threads per workgroup of the pass kernels
#ifndef LDQ_ROWS2D
#define LDQ_ROWS2D 32      // rows per wave tile of the 2-D pass (rounded up so that rows + 2R + 2 is a multiple of 5)
#endif
#define LDQ_ROWS2D_TALL 64  // rows of the tall tile of the FP32 fast 2-D passes (rounded up the same way)
#define LDQ_NQ_BASE 3       // reduced quantities of a pass: gamma, delta, rho (+ one omega per parameter)

namespace ldq {

// ---------------------------------------------------------------- complex FP64
struct cplx {
  double re, im;
};
__host__ __device__ inline cplx cmk(double r, double i) { return cplx{r, i}; }
__host__ __device__ inline cplx cadd(cplx a, cplx b) { return cplx{a.re + b.re, a.im + b.im}; }
__host__ __device__ inline cplx csub(cplx a, cplx b) { return cplx{a.re - b.re, a.im - b.im}; }
__host__ __device__ inline cplx cmul(cplx a, cplx b) {
  return cplx{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__host__ __device__ inline cplx cscale(cplx a, double s) { return cplx{a.re * s, a.im * s}; }
__host__ __device__ inline cplx cdiv(cplx a, cplx b) {
  // Smith's algorithm: avoids overflow of |b|^2 for large or tiny b
  if (fabs(b.re) >= fabs(b.im)) {
    double r = b.im / b.re, d = b.re + b.im * r;
    return cplx{(a.re + a.im * r) / d, (a.im - a.re * r) / d};
  } else {
    double r = b.re / b.im, d = b.re * r + b.im;
    return cplx{(a.re * r + a.im) / d, (a.im * r - a.re) / d};
  }
}
__host__ __device__ inline double cabs2(cplx a) { return a.re * a.re + a.im * a.im; }

// ------------------------------------------------------------ per-probe state
// Scalars of the base CG recurrence of one probe (all FP64).  Iteration k of a
// pass uses alpha = alpha_k and beta_prev = beta_{k-1}; gamma = r_k . r_k.
struct ProbeState {
  double gamma;
  double alpha;
  double alpha_prev;
  double beta_prev;
  double vnorm2;
  double grad[LDQ_MAXP];
  int iter;
  int active;
  int status;   // ldq_status of this probe (0 while fine)
  int colour;   // colour class this probe indicates
};

// Per (probe, shift) state of the multi-shift recurrence.
struct ShiftState {
  cplx zeta, zeta_prev, phi, psi;
  int frozen;
  int pad;
};

// Derivative-operator term applied inside a pass (gradient dot products).
enum GradKind { GK_DIAG = 1, GK_SHIFTED = 2, GK_OBS = 3 };

template <typename T>
struct GradTerm {
  int kind;
  double scale;
  double kappa2;          // GK_SHIFTED with a constant shift
  const T *field;         // GK_DIAG: d[n]; GK_SHIFTED: kappa2 field or null
  const T *obs;           // GK_OBS: 9 x n coefficient planes
};

// Shared tail arguments (reduction + multi-shift recurrences).  Launch g of the
// pass kernel reads the probe states and dot-product partials written by
// launch g - 1 (st_in, part_in) and writes its own (st_out, part_out); the
// host swaps the two buffers between launches, so no workgroup ever waits
// for another one inside a launch.
struct TailArgs {
  const double *part_in;   // [probe][nq][tile] of the previous launch
  double *part_out;        // [probe][nq][tile] of this launch
  const ProbeState *st_in; // [probe] state before this launch
  ProbeState *st_out;      // [probe] state after this launch (written by tile 0)
  ShiftState *sh;          // [probe][nshifts] (read and written by tile 0 only)
  const cplx *sigma;       // [nshifts]
  int nshifts;
  int ngrad;
  double tol2;             // tol^2
  double grad_tol2;        // grad_tol^2
  int max_iter;
  int *active_count;       // probes still iterating (decremented once per finished probe)
  int need_base;           // the base system must reach grad_tol (gradients, enclosure estimate)
  int hist_cap;            // Lanczos coefficients kept per probe (0: none)
  double *hist;            // [probe][hist_cap][2]: (alpha_i, beta_{i-1}) of iteration i
};

enum PassMode { MODE_INIT = 0, MODE_FIRST = 1, MODE_STEP = 2 };

// 2-D lattice pass.
// Entry `site` of random-sign probe j (Sec. 2.1, eq. (6): +1 or -1 with
// probability 1/2, independently): the sign of the top bit of output number
// j * 2^32 + site + 1 of the SplitMix64 generator started from `seed`
// (Steele, Lea and Flood, OOPSLA 2014): z = seed + count * 0x9E3779B97F4A7C15,
// then the generator's output mix of z.  Clear bit: +1.
__host__ __device__ inline double rad_sign(uint64_t seed, int j, int64_t site) {
  uint64_t z = seed + (((uint64_t)(uint32_t)j << 32) + (uint64_t)site + 1u) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (z >> 63) ? -1.0 : 1.0;
}

template <typename T>
struct Pass2D {
  int nx, ny;
  int tiles_x, ntiles;
  int rows;                 // lattice rows per wave tile
  int nprobes;
  // colouring: modular (C > 0) or array; or random signs (rad: probe j has
  // entry rad_sign(seed, j, site) at every site)
  int colC, cola;
  const int32_t *colours;
  int rad;
  uint64_t seed;
  const uint64_t *rmask;    // random signs for the specialised pass: the launch's
                            // probes' strip masks in probe order (rad_masks)
  const double *uvec;       // or given probe vectors, probe-major [probe][n] (FP64)
  // operator
  double kappa2;            // constant shift (SQUARED and unfielded SHIFTED)
  const T *kappa2_field;    // SHIFTED with a field
  double scale;             // operator scale
  double tau;               // observation weight (0: none)
  const T *obs;             // 9 x n planes of A^T A
  GradTerm<T> grad[LDQ_MAXP];
  // vectors, probe-major [probe][n]
  const T *r_in, *p_in;
  T *r_out, *p_out;
  int mode;
  TailArgs tail;
};

// 3-D lattice pass (7-point shifted Laplacian, z marched inside a workgroup).
template <typename T>
struct Pass3D {
  int nx, ny, nz;
  int tiles_x, tiles_y, zseg, nzseg, ntiles;
  int nprobes;
  int colC, cola, colb;
  const int32_t *colours;
  int rad;                  // random-sign probes (as in Pass2D)
  uint64_t seed;
  const double *uvec;       // given probe vectors (as in Pass2D)
  double kappa2;
  const T *kappa2_field;
  double scale;
  GradTerm<T> grad[LDQ_MAXP];
  const T *r_in, *p_in;
  T *r_out, *p_out;
  int mode;
  TailArgs tail;
};

// Many independent 2-D lattices advanced together: every STEP launch covers
// the (field, probe, tile) entries of a work list that holds the tiles of the
// probes still iterating.  Field f's probes are items item_base .. item_base
// + nprobes - 1 (probe states, shift states, history), its vectors start at
// element vec_off of each vector buffer (probe j at vec_off + j n) and its
// partials at part_off of each partial buffer (probe j at part_off + j nq
// ntiles).
struct FieldDesc {
  int nx, ny, tiles_x, ntiles;
  int nprobes, item_base;
  int64_t vec_off, part_off;
  double kappa2;        // Q = (kappa2 I + L)^p
  double kd;            // derivative: gscale (kd I + L)
};

struct WorkItem {
  int field, probe, tile, pad;
};

template <typename T>
struct Batch2D {
  const WorkItem *work;
  const int *count;     // live length of the work list (device; the grid may be longer)
  const FieldDesc *fields;
  const cplx *sigma;    // [field][LDQ_MAXN]
  int rows, colC, cola;
  double gscale;
  const T *r_in, *p_in;
  T *r_out, *p_out;
  TailArgs tail;        // part_in/part_out/st_in/st_out/sh/hist are the buffer bases
};

// General sparse operator.  The rows are cut into slices of 64 (one wave
// each); slice s stores its entries column-major, entry k of row 64 s + l at
// sptr[s] + 64 k + l, for k below the slice width (sptr[s+1] - sptr[s]) / 64.
// The pattern is the union of the patterns of Q and of the derivative
// operators, so val and gval[i] share the slots (zero where an operator has
// no entry).  One iteration is pass A (p_k formed on the fly, r_{k+1} =
// r_k - alpha_k Q p_k, dots gamma', rho', omega_i), pass B (delta' =
// r_{k+1}^T Q r_{k+1}) and the per-probe tail launch.
template <typename T>
struct PassCsr {
  int64_t n;
  int nslices;                  // also the tiles of the partials
  int nprobes;
  int ngrad;
  int nq;
  const int64_t *sptr;
  const int32_t *col;
  const double *val;            // operator values stay FP64 in both precisions
  const double *gval[LDQ_MAXP];
  const int32_t *colours;
  int rad;                      // random-sign probes (rad_sign(seed, j, row)); colours unused
  uint64_t seed;
  const double *uvec;           // given probe vectors [probe][n] (FP64); colours unused
  const ProbeState *st;
  const T *r_in, *p_in;
  T *r_out, *p_out;
  double *part;                 // [probe][nq][slice]
};

}  // namespace ldq
