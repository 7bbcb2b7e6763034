// Small kernels around the Krylov passes: probe-state initialisation, the
// final reduction of the estimator, the contour-quadrature shifts, modular
// colour fills, deterministic min/max/Gershgorin reductions and precision
// conversion.
#include "ldq_internal.h"

namespace ldq {

// ------------------------------------------------------------ probe states
__global__ void init_probes_kernel(ProbeState *st, int nprobes, const int32_t *classes, int *active_count) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < nprobes) {
    ProbeState ps = {};
    ps.active = 1;
    ps.colour = classes[j];
    st[j] = ps;
  }
  if (j == 0) *active_count = nprobes;
}

hipError_t launch_init_probes(ProbeState *st, int nprobes, const int32_t *classes, int *active_count,
                              hipStream_t s) {
  hipLaunchKernelGGL(init_probes_kernel, dim3((nprobes + 255) / 256), dim3(256), 0, s, st, nprobes, classes,
                     active_count);
  return hipGetLastError();
}

// --------------------------------------------------------------- finaliser
// terms[(first + j) * (1 + ngrad) + 0] = Im sum_l c_l psi_jl and + 1 + i = G_ij
// for the probes of one block; status/iteration summaries go to stats.
__global__ void probe_terms_kernel(const ProbeState *st, const ShiftState *sh, const cplx *coef, int nprobes,
                                   int nshifts, int ngrad, double *terms, int first, int *stats) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nprobes) return;
  const ShiftState *s = sh + (size_t)j * nshifts;
  double t = 0.0;
  for (int l = 0; l < nshifts; ++l) t += coef[l].re * s[l].psi.im + coef[l].im * s[l].psi.re;
  double *dst = terms + (size_t)(first + j) * (1 + ngrad);
  dst[0] = t;
  for (int i = 0; i < ngrad; ++i) dst[1 + i] = st[j].grad[i];
  // stats: [0] worst status, [1] max iterations, [2..3] total iterations
  // (64-bit), [6..7] max final ||r|| / ||v|| (a non-negative double: its bit
  // pattern orders like the value)
  atomicMax(stats + 0, st[j].status);
  atomicMax(stats + 1, st[j].iter);
  atomicAdd((unsigned long long *)(stats + 2), (unsigned long long)st[j].iter);
  const double res = st[j].vnorm2 > 0.0 ? sqrt(fmax(st[j].gamma, 0.0) / st[j].vnorm2) : 0.0;
  atomicMax((unsigned long long *)(stats + 6), (unsigned long long)__double_as_longlong(res));
}

// Enclosure check: the CG coefficients of a probe define its Lanczos
// tridiagonal matrix T (diagonal 1/alpha_i + beta_{i-1}/alpha_{i-1},
// off-diagonal squared beta_{i-1}/alpha_{i-1}^2), whose eigenvalues lie in the
// spectrum of Q up to rounding.  Sturm sequences (LDL^T pivots of T - lo I and
// hi I - T) count its eigenvalues below lo and above hi; stats[4] receives the
// number of probes with any.
__global__ void lanczos_check_kernel(const double *hist, const ProbeState *st, int nprobes, int cap, double lo,
                                     double hi, int *stats) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nprobes) return;
  const int K = min(st[j].active ? st[j].iter + 1 : st[j].iter, cap);
  const double *h = hist + (size_t)j * cap * 2;
  double dl = 1.0, dh = 1.0, aprev = 1.0;
  int below = 0, above = 0;
  for (int i = 0; i < K; ++i) {
    const double al = h[2 * i], be = h[2 * i + 1];
    double diag = 1.0 / al, off2 = 0.0;
    if (i > 0) {
      diag += be / aprev;
      off2 = be / (aprev * aprev);
    }
    dl = (diag - lo) - (i > 0 ? off2 / dl : 0.0);
    dh = (hi - diag) - (i > 0 ? off2 / dh : 0.0);
    if (dl == 0.0) dl = -1e-300;
    if (dh == 0.0) dh = -1e-300;
    below += dl < 0.0;
    above += dh < 0.0;
    aprev = al;
  }
  if (below + above > 0) atomicAdd(stats + 4, 1);
}

// The same check for the probes of many fields in one launch: item j
// belongs to field item_field[j], whose interval is lohi[2 f], lohi[2 f + 1]
// and whose count is stats[8 f + 4].
__global__ void batch_lanczos_check_kernel(const double *hist, const ProbeState *st, int nitems, int cap,
                                           const int32_t *item_field, const double *lohi, int *stats) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nitems) return;
  const int f = item_field[j];
  const double lo = lohi[2 * f], hi = lohi[2 * f + 1];
  const int K = min(st[j].active ? st[j].iter + 1 : st[j].iter, cap);
  const double *h = hist + (size_t)j * cap * 2;
  double dl = 1.0, dh = 1.0, aprev = 1.0;
  int below = 0, above = 0;
  for (int i = 0; i < K; ++i) {
    const double al = h[2 * i], be = h[2 * i + 1];
    double diag = 1.0 / al, off2 = 0.0;
    if (i > 0) {
      diag += be / aprev;
      off2 = be / (aprev * aprev);
    }
    dl = (diag - lo) - (i > 0 ? off2 / dl : 0.0);
    dh = (hi - diag) - (i > 0 ? off2 / dh : 0.0);
    if (dl == 0.0) dl = -1e-300;
    if (dh == 0.0) dh = -1e-300;
    below += dl < 0.0;
    above += dh < 0.0;
    aprev = al;
  }
  if (below + above > 0) atomicAdd(stats + 8 * f + 4, 1);
}

hipError_t launch_batch_lanczos_check(const double *hist, const ProbeState *st, int nitems, int cap,
                                      const int32_t *item_field, const double *lohi, int *stats, hipStream_t s) {
  if (cap <= 0 || nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(batch_lanczos_check_kernel, dim3((nitems + 63) / 64), dim3(64), 0, s, hist, st, nitems, cap,
                     item_field, lohi, stats);
  return hipGetLastError();
}

hipError_t launch_lanczos_check(const double *hist, const ProbeState *st, int nprobes, int cap, double lo, double hi,
                                int *stats, hipStream_t s) {
  if (cap <= 0 || nprobes <= 0) return hipSuccess;
  hipLaunchKernelGGL(lanczos_check_kernel, dim3((nprobes + 255) / 256), dim3(256), 0, s, hist, st, nprobes, cap, lo,
                     hi, stats);
  return hipGetLastError();
}

hipError_t launch_probe_terms(const ProbeState *st, const ShiftState *sh, const cplx *coef, int nprobes,
                              int nshifts, int ngrad, double *terms, int first, int *stats, hipStream_t s) {
  hipLaunchKernelGGL(probe_terms_kernel, dim3((nprobes + 255) / 256), dim3(256), 0, s, st, sh, coef, nprobes,
                     nshifts, ngrad, terms, first, stats);
  return hipGetLastError();
}

// Sum the per-probe terms in a fixed order: out[c] = sum_j terms[j * ncol + c].
__global__ void sum_terms_kernel(const double *terms, int nprobes, int ncol, double *out) {
  __shared__ double red[256];
  for (int c = 0; c < ncol; ++c) {
    double acc = 0.0;
    for (int j = threadIdx.x; j < nprobes; j += 256) acc += terms[(size_t)j * ncol + c];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
      if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = red[0];
    __syncthreads();
  }
}

hipError_t launch_sum_terms(const double *terms, int nprobes, int ncol, double *out, hipStream_t s) {
  hipLaunchKernelGGL(sum_terms_kernel, dim3(1), dim3(256), 0, s, terms, nprobes, ncol, out);
  return hipGetLastError();
}

// ------------------------------------------------------------------ shifts
// Complete elliptic integral K(k) = pi / (2 AGM(1, sqrt(1 - k^2))).
__device__ double ellip_k(double k) {
  double a = 1.0, b = sqrt((1.0 - k) * (1.0 + k));
  for (int i = 0; i < 40 && fabs(a - b) > 1e-16 * a; ++i) {
    const double an = 0.5 * (a + b);
    b = sqrt(a * b);
    a = an;
  }
  return M_PI / (2.0 * a);
}

// Jacobi sn, cn, dn of a real argument u for parameter m = k^2 by the
// arithmetic-geometric mean and descending Landen transformation
// (Abramowitz & Stegun 16.4).
__device__ void ellip_j(double u, double m, double *sn, double *cn, double *dn) {
  double a[32], c[32];
  a[0] = 1.0;
  double b = sqrt(1.0 - m);
  c[0] = sqrt(m);
  int nst = 0;
  while (nst < 30 && fabs(c[nst]) > 1e-17) {
    const double an = 0.5 * (a[nst] + b);
    c[nst + 1] = 0.5 * (a[nst] - b);
    b = sqrt(a[nst] * b);
    a[nst + 1] = an;
    ++nst;
  }
  double phi = ldexp(a[nst] * u, nst);
  double phi_prev = phi;
  for (int i = nst; i >= 1; --i) {
    phi_prev = phi;
    phi = 0.5 * (phi + asin(c[i] / a[i] * sin(phi)));
  }
  *sn = sin(phi);
  *cn = cos(phi);
  *dn = (nst == 0) ? 1.0 : cos(phi) / cos(phi_prev - phi);
}

// sigma_l = w_l^2 and c_l = (2K / (pi N)) 4 w_l log(w_l) w'(t_l), with
// w(t) = sqrt(m M)^{1/2} (1/k + sn t) / (1/k - sn t) on the conformal map of
// the square-root spectrum [sqrt m, sqrt M] and midpoint nodes
// t_l = -K + i K'/2 + (l - 1/2) 2K / N (eq. (7); Hale, Higham & Trefethen).
__global__ void shifts_kernel(double lmin, double lmax, int N, cplx *sigma, cplx *coef) {
  const int l = threadIdx.x;
  if (l >= N) return;
  // a near-degenerate enclosure makes the modulus of the map vanish and the
  // elliptic functions lose digits; any wider interval still encloses the spectrum
  lmax = fmax(lmax, 1.01 * lmin);
  const double r = sqrt(sqrt(lmax / lmin));
  const double c0 = sqrt(sqrt(lmin * lmax));
  const double k = (r - 1.0) / (r + 1.0);
  const double m = k * k;
  const double K = ellip_k(k);
  const double Kp = ellip_k(sqrt((1.0 - k) * (1.0 + k)));
  const double x = -K + (l + 0.5) * 2.0 * K / N;
  const double y = 0.5 * Kp;
  double s, c, d, s1, c1, d1;
  ellip_j(x, m, &s, &c, &d);
  ellip_j(y, 1.0 - m, &s1, &c1, &d1);
  const double den = c1 * c1 + m * s * s * s1 * s1;
  const cplx sn = cmk(s * d1 / den, c * d * s1 * c1 / den);
  const cplx cn = cmk(c * c1 / den, -s * d * s1 * d1 / den);
  const cplx dn = cmk(d * c1 * d1 / den, -m * s * c * s1 / den);
  const double ik = 1.0 / k;
  const cplx num = cmk(ik + sn.re, sn.im), dnm = cmk(ik - sn.re, -sn.im);
  const cplx w = cscale(cdiv(num, dnm), c0);
  const cplx dw = cscale(cdiv(cmul(cn, dn), cmul(dnm, dnm)), c0 * 2.0 * ik);
  const cplx logw = cmk(0.5 * log(cabs2(w)), atan2(w.im, w.re));
  sigma[l] = cmul(w, w);
  coef[l] = cscale(cmul(cmul(w, logw), dw), (2.0 * K / (M_PI * N)) * 4.0);
}

hipError_t launch_shifts(double lmin, double lmax, int N, cplx *sigma, cplx *coef, hipStream_t s) {
  hipLaunchKernelGGL(shifts_kernel, dim3(1), dim3(64), 0, s, lmin, lmax, N, sigma, coef);
  return hipGetLastError();
}

// ------------------------------------------------------- modular colouring
__global__ void modular_fill_kernel(int32_t *col, int nx, int ny, int nz, int C, int a, int b) {
  const size_t n = (size_t)nx * ny * nz;
  for (size_t s = (size_t)blockIdx.x * blockDim.x + threadIdx.x; s < n; s += (size_t)gridDim.x * blockDim.x) {
    const int x = (int)(s % nx);
    const size_t t = s / nx;
    const int y = (int)(t % ny), z = (int)(t / ny);
    col[s] = (int32_t)(((int64_t)x + (int64_t)a * y + (int64_t)b * z) % C);
  }
}

hipError_t launch_modular_fill(int32_t *col, int nx, int ny, int nz, int C, int a, int b, hipStream_t s) {
  const size_t n = (size_t)nx * ny * nz;
  const int blocks = (int)std::min<size_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(modular_fill_kernel, dim3(blocks), dim3(256), 0, s, col, nx, ny, nz, C, a, b);
  return hipGetLastError();
}

// Count of sites per colour (integer atomics: order-independent).  Up to
// 4096 colours are counted in a per-workgroup LDS histogram first, so the
// global counters see one atomic per colour and workgroup.
constexpr int LDQ_HIST = 4096;
__global__ void class_count_kernel(const int32_t *col, size_t n, int C, int *count) {
  __shared__ int hist[LDQ_HIST];
  const bool local = C <= LDQ_HIST;
  if (local)
    for (int c = threadIdx.x; c < C; c += blockDim.x) hist[c] = 0;
  __syncthreads();
  for (size_t s = (size_t)blockIdx.x * blockDim.x + threadIdx.x; s < n; s += (size_t)gridDim.x * blockDim.x) {
    const int c = col[s];
    if (c >= 0 && c < C) atomicAdd(local ? hist + c : count + c, 1);
  }
  __syncthreads();
  if (local)
    for (int c = threadIdx.x; c < C; c += blockDim.x)
      if (hist[c]) atomicAdd(count + c, hist[c]);
}

hipError_t launch_class_count(const int32_t *col, size_t n, int C, int *count, hipStream_t s) {
  const int blocks = (int)std::min<size_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(class_count_kernel, dim3(blocks), dim3(256), 0, s, col, n, C, count);
  return hipGetLastError();
}

// Max colour value (for user colour arrays); -1 marks an invalid (negative) colour.
__global__ void colour_max_kernel(const int32_t *col, size_t n, int *out) {
  int m = -1;
  bool neg = false;
  for (size_t s = (size_t)blockIdx.x * blockDim.x + threadIdx.x; s < n; s += (size_t)gridDim.x * blockDim.x) {
    m = max(m, col[s]);
    neg |= col[s] < 0;
  }
  atomicMax(out, m);
  if (neg) atomicMax(out + 1, 1);
}

hipError_t launch_colour_max(const int32_t *col, size_t n, int *out, hipStream_t s) {
  const int blocks = (int)std::min<size_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(colour_max_kernel, dim3(blocks), dim3(256), 0, s, col, n, out);
  return hipGetLastError();
}

// ------------------------------------------------ min / max of a field (FP64)
// Two-stage deterministic reduction: min and max are order independent.
__global__ void minmax_kernel(const double *v, size_t n, double *out) {
  __shared__ double smin[256], smax[256];
  double lo = INFINITY, hi = -INFINITY;
  for (size_t s = (size_t)blockIdx.x * blockDim.x + threadIdx.x; s < n; s += (size_t)gridDim.x * blockDim.x) {
    lo = fmin(lo, v[s]);
    hi = fmax(hi, v[s]);
  }
  smin[threadIdx.x] = lo;
  smax[threadIdx.x] = hi;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (threadIdx.x < w) {
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + w]);
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[2 * blockIdx.x] = smin[0];
    out[2 * blockIdx.x + 1] = smax[0];
  }
}

// Gershgorin row sums of a CSR matrix: rowsum[i] = sum_j |a_ij| (scaled), reduced by minmax.
__global__ void csr_abs_rowsum_kernel(const int32_t *rowptr, const double *val, int64_t n, double *rowsum) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) s += fabs(val[e]);
    rowsum[i] = s;
  }
}

hipError_t launch_minmax(const double *v, size_t n, double *partial /* 2 * 256 */, hipStream_t s) {
  hipLaunchKernelGGL(minmax_kernel, dim3(256), dim3(256), 0, s, v, n, partial);
  return hipGetLastError();
}

hipError_t launch_csr_abs_rowsum(const int32_t *rowptr, const double *val, int64_t n, double *rowsum,
                                 hipStream_t s) {
  const int blocks = (int)std::min<int64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(csr_abs_rowsum_kernel, dim3(blocks), dim3(256), 0, s, rowptr, val, n, rowsum);
  return hipGetLastError();
}

// ------------------------------------------------------------- conversion
__global__ void to_float_kernel(const double *src, float *dst, size_t n) {
  for (size_t s = (size_t)blockIdx.x * blockDim.x + threadIdx.x; s < n; s += (size_t)gridDim.x * blockDim.x)
    dst[s] = (float)src[s];
}

hipError_t launch_to_float(const double *src, float *dst, size_t n, hipStream_t s) {
  const int blocks = (int)std::min<size_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(to_float_kernel, dim3(blocks), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

}  // namespace ldq

namespace ldq {
// y[j][i] (= or +=) w[j][m] x[j][i] over nb vectors of n entries (the
// accumulation of f_N(Q) v = sum_m w_m r_m from the Krylov residuals).
template <typename S>
__global__ void mat_accum_kernel(const S *x, const double *w, int wstride, int m, int nb, int64_t n, double *y,
                                 int init) {
  const size_t total = (size_t)nb * (size_t)n;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
    const int j = (int)(t / (size_t)n);
    const double c = w[(size_t)j * wstride + m];
    y[t] = (init ? 0.0 : y[t]) + c * (double)x[t];
  }
}

template <typename S>
hipError_t launch_mat_accum(const S *x, const double *w, int wstride, int m, int nb, int64_t n, double *y, bool init,
                            hipStream_t s) {
  const size_t total = (size_t)nb * (size_t)n;
  if (total == 0) return hipSuccess;
  const int blocks = (int)std::min<size_t>((total + 255) / 256, 8192);
  hipLaunchKernelGGL(mat_accum_kernel<S>, dim3(blocks), dim3(256), 0, s, x, w, wstride, m, nb, n, y, init ? 1 : 0);
  return hipGetLastError();
}
template hipError_t launch_mat_accum<float>(const float *, const double *, int, int, int, int64_t, double *, bool,
                                            hipStream_t);
template hipError_t launch_mat_accum<double>(const double *, const double *, int, int, int, int64_t, double *, bool,
                                             hipStream_t);
}  // namespace ldq

namespace ldq {
// z[j][l][i] (= or +=) c[j][m][l] x[j][i] for the N shifts l: the shifted
// solutions x^l_j = sum_m c[j][m][l] r_m of probe j, accumulated from its
// residuals (complex coefficients, complex vectors [probe][shift][n]).
template <typename S>
__global__ void mat_accum_shifts_kernel(const S *x, const cplx *c, int cstride, int m, int N, int nb, int64_t n,
                                        cplx *z, int init) {
  const size_t total = (size_t)nb * (size_t)n;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
    const int j = (int)(t / (size_t)n);
    const size_t i = t - (size_t)j * (size_t)n;
    const double xv = (double)x[t];
    const cplx *cj = c + (size_t)j * cstride + (size_t)m * N;
    cplx *zj = z + (size_t)j * N * (size_t)n + i;
    for (int l = 0; l < N; ++l) {
      cplx acc = init ? cmk(0.0, 0.0) : zj[(size_t)l * n];
      acc.re += cj[l].re * xv;
      acc.im += cj[l].im * xv;
      zj[(size_t)l * n] = acc;
    }
  }
}

template <typename S>
hipError_t launch_mat_accum_shifts(const S *x, const cplx *c, int cstride, int m, int N, int nb, int64_t n, cplx *z,
                                   bool init, hipStream_t s) {
  const size_t total = (size_t)nb * (size_t)n;
  if (total == 0) return hipSuccess;
  const int blocks = (int)std::min<size_t>((total + 255) / 256, 8192);
  hipLaunchKernelGGL(mat_accum_shifts_kernel<S>, dim3(blocks), dim3(256), 0, s, x, c, cstride, m, N, nb, n, z,
                     init ? 1 : 0);
  return hipGetLastError();
}
template hipError_t launch_mat_accum_shifts<float>(const float *, const cplx *, int, int, int, int, int64_t, cplx *,
                                                   bool, hipStream_t);
template hipError_t launch_mat_accum_shifts<double>(const double *, const cplx *, int, int, int, int, int64_t, cplx *,
                                                    bool, hipStream_t);

// out[v] = z_v^T dQ z_v (complex bilinear, no conjugation) for the vectors
// v = 0 .. nv - 1 of z (n entries each) and a lattice derivative operator:
// diag (scale * d) or scale * (kd I + L) with Dirichlet L on nx x ny x nz.
// One workgroup per vector; the workgroup's sum is taken in a fixed order.
__global__ void lattice_bilinear_kernel(const cplx *z, int nx, int ny, int nz, int diag, double scale, double kd,
                                        const double *field, const double *planes, cplx *out) {
  const int64_t n = (int64_t)nx * ny * nz;
  const cplx *zz = z + (size_t)blockIdx.x * (size_t)n;
  const int dim = nz > 1 ? 3 : 2;
  double re = 0.0, im = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    const cplx zi = zz[i];
    double sr, si;
    if (planes) {
      // observation gram A^T A (2-D): plane (dy + 1) 3 + (dx + 1) at site i
      // holds the entry from i to i + dx + nx dy
      const int64_t x = i % nx, y = i / nx;
      double nr = 0.0, ni = 0.0;
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          if (x + dx < 0 || x + dx >= nx || y + dy < 0 || y + dy >= ny) continue;
          const double w = planes[(size_t)((dy + 1) * 3 + (dx + 1)) * (size_t)n + i];
          const cplx zo = zz[i + dx + (int64_t)nx * dy];
          nr += w * zo.re;
          ni += w * zo.im;
        }
      sr = scale * nr;
      si = scale * ni;
    } else if (diag) {
      sr = scale * field[i] * zi.re;
      si = scale * field[i] * zi.im;
    } else {
      const int64_t x = i % nx, y = (i / nx) % ny, zc = i / ((int64_t)nx * ny);
      const double k = field ? field[i] : kd;
      double nr = 0.0, ni = 0.0;
      auto add = [&](int64_t o) { nr += zz[o].re; ni += zz[o].im; };
      if (x > 0) add(i - 1);
      if (x + 1 < nx) add(i + 1);
      if (y > 0) add(i - nx);
      if (y + 1 < ny) add(i + nx);
      if (dim == 3) {
        if (zc > 0) add(i - (int64_t)nx * ny);
        if (zc + 1 < nz) add(i + (int64_t)nx * ny);
      }
      sr = scale * ((k + 2.0 * dim) * zi.re - nr);
      si = scale * ((k + 2.0 * dim) * zi.im - ni);
    }
    re += zi.re * sr - zi.im * si;
    im += zi.re * si + zi.im * sr;
  }
  __shared__ double sre[256], sim[256];
  sre[threadIdx.x] = re;
  sim[threadIdx.x] = im;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sre[threadIdx.x] += sre[threadIdx.x + w];
      sim[threadIdx.x] += sim[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = cmk(sre[0], sim[0]);
}

hipError_t launch_lattice_bilinear(const cplx *z, int nv, int nx, int ny, int nz, bool diag, double scale, double kd,
                                   const double *field, const double *planes, cplx *out, hipStream_t s) {
  if (nv <= 0) return hipSuccess;
  hipLaunchKernelGGL(lattice_bilinear_kernel, dim3(nv), dim3(256), 0, s, z, nx, ny, nz, diag ? 1 : 0, scale, kd, field,
                     planes, out);
  return hipGetLastError();
}
}  // namespace ldq
