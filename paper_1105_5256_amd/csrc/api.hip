// Host side of libldq: the C ABI (include/ldq.h), operators, device workspace
// and the driver that launches the Krylov passes until every probe converged.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <array>
#include <complex>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ldq.h"
#include "ldq_internal.h"

namespace ldq {
// launchers (pass2d.hip, pass3d.hip, misc.hip, colour.hip)
template <typename T> hipError_t launch_pass2d(const Pass2D<T> &, bool, bool, bool, hipStream_t);
hipError_t launch_rad_masks(uint64_t *out, uint64_t seed, int first, int nprobes, int nx, int ny, bool squared,
                            hipStream_t stream);
template <typename T> hipError_t launch_pass3d(const Pass3D<T> &, bool, hipStream_t);
void pass2d_tiles(int nx, int ny, bool squared, int rows, int *tiles_x, int *ntiles);
int pass2d_rows(bool squared, int want);
void pass3d_tiles(int nx, int ny, int nz, int zseg, int *tiles_x, int *tiles_y, int *nzseg, int *ntiles);
hipError_t launch_init_probes(ProbeState *, int, const int32_t *, int *, hipStream_t);
hipError_t launch_probe_terms(const ProbeState *, const ShiftState *, const cplx *, int, int, int, double *, int,
                              int *, hipStream_t);
hipError_t launch_sum_terms(const double *, int, int, double *, hipStream_t);
hipError_t launch_shifts(double, double, int, cplx *, cplx *, hipStream_t);
hipError_t launch_modular_fill(int32_t *, int, int, int, int, int, int, hipStream_t);
hipError_t launch_class_count(const int32_t *, size_t, int, int *, hipStream_t);
hipError_t launch_colour_max(const int32_t *, size_t, int *, hipStream_t);
hipError_t launch_minmax(const double *, size_t, double *, hipStream_t);
hipError_t launch_csr_abs_rowsum(const int32_t *, const double *, int64_t, double *, hipStream_t);
hipError_t launch_to_float(const double *, float *, size_t, hipStream_t);
hipError_t launch_jp_round(const int32_t *, const int32_t *, int64_t, int, const int32_t *, int32_t *,
                           unsigned long long *, unsigned long long *, int *, int *, hipStream_t);
// passcsr.hip
struct CsrSrc {
  const int32_t *rowptr, *colind;
  const double *val;
  const double *diag;
};
struct CsrSrcs {
  int nsrc;
  CsrSrc src[1 + LDQ_MAXP];
};
hipError_t launch_csr_slice_width(const CsrSrcs &, int64_t, int, int32_t *, hipStream_t);
hipError_t launch_csr_slab_fill(const CsrSrcs &, int64_t, int, const int64_t *, int32_t *, double *,
                                double *const *, hipStream_t);
int csr_register_width(int maxw, int64_t n, int elem);
template <typename T> hipError_t launch_csr_pass_a(const PassCsr<T> &, int, bool, hipStream_t);
template <typename T> hipError_t launch_csr_pass_b(const PassCsr<T> &, int, bool, hipStream_t);
hipError_t launch_csr_tail(const TailArgs &, int, int, int, hipStream_t);
hipError_t launch_lanczos_check(const double *, const ProbeState *, int, int, double, double, int *, hipStream_t);
hipError_t launch_batch_lanczos_check(const double *, const ProbeState *, int, int, const int32_t *, const double *,
                                      int *, hipStream_t);
template <typename T> hipError_t launch_batch2d(const Batch2D<T> &, int, bool, int, hipStream_t);
template <typename S>
hipError_t launch_mat_accum(const S *x, const double *w, int wstride, int m, int nb, int64_t n, double *y, bool init,
                            hipStream_t s);
template <typename S>
hipError_t launch_mat_accum_shifts(const S *x, const cplx *c, int cstride, int m, int N, int nb, int64_t n, cplx *z,
                                   bool init, hipStream_t s);
hipError_t launch_lattice_bilinear(const cplx *z, int nv, int nx, int ny, int nz, bool diag, double scale, double kd,
                                   const double *field, const double *planes, cplx *out, hipStream_t s);
hipError_t launch_batch_compact(const FieldDesc *, const int32_t *, int, const ProbeState *, ProbeState *, WorkItem *,
                                int *, hipStream_t);
}  // namespace ldq

using namespace ldq;

// ------------------------------------------------------------------ errors
static thread_local std::string g_last_error;

static int fail(int status, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return status;
}

#define HIPCHK(expr)                                                                                \
  do {                                                                                              \
    hipError_t e_ = (expr);                                                                         \
    if (e_ != hipSuccess) return fail(LDQ_E_DEVICE, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                                      __FILE__, __LINE__);                                          \
  } while (0)

#define CHK(expr)            \
  do {                       \
    int s_ = (expr);         \
    if (s_ != LDQ_OK) return s_; \
  } while (0)

extern "C" const char *ldq_status_string(int s) {
  switch (s) {
    case LDQ_OK: return "LDQ_OK";
    case LDQ_E_INVALID: return "LDQ_E_INVALID";
    case LDQ_E_NOT_SPD: return "LDQ_E_NOT_SPD";
    case LDQ_E_NO_CONVERGENCE: return "LDQ_E_NO_CONVERGENCE";
    case LDQ_E_ENCLOSURE: return "LDQ_E_ENCLOSURE";
    case LDQ_E_DEVICE: return "LDQ_E_DEVICE";
    case LDQ_E_NO_MEMORY: return "LDQ_E_NO_MEMORY";
    case LDQ_E_UNSUPPORTED: return "LDQ_E_UNSUPPORTED";
    default: return "LDQ_E_UNKNOWN";
  }
}

extern "C" const char *ldq_last_error(void) { return g_last_error.c_str(); }

// ------------------------------------------------------- device buffers
struct DevBuf {
  void *ptr = nullptr;
  size_t bytes = 0;
  int reserve(size_t want) {
    if (want <= bytes) return LDQ_OK;
    if (ptr) hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
    size_t grow = std::max(want, (size_t)256);
    if (hipMalloc(&ptr, grow) != hipSuccess) {
      ptr = nullptr;
      (void)hipGetLastError();
      return fail(LDQ_E_NO_MEMORY, "hipMalloc of %zu bytes failed", grow);
    }
    bytes = grow;
    return LDQ_OK;
  }
  void release() {
    if (ptr) hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
  }
  template <typename T> T *as() const { return (T *)ptr; }
};

// Concurrent chains of pass launches per probe block, at most (the context
// stream and up to three streams of the library; a process has four hardware
// queues by default).
constexpr int LDQ_MAX_LANES = 4;

struct ldq_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  DevBuf vec, partials, pstate, sstate, shifts, classes, terms, stats, sums, misc, colbuf, jpkey, jpmask, hist;
  DevBuf bfields, bitems, bwork, blohi;   // batched lattice passes
  DevBuf matw;                            // weights of a materialisation of f_N(Q) v
  DevBuf matc, matz, matq;                // consistent gradient: coefficients, shifted solutions, forms
  DevBuf radmask;                         // sign masks of random-sign probes (specialised 2-D pass)
  uint64_t radmask_key[5] = {};           // seed, probes, nx, ny, squared of the masks held
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipEvent_t evp[2] = {nullptr, nullptr};   // convergence polls
  int *hpin = nullptr;                      // pinned host copies of the device counters
  hipStream_t cap = nullptr;                // stream for HIP graph capture (created on first use)
  hipStream_t lane[LDQ_MAX_LANES] = {};     // lanes 1.. of the pass launches (created on first use)
  hipEvent_t evf = nullptr;                 // fork of the lanes from the context stream
  hipEvent_t evj[LDQ_MAX_LANES] = {};       // join of lane l back to it
  std::map<std::string, int> tuned_rows;    // autotuner choices for 2-D lattice problems (rows, lanes)
  std::vector<double> last_terms;
  int last_nparams = 0;
  int64_t last_count = 0;
};

enum OpKind { OPK_LATTICE = 1, OPK_CSR = 2, OPK_DIAG = 3, OPK_OBSGRAM = 4 };

struct ldq_op {
  ldq_ctx *ctx = nullptr;
  int kind = 0;
  int ndim = 0;
  int64_t shape[3] = {1, 1, 1};
  int64_t n = 0;
  int lkind = 0;
  double kappa2 = 0.0, scale = 1.0;
  double k2min = 0.0, k2max = 0.0;
  double *field = nullptr;     // kappa2 field (lattice) or d (diag), FP64 on device
  bool own_field = false;
  float *field32 = nullptr;
  // observation term (2-D lattice, or the gram operator itself)
  double tau = 0.0;
  int64_t nobs = 0;
  double *obs9 = nullptr;      // 9 x n planes, FP64
  float *obs9_32 = nullptr;
  double obs_gersh = 0.0;      // max row sum of |A^T A|
  uint64_t obs_hash = 0;       // FNV-1a of (nobs, corner, weight): equal data gives equal planes
  // CSR
  int64_t nnz = 0;
  int32_t *rowptr = nullptr, *colind = nullptr;
  double *val = nullptr;
  bool own_csr = false;
  uint64_t serial = 0;         // identifies the operator in caches keyed by operators
  double est_lo = 0.0, est_hi = 0.0;   // estimated enclosure of a CSR operator
  bool est_ok = false;
  // non-empty colour classes of the last modular colouring (C, a, b)
  int cls_C = 0, cls_a = 0, cls_b = 0;
  std::vector<int32_t> cls;
  struct Slab *slab = nullptr; // sliced layout of a CSR Q with its derivative operators
};

// Sliced layout of a CSR operator merged with the patterns of the derivative
// operators of a call (built on the device, kept until the key changes).
struct Slab {
  uint64_t key[1 + LDQ_MAXP] = {};
  int nkey = 0;
  int nslices = 0, maxw = 0;
  int64_t nslots = 0;
  DevBuf sptr, col, val, gval[LDQ_MAXP];
  void release() {
    sptr.release();
    col.release();
    val.release();
    for (auto &g : gval) g.release();
  }
};

static uint64_t next_serial() {
  static uint64_t counter = 0;
  return __atomic_add_fetch(&counter, 1, __ATOMIC_RELAXED);
}

static int set_device(ldq_ctx *ctx) {
  HIPCHK(hipSetDevice(ctx->device));
  return LDQ_OK;
}

// ---------------------------------------------------------------- context
extern "C" int ldq_create(int device, void *hip_stream, ldq_ctx **out) {
  if (!out) return fail(LDQ_E_INVALID, "out is NULL");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) {
    (void)hipGetLastError();
    return fail(LDQ_E_DEVICE, "no HIP device available");
  }
  if (device < 0 || device >= ndev) return fail(LDQ_E_INVALID, "device %d out of range (%d devices)", device, ndev);
  ldq_ctx *c = new (std::nothrow) ldq_ctx();
  if (!c) return fail(LDQ_E_NO_MEMORY, "context allocation failed");
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  if (hipSetDevice(device) != hipSuccess || hipEventCreate(&c->ev0) != hipSuccess ||
      hipEventCreate(&c->ev1) != hipSuccess || hipEventCreate(&c->evp[0]) != hipSuccess ||
      hipEventCreate(&c->evp[1]) != hipSuccess || hipHostMalloc((void **)&c->hpin, 16 * sizeof(int)) != hipSuccess) {
    (void)hipGetLastError();
    ldq_destroy(c);
    return fail(LDQ_E_DEVICE, "hipSetDevice/hipEventCreate/hipHostMalloc failed");
  }
  *out = c;
  return LDQ_OK;
}

extern "C" void ldq_destroy(ldq_ctx *c) {
  if (!c) return;
  hipSetDevice(c->device);
  hipStreamSynchronize(c->stream);
  for (DevBuf *b : {&c->vec, &c->partials, &c->pstate, &c->sstate, &c->shifts, &c->classes,
                    &c->terms, &c->stats, &c->sums, &c->misc, &c->colbuf, &c->jpkey, &c->jpmask, &c->hist,
                    &c->bfields, &c->bitems, &c->bwork, &c->blohi, &c->matw, &c->matc, &c->matz, &c->matq,
                    &c->radmask})
    b->release();
  if (c->ev0) hipEventDestroy(c->ev0);
  if (c->ev1) hipEventDestroy(c->ev1);
  for (hipEvent_t e : c->evp)
    if (e) hipEventDestroy(e);
  if (c->cap) hipStreamDestroy(c->cap);
  for (hipStream_t s : c->lane)
    if (s) {
      hipStreamSynchronize(s);
      hipStreamDestroy(s);
    }
  if (c->evf) hipEventDestroy(c->evf);
  for (hipEvent_t e : c->evj)
    if (e) hipEventDestroy(e);
  if (c->hpin) hipHostFree(c->hpin);
  delete c;
}

extern "C" int ldq_set_stream(ldq_ctx *c, void *hip_stream) {
  if (!c) return fail(LDQ_E_INVALID, "ctx is NULL");
  c->stream = (hipStream_t)hip_stream;
  return LDQ_OK;
}

// -------------------------------------------------------------- operators
static int upload(ldq_ctx *c, const void *src, size_t bytes, unsigned flags, void **dst, bool *own) {
  if (flags & LDQ_FLAG_DEVICE_PTR) {
    *dst = (void *)src;
    *own = false;
    return LDQ_OK;
  }
  if (hipMalloc(dst, std::max<size_t>(bytes, 4)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(LDQ_E_NO_MEMORY, "hipMalloc of %zu bytes failed", bytes);
  }
  *own = true;
  HIPCHK(hipMemcpyAsync(*dst, src, bytes, hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return LDQ_OK;
}

// min and max of a device FP64 array (deterministic)
static int device_minmax(ldq_ctx *c, const double *v, size_t n, double *lo, double *hi) {
  CHK(c->misc.reserve(512 * sizeof(double)));
  HIPCHK(launch_minmax(v, n, c->misc.as<double>(), c->stream));
  std::vector<double> h(512);
  HIPCHK(hipMemcpyAsync(h.data(), c->misc.ptr, 512 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  *lo = INFINITY;
  *hi = -INFINITY;
  for (int b = 0; b < 256; ++b) {
    *lo = std::min(*lo, h[2 * b]);
    *hi = std::max(*hi, h[2 * b + 1]);
  }
  return LDQ_OK;
}

extern "C" int ldq_op_lattice(ldq_ctx *c, int ndim, const int64_t *shape, int kind, double kappa2,
                              const double *kappa2_field, double scale, unsigned flags, ldq_op **out) {
  if (!c || !shape || !out) return fail(LDQ_E_INVALID, "NULL argument");
  if (ndim != 2 && ndim != 3) return fail(LDQ_E_INVALID, "ndim must be 2 or 3 (got %d)", ndim);
  if (kind != LDQ_SHIFTED_LAPLACIAN && kind != LDQ_SQUARED_SHIFTED_LAPLACIAN)
    return fail(LDQ_E_INVALID, "unknown lattice kind %d", kind);
  if (kind == LDQ_SQUARED_SHIFTED_LAPLACIAN && (ndim != 2 || kappa2_field))
    return fail(LDQ_E_UNSUPPORTED, "the squared operator is implemented for 2-D lattices with a constant kappa2");
  if (!std::isfinite(kappa2) || !std::isfinite(scale) || scale <= 0.0)
    return fail(LDQ_E_INVALID, "kappa2 and scale must be finite, scale > 0");
  int64_t n = 1;
  for (int d = 0; d < ndim; ++d) {
    if (shape[d] < 1 || shape[d] > (1 << 20)) return fail(LDQ_E_INVALID, "shape[%d] = %lld out of range", d,
                                                           (long long)shape[d]);
    n *= shape[d];
  }
  if (n > (int64_t)1 << 30) return fail(LDQ_E_INVALID, "lattice too large (%lld sites)", (long long)n);
  CHK(set_device(c));
  ldq_op *op = new ldq_op();
  op->serial = next_serial();
  op->ctx = c;
  op->kind = OPK_LATTICE;
  op->ndim = ndim;
  for (int d = 0; d < ndim; ++d) op->shape[d] = shape[d];
  op->n = n;
  op->lkind = kind;
  op->kappa2 = kappa2;
  op->scale = scale;
  op->k2min = op->k2max = kappa2;
  if (kappa2_field) {
    int st = upload(c, kappa2_field, n * sizeof(double), flags, (void **)&op->field, &op->own_field);
    if (st == LDQ_OK) st = device_minmax(c, op->field, n, &op->k2min, &op->k2max);
    if (st != LDQ_OK) {
      ldq_op_destroy(op);
      return st;
    }
    if (!std::isfinite(op->k2min) || !std::isfinite(op->k2max)) {
      ldq_op_destroy(op);
      return fail(LDQ_E_INVALID, "kappa2_field has non-finite values");
    }
  }
  *out = op;
  return LDQ_OK;
}

extern "C" int ldq_op_diag(ldq_ctx *c, int64_t n, const double *d, unsigned flags, ldq_op **out) {
  if (!c || !d || !out || n < 1) return fail(LDQ_E_INVALID, "invalid diagonal operator arguments");
  CHK(set_device(c));
  ldq_op *op = new ldq_op();
  op->serial = next_serial();
  op->ctx = c;
  op->kind = OPK_DIAG;
  op->n = n;
  int st = upload(c, d, n * sizeof(double), flags, (void **)&op->field, &op->own_field);
  if (st != LDQ_OK) {
    ldq_op_destroy(op);
    return st;
  }
  *out = op;
  return LDQ_OK;
}

extern "C" int ldq_op_csr(ldq_ctx *c, int64_t n, int64_t nnz, const int32_t *rowptr, const int32_t *colind,
                          const double *val, unsigned flags, ldq_op **out) {
  if (!c || !rowptr || !colind || !val || !out || n < 1 || nnz < 0 || nnz >= ((int64_t)1 << 31))
    return fail(LDQ_E_INVALID, "invalid CSR arguments");
  if (!(flags & LDQ_FLAG_DEVICE_PTR)) {
    if (rowptr[0] != 0 || rowptr[n] != nnz) return fail(LDQ_E_INVALID, "rowptr[0] must be 0 and rowptr[n] = nnz");
    for (int64_t i = 0; i < n; ++i) {
      if (rowptr[i + 1] < rowptr[i]) return fail(LDQ_E_INVALID, "rowptr not monotone at row %lld", (long long)i);
      for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
        if (colind[e] < 0 || colind[e] >= n)
          return fail(LDQ_E_INVALID, "colind[%d] = %d out of range", e, colind[e]);
        if (e > rowptr[i] && colind[e] <= colind[e - 1])
          return fail(LDQ_E_INVALID, "colind not strictly increasing in row %lld", (long long)i);
      }
    }
  }
  CHK(set_device(c));
  ldq_op *op = new ldq_op();
  op->serial = next_serial();
  op->ctx = c;
  op->kind = OPK_CSR;
  op->n = n;
  op->nnz = nnz;
  bool o1, o2, o3;
  int st = upload(c, rowptr, (n + 1) * sizeof(int32_t), flags, (void **)&op->rowptr, &o1);
  if (st == LDQ_OK) st = upload(c, colind, nnz * sizeof(int32_t), flags, (void **)&op->colind, &o2);
  if (st == LDQ_OK) st = upload(c, val, nnz * sizeof(double), flags, (void **)&op->val, &o3);
  op->own_csr = !(flags & LDQ_FLAG_DEVICE_PTR);
  if (st != LDQ_OK) {
    ldq_op_destroy(op);
    return st;
  }
  *out = op;
  return LDQ_OK;
}

// A^T A as 9 coefficient planes: plane d = (dy + 1) * 3 + (dx + 1) holds the
// entry between site s and s + dx + nx dy.  Accumulated on the host in
// observation order (deterministic), once per operator.
static int build_obs_planes(ldq_op *op, int64_t nobs, const int32_t *corner, const double *weight,
                            std::vector<double> &planes) {
  const int64_t nx = op->shape[0], ny = op->shape[1], n = op->n;
  planes.assign(9 * (size_t)n, 0.0);
  for (int64_t o = 0; o < nobs; ++o) {
    const int32_t *cs = corner + 4 * o;
    const double *ws = weight + 4 * o;
    if (!std::isfinite(ws[0]) || !std::isfinite(ws[1]) || !std::isfinite(ws[2]) || !std::isfinite(ws[3]))
      return fail(LDQ_E_INVALID, "observation %lld has a non-finite weight", (long long)o);
    const int32_t s00 = cs[0];
    if (s00 < 0 || s00 >= n) return fail(LDQ_E_INVALID, "observation %lld: corner out of range", (long long)o);
    const int64_t x0 = s00 % nx, y0 = s00 / nx;
    if (x0 + 1 >= nx || y0 + 1 >= ny || cs[1] != s00 + 1 || cs[2] != s00 + nx || cs[3] != s00 + nx + 1)
      return fail(LDQ_E_INVALID, "observation %lld: corners are not one lattice cell", (long long)o);
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) {
        const int64_t sa = cs[a], sb = cs[b];
        const int dx = (int)((sb % nx) - (sa % nx)), dy = (int)((sb / nx) - (sa / nx));
        planes[(size_t)((dy + 1) * 3 + (dx + 1)) * n + sa] += ws[a] * ws[b];
      }
  }
  double g = 0.0;
  for (int64_t s = 0; s < n; ++s) {
    double r = 0.0;
    for (int d = 0; d < 9; ++d) r += std::fabs(planes[(size_t)d * n + s]);
    g = std::max(g, r);
  }
  op->obs_gersh = g;
  return LDQ_OK;
}

static int set_obs(ldq_op *op, int64_t nobs, const int32_t *corner, const double *weight) {
  std::vector<double> planes;
  CHK(build_obs_planes(op, nobs, corner, weight, planes));
  if (op->obs9) hipFree(op->obs9);
  if (op->obs9_32) hipFree(op->obs9_32);
  op->obs9 = nullptr;
  op->obs9_32 = nullptr;
  bool own;
  CHK(upload(op->ctx, planes.data(), planes.size() * sizeof(double), 0, (void **)&op->obs9, &own));
  op->nobs = nobs;
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](const void *p, size_t bytes) {
    const unsigned char *b = (const unsigned char *)p;
    for (size_t i = 0; i < bytes; ++i) {
      h ^= b[i];
      h *= 1099511628211ull;
    }
  };
  mix(&nobs, sizeof nobs);
  mix(corner, 4 * (size_t)nobs * sizeof(int32_t));
  mix(weight, 4 * (size_t)nobs * sizeof(double));
  op->obs_hash = h;
  return LDQ_OK;
}

extern "C" int ldq_op_add_obs(ldq_op *Q, int64_t nobs, const int32_t *corner, const double *weight, double tau) {
  if (!Q || nobs < 0 || (nobs > 0 && (!corner || !weight)) || !(tau >= 0.0) || !std::isfinite(tau))
    return fail(LDQ_E_INVALID, "invalid observation arguments");
  if (Q->kind != OPK_LATTICE || Q->ndim != 2 || Q->lkind != LDQ_SQUARED_SHIFTED_LAPLACIAN)
    return fail(LDQ_E_UNSUPPORTED, "observation terms are implemented for the 2-D squared operator");
  CHK(set_device(Q->ctx));
  CHK(set_obs(Q, nobs, corner, weight));
  Q->tau = tau;
  return LDQ_OK;
}

extern "C" int ldq_op_obs_gram(ldq_ctx *c, const ldq_op *like, int64_t nobs, const int32_t *corner,
                               const double *weight, ldq_op **out) {
  if (!c || !like || !out || nobs < 0 || (nobs > 0 && (!corner || !weight)))
    return fail(LDQ_E_INVALID, "invalid observation arguments");
  if (like->kind != OPK_LATTICE || like->ndim != 2) return fail(LDQ_E_UNSUPPORTED, "needs a 2-D lattice operator");
  CHK(set_device(c));
  ldq_op *op = new ldq_op();
  op->serial = next_serial();
  op->ctx = c;
  op->kind = OPK_OBSGRAM;
  op->ndim = 2;
  op->shape[0] = like->shape[0];
  op->shape[1] = like->shape[1];
  op->n = like->n;
  op->tau = 1.0;
  int st = set_obs(op, nobs, corner, weight);
  if (st != LDQ_OK) {
    ldq_op_destroy(op);
    return st;
  }
  *out = op;
  return LDQ_OK;
}

extern "C" int64_t ldq_op_size(const ldq_op *op) { return op ? op->n : 0; }

extern "C" void ldq_op_destroy(ldq_op *op) {
  if (!op) return;
  if (op->ctx) {
    hipSetDevice(op->ctx->device);
    hipStreamSynchronize(op->ctx->stream);
  }
  if (op->own_field && op->field) hipFree(op->field);
  if (op->field32) hipFree(op->field32);
  if (op->obs9) hipFree(op->obs9);
  if (op->obs9_32) hipFree(op->obs9_32);
  if (op->own_csr) {
    if (op->rowptr) hipFree(op->rowptr);
    if (op->colind) hipFree(op->colind);
    if (op->val) hipFree(op->val);
  }
  if (op->slab) {
    op->slab->release();
    delete op->slab;
  }
  delete op;
}

// FP32 copies of operator data for LDQ_MIXED (made once, kept by the operator)
static int field_as(ldq_op *op, const float **out) {
  if (!op->field) {
    *out = nullptr;
    return LDQ_OK;
  }
  if (!op->field32) {
    if (hipMalloc(&op->field32, op->n * sizeof(float)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(LDQ_E_NO_MEMORY, "FP32 field copy");
    }
    HIPCHK(launch_to_float(op->field, op->field32, op->n, op->ctx->stream));
  }
  *out = op->field32;
  return LDQ_OK;
}
static int field_as(ldq_op *op, const double **out) {
  *out = op->field;
  return LDQ_OK;
}
static int obs_as(ldq_op *op, const float **out) {
  if (!op->obs9) {
    *out = nullptr;
    return LDQ_OK;
  }
  if (!op->obs9_32) {
    if (hipMalloc(&op->obs9_32, 9 * op->n * sizeof(float)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(LDQ_E_NO_MEMORY, "FP32 observation copy");
    }
    HIPCHK(launch_to_float(op->obs9, op->obs9_32, 9 * op->n, op->ctx->stream));
  }
  *out = op->obs9_32;
  return LDQ_OK;
}
static int obs_as(ldq_op *op, const double **out) {
  *out = op->obs9;
  return LDQ_OK;
}

// ------------------------------------------------------------- options
extern "C" void ldq_options_default(ldq_options *o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->k = 2;
  o->colouring = LDQ_COLOUR_AUTO;
  o->nshifts = 20;
  o->tol = 1e-10;
  o->grad_tol = 0.0;
  o->max_iter = 100000;
  o->precision = LDQ_FP64;
}

// ------------------------------------------------------- a2: enclosure
// Eigenvalues of the 1-D Dirichlet second difference of order m are
// 4 sin^2(pi i / (2 (m + 1))); the lattice Laplacian adds one per axis.
static void lap_extremes(const ldq_op *op, double *lo, double *hi) {
  *lo = 0.0;
  *hi = 0.0;
  for (int d = 0; d < op->ndim; ++d) {
    const double m = (double)op->shape[d];
    const double a = std::sin(M_PI / (2.0 * (m + 1.0))), b = std::sin(M_PI * m / (2.0 * (m + 1.0)));
    *lo += 4.0 * a * a;
    *hi += 4.0 * b * b;
  }
}

static int spectrum(const ldq_op *Q, double *lmin, double *lmax) {
  if (Q->kind == OPK_LATTICE) {
    double llo, lhi;
    lap_extremes(Q, &llo, &lhi);
    // Weyl: diag(kappa2) + L lies between (min kappa2) I + L and (max kappa2) I + L
    double lo = Q->k2min + llo, hi = Q->k2max + lhi;
    if (lo <= 0.0) return fail(LDQ_E_NOT_SPD, "lattice operator is not positive definite (lambda_min bound %g)", lo);
    if (Q->lkind == LDQ_SQUARED_SHIFTED_LAPLACIAN) {
      lo = lo * lo;
      hi = hi * hi;
    }
    lo *= Q->scale;
    hi *= Q->scale;
    // A^T A is positive semidefinite with lambda_max <= its Gershgorin bound
    if (Q->obs9) hi += Q->tau * Q->obs_gersh;
    *lmin = lo;
    *lmax = hi;
    return LDQ_OK;
  }
  if (Q->kind == OPK_DIAG) {
    ldq_ctx *c = Q->ctx;
    CHK(device_minmax(c, Q->field, Q->n, lmin, lmax));
    if (!(*lmin > 0.0)) return fail(LDQ_E_NOT_SPD, "diagonal operator has a non-positive entry");
    return LDQ_OK;
  }
  return fail(LDQ_E_UNSUPPORTED, "no automatic enclosure for this operator kind; pass lambda_min/lambda_max");
}

static int csr_bounds(ldq_ctx *c, ldq_op *Q, double *lo, double *hi);

extern "C" int ldq_spectrum_bounds(ldq_ctx *c, const ldq_op *Q, double *lmin, double *lmax) {
  if (!c || !Q || !lmin || !lmax) return fail(LDQ_E_INVALID, "NULL argument");
  if (Q->ctx != c) return fail(LDQ_E_INVALID, "operator belongs to another context");
  CHK(set_device(c));
  double lo, hi;
  if (Q->kind == OPK_CSR)
    CHK(csr_bounds(c, const_cast<ldq_op *>(Q), &lo, &hi));
  else
    CHK(spectrum(Q, &lo, &hi));
  *lmin = lo;
  *lmax = hi;
  return LDQ_OK;
}

// ------------------------------------------------------------ a3: shifts
extern "C" int ldq_shifts(ldq_ctx *c, double lmin, double lmax, int N, double *sigma, double *coef) {
  if (!c || !sigma || !coef) return fail(LDQ_E_INVALID, "NULL argument");
  if (N < 1 || N > LDQ_MAXN) return fail(LDQ_E_INVALID, "nshifts must be in 1..%d", LDQ_MAXN);
  if (!(lmin > 0.0) || !(lmax >= lmin) || !std::isfinite(lmax))
    return fail(LDQ_E_ENCLOSURE, "invalid enclosure [%g, %g]", lmin, lmax);
  CHK(set_device(c));
  CHK(c->shifts.reserve(2 * LDQ_MAXN * sizeof(cplx)));
  cplx *ds = c->shifts.as<cplx>(), *dc = ds + LDQ_MAXN;
  HIPCHK(launch_shifts(lmin, lmax, N, ds, dc, c->stream));
  HIPCHK(hipMemcpyAsync(sigma, ds, N * sizeof(cplx), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipMemcpyAsync(coef, dc, N * sizeof(cplx), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return LDQ_OK;
}

// ---------------------------------------------------------- a1: colouring
struct Colouring {
  int C = 0, a = 0, b = 0;          // modular parameters when C > 0 and colours == nullptr
  const int32_t *colours = nullptr; // device array otherwise
  int ncolours = 0;                 // C
  bool rad = false;                 // random-sign probes 0 .. ncolours - 1 instead (no classes)
  uint64_t seed = 0;
  const double *uvec = nullptr;     // or given probe vectors 0 .. ncolours - 1 (device, [probe][n])
};

// Smallest C (then smallest coefficients) with x + a y [+ b z] != 0 mod C for
// every nonzero offset of L1 length <= D.  Lattice graph distance is the L1
// distance for the 5/7-point operators and ceil(L1 / 2) for the 13-point one.
static bool modular_ok(int dim, int D, int C, int a, int b) {
  for (int dz = (dim == 3 ? -D : 0); dz <= (dim == 3 ? D : 0); ++dz)
    for (int dy = -D; dy <= D; ++dy)
      for (int dx = -D; dx <= D; ++dx) {
        const int l1 = std::abs(dx) + std::abs(dy) + std::abs(dz);
        if (l1 == 0 || l1 > D) continue;
        long v = (long)dx + (long)a * dy + (long)b * dz;
        if (((v % C) + C) % C == 0) return false;
      }
  return true;
}

// The search result depends only on (dim, D); it is kept for the process
// (the 3-D search at radius 6 visits ~10^7 candidates).
static int modular_params(int dim, int D, int *C, int *a, int *b) {
  static std::mutex mu;
  static std::map<std::pair<int, int>, std::array<int, 3>> found;
  {
    std::lock_guard<std::mutex> lock(mu);
    auto it = found.find({dim, D});
    if (it != found.end()) {
      *C = it->second[0];
      *a = it->second[1];
      *b = it->second[2];
      return LDQ_OK;
    }
  }
  for (int c = 1; c <= 4096; ++c) {
    for (int x = 0; x < c; ++x)
      for (int y = 0; y < (dim == 3 ? c : 1); ++y)
        if (modular_ok(dim, D, c, x, y)) {
          *C = c;
          *a = x;
          *b = y;
          std::lock_guard<std::mutex> lock(mu);
          found[{dim, D}] = {c, x, y};
          return LDQ_OK;
        }
  }
  return fail(LDQ_E_UNSUPPORTED, "no modular colouring with at most 4096 colours for distance %d", D);
}

// CSR pattern of a lattice operator (host-built once for the greedy colouring).
static void lattice_pattern(const ldq_op *op, std::vector<int32_t> &rp, std::vector<int32_t> &ci) {
  const int64_t nx = op->shape[0], ny = op->shape[1], nz = op->ndim == 3 ? op->shape[2] : 1;
  std::vector<int> off;
  const bool sq = op->lkind == LDQ_SQUARED_SHIFTED_LAPLACIAN;
  rp.assign(op->n + 1, 0);
  ci.clear();
  for (int64_t z = 0; z < nz; ++z)
    for (int64_t y = 0; y < ny; ++y)
      for (int64_t x = 0; x < nx; ++x) {
        const int64_t s = (z * ny + y) * nx + x;
        for (int dz = -1; dz <= 1; ++dz)
          for (int dy = -2; dy <= 2; ++dy)
            for (int dx = -2; dx <= 2; ++dx) {
              const int l1 = std::abs(dx) + std::abs(dy) + std::abs(dz);
              const bool in = sq ? (l1 >= 1 && l1 <= 2 && dz == 0) || (op->obs9 && std::abs(dx) <= 1 &&
                                                                         std::abs(dy) <= 1 && l1 >= 1 && dz == 0)
                                 : (l1 == 1 && (op->ndim == 3 || dz == 0));
              if (!in) continue;
              const int64_t xx = x + dx, yy = y + dy, zz = z + dz;
              if (xx < 0 || xx >= nx || yy < 0 || yy >= ny || zz < 0 || zz >= nz) continue;
              ci.push_back((int32_t)((zz * ny + yy) * nx + xx));
            }
        rp[s + 1] = (int32_t)ci.size();
      }
}

static int greedy_device(ldq_ctx *c, const ldq_op *Q, int k, const int32_t *prio_host, int32_t *dcol) {
  const int64_t n = Q->n;
  const int32_t *rp = nullptr, *ci = nullptr;
  DevBuf tmp_rp, tmp_ci, tmp_prio;
  std::vector<int32_t> hrp, hci;
  if (Q->kind == OPK_CSR) {
    rp = Q->rowptr;
    ci = Q->colind;
  } else if (Q->kind == OPK_LATTICE) {
    lattice_pattern(Q, hrp, hci);
    CHK(tmp_rp.reserve(hrp.size() * 4));
    CHK(tmp_ci.reserve(std::max<size_t>(hci.size(), 1) * 4));
    HIPCHK(hipMemcpyAsync(tmp_rp.ptr, hrp.data(), hrp.size() * 4, hipMemcpyHostToDevice, c->stream));
    if (!hci.empty())
      HIPCHK(hipMemcpyAsync(tmp_ci.ptr, hci.data(), hci.size() * 4, hipMemcpyHostToDevice, c->stream));
    rp = tmp_rp.as<int32_t>();
    ci = tmp_ci.as<int32_t>();
  } else {
    return fail(LDQ_E_UNSUPPORTED, "greedy colouring needs a lattice or CSR operator");
  }
  const int32_t *dprio = nullptr;
  if (prio_host) {
    for (int64_t i = 0; i < n; ++i)
      if (prio_host[i] < 0) return fail(LDQ_E_INVALID, "priority values must be >= 0");
    CHK(tmp_prio.reserve(n * 4));
    HIPCHK(hipMemcpyAsync(tmp_prio.ptr, prio_host, n * 4, hipMemcpyHostToDevice, c->stream));
    dprio = tmp_prio.as<int32_t>();
  }
  CHK(c->jpkey.reserve(2 * n * sizeof(unsigned long long)));
  CHK(c->jpmask.reserve(2 * n * 4 * sizeof(unsigned long long)));
  CHK(c->misc.reserve(4 * sizeof(int)));
  HIPCHK(hipMemsetAsync(dcol, 0xff, n * sizeof(int32_t), c->stream));   // -1: uncoloured
  int init[2] = {(int)n, 0};
  HIPCHK(hipMemcpyAsync(c->misc.ptr, init, sizeof init, hipMemcpyHostToDevice, c->stream));
  int h[2] = {(int)n, 0};
  for (int64_t round = 0; h[0] > 0; ++round) {
    if (round > n) return fail(LDQ_E_DEVICE, "greedy colouring made no progress");
    for (int rr = 0; rr < 8; ++rr)
      HIPCHK(launch_jp_round(rp, ci, n, k, dprio, dcol, c->jpkey.as<unsigned long long>(),
                             c->jpmask.as<unsigned long long>(), c->misc.as<int>(), c->misc.as<int>() + 1,
                             c->stream));
    round += 7;
    HIPCHK(hipMemcpyAsync(h, c->misc.ptr, sizeof h, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (h[1]) return fail(LDQ_E_UNSUPPORTED, "greedy colouring needs more than 256 colours");
  }
  HIPCHK(hipStreamSynchronize(c->stream));
  tmp_rp.release();
  tmp_ci.release();
  tmp_prio.release();
  return LDQ_OK;
}

static int lattice_radius(const ldq_op *Q, int k) {
  return Q->lkind == LDQ_SQUARED_SHIFTED_LAPLACIAN ? 2 * k : k;
}

// Resolve the colouring of a call; array colourings are stored in ctx->colbuf.
static int resolve_colouring(ldq_ctx *c, const ldq_op *Q, int k, int method, const int32_t *user,
                             const int32_t *prio, Colouring *col) {
  const int64_t n = Q->n;
  if (method == LDQ_COLOUR_AUTO) method = (Q->kind == OPK_LATTICE) ? LDQ_COLOUR_MODULAR : LDQ_COLOUR_GREEDY;
  if (method == LDQ_COLOUR_RADEMACHER) return LDQ_OK;   // set up by prepare_call
  if (method == LDQ_COLOUR_IDENTITY) {
    if (Q->kind == OPK_LATTICE && n < ((int64_t)1 << 31)) {
      // (x + nx y + nx ny z) mod n is the site index itself
      col->C = (int)n;
      col->a = (int)Q->shape[0];
      col->b = (int)(Q->shape[0] * Q->shape[1]);
      col->ncolours = (int)n;
      return LDQ_OK;
    }
    std::vector<int32_t> iota(n);
    for (int64_t i = 0; i < n; ++i) iota[i] = (int32_t)i;
    CHK(c->colbuf.reserve(n * 4));
    HIPCHK(hipMemcpyAsync(c->colbuf.ptr, iota.data(), n * 4, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    col->colours = c->colbuf.as<int32_t>();
    col->ncolours = (int)n;
    return LDQ_OK;
  }
  if (k < 1 && method != LDQ_COLOUR_USER) return fail(LDQ_E_INVALID, "colouring distance k must be >= 1");
  if (method == LDQ_COLOUR_MODULAR) {
    if (Q->kind != OPK_LATTICE) return fail(LDQ_E_UNSUPPORTED, "modular colouring needs a lattice operator");
    CHK(modular_params(Q->ndim, lattice_radius(Q, k), &col->C, &col->a, &col->b));
    col->ncolours = col->C;
    return LDQ_OK;
  }
  CHK(c->colbuf.reserve(n * 4));
  int32_t *dcol = c->colbuf.as<int32_t>();
  if (method == LDQ_COLOUR_USER) {
    if (!user) return fail(LDQ_E_INVALID, "user_colours is NULL");
    HIPCHK(hipMemcpyAsync(dcol, user, n * 4, hipMemcpyHostToDevice, c->stream));
  } else if (method == LDQ_COLOUR_GREEDY) {
    CHK(greedy_device(c, Q, k, prio, dcol));
  } else {
    return fail(LDQ_E_INVALID, "unknown colouring method %d", method);
  }
  CHK(c->misc.reserve(4 * sizeof(int)));
  int init[2] = {-1, 0};
  HIPCHK(hipMemcpyAsync(c->misc.ptr, init, sizeof init, hipMemcpyHostToDevice, c->stream));
  HIPCHK(launch_colour_max(dcol, n, c->misc.as<int>(), c->stream));
  int h[2];
  HIPCHK(hipMemcpyAsync(h, c->misc.ptr, sizeof h, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  if (h[1]) return fail(LDQ_E_INVALID, "negative colour value");
  col->colours = dcol;
  col->ncolours = h[0] + 1;
  return LDQ_OK;
}

extern "C" int ldq_colouring(ldq_ctx *c, const ldq_op *Q, int k, int method, const int32_t *priority,
                             int32_t *colours, int32_t *ncolours) {
  if (!c || !Q || !colours || !ncolours) return fail(LDQ_E_INVALID, "NULL argument");
  if (method == LDQ_COLOUR_USER || method == LDQ_COLOUR_AUTO) method = (Q->kind == OPK_LATTICE)
                                                                          ? LDQ_COLOUR_MODULAR
                                                                          : LDQ_COLOUR_GREEDY;
  CHK(set_device(c));
  Colouring col;
  CHK(resolve_colouring(c, Q, k, method, nullptr, priority, &col));
  const int64_t n = Q->n;
  if (!col.colours) {
    CHK(c->colbuf.reserve(n * 4));
    HIPCHK(launch_modular_fill(c->colbuf.as<int32_t>(), (int)Q->shape[0], (int)Q->shape[1],
                               Q->ndim == 3 ? (int)Q->shape[2] : 1, col.C, col.a, col.b, c->stream));
    col.colours = c->colbuf.as<int32_t>();
  }
  HIPCHK(hipMemcpyAsync(colours, col.colours, n * 4, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  *ncolours = col.ncolours;
  return LDQ_OK;
}

// --------------------------------------------------------- the Krylov driver
struct Call {
  ldq_ctx *c;
  ldq_op *Q;
  int nparams;
  ldq_op *dQ[LDQ_MAXP];
  ldq_options o;
  Colouring col;
  std::vector<int32_t> classes;   // non-empty colour classes (probe -> colour)
  double lmin, lmax;
  bool estimated;                 // enclosure from the Lanczos estimate (refined when a probe contradicts it)
  int ntiles;
  int stats[8];
  int rows2d;        // 2-D lattices: rows per wave tile (0: the specialised pass's standard tile)
  int lanes;         // lattices: concurrent chains of pass launches per probe block (1..LDQ_MAX_LANES)
  bool force_base;   // the base system must converge even without derivatives (Q^{-1} v)
  // materialising f_N(Q) v (second solve): y_j = sum_m w[j][m] r_m of probe j,
  // accumulated over `mat_steps` iterations (lattice operators, one block)
  const double *mat_w;
  int mat_wstride, mat_steps;
  double *mat_y;
  // ... or the shifted solutions z_jl = sum_m c[j][m][l] r_m themselves
  const cplx *mat_c;
  int mat_cstride;
  cplx *mat_z;
  double *tune_ms;   // non-null: a timing run of the autotuner (a few passes of the first probe block)
};

template <typename T>
static int fill_grad_terms(Call &k, GradTerm<T> *g) {
  for (int i = 0; i < k.nparams; ++i) {
    ldq_op *d = k.dQ[i];
    GradTerm<T> t{};
    if (d->kind == OPK_DIAG) {
      t.kind = GK_DIAG;
      t.scale = 1.0;
      CHK(field_as(d, &t.field));
    } else if (d->kind == OPK_LATTICE && d->lkind == LDQ_SHIFTED_LAPLACIAN) {
      t.kind = GK_SHIFTED;
      t.scale = d->scale;
      t.kappa2 = d->kappa2;
      CHK(field_as(d, &t.field));
    } else if (d->kind == OPK_OBSGRAM) {
      t.kind = GK_OBS;
      t.scale = d->tau;
      CHK(obs_as(d, &t.obs));
    } else {
      return fail(LDQ_E_UNSUPPORTED, "derivative operator %d: only shifted-Laplacian, diagonal and observation-gram"
                  " operators are supported", i);
    }
    g[i] = t;
  }
  return LDQ_OK;
}

// Lanczos coefficients kept per probe: all iterations up to 8192, within
// 64 MiB for the probe block.
static int hist_cap(int block, int max_iter) {
  const int64_t budget = ((int64_t)64 << 20) / (16 * (int64_t)std::max(block, 1));
  return (int)std::max<int64_t>(16, std::min<int64_t>({(int64_t)max_iter + 1, 8192, budget}));
}

// Interval the Lanczos eigenvalues may leave the enclosure [lo, hi] by through
// rounding (vectors of element size elem) before the check reports them.
static void check_interval(double lo, double hi, int elem, double *clo, double *chi) {
  const double eps = elem == 4 ? 5.96e-8 : 1.11e-16;
  const double slack = 256.0 * eps * hi;
  *clo = lo - (1e-3 * lo + slack);
  *chi = hi + (1e-3 * hi + slack);
}

// Extreme eigenvalues of the Lanczos matrix of K recorded CG steps (pairs
// alpha_i, beta_{i-1}), by bisection on Sturm counts.
static int sturm_below(const double *h, int K, double x) {
  double d = 1.0, aprev = 1.0;
  int cnt = 0;
  for (int i = 0; i < K; ++i) {
    double diag = 1.0 / h[2 * i], off2 = 0.0;
    if (i > 0) {
      diag += h[2 * i + 1] / aprev;
      off2 = h[2 * i + 1] / (aprev * aprev);
    }
    d = (diag - x) - (i > 0 ? off2 / d : 0.0);
    if (d == 0.0) d = -1e-300;
    cnt += d < 0.0;
    aprev = h[2 * i];
  }
  return cnt;
}

static void lanczos_extremes(const double *h, int K, double *tmin, double *tmax) {
  std::vector<double> diag(K), off(K + 1, 0.0);   // off[i] couples rows i - 1 and i
  for (int i = 0; i < K; ++i) {
    diag[i] = 1.0 / h[2 * i];
    if (i > 0) {
      diag[i] += h[2 * i + 1] / h[2 * (i - 1)];
      off[i] = std::sqrt(std::max(h[2 * i + 1], 0.0)) / std::fabs(h[2 * (i - 1)]);
    }
  }
  double glo = INFINITY, ghi = -INFINITY;   // Gershgorin interval of T
  for (int i = 0; i < K; ++i) {
    glo = std::min(glo, diag[i] - off[i] - off[i + 1]);
    ghi = std::max(ghi, diag[i] + off[i] + off[i + 1]);
  }
  auto bisect = [&](int target) {   // smallest x with at least `target` eigenvalues below it
    double a = glo, b = ghi;
    for (int it = 0; it < 200 && b - a > 1e-15 * std::max(std::fabs(a), std::fabs(b)); ++it) {
      const double mid = 0.5 * (a + b);
      if (sturm_below(h, K, mid) >= target) b = mid; else a = mid;
    }
    return 0.5 * (a + b);
  };
  *tmin = bisect(1);
  *tmax = bisect(K);
}

// A chunk of pass launches replayed from a HIP graph.  The launches are
// captured once (on the library's own capture stream: capture executes
// nothing, and the legacy default stream cannot be captured) and the graph
// is launched on the context stream for every chunk.
struct ChunkGraph {
  hipGraphExec_t exec = nullptr;
  ~ChunkGraph() {
    if (exec) hipGraphExecDestroy(exec);
  }
};

template <typename F>
static int graph_chunk(ldq_ctx *c, ChunkGraph &g, F enqueue_on, hipStream_t on) {
  if (!g.exec) {
    if (!c->cap) HIPCHK(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    HIPCHK(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
    const int rc = enqueue_on(c->cap);
    const hipError_t ec = hipStreamEndCapture(c->cap, &graph);
    if (rc != LDQ_OK) {
      if (graph) hipGraphDestroy(graph);
      return rc;
    }
    if (ec != hipSuccess) return fail(LDQ_E_DEVICE, "graph capture: %s", hipGetErrorString(ec));
    const hipError_t ei = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (ei != hipSuccess) {
      g.exec = nullptr;
      return fail(LDQ_E_DEVICE, "graph instantiate: %s", hipGetErrorString(ei));
    }
  }
  HIPCHK(hipGraphLaunch(g.exec, on));
  return LDQ_OK;
}

// Streams of lanes 1 .. nlanes - 1 of the pass launches and the events that
// fork them from and join them to the context stream (default priority, like
// the context stream; lane 0 is the context stream itself).
static int ensure_lanes(ldq_ctx *c, int nlanes) {
  for (int l = 1; l < nlanes; ++l) {
    if (!c->lane[l]) HIPCHK(hipStreamCreateWithFlags(&c->lane[l], hipStreamNonBlocking));
    if (!c->evj[l]) HIPCHK(hipEventCreateWithFlags(&c->evj[l], hipEventDisableTiming));
  }
  if (!c->evf) HIPCHK(hipEventCreateWithFlags(&c->evf, hipEventDisableTiming));
  return LDQ_OK;
}

// Queue chunks of launches until the device counter `active` reads 0.  The
// count after chunk c is copied to pinned host memory behind the chunk, and
// the host waits for it only after queueing chunk c + 1, so the device does
// not idle while the host decides; the extra chunk finds every probe stopped
// and its launches return at once.  *stalled when max_chunks are exceeded.
template <typename F>
static int poll_chunks(ldq_ctx *c, const int *active, F enqueue_chunk, int64_t max_chunks, int64_t *chunks,
                       bool *stalled) {
  int slot = 0, pending = -1;
  *chunks = 0;
  *stalled = false;
  for (;;) {
    CHK(enqueue_chunk());
    ++*chunks;
    HIPCHK(hipMemcpyAsync(c->hpin + slot, active, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipEventRecord(c->evp[slot], c->stream));
    if (pending >= 0) {
      HIPCHK(hipEventSynchronize(c->evp[pending]));
      if (c->hpin[pending] == 0) break;
    }
    pending = slot;
    slot ^= 1;
    if (*chunks > max_chunks) {
      *stalled = true;
      break;
    }
  }
  return LDQ_OK;
}

// Reduce the per-probe terms in probe order, bring the sums, the statistics
// and the terms to the host and fill the common fields of info.
static int collect_results(Call &k, int nprobes_total, double kernel_ms, int64_t passes, ldq_info *info,
                           double *out_sums, int64_t *iters_total) {
  ldq_ctx *c = k.c;
  const int P = k.nparams;
  HIPCHK(launch_sum_terms(c->terms.as<double>(), nprobes_total, 1 + P, c->sums.as<double>(), c->stream));
  double sums[1 + LDQ_MAXP];
  HIPCHK(hipMemcpyAsync(sums, c->sums.ptr, (1 + P) * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipMemcpyAsync(k.stats, c->stats.ptr, sizeof k.stats, hipMemcpyDeviceToHost, c->stream));
  c->last_terms.resize((size_t)nprobes_total * (1 + P));
  HIPCHK(hipMemcpyAsync(c->last_terms.data(), c->terms.ptr, c->last_terms.size() * sizeof(double),
                        hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  c->last_nparams = P;
  c->last_count = nprobes_total;
  for (int i = 0; i <= P; ++i) out_sums[i] = sums[i];
  std::memcpy(iters_total, k.stats + 2, sizeof *iters_total);
  if (info) {
    info->ncolours = nprobes_total;
    info->iters_max = k.stats[1];
    info->iters_total = *iters_total;
    info->lambda_min = k.lmin;
    info->lambda_max = k.lmax;
    info->loop_seconds = kernel_ms * 1e-3;
    info->passes = passes;
    info->probe_passes = *iters_total;
    uint64_t rbits;
    std::memcpy(&rbits, k.stats + 6, sizeof rbits);
    info->max_rel_residual = __builtin_bit_cast(double, rbits);
    info->enclosure_violations = k.stats[4];
    info->lanes = 1;
    info->tile_rows = 0;
  }
  return LDQ_OK;
}

static int finish_status(const Call &k, bool stalled) {
  if (stalled) return fail(LDQ_E_NO_CONVERGENCE, "probes did not stop within max_iter");
  if (k.stats[0] == 2) return fail(LDQ_E_NOT_SPD, "the Krylov recurrence met p^T Q p <= 0 or a non-finite value");
  if (k.stats[0] == 3)
    return fail(LDQ_E_NO_CONVERGENCE, "max_iter = %d reached before every shift converged", k.o.max_iter);
  return LDQ_OK;
}

template <typename T>
static int run_krylov(Call &k, ldq_info *info, double *out_sums) {
  ldq_ctx *c = k.c;
  ldq_op *Q = k.Q;
  const int64_t n = Q->n;
  const int N = k.o.nshifts;
  const int P = k.nparams;
  const int nq = LDQ_NQ_BASE + P;
  const int nprobes_total = (int)k.classes.size();
  const int block = (k.o.probe_block > 0) ? std::min(k.o.probe_block, nprobes_total) : nprobes_total;
  const bool is3d = Q->ndim == 3;
  // tiles
  int tiles_x = 0, tiles_y = 0, nzseg = 0, ntiles = 0;
  const int zseg = 64;
  const int rows2d = pass2d_rows(Q->lkind == LDQ_SQUARED_SHIFTED_LAPLACIAN, k.rows2d > 0 ? k.rows2d : LDQ_ROWS2D);
  if (is3d)
    pass3d_tiles((int)Q->shape[0], (int)Q->shape[1], (int)Q->shape[2], zseg, &tiles_x, &tiles_y, &nzseg, &ntiles);
  else
    pass2d_tiles((int)Q->shape[0], (int)Q->shape[1], Q->lkind == LDQ_SQUARED_SHIFTED_LAPLACIAN, rows2d, &tiles_x,
                 &ntiles);
  if ((int64_t)ntiles * block > INT32_MAX) return fail(LDQ_E_UNSUPPORTED, "grid too large");
  // workspace
  CHK(c->vec.reserve(4 * (size_t)block * n * sizeof(T)));
  const size_t part_elems = (size_t)block * ntiles * nq;
  CHK(c->partials.reserve(2 * part_elems * sizeof(double)));
  CHK(c->pstate.reserve(2 * (size_t)block * sizeof(ProbeState)));
  CHK(c->sstate.reserve((size_t)block * N * sizeof(ShiftState)));
  CHK(c->classes.reserve((size_t)nprobes_total * sizeof(int32_t) + 64));
  CHK(c->terms.reserve((size_t)nprobes_total * (1 + P) * sizeof(double) + 64));
  CHK(c->stats.reserve(8 * sizeof(int)));
  CHK(c->sums.reserve(8 * sizeof(double)));
  CHK(c->shifts.reserve(2 * LDQ_MAXN * sizeof(cplx)));
  CHK(c->misc.reserve(8 * sizeof(int)));
  T *vec = c->vec.as<T>();
  T *bufA_r = vec, *bufA_p = vec + (size_t)block * n, *bufB_r = vec + 2 * (size_t)block * n,
    *bufB_p = vec + 3 * (size_t)block * n;
  cplx *dsig = c->shifts.as<cplx>(), *dcoef = dsig + LDQ_MAXN;
  HIPCHK(launch_shifts(k.lmin, k.lmax, N, dsig, dcoef, c->stream));
  HIPCHK(hipMemsetAsync(c->stats.ptr, 0, 8 * sizeof(int), c->stream));
  HIPCHK(hipMemcpyAsync(c->classes.ptr, k.classes.data(), nprobes_total * sizeof(int32_t), hipMemcpyHostToDevice,
                        c->stream));
  int *active_count = c->misc.as<int>();

  double *part[2] = {c->partials.as<double>(), c->partials.as<double>() + part_elems};
  ProbeState *st[2] = {c->pstate.as<ProbeState>(), c->pstate.as<ProbeState>() + block};
  TailArgs ta{};
  ta.sh = c->sstate.as<ShiftState>();
  ta.sigma = dsig;
  ta.nshifts = N;
  ta.ngrad = P;
  ta.tol2 = k.o.tol * k.o.tol;
  const double gt = k.o.grad_tol > 0.0 ? k.o.grad_tol : k.o.tol;
  ta.grad_tol2 = gt * gt;
  ta.max_iter = k.o.max_iter;
  ta.active_count = active_count;
  ta.need_base = P > 0 || k.force_base;
  const int hcap = hist_cap(block, k.o.max_iter);
  CHK(c->hist.reserve((size_t)block * hcap * 2 * sizeof(double)));
  ta.hist = c->hist.as<double>();
  ta.hist_cap = hcap;
  double clo, chi;
  check_interval(k.lmin, k.lmax, (int)sizeof(T), &clo, &chi);

  GradTerm<T> grads[LDQ_MAXP] = {};
  CHK(fill_grad_terms<T>(k, grads));
  const T *kfield = nullptr, *obs = nullptr;
  CHK(field_as(Q, &kfield));
  CHK(obs_as(Q, &obs));

  Pass2D<T> a2{};
  Pass3D<T> a3{};
  if (is3d) {
    a3.nx = (int)Q->shape[0];
    a3.ny = (int)Q->shape[1];
    a3.nz = (int)Q->shape[2];
    a3.tiles_x = tiles_x;
    a3.tiles_y = tiles_y;
    a3.zseg = zseg;
    a3.nzseg = nzseg;
    a3.ntiles = ntiles;
    a3.colC = k.col.colours ? 0 : k.col.C;
    a3.cola = k.col.a;
    a3.colb = k.col.b;
    a3.colours = k.col.colours;
    a3.rad = k.col.rad;
    a3.seed = k.col.seed;
    a3.uvec = k.col.uvec;
    a3.kappa2 = Q->kappa2;
    a3.kappa2_field = kfield;
    a3.scale = Q->scale;
    for (int i = 0; i < P; ++i) a3.grad[i] = grads[i];
    a3.tail = ta;
  } else {
    a2.nx = (int)Q->shape[0];
    a2.ny = (int)Q->shape[1];
    a2.tiles_x = tiles_x;
    a2.ntiles = ntiles;
    a2.rows = rows2d;
    a2.colC = k.col.colours ? 0 : k.col.C;
    a2.cola = k.col.a;
    a2.colours = k.col.colours;
    a2.rad = k.col.rad;
    a2.seed = k.col.seed;
    a2.uvec = k.col.uvec;
    a2.kappa2 = Q->kappa2;
    a2.kappa2_field = kfield;
    a2.scale = Q->scale;
    a2.tau = Q->obs9 ? Q->tau : 0.0;
    a2.obs = obs;
    for (int i = 0; i < P; ++i) a2.grad[i] = grads[i];
    a2.tail = ta;
  }
  const bool sq = Q->lkind == LDQ_SQUARED_SHIFTED_LAPLACIAN;
  const bool has_obs = Q->obs9 != nullptr && Q->tau != 0.0;
  // the specialised 2-D pass: modular colouring, constant kappa2, gradient 0 a
  // shifted Laplacian with a constant shift, gradient 1 (with observations)
  // the observation gram of Q's own observations
  bool fast2d = !is3d && !k.col.colours && !k.col.uvec && !kfield && Q->scale == 1.0 &&
                (double)Q->n * sizeof(T) * (has_obs ? 9.0 : 1.0) < 4294967295.0;
  if (P >= 1) fast2d = fast2d && grads[0].kind == GK_SHIFTED && !grads[0].field;
  if (P >= 2)
    fast2d = fast2d && has_obs && grads[1].kind == GK_OBS && k.dQ[1]->obs_hash == Q->obs_hash &&
             k.dQ[1]->nobs == Q->nobs;
  if (P >= 2 && fast2d) a2.grad[1].scale = k.dQ[1]->tau;
  // random-sign probes take the specialised pass through per-row sign masks
  // of its strips (one 64-bit word per probe, row and strip; kept on the
  // context): without observations and for at most 64 MiB of masks
  const uint64_t *rmask = nullptr;
  if (fast2d && k.col.rad) {
    const size_t words = (size_t)nprobes_total * (size_t)Q->shape[1] * (size_t)tiles_x;
    if (has_obs || words * 8 > ((size_t)64 << 20)) {
      fast2d = false;
    } else {
      const uint64_t key[5] = {k.col.seed, (uint64_t)nprobes_total, (uint64_t)Q->shape[0], (uint64_t)Q->shape[1],
                               (uint64_t)sq};
      if (!c->radmask.ptr || memcmp(key, c->radmask_key, sizeof key) != 0) {
        memset(c->radmask_key, 0, sizeof c->radmask_key);
        CHK(c->radmask.reserve(words * 8));
        HIPCHK(launch_rad_masks(c->radmask.as<uint64_t>(), k.col.seed, 0, nprobes_total, (int)Q->shape[0],
                                (int)Q->shape[1], sq, c->stream));
        memcpy(c->radmask_key, key, sizeof key);
      }
      rmask = c->radmask.as<uint64_t>();
    }
  }
  // the specialised 3-D pass: modular colouring, scale 1, at most two diagonal
  // derivative operators, 32-bit byte offsets
  bool fast3d = is3d && !k.col.colours && !k.col.rad && !k.col.uvec && Q->scale == 1.0 && P <= 2 &&
                (double)Q->n * sizeof(T) < 4294967295.0;
  for (int i = 0; i < P; ++i) fast3d = fast3d && grads[i].kind == GK_DIAG;
  // Launch over probes p0 .. p0 + nprobes - 1 of the block with the probe state
  // and partials read from buffer `in` and written to 1 - in, on stream ls (the
  // context stream, the second lane's stream, or the capture stream while a
  // chunk is captured).  Every per-probe array is probe-major, so a part of
  // the block is the whole-block launch with its base pointers advanced.
  hipStream_t ls = c->stream;
  int blk_first = 0;   // first probe of the block being run
  auto launch = [&](int mode, int nprobes, int in, const T *rin, const T *pin, T *rout, T *pout,
                    int p0 = 0) -> hipError_t {
    TailArgs t = ta;
    const size_t po = (size_t)p0 * nq * ntiles, vo = (size_t)p0 * n;
    t.st_in = st[in] + p0;
    t.st_out = st[1 - in] + p0;
    t.part_in = part[in] + po;
    t.part_out = part[mode == MODE_INIT ? in : 1 - in] + po;
    t.sh = ta.sh + (size_t)p0 * N;
    t.hist = ta.hist + (size_t)p0 * hcap * 2;
    if (rin) rin += vo;
    if (pin) pin += vo;
    if (rout) rout += vo;
    if (pout) pout += vo;
    a2.tail = t;
    a3.tail = t;
    if (is3d) {
      a3.mode = mode;
      a3.nprobes = nprobes;
      a3.r_in = rin;
      a3.p_in = pin;
      a3.r_out = rout;
      a3.p_out = pout;
      return launch_pass3d<T>(a3, fast3d, ls);
    }
    a2.mode = mode;
    a2.nprobes = nprobes;
    // the masks of random-sign probe j (class j) start at word j ny tiles_x
    a2.rmask = rmask ? rmask + (size_t)(blk_first + p0) * (size_t)Q->shape[1] * (size_t)tiles_x : nullptr;
    a2.r_in = rin;
    a2.p_in = pin;
    a2.r_out = rout;
    a2.p_out = pout;
    return launch_pass2d<T>(a2, sq, has_obs, fast2d, ls);
  };
  const bool graphs = k.o.launch_mode != LDQ_LAUNCH_DIRECT;

  // an even number of passes per chunk keeps every chunk on the same buffer parity
  const int check = k.o.check_every > 0 ? 2 * ((k.o.check_every + 1) / 2) : 16;
  int64_t passes = 0;
  bool stalled = false;
  // Device time of the pass kernels: HIP events bracket each chunk of
  // back-to-back pass launches on the context stream (the host polls for
  // convergence between chunks, outside the bracketed spans).
  double kernel_ms = 0.0;
  for (int first = 0; first < nprobes_total; first += block) {
    const int nb = std::min(block, nprobes_total - first);
    blk_first = first;
    // state 0 <- initial; INIT: dots of v -> partials 0; FIRST: tail-init from
    // partials 0, state 0 -> 1, pass -> partials 1, vectors A; then STEP pairs
    // (state 1 -> 0, A -> B) and (state 0 -> 1, B -> A).  The final state is in 1.
    HIPCHK(launch_init_probes(st[0], nb, c->classes.as<int32_t>() + first, active_count, c->stream));
    HIPCHK(hipEventRecord(c->ev0, c->stream));
    HIPCHK(launch(MODE_INIT, nb, 0, nullptr, nullptr, nullptr, nullptr));
    HIPCHK(launch(MODE_FIRST, nb, 0, nullptr, nullptr, bufA_r, bufA_p));
    passes += 2;
    if (k.mat_y || k.mat_z) {
      // second solve of a materialisation: y = w_0 v + sum_{m >= 1} w_m r_m
      // (or each shift's z_l = sum_m c_ml r_m), r_0 = p_0 = v and r_1 from
      // FIRST, r_{m+1} from the m-th STEP pass (the probes stop where the
      // first solve's did; their coefficients are 0 beyond)
      const int N = k.o.nshifts;
      if (k.mat_y) {
        HIPCHK(launch_mat_accum<double>(k.col.uvec, k.mat_w, k.mat_wstride, 0, nb, n, k.mat_y, true, c->stream));
        HIPCHK(launch_mat_accum<T>(bufA_r, k.mat_w, k.mat_wstride, 1, nb, n, k.mat_y, false, c->stream));
      } else {
        HIPCHK(launch_mat_accum_shifts<T>(bufA_p, k.mat_c, k.mat_cstride, 0, N, nb, n, k.mat_z, true, c->stream));
        HIPCHK(launch_mat_accum_shifts<T>(bufA_r, k.mat_c, k.mat_cstride, 1, N, nb, n, k.mat_z, false, c->stream));
      }
      for (int m = 1; m + 1 < k.mat_steps; ++m) {
        const bool odd = (m % 2) == 1;
        HIPCHK(odd ? launch(MODE_STEP, nb, 1, bufA_r, bufA_p, bufB_r, bufB_p)
                   : launch(MODE_STEP, nb, 0, bufB_r, bufB_p, bufA_r, bufA_p));
        const T *rm = odd ? bufB_r : bufA_r;
        if (k.mat_y)
          HIPCHK(launch_mat_accum<T>(rm, k.mat_w, k.mat_wstride, m + 1, nb, n, k.mat_y, false, c->stream));
        else
          HIPCHK(launch_mat_accum_shifts<T>(rm, k.mat_c, k.mat_cstride, m + 1, N, nb, n, k.mat_z, false, c->stream));
        ++passes;
      }
      HIPCHK(hipStreamSynchronize(c->stream));
      continue;
    }
    // the STEP passes of the block in nlanes chains: lane l advances probes
    // lp0[l] .. lp0[l] + lnp[l] - 1 (near-equal shares); lanes 1.. run on
    // streams of their own, forked from and joined to the context stream
    // around every chunk
    const int nlanes = std::max(1, std::min(k.lanes, nb));
    int lnp[LDQ_MAX_LANES] = {}, lp0[LDQ_MAX_LANES] = {};
    for (int l = 0; l < nlanes; ++l) {
      lnp[l] = nb / nlanes + (l < nb % nlanes ? 1 : 0);
      lp0[l] = l ? lp0[l - 1] + lnp[l - 1] : 0;
    }
    auto lane_stream = [&](int l) { return l ? c->lane[l] : c->stream; };
    if (nlanes > 1) CHK(ensure_lanes(c, nlanes));
    auto fork = [&]() -> int {
      if (nlanes > 1) {
        HIPCHK(hipEventRecord(c->evf, c->stream));
        for (int l = 1; l < nlanes; ++l) HIPCHK(hipStreamWaitEvent(c->lane[l], c->evf, 0));
      }
      return LDQ_OK;
    };
    auto join = [&]() -> int {
      for (int l = 1; l < nlanes; ++l) {
        HIPCHK(hipEventRecord(c->evj[l], c->lane[l]));
        HIPCHK(hipStreamWaitEvent(c->stream, c->evj[l], 0));
      }
      return LDQ_OK;
    };
    if (k.tune_ms) {
      // autotuner timing run: one chunk's worth of STEP passes of this block
      // (as forked into lanes in a real run), then stop
      constexpr int TUNE_STEPS = 16;
      HIPCHK(hipEventRecord(c->ev0, c->stream));
      CHK(fork());
      for (int l = 0; l < nlanes; ++l) {
        ls = lane_stream(l);
        for (int i = 0; i < TUNE_STEPS; ++i)
          HIPCHK(i % 2 == 0 ? launch(MODE_STEP, lnp[l], 1, bufA_r, bufA_p, bufB_r, bufB_p, lp0[l])
                            : launch(MODE_STEP, lnp[l], 0, bufB_r, bufB_p, bufA_r, bufA_p, lp0[l]));
      }
      ls = c->stream;
      CHK(join());
      HIPCHK(hipEventRecord(c->ev1, c->stream));
      HIPCHK(hipEventSynchronize(c->ev1));
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, c->ev0, c->ev1));
      *k.tune_ms = ms;
      return LDQ_OK;
    }
    // a chunk is an even number of passes, so every chunk starts from the
    // same buffers and one captured graph per lane serves all chunks of the
    // block
    auto steps = [&](int l, hipStream_t s) -> int {
      ls = s;
      bool in_a = true;
      for (int i = 0; i < check; ++i) {
        const hipError_t e = in_a ? launch(MODE_STEP, lnp[l], 1, bufA_r, bufA_p, bufB_r, bufB_p, lp0[l])
                                  : launch(MODE_STEP, lnp[l], 0, bufB_r, bufB_p, bufA_r, bufA_p, lp0[l]);
        in_a = !in_a;
        if (e != hipSuccess) {
          ls = c->stream;
          return fail(LDQ_E_DEVICE, "pass launch: %s", hipGetErrorString(e));
        }
      }
      ls = c->stream;
      return LDQ_OK;
    };
    ChunkGraph cg[LDQ_MAX_LANES];
    auto chunk = [&]() -> int {
      CHK(fork());
      for (int l = 0; l < nlanes; ++l) {
        hipStream_t on = lane_stream(l);
        auto lane_steps = [&](hipStream_t s) { return steps(l, s); };
        CHK(graphs ? graph_chunk(c, cg[l], lane_steps, on) : steps(l, on));
      }
      return join();
    };
    int64_t chunks = 0;
    bool st_block = false;
    CHK(poll_chunks(c, active_count, chunk, ((int64_t)k.o.max_iter + 2 * check) / check + 1, &chunks, &st_block));
    passes += chunks * check;
    stalled = stalled || st_block;
    HIPCHK(hipEventRecord(c->ev1, c->stream));
    HIPCHK(hipEventSynchronize(c->ev1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    kernel_ms += ms;
    HIPCHK(launch_lanczos_check(ta.hist, st[1], nb, hcap, clo, chi, c->stats.as<int>(), c->stream));
    HIPCHK(launch_probe_terms(st[1], ta.sh, dcoef, nb, N, P, c->terms.as<double>(), first, c->stats.as<int>(),
                              c->stream));
  }
  int64_t iters_total = 0;
  CHK(collect_results(k, nprobes_total, kernel_ms, passes, info, out_sums, &iters_total));
  if (info) {
    info->lanes = std::max(1, std::min(k.lanes, block));
    info->tile_rows = is3d ? 0 : rows2d;
    // vectors: first pass writes r, p; every later pass reads and writes both;
    // operator fields (kappa2 / derivative diagonals / observation planes) once per launch
    const double sv = (double)sizeof(T);
    double fields = 0.0;
    if (kfield) fields += 1.0;
    if (has_obs) fields += 9.0;
    for (int i = 0; i < P; ++i)
      if (grads[i].kind == GK_DIAG || (grads[i].kind == GK_SHIFTED && grads[i].field)) fields += 1.0;
    info->bytes_model = sv * (double)n * (4.0 * (double)iters_total - 2.0 * (double)nprobes_total) +
                        sv * (double)n * fields * (double)(passes - 2);
  }
  return finish_status(k, stalled);
}

// ---------------------------------------------------- general sparse operators
// Sliced layout of Q merged with the derivative operators of the call (values
// in FP64 for both precisions: rounding the operator itself to FP32 would
// perturb Q by its condition number); cached on Q and rebuilt when the
// derivative operators change.
static int csr_slab(Call &k, Slab **out) {
  ldq_ctx *c = k.c;
  ldq_op *Q = k.Q;
  const int P = k.nparams;
  uint64_t key[1 + LDQ_MAXP] = {Q->serial};
  for (int i = 0; i < P; ++i) key[1 + i] = k.dQ[i]->serial;
  Slab *sl = Q->slab;
  if (sl && sl->nkey == 1 + P && std::equal(key, key + 1 + P, sl->key)) {
    *out = sl;
    return LDQ_OK;
  }
  if (!sl) {
    sl = new (std::nothrow) Slab();
    if (!sl) return fail(LDQ_E_NO_MEMORY, "slab descriptor");
    Q->slab = sl;
  }
  sl->nkey = 0;   // invalid until complete
  const int64_t n = Q->n;
  const int64_t nsl = (n + 63) / 64;
  if (nsl > INT32_MAX / 4) return fail(LDQ_E_UNSUPPORTED, "operator too large");
  const int nslices = (int)nsl;
  CsrSrcs S{};
  S.nsrc = 1 + P;
  S.src[0] = CsrSrc{Q->rowptr, Q->colind, Q->val, nullptr};
  for (int i = 0; i < P; ++i) {
    const ldq_op *d = k.dQ[i];
    if (d->kind == OPK_CSR)
      S.src[1 + i] = CsrSrc{d->rowptr, d->colind, d->val, nullptr};
    else
      S.src[1 + i] = CsrSrc{nullptr, nullptr, nullptr, d->field};
  }
  DevBuf wbuf;
  CHK(wbuf.reserve((size_t)nslices * sizeof(int32_t)));
  HIPCHK(launch_csr_slice_width(S, n, nslices, wbuf.as<int32_t>(), c->stream));
  std::vector<int32_t> w(nslices);
  HIPCHK(hipMemcpyAsync(w.data(), wbuf.ptr, (size_t)nslices * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  std::vector<int64_t> sp(nslices + 1);
  sp[0] = 0;
  int maxw = 0;
  for (int i = 0; i < nslices; ++i) {
    maxw = std::max(maxw, (int)w[i]);
    sp[i + 1] = sp[i] + 64 * (int64_t)w[i];
  }
  const int64_t nslots = std::max<int64_t>(sp[nslices], 64);
  if (nslots >= ((int64_t)1 << 40)) return fail(LDQ_E_UNSUPPORTED, "operator too large");
  CHK(sl->sptr.reserve((size_t)(nslices + 1) * sizeof(int64_t)));
  CHK(sl->col.reserve((size_t)nslots * sizeof(int32_t)));
  CHK(sl->val.reserve((size_t)nslots * sizeof(double)));
  double *g[LDQ_MAXP] = {};
  for (int i = 0; i < P; ++i) {
    CHK(sl->gval[i].reserve((size_t)nslots * sizeof(double)));
    g[i] = sl->gval[i].as<double>();
  }
  HIPCHK(hipMemcpyAsync(sl->sptr.ptr, sp.data(), sp.size() * sizeof(int64_t), hipMemcpyHostToDevice, c->stream));
  HIPCHK(launch_csr_slab_fill(S, n, nslices, sl->sptr.as<int64_t>(), sl->col.as<int32_t>(), sl->val.as<double>(), g,
                              c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  wbuf.release();
  sl->nslices = nslices;
  sl->maxw = maxw;
  sl->nslots = sp[nslices];
  std::copy(key, key + 1 + P, sl->key);
  sl->nkey = 1 + P;
  *out = sl;
  return LDQ_OK;
}

// One probe of all ones through the CSR passes with no shifts: its CG
// coefficients give the Lanczos matrix whose extreme eigenvalues approximate
// those of Q from inside.  The upper end of the enclosure is the Gershgorin
// bound of Q; the lower end is half the smallest Lanczos eigenvalue (refined
// later if a probe's own Lanczos matrix reaches below it).
template <typename T>
static int csr_estimate(Call &k, Slab *sl, double *lo, double *hi) {
  ldq_ctx *c = k.c;
  ldq_op *Q = k.Q;
  const int64_t n = Q->n;
  const int L = 200;
  const int W = csr_register_width(sl->maxw, n, (int)sizeof(T));
  DevBuf zcol, cls, vec, part, pst, hist, rs;
  CHK(zcol.reserve(n * sizeof(int32_t)));
  CHK(cls.reserve(sizeof(int32_t)));
  CHK(vec.reserve(4 * n * sizeof(T)));
  CHK(part.reserve((size_t)sl->nslices * LDQ_NQ_BASE * sizeof(double)));
  CHK(pst.reserve(sizeof(ProbeState)));
  CHK(hist.reserve((size_t)(L + 2) * 2 * sizeof(double)));
  CHK(rs.reserve(n * sizeof(double)));
  // misc also serves device_minmax below: size it for that first, so that the
  // counter taken from it now is not reallocated under the queued launches
  CHK(c->misc.reserve(512 * sizeof(double)));
  HIPCHK(hipMemsetAsync(zcol.ptr, 0, n * sizeof(int32_t), c->stream));
  HIPCHK(hipMemsetAsync(cls.ptr, 0, sizeof(int32_t), c->stream));
  int *active = c->misc.as<int>();
  ProbeState *st = pst.as<ProbeState>();
  TailArgs ta{};
  ta.part_in = part.as<double>();
  ta.part_out = part.as<double>();
  ta.st_in = st;
  ta.st_out = st;
  ta.ngrad = 0;
  ta.nshifts = 0;
  ta.grad_tol2 = 1e-20;
  ta.max_iter = L;
  ta.active_count = active;
  ta.need_base = 1;
  ta.hist = hist.as<double>();
  ta.hist_cap = L + 2;
  PassCsr<T> a{};
  a.n = n;
  a.nslices = sl->nslices;
  a.nprobes = 1;
  a.ngrad = 0;
  a.nq = LDQ_NQ_BASE;
  a.sptr = sl->sptr.as<int64_t>();
  a.col = sl->col.as<int32_t>();
  a.val = sl->val.as<double>();
  a.colours = zcol.as<int32_t>();
  a.st = st;
  a.part = part.as<double>();
  T *v = vec.as<T>();
  T *ar = v, *ap = v + n, *br = v + 2 * n, *bp = v + 3 * n;
  HIPCHK(launch_init_probes(st, 1, cls.as<int32_t>(), active, c->stream));
  HIPCHK(launch_csr_pass_b<T>(a, W, true, c->stream));
  HIPCHK(launch_csr_tail(ta, 1, a.nslices, MODE_FIRST, c->stream));
  a.r_out = ar;
  a.p_out = ap;
  HIPCHK(launch_csr_pass_a<T>(a, W, true, c->stream));
  a.r_in = ar;
  HIPCHK(launch_csr_pass_b<T>(a, W, false, c->stream));
  bool in_a = true;
  for (int it = 0; it < L + 1; ++it) {
    HIPCHK(launch_csr_tail(ta, 1, a.nslices, MODE_STEP, c->stream));
    a.r_in = in_a ? ar : br;
    a.p_in = in_a ? ap : bp;
    a.r_out = in_a ? br : ar;
    a.p_out = in_a ? bp : ap;
    HIPCHK(launch_csr_pass_a<T>(a, W, false, c->stream));
    a.r_in = a.r_out;
    HIPCHK(launch_csr_pass_b<T>(a, W, false, c->stream));
    in_a = !in_a;
  }
  // Gershgorin bound of Q
  HIPCHK(launch_csr_abs_rowsum(Q->rowptr, Q->val, n, rs.as<double>(), c->stream));
  double glo, ghi;
  CHK(device_minmax(c, rs.as<double>(), n, &glo, &ghi));
  ProbeState hs;
  std::vector<double> h(2 * (size_t)(L + 2));
  HIPCHK(hipMemcpyAsync(&hs, st, sizeof hs, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipMemcpyAsync(h.data(), hist.ptr, h.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  if (hs.status == 2) return fail(LDQ_E_NOT_SPD, "the Krylov recurrence met p^T Q p <= 0 or a non-finite value");
  const int K = std::min(hs.active ? hs.iter + 1 : hs.iter, L + 2);
  if (K < 1) return fail(LDQ_E_ENCLOSURE, "the enclosure estimate made no progress");
  double tmin, tmax;
  lanczos_extremes(h.data(), K, &tmin, &tmax);
  if (!(tmin > 0.0) || !std::isfinite(tmax)) return fail(LDQ_E_NOT_SPD, "Lanczos estimate of lambda_min is %g", tmin);
  *lo = 0.5 * tmin;
  *hi = std::max(ghi, tmax);
  return LDQ_OK;
}

template <typename T>
static int run_krylov_csr(Call &k, ldq_info *info, double *out_sums) {
  ldq_ctx *c = k.c;
  ldq_op *Q = k.Q;
  const int64_t n = Q->n;
  const int N = k.o.nshifts;
  const int P = k.nparams;
  const int nq = LDQ_NQ_BASE + P;
  const int nprobes_total = (int)k.classes.size();
  const int block = (k.o.probe_block > 0) ? std::min(k.o.probe_block, nprobes_total) : nprobes_total;
  Slab *sl = nullptr;
  CHK(csr_slab(k, &sl));
  if (!(k.lmin > 0.0)) {
    CHK(csr_estimate<T>(k, sl, &k.lmin, &k.lmax));
    k.estimated = true;
  }
  const int W = csr_register_width(sl->maxw, n, (int)sizeof(T));
  const int ntiles = sl->nslices;
  const int hcap = hist_cap(block, k.o.max_iter);
  CHK(c->vec.reserve(4 * (size_t)block * n * sizeof(T)));
  CHK(c->partials.reserve((size_t)block * ntiles * nq * sizeof(double)));
  CHK(c->pstate.reserve((size_t)block * sizeof(ProbeState)));
  CHK(c->sstate.reserve((size_t)block * N * sizeof(ShiftState)));
  CHK(c->classes.reserve((size_t)nprobes_total * sizeof(int32_t) + 64));
  CHK(c->terms.reserve((size_t)nprobes_total * (1 + P) * sizeof(double) + 64));
  CHK(c->stats.reserve(8 * sizeof(int)));
  CHK(c->sums.reserve(8 * sizeof(double)));
  CHK(c->shifts.reserve(2 * LDQ_MAXN * sizeof(cplx)));
  CHK(c->misc.reserve(8 * sizeof(int)));
  CHK(c->hist.reserve((size_t)block * hcap * 2 * sizeof(double)));
  T *vec = c->vec.as<T>();
  T *bufA_r = vec, *bufA_p = vec + (size_t)block * n, *bufB_r = vec + 2 * (size_t)block * n,
    *bufB_p = vec + 3 * (size_t)block * n;
  cplx *dsig = c->shifts.as<cplx>(), *dcoef = dsig + LDQ_MAXN;
  HIPCHK(hipMemcpyAsync(c->classes.ptr, k.classes.data(), nprobes_total * sizeof(int32_t), hipMemcpyHostToDevice,
                        c->stream));
  int *active_count = c->misc.as<int>();
  ProbeState *st = c->pstate.as<ProbeState>();
  double *part = c->partials.as<double>();

  TailArgs ta{};
  ta.sh = c->sstate.as<ShiftState>();
  ta.sigma = dsig;
  ta.nshifts = N;
  ta.ngrad = P;
  ta.tol2 = k.o.tol * k.o.tol;
  const double gt = k.o.grad_tol > 0.0 ? k.o.grad_tol : k.o.tol;
  ta.grad_tol2 = gt * gt;
  ta.max_iter = k.o.max_iter;
  ta.active_count = active_count;
  ta.part_in = part;
  ta.part_out = part;
  ta.st_in = st;
  ta.st_out = st;
  ta.need_base = P > 0;
  ta.hist = c->hist.as<double>();
  ta.hist_cap = hcap;

  PassCsr<T> a{};
  a.n = n;
  a.nslices = ntiles;
  a.ngrad = P;
  a.nq = nq;
  a.sptr = sl->sptr.as<int64_t>();
  a.col = sl->col.as<int32_t>();
  a.val = sl->val.as<double>();
  for (int i = 0; i < P; ++i) a.gval[i] = sl->gval[i].as<double>();
  a.colours = k.col.colours;
  a.rad = k.col.rad;
  a.seed = k.col.seed;
  a.uvec = k.col.uvec;
  a.st = st;
  a.part = part;

  const int check = k.o.check_every > 0 ? k.o.check_every : 16;
  int64_t passes = 0;
  bool stalled = false;
  double kernel_ms = 0.0;
  for (int attempt = 0;; ++attempt) {
    double clo, chi;
    check_interval(k.lmin, k.lmax, (int)sizeof(T), &clo, &chi);
    HIPCHK(launch_shifts(k.lmin, k.lmax, N, dsig, dcoef, c->stream));
    HIPCHK(hipMemsetAsync(c->stats.ptr, 0, 8 * sizeof(int), c->stream));
    passes = 0;
    stalled = false;
    kernel_ms = 0.0;
    bool refine = false;
    for (int first = 0; first < nprobes_total && !refine; first += block) {
      const int nb = std::min(block, nprobes_total - first);
      a.nprobes = nb;
      HIPCHK(launch_init_probes(st, nb, c->classes.as<int32_t>() + first, active_count, c->stream));
      HIPCHK(hipEventRecord(c->ev0, c->stream));
      // INIT: dots of v; FIRST: alpha_0, shifts; pass A from v; pass B
      a.r_in = a.p_in = nullptr;
      HIPCHK(launch_csr_pass_b<T>(a, W, true, c->stream));
      HIPCHK(launch_csr_tail(ta, nb, ntiles, MODE_FIRST, c->stream));
      a.r_out = bufA_r;
      a.p_out = bufA_p;
      HIPCHK(launch_csr_pass_a<T>(a, W, true, c->stream));
      a.r_in = bufA_r;
      HIPCHK(launch_csr_pass_b<T>(a, W, false, c->stream));
      passes += 1;
      bool in_a = true;
      auto chunk = [&]() -> int {
        for (int i = 0; i < check; ++i) {
          HIPCHK(launch_csr_tail(ta, nb, ntiles, MODE_STEP, c->stream));
          a.r_in = in_a ? bufA_r : bufB_r;
          a.p_in = in_a ? bufA_p : bufB_p;
          a.r_out = in_a ? bufB_r : bufA_r;
          a.p_out = in_a ? bufB_p : bufA_p;
          HIPCHK(launch_csr_pass_a<T>(a, W, false, c->stream));
          a.r_in = a.r_out;
          HIPCHK(launch_csr_pass_b<T>(a, W, false, c->stream));
          in_a = !in_a;
        }
        return LDQ_OK;
      };
      int64_t chunks = 0;
      bool st_block = false;
      CHK(poll_chunks(c, active_count, chunk, ((int64_t)k.o.max_iter + 2 * check) / check + 1, &chunks,
                      &st_block));
      passes += chunks * check;
      stalled = stalled || st_block;
      HIPCHK(hipEventRecord(c->ev1, c->stream));
      HIPCHK(hipEventSynchronize(c->ev1));
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, c->ev0, c->ev1));
      kernel_ms += ms;
      HIPCHK(launch_lanczos_check(ta.hist, st, nb, hcap, clo, chi, c->stats.as<int>(), c->stream));
      if (k.estimated && attempt < 3) {
        int viol = 0;
        HIPCHK(hipMemcpyAsync(&viol, c->stats.as<int>() + 4, sizeof viol, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        if (viol > 0) {
          // a probe saw an eigenvalue below the estimated lower end: move
          // the lower end to half the smallest Lanczos eigenvalue seen
          std::vector<ProbeState> hs(nb);
          std::vector<double> h((size_t)nb * hcap * 2);
          HIPCHK(hipMemcpyAsync(hs.data(), st, nb * sizeof(ProbeState), hipMemcpyDeviceToHost, c->stream));
          HIPCHK(hipMemcpyAsync(h.data(), ta.hist, h.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
          HIPCHK(hipStreamSynchronize(c->stream));
          double tmin = k.lmin, tmax = k.lmax;
          for (int j = 0; j < nb; ++j) {
            const int K = std::min(hs[j].active ? hs[j].iter + 1 : hs[j].iter, hcap);
            if (K < 1) continue;
            double a0, a1;
            lanczos_extremes(h.data() + (size_t)j * hcap * 2, K, &a0, &a1);
            tmin = std::min(tmin, a0);
            tmax = std::max(tmax, a1);
          }
          if (!(tmin > 0.0)) return fail(LDQ_E_NOT_SPD, "a probe's Lanczos matrix has eigenvalue %g", tmin);
          k.lmin = 0.5 * tmin;
          k.lmax = std::max(k.lmax, tmax);
          refine = true;
          break;
        }
      }
      HIPCHK(launch_probe_terms(st, ta.sh, dcoef, nb, N, P, c->terms.as<double>(), first, c->stats.as<int>(),
                                c->stream));
    }
    if (!refine) break;
  }
  if (k.estimated) {
    Q->est_lo = k.lmin;
    Q->est_hi = k.lmax;
    Q->est_ok = true;
  }
  int64_t iters_total = 0;
  CHK(collect_results(k, nprobes_total, kernel_ms, passes, info, out_sums, &iters_total));
  if (info) {
    // per probe and iteration: pass A reads r, p and writes r, p, pass B
    // reads r (the first pass A writes only); per iteration the slab once in
    // each pass and the colour array once in each pass
    const double sv = (double)sizeof(T);
    const double slots = (double)sl->nslots, idx = 8.0 * (sl->nslices + 1);
    const double slab_a = slots * (4.0 + 8.0 * (1.0 + P)) + idx, slab_b = slots * 12.0 + idx;
    info->bytes_model = sv * (double)n * (5.0 * (double)iters_total - 2.0 * (double)nprobes_total) +
                        (slab_a + slab_b + 8.0 * (double)n) * (double)passes + slab_b + 4.0 * (double)n;
  }
  return finish_status(k, stalled);
}

static int csr_bounds(ldq_ctx *c, ldq_op *Q, double *lo, double *hi) {
  if (!Q->est_ok) {
    Call k{};
    k.c = c;
    k.Q = Q;
    ldq_options_default(&k.o);
    Slab *sl = nullptr;
    CHK(csr_slab(k, &sl));
    CHK(csr_estimate<double>(k, sl, &Q->est_lo, &Q->est_hi));
    Q->est_ok = true;
  }
  *lo = Q->est_lo;
  *hi = Q->est_hi;
  return LDQ_OK;
}

static int prepare_call(Call &k, ldq_ctx *c, const ldq_op *Q, int nparams, const ldq_op *const *dQ,
                        const ldq_options *opts) {
  if (!c || !Q) return fail(LDQ_E_INVALID, "NULL argument");
  if (Q->ctx != c) return fail(LDQ_E_INVALID, "operator belongs to another context");
  if (nparams < 0 || nparams > LDQ_MAXP) return fail(LDQ_E_INVALID, "nparams must be in 0..%d", LDQ_MAXP);
  if (nparams > 0 && !dQ) return fail(LDQ_E_INVALID, "dQ is NULL");
  k.c = c;
  k.Q = const_cast<ldq_op *>(Q);
  k.nparams = nparams;
  if (opts)
    k.o = *opts;
  else
    ldq_options_default(&k.o);
  if (k.o.nshifts < 1 || k.o.nshifts > LDQ_MAXN) return fail(LDQ_E_INVALID, "nshifts must be in 1..%d", LDQ_MAXN);
  if (!(k.o.tol > 0.0) || !(k.o.grad_tol >= 0.0) || k.o.max_iter < 1)
    return fail(LDQ_E_INVALID, "tol must be > 0, grad_tol >= 0, max_iter >= 1");
  if (k.o.precision != LDQ_FP64 && k.o.precision != LDQ_MIXED) return fail(LDQ_E_INVALID, "unknown precision");
  if (k.o.colouring == LDQ_COLOUR_RADEMACHER) {
    if (k.o.nrandom < 1 || k.o.nrandom > (1 << 20)) return fail(LDQ_E_INVALID, "nrandom must be in 1..2^20");
  }
  if (k.o.lanes < 0 || k.o.lanes > LDQ_MAX_LANES)
    return fail(LDQ_E_INVALID, "lanes must be in 0..%d", LDQ_MAX_LANES);
  if (Q->kind != OPK_LATTICE && Q->kind != OPK_CSR)
    return fail(LDQ_E_UNSUPPORTED, "the Krylov passes are implemented for lattice and CSR operators");
  if (Q->kind == OPK_LATTICE && Q->ndim == 2 && nparams > 2)
    return fail(LDQ_E_UNSUPPORTED, "at most 2 derivative operators on 2-D lattices");
  for (int i = 0; i < nparams; ++i) {
    if (!dQ[i]) return fail(LDQ_E_INVALID, "dQ[%d] is NULL", i);
    if (dQ[i]->n != Q->n) return fail(LDQ_E_INVALID, "dQ[%d] has %lld rows, Q has %lld", i, (long long)dQ[i]->n,
                                      (long long)Q->n);
    if (Q->kind == OPK_CSR && dQ[i]->kind != OPK_CSR && dQ[i]->kind != OPK_DIAG)
      return fail(LDQ_E_UNSUPPORTED, "derivatives of a CSR operator must be CSR or diagonal operators");
    if (dQ[i]->kind == OPK_LATTICE && (dQ[i]->ndim != Q->ndim || dQ[i]->shape[0] != Q->shape[0] ||
                                       dQ[i]->shape[1] != Q->shape[1] || dQ[i]->shape[2] != Q->shape[2]))
      return fail(LDQ_E_INVALID, "dQ[%d] is on another lattice", i);
    if (dQ[i]->kind == OPK_OBSGRAM && (Q->kind != OPK_LATTICE || Q->ndim != 2 || !Q->obs9))
      return fail(LDQ_E_UNSUPPORTED, "an observation-gram derivative needs a 2-D Q with an observation term");
    k.dQ[i] = const_cast<ldq_op *>(dQ[i]);
  }
  CHK(set_device(c));
  // a1: colouring and its non-empty classes (a modular colouring's classes
  // are kept on the operator)
  CHK(resolve_colouring(c, Q, k.o.k, k.o.colouring, k.o.user_colours, k.o.priority, &k.col));
  const bool modular = !k.col.colours;
  if (k.o.colouring == LDQ_COLOUR_RADEMACHER) {
    // Hutchinson's estimator: probes 0 .. s - 1, every one over all sites
    k.col.rad = true;
    k.col.seed = k.o.seed;
    k.col.ncolours = k.o.nrandom;
    k.classes.resize(k.o.nrandom);
    for (int j = 0; j < k.o.nrandom; ++j) k.classes[j] = j;
  } else if (modular && Q->cls_C == k.col.C && Q->cls_a == k.col.a && Q->cls_b == k.col.b && !Q->cls.empty()) {
    k.classes = Q->cls;
  } else {
    const int C = k.col.ncolours;
    DevBuf cnt;
    CHK(cnt.reserve((size_t)C * sizeof(int)));
    HIPCHK(hipMemsetAsync(cnt.ptr, 0, (size_t)C * sizeof(int), c->stream));
    const int32_t *dcol = k.col.colours;
    if (!dcol) {
      CHK(c->colbuf.reserve(Q->n * 4));
      HIPCHK(launch_modular_fill(c->colbuf.as<int32_t>(), (int)Q->shape[0], (int)Q->shape[1],
                                 Q->ndim == 3 ? (int)Q->shape[2] : 1, k.col.C, k.col.a, k.col.b, c->stream));
      dcol = c->colbuf.as<int32_t>();
    }
    HIPCHK(launch_class_count(dcol, Q->n, C, cnt.as<int>(), c->stream));
    std::vector<int> h(C);
    HIPCHK(hipMemcpyAsync(h.data(), cnt.ptr, (size_t)C * sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    cnt.release();
    k.classes.clear();
    for (int j = 0; j < C; ++j)
      if (h[j] > 0) k.classes.push_back(j);
    if (modular) {
      ldq_op *Qm = k.Q;
      Qm->cls = k.classes;
      Qm->cls_C = k.col.C;
      Qm->cls_a = k.col.a;
      Qm->cls_b = k.col.b;
    }
  }
  // a2: enclosure
  if (k.o.lambda_min > 0.0 && k.o.lambda_max > 0.0) {
    k.lmin = k.o.lambda_min;
    k.lmax = k.o.lambda_max;
    if (!(k.lmax >= k.lmin)) return fail(LDQ_E_ENCLOSURE, "lambda_max < lambda_min");
  } else if (Q->kind == OPK_CSR) {
    // estimated by the Krylov driver (Lanczos), or the operator's last estimate
    k.lmin = Q->est_ok ? Q->est_lo : 0.0;
    k.lmax = Q->est_ok ? Q->est_hi : 0.0;
    k.estimated = true;
  } else {
    CHK(spectrum(Q, &k.lmin, &k.lmax));
  }
  return LDQ_OK;
}

// Autotuner for 2-D lattices: the tile height decides the work per wave
// (rows + halo row steps) against the number of waves and, at the standard
// height, selects the specialised pass.  Large lattices have waves to spare
// and want long tiles; small ones are latency-bound and want many short
// tiles.  Each candidate is timed over a few STEP passes of the first probe
// block; the choice is kept on the context for the problem's signature.
static int tune_rows(Call &k) {
  ldq_op *Q = k.Q;
  k.rows2d = 0;
  k.lanes = k.o.lanes > 0 ? k.o.lanes : 1;
  if (Q->ndim != 2) return LDQ_OK;
  const bool sq = Q->lkind == LDQ_SQUARED_SHIFTED_LAPLACIAN;
  if (k.o.tile_rows > 0) {
    k.rows2d = pass2d_rows(sq, k.o.tile_rows);
    return LDQ_OK;
  }
  char key[256];
  std::snprintf(key, sizeof key, "%lld,%lld,%d,%d,%d,%d,%d,%d,%d,%d,%d", (long long)Q->shape[0],
                (long long)Q->shape[1], Q->lkind, k.o.precision, k.nparams, Q->obs9 != nullptr,
                (k.col.colours != nullptr) + 2 * k.col.rad, Q->field != nullptr, (int)k.classes.size(),
                k.o.probe_block, k.o.lanes);
  auto it = k.c->tuned_rows.find(key);
  if (it != k.c->tuned_rows.end()) {
    k.rows2d = it->second % 1000;
    k.lanes = it->second / 1000;
    return LDQ_OK;
  }
  // two and three lanes are timed against one wherever a block has that many
  // probes (two measured 2-10 % faster on 512 x 512 blocks of 13 to 61 probes)
  const int nprobes = (int)k.classes.size();
  const int block = (k.o.probe_block > 0) ? std::min(k.o.probe_block, nprobes) : nprobes;
  int lane_cands[3] = {k.lanes, 0, 0};
  if (k.o.lanes == 0)
    for (int l = 2; l <= 3; ++l)
      if (block >= l) lane_cands[l - 1] = l;
  // the specialised pass's standard tile, its tall tile (FP32), and shorter
  // tiles of the general pass
  const int cands[5] = {LDQ_ROWS2D, LDQ_ROWS2D_TALL, 4, 9, 16};
  int best = 0, best_lanes = 1;
  double best_ms = 0.0;
  for (int lanes : lane_cands) {
    if (lanes == 0) continue;
    for (int want : cands) {
      const int rows = pass2d_rows(sq, want);
      if (want == LDQ_ROWS2D_TALL && (k.o.precision != LDQ_MIXED || k.col.rad)) continue;
      if (want != LDQ_ROWS2D && want != LDQ_ROWS2D_TALL && rows >= pass2d_rows(sq, LDQ_ROWS2D)) continue;
      // the faster of two timing runs of each candidate
      double ms = 0.0;
      k.rows2d = rows;
      k.lanes = lanes;
      for (int rep = 0; rep < 2; ++rep) {
        double t = 0.0;
        k.tune_ms = &t;
        const int st = (k.o.precision == LDQ_MIXED) ? run_krylov<float>(k, nullptr, nullptr)
                                                    : run_krylov<double>(k, nullptr, nullptr);
        k.tune_ms = nullptr;
        if (st != LDQ_OK) return st;
        ms = rep == 0 ? t : std::min(ms, t);
      }
      if (best == 0 || ms < best_ms) {
        best = rows;
        best_lanes = lanes;
        best_ms = ms;
      }
    }
  }
  k.rows2d = best;
  k.lanes = best_lanes;
  k.c->tuned_rows[key] = best + 1000 * best_lanes;
  return LDQ_OK;
}

// The derivative of the probing estimate with the shifts fixed (NEXT row
// f3): dE/d eta_i = -sum_j Im sum_l c_l (x^l_j)^T dQ_i x^l_j.  The shifted
// solutions x^l_j = sum_m zeta^l_m S^l_m r_m are accumulated by a second solve
// from the coefficients of the first (as for f_N(Q) v), then one bilinear form
// per (probe, shift) and derivative.  Replaces grad[0 .. nparams).
static void mat_weights(const double *h, int K, double vnorm2, double tol2, const cplx *sig, const cplx *coef, int N,
                        double *w, cplx *cc);
static int consistent_gradient(Call &k, double *grad) {
  ldq_ctx *c = k.c;
  ldq_op *Q = k.Q;
  const int nb = (int)k.classes.size();
  const int N = k.o.nshifts;
  const int64_t n = Q->n;
  const int hcap = hist_cap(nb, k.o.max_iter);
  std::vector<double> hist((size_t)nb * hcap * 2);
  std::vector<ProbeState> pst(nb);
  std::vector<cplx> sh(2 * LDQ_MAXN);
  HIPCHK(hipMemcpyAsync(hist.data(), c->hist.ptr, hist.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipMemcpyAsync(pst.data(), c->pstate.as<ProbeState>() + nb, nb * sizeof(ProbeState), hipMemcpyDeviceToHost,
                        c->stream));
  HIPCHK(hipMemcpyAsync(sh.data(), c->shifts.ptr, sh.size() * sizeof(cplx), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  int kmax = 1;
  for (const ProbeState &p : pst) kmax = std::max(kmax, p.iter);
  if (kmax > hcap) return fail(LDQ_E_UNSUPPORTED, "%d iterations exceed the %d the coefficient history holds", kmax, hcap);
  const int cstride = (kmax + 1) * N;
  std::vector<cplx> cc((size_t)nb * cstride, cmk(0.0, 0.0));
  std::vector<double> w(kmax + 1);
  for (int j = 0; j < nb; ++j)
    mat_weights(hist.data() + (size_t)j * hcap * 2, pst[j].iter, pst[j].vnorm2, k.o.tol * k.o.tol, sh.data(),
                sh.data() + LDQ_MAXN, N, w.data(), cc.data() + (size_t)j * cstride);
  CHK(c->matc.reserve(cc.size() * sizeof(cplx)));
  CHK(c->matz.reserve((size_t)nb * N * (size_t)n * sizeof(cplx)));
  CHK(c->matq.reserve((size_t)nb * N * sizeof(cplx)));
  HIPCHK(hipMemcpyAsync(c->matc.ptr, cc.data(), cc.size() * sizeof(cplx), hipMemcpyHostToDevice, c->stream));
  Call k2 = k;
  k2.mat_c = c->matc.as<cplx>();
  k2.mat_cstride = cstride;
  k2.mat_z = c->matz.as<cplx>();
  k2.mat_steps = kmax;
  double sums[1 + LDQ_MAXP];
  const int st = (k.o.precision == LDQ_MIXED) ? run_krylov<float>(k2, nullptr, sums) : run_krylov<double>(k2, nullptr, sums);
  if (st != LDQ_OK && st != LDQ_E_NO_CONVERGENCE) return st;
  std::vector<cplx> q((size_t)nb * N);
  for (int i = 0; i < k.nparams; ++i) {
    const ldq_op *d = k.dQ[i];
    const bool diag = d->kind == OPK_DIAG, gram = d->kind == OPK_OBSGRAM;
    // scales as the passes apply them (an observation gram carries its weight in tau)
    HIPCHK(launch_lattice_bilinear(c->matz.as<cplx>(), nb * N, (int)Q->shape[0], (int)Q->shape[1],
                                   Q->ndim == 3 ? (int)Q->shape[2] : 1, diag, gram ? d->tau : d->scale,
                                   diag || gram ? 0.0 : d->kappa2, gram ? nullptr : d->field,
                                   gram ? d->obs9 : nullptr, c->matq.as<cplx>(), c->stream));
    HIPCHK(hipMemcpyAsync(q.data(), c->matq.ptr, q.size() * sizeof(cplx), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    double g = 0.0;
    for (int j = 0; j < nb; ++j)
      for (int l = 0; l < N; ++l) {
        const cplx a = sh[LDQ_MAXN + l], z = q[(size_t)j * N + l];
        g -= a.re * z.im + a.im * z.re;   // Im(a z)
      }
    grad[i] = g;
  }
  return LDQ_OK;
}

static int logdet_impl(ldq_ctx *c, const ldq_op *Q, int nparams, const ldq_op *const *dQ, const ldq_options *opts,
                       double *logdet, double *grad, ldq_info *info) {
  auto t0 = std::chrono::steady_clock::now();
  Call k{};
  CHK(prepare_call(k, c, Q, nparams, dQ, opts));
  const bool consistent = k.o.consistent_grad && nparams > 0;
  if (consistent) {
    if (k.Q->kind != OPK_LATTICE) return fail(LDQ_E_UNSUPPORTED, "the consistent gradient needs a lattice Q");
    for (int i = 0; i < nparams; ++i) {
      const ldq_op *d = k.dQ[i];
      if (!(d->kind == OPK_DIAG || (d->kind == OPK_LATTICE && d->lkind == LDQ_SHIFTED_LAPLACIAN) ||
            (d->kind == OPK_OBSGRAM && k.Q->ndim == 2 && d->obs9)))
        return fail(LDQ_E_UNSUPPORTED,
                    "the consistent gradient takes diagonal, shifted-Laplacian or observation-gram derivatives");
    }
    k.o.probe_block = 0;   // one block: its coefficient history covers every probe
  }
  double sums[1 + LDQ_MAXP] = {};
  ldq_info tmp{};
  int st;
  if (k.Q->kind == OPK_CSR) {
    st = (k.o.precision == LDQ_MIXED) ? run_krylov_csr<float>(k, &tmp, sums) : run_krylov_csr<double>(k, &tmp, sums);
  } else {
    CHK(tune_rows(k));
    if (consistent) k.lanes = 1;
    st = (k.o.precision == LDQ_MIXED) ? run_krylov<float>(k, &tmp, sums) : run_krylov<double>(k, &tmp, sums);
  }
  if (st != LDQ_OK && st != LDQ_E_NO_CONVERGENCE) return st;
  if (consistent && st == LDQ_OK) CHK(consistent_gradient(k, sums + 1));
  if (k.col.rad) {
    // Hutchinson's estimator: the mean over the s probes, and the standard
    // error of that mean from the per-probe terms
    const int s = (int)k.classes.size();
    for (int i = 0; i <= nparams; ++i) sums[i] /= s;
    double m = 0.0, ss = 0.0;
    for (int j = 0; j < s; ++j) m += c->last_terms[(size_t)j * (1 + nparams)];
    m /= s;
    for (int j = 0; j < s; ++j) {
      const double d = c->last_terms[(size_t)j * (1 + nparams)] - m;
      ss += d * d;
    }
    tmp.std_error = s > 1 ? std::sqrt(ss / (s - 1) / s) : INFINITY;
  }
  if (logdet) *logdet = sums[0];
  if (grad)
    for (int i = 0; i < nparams; ++i) grad[i] = sums[1 + i];
  tmp.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (info) *info = tmp;
  return st;
}

extern "C" int ldq_logdet(ldq_ctx *c, const ldq_op *Q, const ldq_options *opts, double *logdet, ldq_info *info) {
  if (!logdet) return fail(LDQ_E_INVALID, "logdet is NULL");
  return logdet_impl(c, Q, 0, nullptr, opts, logdet, nullptr, info);
}

extern "C" int ldq_logdet_grad(ldq_ctx *c, const ldq_op *Q, int nparams, const ldq_op *const *dQ,
                               const ldq_options *opts, double *logdet, double *grad, ldq_info *info) {
  if (!logdet || (nparams > 0 && !grad)) return fail(LDQ_E_INVALID, "NULL output");
  return logdet_impl(c, Q, nparams, dQ, opts, logdet, grad, info);
}

// ------------------------------------------------ f_N(Q) v itself (NEXT row f3)
// The shifted solutions are combinations of the base CG's residuals (Sec. 2.1,
// last paragraph: the shifted iterates follow from the base scalars):
// p^s_0 = r_0, p^s_{k+1} = zeta^s_{k+1} r_{k+1} + beta^s_k p^s_k and
// x^s = sum_{k < F} alpha^s_k p^s_k, so x^s = sum_m zeta^s_m S^s_m r_m with
// S^s_m = alpha^s_m + beta^s_m S^s_{m+1}, S^s_F = 0 (F: the terms the shift took
// before it froze).  Hence f_N(Q) v = Im sum_l a_l x^{s_l} = sum_m w_m r_m with
// real weights w_m = Im sum_l a_l zeta^{s_l}_m S^{s_l}_m, computed here from the
// recorded alpha_k, beta_k of a first solve with the same freezing rule as the
// device; a second, identical solve accumulates the sum.
static void mat_weights(const double *h, int K, double vnorm2, double tol2, const cplx *sig, const cplx *coef, int N,
                        double *w, cplx *cc = nullptr) {
  std::vector<double> alpha(K), beta(std::max(K - 1, 0));
  for (int m = 0; m < K; ++m) alpha[m] = h[2 * m];
  for (int m = 0; m + 1 < K; ++m) beta[m] = h[2 * (m + 1) + 1];
  std::vector<double> gamma(K + 1);
  gamma[0] = vnorm2;
  for (int m = 0; m + 1 < K; ++m) gamma[m + 1] = gamma[m] * beta[m];
  for (int m = 0; m < K; ++m) w[m] = 0.0;
  if (cc)
    for (int m = 0; m < K * N; ++m) cc[m] = cmk(0.0, 0.0);
  using C = std::complex<double>;
  std::vector<C> zeta(K), as(K), bs(K);
  for (int l = 0; l < N; ++l) {
    const C s(sig[l].re, sig[l].im), a(coef[l].re, coef[l].im);
    C z = 1.0, zp = 1.0;
    double akm1 = 1.0, bkm1 = 0.0;
    int F = 0;
    for (int k = 0; k < K; ++k) {
      const double ak = alpha[k];
      const C den = (zp - z) * (ak * bkm1) + zp * akm1 * (1.0 - s * ak);
      const C zn = z * zp * akm1 / den;
      const C ratio = zn / z;
      zeta[k] = z;
      as[k] = ratio * ak;
      F = k + 1;
      if (k + 1 >= K) break;
      bs[k] = ratio * ratio * beta[k];
      if (std::norm(zn) * gamma[k + 1] <= tol2 * vnorm2) break;   // frozen after this term
      zp = z;
      z = zn;
      akm1 = ak;
      bkm1 = beta[k];
    }
    C S = 0.0;
    for (int m = F - 1; m >= 0; --m) {
      S = as[m] + (m + 1 < F ? bs[m] * S : C(0.0));
      w[m] += std::imag(a * zeta[m] * S);
      if (cc) cc[(size_t)m * N + l] = cmk(std::real(zeta[m] * S), std::imag(zeta[m] * S));
    }
  }
}

// The base system alone (sigma = 0: zeta = 1, alpha^s = alpha, beta^s = beta):
// Q^{-1} v = x_K = sum_{m < K} S_m r_m with S_m = alpha_m + beta_m S_{m+1},
// S_K = 0, over every iteration the probe ran (the base system met its
// tolerance by then: the solve forces it).
static void base_weights(const double *h, int K, double *w) {
  double S = 0.0;
  for (int m = K - 1; m >= 0; --m) {
    S = h[2 * m] + (m + 1 < K ? h[2 * (m + 1) + 1] * S : 0.0);
    w[m] = S;
  }
}

// Y = f_N(Q) V (inverse = false) or Q^{-1} V (inverse = true) by two
// identical solves: the first records the base coefficients, the host forms
// the residual weights, the second accumulates Y.
static int materialise(ldq_ctx *c, const ldq_op *Q, int nvec, const double *V, double *Y, const ldq_options *opts,
                       ldq_info *info, bool inverse) {
  if (!c || !Q || nvec < 1 || !V || !Y) return fail(LDQ_E_INVALID, "invalid arguments");
  if (Q->kind != OPK_LATTICE)
    return fail(LDQ_E_UNSUPPORTED, "%s is implemented for lattice operators", inverse ? "Q^-1 v" : "f_N(Q) v");
  CHK(set_device(c));
  // V and Y are read and written by kernels: device (or managed) memory only
  for (const void *ptr : {(const void *)V, (const void *)Y}) {
    hipPointerAttribute_t at{};
    const hipError_t e = hipPointerGetAttributes(&at, ptr);
    if (e != hipSuccess || (at.type != hipMemoryTypeDevice && at.type != hipMemoryTypeManaged)) {
      (void)hipGetLastError();
      return fail(LDQ_E_INVALID, "V and Y must be device memory");
    }
  }
  ldq_options o;
  if (opts)
    o = *opts;
  else
    ldq_options_default(&o);
  // the given vectors are probes 0 .. nvec - 1 of one block, in one chain
  o.colouring = LDQ_COLOUR_RADEMACHER;
  o.nrandom = nvec;
  o.probe_block = 0;
  o.lanes = 1;
  Call k{};
  CHK(prepare_call(k, c, Q, 0, nullptr, &o));
  k.col.rad = false;
  k.col.uvec = V;
  k.force_base = inverse;
  CHK(tune_rows(k));
  k.lanes = 1;
  double sums[1 + LDQ_MAXP] = {};
  ldq_info first{};
  int st = (k.o.precision == LDQ_MIXED) ? run_krylov<float>(k, &first, sums) : run_krylov<double>(k, &first, sums);
  if (st != LDQ_OK) return st;
  // the first solve's coefficients, final states and shifts
  const int hcap = hist_cap(nvec, k.o.max_iter);
  std::vector<double> hist((size_t)nvec * hcap * 2);
  std::vector<ProbeState> pst(nvec);
  std::vector<cplx> sh(2 * LDQ_MAXN);
  HIPCHK(hipMemcpyAsync(hist.data(), c->hist.ptr, hist.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipMemcpyAsync(pst.data(), c->pstate.as<ProbeState>() + nvec, nvec * sizeof(ProbeState),
                        hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipMemcpyAsync(sh.data(), c->shifts.ptr, sh.size() * sizeof(cplx), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  int kmax = 1;
  for (const ProbeState &p : pst) kmax = std::max(kmax, p.iter);
  if (kmax > hcap) return fail(LDQ_E_UNSUPPORTED, "%d iterations exceed the %d the coefficient history holds", kmax, hcap);
  const int ws = kmax + 1;
  std::vector<double> w((size_t)nvec * ws, 0.0);
  for (int j = 0; j < nvec; ++j) {
    if (inverse)
      base_weights(hist.data() + (size_t)j * hcap * 2, pst[j].iter, w.data() + (size_t)j * ws);
    else
      mat_weights(hist.data() + (size_t)j * hcap * 2, pst[j].iter, pst[j].vnorm2, k.o.tol * k.o.tol, sh.data(),
                  sh.data() + LDQ_MAXN, k.o.nshifts, w.data() + (size_t)j * ws);
  }
  CHK(c->matw.reserve(w.size() * sizeof(double)));
  HIPCHK(hipMemcpyAsync(c->matw.ptr, w.data(), w.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
  // the second, identical solve accumulates y
  Call k2 = k;
  k2.mat_w = c->matw.as<double>();
  k2.mat_wstride = ws;
  k2.mat_steps = kmax;
  k2.mat_y = Y;
  st = (k.o.precision == LDQ_MIXED) ? run_krylov<float>(k2, nullptr, sums) : run_krylov<double>(k2, nullptr, sums);
  if (st != LDQ_OK && st != LDQ_E_NO_CONVERGENCE) return st;
  HIPCHK(hipStreamSynchronize(c->stream));
  if (info) *info = first;
  return LDQ_OK;
}

extern "C" int ldq_logm_apply(ldq_ctx *c, const ldq_op *Q, int nvec, const double *V, double *Y,
                              const ldq_options *opts, ldq_info *info) {
  return materialise(c, Q, nvec, V, Y, opts, info, false);
}

extern "C" int ldq_solve(ldq_ctx *c, const ldq_op *Q, int nvec, const double *B, double *X, const ldq_options *opts,
                         ldq_info *info) {
  return materialise(c, Q, nvec, B, X, opts, info, true);
}

extern "C" int ldq_probe_terms(ldq_ctx *c, double *out, int64_t capacity, int64_t *count, int *nparams) {
  if (!c || !count || !nparams) return fail(LDQ_E_INVALID, "NULL argument");
  *count = c->last_count;
  *nparams = c->last_nparams;
  const int64_t need = c->last_count * (1 + c->last_nparams);
  if (out) {
    if (capacity < need) return fail(LDQ_E_INVALID, "capacity %lld < %lld", (long long)capacity, (long long)need);
    std::memcpy(out, c->last_terms.data(), need * sizeof(double));
  }
  return LDQ_OK;
}

// ------------------------------------------------- many lattices at once
// The batched STEP launches need every field to be a 2-D lattice of the same
// kind with a constant shift, scale 1, no observation term and a modular
// colouring of the same (C, a); derivative operators (at most one per field)
// shifted Laplacians with a constant shift.
static bool batchable(const std::vector<Call> &calls) {
  if (calls.empty()) return false;
  const Call &k0 = calls[0];
  if (k0.nparams > 1) return false;
  for (const Call &k : calls) {
    const ldq_op *Q = k.Q;
    if (Q->kind != OPK_LATTICE || Q->ndim != 2 || Q->field || Q->obs9 || Q->scale != 1.0) return false;
    if (Q->lkind != k0.Q->lkind) return false;
    if (k.col.colours || k.col.rad || k.col.C != k0.col.C || k.col.a != k0.col.a) return false;
    if (k.nparams != k0.nparams) return false;
    if (k.nparams == 1) {
      const ldq_op *d = k.dQ[0];
      if (d->kind != OPK_LATTICE || d->lkind != LDQ_SHIFTED_LAPLACIAN || d->field || d->scale != k0.dQ[0]->scale)
        return false;
    }
    if ((double)Q->n * 8.0 >= 4294967295.0) return false;
  }
  return true;
}

template <typename T>
static int run_batched(ldq_ctx *c, std::vector<Call> &calls, double *logdet, double *grad, ldq_info *info) {
  const int nf = (int)calls.size();
  const Call &k0 = calls[0];
  const int P = k0.nparams;
  const int N = k0.o.nshifts;
  const int nq = LDQ_NQ_BASE + P;
  const bool sq = k0.Q->lkind == LDQ_SQUARED_SHIFTED_LAPLACIAN;
  // the batched pass runs the standard tile or, in FP32, the tall one
  const bool tall = sizeof(T) == 4 && k0.rows2d == pass2d_rows(sq, LDQ_ROWS2D_TALL);
  const int rows = pass2d_rows(sq, tall ? LDQ_ROWS2D_TALL : LDQ_ROWS2D);
  std::vector<FieldDesc> fd(nf);
  std::vector<int32_t> item_field, classes;
  int64_t vec_tot = 0, part_tot = 0, work_max = 0;
  int items = 0;
  for (int f = 0; f < nf; ++f) {
    const Call &k = calls[f];
    const int nb = (int)k.classes.size();
    int tx = 0, nt = 0;
    pass2d_tiles((int)k.Q->shape[0], (int)k.Q->shape[1], sq, rows, &tx, &nt);
    fd[f] = FieldDesc{(int)k.Q->shape[0], (int)k.Q->shape[1], tx, nt, nb, items, vec_tot, part_tot, k.Q->kappa2,
                      P ? k.dQ[0]->kappa2 : 0.0};
    items += nb;
    vec_tot += (int64_t)nb * k.Q->n;
    part_tot += (int64_t)nb * nq * nt;
    work_max += (int64_t)nb * nt;
    for (int j = 0; j < nb; ++j) {
      item_field.push_back(f);
      classes.push_back(k.classes[j]);
    }
  }
  if (work_max >= INT32_MAX || items == 0) return fail(LDQ_E_UNSUPPORTED, "batch too large for one work list");
  const int hcap = hist_cap(items, k0.o.max_iter);
  CHK(c->vec.reserve(4 * (size_t)vec_tot * sizeof(T)));
  CHK(c->partials.reserve(2 * (size_t)part_tot * sizeof(double)));
  CHK(c->pstate.reserve(2 * (size_t)items * sizeof(ProbeState)));
  CHK(c->sstate.reserve((size_t)items * N * sizeof(ShiftState)));
  CHK(c->hist.reserve((size_t)items * hcap * 2 * sizeof(double)));
  CHK(c->shifts.reserve((size_t)nf * 2 * LDQ_MAXN * sizeof(cplx)));
  CHK(c->classes.reserve((size_t)items * sizeof(int32_t)));
  CHK(c->terms.reserve((size_t)items * (1 + P) * sizeof(double)));
  CHK(c->stats.reserve((size_t)nf * 8 * sizeof(int)));
  CHK(c->sums.reserve((size_t)nf * (1 + P) * sizeof(double)));
  CHK(c->misc.reserve(8 * sizeof(int)));
  CHK(c->bfields.reserve((size_t)nf * sizeof(FieldDesc)));
  CHK(c->bitems.reserve((size_t)items * sizeof(int32_t)));
  CHK(c->bwork.reserve((size_t)work_max * sizeof(WorkItem)));
  T *vec = c->vec.as<T>();
  T *bufA_r = vec, *bufA_p = vec + vec_tot, *bufB_r = vec + 2 * vec_tot, *bufB_p = vec + 3 * vec_tot;
  cplx *sig = c->shifts.as<cplx>(), *coef = sig + (size_t)nf * LDQ_MAXN;
  double *part[2] = {c->partials.as<double>(), c->partials.as<double>() + part_tot};
  ProbeState *st[2] = {c->pstate.as<ProbeState>(), c->pstate.as<ProbeState>() + items};
  int *counter = c->misc.as<int>();          // work-list length
  int *dummy_active = counter + 1;           // the per-probe countdown is not used here
  HIPCHK(hipMemcpyAsync(c->bfields.ptr, fd.data(), nf * sizeof(FieldDesc), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(c->bitems.ptr, item_field.data(), items * sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(c->classes.ptr, classes.data(), items * sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemsetAsync(c->stats.ptr, 0, (size_t)nf * 8 * sizeof(int), c->stream));
  for (int f = 0; f < nf; ++f)
    HIPCHK(launch_shifts(calls[f].lmin, calls[f].lmax, N, sig + (size_t)f * LDQ_MAXN, coef + (size_t)f * LDQ_MAXN,
                         c->stream));
  HIPCHK(launch_init_probes(st[0], items, c->classes.as<int32_t>(), dummy_active, c->stream));

  TailArgs ta{};
  ta.sh = c->sstate.as<ShiftState>();
  ta.nshifts = N;
  ta.ngrad = P;
  ta.tol2 = k0.o.tol * k0.o.tol;
  const double gt = k0.o.grad_tol > 0.0 ? k0.o.grad_tol : k0.o.tol;
  ta.grad_tol2 = gt * gt;
  ta.max_iter = k0.o.max_iter;
  ta.active_count = dummy_active;
  ta.need_base = P > 0;
  ta.hist = c->hist.as<double>();
  ta.hist_cap = hcap;

  HIPCHK(hipEventRecord(c->ev0, c->stream));
  // INIT and FIRST, one field at a time (the single-lattice generic pass on the
  // field's slice of every buffer)
  for (int f = 0; f < nf; ++f) {
    const FieldDesc &d = fd[f];
    Pass2D<T> a{};
    a.nx = d.nx;
    a.ny = d.ny;
    a.tiles_x = d.tiles_x;
    a.ntiles = d.ntiles;
    a.rows = rows;
    a.nprobes = d.nprobes;
    a.colC = k0.col.C;
    a.cola = k0.col.a;
    a.kappa2 = d.kappa2;
    a.scale = 1.0;
    if (P) {
      a.grad[0].kind = GK_SHIFTED;
      a.grad[0].scale = k0.dQ[0]->scale;
      a.grad[0].kappa2 = d.kd;
    }
    TailArgs t = ta;
    t.sh = ta.sh + (size_t)d.item_base * N;
    t.sigma = sig + (size_t)f * LDQ_MAXN;
    t.hist = ta.hist + (size_t)d.item_base * hcap * 2;
    for (int mode : {(int)MODE_INIT, (int)MODE_FIRST}) {
      t.st_in = st[0] + d.item_base;
      t.st_out = st[1] + d.item_base;
      t.part_in = part[0] + d.part_off;
      t.part_out = (mode == MODE_INIT ? part[0] : part[1]) + d.part_off;
      a.tail = t;
      a.mode = mode;
      a.r_in = a.p_in = nullptr;
      a.r_out = mode == MODE_INIT ? nullptr : bufA_r + d.vec_off;
      a.p_out = mode == MODE_INIT ? nullptr : bufA_p + d.vec_off;
      HIPCHK(launch_pass2d<T>(a, sq, false, false, c->stream));
    }
  }
  Batch2D<T> b{};
  b.work = c->bwork.as<WorkItem>();
  b.count = counter;
  b.fields = c->bfields.as<FieldDesc>();
  b.sigma = sig;
  b.rows = rows;
  b.colC = k0.col.C;
  b.cola = k0.col.a;
  b.gscale = P ? k0.dQ[0]->scale : 0.0;
  b.tail = ta;
  // work list from the states in st[1]; stopped items' states go to st[0] too
  auto compact = [&](int *h_count) -> int {
    HIPCHK(hipMemsetAsync(counter, 0, sizeof(int), c->stream));
    HIPCHK(launch_batch_compact(c->bfields.as<FieldDesc>(), c->bitems.as<int32_t>(), items, st[1], st[0],
                                c->bwork.as<WorkItem>(), counter, c->stream));
    HIPCHK(hipMemcpyAsync(h_count, counter, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return LDQ_OK;
  };
  HIPCHK(hipEventRecord(c->ev1, c->stream));
  int nwork = 0;
  CHK(compact(&nwork));
  double kernel_ms = 0.0;
  {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    kernel_ms += ms;
  }
  const int check = k0.o.check_every > 0 ? 2 * ((k0.o.check_every + 1) / 2) : 16;
  int64_t launches = 2 * (int64_t)nf, steps = 0;
  int64_t tiles_run = 0;
  bool stalled = false;
  // A chunk of passes over the work list: replayed from a graph captured for a
  // grid of `grid` workgroups, which serves while the list (whose live length
  // the kernel reads from the device) is between half that and that long;
  // below half, the chunk is captured again with the current length.
  const bool graphs = k0.o.launch_mode != LDQ_LAUNCH_DIRECT;
  int grid = 0;
  auto chunk_steps = [&](hipStream_t s) -> int {
    for (int i = 0; i < check; ++i) {
      const int in = (i % 2 == 0) ? 1 : 0;
      b.tail.st_in = st[in];
      b.tail.st_out = st[1 - in];
      b.tail.part_in = part[in];
      b.tail.part_out = part[1 - in];
      b.r_in = in ? bufA_r : bufB_r;
      b.p_in = in ? bufA_p : bufB_p;
      b.r_out = in ? bufB_r : bufA_r;
      b.p_out = in ? bufB_p : bufA_p;
      const hipError_t e = launch_batch2d<T>(b, grid, sq, P, s);
      if (e != hipSuccess) return fail(LDQ_E_DEVICE, "batched pass launch: %s", hipGetErrorString(e));
    }
    return LDQ_OK;
  };
  ChunkGraph bg;
  while (nwork > 0) {
    HIPCHK(hipEventRecord(c->ev0, c->stream));
    if (graphs) {
      if (nwork > grid || 2 * nwork < grid) {
        if (bg.exec) HIPCHK(hipGraphExecDestroy(bg.exec));
        bg.exec = nullptr;
        grid = nwork;
      }
      CHK(graph_chunk(c, bg, chunk_steps, c->stream));
    } else {
      grid = nwork;
      CHK(chunk_steps(c->stream));
    }
    HIPCHK(hipEventRecord(c->ev1, c->stream));
    launches += check;
    steps += check;
    tiles_run += (int64_t)check * nwork;
    CHK(compact(&nwork));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    kernel_ms += ms;
    if (steps > (int64_t)k0.o.max_iter + 2 * check) {
      stalled = true;
      break;
    }
  }
  // enclosure check of every probe of every field in one launch
  {
    std::vector<double> lohi(2 * (size_t)nf);
    for (int f = 0; f < nf; ++f)
      check_interval(calls[f].lmin, calls[f].lmax, (int)sizeof(T), &lohi[2 * f], &lohi[2 * f + 1]);
    CHK(c->blohi.reserve(lohi.size() * sizeof(double)));
    HIPCHK(hipMemcpyAsync(c->blohi.ptr, lohi.data(), lohi.size() * sizeof(double), hipMemcpyHostToDevice,
                          c->stream));
    HIPCHK(launch_batch_lanczos_check(ta.hist, st[1], items, hcap, c->bitems.as<int32_t>(), c->blohi.as<double>(),
                                      c->stats.as<int>(), c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));   // lohi is pageable host memory
  }
  // per field: terms and sums (fixed order)
  for (int f = 0; f < nf; ++f) {
    const FieldDesc &d = fd[f];
    int *sf = c->stats.as<int>() + (size_t)f * 8;
    double *tf = c->terms.as<double>() + (size_t)d.item_base * (1 + P);
    HIPCHK(launch_probe_terms(st[1] + d.item_base, ta.sh + (size_t)d.item_base * N, coef + (size_t)f * LDQ_MAXN,
                              d.nprobes, N, P, tf, 0, sf, c->stream));
    HIPCHK(launch_sum_terms(tf, d.nprobes, 1 + P, c->sums.as<double>() + (size_t)f * (1 + P), c->stream));
  }
  std::vector<double> sums((size_t)nf * (1 + P));
  std::vector<int> stats((size_t)nf * 8);
  HIPCHK(hipMemcpyAsync(sums.data(), c->sums.ptr, sums.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipMemcpyAsync(stats.data(), c->stats.ptr, stats.size() * sizeof(int), hipMemcpyDeviceToHost, c->stream));
  c->last_terms.resize((size_t)items * (1 + P));
  HIPCHK(hipMemcpyAsync(c->last_terms.data(), c->terms.ptr, c->last_terms.size() * sizeof(double),
                        hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  c->last_nparams = P;
  c->last_count = items;
  // algorithmic bytes per field: r and p read and written once per probe-site
  // and iteration (the first pass writes only)
  std::vector<double> bytes(nf);
  double bytes_tot = 0.0;
  int worst = 0;
  for (int f = 0; f < nf; ++f) {
    const int *sf = stats.data() + (size_t)f * 8;
    int64_t it_tot;
    std::memcpy(&it_tot, sf + 2, sizeof it_tot);
    const double n = (double)fd[f].nx * fd[f].ny;
    bytes[f] = (double)sizeof(T) * n * (4.0 * (double)it_tot - 2.0 * fd[f].nprobes);
    bytes_tot += bytes[f];
    worst = std::max(worst, sf[0]);
    logdet[f] = sums[(size_t)f * (1 + P)];
    for (int i = 0; i < P; ++i) grad[(size_t)f * P + i] = sums[(size_t)f * (1 + P) + 1 + i];
  }
  if (info) {
    for (int f = 0; f < nf; ++f) {
      const int *sf = stats.data() + (size_t)f * 8;
      ldq_info &o = info[f];
      o = ldq_info{};
      o.ncolours = fd[f].nprobes;
      o.iters_max = sf[1];
      std::memcpy(&o.iters_total, sf + 2, sizeof o.iters_total);
      o.lambda_min = calls[f].lmin;
      o.lambda_max = calls[f].lmax;
      uint64_t rb;
      std::memcpy(&rb, sf + 6, sizeof rb);
      o.max_rel_residual = __builtin_bit_cast(double, rb);
      o.enclosure_violations = sf[4];
      // the launches are shared: each field gets the share of the device time
      // of its algorithmic bytes, and the batch's launch count
      o.loop_seconds = bytes_tot > 0.0 ? kernel_ms * 1e-3 * bytes[f] / bytes_tot : 0.0;
      o.passes = launches;
      o.probe_passes = o.iters_total;
      o.bytes_model = bytes[f];
      o.lanes = 1;
      o.tile_rows = rows;
    }
  }
  (void)tiles_run;
  if (stalled) return fail(LDQ_E_NO_CONVERGENCE, "probes did not stop within max_iter");
  if (worst == 2) return fail(LDQ_E_NOT_SPD, "the Krylov recurrence met p^T Q p <= 0 or a non-finite value");
  if (worst == 3) return fail(LDQ_E_NO_CONVERGENCE, "max_iter = %d reached before every shift converged",
                              k0.o.max_iter);
  return LDQ_OK;
}

extern "C" int ldq_logdet_batched(ldq_ctx *c, int nfields, const ldq_op *const *Q, int nparams,
                                  const ldq_op *const *dQ, const ldq_options *opts, double *logdet, double *grad,
                                  ldq_info *info) {
  if (!c || nfields < 0 || (nfields > 0 && (!Q || !logdet)) || (nparams > 0 && (!dQ || !grad)))
    return fail(LDQ_E_INVALID, "invalid batched arguments");
  if (nfields == 0) return LDQ_OK;
  {
    // one set of batched launches when every field qualifies
    auto t0 = std::chrono::steady_clock::now();
    std::vector<Call> calls(nfields);
    bool ok = true;
    for (int f = 0; f < nfields && ok; ++f) {
      CHK(prepare_call(calls[f], c, Q[f], nparams, nparams ? dQ + (size_t)f * nparams : nullptr, opts));
      ok = calls[f].o.precision == calls[0].o.precision;
    }
    if (ok && batchable(calls)) {
      // tile height: the option when it names the standard or the tall tile
      if (calls[0].o.tile_rows > 0)
        calls[0].rows2d = pass2d_rows(calls[0].Q->lkind == LDQ_SQUARED_SHIFTED_LAPLACIAN, calls[0].o.tile_rows);
      const int st = calls[0].o.precision == LDQ_MIXED ? run_batched<float>(c, calls, logdet, grad, info)
                                                       : run_batched<double>(c, calls, logdet, grad, info);
      const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      if (info)
        for (int f = 0; f < nfields; ++f) info[f].seconds = secs;
      return st;
    }
  }
  int worst = LDQ_OK;
  for (int f = 0; f < nfields; ++f) {
    int st = logdet_impl(c, Q[f], nparams, nparams ? dQ + (size_t)f * nparams : nullptr, opts, logdet + f,
                         nparams ? grad + (size_t)f * nparams : nullptr, info ? info + f : nullptr);
    if (st != LDQ_OK && st != LDQ_E_NO_CONVERGENCE) return st;
    if (st != LDQ_OK) worst = st;
  }
  return worst;
}
