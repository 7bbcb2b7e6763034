/*
 * ldq.h -- C ABI of the MI355X (gfx950) probing / multi-shift Krylov
 * log-determinant library.
 *
 * Method (Aune & Simpson, "Parameter Estimation in High Dimensional Gaussian
 * Distributions", arXiv 1105.5256):
 *   * log det Q = tr log Q (Sec. 2.1, eq. (5));
 *   * tr log Q ~ sum_j v_j^T log(Q) v_j with probing vectors v_j, the 0/1
 *     indicators of the colour classes of a distance-k colouring of the graph
 *     of Q (Sec. 2.1, probing paragraph);
 *   * log(Q) v_j ~ sum_l c_l (Q - sigma_l I)^{-1} v_j, a contour-quadrature
 *     rational approximation that needs an enclosure [lambda_min, lambda_max]
 *     of the spectrum (Sec. 2.1, eq. (7));
 *   * all shifted systems of one probe are solved by one conjugate-gradient
 *     recurrence with per-shift scalar coefficients (CG-M / COCG-M, Sec. 2.1,
 *     last paragraph).
 * The gradient d log det Q / d eta = tr(Q^{-1} dQ/d eta) needed by the
 * hyperparameter optimisation of Sec. 1 (eq. (4)) and Sec. 3 is estimated by
 * probing as sum_j x_j^T (dQ/d eta) v_j with x_j = Q^{-1} v_j from the same
 * Krylov run (the paper gives no gradient; this is the library's reading).
 *
 * Conventions (every entry point):
 *   * Every call returns an ldq_status; nothing is thrown across the ABI and
 *     the process is never terminated.  On failure ldq_last_error() holds a
 *     human-readable detail (thread-local, valid until the next call on the
 *     same thread).
 *   * Output arguments are written only on LDQ_OK, except that
 *     LDQ_E_NO_CONVERGENCE still writes the current estimate and the info.
 *   * Pointers are host pointers unless an argument says otherwise or
 *     LDQ_FLAG_DEVICE_PTR is passed.  Host inputs are copied before the call
 *     returns; the caller keeps ownership.  Device inputs (flag set) are
 *     borrowed and must stay valid until the object that borrows them is
 *     destroyed.  The context owns every device allocation it makes.
 *   * Work is enqueued on the context's HIP stream; calls that return scalars
 *     block until those scalars are on the host.
 *   * A context must not be used by two threads at the same time.
 *   * Lattice sites are numbered s = x + nx * (y + ny * z) (x fastest).
 */
#ifndef LDQ_H
#define LDQ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LDQ_OK = 0,
  LDQ_E_INVALID = 1,         /* an argument is out of range or inconsistent */
  LDQ_E_NOT_SPD = 2,         /* the Krylov run met p^T Q p <= 0 or a non-finite value */
  LDQ_E_NO_CONVERGENCE = 3,  /* max_iter reached; current estimate and info are written */
  LDQ_E_ENCLOSURE = 4,       /* the spectrum enclosure is invalid (lambda_min <= 0, ...) */
  LDQ_E_DEVICE = 5,          /* a HIP runtime call failed */
  LDQ_E_NO_MEMORY = 6,       /* a device or host allocation failed */
  LDQ_E_UNSUPPORTED = 7      /* a valid request this library does not implement */
} ldq_status;

/* Name of a status code (static string). */
const char *ldq_status_string(int status);
/* Detail of the last failure on the calling thread ("" if none). */
const char *ldq_last_error(void);

/* ---------------------------------------------------------------- context */

typedef struct ldq_ctx ldq_ctx;

/* Create a context on HIP device `device`, enqueuing on `hip_stream`
 * (a hipStream_t; NULL = the default stream).  *out receives the handle. */
int ldq_create(int device, void *hip_stream, ldq_ctx **out);
/* Release the context and all device memory it owns (NULL is ignored).
 * Operators created on it must be destroyed first. */
void ldq_destroy(ldq_ctx *ctx);
/* Change the stream later calls enqueue on (NULL = default stream). */
int ldq_set_stream(ldq_ctx *ctx, void *hip_stream);

/* -------------------------------------------------------------- operators */

typedef struct ldq_op ldq_op;

/* Lattice operator kinds (Sec. 3: the SPDE precision on a regular lattice). */
enum {
  LDQ_SHIFTED_LAPLACIAN = 1,         /* M = diag(kappa2) + L: 5-point (2-D) or 7-point (3-D) */
  LDQ_SQUARED_SHIFTED_LAPLACIAN = 2  /* M @ M with constant kappa2: the 13-point 2-D operator */
};
enum { LDQ_FLAG_DEVICE_PTR = 1 };    /* array arguments are device pointers (borrowed) */

/* scale * (kappa2 I + L)^p on an ndim-dimensional box shape[0..ndim-1]
 * (ndim = 2 or 3; every extent >= 1) with Dirichlet boundary: values outside
 * the box are zero, so boundary rows keep the full diagonal.
 *   kind          LDQ_SHIFTED_LAPLACIAN or LDQ_SQUARED_SHIFTED_LAPLACIAN (ndim = 2 only)
 *   kappa2        constant shift (used when kappa2_field is NULL)
 *   kappa2_field  NULL, or n = prod(shape) per-site values of kappa2 (SHIFTED only)
 *   scale         factor applied to the whole operator (e.g. 2 for dQ/dkappa2 = 2M)
 *   flags         0 or LDQ_FLAG_DEVICE_PTR (then kappa2_field is a device pointer) */
int ldq_op_lattice(ldq_ctx *ctx, int ndim, const int64_t *shape, int kind, double kappa2,
                   const double *kappa2_field, double scale, unsigned flags, ldq_op **out);

/* General sparse symmetric operator in CSR form (n rows, nnz entries,
 * rowptr[n + 1], colind[nnz] (int32, strictly ascending within a row),
 * val[nnz] FP64).  The matrix must be symmetric; host arrays are validated
 * and copied, LDQ_FLAG_DEVICE_PTR arrays are borrowed unchecked and must keep
 * their values while the operator lives.  Its log det runs the general sparse
 * passes: the rows in slices of 64 with the union of the patterns of Q and of
 * the call's derivative operators (CSR or diagonal), values kept in FP64 in
 * both precisions (only the Krylov vectors are FP32 in LDQ_MIXED). */
int ldq_op_csr(ldq_ctx *ctx, int64_t n, int64_t nnz, const int32_t *rowptr, const int32_t *colind,
               const double *val, unsigned flags, ldq_op **out);

/* Diagonal operator diag(d), d[n]. */
int ldq_op_diag(ldq_ctx *ctx, int64_t n, const double *d, unsigned flags, ldq_op **out);

/* Gauss-linear observation term (Sec. 1, eq. (1) and the posterior precision
 * Q_p = Q_x + A^T Q_1 A with Q_1 = tau I).  A has nobs rows; row o has the
 * four entries weight[4 o + c] in columns corner[4 o + c] (c = 0..3), which
 * must be sites of one lattice cell: (x, y), (x+1, y), (x, y+1), (x+1, y+1).
 * ldq_op_add_obs adds tau * A^T A to a 2-D lattice operator in place;
 * ldq_op_obs_gram creates A^T A alone (for dQ_p / dtau) on the lattice of
 * `like`.  corner and weight are host arrays. */
int ldq_op_add_obs(ldq_op *Q, int64_t nobs, const int32_t *corner, const double *weight, double tau);
int ldq_op_obs_gram(ldq_ctx *ctx, const ldq_op *like, int64_t nobs, const int32_t *corner,
                    const double *weight, ldq_op **out);

/* Number of rows of an operator. */
int64_t ldq_op_size(const ldq_op *op);
void ldq_op_destroy(ldq_op *op);

/* --------------------------------------------------------------- options */

enum { LDQ_FP64 = 0,    /* vectors stored in FP64, all arithmetic in FP64 */
       LDQ_MIXED = 1 }; /* vectors and operator fields stored in FP32.  The specialised
                           lattice passes apply the stencil in FP32 with the Laplacian's exact
                           coefficients (only kappa2 is rounded) and sum dot products per lane
                           in FP32 over a few rows before adding them in FP64; the other passes
                           compute in FP64.  CG scalars, shifts, recurrences, gradient and
                           log-det accumulation are FP64 throughout. */
enum {
  LDQ_COLOUR_AUTO = 0,     /* modular for lattice operators, greedy for CSR */
  LDQ_COLOUR_MODULAR = 1,  /* (x + a y [+ b z]) mod C, smallest valid C (lattices only) */
  LDQ_COLOUR_GREEDY = 2,   /* sequential greedy in priority order (bit-exact on the device) */
  LDQ_COLOUR_USER = 3,     /* user_colours[n] */
  LDQ_COLOUR_IDENTITY = 4, /* every site its own class (n probes; exact up to quadrature) */
  LDQ_COLOUR_RADEMACHER = 5 /* no colouring: nrandom random-sign probes (Hutchinson's estimator,
                               Sec. 2.1, eq. (6)); lattice and CSR operators, single calls */
};

typedef struct {
  int k;                        /* colouring distance in the graph of Q (>= 1) */
  int colouring;                /* LDQ_COLOUR_* */
  const int32_t *user_colours;  /* host, n entries in [0, C), for LDQ_COLOUR_USER */
  const int32_t *priority;      /* host, n entries or NULL (= natural order): greedy visits
                                   vertices by ascending priority, ties by index */
  int nshifts;                  /* number of complex shifts N (1..64) */
  double tol;                   /* shifted system l stops when |zeta_l| ||r|| / ||v|| <= tol */
  double grad_tol;              /* with a gradient the base system runs until ||r|| / ||v|| <= grad_tol
                                   (0 => tol) */
  int max_iter;                 /* Krylov iteration cap per probe */
  int precision;                /* LDQ_FP64 or LDQ_MIXED */
  double lambda_min, lambda_max;/* spectrum enclosure; 0 => computed by the library */
  int probe_block;              /* probes advanced together (0 = all) */
  int check_every;              /* passes between convergence polls (0 = library default) */
  int launch_mode;              /* LDQ_LAUNCH_*: how each chunk of pass launches between two polls
                                   is issued */
  int tile_rows;                /* 2-D lattices: lattice rows per wave tile; 0 = chosen by the
                                   library's autotuner (timed once per problem shape on the context,
                                   among the specialised pass's tile and shorter tiles of the general
                                   pass) */
  int lanes;                    /* lattices: 1 = the probes of a block advance in one chain of pass
                                   launches; 2..4 = in that many chains over near-equal shares of the
                                   block, run concurrently on the context stream and streams the
                                   library owns (each chain's fixed cost per launch overlaps the
                                   others' streaming); 0 = chosen by the autotuner on 2-D lattices
                                   (1, 2 or 3, timed with the tile heights), 1 elsewhere.  Results
                                   are identical. */
  int nrandom;                  /* LDQ_COLOUR_RADEMACHER: number s of probes; entry i of probe j is
                                   +1 or -1 by the top bit of output j * 2^32 + i + 1 of the SplitMix64
                                   generator (Steele, Lea and Flood 2014) started from `seed` (sites
                                   numbered x + nx (y + ny z)); the result is the mean over probes,
                                   (1/s) sum_j v_j^T log(Q) v_j, and likewise the gradient */
  uint64_t seed;                /* LDQ_COLOUR_RADEMACHER: generator state */
  int consistent_grad;          /* 0: grad_i = sum_j x_j^T dQ_i v_j (x_j = Q^{-1} v_j), the probing
                                   estimate of tr(Q^{-1} dQ_i); 1: the exact derivative of the
                                   log det estimate with the shifts held fixed,
                                   -sum_j Im sum_l c_l (x^l_j)^T dQ_i x^l_j with x^l_j = (Q - sigma_l I)^{-1}
                                   v_j, from a second Krylov solve that accumulates the shifted
                                   solutions (N complex vectors per probe; lattice Q, derivatives
                                   diagonal, scaled shifted Laplacians or, on 2-D lattices,
                                   observation grams; at most 8192 iterations;
                                   LDQ_E_UNSUPPORTED otherwise) */
} ldq_options;

/* launch_mode: AUTO and GRAPH capture one chunk of Krylov pass launches into a HIP graph (on a
 * stream the library owns; capture does not run anything) and replay it on the context stream for
 * every chunk of a probe block; DIRECT enqueues the launches one by one.  Results are identical. */
enum { LDQ_LAUNCH_AUTO = 0, LDQ_LAUNCH_GRAPH = 1, LDQ_LAUNCH_DIRECT = 2 };

/* Defaults: k = 2, AUTO colouring, N = 20, tol = 1e-10 (FP64) / 1e-5 (MIXED),
 * grad_tol = 0, max_iter = 100000, FP64, enclosure computed, all probes. */
void ldq_options_default(ldq_options *o);

typedef struct {
  int32_t ncolours;          /* non-empty colour classes = probes */
  int32_t iters_max;         /* Krylov iterations of the slowest probe */
  int64_t iters_total;       /* sum of iterations over probes */
  double lambda_min, lambda_max;  /* enclosure used */
  double max_rel_residual;   /* max over probes of the final ||r|| / ||v|| */
  double seconds;            /* host wall time of the call */
  double loop_seconds;       /* device time of the pass-kernel launches: HIP events on the ctx stream
                                bracket each chunk of back-to-back launches (host polling excluded) */
  int64_t passes;            /* Krylov iterations launched: one fused pass kernel per lane each on
                                lattice operators; passes A and B and the tail kernel each on CSR
                                operators */
  int64_t probe_passes;      /* sum over iterations of the probes each advanced */
  double bytes_model;        /* algorithmic bytes of those passes.  Lattice: r and p read and written
                                once per probe-site (4 x element size; the first pass writes only),
                                plus each operator field once per launch.  CSR: 5 x element size per
                                probe-site (pass A reads and writes r and p, pass B reads r), plus the
                                sliced operator and the colour array once per pass */
  int32_t enclosure_violations; /* probes whose Lanczos matrix (from their CG coefficients) has an
                                   eigenvalue outside [lambda_min, lambda_max] beyond rounding */
  int32_t lanes;             /* lattices: concurrent chains the passes ran in (a pass is then one
                                launch per lane, over that lane's probes); 1 otherwise */
  int32_t tile_rows;         /* 2-D lattices: lattice rows per wave tile used; 0 otherwise */
  double std_error;          /* LDQ_COLOUR_RADEMACHER: Monte Carlo standard error of the log det
                                estimate (sample standard deviation of the per-probe terms over
                                sqrt(s)); 0 for colourings (the probing estimate is deterministic) */
} ldq_info;

/* ------------------------------------------------------------- the method */

/* a1: the colouring that defines the probes (Sec. 2.1, probing paragraph).
 * method = LDQ_COLOUR_MODULAR / GREEDY / IDENTITY; priority as in ldq_options.
 * colours: host int32[n] output; *ncolours receives C (max colour + 1). */
int ldq_colouring(ldq_ctx *ctx, const ldq_op *Q, int k, int method, const int32_t *priority,
                  int32_t *colours, int32_t *ncolours);

/* a2: enclosure [lambda_min, lambda_max] of the spectrum of Q that the
 * quadrature needs (Sec. 2.1, the paragraph before eq. (7)).  Lattice
 * operators: closed-form eigenvalue extremes of the Laplacian, Weyl's bound
 * for a kappa^2 field, Gershgorin for an observation term.  CSR operators:
 * lambda_max = the Gershgorin bound, lambda_min = half the smallest eigenvalue
 * of the Lanczos matrix of 200 CG steps on the all-ones vector; a log det
 * call lowers it further when a probe's own Lanczos matrix reaches below it,
 * and keeps the result on the operator. */
int ldq_spectrum_bounds(ldq_ctx *ctx, const ldq_op *Q, double *lambda_min, double *lambda_max);

/* a3: shifts sigma_l and weights c_l (l = 1..N) with
 * log(lambda) ~ Im sum_l c_l / (lambda - sigma_l) on [lambda_min, lambda_max]
 * (eq. (7)).  sigma, coef: host double[2 N] as (re, im) pairs. */
int ldq_shifts(ldq_ctx *ctx, double lambda_min, double lambda_max, int nshifts,
               double *sigma, double *coef);

/* a4-a6: log det Q ~ sum_j Im sum_l c_l v_j^T (Q - sigma_l I)^{-1} v_j. */
int ldq_logdet(ldq_ctx *ctx, const ldq_op *Q, const ldq_options *opts, double *logdet,
               ldq_info *info /* nullable */);

/* a4-a7: log det Q and grad[i] ~ sum_j x_j^T dQ[i] v_j, x_j = Q^{-1} v_j,
 * for nparams (0..4) derivative operators dQ[i] on the same lattice:
 * LDQ_SHIFTED_LAPLACIAN (any scale/kappa2), diagonal, or observation gram. */
int ldq_logdet_grad(ldq_ctx *ctx, const ldq_op *Q, int nparams, const ldq_op *const *dQ,
                    const ldq_options *opts, double *logdet, double *grad, ldq_info *info);

/* Per-probe terms of the last ldq_logdet / ldq_logdet_grad call on ctx:
 * out[j * (1 + nparams) + 0] = Im sum_l c_l psi_jl, out[j * (1 + nparams) + 1 + i]
 * = x_j^T dQ[i] v_j, for the j-th non-empty colour class in increasing colour
 * order.  capacity = length of out; *count receives the number of probes. */
int ldq_probe_terms(ldq_ctx *ctx, double *out, int64_t capacity, int64_t *count, int *nparams);

/* Y = f_N(Q) V: the rational approximation of eq. (7) (Sec. 2.1) of log(Q)
 * applied to nvec vectors, Im sum_l c_l (Q - sigma_l I)^{-1} v_j, with the
 * enclosure, shifts and tolerances of opts (colouring fields ignored).
 * V and Y are DEVICE arrays of nvec x n doubles, vector j at [j * n]
 * (owned by the caller; Y is overwritten).  The shifted solutions are not
 * stored: a first Krylov solve records the base CG coefficients, the host
 * forms per-iteration weights w_m = Im sum_l c_l zeta^l_m S^l_m of the
 * residuals (x^l = sum_m zeta^l_m S^l_m r_m), and a second, identical solve
 * accumulates Y = sum_m w_m r_m (two solves and one extra vector per probe).
 * Lattice operators; at most 8192 iterations per vector (LDQ_E_UNSUPPORTED
 * beyond).  info describes the first solve.  v_j^T y_j is the probe term of
 * the log det estimate for probe v_j. */
int ldq_logm_apply(ldq_ctx *ctx, const ldq_op *Q, int nvec, const double *V, double *Y, const ldq_options *opts,
                   ldq_info *info /* nullable */);

/* X = Q^{-1} B for nvec right-hand sides: the base system of the same Krylov
 * iteration (Sec. 2.1: the CG whose coefficients drive every shift), e.g. the
 * posterior mean Q_p^{-1} tau A^T y of the Gauss-linear model (Sec. 2,
 * eq. (3)).  Each system runs until ||r|| <= grad_tol ||b|| (tol when
 * grad_tol <= 0); the solutions are not kept as iterates but formed as
 * x = sum_m S_m r_m, S_m = alpha_m + beta_m S_{m+1}, from a first solve's
 * coefficients and accumulated by a second, identical solve.  B and X are
 * DEVICE arrays of nvec x n doubles, vector j at [j * n] (owned by the
 * caller; X is overwritten, B is not).  Lattice operators (with or without
 * the observation term); at most 8192 iterations per vector
 * (LDQ_E_UNSUPPORTED beyond); LDQ_E_NOT_SPD if a p^T Q p is not positive.
 * info describes the first solve. */
int ldq_solve(ldq_ctx *ctx, const ldq_op *Q, int nvec, const double *B, double *X, const ldq_options *opts,
              ldq_info *info /* nullable */);

/* Many independent fields (e.g. one operator per field); per field f:
 * logdet[f], grad[f * nparams + i] (dQ[f * nparams + i]), info[f] (nullable). */
int ldq_logdet_batched(ldq_ctx *ctx, int nfields, const ldq_op *const *Q, int nparams,
                       const ldq_op *const *dQ, const ldq_options *opts, double *logdet,
                       double *grad, ldq_info *info);

#ifdef __cplusplus
}
#endif
#endif /* LDQ_H */
