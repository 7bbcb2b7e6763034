"""The Hutchinson estimator of log det Q with random-sign probes (oracle; test
infrastructure only: only tests/, the smoke check and the bench's CPU baseline
use this package).

Sec. 2.1, the paragraph on stochastic estimators (eq. (6)): with s vectors v_j
whose entries are +1 or -1 with probability 1/2 each, independently,

    tr log Q  ~  H = (1/s) sum_j v_j^T log(Q) v_j,

an unbiased Monte Carlo estimate, so it comes with confidence regions (by
Monte Carlo statistics or by Hoeffding's inequality, same paragraph).  Here
each v_j^T log(Q) v_j is taken exactly (eigh) or through the rational
approximation of eq. (7) with direct shifted solves, as for the probing
estimator.  The gradient analogue (1/s) sum_j (Q^{-1} v_j)^T dQ v_j is an
unbiased estimate of tr(Q^{-1} dQ).

Random signs.  Entry i of probe j is +1 when the top bit of

    splitmix64(seed, j * 2**32 + i)

is clear and -1 otherwise, where splitmix64(seed, c) is output number c + 1
of the SplitMix64 generator (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) started from state `seed`:
z = seed + (c + 1) * 0x9E3779B97F4A7C15, then z ^= z >> 30, z *= 0xBF58476D1CE4E5B9,
z ^= z >> 27, z *= 0x94D049BB133111EB, z ^= z >> 31 (all modulo 2**64).  Sites are
numbered x + nx * (y + ny * z) on lattices and by row on CSR matrices.
"""
import numpy as np
import scipy.fft as sfft
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import exact

GAMMA = np.uint64(0x9E3779B97F4A7C15)
MIX1 = np.uint64(0xBF58476D1CE4E5B9)
MIX2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed, counter):
    """Output number counter + 1 of SplitMix64 from state `seed` (uint64 arrays)."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (np.asarray(counter, dtype=np.uint64) + np.uint64(1)) * GAMMA
        z = (z ^ (z >> np.uint64(30))) * MIX1
        z = (z ^ (z >> np.uint64(27))) * MIX2
        return z ^ (z >> np.uint64(31))


def rademacher(n, s, seed):
    """n x s matrix of the probes' entries (+1 / -1), probe j in column j."""
    i = np.arange(n, dtype=np.uint64)[:, None]
    j = np.arange(s, dtype=np.uint64)[None, :]
    bits = splitmix64(seed, (j << np.uint64(32)) + i) >> np.uint64(63)
    return 1.0 - 2.0 * bits.astype(np.float64)


def hutchinson_exact(Q, V):
    """H with exact v^T log(Q) v (dense eigh).  Returns (H, per-probe terms)."""
    Qd = Q.toarray() if sp.issparse(Q) else np.asarray(Q, dtype=np.float64)
    lam, U = np.linalg.eigh(Qd)
    W = U.T @ V
    terms = np.sum(np.log(lam)[:, None] * W * W, axis=0)
    return float(np.mean(terms)), terms


def hutchinson_rational(Q, V, sigma, coef):
    """H with eq. (7): terms_j = Im sum_l c_l v_j^T (Q - sigma_l I)^{-1} v_j (sparse LU per shift)."""
    Q = sp.csc_matrix(Q, dtype=np.complex128)
    n = Q.shape[0]
    terms = np.zeros(V.shape[1])
    eye = sp.identity(n, dtype=np.complex128, format="csc")
    Vc = V.astype(np.complex128)
    for s_, c in zip(sigma, coef):
        X = spla.splu((Q - s_ * eye).tocsc()).solve(Vc)
        terms += np.imag(c * np.sum(V * X, axis=0))
    return float(np.mean(terms)), terms


def hutchinson_grad(Q, dQs, V):
    """(1/s) sum_j (Q^{-1} v_j)^T dQ_i v_j for each dQ_i.  Returns (g, per-probe terms [s, nparams])."""
    X = spla.splu(sp.csc_matrix(Q, dtype=np.float64)).solve(V)
    terms = np.stack([np.sum(X * (dQ @ V), axis=0) for dQ in dQs], axis=1)
    return terms.mean(axis=0), terms


def variance_exact(A):
    """Var(v^T A v) for one Rademacher v and symmetric A: 2 (||A||_F^2 - sum_i A_ii^2)."""
    Ad = A.toarray() if sp.issparse(A) else np.asarray(A, dtype=np.float64)
    return float(2.0 * (np.sum(Ad * Ad) - np.sum(np.diag(Ad) ** 2)))


def standard_error(terms):
    """Monte Carlo standard error of the mean of the per-probe terms (sample sd / sqrt(s))."""
    terms = np.asarray(terms, dtype=np.float64)
    return float(np.std(terms, ddof=1) / np.sqrt(len(terms))) if len(terms) > 1 else float("inf")


def hoeffding_halfwidth(n, lmin, lmax, s, delta):
    """Half-width t with P(|H - tr log Q| >= t) <= delta by Hoeffding's inequality: every
    term v^T log(Q) v lies in [n log lmin, n log lmax] (||v||^2 = n), so
    t = n (log lmax - log lmin) sqrt(log(2 / delta) / (2 s))."""
    return float(n * (np.log(lmax) - np.log(lmin)) * np.sqrt(np.log(2.0 / delta) / (2.0 * s)))


def hutchinson_dst(shape, kappa2, V, power=1, dQs=()):
    """Exact per-probe terms for Q = (kappa2 I + L)^power on a Dirichlet
    lattice with constant kappa2 (large lattices): Q = S diag(mu) S with the
    orthonormal DST-I S, so v^T log(Q) v = sum_f log(mu_f) (S v)_f^2 and
    Q^{-1} v = S diag(1/mu) S v.  Returns (H, terms [s], g, gradient terms
    [s, len(dQs)]) with (Q^{-1} v_j)^T dQ_i v_j."""
    shape = tuple(int(m) for m in shape)
    rshape = tuple(reversed(shape))
    mu = (kappa2 + exact.lattice_eigenvalues(shape)) ** power
    logmu = np.log(mu)
    V = np.asarray(V, dtype=np.float64)
    terms = np.empty(V.shape[1])
    gterms = np.zeros((V.shape[1], len(dQs)))
    for j in range(V.shape[1]):
        v = V[:, j]
        sv = sfft.dstn(v.reshape(rshape), type=1, norm="ortho")
        terms[j] = np.sum(logmu * sv * sv)
        if dQs:
            x = sfft.idstn(sv / mu, type=1, norm="ortho").ravel()
            for i, dQ in enumerate(dQs):
                gterms[j, i] = x @ (dQ @ v)
    return float(np.mean(terms)), terms, gterms.mean(axis=0), gterms
