"""The probing estimator of log det Q (oracle; test infrastructure only).

Sec. 2.1: log det Q = tr log Q (eq. (5)) = sum_i e_i^T log(Q) e_i; with
probing vectors v_j (0/1 indicators of the colour classes of a distance-k
colouring) the trace is estimated by

    E(Q; c) = sum_j v_j^T log(Q) v_j            (no 1/s factor, unlike eq. (6)),

and each v_j^T log(Q) v_j is evaluated with the rational approximation of
eq. (7), i.e. sum_j Im sum_l c_l v_j^T (Q - sigma_l I)^{-1} v_j.
With the identity colouring (every vertex its own class) E equals log det Q.

Routes implemented (all float64):
* ``estimator_dst``     exact E for constant-coefficient Dirichlet lattices,
                        log(Q) = S diag(log mu) S with S the orthonormal DST-I;
* ``estimator_eigh``    exact E for small dense Q via eigh;
* ``estimator_logm``    exact E via scipy.linalg.logm (tiny Q only);
* ``estimator_rational_direct``  eq. (7) with a sparse LU per shift;
* ``estimator_cgm``     eq. (7) with the multi-shift CG of ``krylov.cg_m``.
"""
import numpy as np
import scipy.fft as sfft
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import exact, krylov


def probes(colours):
    """Probing vectors as an n x C dense 0/1 matrix, one column per non-empty
    colour class, in increasing colour order (Sec. 2.1, probing)."""
    colours = np.asarray(colours, dtype=np.int64)
    classes = np.unique(colours)
    V = (colours[:, None] == classes[None, :]).astype(np.float64)
    return V, classes


def estimator_dst(shape, kappa2, colours, power=1):
    """Exact E for Q = (kappa2 I + L)^power on a Dirichlet lattice with constant
    kappa2: v^T log(Q) v = sum_f power log(kappa2 + lambda_f) (S v)_f^2.
    Returns (E, per-class terms)."""
    shape = tuple(int(m) for m in shape)
    logmu = power * np.log(kappa2 + exact.lattice_eigenvalues(shape))
    V, _ = probes(colours)
    terms = np.empty(V.shape[1])
    for j in range(V.shape[1]):
        sv = sfft.dstn(V[:, j].reshape(tuple(reversed(shape))), type=1, norm="ortho")
        terms[j] = np.sum(logmu * sv * sv)
    return float(np.sum(terms)), terms


def estimator_eigh(Q, colours):
    """Exact E from the eigen-decomposition Q = V diag(lambda) V^T (eq. (5))."""
    Qd = Q.toarray() if sp.issparse(Q) else np.asarray(Q, dtype=np.float64)
    lam, U = np.linalg.eigh(Qd)
    P, _ = probes(colours)
    W = U.T @ P
    terms = np.sum(np.log(lam)[:, None] * W * W, axis=0)
    return float(np.sum(terms)), terms


def estimator_logm(Q, colours):
    """Exact E with the dense principal matrix logarithm (tiny Q only)."""
    Qd = Q.toarray() if sp.issparse(Q) else np.asarray(Q, dtype=np.float64)
    Lg = np.real(sla.logm(Qd))
    P, _ = probes(colours)
    terms = np.einsum("ij,ik,kj->j", P, Lg, P)
    return float(np.sum(terms)), terms


def estimator_rational_direct(Q, colours, sigma, coef):
    """eq. (7) with exact shifted solves: sum_j Im sum_l c_l v_j^T (Q - sigma_l I)^{-1} v_j."""
    Q = sp.csc_matrix(Q, dtype=np.complex128)
    n = Q.shape[0]
    P, _ = probes(colours)
    terms = np.zeros(P.shape[1])
    eye = sp.identity(n, dtype=np.complex128, format="csc")
    for s, c in zip(sigma, coef):
        lu = spla.splu((Q - s * eye).tocsc())
        X = lu.solve(P.astype(np.complex128))
        psi = np.sum(P * X, axis=0)          # bilinear v^T x, no conjugation
        terms += np.imag(c * psi)
    return float(np.sum(terms)), terms


def estimator_cgm(Q, colours, sigma, coef, tol=1e-12, maxiter=100000):
    """eq. (7) with the textbook multi-shift CG: per probe, psi_l = v^T x^l.
    Returns (E, per-class terms, per-class iteration counts)."""
    P, _ = probes(colours)
    terms = np.zeros(P.shape[1])
    iters = np.zeros(P.shape[1], dtype=np.int64)
    for j in range(P.shape[1]):
        v = P[:, j]
        _, X, it = krylov.cg_m(Q, v, sigma, tol=tol, maxiter=maxiter)
        psi = v @ X
        terms[j] = float(np.imag(np.sum(coef * psi)))
        iters[j] = it
    return float(np.sum(terms)), terms, iters
