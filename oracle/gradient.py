"""Hyperparameter gradient of log det Q (oracle; test infrastructure only).

The hyperparameter step of Sec. 3 (a modified Newton method on the objective
of Sec. 1, eq. (4)) needs d/d eta log det Q(eta) = tr(Q^{-1} dQ/d eta).  The
paper gives no gradient; the quantities here are:

* the exact gradient tr(Q^{-1} dQ) (closed form on lattices, dense solve,
  central finite differences of an exact log det);
* the probing estimate G = sum_j x_j^T dQ v_j with x_j = Q^{-1} v_j and v_j the
  probing vectors of Sec. 2.1.  With the identity colouring G is exact.  G is
  not the derivative of the probing log-det estimate E(Q; c).
"""
import numpy as np
import scipy.fft as sfft
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import exact
from .estimator import probes


def grad_closed_form(shape, kappa2, power=1):
    """d/d kappa2 log det((kappa2 I + L)^power) = power * sum 1 / (kappa2 + lambda)."""
    lam = exact.lattice_eigenvalues(shape)
    return float(power * np.sum(1.0 / (kappa2 + lam)))


def grad_dense(Q, dQ):
    """tr(Q^{-1} dQ) with a dense solve."""
    Qd = Q.toarray() if sp.issparse(Q) else np.asarray(Q, dtype=np.float64)
    Dd = dQ.toarray() if sp.issparse(dQ) else np.asarray(dQ, dtype=np.float64)
    return float(np.trace(np.linalg.solve(Qd, Dd)))


def grad_fd(logdet_of_eta, eta, h=1e-5):
    """Central differences (f(eta + h e_i) - f(eta - h e_i)) / (2 h) per coordinate."""
    eta = np.asarray(eta, dtype=np.float64)
    g = np.zeros_like(eta)
    for i in range(len(eta)):
        e = np.zeros_like(eta)
        e[i] = h
        g[i] = (logdet_of_eta(eta + e) - logdet_of_eta(eta - e)) / (2.0 * h)
    return g


def grad_probing(Q, dQs, colours):
    """G_i = sum_j x_j^T dQ_i v_j with x_j = Q^{-1} v_j from a sparse LU.
    Returns (G (len(dQs)), per-class terms (C x len(dQs)))."""
    P, _ = probes(colours)
    lu = spla.splu(sp.csc_matrix(Q))
    X = lu.solve(P)
    terms = np.stack([np.sum(X * (dQ @ P), axis=0) for dQ in dQs], axis=1)
    return terms.sum(axis=0), terms


def grad_probing_dst(shape, kappa2, power, colours, dQs):
    """Same as ``grad_probing`` for Q = (kappa2 I + L)^power with constant kappa2,
    with x_j = S diag(1/mu) S v_j from the orthonormal DST-I."""
    shape = tuple(int(m) for m in shape)
    rshape = tuple(reversed(shape))
    mu = (kappa2 + exact.lattice_eigenvalues(shape)) ** power
    P, _ = probes(colours)
    terms = np.zeros((P.shape[1], len(dQs)))
    for j in range(P.shape[1]):
        v = P[:, j]
        sv = sfft.dstn(v.reshape(rshape), type=1, norm="ortho")
        x = sfft.idstn(sv / mu, type=1, norm="ortho").ravel()
        for i, dQ in enumerate(dQs):
            terms[j, i] = x @ (dQ @ v)
    return terms.sum(axis=0), terms


def grad_estimator_rational(Q, dQs, colours, sigma, coef):
    """The derivative of the probing estimate E(Q; c) of eq. (7) with the shifts
    held fixed: dE/d eta_i = -sum_j Im sum_l c_l (x_jl)^T dQ_i x_jl with
    x_jl = (Q - sigma_l I)^{-1} v_j (d(A^{-1}) = -A^{-1} dA A^{-1}; Q - sigma_l I
    is complex symmetric, so no conjugation).  Returns (g, per-class terms)."""
    P, _ = probes(colours)
    Qc = sp.csc_matrix(Q, dtype=np.complex128)
    n = Qc.shape[0]
    eye = sp.identity(n, dtype=np.complex128, format="csc")
    terms = np.zeros((P.shape[1], len(dQs)))
    for s, c in zip(sigma, coef):
        X = spla.splu((Qc - s * eye).tocsc()).solve(P.astype(np.complex128))
        for i, dQ in enumerate(dQs):
            terms[:, i] -= np.imag(c * np.sum(X * (dQ @ X), axis=0))
    return terms.sum(axis=0), terms
