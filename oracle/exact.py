"""Exact log-determinants (oracle; test infrastructure only).

Sec. 2 computes log det Q from a Cholesky factor, log det Q = sum_j 2 log l_jj.
Sec. 2.1, eq. (5) writes log det Q = tr log Q = sum_i log lambda_i.  Both are
implemented plainly here, together with the closed-form eigenvalues of the
Dirichlet lattice Laplacian used to pin them.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def lattice_eigenvalues(shape):
    """All eigenvalues of the Dirichlet lattice Laplacian of ``shape``.

    The 1-D second difference of order m has eigenvalues 4 sin^2(pi i / (2 (m + 1))),
    i = 1..m (eigenvectors sin(pi i x / (m + 1))); the Kronecker sum adds them.
    Returned in the ordering of ``scipy.fft.dstn(type=1)`` over an array of shape
    reversed(shape) (x fastest), so that entry f pairs with frequency f of the
    orthonormal DST-I.
    """
    shape = tuple(int(m) for m in shape)
    lam = np.zeros(tuple(reversed(shape)))
    for axis, m in enumerate(shape):
        i = np.arange(1, m + 1)
        e = 4.0 * np.sin(np.pi * i / (2.0 * (m + 1))) ** 2
        view = [1] * len(shape)
        view[len(shape) - 1 - axis] = m
        lam = lam + e.reshape(view)
    return lam


def logdet_closed_form(shape, kappa2, power=1):
    """log det((kappa2 I + L)^power) = power * sum log(kappa2 + lambda) for a
    constant kappa2 (eq. (5) with the lattice eigenvalues)."""
    lam = lattice_eigenvalues(shape)
    return float(power * np.sum(np.log(kappa2 + lam)))


def spectrum_closed_form(shape, kappa2, power=1):
    """Extremal eigenvalues (lambda_min, lambda_max) of (kappa2 I + L)^power."""
    lam = lattice_eigenvalues(shape)
    lo, hi = kappa2 + lam.min(), kappa2 + lam.max()
    return float(lo ** power), float(hi ** power)


def logdet_dense_cholesky(Q):
    """Sec. 2, steps 2-4: Q = L L^T, log det Q = sum 2 log L_jj (dense, no reordering)."""
    Qd = Q.toarray() if sp.issparse(Q) else np.asarray(Q, dtype=np.float64)
    Lc = np.linalg.cholesky(Qd)
    return float(2.0 * np.sum(np.log(np.diag(Lc))))


def logdet_banded_cholesky(Q, bandwidth=None):
    """The same as ``logdet_dense_cholesky`` using banded storage (natural order)."""
    Q = sp.csr_matrix(Q)
    n = Q.shape[0]
    if bandwidth is None:
        coo = Q.tocoo()
        bandwidth = int(np.max(np.abs(coo.row - coo.col)))
    ab = np.zeros((bandwidth + 1, n))
    for d in range(bandwidth + 1):
        diag = Q.diagonal(-d)
        ab[d, :n - d] = diag
    cb = sla.cholesky_banded(ab, lower=True)
    return float(2.0 * np.sum(np.log(cb[0])))


def logdet_splu(Q):
    """log det Q from a sparse LU factorisation: for SPD Q, det Q = prod |U_ii|
    (L has a unit diagonal; the row/column permutations only change the sign)."""
    lu = spla.splu(sp.csc_matrix(Q), permc_spec="MMD_AT_PLUS_A")
    return float(np.sum(np.log(np.abs(lu.U.diagonal()))))


def logdet_eigh(Q):
    """eq. (5) directly: sum of log eigenvalues of the dense symmetric Q."""
    Qd = Q.toarray() if sp.issparse(Q) else np.asarray(Q, dtype=np.float64)
    lam = np.linalg.eigvalsh(Qd)
    return float(np.sum(np.log(lam)))


def gershgorin_upper(Q):
    """Gershgorin bound max_i sum_j |Q_ij| >= lambda_max(Q)."""
    Q = sp.csr_matrix(Q)
    return float(np.max(np.asarray(abs(Q).sum(axis=1)).ravel()))
