"""Sparse precision matrices of the lattice GMRF models (oracle; test infrastructure only).

Site numbering: a lattice of shape (nx, ny) or (nx, ny, nz) numbers site
(x, y[, z]) as s = x + nx * (y + ny * z), x fastest.

Paper passages:
* Sec. 1: Q is a sparse SPD precision matrix of a Gaussian Markov random
  field; the Gauss-linear model y = A x + eps_1, eps_1 ~ N(0, Q_1^{-1})
  (eq. (1)), whose posterior precision is Q_p = Q_x + A^T Q_1 A (stated
  after eq. (3)).
* Sec. 3: the SPDE model tau (kappa - Laplacian) u = W on a lattice; its
  discrete precision is built from M = kappa I + L with L the Dirichlet
  lattice Laplacian, and the squared operator M @ M is the precision of the
  second-order model.
"""
import numpy as np
import scipy.sparse as sp


def second_difference(m):
    """1-D Dirichlet second-difference matrix tridiag(-1, 2, -1) of order m."""
    main = np.full(m, 2.0)
    off = np.full(m - 1, -1.0)
    return sp.diags([off, main, off], [-1, 0, 1], shape=(m, m), format="csr")


def laplacian(shape):
    """Dirichlet lattice Laplacian L = sum over axes of the 1-D second difference.

    Built as a Kronecker sum, so that in 2-D every interior row is the 5-point
    stencil (4, -1, -1, -1, -1) and in 3-D the 7-point stencil (6, -1 x 6); rows
    at the boundary keep the full diagonal (values outside the box are zero).
    """
    shape = tuple(int(m) for m in shape)
    n = int(np.prod(shape))
    L = sp.csr_matrix((n, n))
    for axis, m in enumerate(shape):
        left = int(np.prod(shape[axis + 1:]))    # slower axes
        right = int(np.prod(shape[:axis]))       # faster axes
        term = sp.kron(sp.identity(left, format="csr"),
                       sp.kron(second_difference(m), sp.identity(right, format="csr")))
        L = L + term
    return L.tocsr()


def laplacian_bruteforce(shape):
    """Same matrix as ``laplacian`` built by looping over sites and their lattice
    neighbours (used only to pin ``laplacian`` on tiny shapes)."""
    shape = tuple(int(m) for m in shape)
    d = len(shape)
    n = int(np.prod(shape))
    L = np.zeros((n, n))
    strides = [int(np.prod(shape[:a])) for a in range(d)]
    for s in range(n):
        coord = [(s // strides[a]) % shape[a] for a in range(d)]
        L[s, s] = 2.0 * d
        for a in range(d):
            for step in (-1, 1):
                c = coord[a] + step
                if 0 <= c < shape[a]:
                    L[s, s + step * strides[a]] = -1.0
    return L


def shifted_laplacian(shape, kappa2):
    """M = diag(kappa2) + L; kappa2 is a scalar or one value per site."""
    L = laplacian(shape)
    n = L.shape[0]
    k2 = np.broadcast_to(np.asarray(kappa2, dtype=np.float64), (n,))
    return (sp.diags(k2) + L).tocsr()


def squared(Mop):
    """The matrix product M @ M (the 13-point operator in 2-D, including its
    boundary rows, with no further truncation)."""
    return (Mop @ Mop).tocsr()


def observation_matrix(n, corner, weight):
    """A (nobs x n): row o holds weight[o, c] in column corner[o, c], c = 0..3
    (bilinear interpolation of the field at observation point o; Sec. 1, eq. (1))."""
    corner = np.asarray(corner, dtype=np.int64)
    weight = np.asarray(weight, dtype=np.float64)
    nobs = corner.shape[0]
    rows = np.repeat(np.arange(nobs), corner.shape[1])
    return sp.csr_matrix((weight.ravel(), (rows, corner.ravel())), shape=(nobs, n))


def observation_gram(n, corner, weight):
    """A^T A for the observation matrix above."""
    A = observation_matrix(n, corner, weight)
    return (A.T @ A).tocsr()


def posterior_precision(Qx, corner, weight, tau):
    """Q_p = Q_x + A^T Q_1 A with Q_1 = tau I (the posterior precision stated
    after eq. (3) of Sec. 1)."""
    n = Qx.shape[0]
    return (Qx + tau * observation_gram(n, corner, weight)).tocsr()
