"""f_N(Q) v itself (oracle; test infrastructure only: only tests/, the smoke
check and the bench's CPU baseline use this package).

Sec. 2.1, eq. (7): log(Q) v ~ Im sum_l c_l (Q - sigma_l I)^{-1} v, the rational
approximation the estimator applies inside v^T log(Q) v, here returned as a
vector (the shifted systems solved directly), next to the exact log(Q) v of a
small dense Q (eigh).
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def logm_apply_rational(Q, V, sigma, coef):
    """Im sum_l c_l (Q - sigma_l I)^{-1} V for the columns of V (n x m); sparse LU per shift."""
    Q = sp.csc_matrix(Q, dtype=np.complex128)
    n = Q.shape[0]
    V = np.asarray(V, dtype=np.float64).reshape(n, -1)
    Y = np.zeros(V.shape)
    eye = sp.identity(n, dtype=np.complex128, format="csc")
    for s, c in zip(sigma, coef):
        Y += np.imag(c * spla.splu((Q - s * eye).tocsc()).solve(V.astype(np.complex128)))
    return Y


def logm_apply_exact(Q, V):
    """U diag(log lambda) U^T V with Q = U diag(lambda) U^T (dense, small Q)."""
    Qd = Q.toarray() if sp.issparse(Q) else np.asarray(Q, dtype=np.float64)
    lam, U = np.linalg.eigh(Qd)
    V = np.asarray(V, dtype=np.float64).reshape(Qd.shape[0], -1)
    return U @ (np.log(lam)[:, None] * (U.T @ V))
