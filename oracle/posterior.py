"""The Gauss-linear model of Sec. 1 (oracle; test infrastructure only: only
tests/, the smoke check and the bench's CPU baseline use this package).

Data y = A x + e with a field x ~ N(0, Q_x^{-1}) and noise e ~ N(0, Q_1^{-1}),
Q_1 = tau I (eq. (1)-(3) of Sec. 1).  The posterior of x given y has precision
Q_p = Q_x + A^T Q_1 A and mean mu_p = Q_p^{-1} A^T Q_1 y (stated after
eq. (3)).  The hyperparameters are fitted by maximising the marginal density of
y (Sec. 1, the objective built from eq. (3)); with the constants read as in the
text's definition of the Gaussian density,

    -2 log p(y) = -log det Q_x + log det Q_p - m log tau
                  + tau y^T y - b^T mu_p + m log(2 pi),      b = tau A^T y,

where tau y^T y - b^T mu_p = mu_p^T Q_x mu_p + tau ||y - A mu_p||^2 (the two
quadratic forms of the text at the posterior mean, since Q_p mu_p = b).
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def solve(Q, B):
    """Q^{-1} B for the columns of B (sparse LU)."""
    B = np.asarray(B, dtype=np.float64)
    return spla.splu(sp.csc_matrix(Q, dtype=np.float64)).solve(B)


def posterior_mean(Qx, A, y, tau):
    """mu_p = Q_p^{-1} tau A^T y with Q_p = Q_x + tau A^T A."""
    Qp = (sp.csr_matrix(Qx) + tau * (A.T @ A)).tocsc()
    return solve(Qp, tau * (A.T @ np.asarray(y, dtype=np.float64)))


def _logdet_spd(Q):
    """log det of a symmetric positive definite matrix (dense Cholesky)."""
    L = np.linalg.cholesky(Q.toarray() if sp.issparse(Q) else np.asarray(Q, dtype=np.float64))
    return 2.0 * float(np.sum(np.log(np.diag(L))))


def neg2_loglik(Qx, A, y, tau):
    """-2 log p(y) of the Gauss-linear model through the posterior (formula in the
    module docstring; exact log dets, small problems)."""
    y = np.asarray(y, dtype=np.float64)
    m = y.shape[0]
    Qp = (sp.csr_matrix(Qx) + tau * (A.T @ A)).tocsr()
    mu = posterior_mean(Qx, A, y, tau)
    b = tau * (A.T @ y)
    return (-_logdet_spd(Qx) + _logdet_spd(Qp) - m * np.log(tau) + tau * float(y @ y) - float(b @ mu)
            + m * np.log(2.0 * np.pi))
