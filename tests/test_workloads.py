"""The seeded inputs: the CSR form of the 13-point operator is the product
(kappa2 I + L)^2 of the oracle's lattice matrices, and the random sparse
matrices are symmetric positive definite with the degrees asked for."""
import numpy as np
import scipy.sparse as sp

from oracle import lattice
from paper_1105_5256_amd import workloads


def test_csr_form_of_squared_operator_is_the_matrix_product():
    for shape, kappa2, scale in [((13, 9), 0.3, 1.0), ((5, 31), 0.05, 2.5), ((2, 2), 1.0, 1.0)]:
        rp, ci, v = workloads.lattice2d_sq_csr(*shape, kappa2=kappa2, scale=scale)
        n = shape[0] * shape[1]
        A = sp.csr_matrix((v, ci, rp), shape=(n, n))
        B = scale * lattice.squared(lattice.shifted_laplacian(shape, kappa2))
        assert abs(A - B).max() < 1e-12
        assert all(np.all(np.diff(ci[rp[i]:rp[i + 1]]) > 0) for i in range(n))


def test_csr_form_of_shifted_laplacian():
    for shape, kappa2, scale in [((13, 9), 0.3, 2.0), ((1, 7), 0.05, 1.0)]:
        rp, ci, v = workloads.lattice2d_5pt_csr(*shape, kappa2=kappa2, scale=scale)
        n = shape[0] * shape[1]
        A = sp.csr_matrix((v, ci, rp), shape=(n, n))
        assert abs(A - scale * lattice.shifted_laplacian(shape, kappa2)).max() < 1e-12
        assert all(np.all(np.diff(ci[rp[i]:rp[i + 1]]) > 0) for i in range(n))


def test_random_spd_csr_is_symmetric_positive_definite():
    for signs in (False, True):
        rp, ci, v = workloads.random_spd_csr(600, 2, 9, shift=0.05, seed=4, signs=signs)
        A = sp.csr_matrix((v, ci, rp), shape=(600, 600))
        assert abs(A - A.T).max() == 0.0
        assert np.linalg.eigvalsh(A.toarray())[0] > 0
        assert all(np.all(np.diff(ci[rp[i]:rp[i + 1]]) > 0) for i in range(600))
    # the signs change the matrix but not its spectrum
    a = workloads.random_spd_csr(300, 2, 9, seed=4)
    b = workloads.random_spd_csr(300, 2, 9, seed=4, signs=True)
    ea = np.linalg.eigvalsh(sp.csr_matrix((a[2], a[1], a[0]), shape=(300, 300)).toarray())
    eb = np.linalg.eigvalsh(sp.csr_matrix((b[2], b[1], b[0]), shape=(300, 300)).toarray())
    assert np.allclose(ea, eb, rtol=1e-12, atol=1e-12)


def test_spde_field_sample_has_covariance_q_inverse():
    # x^T Q x of an exact draw from N(0, Q^{-1}) is chi-square with n degrees of freedom
    from oracle import lattice
    shape, k2, tau = (20, 17), 0.5, 2.0
    n = shape[0] * shape[1]
    Q = (tau * tau * lattice.squared(lattice.shifted_laplacian(shape, k2))).tocsr()
    vals = np.array([float(x @ (Q @ x)) for x in (workloads.spde_field_sample(shape, k2, tau, s) for s in range(300))])
    assert abs(vals.mean() - n) < 5 * np.sqrt(2 * n / len(vals))
    assert abs(vals.std() / np.sqrt(2 * n) - 1) < 0.25
