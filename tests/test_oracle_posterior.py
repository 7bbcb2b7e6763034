"""Pins of the Gauss-linear oracle (Sec. 1, eq. (1)-(3)): the solve by its
residual and a dense solve; the posterior mean and the marginal density by
the covariance form of the same model (prior covariance Sigma = Q_x^{-1},
y ~ N(0, A Sigma A^T + tau^{-1} I)), a route that shares no step with the
precision form the oracle takes."""
import numpy as np
import pytest

from oracle import lattice, posterior
from paper_1105_5256_amd import workloads


def model(shape=(8, 7), kappa2=0.4, nobs=23, seed=3):
    n = int(np.prod(shape))
    Qx = lattice.squared(lattice.shifted_laplacian(shape, kappa2))
    corner, weight = workloads.observations(shape, nobs, seed)
    A = lattice.observation_matrix(n, corner, weight)
    return n, Qx, A


def test_solve_residual_and_dense():
    n, Qx, _ = model()
    B = np.random.default_rng(0).standard_normal((n, 3))
    X = posterior.solve(Qx, B)
    assert np.linalg.norm(Qx @ X - B) <= 1e-12 * np.linalg.norm(B)
    assert np.allclose(X, np.linalg.solve(Qx.toarray(), B), rtol=1e-10, atol=0)


@pytest.mark.parametrize("tau", [0.5, 40.0])
def test_posterior_mean_matches_covariance_form(tau):
    n, Qx, A = model()
    y = np.random.default_rng(1).standard_normal(A.shape[0])
    S = np.linalg.inv(Qx.toarray())
    Ad = A.toarray()
    C = Ad @ S @ Ad.T + np.eye(A.shape[0]) / tau
    mu_cov = S @ Ad.T @ np.linalg.solve(C, y)
    mu = posterior.posterior_mean(Qx, A, y, tau)
    assert np.allclose(mu, mu_cov, rtol=1e-9, atol=1e-12 * np.abs(mu_cov).max())


@pytest.mark.parametrize("tau", [0.5, 40.0])
def test_neg2_loglik_matches_marginal_density(tau):
    n, Qx, A = model()
    y = np.random.default_rng(2).standard_normal(A.shape[0])
    S = np.linalg.inv(Qx.toarray())
    Ad = A.toarray()
    C = Ad @ S @ Ad.T + np.eye(A.shape[0]) / tau
    m = A.shape[0]
    direct = np.linalg.slogdet(C)[1] + float(y @ np.linalg.solve(C, y)) + m * np.log(2 * np.pi)
    val = posterior.neg2_loglik(Qx, A, y, tau)
    assert abs(val - direct) <= 1e-9 * abs(direct)
