"""Host logic of the noisy-data fit (no GPU): A^T y of the bilinear
observation operator against the oracle's observation matrix (Sec. 1, eq. (1))."""
import numpy as np

from oracle import lattice
from paper_1105_5256_amd import fit, workloads


def test_obs_adjoint_matches_observation_matrix():
    shape = (13, 11)
    n = 143
    corner, weight = workloads.observations(shape, 57, 4)
    y = np.random.default_rng(5).standard_normal(57)
    A = lattice.observation_matrix(n, corner, weight)
    assert np.allclose(fit.obs_adjoint(y, corner, weight, n), A.T @ y, rtol=1e-14, atol=1e-14)
