"""Pins of oracle/lattice.py against independent constructions (CPU only)."""
import numpy as np
import pytest

from oracle import lattice
from paper_1105_5256_amd import workloads


@pytest.mark.parametrize("shape", [(7,), (4, 3), (3, 5), (3, 4, 2)])
def test_laplacian_matches_neighbour_loop(shape):
    L = lattice.laplacian(shape).toarray()
    assert np.array_equal(L, lattice.laplacian_bruteforce(shape))


def thirteen_point(shape, kappa2):
    """(kappa2 I + L)^2 written entry by entry from the stencil description:
    centre (kappa2 + 4)^2 + (number of in-box axis neighbours), axis neighbours
    -2 (kappa2 + 4), diagonal neighbours +2, second axis neighbours +1."""
    nx, ny = shape
    n = nx * ny
    Q = np.zeros((n, n))
    c = kappa2 + 4.0
    for y in range(ny):
        for x in range(nx):
            s = x + nx * y
            deg = sum(1 for dx, dy in ((1, 0), (-1, 0), (0, 1), (0, -1))
                      if 0 <= x + dx < nx and 0 <= y + dy < ny)
            Q[s, s] = c * c + deg
            for dx, dy, val in ((1, 0, -2 * c), (-1, 0, -2 * c), (0, 1, -2 * c), (0, -1, -2 * c),
                                (1, 1, 2.0), (1, -1, 2.0), (-1, 1, 2.0), (-1, -1, 2.0),
                                (2, 0, 1.0), (-2, 0, 1.0), (0, 2, 1.0), (0, -2, 1.0)):
                xx, yy = x + dx, y + dy
                if 0 <= xx < nx and 0 <= yy < ny:
                    Q[s, xx + nx * yy] = val
    return Q


@pytest.mark.parametrize("shape", [(5, 4), (6, 7), (2, 9)])
def test_squared_operator_is_thirteen_point(shape):
    M = lattice.shifted_laplacian(shape, 0.37)
    Q = lattice.squared(M).toarray()
    assert np.allclose(Q, thirteen_point(shape, 0.37), rtol=0, atol=1e-13)


def test_field_diagonal():
    shape = (3, 4, 2)
    k2 = np.linspace(0.1, 2.0, 24)
    M = lattice.shifted_laplacian(shape, k2).toarray()
    assert np.allclose(np.diag(M), 6.0 + k2)
    assert np.allclose(M - np.diag(np.diag(M)), lattice.laplacian_bruteforce(shape) - 6.0 * np.eye(24))


def test_bilinear_observations_reproduce_linear_functions():
    shape = (9, 7)
    corner, weight = workloads.observations(shape, 50, seed=1)
    n = shape[0] * shape[1]
    A = lattice.observation_matrix(n, corner, weight)
    assert np.allclose(np.asarray(A.sum(axis=1)).ravel(), 1.0)
    xs = np.arange(n) % shape[0]
    ys = np.arange(n) // shape[0]
    f = 0.3 + 1.7 * xs - 0.9 * ys          # bilinear interpolation is exact for affine f
    # recover the points from the weights: x = x0 + fx, fx = weight of the (x0+1) corners
    x0 = corner[:, 0] % shape[0]
    y0 = corner[:, 0] // shape[0]
    px = x0 + weight[:, 1] + weight[:, 3]
    py = y0 + weight[:, 2] + weight[:, 3]
    assert np.allclose(A @ f, 0.3 + 1.7 * px - 0.9 * py)
    G = lattice.observation_gram(n, corner, weight).toarray()
    assert np.allclose(G, G.T)
    assert np.linalg.eigvalsh(G).min() > -1e-12
