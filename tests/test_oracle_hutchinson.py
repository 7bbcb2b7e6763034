"""Pins of the oracle's Hutchinson estimator (Sec. 2.1, eq. (6) and the
paragraph on confidence regions): the sign generator against the published
SplitMix64 outputs, exactness where the estimator is exact (diagonal Q), and
unbiasedness, the variance and the gradient by brute force over every sign
vector of a small matrix."""
import itertools
import os

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import hutchinson as hu
from oracle import lattice, shifts

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_seed0.txt")


def small_spd(n, seed):
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((n, n))
    return B @ B.T + n * np.eye(n)


def logm_spd(A):
    lam, U = np.linalg.eigh(A)
    return (U * np.log(lam)) @ U.T


def test_splitmix64_published_outputs():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    for c, h in rows:
        assert int(hu.splitmix64(0, int(c))) == int(h, 16)


def test_signs_balanced_and_uncorrelated():
    V = hu.rademacher(50000, 4, seed=12345)
    assert set(np.unique(V)) == {-1.0, 1.0}
    N = V.size
    assert abs((V > 0).mean() - 0.5) < 5 * 0.5 / np.sqrt(N)
    for a, b in itertools.combinations(range(4), 2):
        assert abs(np.mean(V[:, a] * V[:, b])) < 5 / np.sqrt(V.shape[0])
    # another seed gives other signs
    assert not np.array_equal(V, hu.rademacher(50000, 4, seed=12346))


def test_diagonal_is_exact_for_every_probe():
    d = np.linspace(0.3, 7.0, 40)
    H, terms = hu.hutchinson_exact(np.diag(d), hu.rademacher(40, 9, seed=3))
    assert np.allclose(terms, np.sum(np.log(d)), rtol=1e-12, atol=0)


def test_unbiased_and_variance_by_brute_force():
    n = 10
    Q = small_spd(n, 1)
    L = logm_spd(Q)
    V = np.array(list(itertools.product([-1.0, 1.0], repeat=n))).T      # every sign vector
    H, terms = hu.hutchinson_exact(Q, V)
    assert abs(H - np.trace(L)) < 1e-12 * abs(np.trace(L)) + 1e-12
    assert abs(np.mean((terms - np.trace(L)) ** 2) - hu.variance_exact(L)) < 1e-9 * hu.variance_exact(L)


def test_generator_mean_within_five_sigma():
    n, s = 12, 20000
    Q = small_spd(n, 2)
    L = logm_spd(Q)
    H, terms = hu.hutchinson_exact(Q, hu.rademacher(n, s, seed=7))
    assert abs(H - np.trace(L)) < 5 * np.sqrt(hu.variance_exact(L) / s)
    assert abs(hu.standard_error(terms) - np.sqrt(hu.variance_exact(L) / s)) < 0.05 * np.sqrt(hu.variance_exact(L) / s)


def test_rational_matches_exact():
    shape = (12, 9)
    Q = lattice.shifted_laplacian(shape, 0.3)
    lam = np.linalg.eigvalsh(Q.toarray())
    sig, coef = shifts.log_shifts(lam[0] * 0.99, lam[-1] * 1.01, 20)
    V = hu.rademacher(Q.shape[0], 6, seed=99)
    He, te = hu.hutchinson_exact(Q, V)
    Hr, tr = hu.hutchinson_rational(Q, V, sig, coef)
    assert np.allclose(tr, te, rtol=1e-8, atol=1e-8 * np.max(np.abs(te)))


def test_gradient_unbiased_by_brute_force():
    n = 10
    Q = small_spd(n, 3)
    rng = np.random.default_rng(4)
    D = rng.standard_normal((n, n))
    dQ = sp.csr_matrix(D + D.T)
    V = np.array(list(itertools.product([-1.0, 1.0], repeat=n))).T
    g, _ = hu.hutchinson_grad(sp.csr_matrix(Q), [dQ], V)
    exact = np.trace(np.linalg.solve(Q, dQ.toarray()))
    assert abs(g[0] - exact) < 1e-10 * max(1.0, abs(exact))


def test_hoeffding_halfwidth_covers():
    shape = (8, 7)
    Q = lattice.shifted_laplacian(shape, 0.5)
    lam = np.linalg.eigvalsh(Q.toarray())
    tr = np.sum(np.log(lam))
    s = 40
    t = hu.hoeffding_halfwidth(Q.shape[0], lam[0], lam[-1], s, 0.01)
    for seed in range(20):
        H, _ = hu.hutchinson_exact(Q, hu.rademacher(Q.shape[0], s, seed))
        assert abs(H - tr) <= t


@pytest.mark.parametrize("power", [1, 2])
def test_dst_route_matches_eigh(power):
    """The DST route for large lattices against the dense eigendecomposition
    (terms) and sparse solves (gradient terms) on a small lattice."""
    shape, k2 = (9, 7), 0.3
    n = 63
    M = lattice.shifted_laplacian(shape, k2)
    Q = lattice.squared(M) if power == 2 else M
    V = hu.rademacher(n, 5, 77)
    dQ = 2 * M
    H, T, g, G = hu.hutchinson_dst(shape, k2, V, power, [dQ])
    He, Te = hu.hutchinson_exact(Q, V)
    ge, Ge = hu.hutchinson_grad(Q, [dQ], V)
    assert np.allclose(T, Te, rtol=1e-11, atol=0) and abs(H - He) <= 1e-11 * abs(He)
    assert np.allclose(G[:, 0], Ge[:, 0], rtol=1e-10, atol=0) and abs(g[0] - ge[0]) <= 1e-10 * abs(ge[0])
