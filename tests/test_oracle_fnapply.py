"""Pins of the oracle's f_N(Q) v (Sec. 2.1, eq. (7) applied to a vector)."""
import numpy as np
import scipy.sparse as sp

from oracle import fnapply, lattice, shifts


def test_diagonal_is_the_scalar_rational_function():
    d = np.linspace(0.2, 9.0, 30)
    sig, coef = shifts.log_shifts(0.19, 9.1, 20)
    V = np.random.default_rng(1).standard_normal((30, 3))
    Y = fnapply.logm_apply_rational(sp.diags(d), V, sig, coef)
    assert np.allclose(Y, shifts.rational_log(d, sig, coef)[:, None] * V, rtol=1e-12, atol=1e-13)
    assert np.allclose(fnapply.logm_apply_exact(np.diag(d), V), np.log(d)[:, None] * V, rtol=1e-13)


def test_rational_matches_exact_within_quadrature_error():
    Q = lattice.shifted_laplacian((11, 9), 0.3)
    lam = np.linalg.eigvalsh(Q.toarray())
    lo, hi = lam[0] * 0.99, lam[-1] * 1.01
    sig, coef = shifts.log_shifts(lo, hi, 20)
    err = np.max(np.abs(shifts.rational_log(np.linspace(lo, hi, 2001), sig, coef) - np.log(np.linspace(lo, hi, 2001))))
    V = np.random.default_rng(2).standard_normal((Q.shape[0], 4))
    Yr = fnapply.logm_apply_rational(Q, V, sig, coef)
    Ye = fnapply.logm_apply_exact(Q, V)
    assert np.all(np.linalg.norm(Yr - Ye, axis=0) <= (1.1 * err + 1e-12) * np.linalg.norm(V, axis=0))
    assert err < 1e-7


def test_unit_vectors_give_the_trace():
    Q = lattice.squared(lattice.shifted_laplacian((7, 6), 0.5))
    lam = np.linalg.eigvalsh(Q.toarray())
    sig, coef = shifts.log_shifts(lam[0] * 0.99, lam[-1] * 1.01, 20)
    n = Q.shape[0]
    Y = fnapply.logm_apply_rational(Q, np.eye(n), sig, coef)
    assert abs(np.trace(Y) - np.sum(shifts.rational_log(lam, sig, coef))) < 1e-10 * abs(np.trace(Y))
