"""Pins of oracle/gradient.py (CPU only)."""
import numpy as np
import scipy.sparse as sp

from oracle import colouring, exact, gradient, lattice
from paper_1105_5256_amd import workloads


def test_gradient_closed_form_dense_and_fd_agree():
    shape, kappa2 = (9, 8), 0.05
    M = lattice.shifted_laplacian(shape, kappa2)
    Q = lattice.squared(M)
    g = gradient.grad_closed_form(shape, kappa2, 2)
    assert abs(gradient.grad_dense(Q, 2 * M) - g) < 1e-10 * abs(g)
    fd = gradient.grad_fd(lambda e: exact.logdet_dense_cholesky(
        lattice.squared(lattice.shifted_laplacian(shape, e[0]))), [kappa2], h=1e-6)
    assert abs(fd[0] - g) < 1e-6 * abs(g)


def test_identity_probing_gradient_is_exact_and_routes_agree():
    shape, kappa2 = (8, 7), 0.1
    M = lattice.shifted_laplacian(shape, kappa2)
    Q = lattice.squared(M)
    G, _ = gradient.grad_probing(Q, [2 * M], np.arange(56))
    g = gradient.grad_closed_form(shape, kappa2, 2)
    assert abs(G[0] - g) < 1e-11 * abs(g)
    C, co = colouring.find_modular(2, 8)
    c = colouring.modular_colouring(shape, C, co)
    G1, t1 = gradient.grad_probing(Q, [2 * M], c)
    G2, t2 = gradient.grad_probing_dst(shape, kappa2, 2, c, [2 * M])
    assert np.allclose(t1, t2, rtol=1e-11, atol=1e-13)


def test_field_model_gradient_matches_finite_differences():
    # Q(eta) = diag(exp(eta0 + eta1 z)) + L, dQ/deta0 = diag(kappa2), dQ/deta1 = diag(kappa2 z)
    shape = (6, 5, 4)
    wl = workloads.lattice3d_field(shape=shape, sigma=1.5, seed=11)
    z = wl["z"]

    def Q_of(eta):
        return lattice.shifted_laplacian(shape, np.exp(eta[0] + eta[1] * z))

    eta = np.array(wl["eta"])
    Q = Q_of(eta)
    k2 = wl["kappa2_field"]
    import scipy.sparse as sp
    dQ = [sp.diags(k2), sp.diags(k2 * z)]
    exact_g = np.array([gradient.grad_dense(Q, d) for d in dQ])
    fd = gradient.grad_fd(lambda e: exact.logdet_dense_cholesky(Q_of(e)), eta, h=1e-6)
    assert np.allclose(fd, exact_g, rtol=1e-6)
    G, _ = gradient.grad_probing(Q, dQ, np.arange(Q.shape[0]))
    assert np.allclose(G, exact_g, rtol=1e-11)


def test_estimator_derivative_matches_finite_differences():
    # the derivative of the probing estimate with fixed shifts, against central
    # differences of the estimate itself (oracle.estimator.estimator_rational_direct)
    from oracle import colouring, estimator, shifts
    shape = (9, 8)
    C, co = colouring.find_modular(2, 2)
    col = colouring.modular_colouring(shape, C, co)
    lam = np.linalg.eigvalsh(lattice.shifted_laplacian(shape, 0.4).toarray())
    sig, coef = shifts.log_shifts(lam[0] * 0.9, lam[-1] * 1.1, 20)
    d = np.linspace(0.5, 1.5, 72)
    g, _ = gradient.grad_estimator_rational(lattice.shifted_laplacian(shape, 0.4), [sp.diags(d)], col, sig, coef)
    h = 1e-5
    Ep, _ = estimator.estimator_rational_direct(lattice.shifted_laplacian(shape, 0.4) + h * sp.diags(d), col, sig, coef)
    Em, _ = estimator.estimator_rational_direct(lattice.shifted_laplacian(shape, 0.4) - h * sp.diags(d), col, sig, coef)
    assert abs(g[0] - (Ep - Em) / (2 * h)) < 1e-7 * abs(g[0])
    # identity probing: the derivative of the rational log det, close to tr(Q^-1 dQ)
    ident = np.arange(72)
    gi, _ = gradient.grad_estimator_rational(lattice.shifted_laplacian(shape, 0.4), [sp.diags(d)], ident, sig, coef)
    assert abs(gi[0] - gradient.grad_dense(lattice.shifted_laplacian(shape, 0.4), sp.diags(d))) < 1e-6 * abs(gi[0])
