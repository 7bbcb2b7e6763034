"""Pins of oracle/estimator.py (CPU only): the probing estimator by independent
routes, the identity-probing invariant and the trend of Table 1."""
import numpy as np
import pytest

from oracle import colouring, estimator, exact, lattice, shifts


def lattice_case(shape, kappa2, power):
    M = lattice.shifted_laplacian(shape, kappa2)
    return M if power == 1 else lattice.squared(M)


@pytest.mark.parametrize("shape,kappa2,power,radius", [((9, 7), 0.1, 1, 2), ((8, 10), 0.05, 2, 8),
                                                       ((5, 4, 6), 0.2, 1, 2)])
def test_exact_estimator_routes_agree(shape, kappa2, power, radius):
    Q = lattice_case(shape, kappa2, power)
    C, co = colouring.find_modular(len(shape), radius)
    c = colouring.modular_colouring(shape, C, co)
    e1, t1 = estimator.estimator_dst(shape, kappa2, c, power)
    e2, t2 = estimator.estimator_eigh(Q, c)
    e3, _ = estimator.estimator_logm(Q, c)
    assert abs(e1 - e2) < 1e-11 * abs(e2) and abs(e3 - e2) < 1e-9 * abs(e2)
    assert np.allclose(t1, t2, rtol=1e-10, atol=1e-12)


def test_identity_probing_is_exact():
    # Sec. 2.1: tr log Q = sum_i e_i^T log(Q) e_i
    shape, kappa2 = (10, 8), 0.1
    Q = lattice_case(shape, kappa2, 2)
    ident = np.arange(80)
    cf = exact.logdet_closed_form(shape, kappa2, 2)
    assert abs(estimator.estimator_dst(shape, kappa2, ident, 2)[0] - cf) < 1e-11 * abs(cf)
    lo, hi = exact.spectrum_closed_form(shape, kappa2, 2)
    s, c = shifts.log_shifts(lo, hi, 24)
    e, _, _ = estimator.estimator_cgm(Q, ident, s, c, tol=1e-12)
    assert abs(e - cf) < 1e-9 * abs(cf)


def test_rational_routes_agree_and_approach_exact():
    shape, kappa2 = (12, 11), 0.05
    Q = lattice_case(shape, kappa2, 2)
    C, co = colouring.find_modular(2, 8)
    c = colouring.modular_colouring(shape, C, co)
    lo, hi = exact.spectrum_closed_form(shape, kappa2, 2)
    exact_e, _ = estimator.estimator_dst(shape, kappa2, c, 2)
    s, w = shifts.log_shifts(lo, hi, 20)
    e_direct, t_direct = estimator.estimator_rational_direct(Q, c, s, w)
    e_cgm, t_cgm, _ = estimator.estimator_cgm(Q, c, s, w, tol=1e-13)
    assert np.allclose(t_direct, t_cgm, rtol=1e-10, atol=1e-12)
    # quadrature error: |f_N - log| <= err on [lo, hi] gives |E_N - E| <= err * sum ||v_j||^2 = err * n
    lam = np.geomspace(lo, hi, 400)
    err = np.max(np.abs(shifts.rational_log(lam, s, w) - np.log(lam)))
    assert abs(e_direct - exact_e) <= 2.0 * err * Q.shape[0] + 1e-10


def test_larger_colouring_distance_approaches_exact():
    # Table 1 / Sec. 3: larger distance colourings give results closer to the exact determinant
    shape, kappa2 = (24, 24), 0.1
    Q = lattice_case(shape, kappa2, 1)
    cf = exact.logdet_closed_form(shape, kappa2, 1)
    errs = []
    for k in (1, 2, 4, 6, 8):
        c = colouring.greedy_colouring(Q, k)
        errs.append(abs(estimator.estimator_dst(shape, kappa2, c, 1)[0] - cf))
    assert all(a > b for a, b in zip(errs, errs[1:]))
