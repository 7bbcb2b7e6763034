"""Pins of oracle/exact.py: closed-form eigenvalues, Cholesky, LU and eigh agree,
and the log det obeys its scaling and squaring identities (CPU only)."""
import numpy as np
import pytest

from oracle import exact, lattice


@pytest.mark.parametrize("shape", [(6,), (5, 4), (3, 4, 5)])
def test_lattice_eigenvalues_match_eigvalsh(shape):
    lam = np.sort(exact.lattice_eigenvalues(shape).ravel())
    ref = np.linalg.eigvalsh(lattice.laplacian_bruteforce(shape))
    assert np.allclose(lam, ref, atol=1e-12)


@pytest.mark.parametrize("shape,kappa2,power", [((9, 8), 0.1, 1), ((7, 9), 0.05, 2), ((4, 5, 3), 0.3, 1)])
def test_logdet_routes_agree(shape, kappa2, power):
    M = lattice.shifted_laplacian(shape, kappa2)
    Q = M if power == 1 else lattice.squared(M)
    cf = exact.logdet_closed_form(shape, kappa2, power)
    ref = np.linalg.slogdet(Q.toarray())
    assert ref[0] == 1.0
    for val in (exact.logdet_dense_cholesky(Q), exact.logdet_banded_cholesky(Q),
                exact.logdet_splu(Q), exact.logdet_eigh(Q)):
        assert abs(val - cf) <= 1e-11 * abs(cf)
    assert abs(ref[1] - cf) <= 1e-11 * abs(cf)


def test_scaling_and_squaring_identities():
    shape = (8, 6)
    M = lattice.shifted_laplacian(shape, 0.2)
    n = 48
    ld = exact.logdet_dense_cholesky(M)
    assert abs(exact.logdet_dense_cholesky(3.5 * M) - (n * np.log(3.5) + ld)) < 1e-11 * abs(ld)
    assert abs(exact.logdet_dense_cholesky(lattice.squared(M)) - 2 * ld) < 1e-11 * abs(ld)


def test_spectrum_closed_form_and_bounds():
    shape = (6, 5)
    lo, hi = exact.spectrum_closed_form(shape, 0.05, 2)
    lam = np.linalg.eigvalsh(lattice.squared(lattice.shifted_laplacian(shape, 0.05)).toarray())
    assert abs(lam[0] - lo) < 1e-12 and abs(lam[-1] - hi) < 1e-11
    assert exact.gershgorin_upper(lattice.squared(lattice.shifted_laplacian(shape, 0.05))) >= hi
    # field diagonal: Weyl's inequality encloses the spectrum by the extremes of kappa2
    k2 = np.random.default_rng(0).uniform(0.01, 1.0, 60)
    Mf = lattice.shifted_laplacian((3, 4, 5), k2).toarray()
    lamL = exact.lattice_eigenvalues((3, 4, 5))
    ev = np.linalg.eigvalsh(Mf)
    assert ev[0] >= k2.min() + lamL.min() - 1e-12 and ev[-1] <= k2.max() + lamL.max() + 1e-12
