"""Pins of oracle/krylov.py (CPU only): CG, COCG and CG-M against sparse direct
solves, and CG-M iterates against separate COCG / CG runs iteration by iteration."""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import exact, krylov, lattice, shifts


def small_problem():
    shape = (11, 9)
    Q = lattice.squared(lattice.shifted_laplacian(shape, 0.3))
    v = np.zeros(99)
    v[::7] = 1.0
    return shape, Q, v


def test_cg_and_cocg_match_direct_solves():
    _, Q, v = small_problem()
    x, _ = krylov.cg(Q, v, tol=1e-13)
    assert np.allclose(x, spla.spsolve(sp.csc_matrix(Q), v), rtol=1e-10, atol=1e-12)
    sigma = -0.4 + 1.3j
    xc, _ = krylov.cocg(Q, sigma, v, tol=1e-13)
    A = sp.csc_matrix(Q, dtype=np.complex128) - sigma * sp.identity(99, format="csc")
    ref = spla.spsolve(A, v.astype(np.complex128))
    assert np.allclose(xc, ref, rtol=1e-9, atol=1e-11)


def test_cgm_matches_direct_solves_for_contour_shifts():
    shape, Q, v = small_problem()
    lo, hi = exact.spectrum_closed_form(shape, 0.3, 2)
    sigma, _ = shifts.log_shifts(lo, hi, 12)
    x, X, _ = krylov.cg_m(Q, v, sigma, tol=1e-13)
    assert np.allclose(x, spla.spsolve(sp.csc_matrix(Q), v), rtol=1e-9, atol=1e-11)
    for l, s in enumerate(sigma):
        A = sp.csc_matrix(Q, dtype=np.complex128) - s * sp.identity(99, format="csc")
        ref = spla.spsolve(A, v.astype(np.complex128))
        assert np.linalg.norm(X[:, l] - ref) <= 1e-9 * np.linalg.norm(ref)


def test_cgm_iterates_equal_separate_cocg_and_cg_iterates():
    # shift invariance of the Krylov space: the k-th CG-M iterate of a shifted
    # system is the k-th iterate of COCG run on that system alone
    _, Q, v = small_problem()
    sig = np.array([-0.8 + 0.5j, 0.2 + 2.0j, -1.5 + 0.0j])     # last one: real shift, Q + 1.5 I
    _, _, _, hist = krylov.cg_m(Q, v, sig, tol=1e-30, maxiter=25, record=True)
    for l, s in enumerate(sig):
        _, _, ref_hist = krylov.cocg(Q, s, v, tol=1e-30, maxiter=25, record=True)
        for k in range(1, 16):
            a, b = hist[k][:, l], ref_hist[k]
            assert np.linalg.norm(a - b) <= 1e-9 * np.linalg.norm(b)
    # the real shift also equals plain CG on Q + 1.5 I
    xr, _ = krylov.cg(Q + 1.5 * sp.identity(99), v, tol=1e-14)
    _, X, _ = krylov.cg_m(Q, v, sig, tol=1e-14)
    assert np.allclose(X[:, 2].real, xr, rtol=1e-9, atol=1e-12)
    assert np.max(np.abs(X[:, 2].imag)) < 1e-12
