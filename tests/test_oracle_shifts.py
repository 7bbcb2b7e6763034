"""Pins of oracle/shifts.py (CPU only): elliptic functions against mpmath, and the
rational approximation against log itself with the geometric convergence rate."""
import mpmath
import numpy as np
import pytest

from oracle import shifts


def test_complex_jacobi_functions_match_mpmath():
    m = 0.37
    for t in (0.3 + 0.2j, -1.1 + 0.9j, 0.7 - 0.4j, -0.2 + 1.3j):
        sn, cn, dn = shifts.jacobi_sn_cn_dn(np.array([t]), m)
        for ours, name in ((sn[0], "sn"), (cn[0], "cn"), (dn[0], "dn")):
            ref = complex(mpmath.ellipfun(name, t, m=m))
            assert abs(ours - ref) < 1e-13 * max(1.0, abs(ref))


@pytest.mark.parametrize("lmin,lmax", [(0.1046, 8.0953), (0.0025, 64.8), (1.06e-4, 81.0), (0.5, 0.5000001)])
def test_rational_log_error_and_rate(lmin, lmax):
    lam = np.geomspace(lmin, lmax, 200)
    errs = {}
    for N in (8, 12, 16, 20, 30):
        s, c = shifts.log_shifts(lmin, lmax, N)
        assert np.all(s.imag > 0)                      # upper half-plane nodes
        errs[N] = np.max(np.abs(shifts.rational_log(lam, s, c) - np.log(lam)))
    rate = 2 * np.pi ** 2 / (np.log(lmax / lmin) + 6.0)
    # the error decays like exp(-rate N) until rounding takes over
    for N in (8, 12, 16, 20, 30):
        assert errs[N] <= max(200.0 * np.exp(-rate * N), 5e-14)
    if errs[12] > 1e-11:
        observed = np.log(errs[8] / errs[12]) / 4.0
        assert 0.7 * rate < observed < 1.4 * rate


def test_shift_rule_scales_with_the_interval():
    # log(c lambda) = log c + log lambda: nodes for [c m, c M] are c sigma and the
    # weights give Im sum c_l' / (c lambda - c sigma_l) = f(lambda) + log c
    s1, c1 = shifts.log_shifts(0.2, 30.0, 20)
    s2, c2 = shifts.log_shifts(0.2 * 7.0, 30.0 * 7.0, 20)
    assert np.allclose(s2, 7.0 * s1, rtol=1e-12)
    lam = np.geomspace(0.2, 30.0, 50)
    assert np.allclose(shifts.rational_log(7.0 * lam, s2, c2),
                       shifts.rational_log(lam, s1, c1) + np.log(7.0), atol=1e-12)
