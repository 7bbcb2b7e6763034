r"""Contour-quadrature rational approximation of log (oracle; test infrastructure only).

Sec. 2.1, eq. (7): log(Q) v ~ f_N(Q) v = sum_{l=1}^N alpha_l (Q - sigma_l I)^{-1} v,
obtained from Cauchy's integral log(Q) = (1 / 2 pi i) \oint log(z) (z I - Q)^{-1} dz
over a contour around the spectrum, discretised by the midpoint rule of
Hale, Higham & Trefethen after a conformal map that needs the extremal
eigenvalues [m, M] of Q.

Reading of the paper (it is garbled here): the 1/(2 pi i) factor and the
integrand log(z) are restored; the nodes are those of the square-root variant
of the conformal map (the spectrum of Q^{1/2} lies in [sqrt m, sqrt M], the
substitution z = w^2 turns the integrand into 4 w log(w) (w^2 - Q)^{-1}), with
N midpoint nodes on the upper half of the contour; the lower half contributes
the complex conjugate, so for real lambda

    log(lambda) ~ Im sum_l c_l / (lambda - sigma_l),   sigma_l = w_l^2,

with c_l = (2K / (pi N)) * 4 w_l log(w_l) w'(t_l) (orientation of the contour
and the sign of (z I - Q)^{-1} versus (Q - sigma I)^{-1} are absorbed in c_l).  N counts the
distinct complex shifts; their conjugates are implicit in "Im".
The error decays like exp(-2 pi^2 N / (log(M/m) + 6)); the paper prints 2 pi N
in the exponent, which the measured convergence does not follow.
"""
import numpy as np
import scipy.special as ss


def jacobi_sn_cn_dn(t, m):
    """sn, cn, dn of a complex argument t = x + i y with parameter m = k^2.

    Uses the addition theorem with Jacobi's imaginary transformation
    (sn, cn, dn of the real parts x at parameter m and of y at 1 - m):
      sn = (s d1 + i c d s1 c1) / D, cn = (c c1 - i s d s1 d1) / D,
      dn = (d c1 d1 - i m s c s1) / D,  D = c1^2 + m s^2 s1^2.
    """
    t = np.asarray(t, dtype=np.complex128)
    s, c, d, _ = ss.ellipj(t.real, m)
    s1, c1, d1, _ = ss.ellipj(t.imag, 1.0 - m)
    den = c1 ** 2 + m * s ** 2 * s1 ** 2
    sn = (s * d1 + 1j * c * d * s1 * c1) / den
    cn = (c * c1 - 1j * s * d * s1 * d1) / den
    dn = (d * c1 * d1 - 1j * m * s * c * s1) / den
    return sn, cn, dn


def log_shifts(lmin, lmax, N):
    """Shifts sigma_l and weights c_l (complex, l = 1..N) of the rational
    approximation log(lambda) ~ Im sum_l c_l / (lambda - sigma_l) on [lmin, lmax]."""
    if not (0.0 < lmin <= lmax):
        raise ValueError("need 0 < lmin <= lmax")
    # A nearly degenerate enclosure makes the modulus of the map vanish and the
    # elliptic functions lose accuracy; any wider interval still encloses the
    # spectrum, so the ratio M/m is raised to at least 1.01.
    lmax = max(lmax, 1.01 * lmin)
    r = (lmax / lmin) ** 0.25                 # sqrt(b / a) for [a, b] = [sqrt m, sqrt M]
    c0 = (lmin * lmax) ** 0.25                # sqrt(a b)
    k = (r - 1.0) / (r + 1.0)                 # modulus of the map
    K = ss.ellipk(k * k)
    Kp = ss.ellipk(1.0 - k * k)
    l = np.arange(1, N + 1)
    t = -K + 0.5j * Kp + (l - 0.5) * 2.0 * K / N
    sn, cn, dn = jacobi_sn_cn_dn(t, k * k)
    w = c0 * (1.0 / k + sn) / (1.0 / k - sn)
    dw = c0 * (2.0 / k) * cn * dn / (1.0 / k - sn) ** 2
    sigma = w * w
    coef = (2.0 * K / (np.pi * N)) * 4.0 * w * np.log(w) * dw
    return sigma, coef


def rational_log(lam, sigma, coef):
    """f_N(lambda) = Im sum_l c_l / (lambda - sigma_l) for real lambda (array)."""
    lam = np.asarray(lam, dtype=np.float64)
    return np.imag(np.sum(coef[None, :] / (lam[:, None] - sigma[None, :]), axis=1))
