"""Textbook Krylov solvers with materialised vectors (oracle; test infrastructure only).

Sec. 2.1, last paragraph: the Krylov spaces of Q and Q - sigma I coincide,
so one CG run on Q x = v yields, with a few scalar recurrences per shift,
the iterates of every shifted system (CG-M of Jegerlehner).  For complex
shifts the bilinear form x^T y replaces the inner product (the COCG variant
of van der Vorst & Melissen); since Q and v are real, the base CG stays real
and only the per-shift coefficients are complex.

Shift convention here: the systems are (Q - sigma_l I) x = v, as in eq. (7).
"""
import numpy as np


def cg(Q, b, tol=1e-12, maxiter=100000):
    """Plain conjugate gradients for SPD Q (real b).  Returns (x, iterations).
    Stops when ||r|| <= tol ||b||."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = r @ r
    bnorm = np.sqrt(b @ b)
    it = 0
    while np.sqrt(rr) > tol * bnorm and it < maxiter:
        q = Q @ p
        alpha = rr / (p @ q)
        x += alpha * p
        r -= alpha * q
        rr_new = r @ r
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    return x, it


def cocg(Q, sigma, b, tol=1e-12, maxiter=100000, record=False):
    """COCG for the complex symmetric system (Q - sigma I) x = b: CG with the
    bilinear form u^T w in place of the inner product.  With ``record`` the
    list of iterates x_0, x_1, ... is returned as well."""
    b = np.asarray(b, dtype=np.complex128)
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = r @ r
    bnorm = np.sqrt(np.real(np.conj(b) @ b))
    hist = [x.copy()]
    it = 0
    while np.sqrt(np.real(np.conj(r) @ r)) > tol * bnorm and it < maxiter:
        q = Q @ p - sigma * p
        alpha = rr / (p @ q)
        x = x + alpha * p
        r = r - alpha * q
        rr_new = r @ r
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
        if record:
            hist.append(x.copy())
    return (x, it, hist) if record else (x, it)


def cg_m(Q, v, sigma, tol=1e-12, maxiter=100000, record=False):
    """Multi-shift CG (CG-M) with per-shift solution and direction vectors.

    One real CG on Q x = v supplies alpha_k, beta_k; each shifted system
    (Q - sigma_l I) x^l = v gets
        zeta^l_{k+1} = zeta^l_k zeta^l_{k-1} alpha_{k-1} /
                       ( alpha_k beta_{k-1} (zeta^l_{k-1} - zeta^l_k)
                         + zeta^l_{k-1} alpha_{k-1} (1 - sigma_l alpha_k) ),
        alpha^l_k = alpha_k zeta^l_{k+1} / zeta^l_k,
        x^l += alpha^l_k p^l,
        beta^l_k = (zeta^l_{k+1} / zeta^l_k)^2 beta_k,
        p^l = zeta^l_{k+1} r_{k+1} + beta^l_k p^l,
    starting from zeta_{-1} = zeta_0 = 1, alpha_{-1} = 1, beta_{-1} = 0,
    p^l_0 = v (the shifted residual is zeta^l_k r_k).  A shifted system stops
    being updated once |zeta^l_{k+1}| ||r_{k+1}|| <= tol ||v||; the base system
    runs until every shift has stopped and ||r|| <= tol ||v||.

    Returns (x_base, X_shift (n x N complex), iterations); with ``record`` also
    the list of X_shift after every iteration.
    """
    v = np.asarray(v, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.complex128)
    N = len(sigma)
    n = len(v)
    x = np.zeros(n)
    r = v.copy()
    p = v.copy()
    rr = r @ r
    vnorm = np.sqrt(rr)
    X = np.zeros((n, N), dtype=np.complex128)
    P = np.tile(v[:, None], (1, N)).astype(np.complex128)
    zeta = np.ones(N, dtype=np.complex128)
    zeta_prev = np.ones(N, dtype=np.complex128)
    active = np.ones(N, dtype=bool)
    alpha_prev, beta_prev = 1.0, 0.0
    hist = [X.copy()] if record else None
    it = 0
    if vnorm == 0.0:
        return x, X, 0
    while it < maxiter:
        q = Q @ p
        alpha = rr / (p @ q)
        for l in np.nonzero(active)[0]:
            den = (alpha * beta_prev * (zeta_prev[l] - zeta[l])
                   + zeta_prev[l] * alpha_prev * (1.0 - sigma[l] * alpha))
            zeta_next = zeta[l] * zeta_prev[l] * alpha_prev / den
            alpha_l = alpha * zeta_next / zeta[l]
            X[:, l] += alpha_l * P[:, l]
            zeta_prev[l], zeta[l] = zeta[l], zeta_next
        x += alpha * p
        r -= alpha * q
        rr_new = r @ r
        beta = rr_new / rr
        for l in np.nonzero(active)[0]:
            beta_l = (zeta[l] / zeta_prev[l]) ** 2 * beta
            P[:, l] = zeta[l] * r + beta_l * P[:, l]
        p = r + beta * p
        rr = rr_new
        alpha_prev, beta_prev = alpha, beta
        it += 1
        if record:
            hist.append(X.copy())
        rnorm = np.sqrt(rr)
        active &= np.abs(zeta) * rnorm > tol * vnorm
        if not active.any() and rnorm <= tol * vnorm:
            break
    return (x, X, it, hist) if record else (x, X, it)
