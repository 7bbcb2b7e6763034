"""Hyperparameter estimation for a directly observed lattice SPDE field.

Sec. 3, first experiment (with the objective of Sec. 1, eq. (4), for a field
observed without noise): the field x on an mx x my lattice has precision

    Q(eta) = tau^2 (kappa2 I + L)^2,   eta = (log kappa2, log tau),

L the 5-point Dirichlet Laplacian, and the negative log-likelihood is, up to
a constant,

    f(eta) = -1/2 log det Q(eta) + 1/2 x^T Q(eta) x,
    df/dlog kappa2 = -1/2 kappa2 tr(Q^{-1} dQ/dkappa2) + tau^2 kappa2 x^T (kappa2 I + L) x,
    df/dlog tau    = -n + tau^2 |(kappa2 I + L) x|^2,

with dQ/dkappa2 = 2 tau^2 (kappa2 I + L) and tr(Q^{-1} dQ/dlog tau) = 2n
exactly (Q scales with tau^2).  log det Q and tr(Q^{-1} dQ/dkappa2) are the
library's probing estimates at colouring distance k (or its identity probing,
exact up to the quadrature); the quadratic form runs on the device (torch,
FP64).  The minimiser is scipy's L-BFGS-B.  The paper's point (its Table 1)
is that the estimates approach those with the exact log det as k grows and
that small kappa needs larger k; `fit_spde` returns what is needed to show
that.  The paper also schedules the distance (small k early, large k late):
`fit_spde_schedule` warm-starts each distance from the previous estimate.

Noisy observations (the Gauss-linear model of Sec. 1, eq. (1)-(3)):
`objective_noisy` / `fit_noisy` take data y = A x + e, with the posterior
mean from the library's solve (ldq_solve) and both log dets (field and
posterior precision) from its estimates.
"""
import time

import numpy as np

from . import ldq


def _apply_m(xg, kappa2):
    """(kappa2 I + L) x on the lattice (x as an (my, mx) torch tensor, zero outside)."""
    import torch.nn.functional as F
    p = F.pad(xg[None, None], (1, 1, 1, 1))[0, 0]
    return (kappa2 + 4.0) * xg - (p[:-2, 1:-1] + p[2:, 1:-1] + p[1:-1, :-2] + p[1:-1, 2:])


def objective(ctx, x, shape, eta, opts):
    """(f, grad f) at eta = (log kappa2, log tau) for the field x (torch FP64 on the device)."""
    kappa2, tau = float(np.exp(eta[0])), float(np.exp(eta[1]))
    n = int(np.prod(shape))
    h = ctx.handle
    Q = ldq.ldq_op_lattice(h, shape, ldq.LDQ_SQUARED_SHIFTED_LAPLACIAN, kappa2, scale=tau * tau)
    dQ = ldq.ldq_op_lattice(h, shape, ldq.LDQ_SHIFTED_LAPLACIAN, kappa2, scale=2.0 * tau * tau)
    try:
        ld, g, info = ldq.ldq_logdet_grad(h, Q, [dQ], opts)
    finally:
        ldq.ldq_op_destroy(Q)
        ldq.ldq_op_destroy(dQ)
    xg = x.reshape(shape[1], shape[0])
    mx_ = _apply_m(xg, kappa2)
    xmx = float((xg * mx_).sum())
    mm = float((mx_ * mx_).sum())
    f = -0.5 * ld + 0.5 * tau * tau * mm
    df = np.array([-0.5 * kappa2 * g[0] + tau * tau * kappa2 * xmx, -n + tau * tau * mm])
    return f, df, info


def fit_spde(ctx, x, shape, k, eta0, colouring=ldq.LDQ_COLOUR_MODULAR, tol=1e-9, precision=ldq.LDQ_FP64,
             gtol=1e-7, maxiter=200):
    """Estimate eta = (log kappa2, log tau) from the field x with the probing
    estimate at colouring distance k.  Returns a dict with the estimate, the
    objective, the evaluations made, their Krylov iterations and seconds."""
    from scipy.optimize import minimize
    import torch
    xt = torch.as_tensor(np.asarray(x, dtype=np.float64), device="cuda")
    opts = ldq.ldq_options_default(k=k, colouring=colouring, tol=tol, grad_tol=tol, precision=precision)
    stats = {"evals": 0, "iters": 0, "probes": 0}

    def fg(eta):
        f, df, info = objective(ctx, xt, shape, eta, opts)
        stats["evals"] += 1
        stats["iters"] += info["iters_total"]
        stats["probes"] = info["ncolours"]
        return f, df

    t0 = time.perf_counter()
    res = minimize(fg, np.asarray(eta0, dtype=np.float64), jac=True, method="L-BFGS-B",
                   options={"gtol": gtol, "maxiter": maxiter})
    secs = time.perf_counter() - t0
    return {"k": k, "eta": res.x, "kappa2": float(np.exp(res.x[0])), "tau": float(np.exp(res.x[1])),
            "f": float(res.fun), "evals": stats["evals"], "krylov_iters": stats["iters"], "probes": stats["probes"],
            "seconds": secs, "converged": bool(res.success)}


def fit_spde_schedule(ctx, x, shape, ks, eta0, **kw):
    """The distance schedule: fit at ks[0], then warm-start each larger distance."""
    out, eta = [], np.asarray(eta0, dtype=np.float64)
    for k in ks:
        r = fit_spde(ctx, x, shape, k, eta, **kw)
        out.append(r)
        eta = r["eta"]
    return out


# ----------------------------------------------- noisy observations (Sec. 1)
def obs_adjoint(y, corner, weight, n):
    """A^T y for the bilinear observation operator (host, once per data set)."""
    out = np.zeros(n)
    np.add.at(out, np.asarray(corner, dtype=np.int64).ravel(),
              (np.asarray(weight, dtype=np.float64) * np.asarray(y, dtype=np.float64)[:, None]).ravel())
    return out


def objective_noisy(ctx, data, shape, theta, opts):
    """(F, grad F, info) at theta = (log kappa2, log tau_x, log tau_y) for data
    y = A x + e of the Gauss-linear model of Sec. 1 (eq. (1)-(3)): field
    precision Q_x = tau_x^2 (kappa2 I + L)^2, noise precision tau_y I,
    posterior precision Q_p = Q_x + tau_y A^T A, b = tau_y A^T y,
    mu = Q_p^{-1} b (ldq_solve), and

        F = -2 log p(y) = -log det Q_x + log det Q_p - m log tau_y
                          + tau_y y^T y - b^T mu + m log(2 pi).

    With M = kappa2 I + L and the envelope identity d(b^T Q_p^{-1} b) =
    2 db^T mu - mu^T dQ_p mu:
      dF/dlog kappa2 = kappa2 (-tr(Q_x^{-1} dQ) + tr(Q_p^{-1} dQ) + mu^T dQ mu),
                       dQ = 2 tau_x^2 M;
      dF/dlog tau_x  = -2n + 2 (n - tau_y tr(Q_p^{-1} A^T A)) + 2 tau_x^2 |M mu|^2;
      dF/dlog tau_y  = tau_y tr(Q_p^{-1} A^T A) - m + tau_y |y - A mu|^2.
    The log dets and traces are the library's estimates (opts), mu its solve;
    `data` holds y, corner, weight (host arrays) and their device copies."""
    import torch
    kappa2, taux, tauy = (float(v) for v in np.exp(np.asarray(theta, dtype=np.float64)))
    n = int(np.prod(shape))
    y, corner, weight = data["y"], data["corner"], data["weight"]
    m = y.shape[0]
    h = ctx.handle
    Qx = ldq.ldq_op_lattice(h, shape, ldq.LDQ_SQUARED_SHIFTED_LAPLACIAN, kappa2, scale=taux * taux)
    Qp = ldq.ldq_op_lattice(h, shape, ldq.LDQ_SQUARED_SHIFTED_LAPLACIAN, kappa2, scale=taux * taux)
    dQ = ldq.ldq_op_lattice(h, shape, ldq.LDQ_SHIFTED_LAPLACIAN, kappa2, scale=2.0 * taux * taux)
    G = None
    try:
        ldq.ldq_op_add_obs(Qp, corner, weight, tauy)
        G = ldq.ldq_op_obs_gram(h, Qp, corner, weight)
        ldx, gx, info = ldq.ldq_logdet_grad(h, Qx, [dQ], opts)
        ldp, gp, _ = ldq.ldq_logdet_grad(h, Qp, [dQ, G], opts)
        b = tauy * data["aty_d"]
        mu = ldq.ldq_solve(h, Qp, b[None].contiguous(), opts)[0][0]
    finally:
        for op in (Qx, Qp, dQ, G):
            if op is not None:
                ldq.ldq_op_destroy(op)
    yd, cd, wd = data["y_d"], data["corner_d"], data["weight_d"]
    amu = (wd * mu[cd]).sum(dim=1)
    mg = mu.reshape(shape[1], shape[0])
    mmu = _apply_m(mg, kappa2)
    mu_m_mu = float((mg * mmu).sum())
    m_mu2 = float((mmu * mmu).sum())
    res2 = float(((yd - amu) ** 2).sum())
    F = -ldx + ldp - m * np.log(tauy) + tauy * float(yd @ yd) - float(b @ mu) + m * np.log(2.0 * np.pi)
    dF = np.array([kappa2 * (-gx[0] + gp[0] + 2.0 * taux * taux * mu_m_mu),
                   -2.0 * n + 2.0 * (n - tauy * gp[1]) + 2.0 * taux * taux * m_mu2,
                   tauy * gp[1] - m + tauy * res2])
    return F, dF, info


def noisy_data(y, corner, weight, shape):
    """The data of objective_noisy: host arrays and their device copies."""
    import torch
    n = int(np.prod(shape))
    y = np.asarray(y, dtype=np.float64)
    corner = np.ascontiguousarray(corner, dtype=np.int32)
    weight = np.ascontiguousarray(weight, dtype=np.float64)
    dev = dict(device="cuda")
    return dict(y=y, corner=corner, weight=weight,
                y_d=torch.as_tensor(y, **dev), corner_d=torch.as_tensor(corner.astype(np.int64), **dev),
                weight_d=torch.as_tensor(weight, **dev),
                aty_d=torch.as_tensor(obs_adjoint(y, corner, weight, n), **dev))


def fit_noisy(ctx, y, corner, weight, shape, k, theta0, colouring=ldq.LDQ_COLOUR_MODULAR, tol=1e-9,
              precision=ldq.LDQ_FP64, gtol=1e-7, maxiter=200):
    """Estimate theta = (log kappa2, log tau_x, log tau_y) from noisy
    observations y = A x + e by minimising objective_noisy (L-BFGS-B).
    Returns a dict with the estimate, the objective and the evaluations made."""
    from scipy.optimize import minimize
    data = noisy_data(y, corner, weight, shape)
    opts = ldq.ldq_options_default(k=k, colouring=colouring, tol=tol, grad_tol=tol, precision=precision)
    stats = {"evals": 0, "iters": 0}

    def fg(theta):
        F, dF, info = objective_noisy(ctx, data, shape, theta, opts)
        stats["evals"] += 1
        stats["iters"] += info["iters_total"]
        return F, dF

    t0 = time.perf_counter()
    res = minimize(fg, np.asarray(theta0, dtype=np.float64), jac=True, method="L-BFGS-B",
                   options={"gtol": gtol, "maxiter": maxiter})
    return dict(theta=res.x, f=float(res.fun), success=bool(res.success), seconds=time.perf_counter() - t0,
                **stats)
