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
