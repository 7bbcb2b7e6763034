"""The hyperparameter fit of a directly observed lattice SPDE field (Sec. 3,
first experiment; NEXT row f1) against the oracle's exact maximiser (the
closed-form log det on the Dirichlet lattice): identity probing reproduces
it, and the probing estimates approach it as the colouring distance grows
(the trend of the paper's Table 1)."""
import sys

import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import exact, lattice
from paper_1105_5256_amd import fit, ldq, workloads

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = ldq.Context(0)
    yield c
    c.close()


def exact_fit(x, shape, eta0):
    lam = exact.lattice_eigenvalues(shape).ravel()
    n = lam.size
    L = lattice.laplacian(shape).tocsr()

    def fg(eta):
        k2, tau = np.exp(eta[0]), np.exp(eta[1])
        mx = k2 * x + L @ x
        f = -0.5 * np.sum(np.log(tau * tau * (k2 + lam) ** 2)) + 0.5 * tau * tau * (mx @ mx)
        g0 = -0.5 * k2 * np.sum(2.0 / (k2 + lam)) + tau * tau * k2 * (x @ mx)
        g1 = -n + tau * tau * (mx @ mx)
        return f, np.array([g0, g1])
    r = minimize(fg, np.asarray(eta0, float), jac=True, method="L-BFGS-B", options={"gtol": 1e-9})
    return r.x


@pytest.mark.parametrize("kappa2", [0.5, 0.05])
def test_fit_approaches_exact_with_distance(ctx, kappa2):
    shape, tau = (40, 36), 2.0
    say(f"fit {shape} kappa2={kappa2} tau={tau}")
    x = workloads.spde_field_sample(shape, kappa2, tau, seed=11)
    eta0 = (np.log(1.0), np.log(1.0))
    ex = exact_fit(x, shape, eta0)
    ident = fit.fit_spde(ctx, x, shape, 1, eta0, colouring=ldq.LDQ_COLOUR_IDENTITY)
    print(f"exact  kappa2 {np.exp(ex[0]):.6f} tau {np.exp(ex[1]):.6f}")
    print(f"ident  kappa2 {ident['kappa2']:.6f} tau {ident['tau']:.6f} evals {ident['evals']}")
    assert np.max(np.abs(ident["eta"] - ex)) < 1e-5
    errs = []
    for k in (1, 2, 3, 4, 6):
        r = fit.fit_spde(ctx, x, shape, k, eta0)
        err = float(np.max(np.abs(r["eta"] - ex)))
        errs.append(err)
        print(f"k={k}: probes {r['probes']:3d} kappa2 {r['kappa2']:.6f} tau {r['tau']:.6f} |eta - exact| {err:.2e} "
              f"evals {r['evals']} krylov iters {r['krylov_iters']} {r['seconds']:.2f} s")
        assert r["converged"]
    # the error falls with every step of the distance (small kappa2 starts further away)
    assert all(b < a for a, b in zip(errs, errs[1:]))
    assert errs[-1] < 0.1 * errs[0]
    # the schedule ends where the largest distance alone does
    sched = fit.fit_spde_schedule(ctx, x, shape, (1, 6), eta0)
    assert np.max(np.abs(sched[-1]["eta"] - ex)) < errs[-1] + 1e-5
