"""GPU parity of the consistent gradient (the derivative of the probing log
det estimate with the shifts fixed; NEXT row f3) against the oracle's direct
shifted solves on the same colouring and shifts.  Bound: the Krylov stopping
error (FP64 tol 1e-11: 1e-7 relative; mixed: 1e-3)."""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import colouring, gradient, lattice, shifts
from paper_1105_5256_amd import ldq

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


def rel(a, b):
    return abs(a - b) / abs(b)


@pytest.mark.parametrize("shape,kind,k,precision,tol,bound", [
    ((30, 25), ldq.LDQ_SHIFTED_LAPLACIAN, 2, ldq.LDQ_FP64, 1e-11, 1e-7),
    ((24, 21), ldq.LDQ_SQUARED_SHIFTED_LAPLACIAN, 2, ldq.LDQ_FP64, 1e-11, 1e-7),
    ((10, 9, 8), ldq.LDQ_SHIFTED_LAPLACIAN, 2, ldq.LDQ_FP64, 1e-11, 1e-7),
    ((30, 25), ldq.LDQ_SHIFTED_LAPLACIAN, 2, ldq.LDQ_MIXED, 1e-6, 1e-3)])
def test_consistent_gradient_matches_oracle(ctx, shape, kind, k, precision, tol, bound):
    say(f"consistent gradient {shape} kind={kind} precision={precision}")
    n = int(np.prod(shape))
    k2 = 0.3
    Q = ctx.op(ldq.ldq_op_lattice(ctx.handle, shape, kind, k2))
    M = lattice.shifted_laplacian(shape, k2)
    d = np.random.default_rng(1).uniform(0.2, 3.0, n)   # uneven: the two gradients differ
    D = ctx.op(ldq.ldq_op_diag(ctx.handle, d))
    if kind == ldq.LDQ_SQUARED_SHIFTED_LAPLACIAN:
        Qo = lattice.squared(M)
        S = ctx.op(ldq.ldq_op_lattice(ctx.handle, shape, ldq.LDQ_SHIFTED_LAPLACIAN, k2, scale=2.0))
        dQs, dQo = [S, D], [2 * M, sp.diags(d)]
        radius = 2 * k
    else:
        Qo = M
        S = ctx.op(ldq.ldq_op_lattice(ctx.handle, shape, ldq.LDQ_SHIFTED_LAPLACIAN, 0.7, scale=0.5))
        dQs, dQo = [D, S], [sp.diags(d), 0.5 * lattice.shifted_laplacian(shape, 0.7)]
        radius = k
    opts = ldq.ldq_options_default(k=k, tol=tol, grad_tol=tol, precision=precision, consistent_grad=1)
    v, g, info = ldq.ldq_logdet_grad(ctx.handle, Q, dQs, opts)
    C, co = colouring.find_modular(len(shape), radius)
    col = colouring.modular_colouring(shape, C, co)
    sig, coef = shifts.log_shifts(info["lambda_min"], info["lambda_max"], 20)
    G, _ = gradient.grad_estimator_rational(Qo, dQo, col, sig, coef)
    # the probing gradient (default) differs from the derivative of the estimate
    _, gp, _ = ldq.ldq_logdet_grad(ctx.handle, Q, dQs, ldq.ldq_options_default(k=k, tol=tol, grad_tol=tol,
                                                                               precision=precision))
    print(f"consistent {g} oracle {G} rel {[rel(a, b) for a, b in zip(g, G)]}; probing gradient {gp}")
    assert info["ncolours"] == C
    for a, b in zip(g, G):
        assert rel(a, b) < bound
    # the diagonal derivative: the probing gradient misses the estimate's derivative by far more
    idiag = 1 if kind == ldq.LDQ_SQUARED_SHIFTED_LAPLACIAN else 0
    assert rel(gp[idiag], G[idiag]) > 1e-4 and rel(gp[idiag], G[idiag]) > 100 * rel(g[idiag], G[idiag])


@pytest.mark.parametrize("precision,tol,bound", [(ldq.LDQ_FP64, 1e-11, 1e-7), (ldq.LDQ_MIXED, 1e-6, 1e-3)])
def test_consistent_gradient_observation_gram(ctx, precision, tol, bound):
    """The posterior precision Q_p = (kappa2 I + L)^2 + tau A^T A with the
    derivatives 2 (kappa2 I + L) and the observation gram A^T A."""
    from paper_1105_5256_amd import workloads
    shape, k2, tau, k = (26, 22), 0.3, 4.0, 2
    say(f"consistent gradient, observation gram {shape} precision={precision}")
    n = int(np.prod(shape))
    corner, weight = workloads.observations(shape, 120, 3)
    Q = ctx.op(ldq.ldq_op_lattice(ctx.handle, shape, ldq.LDQ_SQUARED_SHIFTED_LAPLACIAN, k2))
    ldq.ldq_op_add_obs(Q, corner, weight, tau)
    S = ctx.op(ldq.ldq_op_lattice(ctx.handle, shape, ldq.LDQ_SHIFTED_LAPLACIAN, k2, scale=2.0))
    G = ctx.op(ldq.ldq_op_obs_gram(ctx.handle, Q, corner, weight))
    M = lattice.shifted_laplacian(shape, k2)
    Qo = lattice.posterior_precision(lattice.squared(M), corner, weight, tau)
    dQo = [2 * M, lattice.observation_gram(n, corner, weight)]
    opts = ldq.ldq_options_default(k=k, tol=tol, grad_tol=tol, precision=precision, consistent_grad=1)
    v, g, info = ldq.ldq_logdet_grad(ctx.handle, Q, [S, G], opts)
    C, co = colouring.find_modular(2, 2 * k)
    col = colouring.modular_colouring(shape, C, co)
    sig, coef = shifts.log_shifts(info["lambda_min"], info["lambda_max"], 20)
    Gr, _ = gradient.grad_estimator_rational(Qo, dQo, col, sig, coef)
    print(f"consistent {g} oracle {Gr} rel {[rel(a, b) for a, b in zip(g, Gr)]}")
    assert info["ncolours"] == C
    for a, b in zip(g, Gr):
        assert rel(a, b) < bound
