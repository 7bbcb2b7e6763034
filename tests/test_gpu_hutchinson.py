"""GPU parity of Hutchinson's estimator with random-sign probes (Sec. 2.1,
eq. (6) and the paragraph on confidence regions) against the oracle on the
same probes: the library draws the signs in its kernels, the oracle from its
own implementation of the same generator; every per-probe term, the mean,
the gradient and the standard error are compared.  Bounds: FP64 passes at
tol 1e-10 agree with the oracle's direct shifted solves to the Krylov
stopping error (<= 1e-8 relative); the mixed form to 1e-4 (the method's gate).
"""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import exact, hutchinson as hu, lattice, shifts
from paper_1105_5256_amd import ldq, workloads

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


def hopts(s, seed, **kw):
    return ldq.ldq_options_default(colouring=ldq.LDQ_COLOUR_RADEMACHER, nrandom=s, seed=seed, nshifts=20, **kw)


@pytest.mark.parametrize("shape,kind,precision,tol,bound", [
    ((40, 33), ldq.LDQ_SHIFTED_LAPLACIAN, ldq.LDQ_FP64, 1e-10, 1e-8),
    ((37, 29), ldq.LDQ_SQUARED_SHIFTED_LAPLACIAN, ldq.LDQ_FP64, 1e-10, 1e-8),
    ((37, 29), ldq.LDQ_SQUARED_SHIFTED_LAPLACIAN, ldq.LDQ_MIXED, 1e-5, 1e-4),
    ((16, 13, 11), ldq.LDQ_SHIFTED_LAPLACIAN, ldq.LDQ_FP64, 1e-10, 1e-8)])
def test_hutchinson_matches_oracle(ctx, shape, kind, precision, tol, bound):
    s, seed, k2 = 12, 20260101, 0.2
    say(f"hutchinson {shape} kind={kind} precision={precision} s={s}")
    n = int(np.prod(shape))
    Q = ctx.op(ldq.ldq_op_lattice(ctx.handle, shape, kind, k2))
    M = lattice.shifted_laplacian(shape, k2)
    if kind == ldq.LDQ_SQUARED_SHIFTED_LAPLACIAN:
        Qo = lattice.squared(M)
        dQ = ctx.op(ldq.ldq_op_lattice(ctx.handle, shape, ldq.LDQ_SHIFTED_LAPLACIAN, k2, scale=2.0))
        dQo = 2 * M
    else:
        Qo = M
        d = np.linspace(0.5, 1.5, n)
        dQ = ctx.op(ldq.ldq_op_diag(ctx.handle, d))
        dQo = sp.diags(d)
    v, g, info = ldq.ldq_logdet_grad(ctx.handle, Q, [dQ], hopts(s, seed, tol=tol, grad_tol=tol, precision=precision))
    terms = ldq.ldq_probe_terms(ctx.handle)
    V = hu.rademacher(n, s, seed)
    sig, coef = shifts.log_shifts(info["lambda_min"], info["lambda_max"], 20)
    H, T = hu.hutchinson_rational(Qo, V, sig, coef)
    G, _ = hu.hutchinson_grad(Qo, [dQo], V)
    print(f"logdet rel {rel(v, H):.1e}, grad rel {rel(g[0], G[0]):.1e}, max term rel "
          f"{np.max(np.abs(terms[:, 0] - T) / np.abs(T)):.1e}, std_error {info['std_error']:.3e} "
          f"vs {hu.standard_error(T):.3e}, iters {info['iters_max']}")
    assert info["ncolours"] == s and terms.shape[0] == s
    assert np.allclose(terms[:, 0], T, rtol=bound, atol=0)
    assert rel(v, H) < bound and rel(g[0], G[0]) < 10 * bound
    assert rel(info["std_error"], hu.standard_error(T)) < 1e-3 if precision == ldq.LDQ_MIXED else \
        rel(info["std_error"], hu.standard_error(T)) < 1e-6


@pytest.mark.parametrize("shape,kind,precision,with_grad", [
    ((124, 80), ldq.LDQ_SQUARED_SHIFTED_LAPLACIAN, ldq.LDQ_MIXED, True),
    ((124, 80), ldq.LDQ_SQUARED_SHIFTED_LAPLACIAN, ldq.LDQ_FP64, False),
    ((126, 80), ldq.LDQ_SHIFTED_LAPLACIAN, ldq.LDQ_MIXED, False),
    ((126, 80), ldq.LDQ_SHIFTED_LAPLACIAN, ldq.LDQ_FP64, True)])
def test_hutchinson_specialised_pass(ctx, shape, kind, precision, with_grad):
    """Random signs in the specialised 2-D pass (per-row sign masks of the
    strips; standard tiles) on lattices with interior, boundary and ragged
    tiles, in two probe blocks of two lanes each (masks offset by block and
    lane): against the oracle and against the general pass (short tiles)."""
    s, seed, k2 = 7, 0xC0FFEE, 0.3
    say(f"hutchinson specialised pass {shape} kind={kind} precision={precision} grad={with_grad}")
    n = int(np.prod(shape))
    Q = ctx.op(ldq.ldq_op_lattice(ctx.handle, shape, kind, k2))
    M = lattice.shifted_laplacian(shape, k2)
    if kind == ldq.LDQ_SQUARED_SHIFTED_LAPLACIAN:
        Qo, kd, sc = lattice.squared(M), k2, 2.0
    else:
        Qo, kd, sc = M, 1.3, 0.5
    dQ = ctx.op(ldq.ldq_op_lattice(ctx.handle, shape, ldq.LDQ_SHIFTED_LAPLACIAN, kd, scale=sc))
    dQo = sc * lattice.shifted_laplacian(shape, kd)
    tol = 1e-5 if precision == ldq.LDQ_MIXED else 1e-10
    bound = 1e-4 if precision == ldq.LDQ_MIXED else 1e-8
    # standard tiles (specialised pass) and short ones (general pass): rows
    # plus twice the halo is a multiple of five
    std_rows, gen_rows = (34, 9) if kind == ldq.LDQ_SQUARED_SHIFTED_LAPLACIAN else (36, 11)

    def run(rows):
        o = hopts(s, seed, tol=tol, grad_tol=tol, precision=precision, tile_rows=rows, lanes=2, probe_block=4)
        if with_grad:
            v, g, info = ldq.ldq_logdet_grad(ctx.handle, Q, [dQ], o)
        else:
            (v, info), g = ldq.ldq_logdet(ctx.handle, Q, o), None
        assert info["tile_rows"] == rows
        return v, g, ldq.ldq_probe_terms(ctx.handle), info

    v, g, terms, info = run(std_rows)
    vg, gg, terms_g, _ = run(gen_rows)
    V = hu.rademacher(n, s, seed)
    sig, coef = shifts.log_shifts(info["lambda_min"], info["lambda_max"], 20)
    H, T = hu.hutchinson_rational(Qo, V, sig, coef)
    print(f"logdet {v:.10g} general pass {vg:.10g} oracle {H:.10g}: rel {rel(v, H):.1e} / {rel(vg, H):.1e}; "
          f"max term rel {np.max(np.abs(terms[:, 0] - T) / np.abs(T)):.1e}; iters {info['iters_max']}")
    assert terms.shape[0] == s
    assert np.allclose(terms[:, 0], T, rtol=bound, atol=0) and np.allclose(terms_g[:, 0], T, rtol=bound, atol=0)
    assert rel(v, H) < bound and rel(vg, H) < bound
    assert np.allclose(terms[:, 0], terms_g[:, 0], rtol=bound, atol=0)
    if with_grad:
        G, _ = hu.hutchinson_grad(Qo, [dQo], V)
        print(f"grad {g[0]:.10g} general pass {gg[0]:.10g} oracle {G[0]:.10g}")
        assert rel(g[0], G[0]) < 10 * bound and rel(gg[0], G[0]) < 10 * bound


def test_hutchinson_seed_changes_probes_and_estimate_covers_exact(ctx):
    shape = (64, 64)
    say(f"hutchinson statistics {shape}")
    Q = ctx.op(ldq.ldq_op_lattice(ctx.handle, shape, ldq.LDQ_SHIFTED_LAPLACIAN, 0.3))
    exact_val = float(np.sum(np.log(0.3 + exact.lattice_eigenvalues(shape))))
    vals = []
    for seed in (1, 2, 3):
        v, info = ldq.ldq_logdet(ctx.handle, Q, hopts(64, seed, tol=1e-10))
        vals.append(v)
        print(f"seed {seed}: {v:.6f} exact {exact_val:.6f} std_error {info['std_error']:.4f}")
        assert abs(v - exact_val) <= 5 * info["std_error"]
    assert len(set(vals)) == 3


# general sparse operators: the CSR passes draw the same signs per row
@pytest.mark.parametrize("n,wide,precision,bound", [(700, False, ldq.LDQ_FP64, 1e-8),
                                                    (900, True, ldq.LDQ_FP64, 1e-8),
                                                    (700, False, ldq.LDQ_MIXED, 1e-4)])
def test_hutchinson_csr_matches_oracle(ctx, n, wide, precision, bound):
    s, seed = 10, 77
    say(f"hutchinson CSR n={n} wide={wide} precision={precision}")
    rp, ci, v = workloads.random_spd_csr(n, 20 if wide else 2, 60 if wide else 8, shift=0.05, seed=n)
    Q = ctx.op(ldq.ldq_op_csr(ctx.handle, n, rp, ci, v))
    Qm = sp.csr_matrix((v, ci, rp), shape=(n, n))
    d = np.linspace(0.5, 2.0, n)
    D = ctx.op(ldq.ldq_op_diag(ctx.handle, d))
    val, g, info = ldq.ldq_logdet_grad(ctx.handle, Q, [D], hopts(s, seed, tol=1e-10 if precision == ldq.LDQ_FP64
                                                                    else 1e-5, grad_tol=1e-10 if precision ==
                                                                    ldq.LDQ_FP64 else 1e-5, precision=precision))
    terms = ldq.ldq_probe_terms(ctx.handle)
    V = hu.rademacher(n, s, seed)
    sig, coef = shifts.log_shifts(info["lambda_min"], info["lambda_max"], 20)
    H, T = hu.hutchinson_rational(Qm, V, sig, coef)
    G, _ = hu.hutchinson_grad(Qm, [sp.diags(d)], V)
    print(f"logdet rel {rel(val, H):.1e}, grad rel {rel(g[0], G[0]):.1e}, max term rel "
          f"{np.max(np.abs(terms[:, 0] - T) / np.abs(T)):.1e}, iters {info['iters_max']}")
    assert np.allclose(terms[:, 0], T, rtol=bound, atol=0)
    assert rel(val, H) < bound and rel(g[0], G[0]) < 10 * bound
    assert rel(info["std_error"], hu.standard_error(T)) < (1e-3 if precision == ldq.LDQ_MIXED else 1e-6)


def test_hutchinson_error_paths(ctx):
    say("hutchinson error paths")
    Q = ctx.op(ldq.ldq_op_lattice(ctx.handle, (20, 20), ldq.LDQ_SHIFTED_LAPLACIAN, 0.3))
    for s in (0, -3):
        with pytest.raises(ldq.LdqError) as e:
            ldq.ldq_logdet(ctx.handle, Q, hopts(s, 1))
        assert e.value.status == ldq.LDQ_E_INVALID
