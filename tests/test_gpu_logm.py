"""GPU parity of f_N(Q) V (the rational approximation of log(Q), eq. (7) of
Sec. 2.1, applied to vectors; NEXT row f3) against the oracle's direct
shifted solves with the same shifts.  Bound: the Krylov stopping error of the
two solves (FP64, tol 1e-11: 1e-8 relative in the 2-norm; mixed: 1e-4)."""
import sys

import numpy as np
import pytest

from oracle import fnapply, lattice, shifts
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


@pytest.mark.parametrize("shape,kind,precision,tol,bound", [
    ((30, 25), ldq.LDQ_SHIFTED_LAPLACIAN, ldq.LDQ_FP64, 1e-11, 1e-8),
    ((24, 21), ldq.LDQ_SQUARED_SHIFTED_LAPLACIAN, ldq.LDQ_FP64, 1e-11, 1e-8),
    ((10, 9, 8), ldq.LDQ_SHIFTED_LAPLACIAN, ldq.LDQ_FP64, 1e-11, 1e-8),
    ((30, 25), ldq.LDQ_SHIFTED_LAPLACIAN, ldq.LDQ_MIXED, 1e-6, 1e-4)])
def test_logm_apply_matches_oracle(ctx, shape, kind, precision, tol, bound):
    import torch
    say(f"f_N(Q) V {shape} kind={kind} precision={precision}")
    n = int(np.prod(shape))
    k2 = 0.3
    Q = ctx.op(ldq.ldq_op_lattice(ctx.handle, shape, kind, k2))
    M = lattice.shifted_laplacian(shape, k2)
    Qo = lattice.squared(M) if kind == ldq.LDQ_SQUARED_SHIFTED_LAPLACIAN else M
    rng = np.random.default_rng(7)
    V = np.zeros((4, n))
    V[:3] = rng.standard_normal((3, n))
    V[3, n // 2 + shape[0] // 2] = 1.0                  # a unit vector near the centre
    Vt = torch.tensor(V, dtype=torch.float64, device="cuda")
    opts = ldq.ldq_options_default(tol=tol, precision=precision, nshifts=20)
    Y, info = ldq.ldq_logm_apply(ctx.handle, Q, Vt, opts)
    Y = Y.cpu().numpy()
    sig, coef = shifts.log_shifts(info["lambda_min"], info["lambda_max"], 20)
    Yo = fnapply.logm_apply_rational(Qo, V.T, sig, coef).T
    err = np.linalg.norm(Y - Yo, axis=1) / np.linalg.norm(Yo, axis=1)
    print(f"rel errors {err}, iterations {info['iters_max']}")
    assert np.all(err < bound)
    # v^T f_N(Q) v is the probe's log det term
    assert np.allclose(np.sum(V * Y, axis=1), np.sum(V * Yo, axis=1), rtol=10 * bound)


def test_logm_apply_error_paths(ctx):
    import torch
    say("f_N(Q) V error paths")
    rp = np.arange(5, dtype=np.int32)
    ci = np.arange(4, dtype=np.int32)
    C = ctx.op(ldq.ldq_op_csr(ctx.handle, 4, rp, ci, np.full(4, 2.0)))
    with pytest.raises(ldq.LdqError) as e:
        ldq.ldq_logm_apply(ctx.handle, C, torch.ones(1, 4, dtype=torch.float64, device="cuda"))
    assert e.value.status == ldq.LDQ_E_UNSUPPORTED
    # host memory is refused through the C ABI (the kernels could not read it)
    import ctypes
    Q = ctx.op(ldq.ldq_op_lattice(ctx.handle, (6, 5), ldq.LDQ_SHIFTED_LAPLACIAN, 0.5))
    host = np.ones(30)
    out = np.zeros(30)
    opts = ldq.ldq_options_default()
    st = ldq.load().ldq_logm_apply(ctx.handle, Q, 1, host.ctypes.data_as(ctypes.c_void_p),
                                   out.ctypes.data_as(ctypes.c_void_p), ctypes.byref(opts), None)
    assert st == ldq.LDQ_E_INVALID
