"""LogDetFn: forward value and backward gradient of log det Q(eta) through
torch autograd, for the 3-D field model log kappa2(s) = eta0 + eta1 z(s).
With identity probing both are exact: they are checked against the oracle's
exact log det (sparse LU) and central finite differences of it, and against
the oracle's exact gradient tr(Q^{-1} dQ/deta_i)."""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import exact, gradient, lattice
from paper_1105_5256_amd import ldq, workloads

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def test_logdetfn_identity_probing_matches_finite_differences():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1105_5256_amd.autograd import logdet

    shape = (12, 10, 8)
    n = int(np.prod(shape))
    say(f"LogDetFn 3-D field {shape}, identity probing ({n} probes), FP64")
    z = workloads.smooth_field(shape, 2.0, seed=3).ravel()
    ctx = ldq.Context(0)
    try:
        def build(e):
            k2 = np.exp(e[0] + e[1] * z)
            Q = ctx.op(ldq.ldq_op_lattice(ctx.handle, shape, ldq.LDQ_SHIFTED_LAPLACIAN, 0.0, kappa2_field=k2))
            d0 = ctx.op(ldq.ldq_op_diag(ctx.handle, k2))
            d1 = ctx.op(ldq.ldq_op_diag(ctx.handle, k2 * z))
            return Q, [d0, d1]

        opts = ldq.ldq_options_default(colouring=ldq.LDQ_COLOUR_IDENTITY, nshifts=24, tol=1e-11,
                                       grad_tol=1e-11)
        eta0 = np.array([np.log(0.1), 0.5])
        eta = torch.tensor(eta0, dtype=torch.float64, requires_grad=True)
        val = logdet(eta, ctx, build, opts)
        (2.5 * val).backward()

        def exact_logdet(e):
            return exact.logdet_splu(lattice.shifted_laplacian(shape, np.exp(e[0] + e[1] * z)))

        ref = exact_logdet(eta0)
        fd = gradient.grad_fd(exact_logdet, eta0, h=1e-5)
        Qm = lattice.shifted_laplacian(shape, np.exp(eta0[0] + eta0[1] * z))
        k2 = np.exp(eta0[0] + eta0[1] * z)
        gex = np.array([gradient.grad_dense(Qm, sp.diags(k2)), gradient.grad_dense(Qm, sp.diags(k2 * z))])
        g = eta.grad.numpy() / 2.5
        print(f"logdet {val.item()!r} exact {ref!r}; grad {g} fd {fd} exact {gex}")
        assert val.dtype == torch.float64 and val.dim() == 0
        assert abs(val.item() - ref) < 1e-6 * abs(ref)
        assert np.allclose(g, gex, rtol=1e-6)
        assert np.allclose(g, fd, rtol=1e-5)
    finally:
        ctx.close()
