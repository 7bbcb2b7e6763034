"""log det Q(eta) as a differentiable torch function.

The forward pass runs the library's log det and gradient in one call (the
gradient g_i = sum_j x_j^T (dQ/deta_i) v_j comes from the same Krylov run as
the log det); the backward pass only scales the saved gradient by the
incoming gradient, so no second Krylov run is needed.  The gradient is the
probing estimate of tr(Q^{-1} dQ/deta_i) -- with identity probing it is the
exact derivative of log det Q.
"""
import numpy as np
import torch

from . import ldq


class LogDetFn(torch.autograd.Function):
    """LogDetFn.apply(eta, context, build, opts) -> 0-dim FP64 tensor.

    eta      1-D tensor of hyperparameters (any device; FP64 recommended)
    context  an ldq.Context
    build    callable(eta as a numpy array) -> (Q handle, [dQ/deta_i handles]);
             the handles are owned by the caller (e.g. registered with
             context.op) and must stay valid during the call
    opts     ldq_options (None: library defaults)
    """

    @staticmethod
    def forward(ctx, eta, context, build, opts=None):
        e = eta.detach().to("cpu", torch.float64).numpy()
        Q, dQ = build(e)
        if len(dQ) != e.size:
            raise ValueError(f"build returned {len(dQ)} derivative operators for {e.size} parameters")
        val, grad, info = ldq.ldq_logdet_grad(context.handle, Q, list(dQ), opts)
        ctx.save_for_backward(torch.as_tensor(np.asarray(grad, dtype=np.float64)).to(eta.device))
        ctx.eta_dtype = eta.dtype
        ctx.info = info
        return torch.tensor(val, dtype=torch.float64, device=eta.device)

    @staticmethod
    def backward(ctx, grad_output):
        (g,) = ctx.saved_tensors
        return (grad_output * g).to(ctx.eta_dtype), None, None, None


def logdet(eta, context, build, opts=None):
    """Differentiable log det Q(eta); see LogDetFn."""
    return LogDetFn.apply(eta, context, build, opts)
