"""torch.autograd binding of the pseudofermion action of the red/black
Moebius operator:

    S(U, phi) = phi_o^+ (D_pre^+ D_pre)^-1 phi_o,   D_pre = 1 - I^-1 D_oe I^-1 D_eo,

phi_o the odd-parity part of phi.  The forward pass runs the CG solve on the
normal operator and the hand-written link-derivative kernel in one library
call (mobius_force); backward only scales the stored gradients by the
incoming gradient.  Gradients follow PyTorch's convention for a real function
of complex inputs (dS/dRe z + i dS/dIm z): dS/dU for every link entry as an
independent complex number, and dS/dphi = 2 X on odd sites (0 on even ones).
"""
from __future__ import annotations

import torch

from . import mobius


class MobiusAction(torch.autograd.Function):
    """S = phi_o^+ (D_pre^+ D_pre)^-1 phi_o as a differentiable function of the
    links and of phi (both complex128 CUDA tensors in the canonical layouts).
    The link-derivative pass runs only when the links need a gradient."""

    @staticmethod
    def forward(ctx, links, phi, dims, Ls, M5, mf, b5, c5, tol, maxiter, inner_prec, op):
        want_links = ctx.needs_input_grad[0]
        own = op is None
        if own:
            op = mobius.Operator(dims, Ls, M5, mf, b5, c5, links.detach().contiguous())
        try:
            S, g_links, g_phi, info, rc = op.force(phi.detach().contiguous(), tol=tol,
                                                   maxiter=maxiter, inner_prec=inner_prec,
                                                   link_grad=want_links)
        finally:
            if own:
                op.close()
        if rc != mobius.OK:
            raise mobius.MobiusError(f"force solve did not converge: {info}")
        ctx.save_for_backward(g_links if want_links else None, g_phi)
        ctx.info = info
        return torch.tensor(S, dtype=torch.float64, device=links.device)

    @staticmethod
    def backward(ctx, grad_out):
        g_links, g_phi = ctx.saved_tensors
        gl = grad_out * g_links if ctx.needs_input_grad[0] else None
        gp = grad_out * g_phi if ctx.needs_input_grad[1] else None
        return gl, gp, None, None, None, None, None, None, None, None, None, None


def action(links, phi, dims, Ls, M5, mf, b5, c5, tol=1e-12, maxiter=20000, inner_prec=mobius.F64,
           op=None):
    """Differentiable S(U, phi) (a float64 scalar tensor on the links' device).
    op: an existing mobius.Operator built on these same links and parameters
    (saves packing the links again); None builds one for the call."""
    return MobiusAction.apply(links, phi, tuple(dims), int(Ls), float(M5), float(mf), float(b5),
                              float(c5), float(tol), int(maxiter), int(inner_prec), op)
