"""torch.autograd.Function for the pseudofermion action S = phi^+ (Mhat^+ Mhat)^-1 phi.

Forward: one solve A X = phi in the HIP library (plain CG or MSPCG).
Backward: the adjoint force kernel gives dS/dU for every link from X and
Y = Mhat X (one more operator application); dS/dphi = 2 X.  PyTorch's complex
convention is used: for a real loss L, the gradient g of a complex input z
satisfies dL = Re sum conj(g) dz.
"""
from __future__ import annotations

import torch

from . import mspcg


class PseudofermionAction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U, phi, context: "mspcg.Context", params: "mspcg.SolveParams"):
        context.load_gauge(U.detach().contiguous())
        p = mspcg.SolveParams.from_buffer_copy(params)
        p.rhs_normal = 1
        X = torch.zeros_like(phi)
        context.solve(phi.detach().contiguous(), X, p)
        S = torch.vdot(phi.detach().reshape(-1), X.reshape(-1)).real
        ctx.save_for_backward(X)
        ctx.context = context
        return S

    @staticmethod
    def backward(ctx, gS):
        (X,) = ctx.saved_tensors
        c = ctx.context
        Y = torch.zeros_like(X)
        c.apply(mspcg.OP_MHAT, X, Y)
        G = torch.zeros(c.gshape, dtype=torch.complex128, device=X.device)
        c.force(X, Y, None, G)
        return gS * G, 2.0 * gS * X, None, None


def pseudofermion_action(U, phi, context, params=None):
    """S = phi^+ A^-1 phi with gradients to U (links) and phi (even field)."""
    if params is None:
        params = mspcg.make_params(tol=1e-12, maxiter=20000)
    return PseudofermionAction.apply(U, phi, context, params)
