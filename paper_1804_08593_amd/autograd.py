"""torch.autograd.Function for the pseudofermion action S = phi^+ (Mhat^+ Mhat)^-1 phi.

Forward: mspcg_pseudofermion_action solves A X = phi in the HIP library and
returns S and dS/dphi = 2 X.  Backward: the adjoint force kernel gives dS/dU
for every link from X and Y = Mhat X (one more operator application); the
links used are those of the forward pass (the context's gauge generation is
checked and the saved links reloaded when something else loaded a gauge
field in between).  Only the chain rule's scaling by the incoming gradient
happens here.  PyTorch's complex convention is used: for a real loss L, the
gradient g of a complex input z satisfies dL = Re sum conj(g) dz.
"""
from __future__ import annotations

import torch

from . import mspcg


class PseudofermionAction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U, phi, context: "mspcg.Context", params: "mspcg.SolveParams"):
        Uc = U.detach().contiguous()
        context.load_gauge(Uc)
        X = torch.zeros_like(phi)
        dphi = torch.zeros_like(phi)
        S, _ = context.pseudofermion_action(phi.detach().contiguous(), X, dphi, params)
        ctx.save_for_backward(Uc, X, dphi)
        ctx.context = context
        ctx.gauge_generation = context.gauge_generation
        return torch.tensor(S, dtype=torch.float64, device=phi.device)

    @staticmethod
    def backward(ctx, gS):
        Uc, X, dphi = ctx.saved_tensors
        c = ctx.context
        if c.gauge_generation != ctx.gauge_generation:
            c.load_gauge(Uc)
        Y = torch.zeros_like(X)
        c.apply(mspcg.OP_MHAT, X, Y)
        G = torch.zeros(c.gshape, dtype=torch.complex128, device=X.device)
        c.force(X, Y, None, G)
        return gS * G, gS * dphi, None, None


def pseudofermion_action(U, phi, context, params=None):
    """S = phi^+ A^-1 phi with gradients to U (links) and phi (even field)."""
    if params is None:
        params = mspcg.make_params(tol=1e-12, maxiter=20000)
    return PseudofermionAction.apply(U, phi, context, params)
