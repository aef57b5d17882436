"""torch.autograd.Function over the adjoint backward (Sec. 3.3, Alg. 2;
Sec. 3.5 for density matrices).

``energy(circuit, theta, terms)`` returns the differentiable loss
Re<psi(theta)|H|psi(theta)> (pure) or Tr(H rho(theta)) (mixed); its backward
runs ``vqc_backward`` (uncomputing Phi for pure circuits, checkpoints for
mixed ones) and scales the gradient by the incoming grad_output.  Only the
final state is kept between forward and backward.
"""
from __future__ import annotations

import torch

from .api import Circuit, State


class VQCEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, circuit: Circuit, terms):
        theta_c = theta.detach().contiguous()
        st = State(circuit.n, mixed=circuit.mixed, device=theta.device)
        circuit.apply(st, theta_c)
        ctx.circuit, ctx.terms, ctx.state, ctx.theta = circuit, terms, st, theta_c
        e = st.expectation(terms)
        return torch.tensor(e.real, dtype=torch.float64, device=theta.device)

    @staticmethod
    def backward(ctx, grad_out):
        g, _ = ctx.circuit.backward(ctx.theta, ctx.state, ctx.terms, energy=False)
        ctx.state = None
        return grad_out * g, None, None


def energy(circuit: Circuit, theta: torch.Tensor, terms) -> torch.Tensor:
    return VQCEnergy.apply(theta, circuit, terms)
