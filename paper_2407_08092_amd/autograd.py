"""torch.autograd.Function for y_e = D_S(U) phi_e (eq. 3), FP64.

forward runs the HIP Schur apply; backward returns dL/dphi_e = D_S^H g (adjoint
apply) and dL/dU (the link force kernel, both the hopping and the clover terms),
in torch's convention for complex gradients.  The lattice handle must already hold
the links U (ddq_set_gauge) and the clover term (ddq_set_clover); U is passed so
that autograd can route its gradient.
"""
from __future__ import annotations

import torch

from . import api


class DiracSchur(torch.autograd.Function):
    @staticmethod
    def forward(ctx, phi_e: torch.Tensor, U: torch.Tensor, lat: api.Lattice):
        if phi_e.dtype != torch.complex128:
            raise TypeError("DiracSchur differentiates the FP64 path: phi_e must be complex128")
        ctx.lat = lat
        ctx.save_for_backward(phi_e)
        return api.apply_schur(lat, phi_e.contiguous())

    @staticmethod
    def backward(ctx, g: torch.Tensor):
        (phi_e,) = ctx.saved_tensors
        lat = ctx.lat
        g = g.contiguous()
        grad_phi = grad_U = None
        if ctx.needs_input_grad[0]:
            grad_phi = api.backward_apply(lat, g)
        if ctx.needs_input_grad[1]:
            grad_U, _ = api.backward_link_force(lat, g, phi_e.contiguous(), want_G=True)
        return grad_phi, grad_U, None


def dirac_schur(phi_e: torch.Tensor, U: torch.Tensor, lat: api.Lattice) -> torch.Tensor:
    """Differentiable y_e = D_S(U) phi_e; `lat` must hold U and its clover term."""
    return DiracSchur.apply(phi_e, U, lat)
