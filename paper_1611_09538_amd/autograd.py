"""torch.autograd wrappers around the SE1P C ABI.

The SE1P potential is linear in the charges, phi = A(x) q, with A symmetric:
the real-space and self parts are pair/diagonal terms, and the k-space part
is G^T S G with G the Gaussian gridding of step 2 of Algorithm 1 and S the
real, even scaling of eq. scale_1p, so gathering is exactly the transpose of
gridding.  Hence, with U = 1/2 q^T A q (section 3.5 read with the usual 1/2):

  dU/dq_m = phi_m
  dU/dx_m = -q_m E_m            (E = -grad phi, the gather gradient of
                                 eq. force_se1p for the k-space part; the
                                 library returns q_m E_m itself, SE1P_FORCE)

and for a loss L(phi) with upstream gradient g = dL/dphi:

  dL/dq   = A g                  (one more evaluation with charges g)
  dL/dx_m = -g_m E[q]_m - q_m E[g]_m

Every number comes from the HIP library; this module only combines device
tensors.
"""
from __future__ import annotations

import torch

from . import se1p


class SE1PEnergy(torch.autograd.Function):
    """U = 1/2 sum q phi for a neutral system; backward gives forces and
    dU/dq through the saved potential and field (no extra pass)."""

    @staticmethod
    def forward(ctx, x, q, plan):
        # the library writes the force q_m E_m (SE1P_FORCE) next to phi
        phi, F, U = plan.eval(x, q, flags=se1p.ALL | se1p.FORCE)
        ctx.save_for_backward(phi, F)
        return U.reshape(())

    @staticmethod
    def backward(ctx, gU):
        phi, F = ctx.saved_tensors
        g = gU.to(phi.dtype)
        grad_x = grad_q = None
        if ctx.needs_input_grad[0]:
            grad_x = -g * F
        if ctx.needs_input_grad[1]:
            grad_q = g * phi
        return grad_x, grad_q, None


class SE1PPotential(torch.autograd.Function):
    """phi = A(x) q with the general adjoint for an upstream gradient."""

    @staticmethod
    def forward(ctx, x, q, plan, neutral_check=False):
        flags = se1p.ALL | (se1p.CHECK_INPUT if neutral_check else 0)
        phi, E, _ = plan.eval(x, q, flags=flags, want_energy=False)
        ctx.plan = plan
        ctx.save_for_backward(x, q, E)
        return phi

    @staticmethod
    def backward(ctx, gphi):
        x, q, E = ctx.saved_tensors
        plan = ctx.plan
        g = gphi.contiguous().to(q.dtype)
        phi_g, E_g, _ = plan.eval(x, g, flags=se1p.ALL | se1p.NO_NEUTRAL,
                                  want_energy=False)
        grad_x = grad_q = None
        if ctx.needs_input_grad[0]:
            grad_x = -g[:, None] * E - q[:, None] * E_g
        if ctx.needs_input_grad[1]:
            grad_q = phi_g
        return grad_x, grad_q, None, None


def energy(x, q, plan):
    return SE1PEnergy.apply(x, q, plan)


def potential(x, q, plan, neutral_check=False):
    return SE1PPotential.apply(x, q, plan, neutral_check)
