"""log Z/V of the 4D Ising model by triad-ATRG as a torch.autograd.Function.

forward(beta, h) runs the RG flow on the GPU (the C ABI, on torch's current
stream) and returns log Z/V; backward returns grad * (d/dbeta, d/dh) log Z/V,
i.e. minus the internal energy per site and the magnetisation per site (the
field enters as exp(h s)).

The derivatives come from the same forward run: the solver carries the
impurity tangents of the site tensor (impurity_derivatives in the C ABI,
Sec. III D) through every step, so backward costs no further solve.  They
are exact where no truncation acts and differ from the derivative of the
truncated flow by terms of the order of the truncation.  The beta tangent
needs beta > 0 (the CP factor sqrt(sinh beta) is not differentiable at 0);
at beta = 0 the beta derivative is the closed form 4 tanh(h)^2 of
independent spins.
"""
import math

import torch

from .binding import Solver, FP64, TAN_BETA, TAN_H


def solve(beta, h, D, nsteps, seed=0, r=7, precision=FP64, tau_deg=0.0, stream=None, tangents=TAN_BETA | TAN_H):
    """(log Z/V, d/dbeta, d/dh) of an nsteps triad-ATRG flow (axes cycling 0..3)."""
    if beta == 0.0:
        tangents &= ~TAN_BETA
    s = Solver(seed=seed, r=r, precision=precision, tau_deg=tau_deg, stream=stream, tangents=tangents)
    try:
        s.tensor_init(0, float(beta), float(h), D)
        for k in range(nsteps):
            s.triad_atrg_step(k % 4)
        f = s.log_z_per_site()
        db, dh = s.impurity_derivatives() if tangents else (math.nan, math.nan)
    finally:
        s.close()
    if beta == 0.0:
        db = 4.0 * math.tanh(h) ** 2
    return f, db, dh


def _stream():
    if torch.cuda.is_available():
        return torch.cuda.current_stream().cuda_stream
    return None


class TriadFreeEnergy(torch.autograd.Function):
    """log Z/V (beta, h) with impurity-tensor derivatives; see the module docstring."""

    @staticmethod
    def forward(ctx, beta, h, D=8, nsteps=40, seed=0, r=7, precision=FP64, tau_deg=0.0):
        b, hv = float(beta), float(h)
        f, db, dh = solve(b, hv, D, nsteps, seed, r, precision, tau_deg, _stream())
        ctx.grads = (db, dh)
        dev = beta.device if torch.is_tensor(beta) else None
        return torch.tensor(f, dtype=torch.float64, device=dev)

    @staticmethod
    def backward(ctx, grad):
        db, dh = ctx.grads
        out_b = grad * torch.tensor(db, dtype=torch.float64, device=grad.device) if ctx.needs_input_grad[0] else None
        out_h = grad * torch.tensor(dh, dtype=torch.float64, device=grad.device) if ctx.needs_input_grad[1] else None
        return (out_b, out_h) + (None,) * 6
