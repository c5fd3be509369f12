"""log Z/V of the 4D Ising model by triad-ATRG as a torch.autograd.Function.

forward(beta, h) runs the RG flow on the GPU (the C ABI, on torch's current
stream) and returns log Z/V; backward returns (d/dbeta, d/dh) log Z/V, i.e.
minus the internal energy per site and the magnetisation per site with the
field entering as exp(h s).

The derivatives are central differences of the same deterministic flow (same
seed, so the same sketches): 2 extra solves per variable.  The steps of h
stay inside h's sign (delta_h <= |h| / 2 when h != 0), because for beta above
the critical coupling log Z/V has a kink at h = 0.
"""
import torch

from .binding import Solver, FP64


def _log_z(beta, h, D, nsteps, seed, r, precision, tau_deg, stream):
    s = Solver(seed=seed, r=r, precision=precision, tau_deg=tau_deg, stream=stream)
    try:
        s.tensor_init(0, float(beta), float(h), D)
        for k in range(nsteps):
            s.triad_atrg_step(k % 4)
        return s.log_z_per_site()
    finally:
        s.close()


def _stream():
    if torch.cuda.is_available():
        return torch.cuda.current_stream().cuda_stream
    return None


class TriadFreeEnergy(torch.autograd.Function):
    """log Z/V (beta, h) with derivatives; see the module docstring."""

    @staticmethod
    def forward(ctx, beta, h, D=8, nsteps=40, seed=0, r=7, precision=FP64, tau_deg=0.0, delta_beta=1e-4,
                delta_h=1e-4):
        b, hv = float(beta), float(h)
        st = _stream()
        f = _log_z(b, hv, D, nsteps, seed, r, precision, tau_deg, st)
        ctx.args = (b, hv, D, nsteps, seed, r, precision, tau_deg, delta_beta, delta_h)
        return torch.tensor(f, dtype=torch.float64, device=beta.device if torch.is_tensor(beta) else None)

    @staticmethod
    def backward(ctx, grad):
        b, hv, D, nsteps, seed, r, precision, tau_deg, db, dh = ctx.args
        st = _stream()

        def f(x, y):
            return _log_z(x, y, D, nsteps, seed, r, precision, tau_deg, st)

        gb = gh = None
        if ctx.needs_input_grad[0]:
            d = min(db, b) if b > 0 else db          # beta stays >= 0
            if b - d < 0:
                gb = (f(b + d, hv) - f(b, hv)) / d
            else:
                gb = (f(b + d, hv) - f(b - d, hv)) / (2 * d)
        if ctx.needs_input_grad[1]:
            d = min(dh, abs(hv) / 2) if hv != 0 else dh
            gh = (f(b, hv + d) - f(b, hv - d)) / (2 * d)
        out_b = None if gb is None else grad * torch.tensor(gb, dtype=torch.float64, device=grad.device)
        out_h = None if gh is None else grad * torch.tensor(gh, dtype=torch.float64, device=grad.device)
        return (out_b, out_h) + (None,) * 8
