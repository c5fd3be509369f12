"""TriadFreeEnergy: d log Z/V / d beta and d / dh against closed forms."""
import math

import pytest

pytestmark = pytest.mark.gpu


def _grads(beta, h, D, nsteps):
    import torch
    from paper_2507_21909_amd.autograd import TriadFreeEnergy
    b = torch.tensor(beta, dtype=torch.float64, requires_grad=True)
    hh = torch.tensor(h, dtype=torch.float64, requires_grad=True)
    f = TriadFreeEnergy.apply(b, hh, D, nsteps, 0x2507219090000000 + 5000)
    f.backward()
    return float(f), float(b.grad), float(hh.grad)


def test_beta_zero_field_derivative_is_tanh():
    # at beta = 0 the spins are independent: log Z/V = ln(2 cosh h) exactly
    f, gb, gh = _grads(0.0, 0.3, 4, 8)
    assert abs(f - math.log(2 * math.cosh(0.3))) < 1e-13
    assert abs(gh - math.tanh(0.3)) < 1e-8
    # d/dbeta at beta = 0: sum over the 4 bonds of <s s'> = 4 tanh^2 h (one-sided step, O(delta) error)
    assert abs(gb - 4 * math.tanh(0.3) ** 2) < 2e-3


def test_high_temperature_energy():
    # log Z/V = ln 2 + 4 ln cosh b + 6 t^4 + 76 t^6 + O(t^8), t = tanh b.  The
    # truncated flow at D = 8 carries the plaquette term only in part (the
    # oracle's own series pin has the same bound), so the closed form pins the
    # leading term to within the plaquette term's derivative, and the oracle's
    # central difference on the same seed pins the rest.
    from oracle import trg as otrg
    b, D, nsteps, seed = 0.01, 8, 40, 0x2507219090000000 + 5000
    t = math.tanh(b)
    f, gb, gh = _grads(b, 0.0, D, nsteps)
    assert abs(gb - 4 * t) < 24 * t ** 3
    assert abs(gh) < 1e-6          # Z2 symmetry at h = 0

    def oracle_f(x):
        prm = otrg.Params(D=D, seed=seed)
        return otrg.run(x, 0.0, prm, nsteps)[0]
    go = (oracle_f(b + 1e-4) - oracle_f(b - 1e-4)) / 2e-4
    assert abs(gb - go) < 1e-8
