"""TriadFreeEnergy: derivatives of log Z/V from the impurity tangents, against closed forms and the oracle."""
import math

import pytest

pytestmark = pytest.mark.gpu


def _grads(beta, h, D, nsteps, seed=0x2507219090000000 + 5000):
    import torch
    from paper_2507_21909_amd.autograd import TriadFreeEnergy
    b = torch.tensor(beta, dtype=torch.float64, requires_grad=True)
    hh = torch.tensor(h, dtype=torch.float64, requires_grad=True)
    f = TriadFreeEnergy.apply(b, hh, D, nsteps, seed)
    f.backward()
    return float(f.detach()), float(b.grad), float(hh.grad)


def test_beta_zero_field_derivative_is_tanh():
    # at beta = 0 the spins are independent: log Z/V = ln(2 cosh h), d/dh = tanh h exactly
    f, gb, gh = _grads(0.0, 0.3, 4, 8)
    assert abs(f - math.log(2 * math.cosh(0.3))) < 1e-13
    assert abs(gh - math.tanh(0.3)) < 1e-14
    assert abs(gb - 4 * math.tanh(0.3) ** 2) < 1e-15


def test_matches_the_oracle_impurity_method():
    from oracle import trg as otrg, impurity
    b, h, D, nsteps, seed = 0.1497, 1e-3, 6, 12, 0x2507219090000000 + 5000
    f, gb, gh = _grads(b, h, D, nsteps, seed)
    (ob, oh), ist = impurity.run(b, h, otrg.Params(D=D, seed=seed), nsteps, "triad")
    assert abs(f - otrg.log_z_per_site(ist.pure)) < 1e-10 * abs(f)
    assert abs(gb - ob) < 1e-8 * abs(ob)
    assert abs(gh - oh) < 1e-8 * abs(oh)
