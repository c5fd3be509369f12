"""Impurity-tensor derivatives (Sec. III D) on the GPU against the oracle and exact tori.

d(log Z/V)/d(beta) and d(log Z/V)/dh after every step.  Exact tori: the
untruncated first steps must equal the enumerated Boltzmann averages to
1e-12.  Flows: log Z/V at 1e-10 relative after every step; the derivatives at
1e-7 relative (d/dh, which passes through zero at h = 0, relative to
1e-3 |d/dbeta| at least); measured 3.9e-12 (D = 6, h = 1e-3), 2.9e-9
(D = 8, h = 0), 5.6e-10 (D = 6, beta = 0.3) and 4.3e-9 (D = 16, h = 1e-4).
Both sides leave out of the isometry derivative the kept / discarded
eigenvalue pairs closer than 1e-12 of the largest: at D = 8, h = 0 the cut
falls between Gram eigenvalues of 1.2e-14 and 6.6e-15 of the largest, whose
eigenvectors the Gram does not determine, and with those pairs in, the two
eigen-routes (pivoted Cholesky with one-sided Jacobi here, two-sided Jacobi
in the oracle) gave derivatives 1e-6 to 4e-6 apart.
"""
import math
import sys

import numpy as np
import pytest

import paper_2507_21909_amd as trg
from oracle import trg as otrg, impurity
from oracle.ising import enumerate_derivatives_per_site

pytestmark = pytest.mark.gpu
TOL = 1e-7


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_exact_tori():
    _say("impurity exact tori")
    beta, h = 0.1497, 0.15
    s = trg.Solver(seed=3, tangents=trg.TAN_BETA | trg.TAN_H)
    s.tensor_init(trg.MODEL_ISING, beta, h, 16)
    ref = enumerate_derivatives_per_site(beta, h, (1, 1, 1, 1))
    assert np.allclose(s.impurity_derivatives(), ref, rtol=1e-13, atol=1e-14)
    for nst, ext in [(1, (2, 1, 1, 1)), (2, (2, 2, 1, 1))]:
        s.triad_atrg_step(nst - 1)
        ref = enumerate_derivatives_per_site(beta, h, ext)
        got = s.impurity_derivatives()
        _say("  step %d  gpu %r  exact %r" % (nst, got, ref))
        assert abs(got[0] - ref[0]) < 1e-12 * abs(ref[0])
        assert abs(got[1] - ref[1]) < 1e-12 * abs(ref[1])


def test_beta_zero_magnetisation():
    s = trg.Solver(seed=1, tangents=trg.TAN_H)
    s.tensor_init(trg.MODEL_ISING, 0.0, 0.3, 4)
    for i in range(6):
        s.triad_atrg_step(i % 4)
        db, dh = s.impurity_derivatives()
        assert math.isnan(db) and abs(dh - math.tanh(0.3)) < 1e-14


@pytest.mark.parametrize("D,nsteps,beta,h", [(6, 12, 0.1497, 1e-3), (8, 10, 0.1497, 0.0), (6, 10, 0.3, 0.0),
                                             (16, 6, 0.1497, 1e-4)])
def test_matches_oracle_every_step(D, nsteps, beta, h):
    _say("impurity vs oracle D=%d beta=%g h=%g" % (D, beta, h))
    prm = otrg.Params(D=D, seed=29)
    ist = impurity.ImpurityState(beta, h, 4)
    s = trg.Solver(seed=29, tangents=trg.TAN_BETA | trg.TAN_H)
    s.tensor_init(trg.MODEL_ISING, beta, h, D)
    worst = 0.0
    for i in range(nsteps):
        impurity.step(ist, i % 4, prm, "triad")
        s.triad_atrg_step(i % 4)
        ob, oh = impurity.derivatives(ist)
        gb, gh = s.impurity_derivatives()
        fo, fg = otrg.log_z_per_site(ist.pure), s.log_z_per_site()
        assert abs(fg - fo) <= 1e-10 * abs(fo)
        eb = abs(gb - ob) / abs(ob)
        eh = abs(gh - oh) / max(abs(oh), 1e-3 * abs(ob))
        worst = max(worst, eb, eh)
        _say("  step %2d  d/dbeta gpu %.15f oracle %.15f   d/dh gpu %.3e oracle %.3e" % (i, gb, ob, gh, oh))
    _say("  worst %.2e" % worst)
    assert worst <= TOL, worst


def test_errors():
    s = trg.Solver(seed=1)
    s.tensor_init(trg.MODEL_ISING, 0.1, 0.0, 4)
    with pytest.raises(trg.TrgError) as e:
        s.impurity_derivatives()
    assert e.value.code == -2
    t = trg.Solver(seed=1, tangents=trg.TAN_BETA)
    with pytest.raises(trg.TrgError) as e:
        t.tensor_init(trg.MODEL_ISING, 0.0, 0.0, 4)       # no beta tangent at beta = 0
    assert e.value.code == -1
    t.tensor_init(trg.MODEL_ISING, 0.1, 0.0, 4)
    with pytest.raises(trg.TrgError) as e:
        t.atrg_step(0)                                     # tangents ride on the triad step only
    assert e.value.code == -6
