"""Pins of the oracle's ILO triad-ATRG (Sec. II C; App. A with r_bond > 1).

With r_bond > 1 the bond swap keeps r_bond D singular values, the sketch is
eta D = (r_bond + 1) D wide (App. A footnote), and the next step's alpha and
beta carry the overspanned bond through the re-split.  Pins:

* r_bond = 1 is the plain bond swap (identical flow);
* untruncated first steps still equal the enumerated tori, and beta = 0
  still gives ln(2 cosh h), with the overspanned bond;
* with R = D^2 the triad representation truncates nothing, so ILO triad-ATRG
  equals ILO ATRG with the same r_bond (the triad identity of Sec. II B);
* the state's bond settles at r_bond D;
* the paper's accuracy claim, checked where the answer is known: in 2D the
  free energy with r_bond = 2 is markedly closer to Onsager's than with
  r_bond = 1 at the same D.
"""
import math

import pytest

from oracle import trg
from oracle.ising import enumerate_log_z_per_site, onsager_log_z


def test_rbond_one_is_the_plain_bond_swap():
    a, _ = trg.run(0.1497, 1e-3, trg.Params(D=6, seed=9), 8, "triad")
    b, _ = trg.run(0.1497, 1e-3, trg.Params(D=6, seed=9, r_bond=1, sketch_mult=2), 8, "triad")
    assert a == b


@pytest.mark.parametrize("method", ["triad", "atrg"])
def test_exact_steps_with_overspanned_bond(method):
    beta, h = 0.1497, 0.15
    st = trg.init_ising(beta, h, 4)
    prm = trg.Params(D=16, seed=7, r_bond=2, sketch_mult=3)
    for nst, ext in [(1, (2, 1, 1, 1)), (2, (2, 2, 1, 1))]:
        trg.rg_step(st, nst - 1, prm, method)
        assert abs(trg.log_z_per_site(st) - enumerate_log_z_per_site(beta, h, ext)) < 1e-13


def test_beta_zero():
    f, _ = trg.run(0.0, 0.2, trg.Params(D=4, seed=1, r_bond=2, sketch_mult=3), 8, "triad")
    assert abs(f - math.log(2 * math.cosh(0.2))) < 1e-14


def test_triad_with_full_overspan_is_atrg():
    prm_t = trg.Params(D=4, r=4, seed=3, r_bond=2, sketch_mult=3)
    prm_a = trg.Params(D=4, seed=3, r_bond=2, sketch_mult=3)
    lt, _ = trg.run(0.1497, 0.01, prm_t, 8, "triad")
    la, _ = trg.run(0.1497, 0.01, prm_a, 8, "atrg")
    assert abs(lt - la) < 1e-13


def test_bond_settles_at_rbond_d():
    st = trg.init_ising(0.1497, 0.0, 4)
    prm = trg.Params(D=4, seed=5, r_bond=2, sketch_mult=3)
    for i in range(6):
        trg.rg_step(st, i % 4, prm, "triad")
    assert st.phi.shape[-1] == 8 and st.log[-1]["bond"]["kept"] == 8
    assert max(st.phi.shape[:-1]) == 4


@pytest.mark.parametrize("beta", [0.40, 0.44])
def test_two_dimensional_accuracy_gain(beta):
    ref = onsager_log_z(beta)
    err = {}
    for rb in (1, 2):
        f, _ = trg.run(beta, 0.0, trg.Params(D=8, seed=4, r_bond=rb, sketch_mult=rb + 1), 40, "atrg", d=2)
        err[rb] = abs(f - ref) / abs(ref)
    assert err[2] < 0.5 * err[1], err
