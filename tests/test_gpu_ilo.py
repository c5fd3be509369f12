"""ILO triad-ATRG (Sec. II C, App. A with r_bond > 1) on the GPU against the oracle.

The bond swap keeps r_bond D values with a sketch (r_bond + 1) D wide; the
next step's re-split carries the overspanned bond.  Bonds and sketches wider
than 64 go through the blocked Householder QR over TSQR panels.  Tolerance:
log Z/V within 1e-10 relative after every step (the FP64 parity target), the
kept bond count equal and the kept bond spectrum within 1e-10 of its largest
value.
"""
import math
import os
import sys

import numpy as np
import pytest

import paper_2507_21909_amd as trg
from oracle import trg as otrg
from oracle.ising import enumerate_log_z_per_site

pytestmark = pytest.mark.gpu
TOL = 1e-10


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _pair(beta, h, D, rb, sm, nsteps, method, seed=13):
    prm = otrg.Params(D=D, seed=seed, r_bond=rb, sketch_mult=sm)
    st = otrg.init_ising(beta, h, 4)
    s = trg.Solver(seed=seed, r_bond=rb, sketch_mult=sm)
    s.tensor_init(trg.MODEL_ISING, beta, h, D)
    worst = 0.0
    for i in range(nsteps):
        otrg.rg_step(st, i % 4, prm, method)
        (s.triad_atrg_step if method == "triad" else s.atrg_step)(i % 4)
        fo, fg = otrg.log_z_per_site(st), s.log_z_per_site()
        rel = abs(fg - fo) / abs(fo)
        worst = max(worst, rel)
        b = st.log[-1]["bond"]
        sig = s.export(trg.T_SIGMA)
        kept = int(np.count_nonzero(sig))
        assert kept == b["kept"], (i, kept, b["kept"])
        assert np.max(np.abs(sig[:kept] - b["sig"][:kept])) <= TOL * sig[0]
        _say("  step %2d  chi %3d  gpu %.16f  oracle %.16f  rel %.2e" % (i, s.shape()[1], fg, fo, rel))
    assert worst <= TOL, worst
    return s, st


@pytest.mark.parametrize("method", ["triad", "atrg"])
def test_exact_steps(method):
    _say("ilo exact steps", method)
    beta, h = 0.1497, 0.15
    s = trg.Solver(seed=7, r_bond=2, sketch_mult=3)
    s.tensor_init(trg.MODEL_ISING, beta, h, 16)
    for nst, ext in [(1, (2, 1, 1, 1)), (2, (2, 2, 1, 1))]:
        (s.triad_atrg_step if method == "triad" else s.atrg_step)(nst - 1)
        assert abs(s.log_z_per_site() - enumerate_log_z_per_site(beta, h, ext)) < 1e-13


def test_beta_zero():
    s = trg.Solver(seed=1, r_bond=3, sketch_mult=4)
    s.tensor_init(trg.MODEL_ISING, 0.0, 0.2, 4)
    for i in range(6):
        s.triad_atrg_step(i % 4)
    assert abs(s.log_z_per_site() - math.log(2 * math.cosh(0.2))) < 1e-14


@pytest.mark.parametrize("D,rb,h", [(8, 5, 1e-4), (6, 2, 0.0)])
def test_triad_matches_oracle(D, rb, h):
    _say("ilo triad D=%d r_bond=%d" % (D, rb))
    s, st = _pair(0.1497, h, D, rb, rb + 1, 8, "triad")
    assert s.shape()[1] == rb * D


def test_atrg_matches_oracle():
    _say("ilo atrg D=6 r_bond=3")
    _pair(0.1497, 1e-4, 6, 3, 4, 8, "atrg")


def test_options_are_checked():
    with pytest.raises(trg.TrgError) as e:
        trg.Solver(r_bond=3, sketch_mult=2)
    assert e.value.code == -1
    s = trg.Solver(r_bond=20, sketch_mult=21)
    with pytest.raises(trg.TrgError) as e:
        s.tensor_init(trg.MODEL_ISING, 0.1, 0.0, 16)   # r_bond D = 320 > 256
    assert e.value.code == -6


@pytest.mark.parametrize("name", ["ilo_d16_rb2_16steps", "ilo_d12_rb6_8steps", "ilo_d16_rb5_6steps"])
def test_against_stored_oracle_flows(name):
    from test_gpu_grid import _golden, run_against
    _say("ilo reference flow", name)
    run_against(_golden(name))


def test_d32_overspanned_bond():
    """D = 32, r_bond = 2: a 64-wide bond and a 96-wide sketch (blocked QR).  The
    first three steps are cheap for the oracle and are compared directly; the
    flow then continues to the saturated shapes and must stay finite, keep a
    64-wide bond and stay within the truncation error of the plain flow."""
    _say("ilo D=32 r_bond=2")
    s, st = _pair(0.1497, 0.0, 32, 2, 3, 3, "triad", seed=17)
    for i in range(3, 8):
        s.triad_atrg_step(i % 4)
    f_ilo = s.log_z_per_site()
    assert s.shape()[1] == 64 and max(s.shape()[0]) == 32
    p = trg.Solver(seed=17)
    p.tensor_init(trg.MODEL_ISING, 0.1497, 0.0, 32)
    for i in range(8):
        p.triad_atrg_step(i % 4)
    f_plain = p.log_z_per_site()
    _say("  8 steps: ILO %.12f  plain %.12f" % (f_ilo, f_plain))
    assert abs(f_ilo - f_plain) <= 1e-3 * abs(f_plain)
