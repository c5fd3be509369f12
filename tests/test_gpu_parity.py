"""End-to-end parity of the HIP path with the FP64 oracle (through the C ABI).

Tolerance: relative error of log Z/V at most 1e-10 on the FP64 path (the
FP64 parity target), step by step on the same seeded sketch.
"""
import math
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


def _run_pair(beta, h, D, nsteps, method, seed=11, bond="sketch", r=7):
    prm = otrg.Params(D=D, r=r, seed=seed, bond_svd=bond)
    st = otrg.init_ising(beta, h, 4)
    s = trg.Solver(seed=seed, r=r, bond_svd=trg.SVD_EXACT if bond == "exact" else trg.SVD_SKETCH)
    s.tensor_init(trg.MODEL_ISING, beta, h, D)
    out = []
    for i in range(nsteps):
        ax = i % 4
        otrg.rg_step(st, ax, prm, method)
        (s.triad_atrg_step if method == "triad" else s.atrg_step)(ax)
        f_o = otrg.log_z_per_site(st)
        f_g = s.log_z_per_site()
        out.append((f_g, f_o))
        _say("  step %2d  gpu %.16f  oracle %.16f  rel %.2e" % (i, f_g, f_o, abs(f_g - f_o) / abs(f_o)))
    return out, s, st


@pytest.mark.parametrize("h", [0.0, 0.2])
def test_beta_zero_exact(h):
    s = trg.Solver(seed=1)
    s.tensor_init(trg.MODEL_ISING, 0.0, h, 4)
    for i in range(6):
        s.triad_atrg_step(i % 4)
    assert abs(s.log_z_per_site() - math.log(2 * math.cosh(h))) < 1e-13


@pytest.mark.parametrize("method", ["triad", "atrg"])
def test_first_two_steps_exact(method):
    _say("exact steps", method)
    s = trg.Solver(seed=3)
    s.tensor_init(trg.MODEL_ISING, 0.1497, 0.15, 16)
    for nst, ext in [(1, (2, 1, 1, 1)), (2, (2, 2, 1, 1))]:
        (s.triad_atrg_step if method == "triad" else s.atrg_step)(nst - 1)
        assert abs(s.log_z_per_site() - enumerate_log_z_per_site(0.1497, 0.15, ext)) < 1e-13


def test_atrg_d6_exact_svd_config():
    """Plain ATRG, beta 0.1497, h 0, D 6, exact bond-swap SVD, L = 8 (12 steps)."""
    _say("atrg D=6 exact 12 steps")
    out, s, st = _run_pair(0.1497, 0.0, 6, 12, "atrg", bond="exact")
    for f_g, f_o in out:
        assert abs(f_g - f_o) <= TOL * abs(f_o)


@pytest.mark.parametrize("D,nsteps,h", [(6, 8, 0.0), (8, 12, 1e-4)])
def test_triad_sketch(D, nsteps, h):
    _say("triad D=%d %d steps" % (D, nsteps))
    out, s, st = _run_pair(0.1497, h, D, nsteps, "triad")
    for f_g, f_o in out:
        assert abs(f_g - f_o) <= TOL * abs(f_o)
    # state tensors agree element by element (sign convention fixes the gauge)
    phi = s.export(0)
    assert phi.shape == st.phi.shape
    assert np.max(np.abs(phi - st.phi)) < 1e-8 * np.max(np.abs(st.phi))


def test_error_codes():
    s = trg.Solver()
    with pytest.raises(trg.TrgError) as e:
        s.triad_atrg_step(0)
    assert e.value.code == -2
    s.tensor_init(trg.MODEL_ISING, 0.1, 0.0, 4)
    with pytest.raises(trg.TrgError) as e:
        s.atrg_step(4)
    assert e.value.code == -1
    with pytest.raises(trg.TrgError) as e:
        s.tensor_init(trg.MODEL_ISING, -0.1, 0.0, 4)
    assert e.value.code == -1


def _golden(name):
    import json
    import os
    p = os.path.join(os.path.dirname(__file__), "golden", name + ".json")
    if not os.path.exists(p):
        pytest.skip("golden values %s not generated (tests/golden/make_golden.py)" % name)
    return json.load(open(p))


@pytest.mark.parametrize("name", ["triad_d16_l1024", "triad_d16_h1e-4_16steps", "triad_d32_12steps"])
def test_triad_against_stored_oracle_values(name):
    """Full-size parity: the FP64 GPU path vs oracle values stored by make_golden.py."""
    g = _golden(name)
    c = g["params"]
    n = len(g["log_z"])
    if n < c["nsteps"]:
        pytest.skip("golden file %s incomplete (%d of %d steps)" % (name, n, c["nsteps"]))
    _say("golden", name)
    s = trg.Solver(seed=c["seed"])
    s.tensor_init(trg.MODEL_ISING, c["beta"], c["h"], c["D"])
    worst = 0.0
    for i in range(n):
        s.triad_atrg_step(i % 4)
        f = s.log_z_per_site()
        rel = abs(f - g["log_z"][i]) / abs(g["log_z"][i])
        worst = max(worst, rel)
        _say("  step %2d  gpu %.16f  oracle %.16f  rel %.2e" % (i, f, g["log_z"][i], rel))
    assert worst <= TOL
