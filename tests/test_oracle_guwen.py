"""Pins of the oracle's Gu-Wen ratio X = (Tr A)^2 / Tr(A A) (Sec. III D).

* Untruncated tensors: Tr A is the partition function of the torus the
  tensor stands for and Tr(A A) that of the torus with the open axis doubled
  (two copies glued along it), so X = Z(L)^2 / Z(L with L_axis doubled),
  checked against brute-force enumeration on tiny tori.  This fixes both
  traces, the leg pairing (forward with backward) and the axis bookkeeping.
* beta = 0: the tensor has rank one, X = 1 exactly.
* the two phases: X tends to 2 deep in the ordered phase (two ground states)
  and to 1 in the disordered phase, the behaviour the paper uses to locate T_c.
"""
import math

import numpy as np
import pytest

from oracle import trg
from oracle.ising import enumerate_log_z_per_site


def _z(beta, h, ext):
    return math.exp(int(np.prod(ext)) * enumerate_log_z_per_site(beta, h, ext))


def _x_enum(beta, h, ext, axis):
    dbl = list(ext)
    dbl[axis] *= 2
    return _z(beta, h, ext) ** 2 / _z(beta, h, dbl)


@pytest.mark.parametrize("axis", [0, 1, 2, 3])
@pytest.mark.parametrize("h", [0.0, 0.2])
def test_initial_tensor_is_exact(axis, h):
    beta = 0.31
    st = trg.init_ising(beta, h, 4)
    assert abs(trg.gu_wen_x(st, axis) - _x_enum(beta, h, (1, 1, 1, 1), axis)) < 1e-13


@pytest.mark.parametrize("method", ["triad", "atrg"])
@pytest.mark.parametrize("axis", [0, 2, 3])
def test_exact_steps(method, axis):
    beta, h = 0.1497, 0.1
    st = trg.init_ising(beta, h, 4)
    prm = trg.Params(D=16, seed=3)
    for nst, ext in [(1, (2, 1, 1, 1)), (2, (2, 2, 1, 1))]:
        trg.rg_step(st, nst - 1, prm, method)
        ref = _x_enum(beta, h, ext, axis)
        assert abs(trg.gu_wen_x(st, axis) - ref) < 1e-12 * ref


def test_two_dimensional_exact_steps():
    # 2D ATRG, D = 64: three steps are exact (4 x 2 torus), X along both axes
    beta, h = 0.44, 0.05
    st = trg.init_ising(beta, h, 2)
    prm = trg.Params(D=64, seed=1)
    exts = [(2, 1), (2, 2), (4, 2)]
    for i, ext in enumerate(exts):
        trg.rg_step(st, i % 2, prm, "atrg")
        for axis in (0, 1):
            ref = _x_enum(beta, h, ext, axis)
            assert abs(trg.gu_wen_x(st, axis) - ref) < 1e-12 * ref


def test_beta_zero_is_one():
    st = trg.init_ising(0.0, 0.3, 4)
    prm = trg.Params(D=4, seed=2)
    for i in range(6):
        trg.rg_step(st, i % 4, prm, "triad")
        assert abs(trg.gu_wen_x(st) - 1.0) < 1e-14


def test_ordered_phase_plateau():
    # deep in the ordered phase (beta_c ~ 0.1496 in 4D, 0.4407 in 2D) the ratio
    # counts the two ground states once the torus has grown past a few sites.
    # The randomized sketch does not respect the spin-flip symmetry exactly,
    # so the degeneracy of the two sectors decays again after many steps at
    # finite D; X is read on its plateau (4 to 8 sites per axis)
    st = trg.init_ising(0.6, 0.0, 4)
    prm = trg.Params(D=6, seed=4)
    xs = []
    for i in range(12):
        trg.rg_step(st, i % 4, prm, "triad")
        xs.append(trg.gu_wen_x(st))
    assert max(abs(x - 2.0) for x in xs[7:12]) < 1e-5, xs
    st = trg.init_ising(0.6, 0.0, 2)
    prm = trg.Params(D=8, seed=4)
    xs = []
    for i in range(24):
        trg.rg_step(st, i % 2, prm, "atrg")
        xs.append(trg.gu_wen_x(st))
    assert max(abs(x - 2.0) for x in xs[7:24]) < 1e-5, xs


@pytest.mark.parametrize("d,beta,D,method", [(4, 0.10, 6, "triad"), (2, 0.30, 8, "atrg")])
def test_disordered_phase(d, beta, D, method):
    st = trg.init_ising(beta, 0.0, d)
    prm = trg.Params(D=D, seed=4)
    for i in range(24):
        trg.rg_step(st, i % d, prm, method)
    assert abs(trg.gu_wen_x(st) - 1.0) < 1e-6
