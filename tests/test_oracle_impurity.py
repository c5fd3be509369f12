"""Pins of the oracle's impurity-tensor derivatives (Sec. III D).

* Untruncated tori: the first two steps at D = 16 (and the initial tensor)
  truncate nothing, so d(log Z/V)/d(beta) and d(log Z/V)/dh must equal the
  Boltzmann averages <sum s s>/V and <sum s>/V of the enumerated torus.
* beta = 0: m = tanh h exactly, at any step.
* 2D thermodynamic limit: the internal energy of ATRG at D = 8 equals
  Onsager's closed form within the truncation error of the flow (measured
  3.6e-5 at beta = 0.3 and 7e-5 at 0.6), the closed form itself checked
  against the derivative of the pinned Onsager free energy; in the ordered
  phase the field derivative is Yang's spontaneous magnetisation.
* 4D, high temperature: the impurity energy agrees with a central difference
  of the same truncated flow and with the high-temperature series to the
  truncation level, and the field derivative vanishes at h = 0.
* 4D near T_c (D = 8, exact bond-swap SVD): with the triad isometries
  differentiated, the tangent is the flow's own derivative up to the held
  squeezers and the bond swap's tangent-space form (measured 4e-4 relative
  against a central difference); holding the isometries instead reproduces
  the central difference of the flow with its isometries and squeezers
  frozen (9e-4), 12 % away from the flow's derivative.
* The isometry derivative alone: on a Gram with separated eigenvalues the
  projector's first-order change (dU U^T + U dU^T) equals a central
  difference of the exact eigen-decomposition; a kept / discarded pair
  closer than 1e-12 of the largest eigenvalue gets no rotation, the other
  pairs the textbook coefficient w_j^T dG u_i / (lam_i - lam_j).
"""
import math

import numpy as np
import pytest

from oracle import trg, impurity
from oracle.ising import enumerate_derivatives_per_site, hte_4d, onsager_energy, onsager_log_z_1d


@pytest.mark.parametrize("method", ["triad", "atrg"])
@pytest.mark.parametrize("h", [0.0, 0.15])
def test_exact_tori(method, h):
    beta = 0.1497
    ist = impurity.ImpurityState(beta, h, 4)
    ref = enumerate_derivatives_per_site(beta, h, (1, 1, 1, 1))
    assert np.allclose(impurity.derivatives(ist), ref, rtol=1e-13, atol=1e-14)
    prm = trg.Params(D=16, seed=3)
    for nst, ext in [(1, (2, 1, 1, 1)), (2, (2, 2, 1, 1))]:
        impurity.step(ist, nst - 1, prm, method)
        ref = enumerate_derivatives_per_site(beta, h, ext)
        got = impurity.derivatives(ist)
        assert abs(got[0] - ref[0]) < 1e-12 * abs(ref[0]), (got, ref)
        assert abs(got[1] - ref[1]) < 1e-12 + 1e-12 * abs(ref[1]), (got, ref)


def test_beta_zero_magnetisation():
    h = 0.3
    ist = impurity.ImpurityState(0.0, h, 4, wrt=("h",))
    prm = trg.Params(D=4, seed=2)
    for i in range(8):
        impurity.step(ist, i % 4, prm, "triad")
        assert abs(impurity.derivatives(ist)[0] - math.tanh(h)) < 1e-14


def test_onsager_energy_closed_form():
    for beta in (0.2, 0.3, 0.6):
        e = 1e-5
        fd = (onsager_log_z_1d(beta + e) - onsager_log_z_1d(beta - e)) / (2 * e)
        assert abs(onsager_energy(beta) + fd) < 1e-8


@pytest.mark.parametrize("beta,tol", [(0.3, 1e-4), (0.6, 2e-4)])
def test_two_dimensional_energy_and_magnetisation(beta, tol):
    prm = trg.Params(D=8, seed=4)
    (db, dh), _ = impurity.run(beta, 0.0, prm, 40, "atrg", d=2)
    assert abs(-db - onsager_energy(beta)) < tol
    if beta < 0.4407:
        assert abs(dh) < 1e-6          # disordered: no magnetisation
    else:
        # ordered: the truncated flow settles in one of the two ground states,
        # and |m| is Yang's spontaneous magnetisation (1 - sinh(2b)^-4)^(1/8)
        assert abs(abs(dh) - (1 - math.sinh(2 * beta) ** -4) ** 0.125) < 1e-4


def test_four_dimensional_high_temperature():
    # beta = 0.02: the flow's own derivative (central difference) and the
    # impurity energy agree to the truncation level, and both sit within the
    # D = 6 truncation error of the high-temperature series (through t^8,
    # remainder ~1e-10 here)
    beta = 0.02
    prm = trg.Params(D=6, seed=8)
    (db, dh), _ = impurity.run(beta, 0.0, prm, 24, "triad")
    d = 1e-5
    fp, _ = trg.run(beta + d, 0.0, prm, 24, "triad")
    fm, _ = trg.run(beta - d, 0.0, prm, 24, "triad")
    fb = (fp - fm) / (2 * d)
    hb = (hte_4d(beta + d) - hte_4d(beta - d)) / (2 * d)
    assert abs(db - fb) < 1e-4 * abs(fb), (db, fb)
    assert abs(db - hb) < 2e-3 * abs(hb), (db, hb)
    # the Gaussian sketch respects the spin-flip symmetry only to rounding
    assert abs(dh) < 1e-8


class _Freezer:
    """Records a flow's triad isometries and squeezers, then replays them (frozen) in later flows."""

    def __init__(self, monkeypatch):
        self.iso, self.sq, self.mode, self.i, self.j = [], [], "record", 0, 0
        self.fi = self.fs = False
        orig_iso, orig_sq = trg.triad_isometry, trg.squeezer

        def iso(gram, d1, d2, cap, prm, name, logrec):
            if self.mode == "replay" and self.fi:
                self.i += 1
                return self.iso[self.i - 1]
            u = orig_iso(gram, d1, d2, cap, prm, name, logrec)
            if self.mode == "record":
                self.iso.append(u)
            return u

        def sq(kf, kb, dt, db, prm, name, logrec):
            if self.mode == "replay" and self.fs:
                self.j += 1
                return self.sq[self.j - 1]
            r = orig_sq(kf, kb, dt, db, prm, name, logrec)
            if self.mode == "record":
                self.sq.append(r)
            return r
        monkeypatch.setattr(trg, "triad_isometry", iso)
        monkeypatch.setattr(trg, "squeezer", sq)

    def flow(self, beta, prm, nsteps, mode, fi=False, fs=False):
        self.mode, self.fi, self.fs, self.i, self.j = mode, fi, fs, 0, 0
        f, _ = trg.run(beta, 0.0, prm, nsteps, "triad")
        self.mode = None
        return f


def test_four_dimensional_near_tc_isometry_derivative(monkeypatch):
    beta, nsteps, d = 0.149, 8, 1e-5
    prm = trg.Params(D=8, seed=12345, bond_svd="exact")
    fz = _Freezer(monkeypatch)
    fz.flow(beta, prm, nsteps, "record")
    u_free = -(fz.flow(beta + d, prm, nsteps, "replay") - fz.flow(beta - d, prm, nsteps, "replay")) / (2 * d)
    u_frozen = -(fz.flow(beta + d, prm, nsteps, "replay", True, True) -
                 fz.flow(beta - d, prm, nsteps, "replay", True, True)) / (2 * d)
    (db,), _ = impurity.run(beta, 0.0, prm, nsteps, "triad", wrt=("beta",))
    (db_held,), _ = impurity.run(beta, 0.0, prm, nsteps, "triad", wrt=("beta",), iso=False)
    assert abs(-db - u_free) < 2e-3 * abs(u_free), (-db, u_free)
    assert abs(-db_held - u_frozen) < 2e-3 * abs(u_frozen), (-db_held, u_frozen)
    # the isometries' share of the derivative is not small here: the pin above
    # would fail with the isometries held
    assert abs(u_frozen - u_free) > 0.05 * abs(u_free)


def _gram(lam, seed):
    rng = np.random.default_rng(seed)
    w, _ = np.linalg.qr(rng.standard_normal((len(lam), len(lam))))
    return (w * np.asarray(lam)[None, :]) @ w.T, w


def _projector(g, kept):
    lam, w = np.linalg.eigh(g)
    u = w[:, np.argsort(lam)[::-1][:kept]]
    return u @ u.T


def test_isometry_derivative_is_the_projector_derivative():
    d1, d2, cap = 3, 4, 5
    lam = [3.0, 2.2, 1.7, 1.1, 0.8, 0.31, 0.2, 0.12, 0.05, 0.02, 0.0, 0.0]   # rank 10, gap at the cut
    g, _ = _gram(lam, 4)
    rng = np.random.default_rng(5)
    dg = rng.standard_normal((12, 12))
    dg = dg + dg.T
    prm = trg.Params(D=cap, tau_deg=0.0)
    u = trg.triad_isometry(g, d1, d2, cap, prm, "t", {})
    du = impurity._iso_tangent(g, dg, d1, d2, cap, prm).reshape(12, cap)
    dp = du @ u.T + u @ du.T
    eps = 1e-5
    fd = (_projector(g + eps * dg, cap) - _projector(g - eps * dg, cap)) / (2 * eps)
    assert np.max(np.abs(dp - fd)) <= 1e-8 * np.max(np.abs(fd))
    # dU is orthogonal to the kept subspace (a rotation inside it cancels)
    assert np.max(np.abs(u.T @ du)) <= 1e-13


def test_isometry_derivative_leaves_out_pairs_closer_than_1e12():
    d1, d2, cap = 2, 4, 4
    lam = [1.0, 0.5, 0.2, 3e-13, 2e-13, 0.0, 0.0, 0.0]   # kept 4; the cut pair 1e-13 apart
    g, w = _gram(lam, 6)
    rng = np.random.default_rng(7)
    dg = rng.standard_normal((8, 8))
    dg = dg + dg.T
    prm = trg.Params(D=cap, tau_deg=0.0)
    u = trg.triad_isometry(g, d1, d2, cap, prm, "t", {})
    du = impurity._iso_tangent(g, dg, d1, d2, cap, prm).reshape(8, cap)
    lam_c, w_c = trg.jacobi_eigh(g)
    assert trg.kept_count(lam_c, cap, prm.eps_lam, prm.tau_deg) == 4
    w4 = w_c[:, 4]   # the discarded partner of the smallest kept value
    # no rotation between the pair: u_3 does not move along w_4
    assert abs(w4 @ du[:, 3]) <= 1e-12 * np.max(np.abs(du))
    # a separated pair keeps the first-order coefficient
    i0 = int(np.argmax(np.abs(u.T @ w_c[:, 0])))   # the column of u along the top eigenvector
    coef = (w4 @ dg @ u[:, i0]) / (lam_c[0] - lam_c[4])
    assert abs(w4 @ du[:, i0] - coef) <= 1e-10 * abs(coef)
