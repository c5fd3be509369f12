"""Pins of the Ising initial tensor and of the exact results used as references."""
import itertools
import math

import numpy as np
import pytest

from oracle.ising import (ising_w, ising_tensor, ising_cp, enumerate_log_z_per_site,
                          onsager_log_z, onsager_log_z_1d, hte_4d, lte_4d, hte_series, HTE_COEFFS)


@pytest.mark.parametrize("beta", [0.0, 0.1497, 0.7])
def test_w_reproduces_bond_weight(beta):
    w = ising_w(beta)
    s = np.array([1.0, -1.0])
    assert np.allclose(w @ w.T, np.exp(beta * np.outer(s, s)), rtol=1e-15, atol=0)


def test_tensor_rank_and_symmetry():
    t = ising_tensor(0.2, 0.1, 4)
    m = t.reshape(16, 16)
    sv = np.linalg.svd(m, compute_uv=False)
    assert np.sum(sv > 1e-12 * sv[0]) == 2
    t0 = ising_tensor(0.0, 0.1, 4).reshape(16, 16)
    sv0 = np.linalg.svd(t0, compute_uv=False)
    assert np.sum(sv0 > 1e-12 * sv0[0]) == 1
    # axis permutation symmetry of T (h = 0)
    t = ising_tensor(0.3, 0.0, 4)
    tp = np.transpose(t, (1, 2, 0, 3, 5, 6, 4, 7))
    assert np.allclose(t, tp, rtol=1e-15, atol=0)


def test_single_site_torus():
    # one site with all legs self-traced: every axis gives a self-bond s s = 1
    for d in (2, 4):
        t = ising_tensor(0.3, 0.2, d).reshape(2 ** d, 2 ** d)
        ref = math.log(math.exp(d * 0.3) * 2 * math.cosh(0.2))
        assert abs(math.log(np.trace(t)) - ref) < 1e-14
        assert abs(enumerate_log_z_per_site(0.3, 0.2, (1,) * d) - ref) < 1e-14


@pytest.mark.parametrize("length", [3, 6, 11])
def test_enumeration_vs_transfer_matrix_1d(length):
    beta, h = 0.37, 0.21
    # symmetric transfer matrix exp(beta s s' + h (s + s')/2)
    tm = np.array([[math.exp(beta + h), math.exp(-beta)], [math.exp(-beta), math.exp(beta - h)]])
    ev = np.linalg.eigvalsh(tm)
    ref = math.log(np.sum(ev ** length)) / length
    assert abs(enumerate_log_z_per_site(beta, h, (length,)) - ref) < 1e-13


def test_enumeration_vs_tensor_network_2x2():
    # brute-force contraction of the 2x2 torus from the dense tensor
    beta, h = 0.41, 0.07
    t = ising_tensor(beta, h, 2)      # legs f_x, f_y, b_x, b_y
    sites = [(0, 0), (1, 0), (0, 1), (1, 1)]
    # bond variable names: xb[s] forward x of s, yb[s] forward y of s
    letters = "abcdefgh"
    xb = {s: letters[i] for i, s in enumerate(sites)}
    yb = {s: letters[4 + i] for i, s in enumerate(sites)}
    terms = []
    for (x, y) in sites:
        fx = xb[(x, y)]
        fy = yb[(x, y)]
        bx = xb[((x - 1) % 2, y)]
        by = yb[(x, (y - 1) % 2)]
        terms.append(fx + fy + bx + by)
    z = np.einsum(",".join(terms) + "->", t, t, t, t)
    assert abs(math.log(z) / 4 - enumerate_log_z_per_site(beta, h, (2, 2))) < 1e-14


@pytest.mark.parametrize("beta", [0.2, 0.3, 0.6, 0.9])
def test_onsager_two_forms_agree(beta):
    assert abs(onsager_log_z(beta) - onsager_log_z_1d(beta)) < 1e-13


def test_onsager_limits():
    # high temperature: ln 2 + 2 ln cosh b + t^4 + 2 t^6 + 9/2 t^8 (2D square lattice)
    b = 0.02
    t = math.tanh(b)
    hte2 = math.log(2) + 2 * math.log(math.cosh(b)) + t ** 4 + 2 * t ** 6 + 4.5 * t ** 8
    assert abs(onsager_log_z(b) - hte2) < 1e-14
    # low temperature (dual of the high-T series): 2b + u^2 + 2u^3 + 9/2 u^4 + 12 u^5, u = e^{-4b}
    b = 1.5
    u = math.exp(-4 * b)
    lte2 = 2 * b + u ** 2 + 2 * u ** 3 + 4.5 * u ** 4 + 12 * u ** 5
    assert abs(onsager_log_z(b) - lte2) < 1e-12


def test_series_4d_leading_terms():
    assert abs(hte_4d(0.0) - math.log(2)) < 1e-16
    assert lte_4d(5.0) == pytest.approx(20.0, abs=1e-30)
    # CP factors reproduce T
    phi, psi = ising_cp(0.3, 0.1, 4)
    assert np.allclose(np.tensordot(phi, psi, ([4], [4])), ising_tensor(0.3, 0.1, 4))


# ---------------------------------------------------------------- series coefficients

def _closed_walks(d, n):
    """Rooted, directed closed self-avoiding walks of n steps on Z^d (brute force)."""
    steps = []
    for mu in range(d):
        for s in (1, -1):
            v = [0] * d
            v[mu] = s
            steps.append(tuple(v))
    origin = (0,) * d
    seen = {origin}
    count = 0

    def walk(pos, k):
        nonlocal count
        if k == n - 1:
            if sum(abs(a) for a in pos) == 1:
                count += 1
            return
        for st in steps:
            nxt = tuple(a + b for a, b in zip(pos, st))
            if nxt in seen or sum(abs(a) for a in nxt) > n - k - 1:
                continue
            seen.add(nxt)
            walk(nxt, k + 1)
            seen.discard(nxt)

    walk(origin, 0)
    return count


def _plaquette_overlaps(d):
    """For the plaquette at the origin in the (0, 1) plane: number of other plaquettes
    sharing an edge with it and sharing exactly one site with it (brute force)."""
    def sites(base, mu, nu):
        e = [0] * d
        f = [0] * d
        e[mu] = 1
        f[nu] = 1
        b = tuple(base)
        return {b, tuple(x + y for x, y in zip(b, e)), tuple(x + y for x, y in zip(b, f)),
                tuple(x + y + z for x, y, z in zip(b, e, f))}

    ref = sites((0,) * d, 0, 1)
    edge = corner = 0
    for base in itertools.product(range(-1, 2), repeat=d):
        for mu in range(d):
            for nu in range(mu + 1, d):
                s = sites(base, mu, nu)
                if s == ref:
                    continue
                k = len(s & ref)
                if k == 2:
                    edge += 1
                elif k == 1:
                    corner += 1
    return edge, corner


@pytest.mark.parametrize("d", [2, 3, 4])
def test_series_coefficients_from_polygon_counts(d):
    # a_4 = p_4, a_6 = p_6, a_8 = p_8 + f_8 - c_8 / 2 (cluster expansion of log of
    # the even-subgraph sum); every count is done here by brute force
    p = {n: _closed_walks(d, n) / (2 * n) for n in (4, 6, 8)}
    nplaq = d * (d - 1) // 2
    edge, corner = _plaquette_overlaps(d)
    f8 = nplaq * corner / 2.0
    c8 = nplaq * (1 + edge + corner)
    a = (p[4], p[6], p[8] + f8 - c8 / 2.0)
    assert a == HTE_COEFFS[d]


@pytest.mark.parametrize("beta", [0.05, 0.08])
def test_2d_series_against_onsager(beta):
    # the same derivation in 2D against the exact solution: the residual after t^8
    # is the t^10 term (12 t^10)
    t = math.tanh(beta)
    assert abs(onsager_log_z(beta) - hte_series(beta, 2, 8)) < 13 * t ** 10
    assert abs(onsager_log_z(beta) - hte_series(beta, 2, 6)) > 4 * t ** 8
