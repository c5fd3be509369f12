"""Ising model: initial tensor and the exact results that pin the oracle.

Test infrastructure only.

Model (Sec. III): H = -sum_<ij> s_i s_j with s = +-1; here with a site
field, Z = sum_s exp(beta sum_{n,mu} s_n s_{n+mu} + h sum_n s_n) on a periodic
torus.  The field enters the site tensor as exp(h s) (no factor beta).

Initial tensor (Sec. III, CP form):
    T[i_1..i_d; j_1..j_d] = sum_a exp(h s_a) prod_mu W[a, i_mu] W[a, j_mu],
    W = [[sqrt(cosh b), sqrt(sinh b)], [sqrt(cosh b), -sqrt(sinh b)]],
row a = 0 <-> s = +1, row a = 1 <-> s = -1, so that sum_i W[a,i] W[b,i] =
exp(beta s_a s_b).  It is returned as the pair (Phi, Psi) with
T = sum_a Phi[..., a] Psi[..., a], which is the state the RG step consumes.
"""
import itertools
import math

import numpy as np


def ising_w(beta):
    cb = math.sqrt(math.cosh(beta))
    sb = math.sqrt(math.sinh(beta))
    return np.array([[cb, sb], [cb, -sb]], dtype=np.float64)


def ising_cp(beta, h, d):
    """CP factors (Phi, Psi), each of shape (2,)*d + (2,)."""
    w = ising_w(beta)
    spins = np.array([1.0, -1.0])
    phi = np.empty((2,) * d + (2,))
    psi = np.empty((2,) * d + (2,))
    for a in range(2):
        prod = np.ones((2,) * d)
        for mu in range(d):
            shape = [1] * d
            shape[mu] = 2
            prod = prod * w[a].reshape(shape)
        psi[..., a] = prod
        phi[..., a] = math.exp(h * spins[a]) * prod
    return phi, psi


def ising_tensor(beta, h, d):
    """Dense T[i_1..i_d, j_1..j_d]."""
    phi, psi = ising_cp(beta, h, d)
    return np.tensordot(phi, psi, axes=([d], [d]))


def _logsumexp(x):
    m = np.max(x)
    return m + math.log(np.sum(np.exp(x - m)))


def enumerate_log_z_per_site(beta, h, extents):
    """log Z / V by summing all 2^V configurations of a periodic torus.

    Bonds are sum over sites n and axes mu of s_n s_{n + mu (mod L_mu)}: an
    axis of extent 1 gives the self-bond s_n s_n = 1 and an axis of extent 2
    counts each neighbour pair twice, exactly as the tensor network does.
    """
    extents = tuple(int(e) for e in extents)
    v = int(np.prod(extents))
    if v > 22:
        raise ValueError("enumeration limited to V <= 22")
    sites = list(itertools.product(*[range(e) for e in extents]))
    index = {s: i for i, s in enumerate(sites)}
    bonds = []
    for s in sites:
        for mu, e in enumerate(extents):
            t = list(s)
            t[mu] = (t[mu] + 1) % e
            bonds.append((index[s], index[tuple(t)]))
    bonds = np.array(bonds, dtype=np.int64)
    n = np.arange(2 ** v, dtype=np.int64)
    spins = 1 - 2 * ((n[:, None] >> np.arange(v)[None, :]) & 1)
    e_bond = np.sum(spins[:, bonds[:, 0]] * spins[:, bonds[:, 1]], axis=1)
    mag = np.sum(spins, axis=1)
    return _logsumexp(beta * e_bond + h * mag) / v


def enumerate_derivatives_per_site(beta, h, extents):
    """(d/dbeta, d/dh) of log Z / V on the same torus by enumeration:
    <sum_{n,mu} s_n s_{n+mu}> / V and <sum_n s_n> / V (Boltzmann averages)."""
    extents = tuple(int(e) for e in extents)
    v = int(np.prod(extents))
    if v > 22:
        raise ValueError("enumeration limited to V <= 22")
    sites = list(itertools.product(*[range(e) for e in extents]))
    index = {s: i for i, s in enumerate(sites)}
    bonds = []
    for s in sites:
        for mu, e in enumerate(extents):
            t = list(s)
            t[mu] = (t[mu] + 1) % e
            bonds.append((index[s], index[tuple(t)]))
    bonds = np.array(bonds, dtype=np.int64)
    n = np.arange(2 ** v, dtype=np.int64)
    spins = 1 - 2 * ((n[:, None] >> np.arange(v)[None, :]) & 1)
    e_bond = np.sum(spins[:, bonds[:, 0]] * spins[:, bonds[:, 1]], axis=1).astype(np.float64)
    mag = np.sum(spins, axis=1).astype(np.float64)
    x = beta * e_bond + h * mag
    w = np.exp(x - np.max(x))
    z = np.sum(w)
    return float(np.sum(w * e_bond) / z / v), float(np.sum(w * mag) / z / v)


def onsager_energy(beta):
    """Onsager's internal energy per site of the 2D model (H = -sum s s):
    u = -coth(2b) [1 + (2/pi)(2 tanh^2(2b) - 1) K(k)], k = 2 sinh 2b / cosh^2 2b,
    with K the complete elliptic integral of the first kind (here by the
    arithmetic-geometric mean: K(k) = pi / (2 AGM(1, sqrt(1 - k^2))))."""
    k = 2 * math.sinh(2 * beta) / math.cosh(2 * beta) ** 2
    a, b = 1.0, math.sqrt(max(0.0, 1.0 - k * k))
    for _ in range(60):
        a, b = 0.5 * (a + b), math.sqrt(a * b)
    kk = math.pi / (2 * a)
    return -(1.0 / math.tanh(2 * beta)) * (1 + (2 / math.pi) * (2 * math.tanh(2 * beta) ** 2 - 1) * kk)


# Coefficients a_4, a_6, a_8 of the high-temperature series of log Z/V on the
# d-dimensional hypercubic lattice (h = 0), in t = tanh(beta):
#   log Z/V = ln 2 + d ln cosh(beta) + a_4 t^4 + a_6 t^6 + a_8 t^8 + O(t^10).
# With Z = 2^V cosh^{dV}(beta) sum_G t^|G| over the even bond subgraphs G, the
# cluster expansion of the logarithm gives a_4 = p_4, a_6 = p_6 (polygons per
# site) and a_8 = p_8 + f_8 - c_8 / 2: f_8 pairs of plaquettes touching at one
# site only (a connected even subgraph), c_8 ordered pairs of plaquettes that
# share at least one site, a plaquette with itself included.  Per plaquette,
# 2d - 3 others share each of its 4 edges and 8d^2 - 24d + 20 others share a
# single site, so f_8 - c_8 / 2 = -(d(d-1)/4) (1 + 4(2d - 3)).  The polygon
# counts p_n are 1, 2, 7 (2D), 3, 22, 207 (3D) and 6, 76, 1434 (4D).
HTE_COEFFS = {2: (1.0, 2.0, 4.5), 3: (3.0, 22.0, 187.5), 4: (6.0, 76.0, 1371.0)}


def hte_series(beta, d=4, order=8):
    """High-temperature series of log Z/V (h = 0, thermodynamic limit) through t^order."""
    t = math.tanh(beta)
    a4, a6, a8 = HTE_COEFFS[d]
    val = math.log(2.0) + d * math.log(math.cosh(beta))
    for n, a in ((4, a4), (6, a6), (8, a8)):
        if n <= order:
            val += a * t ** n
    return val


def hte_4d(beta):
    """High-temperature series of log Z/V (4D, h=0) through t^8, t = tanh beta.

    log Z/V = ln 2 + 4 ln cosh b + 6 t^4 + 76 t^6 + 1371 t^8 + O(t^10).
    """
    return hte_series(beta, 4, 8)


def lte_4d(beta):
    """Low-temperature series of log Z/V (4D, h=0, thermodynamic limit).

    One flipped spin breaks 8 bonds, an adjacent pair 14 (4 per site); the
    disconnected-pair term of the logarithm gives -(1 + 2d)/2 = -9/2 at e^{-32b}.
    """
    return 4.0 * beta + math.exp(-16 * beta) + 4.0 * math.exp(-28 * beta) - 4.5 * math.exp(-32 * beta)


def onsager_log_z(beta, n=1024):
    """Onsager: log Z/V = ln 2 + (1/8 pi^2) int int ln[cosh^2 2b - sinh 2b (cos t1 + cos t2)].

    The integrand is periodic and analytic off criticality, so the trapezoid
    rule on n x n points converges exponentially.
    """
    th = 2.0 * np.pi * np.arange(n) / n
    c = np.cos(th)
    val = np.log(math.cosh(2 * beta) ** 2 - math.sinh(2 * beta) * (c[:, None] + c[None, :]))
    return math.log(2.0) + 0.5 * float(np.mean(val))


def onsager_log_z_1d(beta, n=4096):
    """Onsager's single-integral form (independent of the double integral):

    log Z/V = ln(2 cosh 2b) + (1/2pi) int_0^pi ln[(1 + sqrt(1 - k^2 sin^2 th))/2] dth,
    k = 2 sinh 2b / cosh^2 2b; trapezoid on the periodic integrand.
    """
    k = 2 * math.sinh(2 * beta) / math.cosh(2 * beta) ** 2
    th = np.pi * np.arange(n) / n
    val = np.log(0.5 * (1.0 + np.sqrt(1.0 - (k * np.sin(th)) ** 2)))
    return math.log(2 * math.cosh(2 * beta)) + 0.5 * float(np.mean(val))
