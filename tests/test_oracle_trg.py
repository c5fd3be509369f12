"""Pins of the oracle's RG step against exact results and brute-force definitions.

* exact finite tori: the first two steps at D = 16 truncate nothing (ranks are
  at most 2^(#spins in the block)), so log Z/V must equal the enumeration of
  the 2x1x1x1 and 2x2x1x1 tori; two steps plus an exact contraction of the
  residual 1x1x2x2 network must equal the 2^16-configuration sum of the
  L = 2 hypercubic torus; in 2D three exact steps plus the residual trace
  must equal the 4x4 enumeration;
* beta = 0: log Z/V = ln(2 cosh h) for any D and number of steps;
* series and Onsager: thermodynamic-limit values within the truncation error;
* structural identities: triad-ATRG with R = D^2 is ATRG (Sec. II B), and the
  free energy does not depend on the axis the cycle starts on;
* each truncation against its definition on tiny explicit networks.
"""
import math

import numpy as np
import pytest

from oracle import trg
from oracle.ising import enumerate_log_z_per_site, hte_4d, lte_4d, onsager_log_z
from oracle.linalg import qr_pos


# ---------------------------------------------------------------- exact tori

@pytest.mark.parametrize("method", ["triad", "atrg"])
@pytest.mark.parametrize("mode", ["sketch", "exact"])
@pytest.mark.parametrize("h", [0.0, 0.15])
def test_first_two_steps_are_exact(method, mode, h):
    beta = 0.1497
    st = trg.init_ising(beta, h, 4)
    prm = trg.Params(D=16, bond_svd=mode, seed=7)
    for nst, ext in [(1, (2, 1, 1, 1)), (2, (2, 2, 1, 1))]:
        trg.rg_step(st, nst - 1, prm, method)
        ref = enumerate_log_z_per_site(beta, h, ext)
        assert abs(trg.log_z_per_site(st) - ref) < 1e-13


def _residual_4d(st):
    """log Z of the 1 x 1 x 2 x 2 torus built from the current coarse tensor."""
    tz = np.einsum("xyzwg,xyuvg->zwuv", st.phi, st.psi)   # x, y legs self-traced
    # sites (a, b) on the (z, t) torus; Z[a,b] forward z bond, W[a,b] forward t bond
    names = {}
    letters = iter("abcdefgh")
    for a in range(2):
        for b in range(2):
            names[("z", a, b)] = next(letters)
            names[("t", a, b)] = next(letters)
    terms = []
    for a in range(2):
        for b in range(2):
            terms.append(names[("z", a, b)] + names[("t", a, b)]
                         + names[("z", (a - 1) % 2, b)] + names[("t", a, (b - 1) % 2)])
    return math.log(np.einsum(",".join(terms) + "->", tz, tz, tz, tz, optimize=True))


@pytest.mark.parametrize("method", ["triad", "atrg"])
def test_full_4d_l2_torus(method):
    beta, h = 0.1497, 0.05
    st = trg.init_ising(beta, h, 4)
    prm = trg.Params(D=16)
    trg.rg_step(st, 0, prm, method)
    trg.rg_step(st, 1, prm, method)
    lz = st.logacc + _residual_4d(st) / 16.0
    assert abs(lz - enumerate_log_z_per_site(beta, h, (2, 2, 2, 2))) < 1e-13


def test_2d_4x4_torus():
    beta, h = 0.44, 0.03
    st = trg.init_ising(beta, h, 2)
    prm = trg.Params(D=64)
    for ax in (0, 1, 0):
        trg.rg_step(st, ax, prm, "atrg")
    # residual: two tensors along y, x self-traced
    ty = np.einsum("xag,xbg->ab", st.phi, st.psi)
    lz = st.logacc + math.log(np.trace(ty @ ty)) / 16.0
    assert abs(lz - enumerate_log_z_per_site(beta, h, (4, 4))) < 1e-13


@pytest.mark.parametrize("method", ["triad", "atrg"])
@pytest.mark.parametrize("h", [0.0, 0.3, -1.2])
def test_beta_zero(method, h):
    lz, _ = trg.run(0.0, h, trg.Params(D=4), 8, method)
    assert abs(lz - math.log(2 * math.cosh(h))) < 1e-14


# ---------------------------------------------------- thermodynamic-limit pins

def test_high_temperature_series():
    beta = 0.001
    lz, _ = trg.run(beta, 0.0, trg.Params(D=8), 12, "triad")
    # ln 2 + 4 ln cosh b is reproduced to well inside the plaquette term 6 t^4
    assert abs(lz - hte_4d(beta)) < 6 * math.tanh(beta) ** 4


def test_high_temperature_deviation_shrinks_with_D():
    # At beta = 0.05 the truncation error at D <= 8 is itself of order t^4 (the
    # bond states that carry plaquettes across block faces outnumber D): the
    # deviation from the series is 1.6e-5, 1.15e-5, 8.9e-6 at D = 4, 6, 8, above
    # 76 t^6 = 1.2e-6, so the t^6 and t^8 terms are not resolved by the flow.
    # What is checked: the flow lies below the series and approaches it as D grows.
    beta = 0.05
    t = math.tanh(beta)
    dev = []
    for D in (4, 6, 8):
        lz, _ = trg.run(beta, 0.0, trg.Params(D=D, seed=1), 20, "triad")
        dev.append(lz - hte_4d(beta))
    assert all(v < 0 for v in dev)
    assert abs(dev[0]) > abs(dev[1]) > abs(dev[2])
    assert abs(dev[2]) < 1.5 * t ** 4


def test_low_temperature_series():
    beta = 1.0
    lz, _ = trg.run(beta, 0.0, trg.Params(D=4), 40, "triad")
    assert abs(lz - lte_4d(beta)) < 1e-9          # e^{-16 b} = 1.1e-7 is resolved


@pytest.mark.parametrize("beta", [0.3, 0.6])
def test_onsager_2d(beta):
    lz, _ = trg.run(beta, 0.0, trg.Params(D=8), 40, "atrg", d=2)
    assert abs(lz - onsager_log_z(beta)) < 3e-6


# ------------------------------------------------------ structural identities

def test_triad_with_full_overspan_is_atrg():
    prm_t = trg.Params(D=5, r=5, seed=3)
    prm_a = trg.Params(D=5, seed=3)
    lt, _ = trg.run(0.1497, 0.01, prm_t, 8, "triad")
    la, _ = trg.run(0.1497, 0.01, prm_a, 8, "atrg")
    assert abs(lt - la) < 1e-13


def test_axis_relabelling():
    prm = trg.Params(D=6, seed=5)
    la, _ = trg.run(0.1497, 0.0, prm, 8, "triad", start_axis=0)
    lb, _ = trg.run(0.1497, 0.0, prm, 8, "triad", start_axis=2)
    assert abs(la - lb) < 1e-13


# ---------------------------------------------------- pieces vs definitions

def _iso(rng, rows, cols):
    q, _ = qr_pos(rng.standard_normal((rows, cols)))
    return q


def test_resplit():
    rng = np.random.default_rng(0)
    phi = rng.standard_normal((2, 3, 2, 3, 5))
    psi = rng.standard_normal((2, 3, 2, 3, 5))
    a, b, c, d, cn, s = trg.resplit(phi, psi, 1e-14)
    t = phi.reshape(36, 5) @ psi.reshape(36, 5).T
    assert abs(cn - np.linalg.svd(t, compute_uv=False)[0]) < 1e-13 * cn
    assert np.max(np.abs(a @ b.T - t / cn)) < 1e-14
    assert np.max(np.abs(c @ d.T - t / cn)) < 1e-14
    assert np.max(np.abs(a.T @ a - np.eye(5))) < 1e-14
    assert np.max(np.abs(d.T @ d - np.eye(5))) < 1e-14


def _explicit_m(bt, ct):
    """M[(alpha, i_perp), (beta, j_perp)] = sum_x B[x, j_perp, alpha] C[x, i_perp, beta]."""
    xd, chia, chib = bt.shape[0], bt.shape[-1], ct.shape[-1]
    jn = int(np.prod(bt.shape[1:-1]))
    inn = int(np.prod(ct.shape[1:-1]))
    b3 = bt.reshape(xd, jn, chia)
    c3 = ct.reshape(xd, inn, chib)
    return np.einsum("xja,xib->aibj", b3, c3).reshape(chia * inn, chib * jn)


def test_bond_swap_exact_is_eckart_young():
    rng = np.random.default_rng(1)
    bt = rng.standard_normal((3, 2, 2, 2, 3))
    ct = rng.standard_normal((3, 2, 2, 2, 3))
    m = _explicit_m(bt, ct)
    prm = trg.Params(D=5, bond_svd="exact")
    x, sig, y = trg.bond_swap(bt, ct, prm, 0, {})
    xm = x.reshape(-1, x.shape[-1])
    ym = y.reshape(-1, y.shape[-1])
    sv = np.linalg.svd(m, compute_uv=False)
    assert np.allclose(sig, sv[:5], rtol=1e-13, atol=0)
    resid = np.linalg.norm(m - xm @ np.diag(sig) @ ym.T) ** 2
    assert abs(resid - np.sum(sv[5:] ** 2)) < 1e-12 * np.sum(sv ** 2)
    assert np.max(np.abs(xm.T @ xm - np.eye(5))) < 1e-13
    assert np.max(np.abs(ym.T @ ym - np.eye(5))) < 1e-13


def test_bond_swap_sketch_is_exact_when_the_sketch_spans_the_range():
    # B rank one in j_perp makes rank(M) <= chi = 2 = m < dim N: the randomized
    # SVD then spans the whole range and must equal the exact SVD
    rng = np.random.default_rng(2)
    bt = np.einsum("xa,j->xja", rng.standard_normal((2, 2)), rng.standard_normal(8)).reshape(2, 2, 2, 2, 2)
    ct = rng.standard_normal((2, 2, 2, 2, 2))
    m = _explicit_m(bt, ct)
    assert np.linalg.matrix_rank(m) <= 2
    rec = {}
    x, sig, y = trg.bond_swap(bt, ct, trg.Params(D=1, seed=11), 3, rec)
    assert rec["bond"]["mode"] == "sketch"
    x2, sig2, y2 = trg.bond_swap(bt, ct, trg.Params(D=1, bond_svd="exact"), 3, {})
    assert np.allclose(sig, sig2, rtol=1e-13, atol=0)
    p1 = x.reshape(-1, 1) @ np.diag(sig) @ y.reshape(-1, 1).T
    p2 = x2.reshape(-1, 1) @ np.diag(sig2) @ y2.reshape(-1, 1).T
    assert np.max(np.abs(p1 - p2)) < 1e-13 * sig[0]


@pytest.mark.parametrize("power_iters", [0, 1, 2])
def test_bond_swap_sketch_is_subspace_iteration(power_iters):
    # rank(M) = 27 > m = 6: the randomized SVD is an approximation, and it must be
    # the one of subspace iteration (Halko, Martinsson, Tropp, SIAM Rev. 2011):
    # Q = orth((M M^T)^(q-1) M Omega) with q = power_iters + 1 passes, Omega the
    # sketch drawn in M's column index (beta, j_perp), and the kept triplets those
    # of the SVD of Q^T M, mapped back through Q.  Computed here on the explicit M.
    from oracle.philox import sketch_omega
    rng = np.random.default_rng(21)
    xd, chi, tdim = 3, 3, (4, 4, 4)
    bt = rng.standard_normal((xd,) + tdim + (chi,))
    ct = rng.standard_normal((xd,) + tdim + (chi,))
    m = _explicit_m(bt, ct)                          # (alpha, i_perp) x (beta, j_perp)
    assert np.linalg.matrix_rank(m) == 27
    D, step, seed = 3, 5, 99
    prm = trg.Params(D=D, sketch_mult=2, power_iters=power_iters, seed=seed)
    rec = {}
    x, sig, y = trg.bond_swap(bt, ct, prm, step, rec)
    assert rec["bond"]["mode"] == "sketch"
    om = sketch_omega(seed, step, 0, chi, tdim, 2 * D).reshape(chi * 64, 2 * D)
    yk = np.linalg.matrix_power(m @ m.T, power_iters) @ m @ om
    q, _ = np.linalg.qr(yk)
    u, sv, vt = np.linalg.svd(q.T @ m)
    k = rec["bond"]["kept"]
    assert k == D
    assert np.allclose(sig[:k], sv[:k], rtol=1e-11, atol=0)
    approx_ref = (q @ u[:, :k]) @ np.diag(sv[:k]) @ vt[:k]
    xm = x.reshape(-1, x.shape[-1])[:, :k]
    ym = y.reshape(-1, y.shape[-1])[:, :k]
    assert np.max(np.abs(xm @ np.diag(sig[:k]) @ ym.T - approx_ref)) < 1e-11 * sv[0]
    # the sketch is not the exact SVD here (so the check above is not vacuous)
    assert np.max(np.abs(sig[:k] - np.linalg.svd(m, compute_uv=False)[:k])) > 1e-6 * sv[0]


def _explicit_gamma(a, xs, y, dt):
    """Gamma[i_a, t.., b.., t'.., j_a, b'..] = sum A X sigma Y D (legs of dim 2, d = 4)."""
    up = np.einsum("xijka,aLMNg->xijkLMNg", a, xs)      # i_a, top fwd, bottom fwd, g
    lo = np.einsum("bPQRg,yUVWb->PQRyUVWg", y, dt)      # top bwd, j_a, bottom bwd, g
    return up, lo


def test_env_grams_match_explicit_cell():
    rng = np.random.default_rng(4)
    a = rng.standard_normal((2, 2, 2, 2, 3))
    xs = rng.standard_normal((3, 2, 2, 2, 4))
    y = rng.standard_normal((3, 2, 2, 2, 4))
    dt = rng.standard_normal((2, 2, 2, 2, 3))
    up, lo = _explicit_gamma(a, xs, y, dt)
    pl = np.einsum("PQRyUVWg,PQRyUVWh->gh", lo, lo)     # lower-block Gram
    ou = np.einsum("xijkLMNg,xijkLMNh->gh", up, up)     # upper-block Gram
    gam = np.einsum("xijkLMNg,PQRyUVWg->xijkLMNPQRyUVW", up, lo)
    for pos in range(3):
        kf, kb = trg.env_grams(a, xs, pl, y, dt, ou, pos)
        # forward pair: top leg axis 1+pos, bottom leg axis 4+pos of gam
        g1 = np.moveaxis(gam, [1 + pos, 4 + pos], [-2, -1]).reshape(-1, 4)
        assert np.max(np.abs(kf - g1.T @ g1)) < 1e-12 * np.max(np.abs(kf))
        # backward pair: top (Y) leg axis 7+pos, bottom (D) leg axis 11+pos
        g2 = np.moveaxis(gam, [7 + pos, 11 + pos], [-2, -1]).reshape(-1, 4)
        assert np.max(np.abs(kb - g2.T @ g2)) < 1e-12 * np.max(np.abs(kb))


def test_squeezer_is_optimal_on_the_bond():
    rng = np.random.default_rng(5)
    npair, k = 9, 4
    zx = rng.standard_normal((30, npair)) @ np.diag(0.6 ** np.arange(npair))
    zy = rng.standard_normal((25, npair)) @ np.diag(0.7 ** np.arange(npair))
    prm = trg.Params(D=k)
    e, f = trg.squeezer(zx.T @ zx, zy.T @ zy, 3, 3, prm, "sq", {})
    e = e.reshape(npair, k)
    f = f.reshape(npair, k)
    bond = zx @ zy.T
    u, s, vt = np.linalg.svd(bond)
    best = u[:, :k] @ np.diag(s[:k]) @ vt[:k]
    assert np.max(np.abs(zx @ e @ f.T @ zy.T - best)) < 1e-12 * s[0]
    assert np.max(np.abs(f.T @ e - np.eye(k))) < 1e-11


def test_triad_grams_are_hosvd_of_canonical_gamma():
    rng = np.random.default_rng(6)
    a = _iso(rng, 16, 3).reshape(2, 2, 2, 2, 3)
    x = _iso(rng, 24, 4).reshape(3, 2, 2, 2, 4)
    y = _iso(rng, 24, 4).reshape(3, 2, 2, 2, 4)
    dt = _iso(rng, 16, 3).reshape(2, 2, 2, 2, 3)
    sig = np.array([1.0, 0.6, 0.3, 0.05])
    up, lo = _explicit_gamma(a, x * sig, y, dt)
    gam = np.einsum("xijkLMNg,PQRyUVWg->xijkLMNPQRyUVW", up, lo)
    grams = trg.triad_grams(a, x, sig, y, dt)
    pairs = [(1, 2), (4, 5), (7, 8), (11, 12)]        # (t1, t2) of A, X, Y, D
    for gm, (p1, p2) in zip(grams, pairs):
        g = np.moveaxis(gam, [p1, p2], [-2, -1]).reshape(-1, 4)
        assert np.max(np.abs(gm - g.T @ g)) < 1e-13


def test_make_phi_is_the_naive_contraction():
    rng = np.random.default_rng(7)
    e = rng.standard_normal((2, 3, 2, 2))     # E[i_a, kA, t3, alpha]
    f = rng.standard_normal((2, 3, 2, 3))     # F[alpha, kX, t3, g]
    ti = rng.standard_normal((2, 2, 3))
    tj = rng.standard_normal((2, 2, 3))
    m1, m2, m3 = (rng.standard_normal((2, 2, 3)) for _ in range(3))
    phi = trg.make_phi(e, f, ti, tj, m1, m2, m3)
    at = np.einsum("xkta,ijk->xijta", e, ti)
    xt = np.einsum("aktg,ijk->aijtg", f, tj)
    ref = np.einsum("xijta,apqsg,ipk,jql,tsc->xklcg", at, xt, m1, m2, m3)
    assert np.max(np.abs(phi - ref)) < 1e-12
    psi = trg.make_psi(f.transpose(0, 1, 2, 3), e.transpose(0, 1, 2, 3), ti, tj, m1, m2, m3)
    yt = np.einsum("bktg,ijk->bijtg", f, ti)
    dtt = np.einsum("xktb,ijk->xijtb", e, tj)
    ref2 = np.einsum("bijtg,xpqsb,ipk,jql,tsc->xklcg", yt, dtt, m1, m2, m3)
    assert np.max(np.abs(psi - ref2)) < 1e-12
