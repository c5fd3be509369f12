"""Impurity-tensor derivatives of log Z/V (Sec. III D) in FP64 (test infrastructure only).

The paper obtains the internal energy from a network that carries impurity
tensors through the same coarse-graining as the pure tensor.  Here the
impurity is the derivative of the site tensor, dT = dT/d(theta) for theta =
beta or h, summed over every site: with every truncation of the pure flow
held fixed (bond-swap subspaces, triad isometries, squeezers, norms c_k),
each coarse tensor is multilinear in the finer ones, so the product rule
carries the summed impurity from level to level, and

    d(log Z/V)/d(theta) = 2^-n Tr(dT^(n)) / Tr(T^(n)).

u = -d(log Z/V)/d(beta) is the internal energy per site (H = -sum s s) and
m = d(log Z/V)/dh the magnetisation.  Where no truncation acts (exact finite
tori, beta = 0) this is the exact derivative; otherwise it differs from the
derivative of the truncated flow by terms of the order of the truncation.

Readings (the paper gives no formulas for this part):
* the state (Phi, Psi) carries a tangent (dPhi, dPsi), T + e dT =
  (Phi + e dPhi)(Psi + e dPsi)^T to first order;
* re-split: T/c = A B^T = C D^T with A, D isometric is exact for the pure
  tensor; the tangent is written in the tangent space of the rank-chi
  matrices at T with the gauge A^T dA = 0 (resp. D^T dD = 0):
  dT/c = dA B^T + A dB^T,  dB = (dT/c)^T A,  dA = (1 - A A^T)(dT/c) D S'^+,
  dT/c = dC D^T + C dD^T,  dC = (dT/c) D,  dD = (1 - D D^T)(dT/c)^T A S'^+,
  S' the re-split's (canonical) singular-value matrix, S'^+ its inverse on
  the kept values;
* bond swap: the tangent of the truncated product X sigma Y^T is taken in the
  tangent space of the rank-chi matrices at it (the first-order change of a
  truncated SVD when the discarded values are negligible), and split over
  both factors: d(X sigma) = dM Y, dY = (1 - Y Y^T) dM^T X sigma^+ with
  dM = dB C + B dC, so F = (X sigma) U^X and G = Y U^Y both move;
* triad isometries: the coarse tensor depends on each U only through its
  projector U U^T (E = A U^A meets I = U^A in makeMG, and so on), so a
  first-order change of U within its kept subspace cancels.  The kept
  subspace moves with the Gram (eq. HOSVD): dU = W C, W the discarded
  eigenvectors and C[j, i] = w_j^T dG u_i / (lam_i - lam_j) (first-order
  perturbation of an invariant subspace), with dG the Gram's tangent from
  dA, d(X sigma), dY, dD.  Pairs with lam_i - lam_j <= 1e-12 lam_1 are left
  out (C = 0): eigen-directions whose eigenvalues lie that close are not
  determined by the Gram (at D = 8, h = 0 the kept/discarded cut falls
  between eigenvalues of 1.2e-14 and 6.6e-15 of the largest, within a few
  rounding errors eps lam_1 of each other), so the rotation between them
  has no derivative; the pair is treated as degenerate, as a multiplet.  Holding U instead (iso=False) gives the
  derivative of the flow with its isometries frozen, which near T_c differs
  from the flow's own derivative by 10 % or more; the squeezers are held
  (freezing them moves the derivative by about 1e-3 at D = 8);
* E..H take dA, d(X sigma), dY, dD and A dU^A, (X sigma) dU^X, Y dU^Y, D dU^D,
  and the triad tensors I..L in makeMG / makeMH take dU as well.
"""
import math

import numpy as np

from . import trg
from .ising import ising_w


def ising_cp_tangent(beta, h, d, wrt):
    """(dPhi, dPsi) of the CP factors with respect to ``wrt`` = "beta" (beta > 0) or "h"."""
    w = ising_w(beta)
    spins = np.array([1.0, -1.0])
    if wrt == "beta":
        if not beta > 0.0:
            raise ValueError("the CP factors are not differentiable in beta at beta = 0")
        cb, sb = math.sqrt(math.cosh(beta)), math.sqrt(math.sinh(beta))
        dw = np.array([[math.sinh(beta) / (2 * cb), math.cosh(beta) / (2 * sb)],
                       [math.sinh(beta) / (2 * cb), -math.cosh(beta) / (2 * sb)]])
    elif wrt != "h":
        raise ValueError("wrt must be 'beta' or 'h'")
    dphi = np.zeros((2,) * d + (2,))
    dpsi = np.zeros((2,) * d + (2,))
    for a in range(2):
        def outer(rows):
            prod = np.ones((2,) * d)
            for mu in range(d):
                shape = [1] * d
                shape[mu] = 2
                prod = prod * rows[mu].reshape(shape)
            return prod
        fa = math.exp(h * spins[a])
        if wrt == "h":
            dphi[..., a] = spins[a] * fa * outer([w[a]] * d)
        else:
            dprod = np.zeros((2,) * d)
            for mu in range(d):
                rows = [w[a]] * d
                rows[mu] = dw[a]
                dprod += outer(rows)
            dphi[..., a] = fa * dprod
            dpsi[..., a] = dprod
    return dphi, dpsi


class ImpurityState:
    """Pure state plus its tangents (one per derivative)."""

    def __init__(self, beta, h, d=4, wrt=("beta", "h")):
        self.pure = trg.init_ising(beta, h, d)
        self.wrt = tuple(wrt)
        self.tan = [ising_cp_tangent(beta, h, d, v) for v in self.wrt]


def _resplit_tangent(kp, dphi, dpsi):
    """(dA, dB, dC, dD) as natural-order matrices (rows = legs, cols = bond)."""
    phi, psi = kp["phi"], kp["psi"]
    f = int(np.prod(phi.shape[:-1]))
    ph, ps = phi.reshape(f, -1), psi.reshape(f, -1)
    dph, dps = dphi.reshape(f, -1), dpsi.reshape(f, -1)
    a, dm, c, s, rot = kp["am"], kp["dm"], kp["c"], kp["s"], kp["rot"]
    sinv = np.where(s > 0.0, 1.0 / np.where(s > 0.0, s, 1.0), 0.0)
    spp = rot.T @ np.diag(sinv) @ rot
    z1 = (dph @ (ps.T @ dm) + ph @ (dps.T @ dm)) / c     # (dT/c) D
    z2 = (ps @ (dph.T @ a) + dps @ (ph.T @ a)) / c       # (dT/c)^T A
    da = (z1 - a @ (a.T @ z1)) @ spp
    ddm = (z2 - dm @ (dm.T @ z2)) @ spp
    return da, z2, z1, ddm


def _bond_tangent(kp, db, dcc):
    """Tangents of the two bond-swap factors, X sigma Y^T ~ M = sum_x B C.

    With dM = dB C + B dC, the first-order change of the truncated product in
    the tangent space of the rank-chi matrices is P_X dM + dM P_Y - P_X dM P_Y,
    written as d(X sigma) Y^T + X sigma dY^T with d(X sigma) = dM Y and
    dY = (1 - Y Y^T) dM^T X sigma^+.  Returns (d(X sigma), dY) shaped like X, Y.
    """
    x, y, b, cc, sig = kp["x"], kp["y"], kp["b"], kp["cc"], kp["sig"]
    xd, chia = b.shape[0], b.shape[-1]
    chib = cc.shape[-1]
    g = x.shape[-1]
    xm = x.reshape(chia, -1, g)
    ym = y.reshape(chib, -1, g)
    bm, ccm = b.reshape(xd, -1, chia), cc.reshape(xd, -1, chib)
    dbm, dccm = db.reshape(xd, -1, chia), dcc.reshape(xd, -1, chib)
    # (dM Y)[alpha, i, g] = sum_{x, beta, j} (dB[x, j, alpha] C[x, i, beta] + B dC) Y[beta, j, g]
    by = np.einsum("xja,bjh->xabh", bm, ym, optimize=True)
    dby = np.einsum("xja,bjh->xabh", dbm, ym, optimize=True)
    dxs = (np.einsum("xib,xabh->aih", ccm, dby, optimize=True) +
           np.einsum("xib,xabh->aih", dccm, by, optimize=True))
    # (dM^T X)[beta, j, g] = sum_{x, alpha, i} (dB C + B dC)[x; alpha, i; beta, j] X[alpha, i, g]
    cx = np.einsum("xib,aig->xabg", ccm, xm, optimize=True)
    dcx = np.einsum("xib,aig->xabg", dccm, xm, optimize=True)
    dmtx = (np.einsum("xja,xabg->bjg", dbm, cx, optimize=True) +
            np.einsum("xja,xabg->bjg", bm, dcx, optimize=True))
    sinv = np.where(sig > 0.0, 1.0 / np.where(sig > 0.0, sig, 1.0), 0.0)
    dy = dmtx * sinv
    dy = dy - np.einsum("bjh,ckh,ckg->bjg", ym, ym, dy, optimize=True)
    return dxs.reshape(x.shape), dy.reshape(y.shape)


def _gram_tangents(a, x, sig, y, dt, da, dxs, dy, ddm):
    """Tangents of the four triad Grams (see trg.triad_grams).

    With M_k = X sigma Y^T the truncated bond-swap product, X sigma^2 X^T =
    M_k M_k^T and Y sigma^2 Y^T = M_k^T M_k; along dM_k = d(X sigma) Y^T + X
    sigma dY^T with Y^T dY = 0 they move by d(X sigma)(X sigma)^T + transpose
    and by Y Wg Y^T + dY sigma^2 Y^T + transpose, Wg = (X sigma)^T d(X sigma) + transpose.
    """
    def sym(g):
        return g + g.transpose(2, 3, 0, 1)
    xs = x * sig
    s2 = sig * sig
    xsx = np.einsum("aijtg,bijtg->ab", xs, xs, optimize=True)
    dxsx = np.einsum("aijtg,bijtg->ab", dxs, xs, optimize=True)
    dxsx = dxsx + dxsx.T
    wg = np.einsum("aijtg,aijth->gh", xs, dxs, optimize=True)
    wg = wg + wg.T
    ysy = np.einsum("aijtg,g,bijtg->ab", y, s2, y, optimize=True)
    dysy = np.einsum("aijtg,g,bijtg->ab", dy, s2, y, optimize=True)
    dysy = dysy + dysy.T + np.einsum("aijtg,gh,bijth->ab", y, wg, y, optimize=True)
    dga = sym(np.einsum("xijta,ab,xkltb->ijkl", da, xsx, a, optimize=True)) + \
        np.einsum("xijta,ab,xkltb->ijkl", a, dxsx, a, optimize=True)
    dgx = sym(np.einsum("aijtg,akltg->ijkl", dxs, xs, optimize=True))
    dgy = sym(np.einsum("aijtg,g,akltg->ijkl", dy, s2, y, optimize=True)) + \
        np.einsum("aijtg,gh,aklth->ijkl", y, wg, y, optimize=True)
    dgd = sym(np.einsum("xijta,ab,xkltb->ijkl", ddm, ysy, dt, optimize=True)) + \
        np.einsum("xijta,ab,xkltb->ijkl", dt, dysy, dt, optimize=True)
    nn = a.shape[1] * a.shape[2]
    return [g.reshape(nn, nn) for g in (dga, dgx, dgy, dgd)]


ISO_GAP = 1e-12   # eigenvalue gaps (relative to the largest) below which a pair has no derivative


def _iso_tangent(gram, dgram, d1, d2, cap, prm):
    """dU of a truncated HOSVD isometry (trg.triad_isometry) along dgram, [d1, d2, cap]."""
    n = d1 * d2
    if n <= cap:
        return np.zeros((d1, d2, n))                 # identity: nothing truncated
    lam, w = trg.jacobi_eigh(gram)
    kept = trg.kept_count(lam, cap, prm.eps_lam, prm.tau_deg)
    u, wd = w[:, :kept], w[:, kept:]
    sg = trg.fix_signs(u, (d1, d2))
    gap = lam[None, :kept] - lam[kept:, None]
    ok = gap > ISO_GAP * lam[0]
    cm = np.where(ok, wd.T @ dgram @ u, 0.0) / np.where(ok, gap, 1.0)
    out = np.zeros((n, cap))
    out[:, :kept] = (wd @ cm) * sg
    return out.reshape(d1, d2, cap)


def step(ist, axis, prm, method, iso=True):
    """One coarse-graining step of the pure state and of every tangent.

    iso: differentiate the triad isometries (True) or hold them (False)."""
    kp = {}
    st = ist.pure
    d = st.d
    trg.rg_step(st, axis, prm, method, keep=kp)
    order = kp["order"]
    dims = kp["phi"].shape[:-1]
    inv = list(np.argsort(order)) + [d]
    new = []
    for dphi, dpsi in ist.tan:
        da, db, dcc, ddm = _resplit_tangent(kp, dphi, dpsi)
        da, db = trg._to_step_order(da, dims, order), trg._to_step_order(db, dims, order)
        dcc, ddm = trg._to_step_order(dcc, dims, order), trg._to_step_order(ddm, dims, order)
        dxs, dy = _bond_tangent(kp, db, dcc)
        if method == "triad":
            ti, tj, tk, tl = kp["ti"], kp["tj"], kp["tk"], kp["tl"]
            m1, m2, m3 = kp["m"]
            n1, n2, n3 = kp["n"]
            de = np.einsum("xijta,ijk->xkta", da, ti, optimize=True)      # E = A U^A
            df = np.einsum("aijtg,ijk->aktg", dxs, tj, optimize=True)     # F = (X sigma) U^X
            dg = np.einsum("bijtg,ijk->bktg", dy, tk, optimize=True)      # G = Y U^Y
            dh = np.einsum("xijtb,ijk->xktb", ddm, tl, optimize=True)     # H = D U^D
            dphi_n = trg.make_phi(de, kp["f"], ti, tj, m1, m2, m3) + trg.make_phi(kp["e"], df, ti, tj, m1, m2, m3)
            dpsi_n = trg.make_psi(dg, kp["h"], tk, tl, n1, n2, n3) + trg.make_psi(kp["g"], dh, tk, tl, n1, n2, n3)
            if iso:
                a, x, sig, y, dt = kp["a"], kp["x"], kp["sig"], kp["y"], kp["dd"]
                d1, d2, cap = ti.shape
                grams = trg.triad_grams(a, x, sig, y, dt)
                dgr = _gram_tangents(a, x, sig, y, dt, da, dxs, dy, ddm)
                dti, dtj, dtk, dtl = (_iso_tangent(gm, dgm, d1, d2, cap, prm) for gm, dgm in zip(grams, dgr))
                de2 = np.einsum("xijta,ijk->xkta", a, dti, optimize=True)
                df2 = np.einsum("aijtg,ijk,g->aktg", x, dtj, sig, optimize=True)
                dg2 = np.einsum("bijtg,ijk->bktg", y, dtk, optimize=True)
                dh2 = np.einsum("xijtb,ijk->xktb", dt, dtl, optimize=True)
                e, f, g, h = kp["e"], kp["f"], kp["g"], kp["h"]
                dphi_n = dphi_n + trg.make_phi(de2, f, ti, tj, m1, m2, m3) + trg.make_phi(e, df2, ti, tj, m1, m2, m3) \
                    + trg.make_phi(e, f, dti, tj, m1, m2, m3) + trg.make_phi(e, f, ti, dtj, m1, m2, m3)
                dpsi_n = dpsi_n + trg.make_psi(dg2, h, tk, tl, n1, n2, n3) + trg.make_psi(g, dh2, tk, tl, n1, n2, n3) \
                    + trg.make_psi(g, h, dtk, tl, n1, n2, n3) + trg.make_psi(g, h, tk, dtl, n1, n2, n3)
        else:
            dphi_n, dpsi_n = _atrg_tangent(kp, da, dxs, dy, ddm)
        new.append((np.ascontiguousarray(np.transpose(dphi_n, inv)),
                    np.ascontiguousarray(np.transpose(dpsi_n, inv))))
    ist.tan = new
    return ist


def _atrg_tangent(kp, da, dxs, dy, ddm):
    """makeG / makeH with one factor replaced by its tangent (ATRG, Sec. II A)."""
    a, x, sig, y, dt = kp["a"], kp["x"], kp["sig"], kp["y"], kp["dd"]
    es, fs = kp["es"], kp["fs"]
    nd = a.ndim - 1
    xs = x * sig
    ia, al, g = 0, 1, 2
    tl = [10 + p for p in range(nd - 1)]
    bl = [20 + p for p in range(nd - 1)]
    kl = [30 + p for p in range(nd - 1)]
    ja, be = 3, 4

    def make_g(at, xt):
        return trg._chain([(at, [ia] + tl + [al]), (es[0], [tl[0], bl[0], kl[0]]), (xt, [al] + bl + [g])]
                          + [(es[p], [tl[p], bl[p], kl[p]]) for p in range(1, nd - 1)], [ia] + kl + [g])

    def make_h(dtt, yt):
        return trg._chain([(dtt, [ja] + bl + [be]), (fs[0], [tl[0], bl[0], kl[0]]), (yt, [be] + tl + [g])]
                          + [(fs[p], [tl[p], bl[p], kl[p]]) for p in range(1, nd - 1)], [ja] + kl + [g])
    return make_g(da, xs) + make_g(a, dxs), make_h(ddm, y) + make_h(dt, dy)


def derivatives(ist):
    """d(log Z/V)/d(theta) for each tangent: 2^-n Tr(dT) / Tr(T)."""
    st = ist.pure
    tr = float(np.sum(st.phi * st.psi))
    out = []
    for dphi, dpsi in ist.tan:
        dtr = float(np.sum(dphi * st.psi) + np.sum(st.phi * dpsi))
        out.append(2.0 ** (-st.k) * dtr / tr)
    return out


def run(beta, h, prm, nsteps, method="triad", d=4, wrt=("beta", "h"), iso=True):
    ist = ImpurityState(beta, h, d, wrt)
    for i in range(nsteps):
        step(ist, i % d, prm, method, iso)
    return derivatives(ist), ist
