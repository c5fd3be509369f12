"""ATRG and triad-ATRG RG steps in FP64 (test infrastructure only).

State.  The coarse tensor after k steps is kept as a pair (Phi, Psi) with
    T[f_0..f_{d-1}; b_0..b_{d-1}] = sum_g Phi[f_0..f_{d-1}, g] Psi[b_0..b_{d-1}, g],
f_mu the forward leg along axis mu (i_mu(n)), b_mu the backward leg
(j_mu(n)), both of dim dims[mu], legs in natural axis order.  The Ising
tensor in CP form is the initial state.

One step along axis a (Sec. II A-B, Fig. 5), transverse axes
(t_1, .., t_{d-1}) = (a+1, .., a+d-1) mod d:
 1. re-split (Fig. 5f): T = Phi Psi^T has rank <= chi, so QR(Phi), QR(Psi) and
    the SVD of R_Phi R_Psi^T give T = A B^T = C D^T exactly (eq. ABCD), with A,
    D isometric, B = D-side vectors times s, C = A times s.  The largest
    singular value c_k normalises T and log Z/V accumulates 2^-k log c_k.
 2. bond swap (eq. of the bond swap; App. A): the truncated SVD of
    sum_{i_a(n)} B C = X sigma Y, exact or by the randomized SVD of App. A.
 3. ATRG: squeezers from the canonical Gamma^ATRG and makeG / makeH; or
    triad-ATRG (d = 4): triad isometries from the truncated HOSVD of
    Gamma^ATRG (eq. HOSVD), the triad tensors E..L, squeezers from
    Gamma^Triad with the Gram matrices O and P, and makeMG / makeMH.
 4. The new (Phi, Psi) = (G, H) or (Phi, Psi) of makeMG / makeMH.

Squeezers (the oblique projector pair of the papers cited in Sec. II A):
with K_f the Gram of the unit cell over every leg except the forward pair
(i_mu(n+a), i_mu(n)) and K_b that of the next cell over every leg except the
backward pair (j_mu(n+a), j_mu(n)), R_f^T R_f = K_f, R_b^T R_b = K_b, and
R_f R_b^T = U S V^T truncated to D:  E = R_b^T V S^-1/2 acts on the forward
pair, F = R_f^T U S^-1/2 on the backward pair.  Pairs are ordered
(top-site leg, bottom-site leg) on both sides.

Readings where the paper is silent are listed in the design notes and in
the docstrings below (sign convention, truncation rule, sketch layout,
power-iteration count).
"""
from dataclasses import dataclass, field
import math

import numpy as np

from .linalg import qr_pos, jacobi_eigh, jacobi_svd, kept_count, fix_signs, canonical_rotation
from .philox import sketch_omega
from .ising import ising_cp


@dataclass
class Params:
    D: int
    r: int = 7
    sketch_mult: int = 2          # sketch width m = sketch_mult * D (App. A footnote: eta = r_bond + 1)
    r_bond: int = 1               # bond-swap overspanning (Sec. II C): keep r_bond * D bond values
    power_iters: int = 1
    seed: int = 0
    instance: int = 0
    bond_svd: str = "sketch"      # "sketch" (App. A) or "exact"
    eps_s: float = 1e-14          # singular values <= eps_s * top are zero
    eps_lam: float = 1e-14        # Gram eigenvalues <= eps_lam * top are zero
    tau_deg: float = 1e-9         # multiplet width (relative to the largest value)
    eps_sq: float = 1e-14         # squeezer singular values <= eps_sq * top are dropped


@dataclass
class State:
    d: int
    phi: np.ndarray
    psi: np.ndarray
    k: int = 0
    logacc: float = 0.0
    nsteps_axis: list = field(default_factory=list)
    log: list = field(default_factory=list)

    @property
    def dims(self):
        return tuple(self.phi.shape[:-1])


def init_ising(beta, h, d=4):
    phi, psi = ising_cp(beta, h, d)
    return State(d=d, phi=phi, psi=psi, nsteps_axis=[0] * d)


# ----------------------------------------------------------------------------
# step pieces
# ----------------------------------------------------------------------------

def resplit(phi, psi, eps_s, tau_deg=1e-9, keep=None):
    """Exact SVD of T = Phi Psi^T through two QRs and a small SVD.

    Returns (A, B, C, Dm, c, s) as matrices with rows = legs in natural order:
    T / c = A B^T = C Dm^T with A and Dm isometric on the kept columns.  The
    bond basis is canonical: within each multiplet of singular values the
    columns of A (and Dm) are rotated by the canonical rotation R, and
    B = Dm S', C = A S' with S' = R^T diag(s) R.  Columns whose singular value
    is <= eps_s are zero in all four.  ``keep`` (a dict), if given, receives
    the canonical rotation R.
    """
    dims = phi.shape[:-1]
    f = int(np.prod(dims))
    q1, r1 = qr_pos(phi.reshape(f, -1))
    q2, r2 = qr_pos(psi.reshape(f, -1))
    u, s, v = jacobi_svd(r1 @ r2.T)
    c = s[0]
    if not (c > 0 and np.isfinite(c)):
        raise FloatingPointError("re-split: non-positive or non-finite norm %r" % c)
    s = s / c
    s = np.where(s > eps_s, s, 0.0)
    k = int(np.count_nonzero(s))
    a = q1 @ u
    dm = q2 @ v
    rot = np.eye(len(s))
    rot[:k, :k] = canonical_rotation(a[:, :k], s, k, dims, tau_deg)
    a = a @ rot
    dm = dm @ rot
    a[:, k:] = 0.0
    dm[:, k:] = 0.0
    sp = rot.T @ np.diag(s) @ rot
    if keep is not None:
        keep["rot"] = rot
    return a, dm @ sp, a @ sp, dm, c, s


def _to_step_order(mat, dims, order):
    """Matrix with rows = natural-order legs -> tensor [legs in ``order``, col]."""
    t = mat.reshape(tuple(dims) + (mat.shape[1],))
    return np.transpose(t, list(order) + [len(dims)])


def bond_swap(bt, ct, prm, step, logrec):
    """Truncated SVD of M[(alpha, i_perp), (beta, j_perp)] = sum_x B[x, j_perp, alpha] C[x, i_perp, beta].

    ``bt`` = B[x, j_t.., alpha] (top site, x = j_a(n+a) = i_a(n)),
    ``ct`` = C[x, i_t.., beta]  (bottom site).
    Follows App. A: QR of B over (j_perp) x (x, alpha) and of C, the core
    N[(alpha, q), (beta, p)] = sum_x R^B[p, x, alpha] R^C[q, x, beta], then
    either the exact SVD of N or the randomized loop of App. A with q_loop =
    power_iters + 1 passes.  The Gaussian sketch is drawn in the (beta, j_perp)
    index space of M and projected on the QR basis of B.
    Returns X[alpha, i_t.., g], sigma[g], Y[beta, j_t.., g] with g padded to
    min(r_bond D, rows(N), cols(N)): with r_bond > 1 the bond is overspanned
    (ILO triad-ATRG, Sec. II C), and the next step's alpha and beta carry
    r_bond D values through the re-split.
    """
    xdim = bt.shape[0]
    chia = bt.shape[-1]
    chib = ct.shape[-1]
    jdims = bt.shape[1:-1]
    idims = ct.shape[1:-1]
    jn = int(np.prod(jdims))
    inn = int(np.prod(idims))
    bm = np.moveaxis(bt, 0, -2).reshape(jn, xdim * chia)
    cm = np.moveaxis(ct, 0, -2).reshape(inn, xdim * chib)
    qb, rb = qr_pos(bm)
    qc, rc = qr_pos(cm)
    p = rb.shape[0]
    q = rc.shape[0]
    rb3 = rb.reshape(p, xdim, chia)
    rc3 = rc.reshape(q, xdim, chib)
    rows, cols = chia * q, chib * p
    gcap = min(prm.r_bond * prm.D, rows, cols)
    m = prm.sketch_mult * prm.D
    if prm.bond_svd == "exact" or m >= min(rows, cols):
        n = np.einsum("pxa,qxb->aqbp", rb3, rc3).reshape(rows, cols)
        ub, sig, vb = jacobi_svd(n)
        mode = "exact"
    else:
        # the core is never formed: eq. bond1 applies R^B to the sketch, then
        # R^C; eq. bond2 applies R^C to Q, then R^B
        def apply_n(om):
            t = np.einsum("pxa,bpm->xabm", rb3, om.reshape(chib, p, -1), optimize=True)
            return np.einsum("qxb,xabm->aqm", rc3, t, optimize=True).reshape(rows, -1)

        def apply_nt(qm):
            t = np.einsum("qxb,aqm->xabm", rc3, qm.reshape(chia, q, -1), optimize=True)
            return np.einsum("pxa,xabm->bpm", rb3, t, optimize=True).reshape(cols, -1)

        om_full = sketch_omega(prm.seed, step, prm.instance, chib, jdims, m)
        om = np.einsum("jp,bjm->bpm", qb, om_full.reshape(chib, jn, m)).reshape(chib * p, m)
        qy = None
        rp = None
        for _ in range(prm.power_iters + 1):
            y = apply_n(om)
            qy, _r = qr_pos(y)
            yt = apply_nt(qy)
            qp, rp = qr_pos(yt)
            om = qp
        ut, sig, w = jacobi_svd(rp.T)
        ub = qy @ ut
        vb = om @ w
        mode = "sketch"
    kept = kept_count(sig, gcap, prm.eps_s, prm.tau_deg)
    logrec["bond"] = dict(mode=mode, kept=kept, cap=gcap, sig=sig[: gcap + 1].copy(),
                          gap=_gap(sig, kept, gcap))
    ub = ub[:, :kept]
    vb = vb[:, :kept]
    sigk = sig[:kept]
    x = np.einsum("aqg,iq->aig", ub.reshape(chia, q, kept), qc)
    y = np.einsum("bpg,jp->bjg", vb.reshape(chib, p, kept), qb)
    sg = fix_signs(x.reshape(chia * inn, kept), (chia,) + tuple(idims))
    x = x * sg
    y = y * sg
    xo = np.zeros((chia, inn, gcap))
    yo = np.zeros((chib, jn, gcap))
    so = np.zeros(gcap)
    xo[:, :, :kept] = x
    yo[:, :, :kept] = y
    so[:kept] = sigk
    return (xo.reshape((chia,) + tuple(idims) + (gcap,)), so,
            yo.reshape((chib,) + tuple(jdims) + (gcap,)))


def _gap(vals, kept, cap):
    if kept < len(vals) and kept > 0 and vals[0] > 0:
        return float((vals[kept - 1] - vals[kept]) / vals[0])
    return None


def _partial_gram(t, pos, penv=None, env_axis=None):
    """Z[c, x, c', x'] = sum over the other legs of t[.., x, .., c] t[.., x', .., c'].

    ``pos`` is the axis of t kept open as x, c is the last axis (the bond to
    the other half of the cell).  If ``penv`` is given, axis ``env_axis`` of
    t is contracted through it: t[.., g] penv[g, g'] t[.., g'], and the open
    bond c is then axis 0.
    """
    nd = t.ndim
    if penv is None:
        cax = nd - 1
        a1 = list(range(nd))
        a2 = list(range(nd))
        a2[pos] = 40
        a2[cax] = 41
        return np.einsum(t, a1, t, a2, [cax, pos, 41, 40], optimize=True)
    cax = 0
    tp = np.tensordot(t, penv, axes=([env_axis], [0]))
    tp = np.moveaxis(tp, -1, env_axis)
    a1 = list(range(nd))
    a2 = list(range(nd))
    a2[pos] = 40
    a2[cax] = 41
    return np.einsum(tp, a1, t, a2, [cax, pos, 41, 40], optimize=True)


def env_grams(top_f, bot_f, penv, top_b, bot_b, oenv, pos):
    """K_f and K_b of the squeezer along transverse position ``pos`` (0-based).

    Upper half of the cell = top_f[i_a, t.., alpha] bot_f[alpha, b.., g] (g
    closed through the lower-half Gram ``penv``); lower half =
    top_b[beta, t.., g] bot_b[j_a, b.., beta] (g closed through ``oenv``).
    K_f[(t, b), (t', b')] and K_b[(t, b), (t', b')] as matrices.
    """
    zt = _partial_gram(top_f, pos + 1)                              # [a, t, a', t']
    zb = _partial_gram(bot_f, pos + 1, penv, bot_f.ndim - 1)        # [a, b, a', b']
    kf = np.einsum("atcu,abcd->tbud", zt, zb, optimize=True)
    zy = _partial_gram(top_b, pos + 1, oenv, top_b.ndim - 1)        # [b, t, b', t']
    zd = _partial_gram(bot_b, pos + 1)                              # [b, x, b', x']
    kb = np.einsum("btcu,bxcy->txuy", zy, zd, optimize=True)
    dt = kf.shape[0]
    db = kf.shape[1]
    return kf.reshape(dt * db, dt * db), kb.reshape(dt * db, dt * db)


def sqrt_psd(k, eps_lam):
    """R with R^T R = K from the Jacobi eigen-decomposition; eigenvalues <= eps_lam*top -> 0."""
    lam, w = jacobi_eigh(k)
    top = lam[0] if lam[0] > 0 else 0.0
    lam = np.where(lam > eps_lam * top, lam, 0.0)
    return np.sqrt(lam)[:, None] * w.T


def squeezer(kf, kb, dt, db, prm, name, logrec):
    """Projector pair (E on the forward pair, F on the backward pair), [dt, db, k]."""
    npair = dt * db
    if npair <= prm.D:
        e = np.eye(npair).reshape(dt, db, npair)
        logrec[name] = dict(identity=True)
        return e, e.copy()
    rf = sqrt_psd(kf, prm.eps_lam)
    rb = sqrt_psd(kb, prm.eps_lam)
    u, s, v = jacobi_svd(rf @ rb.T)
    kept = kept_count(s, prm.D, prm.eps_sq, prm.tau_deg)
    logrec[name] = dict(kept=kept, s=s[: prm.D + 1] / (s[0] if s[0] > 0 else 1.0),
                        gap=_gap(s, kept, prm.D))
    isq = 1.0 / np.sqrt(s[:kept])
    e = rb.T @ v[:, :kept] * isq[None, :]
    f = rf.T @ u[:, :kept] * isq[None, :]
    rot = canonical_rotation(e, s, kept, (dt, db), prm.tau_deg)
    e = e @ rot
    f = f @ rot
    eo = np.zeros((npair, prm.D))
    fo = np.zeros((npair, prm.D))
    eo[:, :kept] = e
    fo[:, :kept] = f
    return eo.reshape(dt, db, prm.D), fo.reshape(dt, db, prm.D)


def atrg_coarse(a, x, sig, y, dt, prm, logrec, keep=None):
    """ATRG coarse-graining (makeG / makeH) with squeezers from canonical Gamma^ATRG.

    a[i_a, t.., alpha], x[alpha, b.., g], y[beta, t.., g], dt[j_a, b.., beta].
    Canonical form: the lower half is isometric (P = 1) and the upper half
    has Gram O = diag(sigma^2).
    """
    d = a.ndim - 1
    xs = x * sig
    ng = sig.shape[0]
    penv = np.eye(ng)
    oenv = np.diag(sig * sig)
    es, fs = [], []
    for pos in range(d - 1):
        dtr = a.shape[pos + 1]
        dbr = x.shape[pos + 1]
        if dtr * dbr <= prm.D:
            e, f = squeezer(None, None, dtr, dbr, prm, "sq%d" % pos, logrec)
        else:
            kf, kb = env_grams(a, xs, penv, y, dt, oenv, pos)
            e, f = squeezer(kf, kb, dtr, dbr, prm, "sq%d" % pos, logrec)
        es.append(e)
        fs.append(f)
    # makeG: G[i_a, k.., g] = sum A X sigma prod E, as a chain of pairwise contractions
    ia, al, g = 0, 1, 2
    tl = [10 + p for p in range(d - 1)]
    bl = [20 + p for p in range(d - 1)]
    kl = [30 + p for p in range(d - 1)]
    gnew = _chain([(a, [ia] + tl + [al]), (es[0], [tl[0], bl[0], kl[0]]), (xs, [al] + bl + [g])]
                  + [(es[p], [tl[p], bl[p], kl[p]]) for p in range(1, d - 1)], [ia] + kl + [g])
    # makeH: H[j_a, k'.., g] = sum D Y prod F
    ja, be = 3, 4
    hnew = _chain([(dt, [ja] + bl + [be]), (fs[0], [tl[0], bl[0], kl[0]]), (y, [be] + tl + [g])]
                  + [(fs[p], [tl[p], bl[p], kl[p]]) for p in range(1, d - 1)], [ja] + kl + [g])
    if keep is not None:
        keep.update(es=es, fs=fs)
    return gnew, hnew


def _chain(ops, out):
    """Contract (tensor, labels) operands left to right, pairwise (BLAS), into labels ``out``."""
    cur, lab = ops[0]
    for t, lt in ops[1:]:
        keep = [x for x in lab if x not in lt or x in out] + [x for x in lt if x not in lab]
        cur = np.einsum(cur, lab, t, lt, keep, optimize=True)
        lab = keep
    return np.einsum(cur, lab, out)


def triad_isometry(gram, d1, d2, cap, prm, name, logrec):
    """Truncated HOSVD isometry U[(t1, t2), k] of a pair Gram (eq. HOSVD)."""
    n = d1 * d2
    if n <= cap:
        logrec[name] = dict(identity=True)
        return np.eye(n)
    lam, w = jacobi_eigh(gram)
    kept = kept_count(lam, cap, prm.eps_lam, prm.tau_deg)
    logrec[name] = dict(kept=kept, cap=cap, gap=_gap(lam, kept, cap))
    u = w[:, :kept]
    u = u * fix_signs(u, (d1, d2))
    out = np.zeros((n, cap))
    out[:, :kept] = u
    return out


def triad_grams(a, x, sig, y, dt):
    """Pair Grams of canonical Gamma^ATRG for the triad isometries (eq. HOSVD).

    G_A[(t1,t2),(t1',t2')] = sum A[.., t1, t2, .., a] (X s^2 X^T)[a, a'] A[.., t1', t2', .., a']
    (the lower half is isometric, A is the only other factor on its legs);
    G_X = sum X s^2 X over (alpha, t3, g); G_Y likewise; G_D with (Y s^2 Y^T).
    """
    s2 = sig * sig
    xsx = np.einsum("aijtg,g,bijtg->ab", x, s2, x, optimize=True)
    ysy = np.einsum("aijtg,g,bijtg->ab", y, s2, y, optimize=True)
    ga = np.einsum("xijta,ab,xkltb->ijkl", a, xsx, a, optimize=True)
    gx = np.einsum("aijtg,g,akltg->ijkl", x, s2, x, optimize=True)
    gy = np.einsum("aijtg,g,akltg->ijkl", y, s2, y, optimize=True)
    gd = np.einsum("xijta,ab,xkltb->ijkl", dt, ysy, dt, optimize=True)
    nn = a.shape[1] * a.shape[2]
    return [g.reshape(nn, nn) for g in (ga, gx, gy, gd)]


def make_phi(e, f, ti, tj, m1, m2, m3):
    """makeMG: Phi[i_a, k1, k2, k3, g] = (E F M3)(I J M1 M2), contracted over kA, kX."""
    efm = np.einsum("xAta,aXsg,tsc->xAXcg", e, f, m3, optimize=True)
    ijmm = np.einsum("ijA,pqX,ipk,jql->AXkl", ti, tj, m1, m2, optimize=True)
    return np.einsum("xAXcg,AXkl->xklcg", efm, ijmm, optimize=True)


def make_psi(g, h, tk, tl, n1, n2, n3):
    """makeMH: Psi[j_a, k1', k2', k3', g] = (G H N3)(K L N1 N2), contracted over kY, kD."""
    ghn = np.einsum("bYtg,xDsb,tsc->xYDcg", g, h, n3, optimize=True)
    klnn = np.einsum("ijY,pqD,ipk,jql->YDkl", tk, tl, n1, n2, optimize=True)
    return np.einsum("xYDcg,YDkl->xklcg", ghn, klnn, optimize=True)


def triad_coarse(a, x, sig, y, dt, prm, logrec, keep=None):
    """Triad-ATRG coarse-graining (Sec. II B), d = 4.

    a[i_a, t1, t2, t3, alpha], x[alpha, t1, t2, t3, g], y[beta, t1, t2, t3, g],
    dt[j_a, t1, t2, t3, beta]; t1, t2 are bundled into triads, t3 stays on the
    four-leg tensors.
    """
    d1, d2, d3 = a.shape[1], a.shape[2], a.shape[3]
    rcap = min(prm.r * prm.D, d1 * d2)
    ga, gx, gy, gd = triad_grams(a, x, sig, y, dt)
    ua = triad_isometry(ga, d1, d2, rcap, prm, "UA", logrec)
    ux = triad_isometry(gx, d1, d2, rcap, prm, "UX", logrec)
    uy = triad_isometry(gy, d1, d2, rcap, prm, "UY", logrec)
    ud = triad_isometry(gd, d1, d2, rcap, prm, "UD", logrec)
    # triad tensors E..L (eqs. for E, F, G, H, I, J, K, L)
    ti = ua.reshape(d1, d2, -1)
    tj = ux.reshape(d1, d2, -1)
    tk = uy.reshape(d1, d2, -1)
    tl = ud.reshape(d1, d2, -1)
    e = np.einsum("xijta,ijk->xkta", a, ti, optimize=True)          # E[i_a, kA, t3, alpha]
    f = np.einsum("aijtg,ijk,g->aktg", x, tj, sig, optimize=True)   # F[alpha, kX, t3, g]
    g = np.einsum("bijtg,ijk->bktg", y, tk, optimize=True)          # G[beta, kY, t3, g]
    h = np.einsum("xijtb,ijk->xktb", dt, tl, optimize=True)         # H[j_a, kD, t3, beta]
    # Gram matrices of the upper (E, F, I, J) and lower (G, H, K, L) blocks
    ee = np.einsum("xkta,xktb->ab", e, e, optimize=True)
    o = np.einsum("ab,aktg,bkth->gh", ee, f, f, optimize=True)
    hh = np.einsum("xktb,xktc->bc", h, h, optimize=True)
    p = np.einsum("bc,bktg,ckth->gh", hh, g, g, optimize=True)
    # Gamma^Triad with the triad bonds contracted: projected A, X sigma, Y, D
    at = np.einsum("xkta,ijk->xijta", e, ti, optimize=True)
    xt = np.einsum("aktg,ijk->aijtg", f, tj, optimize=True)
    yt = np.einsum("bktg,ijk->bijtg", g, tk, optimize=True)
    dtt = np.einsum("xktb,ijk->xijtb", h, tl, optimize=True)
    sq = []
    for pos, dd in enumerate((d1, d2, d3)):
        if dd * dd <= prm.D:
            mm, nm = squeezer(None, None, dd, dd, prm, "sq%d" % pos, logrec)
        else:
            kf, kb = env_grams(at, xt, p, yt, dtt, o, pos)
            mm, nm = squeezer(kf, kb, dd, dd, prm, "sq%d" % pos, logrec)
        sq.append((mm, nm))
    (m1, n1), (m2, n2), (m3, n3) = sq
    phi = make_phi(e, f, ti, tj, m1, m2, m3)
    psi = make_psi(g, h, tk, tl, n1, n2, n3)
    if keep is not None:
        keep.update(e=e, f=f, g=g, h=h, ti=ti, tj=tj, tk=tk, tl=tl, m=(m1, m2, m3), n=(n1, n2, n3))
    return phi, psi


def rg_step(state, axis, prm, method, keep=None):
    """One coarse-graining step along ``axis`` ("atrg" or "triad").

    ``keep`` (a dict), if given, receives the step's inputs, its re-split, bond
    swap, isometries and squeezers (the impurity method reuses them)."""
    d = state.d
    if not 0 <= axis < d:
        raise ValueError("axis out of range")
    if method == "triad" and d != 4:
        raise ValueError("triad-ATRG is defined for d = 4")
    order = [axis] + [(axis + i) % d for i in range(1, d)]
    rec = dict(step=state.k, axis=axis, method=method)
    if keep is not None:
        keep.update(phi=state.phi, psi=state.psi, order=order, k=state.k)
    am, bm, cm, dm, c, s = resplit(state.phi, state.psi, prm.eps_s, prm.tau_deg, keep)
    state.logacc += 2.0 ** (-state.k) * math.log(c)
    rec["c"] = c
    rec["s"] = s.copy()
    dims = state.dims
    a = _to_step_order(am, dims, order)
    b = _to_step_order(bm, dims, order)
    cc = _to_step_order(cm, dims, order)
    dd = _to_step_order(dm, dims, order)
    x, sig, y = bond_swap(b, cc, prm, state.k, rec)
    if keep is not None:
        keep.update(am=am, dm=dm, c=c, s=s, a=a, b=b, cc=cc, dd=dd, x=x, sig=sig, y=y)
    if method == "atrg":
        gnew, hnew = atrg_coarse(a, x, sig, y, dd, prm, rec, keep)
    else:
        gnew, hnew = triad_coarse(a, x, sig, y, dd, prm, rec, keep)
    inv = list(np.argsort(order)) + [d]
    state.phi = np.ascontiguousarray(np.transpose(gnew, inv))
    state.psi = np.ascontiguousarray(np.transpose(hnew, inv))
    state.k += 1
    state.nsteps_axis[axis] += 1
    state.log.append(rec)
    return state


def trace(state):
    """tTr of the single coarse tensor: sum_I sum_g Phi[I, g] Psi[I, g]."""
    return float(np.sum(state.phi * state.psi))


def log_z_per_site(state):
    tr = trace(state)
    if not (tr > 0 and np.isfinite(tr)):
        raise FloatingPointError("final trace %r is not positive" % tr)
    return state.logacc + 2.0 ** (-state.k) * math.log(tr)


def gu_wen_matrix(state, axis):
    """A[k, l] = sum of T over every leg pair but ``axis`` traced (forward leg =
    backward leg), with k the forward and l the backward leg along ``axis``
    (Sec. III D, the matrix of the dimensionless ratio X).  With
    T = sum_g Phi[.., g] Psi[.., g]: A = sum_{I, g} Phi[I_k, g] Psi[I_l, g]."""
    n = state.phi.shape[axis]
    phi = np.moveaxis(state.phi, axis, 0).reshape(n, -1)
    psi = np.moveaxis(state.psi, axis, 0).reshape(n, -1)
    return phi @ psi.T


def gu_wen_x(state, axis=None):
    """X = (Tr A)^2 / Tr(A A) of the current coarse tensor (Sec. III D); the
    paper's A keeps the fourth leg open, which is the default axis d - 1.
    X is 1 for a tensor of rank one along ``axis`` (disordered phase) and 2 for
    two degenerate ground states (ordered phase)."""
    if axis is None:
        axis = state.d - 1
    if not 0 <= axis < state.d:
        raise ValueError("axis out of range")
    a = gu_wen_matrix(state, axis)
    return float(np.trace(a) ** 2 / np.trace(a @ a))


def run(beta, h, prm, nsteps, method="triad", d=4, start_axis=0):
    """Cycle the axes start_axis, start_axis+1, .. for ``nsteps`` steps; return (log Z/V, state)."""
    st = init_ising(beta, h, d)
    for i in range(nsteps):
        rg_step(st, (start_axis + i) % d, prm, method)
    return log_z_per_site(st), st
