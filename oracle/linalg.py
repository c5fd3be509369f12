"""Dense FP64 linear algebra of the oracle (test infrastructure only).

* ``qr_pos``      thin Householder QR (LAPACK ``dgeqrf`` through numpy, used as
                  a library primitive) normalised to a non-negative diagonal of R.
* ``jacobi_eigh`` the oracle's own cyclic two-sided Jacobi eigensolver for
                  symmetric matrices (Rutishauser's rotation formulas).
* ``jacobi_svd``  the oracle's own one-sided (Hestenes) Jacobi SVD.
* ``kept_count``  the truncation rule shared by every truncated decomposition
                  of the method: keep at most ``cap`` values, drop values at or
                  below ``eps_rel`` times the largest, and never cut through a
                  multiplet (values closer than ``tau_deg`` times the largest are
                  kept or dropped together).
* ``sign_weights`` / ``fix_signs``  the sign convention that fixes the basis
                  of every kept singular/eigen vector: column j is flipped so
                  that sum_i w(i) Q[i, j] > 0, with w a fixed irregular weight of
                  the multi-index of the row.
* ``canonical_rotation``  the same convention for a multiplet of d nearly
                  equal values: the columns of the multiplet are rotated to
                  Q_m Q_z, Q_z the Q factor (diag R > 0) of Z = Q_m^T W_d with d
                  fixed weight vectors w_0..w_{d-1}; the result depends only on
                  the subspace the multiplet spans (for d = 1 it is the sign
                  convention).

Both Jacobi routines (their loops are in ``jacobi.c``) process the disjoint
index pairs of a round-robin schedule simultaneously; this is the textbook
parallel ordering and changes nothing about what is computed.
"""
import numpy as np

EPS = np.finfo(np.float64).eps
GOLDEN = 0.6180339887498949
SQRT2M1 = 0.41421356237309515
RADIX = 131


def qr_pos(a):
    """Thin QR, a = q r with q (m x k), r (k x n), k = min(m, n), diag(r) >= 0."""
    a = np.asarray(a, dtype=np.float64)
    q, r = np.linalg.qr(a, mode="reduced")
    d = np.sign(np.diagonal(r)).copy()
    d[d == 0] = 1.0
    return q * d[None, :], r * d[:, None]


_LIB = None


def _lib():
    """The oracle's C Jacobi kernels (oracle/jacobi.c), compiled with gcc on first use."""
    global _LIB
    if _LIB is None:
        import ctypes
        import os
        import subprocess
        here = os.path.dirname(os.path.abspath(__file__))
        so = os.path.join(here, "libjacobi.so")
        src = os.path.join(here, "jacobi.c")
        if not os.path.exists(so) or os.path.getmtime(so) < os.path.getmtime(src):
            subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", so, src, "-lm"])
        lib = ctypes.CDLL(so)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_jacobi_eigh.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int]
        lib.oracle_jacobi_eigh.restype = ctypes.c_int
        lib.oracle_jacobi_svd.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, ctypes.c_int]
        lib.oracle_jacobi_svd.restype = ctypes.c_int
        _LIB = lib
    return _LIB


def _ptr(x):
    import ctypes
    return x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def jacobi_eigh(k, max_sweeps=80):
    """Eigen-decomposition of a symmetric matrix by cyclic two-sided Jacobi.

    Returns (lam, v) with lam sorted descending and k = v diag(lam) v^T.
    A rotation of pair (p, q) is skipped when |a_pq| <= n eps sqrt|a_pp| sqrt|a_qq|;
    the iteration stops after the first sweep that performs no rotation.
    """
    a = np.array(k, dtype=np.float64, order="C", copy=True)
    n = a.shape[0]
    scale = float(np.max(np.abs(a))) if a.size else 0.0
    if scale > 0:
        a /= scale
    v = np.empty((n, n), dtype=np.float64)
    rc = _lib().oracle_jacobi_eigh(n, _ptr(a), _ptr(v), max_sweeps)
    if rc < 0:
        raise RuntimeError("jacobi_eigh: no convergence in %d sweeps" % max_sweeps)
    lam = np.diagonal(a).copy() * (scale if scale > 0 else 1.0)
    order = np.argsort(-lam, kind="stable")
    return lam[order], v[:, order]


def jacobi_svd(a, max_sweeps=80):
    """Thin SVD a = u diag(s) v^T by one-sided (Hestenes) Jacobi.

    u (m x k), s (k,) descending, v (n x k), k = min(m, n).  A pair (p, q) is
    rotated while |u_p . u_q| > sqrt(m) eps |u_p| |u_q| (the tolerance of
    LAPACK's dgesvj).  Columns of u belonging to zero singular values are
    returned as zero vectors.
    """
    a = np.asarray(a, dtype=np.float64)
    m, n = a.shape
    if m < n:
        ut, s, vt = jacobi_svd(a.T, max_sweeps)
        return vt, s, ut
    ut = np.array(a.T, dtype=np.float64, order="C", copy=True)
    scale = float(np.max(np.abs(ut))) if ut.size else 0.0
    if scale > 0:
        ut /= scale
    vt = np.empty((n, n), dtype=np.float64)
    rc = _lib().oracle_jacobi_svd(m, n, _ptr(ut), _ptr(vt), max_sweeps)
    if rc < 0:
        raise RuntimeError("jacobi_svd: no convergence in %d sweeps" % max_sweeps)
    u = ut.T
    v = vt.T
    s = np.sqrt(np.einsum("ij,ij->j", u, u))
    order = np.argsort(-s, kind="stable")
    s = s[order]
    u = u[:, order]
    v = v[:, order]
    nz = s > 0
    u[:, nz] = u[:, nz] / s[nz][None, :]
    u[:, ~nz] = 0.0
    return np.ascontiguousarray(u), s * (scale if scale > 0 else 1.0), np.ascontiguousarray(v)


def kept_count(vals, cap, eps_rel, tau_deg):
    """Number of leading values kept by a truncation (vals sorted descending).

    At most ``cap``; none at or below ``eps_rel * vals[0]``; and if the cut
    would separate two values closer than ``tau_deg * vals[0]`` the whole
    multiplet at the cut is dropped.
    """
    vals = np.asarray(vals, dtype=np.float64)
    if vals.size == 0 or not vals[0] > 0:
        return 0
    top = vals[0]
    nz = int(np.count_nonzero(vals > eps_rel * top))
    k = min(cap, nz)
    if k < nz:
        while k > 0 and (vals[k - 1] - vals[k]) <= tau_deg * top:
            k -= 1
    return k


def sign_weights(dims):
    """Weight w of every multi-index of a row space with leg dims ``dims``.

    w(i_0, ..., i_{n-1}) = 0.5 + frac(g * (1 + sum_l i_l * 131^l)), g the
    golden-ratio conjugate.  Defined on the multi-index, so it does not depend
    on how a leg is padded or laid out in memory.
    """
    code = np.zeros(tuple(dims), dtype=np.float64)
    mult = 1.0
    for ax, d in enumerate(dims):
        shape = [1] * len(dims)
        shape[ax] = d
        code = code + (np.arange(d, dtype=np.float64) * mult).reshape(shape)
        mult *= RADIX
    x = GOLDEN * (1.0 + code)
    return (0.5 + (x - np.floor(x))).reshape(-1)


def fix_signs(q, dims):
    """Sign of each column of q (rows = multi-index over ``dims``) per the convention.

    Returns the vector of +-1 factors; the caller multiplies q and every
    partner factor by it.
    """
    w = sign_weights(dims)
    proj = w @ q
    return np.where(proj < 0, -1.0, 1.0)


def basis_weights(dims, count):
    """Weight vectors w_j(i) = 0.5 + frac(g (1 + code(i)) + j (sqrt 2 - 1)), j < count."""
    code = np.zeros(tuple(dims), dtype=np.float64)
    mult = 1.0
    for ax, d in enumerate(dims):
        shape = [1] * len(dims)
        shape[ax] = d
        code = code + (np.arange(d, dtype=np.float64) * mult).reshape(shape)
        mult *= RADIX
    x = (GOLDEN * (1.0 + code)).reshape(-1)
    w = np.empty((x.size, count))
    for j in range(count):
        y = x + j * SQRT2M1
        w[:, j] = 0.5 + (y - np.floor(y))
    return w


def multiplets(vals, k, tau_deg):
    """Groups (start, size) of the first k values: neighbours closer than tau_deg * vals[0] share a group."""
    groups = []
    a = 0
    for i in range(1, k + 1):
        if i == k or (vals[i - 1] - vals[i]) > tau_deg * vals[0]:
            groups.append((a, i - a))
            a = i
    return groups


def canonical_rotation(q, vals, k, dims, tau_deg):
    """Block-diagonal orthogonal R (k x k) that puts the first k columns of q in canonical form."""
    rot = np.eye(k)
    if k == 0:
        return rot
    groups = multiplets(vals, k, tau_deg)
    dmax = max(d for _, d in groups)
    w = basis_weights(dims, dmax)
    for a, d in groups:
        z = q[:, a:a + d].T @ w[:, :d]
        qz, _ = qr_pos(z)
        rot[a:a + d, a:a + d] = qz
    return rot
