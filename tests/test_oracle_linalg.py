"""Pins of the oracle's own linear algebra against LAPACK and the definitions."""
import numpy as np
import pytest

from oracle.linalg import qr_pos, jacobi_eigh, jacobi_svd, kept_count, sign_weights, fix_signs


@pytest.mark.parametrize("n", [1, 2, 3, 17, 64, 131])
def test_jacobi_eigh_matches_lapack(n):
    rng = np.random.default_rng(n)
    a = rng.standard_normal((n, n))
    k = a + a.T
    lam, v = jacobi_eigh(k)
    ref = np.linalg.eigvalsh(k)[::-1]
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(lam - ref)) <= 20 * n * 2.2e-16 * scale
    assert np.max(np.abs(v.T @ v - np.eye(n))) < 1e-13
    assert np.max(np.abs(v @ np.diag(lam) @ v.T - k)) < 1e-13 * n * scale
    assert np.all(np.diff(lam) <= 0)


def test_jacobi_eigh_graded_psd_relative_accuracy():
    # Graded PSD matrix D H D: Jacobi keeps high relative accuracy on tiny eigenvalues.
    rng = np.random.default_rng(3)
    n = 12
    h = rng.standard_normal((n, n))
    h = h @ h.T + n * np.eye(n)
    d = np.diag(10.0 ** (-np.arange(n)))
    k = d @ h @ d
    lam, _ = jacobi_eigh(k)
    # reference: eigenvalues of the scaled problem via a Cholesky route in extended range
    l = np.linalg.cholesky(h)
    ref = np.linalg.svd(d @ l, compute_uv=False) ** 2
    assert np.max(np.abs(lam - ref) / ref) < 1e-10


def test_jacobi_eigh_degenerate():
    q, _ = np.linalg.qr(np.random.default_rng(5).standard_normal((6, 6)))
    lam0 = np.array([3.0, 3.0, 1.0, 1.0, 1.0, 0.0])
    k = q @ np.diag(lam0) @ q.T
    lam, v = jacobi_eigh(k)
    assert np.allclose(lam, lam0, atol=1e-14)
    # the 3-fold subspace is reproduced as a subspace
    p1 = v[:, 2:5] @ v[:, 2:5].T
    p0 = q[:, 2:5] @ q[:, 2:5].T
    assert np.max(np.abs(p1 - p0)) < 1e-13


@pytest.mark.parametrize("m,n", [(1, 1), (5, 3), (3, 5), (40, 40), (100, 37), (37, 100)])
def test_jacobi_svd_matches_lapack(m, n):
    rng = np.random.default_rng(m * 101 + n)
    a = rng.standard_normal((m, n))
    u, s, v = jacobi_svd(a)
    ref = np.linalg.svd(a, compute_uv=False)
    k = min(m, n)
    assert u.shape == (m, k) and v.shape == (n, k) and s.shape == (k,)
    assert np.max(np.abs(s - ref)) < 1e-13 * ref[0]
    assert np.max(np.abs(u @ np.diag(s) @ v.T - a)) < 1e-13 * ref[0]
    assert np.max(np.abs(u.T @ u - np.eye(k))) < 1e-13
    assert np.max(np.abs(v.T @ v - np.eye(k))) < 1e-13


def test_jacobi_svd_rank_deficient_and_graded():
    rng = np.random.default_rng(11)
    a = rng.standard_normal((9, 3)) @ rng.standard_normal((3, 7))
    u, s, v = jacobi_svd(a)
    assert np.sum(s > 1e-12 * s[0]) == 3
    assert np.max(np.abs(u @ np.diag(s) @ v.T - a)) < 1e-13 * s[0]
    # columns spanning 1 .. 1e-170: must converge (squared norms underflow)
    g = np.tril(rng.standard_normal((8, 8))) * (10.0 ** (-25.0 * np.arange(8)))[:, None]
    g[0, 0] = 1.0
    u, s, v = jacobi_svd(g)
    assert abs(s[0] - np.linalg.svd(g, compute_uv=False)[0]) < 1e-14


@pytest.mark.parametrize("m,n", [(10, 4), (4, 10), (50, 50)])
def test_qr_pos(m, n):
    a = np.random.default_rng(m + n).standard_normal((m, n))
    q, r = qr_pos(a)
    k = min(m, n)
    assert q.shape == (m, k) and r.shape == (k, n)
    assert np.max(np.abs(q @ r - a)) < 1e-13
    assert np.max(np.abs(q.T @ q - np.eye(k))) < 1e-13
    assert np.all(np.diagonal(r) >= 0)
    assert np.allclose(np.tril(r, -1), 0)


def test_kept_count_rules():
    v = np.array([1.0, 0.5, 0.5, 0.1, 1e-15, 0.0])
    assert kept_count(v, 10, 1e-14, 1e-12) == 4          # eps cut
    assert kept_count(v, 3, 1e-14, 1e-12) == 3
    assert kept_count(v, 2, 1e-14, 1e-12) == 1          # 0.5, 0.5 multiplet dropped whole
    assert kept_count(v, 1, 1e-14, 1e-12) == 1
    assert kept_count(np.zeros(3), 2, 1e-14, 1e-12) == 0
    w = np.array([1.0, 0.5, 0.5 - 1e-13, 0.2])
    assert kept_count(w, 2, 1e-14, 1e-12) == 1          # split below tau_deg counts as a multiplet
    assert kept_count(w, 2, 1e-14, 1e-14) == 2


def test_sign_weights_do_not_depend_on_padding():
    w1 = sign_weights((3, 4)).reshape(3, 4)
    w2 = sign_weights((5, 6)).reshape(5, 6)
    assert np.array_equal(w1, w2[:3, :4])
    assert np.all((w1 >= 0.5) & (w1 < 1.5))
    # an antisymmetric vector under leg exchange is not orthogonal to w
    x = np.random.default_rng(2).standard_normal((4, 4))
    anti = (x - x.T).reshape(16, 1)
    assert abs(float(sign_weights((4, 4)) @ anti[:, 0])) > 1e-3
    sg = fix_signs(np.hstack([anti, -anti]), (4, 4))
    assert sg[0] == -sg[1]


def test_canonical_rotation_depends_only_on_the_subspace():
    from oracle.linalg import canonical_rotation
    rng = np.random.default_rng(21)
    dims = (3, 4, 2)
    n = 24
    q, _ = np.linalg.qr(rng.standard_normal((n, 6)))
    vals = np.array([1.0, 0.5, 0.5, 0.5, 0.2, 0.1])
    rot = canonical_rotation(q, vals, 6, dims, 1e-9)
    c1 = q @ rot
    # rotate the 3-fold multiplet (and flip a singlet): same canonical basis
    r3, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    q2 = q.copy()
    q2[:, 1:4] = q[:, 1:4] @ r3
    q2[:, 4] *= -1
    c2 = q2 @ canonical_rotation(q2, vals, 6, dims, 1e-9)
    assert np.max(np.abs(c1 - c2)) < 1e-13
    # singlets: the sign convention
    single = canonical_rotation(q, np.array([6, 5, 4, 3, 2, 1.0]), 6, dims, 1e-9)
    assert np.allclose(single, np.diag(fix_signs(q, dims)))


def test_resplit_basis_is_gauge_invariant():
    from oracle import trg
    rng = np.random.default_rng(22)
    dims = (2, 3, 2, 2)
    f = int(np.prod(dims))
    u, _ = np.linalg.qr(rng.standard_normal((f, 5)))
    v, _ = np.linalg.qr(rng.standard_normal((f, 5)))
    s = np.array([2.0, 1.0, 1.0, 0.3, 0.3])          # two degenerate pairs
    g = rng.standard_normal((5, 5)) + 3 * np.eye(5)
    phi1 = (u * s).reshape(dims + (5,))
    psi1 = v.reshape(dims + (5,))
    phi2 = (u * s @ g).reshape(dims + (5,))
    psi2 = (v @ np.linalg.inv(g).T).reshape(dims + (5,))
    a1, b1, _c1, d1, _, _ = trg.resplit(phi1, psi1, 1e-14)
    a2, b2, _c2, d2, _, _ = trg.resplit(phi2, psi2, 1e-14)
    assert np.max(np.abs(a1 - a2)) < 1e-12
    assert np.max(np.abs(d1 - d2)) < 1e-12
    assert np.max(np.abs(a1 @ b1.T - (u * s) @ v.T / 2.0)) < 1e-13
