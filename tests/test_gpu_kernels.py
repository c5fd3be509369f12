"""GPU kernels of the path against numpy and the oracle (through the C ABI)."""
import sys

import numpy as np
import pytest

import paper_2507_21909_amd as trg
from oracle.philox import sketch_omega

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


# (5, 64, 64, 64), (2, 128, 192, 64), (1, 256, 64, 1024): every tile inside C and
# K a multiple of 32, the vector-load kernel; (2, 128, 224, 64): its first 192
# columns on the vector kernel, the last 32 on the general one; the others the
# general one
@pytest.mark.parametrize("shape", [(1, 16, 16, 4), (3, 67, 45, 33), (2, 130, 70, 129), (1, 1, 200, 17),
                                   (5, 64, 64, 64), (1, 300, 1, 7), (2, 128, 192, 64), (1, 256, 64, 1024), (1, 64, 128, 48),
                                   (2, 128, 224, 64)])
@pytest.mark.parametrize("ta,tb", [(False, False), (True, False), (False, True), (True, True)])
def test_gemm_f64(shape, ta, tb):
    batch, m, n, k = shape
    _say("gemm f64", shape, ta, tb)
    rng = np.random.default_rng(m * n + k)
    a = rng.standard_normal((batch, k, m) if ta else (batch, m, k))
    b = rng.standard_normal((batch, n, k) if tb else (batch, k, n))
    c = trg.selftest_gemm(a, b, ta, tb)
    aa = np.swapaxes(a, 1, 2) if ta else a
    bb = np.swapaxes(b, 1, 2) if tb else b
    ref = aa @ bb
    assert np.max(np.abs(c - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref))) * np.sqrt(k)


# every path of the library's permute: two contiguous groups swapped (tiled
# transpose), the source's unit-stride axis moved (tiled through LDS), and the
# element-wise kernel (the unit-stride axis kept last with the other axes
# reordered, as in the step's 32^5 tensors, with short, ragged and long rows,
# or a short destination row); a single axis is a copy
@pytest.mark.parametrize("shape,perm", [((3, 40, 70), (0, 2, 1)), ((17, 5, 33, 40), (3, 1, 0, 2)),
                                        ((16, 16, 16, 16, 32), (1, 2, 3, 0, 4)), ((5, 9, 11, 13, 24), (3, 0, 1, 2, 4)),
                                        ((32, 10, 20, 16), (2, 0, 1, 3)), ((9, 8, 64), (1, 0, 2)),
                                        ((6, 7, 9, 64), (2, 0, 1, 3)), ((5, 3, 11, 13), (1, 2, 0, 3)),
                                        ((64, 32, 32, 64), (1, 0, 2, 3)), ((4, 5, 6, 3), (2, 1, 0, 3)),
                                        ((2, 1, 3, 1, 200), (4, 2, 0, 1, 3)), ((7,), (0,))])
def test_permute_exact(shape, perm):
    _say("permute", shape, perm)
    a = np.random.default_rng(len(shape) * 100 + shape[0]).standard_normal(shape)
    assert np.array_equal(trg.selftest_permute(a, perm), np.transpose(a, perm))


def test_permute_rejects_bad_permutations():
    a = np.zeros((2, 3))
    for perm in [(0, 0), (0, 2)]:
        with pytest.raises(trg.TrgError) as e:
            trg.selftest_permute(a, perm)
        assert e.value.code == -1


@pytest.mark.parametrize("m,n", [(4, 4), (37, 5), (256, 64), (1000, 33), (5000, 64), (70000, 17), (300000, 2),
                                 (64, 64), (257, 40), (100003, 64)])
def test_tsqr(m, n):
    _say("tsqr", m, n)
    rng = np.random.default_rng(m + n)
    a = rng.standard_normal((m, n)) * (10.0 ** -np.linspace(0, 8, n))[None, :]
    q, r = trg.selftest_tsqr(a)
    assert np.max(np.abs(q @ r - a)) < 1e-13 * np.max(np.abs(a))
    assert np.max(np.abs(q.T @ q - np.eye(n))) < 1e-13
    assert np.all(np.diagonal(r) >= 0)
    assert np.allclose(np.tril(r, -1), 0)
    # unique QR (full column rank): matches LAPACK up to column signs
    q2, r2 = np.linalg.qr(a)
    sg = np.sign(np.diagonal(r2))
    assert np.max(np.abs(r - r2 * sg[:, None])) < 1e-12 * np.max(np.abs(r))


def test_tsqr_rank_deficient():
    rng = np.random.default_rng(3)
    a = rng.standard_normal((3000, 4)) @ rng.standard_normal((4, 12))
    q, r = trg.selftest_tsqr(a)
    assert np.max(np.abs(q @ r - a)) < 1e-12 * np.max(np.abs(a))
    assert np.max(np.abs(q.T @ q - np.eye(12))) < 1e-12
    # 64 columns: rank 20 with zero and repeated columns (column-per-lane blocks)
    a = rng.standard_normal((9000, 20)) @ rng.standard_normal((20, 64))
    a[:, 7] = 0.0
    a[:, 40] = a[:, 2]
    q, r = trg.selftest_tsqr(a)
    assert np.max(np.abs(q @ r - a)) < 1e-12 * np.max(np.abs(a))
    assert np.max(np.abs(q.T @ q - np.eye(64))) < 1e-12
    assert np.all(np.diagonal(r) >= 0)


# wide QR (n > 64): blocked Householder over 64-column TSQR panels; ragged
# last panels, square, and sketch-like heights
@pytest.mark.parametrize("m,n", [(65, 65), (1000, 65), (777, 130), (5000, 96), (300, 200), (200000, 160),
                                 (2000, 512)])
def test_tsqr_wide(m, n):
    _say("tsqr wide", m, n)
    rng = np.random.default_rng(m + 3 * n)
    a = rng.standard_normal((m, n)) * (10.0 ** -np.linspace(0, 8, n))[None, :]
    q, r = trg.selftest_tsqr(a)
    assert np.max(np.abs(q @ r - a)) < 1e-13 * np.max(np.abs(a))
    assert np.max(np.abs(q.T @ q - np.eye(n))) < 1e-13
    assert np.all(np.diagonal(r) >= 0)
    assert np.all(np.tril(r, -1) == 0)
    q2, r2 = np.linalg.qr(a)
    sg = np.sign(np.diagonal(r2))
    assert np.max(np.abs(r - r2 * sg[:, None])) < 1e-12 * np.max(np.abs(r))


def test_tsqr_wide_rank_deficient():
    # zero-padded and repeated columns, as a padded bond gives them
    rng = np.random.default_rng(5)
    a = rng.standard_normal((4000, 140))
    a[:, 70:95] = 0.0
    a[:, 5] = 0.0
    a[:, 120] = a[:, 3]
    q, r = trg.selftest_tsqr(a)
    assert np.max(np.abs(q @ r - a)) < 1e-12 * np.max(np.abs(a))
    assert np.max(np.abs(q.T @ q - np.eye(140))) < 1e-13
    assert np.all(np.diagonal(r) >= 0)


@pytest.mark.parametrize("m,n", [(1, 1), (8, 8), (64, 64), (40, 17), (200, 120), (300, 300)])
def test_jacobi_svd(m, n):
    _say("svd", m, n)
    rng = np.random.default_rng(m * 7 + n)
    a = rng.standard_normal((m, n))
    u, s, v, sweeps = trg.selftest_svd(a)
    ref = np.linalg.svd(a, compute_uv=False)
    assert np.max(np.abs(s - ref)) < 1e-13 * ref[0] * np.sqrt(n)
    assert np.max(np.abs(u @ np.diag(s) @ v.T - a)) < 1e-13 * ref[0] * np.sqrt(n)
    assert np.max(np.abs(v.T @ v - np.eye(n))) < 1e-13 * np.sqrt(n)
    assert sweeps < 40


@pytest.mark.parametrize("m,n", [(1000, 517), (1024, 1024), (97, 97), (257, 130)])
def test_panel_jacobi_svd(m, n):
    """n > 96 runs the register-panel block Jacobi (rows per thread 1, 2 or 4)."""
    _say("panel svd", m, n)
    rng = np.random.default_rng(m + 3 * n)
    a = rng.standard_normal((m, n))
    u, s, v, sweeps = trg.selftest_svd(a)
    ref = np.linalg.svd(a, compute_uv=False)
    assert np.max(np.abs(s - ref)) < 1e-13 * ref[0] * np.sqrt(n)
    assert np.max(np.abs(u @ np.diag(s) @ v.T - a)) < 1e-13 * ref[0] * np.sqrt(n)
    assert np.max(np.abs(v.T @ v - np.eye(n))) < 1e-13 * np.sqrt(n)
    assert np.max(np.abs(u.T @ u - np.eye(n))) < 1e-12 * np.sqrt(n)
    assert sweeps < 40


def test_panel_jacobi_svd_squeezer_shape():
    """M = Df C Db (C orthogonal, Df, Db graded over 7 decades), the shape of the
    squeezer matrix: the leading singular values keep high relative accuracy."""
    rng = np.random.default_rng(77)
    n = 1024
    c, _ = np.linalg.qr(rng.standard_normal((n, n)))
    df = 10.0 ** -np.linspace(0, 7, n)
    db = 10.0 ** -np.linspace(0, 7, n)[rng.permutation(n)]
    a = (df[:, None] * c) * db[None, :]
    u, s, v, _ = trg.selftest_svd(a)
    ref = np.linalg.svd(a, compute_uv=False)
    assert np.max(np.abs(s[:40] - ref[:40]) / ref[:40]) < 1e-12
    assert np.max(np.abs(u[:, :40] * s[:40] - a @ v[:, :40])) < 1e-13 * s[0]


def test_jacobi_svd_graded_psd_eigen():
    rng = np.random.default_rng(9)
    n = 150
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = 10.0 ** -np.linspace(0, 12, n)
    k = (q * lam) @ q.T
    k = 0.5 * (k + k.T)
    _u, s, v, _ = trg.selftest_svd(k)
    # k carries its own rounding (about n eps): compare with LAPACK on the same k;
    # the block (panel) Jacobi applies more, smaller rotations than the cyclic one
    ref = np.linalg.svd(k, compute_uv=False)
    assert np.max(np.abs(s - ref) / lam[0]) < 3e-13
    assert np.max(np.abs(s - lam) / lam[0]) < 20 * n * 2.2e-16
    # leading eigenvectors (well separated) match up to sign
    for j in range(10):
        assert abs(abs(v[:, j] @ q[:, j]) - 1.0) < 1e-10


@pytest.mark.parametrize("n,count", [(1, 1), (5, 2), (64, 1), (65, 3), (100, 2), (256, 1), (300, 2)])
def test_block_jacobi_eigh(n, count):
    _say("eigh", n, count)
    rng = np.random.default_rng(n * 13 + count)
    x = rng.standard_normal((count, n, n))
    k = x + x.transpose(0, 2, 1)
    lam, v, sweeps = trg.selftest_eigh(k)
    for b in range(count):
        ref = np.linalg.eigvalsh(k[b])[::-1]
        scale = np.max(np.abs(ref))
        assert np.max(np.abs(lam[b] - ref)) < 20 * n * 2.2e-16 * scale
        assert np.all(np.diff(lam[b]) <= 0)
        assert np.max(np.abs(v[b].T @ v[b] - np.eye(n))) < 1e-12
        assert np.max(np.abs(k[b] @ v[b] - v[b] * lam[b])) < 20 * n * 2.2e-16 * scale
    assert sweeps < 30


def test_block_jacobi_eigh_graded_and_rank_deficient_gram():
    """A Gram X X^T of rank 120 in 520 dims with a spectrum graded over 12 decades:
    the shape of the triad and squeezer Grams (most eigenvalues at the rounding floor)."""
    rng = np.random.default_rng(31)
    n, k = 520, 120
    qx, _ = np.linalg.qr(rng.standard_normal((n, k)))
    sv = 10.0 ** -np.linspace(0, 6, k)
    g = (qx * sv ** 2) @ qx.T
    lam, v, sweeps = trg.selftest_eigh(g)
    assert sweeps < 30
    # g itself carries rounding noise of order n eps (its null space is not exact)
    ref = np.linalg.eigvalsh(g)[::-1]
    floor = 20 * n * 2.2e-16
    assert np.max(np.abs(lam - ref)) < floor
    assert np.max(np.abs(lam[:k] - sv ** 2)) < floor
    assert np.max(np.abs(lam[k:])) < floor
    # eigenvectors up to sign where the gap (about 0.2 lambda_j) dwarfs g's own noise
    for j in range(0, k, 7):
        if sv[j] ** 2 > 1e-4:
            assert abs(abs(v[:, j] @ qx[:, j]) - 1.0) < 1e-8
    assert np.max(np.abs(v.T @ v - np.eye(n))) < 1e-12


def test_block_jacobi_eigh_degenerate():
    rng = np.random.default_rng(32)
    n = 130
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam0 = np.repeat([4.0, 2.0, 1.0, 0.5, 0.0], [3, 40, 1, 60, 26])
    k = (q * lam0) @ q.T
    lam, v, _ = trg.selftest_eigh(k)
    assert np.max(np.abs(lam - lam0)) < 1e-13
    p = v[:, 3:43] @ v[:, 3:43].T
    p0 = q[:, 3:43] @ q[:, 3:43].T
    assert np.max(np.abs(p - p0)) < 1e-12


def _lower_up_to_rows(x):
    """Rows of X = P L reordered into L: row r of L ends at column r, so each
    row's last nonzero column names its place (-1 for a zero row)."""
    n = x.shape[0]
    last = np.array([np.flatnonzero(x[i])[-1] if np.any(x[i]) else -1 for i in range(n)])
    return last


@pytest.mark.parametrize("n,count", [(1, 1), (63, 2), (200, 3), (1024, 2)])
def test_pivoted_cholesky_full_rank(n, count):
    _say("pchol", n, count)
    rng = np.random.default_rng(100 + n)
    a = rng.standard_normal((count, n, n + 8))
    k = a @ a.transpose(0, 2, 1)
    x, rank = trg.selftest_pchol(k, tol=0.0)
    for b in range(count):
        scale = np.max(np.abs(k[b]))
        assert rank[b] == n
        assert np.max(np.abs(x[b] @ x[b].T - k[b])) < 20 * n * 2.2e-16 * scale
        # X = P L with L lower triangular: the rows' last nonzero columns are a permutation
        last = _lower_up_to_rows(x[b])
        assert sorted(last) == list(range(n))
        # diagonal pivoting: L's diagonal is positive and non-increasing
        diag = np.array([x[b][np.flatnonzero(last == j)[0], j] for j in range(n)])
        assert np.all(diag > 0) and np.all(np.diff(diag) <= 1e-12 * diag[0])


def test_pivoted_cholesky_truncates_at_tolerance():
    """Rank 120 in 300 dims, spectrum graded over 10 decades: the factor stops at
    a rounding-level pivot and its columns from there on are exactly zero."""
    rng = np.random.default_rng(41)
    n, r = 300, 120
    q, _ = np.linalg.qr(rng.standard_normal((n, r)))
    g = (q * (10.0 ** -np.linspace(0, 10, r))) @ q.T
    z = np.zeros((n, n))
    x, rank = trg.selftest_pchol(np.stack([g, z]), tol=2.220446049250313e-16)
    assert r <= rank[0] < n
    assert np.all(x[0][:, rank[0]:] == 0.0)
    assert np.max(np.abs(x[0] @ x[0].T - g)) < 20 * n * 2.2e-16
    # the zero matrix has rank 0 and factor 0
    assert rank[1] == 0 and np.all(x[1] == 0.0)
    # without a tolerance a zero pivot is an error
    with pytest.raises(trg.TrgError):
        trg.selftest_pchol(z, tol=0.0)


def test_gram_eig_graded_rank_deficient():
    """The triad-isometry route (pivoted Cholesky, then one-sided Jacobi on the
    factor) on a Gram of rank 120 in 520 dims graded over 12 decades."""
    rng = np.random.default_rng(31)
    n, k = 520, 120
    qx, _ = np.linalg.qr(rng.standard_normal((n, k)))
    sv = 10.0 ** -np.linspace(0, 6, k)
    g = (qx * sv ** 2) @ qx.T
    lam, v, sweeps = trg.selftest_gram_eig(g)
    assert sweeps < 30
    ref = np.linalg.eigvalsh(g)[::-1]
    floor = 20 * n * 2.2e-16
    assert np.all(np.diff(lam) <= 0) and np.all(lam >= 0)
    assert np.max(np.abs(lam - ref)) < floor
    assert np.max(np.abs(lam[:k] - sv ** 2)) < floor
    for j in range(0, k, 7):
        if sv[j] ** 2 > 1e-4:
            assert abs(abs(v[:, j] @ qx[:, j]) - 1.0) < 1e-8
    # the kept part of the basis is orthonormal and satisfies g v = v lam
    vk = v[:, :k]
    assert np.max(np.abs(vk.T @ vk - np.eye(k))) < 1e-12
    assert np.max(np.abs(g @ vk - vk * lam[:k])) < floor


def test_gram_eig_triad_shape():
    """Four 1024 x 1024 Grams of rank 1023 with a steep graded spectrum, the shape
    of the D = 32 triad Grams: eigenvalues to the rounding floor, the leading 224
    eigenvectors up to sign, in far fewer sweeps than the two-sided solver."""
    rng = np.random.default_rng(77)
    n, count = 1024, 4
    sv = np.exp(-np.linspace(0, 18, n - 1))
    gs, qs = [], []
    for b in range(count):
        q, _ = np.linalg.qr(rng.standard_normal((n, n - 1)))
        qs.append(q)
        gs.append((q * sv ** 2) @ q.T)
    g = np.stack(gs)
    lam, v, sweeps = trg.selftest_gram_eig(g)
    _say("gram eig sweeps", sweeps)
    assert sweeps <= 20
    floor = 20 * n * 2.2e-16
    for b in range(count):
        assert np.max(np.abs(lam[b][:n - 1] - sv ** 2)) < floor
        ov = np.abs(np.sum(v[b][:, :224] * qs[b][:, :224], axis=0))
        assert np.max(np.abs(ov - 1.0)) < 1e-9
        vk = v[b][:, :224]
        assert np.max(np.abs(vk.T @ vk - np.eye(224))) < 1e-12


def test_sketch_matches_oracle():
    _say("sketch")
    g = trg.selftest_sketch(0x2507219090000000, 5, 3, 7, (5, 4, 3), 9)
    o = sketch_omega(0x2507219090000000, 5, 3, 7, (5, 4, 3), 9)
    assert g.shape == o.shape
    assert np.max(np.abs(g - o)) < 1e-13


@pytest.mark.parametrize("prec,tol", [(trg.FP32, 2e-6), (trg.BF16X3, 1e-4), (trg.BF16X6, 2e-6)])
@pytest.mark.parametrize("shape", [(1, 64, 64, 64), (2, 100, 70, 3000), (1, 33, 130, 47)])
@pytest.mark.parametrize("ta,tb", [(False, False), (True, True)])
def test_gemm_mixed(prec, tol, shape, ta, tb):
    batch, m, n, k = shape
    _say("gemm mixed", prec, shape, ta, tb)
    rng = np.random.default_rng(m + 3 * n + k)
    a = rng.standard_normal((batch, k, m) if ta else (batch, m, k))
    b = rng.standard_normal((batch, n, k) if tb else (batch, k, n))
    c = trg.selftest_gemm(a, b, ta, tb, precision=prec)
    aa = np.swapaxes(a, 1, 2) if ta else a
    bb = np.swapaxes(b, 1, 2) if tb else b
    ref = aa @ bb
    # error relative to the natural scale of the sum, sqrt(K) for unit normals
    err = np.max(np.abs(c - ref)) / np.sqrt(k)
    assert err < tol, err
