"""trg_qr_noalloc (no device allocation, fixed scratch) against trg_qr through the C ABI.

Both run the same TSQR kernels, so Q and R must agree bit for bit; the pair
is also checked against the oracle's Householder QR (diag(R) >= 0).  Two
calls in a row, the second smaller, show that the scratch left by the first
call does not leak into the second.
"""
import sys

import numpy as np
import pytest

import paper_2507_21909_amd as trg
from oracle.linalg import qr_pos

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _mat(m, n, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((m, n)) * (10.0 ** -np.linspace(0, 5, n))[None, :]


def _check_pair(a_np, q, r):
    q, r = q.cpu().numpy(), r.cpu().numpy()
    qo, ro = qr_pos(a_np)
    n = a_np.shape[1]
    assert np.max(np.abs(r - ro)) <= 1e-12 * np.max(np.abs(ro))
    assert np.max(np.abs(q - qo)) <= 1e-8
    assert np.max(np.abs(q.T @ q - np.eye(n))) <= 1e-13
    assert np.all(np.diagonal(r) >= 0) and np.all(np.tril(r, -1) == 0)


def test_noalloc_qr_equals_allocating_qr_twice():
    import torch
    torch.cuda.init()
    # the largest m the fixed scratch takes at n = 64, then a smaller ragged one
    for (m, n) in [(35584, 64), (777, 13)]:
        _say("trg_qr_noalloc", m, n)
        a_np = _mat(m, n, 11 * m + n)
        a = torch.from_numpy(a_np).cuda()
        q0, r0 = trg.qr(a)
        q1 = torch.full((m, n), float("nan"), dtype=torch.float64, device="cuda")
        r1 = torch.full((n, n), float("nan"), dtype=torch.float64, device="cuda")
        trg.qr_noalloc(a, q1, r1)
        torch.cuda.synchronize()
        assert torch.equal(q0, q1) and torch.equal(r0, r1)
        _check_pair(a_np, q1, r1)


def test_noalloc_qr_rejects_sizes_above_its_scratch():
    import torch
    lib = trg.load_library()
    a = torch.zeros((35585, 64), dtype=torch.float64, device="cuda")
    q = torch.empty_like(a)
    r = torch.empty((64, 64), dtype=torch.float64, device="cuda")
    # host-side checks, nothing is enqueued
    assert lib.trg_qr_noalloc(a.data_ptr(), 35585, 64, q.data_ptr(), r.data_ptr(), None) == -6
    assert b"scratch" in lib.trg_last_error(None)
    assert lib.trg_qr_noalloc(None, 10, 4, None, None, None) == -1
    assert lib.trg_qr_noalloc(a.data_ptr(), 10, 65, q.data_ptr(), r.data_ptr(), None) == -1
