"""Device-memory entry points (torch CUDA tensors through the C ABI) against the oracle."""
import sys

import numpy as np
import pytest

import paper_2507_21909_amd as trg
from oracle.linalg import qr_pos

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


# ragged row counts (not multiples of the 256-row blocks), one column, the
# largest column count, graded columns
@pytest.mark.parametrize("m,n", [(1, 1), (300, 1), (777, 13), (4096, 32), (70001, 64), (20000, 48)])
def test_qr_matches_oracle(m, n):
    import torch
    _say("trg_qr", m, n)
    rng = np.random.default_rng(7 * m + n)
    a = rng.standard_normal((m, n)) * (10.0 ** -np.linspace(0, 6, n))[None, :]
    q, r = trg.qr(torch.from_numpy(a).cuda())
    torch.cuda.synchronize()
    q, r = q.cpu().numpy(), r.cpu().numpy()
    qo, ro = qr_pos(a)
    # full column rank: the QR with diag(R) >= 0 is unique
    assert np.max(np.abs(r - ro)) <= 1e-12 * np.max(np.abs(ro))
    scale = np.abs(np.diagonal(ro))
    # column j of Q is determined to about eps * cond of the leading j columns
    assert np.max(np.abs(q - qo)) <= 1e-8
    assert np.max(np.abs(q.T @ q - np.eye(n))) <= 1e-13
    assert np.max(np.abs(q @ r - a)) <= 1e-13 * np.max(np.abs(a))
    assert np.all(np.diagonal(r) >= 0) and np.all(np.tril(r, -1) == 0)
    assert scale.min() > 0


def test_qr_rejects_bad_sizes():
    import torch
    a = torch.zeros((10, 65), dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        trg.qr(a)
    lib = trg.load_library()
    # host-side checks: nothing is launched
    assert lib.trg_qr(None, 10, 4, None, None, None) == -1
    assert lib.trg_qr(a.data_ptr(), 3, 4, a.data_ptr(), a.data_ptr(), None) == -1
