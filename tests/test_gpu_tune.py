"""The GEMMs' tile-walk autotuner is bit-neutral.

The group size of the L2-aware tile walk only decides which workgroup takes
which output tile, never the order of any sum, so every choice must give the
same bits.  Each choice runs in a fresh process (TRG_GEMM_GM fixes it for the
process); the in-process run lets the tuner pick, and must agree as well.
"""
import os
import subprocess
import sys

import numpy as np
import pytest

import paper_2507_21909_amd as trg

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# (batch, M, N, K, ta, tb, precision): 2 M N K batch >= 2e10, so the tuner is eligible
CASES = [(2, 2048, 1536, 4096, 0, 0, trg.FP64), (2, 2048, 1536, 4096, 1, 0, trg.FP64),
         (1, 2048, 2048, 2048, 0, 0, trg.BF16X6)]

CHILD = r"""
import sys, numpy as np
import paper_2507_21909_amd as trg
batch, m, n, k, ta, tb, prec = map(int, sys.argv[1:8])
rng = np.random.default_rng(m + n + k)
a = rng.standard_normal((batch, k, m) if ta else (batch, m, k))
b = rng.standard_normal((batch, k, n))
np.save(sys.argv[8], trg.selftest_gemm(a, b, bool(ta), bool(tb), prec))
"""


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _child(case, out, env_extra):
    env = dict(os.environ)
    env.update(env_extra)
    env["PYTHONPATH"] = ROOT + os.pathsep + env.get("PYTHONPATH", "")
    args = [sys.executable, "-c", CHILD] + [str(int(x)) for x in case] + [out]
    r = subprocess.run(args, env=env, capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    return r.stderr


@pytest.mark.parametrize("case", CASES, ids=["f64_nn", "f64_tn", "bf16x6"])
def test_group_size_is_bit_neutral(case, tmp_path):
    _say("tile walk", case)
    res = {}
    for gm in (4, 8, 16, 3):
        out = str(tmp_path / ("c%d.npy" % gm))
        _child(case, out, {"TRG_GEMM_GM": str(gm)})
        res[gm] = np.load(out)
    for gm in (8, 16, 3):
        assert np.array_equal(res[gm], res[4]), gm
    # tuned in a fresh process (the trace names the choice), then again from the cache
    out = str(tmp_path / "tuned.npy")
    err = _child(case, out, {"TRG_GEMM_TRACE": "1"})
    assert "[tune]" in err
    assert np.array_equal(np.load(out), res[4])
    batch, m, n, k, ta, tb, prec = case
    rng = np.random.default_rng(m + n + k)
    a = rng.standard_normal((batch, k, m) if ta else (batch, m, k))
    b = rng.standard_normal((batch, k, n))
    assert np.array_equal(trg.selftest_gemm(a, b, bool(ta), bool(tb), prec), res[4])
    assert np.array_equal(trg.selftest_gemm(a, b, bool(ta), bool(tb), prec), res[4])
