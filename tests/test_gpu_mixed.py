"""Mixed-precision contractions (FP32 / BF16 split on the matrix cores) against
the FP64 GPU path on the same seeded flow.

The coarse-graining GEMMs carry a relative arithmetic error of about 1e-8
(FP32, BF16x6) or 5e-7 (BF16x3).  A truncation whose cut separates two values
closer than that error can keep either of them, and the two flows then differ
by the truncation error itself (1e-5 .. 1e-4 here, the same as changing the
sketch seed).  Both runs therefore use the multiplet tolerance tau_deg = 1e-7
(values closer than 1e-7 of the largest at a cut are kept or dropped
together), which the FP32 and BF16x6 errors stay below.
"""
import sys

import pytest

import paper_2507_21909_amd as trg

pytestmark = pytest.mark.gpu
TAU = 1e-7


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _flow(prec, D, nsteps, seed, tau=TAU, beta=0.1497, h=0.0):
    s = trg.Solver(seed=seed, precision=prec, tau_deg=tau)
    s.tensor_init(trg.MODEL_ISING, beta, h, D)
    out = []
    for i in range(nsteps):
        s.triad_atrg_step(i % 4)
        out.append(s.log_z_per_site())
    return out


@pytest.mark.parametrize("D,nsteps,seed", [(16, 40, 0x2507219090000000 + 2000),
                                           (32, 12, 0x2507219090000000 + 3000)])
def test_fp32_and_bf16x6_within_1e7_of_fp64(D, nsteps, seed):
    ref = _flow(trg.FP64, D, nsteps, seed)
    for name, prec, tol in (("fp32", trg.FP32, 1e-7), ("bf16x6", trg.BF16X6, 1.5e-7)):
        got = _flow(prec, D, nsteps, seed)
        err = max(abs(a - b) / abs(b) for a, b in zip(got, ref))
        _say("D=%d %s: max rel err of log Z/V over %d steps %.2e" % (D, name, nsteps, err))
        assert err <= tol


def test_untruncated_steps_show_the_arithmetic_error():
    """The first two steps truncate nothing: the difference is the GEMM rounding alone."""
    seed = 0x2507219090000000 + 3000
    ref = _flow(trg.FP64, 32, 2, seed)
    for prec, tol in ((trg.FP32, 1e-7), (trg.BF16X6, 1e-7), (trg.BF16X3, 2e-6)):
        got = _flow(prec, 32, 2, seed)
        assert max(abs(a - b) / abs(b) for a, b in zip(got, ref)) <= tol
