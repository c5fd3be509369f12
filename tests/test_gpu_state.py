"""State handling at the boundary: failed steps and failed re-initialisation."""
import sys

import pytest

import paper_2507_21909_amd as trg

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_failed_step_keeps_log_z():
    """A step that fails after its re-split has added 2^-k log c_k gives the accumulator back.

    max_sweeps = 2 lets the 2 x 2 re-split SVD of the first step converge (one
    rotation, one clean sweep) and stops the bond swap's larger exact SVD: a
    host-side limit, every kernel exits normally.
    """
    _say("failed step rollback")
    s = trg.Solver(seed=5, max_sweeps=2)
    s.tensor_init(trg.MODEL_ISING, 0.1497, 0.05, 6)
    before = s.log_z_per_site()
    with pytest.raises(trg.TrgError) as ei:
        s.triad_atrg_step(0)
    assert ei.value.code == -4
    msg = str(ei.value)
    assert "did not converge" in msg and "n 2)" not in msg, msg
    assert s.shape()[2] == 0
    assert s.log_z_per_site() == before
    # the state is still usable: a new solver with the default limit gives the same first step
    s2 = trg.Solver(seed=5)
    s2.tensor_init(trg.MODEL_ISING, 0.1497, 0.05, 6)
    s2.triad_atrg_step(0)
    assert s2.log_z_per_site() != before


def test_failed_reinit_invalidates_state():
    _say("failed re-init")
    s = trg.Solver(seed=5)
    s.tensor_init(trg.MODEL_ISING, 0.1497, 0.0, 4)
    s.triad_atrg_step(0)
    # D = 400 is outside the kernels' limits: refused before anything changes
    with pytest.raises(trg.TrgError) as ei:
        s.tensor_init(trg.MODEL_ISING, 0.1497, 0.0, 400)
    assert ei.value.code == -6
    s.log_z_per_site()
    # D = 200: two D^5 FP64 tensors of 2.6 TB each cannot be allocated
    with pytest.raises(trg.TrgError) as ei:
        s.tensor_init(trg.MODEL_ISING, 0.1497, 0.0, 200)
    assert ei.value.code == -3
    with pytest.raises(trg.TrgError) as ei:
        s.triad_atrg_step(1)
    assert ei.value.code == -2
    with pytest.raises(trg.TrgError) as ei:
        s.log_z_per_site()
    assert ei.value.code == -2
    # and a valid tensor_init brings it back
    s.tensor_init(trg.MODEL_ISING, 0.0, 0.0, 4)
    s.triad_atrg_step(0)
    import math
    assert abs(s.log_z_per_site() - math.log(2.0)) < 1e-14
