"""trg_batch: many (beta, h, D) solves at once, each equal bit for bit to a lone solver."""
import sys
import time

import numpy as np
import pytest

import paper_2507_21909_amd as trg

pytestmark = pytest.mark.gpu
SEED = 0x2507219090000000 + 4000


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _alone(beta, h, D, instance, nsteps):
    s = trg.Solver(seed=SEED, instance=instance)
    s.tensor_init(trg.MODEL_ISING, beta, h, D)
    for k in range(nsteps):
        s.triad_atrg_step(k % 4)
    return s.log_z_per_site()


def test_batch_equals_sequential_bitwise():
    betas = [0.140, 0.1497, 0.160, 0.1497, 0.150, 0.145]
    hs = [0.0, 1e-4, 0.0, 1e-3, 1e-2, 0.0]
    Ds = [8, 12, 6, 8, 12, 4]
    nsteps = 12
    _say("batch of", len(betas))
    b = trg.Batch(betas, hs, Ds, seed=SEED)
    t0 = time.perf_counter()
    b.run(nsteps)
    got = b.log_z_per_site()
    t_batch = time.perf_counter() - t0
    t0 = time.perf_counter()
    ref = [_alone(be, h, D, i, nsteps) for i, (be, h, D) in enumerate(zip(betas, hs, Ds))]
    t_seq = time.perf_counter() - t0
    _say("batch %.3f s, sequential %.3f s, instance-steps/s %.1f vs %.1f" % (
        t_batch, t_seq, len(betas) * nsteps / t_batch, len(betas) * nsteps / t_seq))
    assert np.array_equal(got, np.array(ref))


def test_batch_graphs_equal_eager_bitwise():
    """trg_batch_run_graphs replays the steady steps from graphs: same bits as the eager batch."""
    betas = [0.140, 0.1497, 0.160, 0.1497, 0.150, 0.145, 0.1497, 0.155]
    hs = [0.0, 1e-4, 0.0, 1e-3, 1e-2, 0.0, 1e-4, 1e-3]
    Ds = [8, 12, 16, 24, 12, 4, 8, 16]
    nsteps = 16
    _say("graph batch of", len(betas))
    b = trg.Batch(betas, hs, Ds, seed=SEED)
    t0 = time.perf_counter()
    b.run(nsteps)
    ref = b.log_z_per_site()
    t_eager = time.perf_counter() - t0
    b.close()
    g = trg.Batch(betas, hs, Ds, seed=SEED)
    t0 = time.perf_counter()
    g.run(nsteps, graphs=True)
    got = g.log_z_per_site()
    t_graph = time.perf_counter() - t0
    _say("eager %.3f s, graphs %.3f s" % (t_eager, t_graph))
    assert np.array_equal(got, ref)
    # a second run continues the flows: the graphs of the first run were retired with it
    g.run(4, axes=[1, 2, 3, 0], graphs=True)
    b2 = trg.Batch(betas, hs, Ds, seed=SEED)
    b2.run(nsteps)
    b2.run(4, axes=[1, 2, 3, 0])
    assert np.array_equal(g.log_z_per_site(), b2.log_z_per_site())


def test_batch_graphs_fall_back_to_eager(monkeypatch):
    """Replays that exceed their recorded sweeps are rolled back and taken eagerly: same bits."""
    betas, hs, Ds = [0.1497, 0.160, 0.150], [1e-4, 0.0, 1e-3], [12, 16, 12]
    nsteps = 10
    _say("graph batch fallback")
    b = trg.Batch(betas, hs, Ds, seed=SEED)
    b.run(nsteps)
    ref = b.log_z_per_site()
    monkeypatch.setenv("TRG_GRAPH_SWEEP_CAP", "2")
    g = trg.Batch(betas, hs, Ds, seed=SEED)
    g.run(nsteps, graphs=True)
    monkeypatch.delenv("TRG_GRAPH_SWEEP_CAP")
    assert np.array_equal(g.log_z_per_site(), ref)


def test_batch_custom_axes_and_errors():
    b = trg.Batch([0.0, 0.0], [0.3, 0.0], [4, 6], seed=SEED)
    b.run(6, axes=[3, 2, 1, 0, 3, 2])
    got = b.log_z_per_site()
    assert np.allclose(got, [np.log(2 * np.cosh(0.3)), np.log(2.0)], atol=1e-13)
    with pytest.raises(trg.TrgError):
        b.run(1, axes=[4])
    with pytest.raises(trg.TrgError):
        trg.Batch([0.1], [0.0], [1])          # D < 2 is rejected at creation
