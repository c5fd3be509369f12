"""Benchmark: 4D Ising triad-ATRG RG steps per second at D = 32 on one MI355X.

One "step" is one full triad-ATRG coarse-graining step (re-split, bond swap,
triad representation, squeezers, makeMG / makeMH) on the device state.
Warm-up steps run the RG flow until the leg dimensions saturate at D; the
timed steps continue the same flow.  Prints one JSON line.

The roofline entry is for the coarse-graining GEMMs (makeMG / makeMH), the
dominant kernel: algorithmic flops per launch (2 M N K of the contraction)
over the launch's average duration from HIP events on the library's stream.
The CPU baseline times the FP64 oracle on a bounded sample of the same step
(see cpu_baseline.sample).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0}   # dense MFMA TFLOP/s, MI355X
DTYPE = {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3"}


def cpu_baseline(D, r):
    """Time the oracle's makeMG at D, R = r D on 1 and 2 of the D i_a slabs.

    The marginal per-slab time (2 slabs minus 1) times D plus the slab-free
    part (T23) gives Phi; Phi and Psi together are 85% of the algorithmic
    flops of a steady step at D = 32, which scales the sample to one step.
    """
    import numpy as np
    from oracle import trg as otrg
    R = r * D
    rng = np.random.default_rng(0)
    f = rng.standard_normal((D, R, D, D))           # F[alpha, kX, t3, g]
    ti = rng.standard_normal((D, D, R))
    tj = rng.standard_normal((D, D, R))
    m = [rng.standard_normal((D, D, D)) for _ in range(3)]
    threads = os.environ.get("OMP_NUM_THREADS") or str(os.cpu_count())
    times = []
    for slabs in (1, 2):
        e = rng.standard_normal((slabs, R, D, D))   # E[i_a, kA, t3, alpha] on `slabs` i_a values
        t0 = time.perf_counter()
        otrg.make_phi(e, f, ti, tj, *m)
        times.append(time.perf_counter() - t0)
    per_slab = max(times[1] - times[0], 1e-9)
    fixed = max(times[0] - per_slab, 0.0)
    a7 = 2 * (fixed + D * per_slab)              # Phi and Psi, all D slabs
    step = a7 / 0.85
    return {"value": 1.0 / step, "unit": "RG steps/s", "cores": int(threads), "kind": "oracle",
            "sample": "oracle makeMG at D=%d, R=%d on 1 and 2 of the %d i_a slabs (%.1f s, %.1f s); per-slab "
                      "and slab-free parts scaled to Phi+Psi of one step and by the 85%% flop share of "
                      "makeMG/makeMH in a steady step" % (D, R, D, times[0], times[1])}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=6)
    ap.add_argument("--D", type=int, default=32)
    ap.add_argument("--r", type=int, default=7)
    ap.add_argument("--beta", type=float, default=0.1497)
    ap.add_argument("--h", type=float, default=0.0)
    ap.add_argument("--precision", default="fp64", choices=list(PEAK))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build runs the RG step on a single MI355X "
              "(no multi-GPU path); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import paper_2507_21909_amd as trg
    prec = {"fp64": trg.FP64, "fp32": trg.FP32, "bf16x3": trg.BF16X3}[args.precision]
    seed = 0x2507219090000000 + 3000
    s = trg.Solver(seed=seed, r=args.r, precision=prec)
    s.tensor_init(trg.MODEL_ISING, args.beta, args.h, args.D)
    for i in range(args.warmup):
        s.triad_atrg_step(i % 4)
        print("warmup step %d done, dims %s" % (i, s.shape()[0]), file=sys.stderr, flush=True)
    s.log_z_per_site()                 # synchronises the stream
    s.set_timing(True)
    s.kernel_time()                    # reset counters
    t0 = time.perf_counter()
    for i in range(args.warmup, args.warmup + args.steps):
        s.triad_atrg_step(i % 4)
        print("timed step %d done" % i, file=sys.stderr, flush=True)
    f = s.log_z_per_site()             # synchronises the stream
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    kms, kflops, nl = s.kernel_time()
    R = args.r * args.D
    step_flops = 8.0 * R * R * args.D ** 5  # makeMG + makeMH algorithmic flops per steady step
    roof = None
    if nl > 0 and kms > 0:
        achieved = kflops / (kms * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": PEAK[args.precision], "unit": "TFLOP/s",
                "frac": achieved / PEAK[args.precision], "traffic": None,
                "kernel": "gemm (makeMG/makeMH)", "launches": nl, "avg_ms": kms / nl}
    out = {
        "metric": "4D triad-ATRG RG steps/s at D=32",
        "value": 1e3 / ms_step,
        "unit": "RG steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.precision],
        "data": "synthetic (4D Ising tensor from beta, h; seeded Philox sketch)",
        "config": {"workload": "triad-ATRG 4D Ising, beta=%g, h=%g, D=%d, r=%d (R=%d), sketch 2D, 1 power "
                               "iteration, steady-state steps %d..%d of the flow" % (
                                   args.beta, args.h, args.D, args.r, R, args.warmup, args.warmup + args.steps - 1),
                   "D": args.D, "R": R, "precision": args.precision},
        "tflops_makeMG_makeMH_per_step": step_flops / (ms_step * 1e-3) / 1e12,
        "log_z_per_site": f,
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.D, args.r)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
