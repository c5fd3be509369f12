"""Benchmark: 4D Ising triad-ATRG RG steps per second at D = 32 on one MI355X.

One "step" is one full triad-ATRG coarse-graining step (re-split, bond swap,
triad representation, squeezers, makeMG / makeMH) on the device state.
Warm-up steps run the RG flow until the leg dimensions saturate at D; the
timed steps continue the same flow.  Prints one JSON line.

The roofline entry is for the coarse-graining GEMMs (makeMG / makeMH), the
dominant kernel: algorithmic flops per launch (2 M N K of the contraction)
over the launch's average duration from HIP events on the library's stream.
The CPU baseline times one steady-state step of the FP64 oracle at D = 16 on
the host and scales it to D by the step's algorithmic flop ratio (see
cpu_baseline.sample).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0, "bf16x6": 2500.0}   # dense MFMA TFLOP/s, MI355X
# MFMA products executed per algorithmic multiply-add (split-BF16 paths)
EXECUTED = {"fp64": 1, "fp32": 1, "bf16x3": 3, "bf16x6": 6}
# HBM bytes per makeMG/makeMH launch (FETCH_SIZE + WRITE_SIZE from two rocprofv3
# --pmc runs of this benchmark, each scaled by the counter's reading for a plain
# 1 GiB copy) for the FP64 kernel at D = 32, r = 7; None for other settings.
TRAFFIC = {("fp64", 32, 7): 5.30e9}
DTYPE = {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3", "bf16x6": "bf16x6"}


def cpu_baseline(D, r, beta, h, seed):
    """Time one steady-state oracle step at D = 16 and scale it to D.

    The oracle (numpy FP64 with its own C Jacobi solvers) runs the same flow
    (beta, h, r, seed) for 4 warm-up steps, until the leg dimensions saturate
    at 16, then one timed step.  That step's time is scaled to D by the ratio
    of the step's algorithmic flops: 8 R^2 D^5 (makeMG/makeMH) + 24 R^2 D^4
    (squeezers) + 8 D^7 + 8 R D^5 (triad) + 8 D^7 + 4 D^7 (bond swap).
    """
    from oracle import trg as otrg

    def step_flops(d):
        rr = r * d
        return 8.0 * rr * rr * d ** 5 + 24.0 * rr * rr * d ** 4 + 8.0 * d ** 7 + 8.0 * rr * d ** 5 + 12.0 * d ** 7

    d0 = 16
    prm = otrg.Params(D=d0, r=r, seed=seed)
    st = otrg.init_ising(beta, h, 4)
    for i in range(4):
        otrg.rg_step(st, i % 4, prm, "triad")
    t0 = time.perf_counter()
    otrg.rg_step(st, 4 % 4, prm, "triad")
    t_step = time.perf_counter() - t0
    scale = step_flops(D) / step_flops(d0)
    threads = os.environ.get("OMP_NUM_THREADS") or str(os.cpu_count())
    return {"value": 1.0 / (t_step * scale), "unit": "RG steps/s", "cores": int(threads), "kind": "oracle",
            "extrapolated": True, "measured_steps_per_s_at_D16": 1.0 / t_step,
            "sample": "one steady-state oracle step (the 5th) of the same flow at D=16, R=%d: %.1f s on %s host "
                      "threads, scaled to D=%d by the step's algorithmic flop ratio %.1f" % (
                          r * d0, t_step, threads, D, scale)}


def batch_main(args):
    """The 128-instance parameter scan (the T_c search workload): beta_j = 0.140 + 0.020 j / 31
    (j = 0..31) x h_l in {0, 1e-4, 1e-3, 1e-2}, instance i = j + 32 l, D = (8, 12, 16, 24)[i mod 4],
    r = 7, L = 2^10 per axis (40 steps).  The 128 instances run as eight trg_batch objects of 16
    (instance words 0, 16, .., 112, so every instance draws the sketches it would in one batch of
    128), with trg_batch_run; a sample of instances must equal lone solves bit for bit, eagerly and
    with their steady steps replayed from HIP graphs.  The sequential time of all 128 is estimated from the sample's per-D
    times."""
    import numpy as np
    import paper_2507_21909_amd as trg
    seed = 0x2507219090000000 + 4000
    betas, hs, Ds = [], [], []
    for i in range(128):
        j, l = i % 32, i // 32
        betas.append(0.140 + 0.020 * j / 31)
        hs.append([0.0, 1e-4, 1e-3, 1e-2][l])
        Ds.append([8, 12, 16, 24][i % 4])
    nsteps = args.batch_steps

    def run(graphs):
        out = np.empty(128)
        wall = 0.0
        for g in range(8):
            idx = slice(16 * g, 16 * g + 16)
            b = trg.Batch(betas[idx], hs[idx], Ds[idx], seed=seed, instance=16 * g)
            t0 = time.perf_counter()
            b.run(nsteps, graphs=graphs)
            out[idx] = b.log_z_per_site()
            wall += time.perf_counter() - t0
            b.close()
            print("batch (%s): instances %d..%d done, %.1f s" % ("graphs" if graphs else "eager", 16 * g,
                                                                 16 * g + 15, wall), file=sys.stderr, flush=True)
        return out, wall

    got, t_eager = run(False)
    sample = [0, 1, 2, 3, 45, 46, 47, 60, 66, 79, 93, 98, 103, 113, 126, 127]
    t_by_d, tg_by_d = {}, {}

    def lone(i, graphs):
        s = trg.Solver(seed=seed, instance=i)
        s.tensor_init(trg.MODEL_ISING, betas[i], hs[i], Ds[i])
        t0 = time.perf_counter()
        rec, k = None, 0
        while k < nsteps:
            if rec:
                try:   # checked: a replay that needs more sweeps than recorded is rolled back
                    rec[k % 4].launch(check=True)
                except trg.TrgError:
                    for g in rec:
                        g.close()
                    s.triad_atrg_step(k % 4)   # eagerly (logs the sweeps), then record again
                    rec = [s.capture(a) for a in range(4)] if k + 1 < nsteps else None
                k += 1
                continue
            before = s.shape()[:2]
            s.triad_atrg_step(k % 4)
            k += 1
            if graphs and s.shape()[:2] == before and k < nsteps:
                rec = [s.capture(a) for a in range(4)]
        f = s.log_z_per_site()
        dt = time.perf_counter() - t0
        for g in rec or []:
            g.close()
        s.close()
        return f, dt

    for i in sample:
        f, dt = lone(i, False)
        t_by_d.setdefault(Ds[i], []).append(dt)
        fg, dtg = lone(i, True)
        tg_by_d.setdefault(Ds[i], []).append(dtg)
        print("lone solves of instance %d (D=%d) done: eager %.3f s, graphs %.3f s" % (i, Ds[i], dt, dtg),
              file=sys.stderr, flush=True)
        if f != got[i] or fg != got[i]:
            print("instance %d differs: batch %.17g alone %.17g graphs %.17g" % (i, got[i], f, fg), file=sys.stderr)
            sys.exit(1)
    t_seq = sum(32 * float(np.mean(v)) for v in t_by_d.values())
    out = {"metric": "batched triad-ATRG instance-steps/s (128 instances, D in {8,12,16,24})",
           "value": 128 * nsteps / t_eager, "unit": "instance-steps/s", "n_gpus": 1, "steps": nsteps,
           "higher_is_better": True, "dtype": "f64", "data": "synthetic (4D Ising tensors from beta, h)",
           "config": {"workload": "128-instance beta x h scan, r=7, %d steps" % nsteps},
           "batch_wall_s": t_eager,
           "sequential_wall_s_estimated": t_seq,
           "sequential_instance_steps_per_s": 128 * nsteps / t_seq,
           "sequential_s_per_solve_by_D": {str(k): float(np.mean(v)) for k, v in sorted(t_by_d.items())},
           "lone_graph_s_per_solve_by_D": {str(k): float(np.mean(v)) for k, v in sorted(tg_by_d.items())},
           "bitwise_equal_sample": len(sample)}
    print(json.dumps(out), flush=True)


def derivative_main(args):
    """Internal energy and magnetisation over a beta scan by the impurity tangents: D = 24
    (R = 168), L = 2^10 per axis (40 steps), beta_j = 0.148 + 0.003 j / 15 (j = 0..15), h = 1e-5,
    contractions in the chosen precision.  For each beta: u = -d(log Z/V)/d(beta) and
    m = d(log Z/V)/dh from one forward run carrying both tangents, the central differences of
    the same flow (delta_beta = 1e-4, delta_h = h / 2, so h - delta_h keeps h's sign), and the
    cost of the tangents as (time with tangents) / (time without)."""
    import numpy as np
    import paper_2507_21909_amd as trg
    prec = {"fp64": trg.FP64, "fp32": trg.FP32, "bf16x3": trg.BF16X3, "bf16x6": trg.BF16X6}[args.precision]
    seed = 0x2507219090000000 + 5000
    D, nsteps, h = args.D, 40, 1e-5
    rows = []

    def flow(beta, hh, tangents):
        s = trg.Solver(seed=seed, precision=prec, tangents=tangents)
        s.tensor_init(trg.MODEL_ISING, beta, hh, D)
        t0 = time.perf_counter()
        for k in range(nsteps):
            s.triad_atrg_step(k % 4)
        f = s.log_z_per_site()
        t = time.perf_counter() - t0
        d = s.impurity_derivatives() if tangents else (None, None)
        s.close()
        return f, d, t

    for j in range(args.derivative_first, args.derivative_first + args.derivative_points):
        beta = 0.148 + 0.003 * j / 15
        try:
            f, (db, dh), t_tan = flow(beta, h, trg.TAN_BETA | trg.TAN_H)
            _, _, t_plain = flow(beta, h, 0)
            fbp, _, _ = flow(beta + 1e-4, h, 0)
            fbm, _, _ = flow(beta - 1e-4, h, 0)
            fhp, _, _ = flow(beta, h + h / 2, 0)
            fhm, _, _ = flow(beta, h - h / 2, 0)
        except trg.TrgError as e:
            # a flow of this point failed (e.g. a cut inside a multiplet too large for the canonical basis)
            rows.append({"beta": beta, "error": str(e)})
            print("beta %.5f  failed: %s" % (beta, e), file=sys.stderr, flush=True)
            continue
        ufd, mfd = -(fbp - fbm) / 2e-4, (fhp - fhm) / h
        rows.append({"beta": beta, "log_z": f, "u": -db, "m": dh, "u_fd": ufd, "m_fd": mfd,
                     "t_with_tangents_s": t_tan, "t_plain_s": t_plain})
        print("beta %.5f  u %.10f (fd %.10f)  m %.6e (fd %.6e)  tangents/plain %.2f" % (
            beta, -db, ufd, dh, mfd, t_tan / t_plain), file=sys.stderr, flush=True)
    ok = [r for r in rows if "error" not in r]
    ratio = float(np.mean([r["t_with_tangents_s"] / r["t_plain_s"] for r in ok])) if ok else None
    out = {"metric": "impurity derivatives of log Z/V over a beta scan (D=%d)" % D,
           "value": ratio, "unit": "time with both tangents / time without", "n_gpus": 1, "steps": nsteps,
           "higher_is_better": False, "dtype": DTYPE[args.precision], "data": "synthetic (4D Ising)",
           "config": {"workload": "triad-ATRG D=%d, r=7, 40 steps, h=1e-5, %d beta values in [0.148, 0.151]" % (
               D, len(rows))},
           "max_rel_u_vs_fd": max((abs(r["u"] - r["u_fd"]) / abs(r["u_fd"]) for r in ok), default=None),
           "failed_points": len(rows) - len(ok),
           "points": rows}
    print(json.dumps(out), flush=True)


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
    ap.add_argument("--batch", action="store_true", help="run the 128-instance scan instead of the D=32 step")
    ap.add_argument("--batch-steps", type=int, default=40)
    ap.add_argument("--derivatives", action="store_true",
                    help="internal energy / magnetisation scan by the impurity tangents (use --D 24)")
    ap.add_argument("--derivative-points", type=int, default=16)
    ap.add_argument("--derivative-first", type=int, default=0,
                    help="first beta index j of the scan (beta_j = 0.148 + 0.003 j / 15)")
    ap.add_argument("--graphs", action="store_true",
                    help="time steps replayed from HIP graphs recorded after the warmup (no kernel timing)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library runs the RG step on a single MI355X "
              "(no multi-GPU path); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.batch:
        batch_main(args)
        return
    if args.derivatives:
        derivative_main(args)
        return
    import paper_2507_21909_amd as trg
    prec = {"fp64": trg.FP64, "fp32": trg.FP32, "bf16x3": trg.BF16X3, "bf16x6": trg.BF16X6}[args.precision]
    seed = 0x2507219090000000 + 3000
    s = trg.Solver(seed=seed, r=args.r, precision=prec)
    s.tensor_init(trg.MODEL_ISING, args.beta, args.h, args.D)
    for i in range(args.warmup):
        s.triad_atrg_step(i % 4)
        print("warmup step %d done, dims %s" % (i, s.shape()[0]), file=sys.stderr, flush=True)
    s.log_z_per_site()                 # synchronises the stream
    graphs = None
    if args.graphs:
        before = s.shape()[:2]
        s.triad_atrg_step(args.warmup % 4)   # one more eager step: it must leave the shapes unchanged
        args.warmup += 1
        if s.shape()[:2] != before:
            print("shapes still changing after the warmup: raise --warmup", file=sys.stderr)
            sys.exit(1)
        graphs = [s.capture(a) for a in range(4)]
        print("4 steps recorded", file=sys.stderr, flush=True)
    else:
        s.set_timing(True)
        s.kernel_time()                # reset counters
    t0 = time.perf_counter()
    for i in range(args.warmup, args.warmup + args.steps):
        if graphs:
            graphs[i % 4].launch()
            continue
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
        algorithmic = kflops / (kms * 1e-3) / 1e12
        achieved = algorithmic * EXECUTED[args.precision]     # executed MFMA flops
        roof = {"bound": "mfma", "achieved": achieved, "peak": PEAK[args.precision], "unit": "TFLOP/s",
                "frac": achieved / PEAK[args.precision],
                "traffic": TRAFFIC.get((args.precision, args.D, args.r)),
                "kernel": "gemm (makeMG/makeMH)", "launches": nl, "avg_ms": kms / nl,
                "algorithmic_tflops": algorithmic}
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
                               "iteration, steady-state steps %d..%d of the flow%s" % (
                                   args.beta, args.h, args.D, args.r, R, args.warmup, args.warmup + args.steps - 1,
                                   ", replayed from HIP graphs" if graphs else ""),
                   "D": args.D, "R": R, "precision": args.precision},
        "makeMG_makeMH_tflops_over_step_time": step_flops / (ms_step * 1e-3) / 1e12,
        "log_z_per_site": f,
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.D, args.r, args.beta, args.h, seed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
