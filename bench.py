"""Benchmark of the FED-FEM time step on one MI355X.

Workload: the nonlinear hexahedral case - 0.1 m cube, 64^3 8-node hexahedra
(262,144 elements, 274,625 nodes), orthotropic D(T) = diag(1,2,0.5)(1+0.005T),
c(T) = 1000 + 2T, convection on all faces, radiation on the top face and a
flux patch on the bottom, seeded random T0 - in compensated FP32, with the
same steps in FP64 timed for the speed ratio.  A step is one pass of the
whole hot path (element loads, nodal sums, surface loads, explicit update).

Prints one JSON line.  `value` is element-updates/s (elements x steps / s)
with all inputs resident on the GPU when the timed region starts.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0   # MI355X HBM3E peak


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--n", type=int, default=64, help="cells per cube edge")
    ap.add_argument("--graph-steps", type=int, default=100)
    ap.add_argument("--tile-nodes", type=int, default=0)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--fuse", type=int, default=0, help="steps per kernel launch (0 = default)")
    ap.add_argument("--oracle-steps", type=int, default=200,
                    help="steps of the CPU oracle sample (timed baseline and error reference)")
    ap.add_argument("--no-oracle", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    return ap.parse_args()


def timed_run(sim, steps, warmup, graph_steps):
    import torch
    sim.set_temperature()
    sim.step(warmup, graph_steps=graph_steps)
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    sim.step(steps, graph_steps=graph_steps)
    stop.record()
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / 1e3


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the method's "
              "multi-GPU sharding is described in DESIGN.md and not built.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1909_03355_amd import Simulation
    from workloads import problems as P

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    prob = P.cube_nonlinear_hex(args.n, args.steps)
    E, N = prob["conn"].shape[1], prob["x"].size

    res = {}
    for prec in (["fp32c"] if args.no_fp64 else ["fp32c", "fp64"]):
        sim = Simulation(prob, prec=prec, tile_nodes=args.tile_nodes, block_threads=args.block,
                         fuse_steps=args.fuse)
        t = timed_run(sim, args.steps, args.warmup, args.graph_steps)
        res[prec] = dict(t=t, info=sim.info, dt=float(sim.dt[0]))
        sim.close()
        print(f"[bench] {prec}: {args.steps} steps in {t * 1e3:.2f} ms "
              f"({t / args.steps * 1e6:.2f} us/step)", file=sys.stderr, flush=True)

    # accuracy against the FP64 oracle on a bounded sample, which is also the
    # timed CPU baseline
    cpu = None
    errs = {}
    if not args.no_oracle:
        import oracle
        o = oracle.Oracle(prob)
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        t0 = time.perf_counter()
        ref = o.run(args.oracle_steps)
        tc = time.perf_counter() - t0
        cpu = dict(value=E * args.oracle_steps / tc, unit="element-updates/s", cores=threads,
                   kind="oracle",
                   sample=f"{args.oracle_steps} steps of the same {args.n}^3 workload, FP64 C "
                          f"oracle, OpenMP element loop, {tc:.2f} s")
        for prec in res:
            sim = Simulation(prob, prec=prec)
            sim.set_temperature()
            sim.step(args.oracle_steps)
            errs[prec] = oracle.err_max(sim.temperature(), ref)
            sim.close()
        print(f"[bench] oracle {args.oracle_steps} steps {tc:.2f} s; err_max {errs}",
              file=sys.stderr, flush=True)

    r32 = res["fp32c"]
    t = r32["t"]
    ms = t / args.steps * 1e3
    info = r32["info"]
    K = info["fuse_steps"]
    launches = -(-args.steps // K)
    alg = info["algorithmic_bytes_per_launch"]
    achieved = alg / (t / launches) / 1e9
    line = {
        "metric": "element-updates/s & HBM GB/s, FP32-compensated vs FP64 on GPU at stated error",
        "value": E * args.steps / t,
        "unit": "element-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32-compensated",
        "data": "synthetic (seeded)",
        "config": {"workload": f"nonlinear_hex{args.n}: 0.1 m cube, {args.n}^3 hex8 "
                               f"({E} elements, {N} nodes), orthotropic D(T), c(T), "
                               "convection+radiation+flux", "elements": E, "nodes": N,
                   "precision": "fp32c", "graph_steps": args.graph_steps,
                   "steps_per_launch": K, "tiles": info["n_tiles"],
                   "block_threads": info["block_threads"]},
        "hbm_gbs_algorithmic": achieved,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS, "traffic": None,
                     "kernel": "k_step", "us_per_launch": t / launches * 1e6,
                     "bytes_per_launch_algorithmic": alg,
                     "bytes_per_launch_moved": info["moved_bytes_per_launch"]},
        "cpu_baseline": cpu,
    }
    if "fp64" in res:
        t64 = res["fp64"]["t"]
        i64 = res["fp64"]["info"]
        l64 = -(-args.steps // i64["fuse_steps"])
        line["fp64"] = {"value": E * args.steps / t64, "ms_per_step": t64 / args.steps * 1e3,
                        "hbm_gbs_algorithmic": i64["algorithmic_bytes_per_launch"]
                        / (t64 / l64) / 1e9,
                        "steps_per_launch": i64["fuse_steps"],
                        "speedup_fp32c_over_fp64": t64 / t}
    if errs:
        line["err_max_vs_oracle"] = {k: v for k, v in errs.items()}
        line["err_steps"] = args.oracle_steps
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
