"""Benchmark of the FED-FEM time step on one MI355X.

Default workload (the one the metric is quoted on): the nonlinear hexahedral
case - 0.1 m cube, 64^3 8-node hexahedra (262,144 elements, 274,625 nodes),
orthotropic D(T) = diag(1,2,0.5)(1+0.005T), c(T) = 1000 + 2T, convection on
all faces, radiation on the top face and a flux patch on the bottom, seeded
random T0 - in compensated FP32, with the same steps in FP64 timed for the
speed ratio.  A step is one pass of the whole hot path (element loads, nodal
sums, surface loads, explicit update).  Other workloads (--workload):
aniso_tet128, batched_hex256, adjoint_hex48 (forward + adjoint), and the
follow-up features at the 64^3 size: tables_hex64 (tabulated D(T), c(T)),
meanhex_hex64 (uniform-gradient hexahedron on a distorted mesh), meanhg_hex64
(the same with hourglass control),
nladjoint_hex64 (adjoint through D(T), c(T) and radiation) and
moving_source_hex64 (a point source moved one node every step by a point-load
schedule).

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
# sources that decide a kernel's memory traffic: the kernels, the tiler, the launches
TRAFFIC_SRC = [os.path.join(ROOT, "paper_1909_03355_amd", "csrc", f)
               for f in ("fed_kernels.hip", "fed_kernels.h", "fed_tiling.cpp")]
# Memory traffic of the dominant kernel, from rocprofv3 counter runs
# (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled by what the
# counter reads for a copy kernel of known size (FETCH_SIZE x 2.0, WRITE_SIZE
# x 1.0): bytes per launch for a one-step kernel; for resident stepping (one
# launch for all steps) bytes once per launch plus bytes per step, from two
# launches of different step counts.  Valid only for the launch shape the
# counters were taken in (tiles, block threads, steps per launch, resident) and
# for the kernel sources and the tiler (TRAFFIC_SRC, concatenated) with this
# SHA-1; anything else reports null.
#   workload -> (sha1, kernel, shape, bytes per launch or once, bytes per step)
TRAFFIC = {
    "nonlinear_hex64": ("eb0df3699702a93322f4d258c73abbcc6e2d8da9", "k_resident", (256, 1024, 1, 1), 21584073.0, 2352607.6),
    "aniso_tet128": ("eb0df3699702a93322f4d258c73abbcc6e2d8da9", "k_step1", (4194, 512, 1, 0), 662686128.2, 0.0),
    "batched_hex256": ("eb0df3699702a93322f4d258c73abbcc6e2d8da9", "k_step1", (6437, 512, 1, 0), 470461989.5, 0.0),
    "tables_hex64": ("eb0df3699702a93322f4d258c73abbcc6e2d8da9", "k_resident", (256, 1024, 1, 1), 20650261.5, 2398120.7),
    "meanhex_hex64": ("eb0df3699702a93322f4d258c73abbcc6e2d8da9", "k_resident", (256, 1024, 1, 1), 49962242.5, 5398764.8),
    "meanhg_hex64": ("eb0df3699702a93322f4d258c73abbcc6e2d8da9", "k_resident", (256, 1024, 1, 1), 9629230.1, 59085754.9),
    "moving_source_hex64": ("eb0df3699702a93322f4d258c73abbcc6e2d8da9", "k_resident", (256, 1024, 1, 1), 23536070.2, 2355051.3),
    "paper_standin_ti": ("eb0df3699702a93322f4d258c73abbcc6e2d8da9", "k_resident", (250, 1024, 1, 1), 2936819.7, 201860.7),
    "paper_standin_td": ("eb0df3699702a93322f4d258c73abbcc6e2d8da9", "k_resident", (250, 1024, 1, 1), 2962830.1, 202972.8),
}
METRIC = "element-updates/s & HBM GB/s, FP32-compensated vs FP64 on GPU at stated error"

WORKLOADS = {
    # name: (builder, default steps, oracle sample steps, description, default launch
    #        shape, kind: "steps" | "adjoint" (forward + adjoint) | "moving" (a point
    #        source moved every step))
    "nonlinear_hex64": ("cube_nonlinear_hex", 10000, 200,
                        "0.1 m cube, 64^3 hex8, orthotropic D(T), c(T), convection+radiation+flux",
                        dict(resident=True), "steps"),
    "aniso_tet128": ("cube_aniso_tet", 2000, 4,
                     "0.1 m cube, 128^3 x 6 Kuhn tet4, per-element SPD conductivity, c(T), "
                     "convection", dict(tile_nodes=1024, block_threads=512), "steps"),
    "batched_hex256": ("batched_hex", 5000, 10,
                       "256 hex8 boxes with 8..48 cells per axis, per-instance k, c, h, eps, T0, dt",
                       dict(tile_nodes=1024, block_threads=512), "steps"),
    "adjoint_hex48": ("adjoint_hex", 2000, 100,
                      "48^3 hex8, log-normal k field, convection; forward + adjoint with "
                      "checkpoints every 100 steps", dict(resident=True), "adjoint"),
    # the follow-up features at the size of nonlinear_hex64
    "tables_hex64": ("cube_nonlinear_hex_tables", 10000, 200,
                     "nonlinear_hex64 with D(T) and c(T) as piecewise-linear multiplier tables",
                     dict(resident=True), "steps"),
    "meanhex_hex64": ("cube_nonlinear_hex_mean", 2000, 100,
                      "nonlinear_hex64 on a distorted mesh (interior nodes moved up to 0.25 h) "
                      "with the uniform-gradient hexahedron", dict(resident=True), "steps"),
    "meanhg_hex64": ("cube_nonlinear_hex_mean_hg", 2000, 100,
                     "meanhex_hex64 with hourglass control (eps 0.3, 40 values per element)",
                     dict(resident=True), "steps"),
    "nladjoint_hex64": ("nonlinear_adjoint_hex", 2000, 100,
                        "nonlinear_hex64 (D(T), c(T), radiation) as the forward model of a sensor "
                        "loss; forward + adjoint with checkpoints every 100 steps",
                        dict(resident=True), "adjoint"),
    "moving_source_hex64": ("moving_source_hex", 2000, 200,
                            "nonlinear_hex64 with a 2 W point source moved one node along the "
                            "top face every step (a point-load schedule)",
                            dict(resident=True), "moving"),
    # the paper's timing study (Sec. 4.6) on a synthetic cube of its size: the
    # oracle runs all the steps on one thread and on all threads, beside the
    # paper's single-thread times (context, not a target)
    "paper_standin_ti": ("paper_standin", 2000, 2000,
                         "0.1 m cube, 19^3 x 6 Kuhn tet4 (the paper's timing-study size), k=200, "
                         "rho=1000, c=2000, dt=0.005 s, back face 37 C, 0.2 W point loads",
                         dict(resident=True), "standin"),
    "paper_standin_td": ("paper_standin", 2000, 2000,
                         "paper_standin_ti with k(T), c(T) rising 6 and 20 per C (Sec. 4.2.2)",
                         dict(resident=True), "standin"),
}
# the paper's single-thread C++ times of the timing study (Sec. 4.6), quoted as
# context: 40,021 tetrahedra / 7,872 nodes on an Intel i7-6700 at 3.40 GHz
PAPER_STANDIN = {"paper_standin_ti": 2.376, "paper_standin_td": 4.656}
# a launch shape chosen by the project's autotuner (cached per problem class)
AUTOTUNED = {"batched_hex256"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="nonlinear_hex64", choices=sorted(WORKLOADS))
    ap.add_argument("--steps", type=int, default=0, help="timed steps (0 = the workload's)")
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--graph-steps", type=int, default=100)
    ap.add_argument("--tile-nodes", type=int, default=0)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--fuse", type=int, default=0, help="steps per kernel launch (0 = default)")
    ap.add_argument("--autotune", action="store_true", help="pick the launch shape by timing")
    ap.add_argument("--resident", choices=["default", "on", "off"], default="default",
                    help="resident stepping (one launch for all steps, tiles held in registers)")
    ap.add_argument("--oracle-steps", type=int, default=0,
                    help="steps of the CPU oracle sample (timed baseline and error reference)")
    ap.add_argument("--no-oracle", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-golden", action="store_true",
                    help="skip the full-horizon error run against the stored oracle temperatures")
    ap.add_argument("--no-autotune", action="store_true",
                    help="workloads timed with the autotuner's shape: use the fixed one")
    return ap.parse_args()


def timed_steps(sim, steps, warmup, graph_steps):
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


def timed_adjoint(sim, steps, prob, keep=True):
    """Forward with checkpoints plus the adjoint of an MSE sensor loss; with
    keep on, a resident context keeps every forward state, so the backward
    pass does not recompute the checkpoint segments."""
    import torch
    sens = prob["meta"]["sensors"]
    sim.checkpoint_every(prob["meta"]["ckpt_every"])
    if sim.info["resident"]:
        sim.keep_states(keep)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.set_temperature()
    sim.step(steps)
    T = sim.temperature()
    t1 = time.perf_counter()
    lam = np.zeros(T.size)
    lam[sens] = 2.0 * (T[sens] - 60.0) / sens.size
    sim.backward(lam)
    t2 = time.perf_counter()
    return t1 - t0, t2 - t1


def moving_rows(prob):
    """The source's path as a point-load schedule: row i loads the i-th node of
    the line with the source power, the other listed nodes with nothing."""
    n = prob["pt_nodes"].size
    return np.diag(np.full(n, prob["meta"]["source_power"]))


def timed_moving_host(sim, steps, prob, warmup):
    """The same path driven from the host: the loads replaced (device-side rows,
    no host transfer) before every one-step call."""
    import torch
    W = torch.tensor(moving_rows(prob), device="cuda")
    n = W.shape[0]
    sim.set_temperature()
    for i in range(warmup):
        sim.set_bc(pt_W=W[i % n])
        sim.step(1)
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for i in range(steps):
        sim.set_bc(pt_W=W[i % n])
        sim.step(1)
    stop.record()
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / 1e3


def cpu_info():
    """Model name, logical CPUs and physical cores of the host (/proc/cpuinfo)."""
    model, cores, logical = None, set(), 0
    phys = core = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                k, _, v = line.partition(":")
                k, v = k.strip(), v.strip()
                if k == "processor":
                    logical += 1
                elif k == "model name" and model is None:
                    model = v
                elif k == "physical id":
                    phys = v
                elif k == "core id":
                    core = v
                elif not k and phys is not None:
                    cores.add((phys, core))
                    phys = core = None
        if phys is not None:
            cores.add((phys, core))
    except OSError:
        pass
    return {"model": model, "logical_cpus": logical or os.cpu_count(),
            "physical_cores": len(cores) or None}


def golden_error(name, sim_factory, steps):
    """err_max of a fresh run of the workload's full step count against the
    oracle's stored temperatures at sampled nodes (tests/golden), with the
    health record of that run, or None.  sim_factory(check_every) makes the
    simulation."""
    sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
    try:
        import make_golden as G
    finally:
        sys.path.pop(0)
    gsteps = G.WORKLOADS.get(name, (None, None))[1]
    if gsteps is None or not os.path.exists(G.path_of(name, gsteps)):
        return None
    head, ids, vals = G.read(name, gsteps)
    # ten energy checks along the run (each in the one-step kernel)
    with sim_factory(max(1, gsteps // 10)) as sim:
        sim.set_temperature()
        sim.step(gsteps, graph_steps=100)
        T = sim.temperature()
        health = sim.health()
    err = float(np.max(np.abs(T[ids] - vals)) / float(head["max_abs"]))
    out = {"err_max": err, "steps": gsteps, "nodes": int(ids.size),
           "reference": f"tests/golden/{name}_{gsteps}.txt (oracle, sampled nodes)"}
    out["energy_residual"] = health["energy_residual"]
    out["energy_checks"] = health["energy_checks"]
    out["first_step_outside_window"] = health["first_bad_step"]
    out["window"] = [health["window_lo"], health["window_hi"]]
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the method's "
              "multi-GPU sharding is described in DESIGN.md and not built.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1909_03355_amd import Simulation
    from paper_1909_03355_amd.autotune import autotune, launch_kwargs
    from workloads import problems as P

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    builder, dsteps, osteps, desc, shape, kind = WORKLOADS[args.workload]
    steps = args.steps or dsteps
    osteps = args.oracle_steps or osteps
    bargs = dict(nsteps=steps)
    if kind == "standin":
        bargs["td"] = args.workload.endswith("_td")
    prob = getattr(P, builder)(**bargs)
    E, N = prob["conn"].shape[1], prob["x"].size
    log = lambda m: print(f"[bench] {m}", file=sys.stderr, flush=True)

    kw = dict(shape)
    for k, v in (("tile_nodes", args.tile_nodes), ("block_threads", args.block),
                 ("fuse_steps", args.fuse)):
        if v:
            kw[k] = v
    if args.resident != "default":
        kw["resident"] = args.resident == "on"
    tuned = None
    if args.autotune or (args.workload in AUTOTUNED and not args.no_autotune
                         and not (args.tile_nodes or args.block or args.fuse)):
        tuned = autotune(prob, "fp32c", steps=200, log=log)
        kw = launch_kwargs(tuned)
        log(f"autotuned: {tuned}")

    res = {}
    precs = ["fp32c"] if args.no_fp64 else ["fp32c", "fp64"]
    for prec in precs:
        with Simulation(prob, prec=prec, **kw) as sim:
            if kind == "adjoint":
                # spec: checkpoints every K steps, each segment recomputed
                # in the backward pass; the kept-states variant is timed beside it
                if args.warmup:
                    timed_adjoint(sim, steps, prob, False)  # first-use allocations, module loads
                tf, tb = timed_adjoint(sim, steps, prob, False)
                t = tf + tb
                log(f"{prec}: forward {tf * 1e3:.1f} ms + adjoint {tb * 1e3:.1f} ms for {steps} "
                    "steps (segments recomputed)")
                extra = dict(forward_s=tf, backward_s=tb)
                if sim.info["resident"]:
                    timed_adjoint(sim, steps, prob, True)
                    kf, kb = timed_adjoint(sim, steps, prob, True)
                    log(f"{prec}: kept states: forward {kf * 1e3:.1f} ms + adjoint "
                        f"{kb * 1e3:.1f} ms")
                    extra["kept_states"] = dict(forward_s=kf, backward_s=kb)
                res[prec] = dict(t=t, info=sim.info, **extra)
                continue
            if kind == "moving":
                sim.set_point_schedule(moving_rows(prob))
                t = timed_steps(sim, steps, args.warmup, args.graph_steps)
                log(f"{prec}: {steps} scheduled steps, the source one node further each step, "
                    f"in {t * 1e3:.2f} ms ({t / steps * 1e6:.2f} us/step)")
            else:
                t = timed_steps(sim, steps, args.warmup, args.graph_steps)
                log(f"{prec}: {steps} steps in {t * 1e3:.2f} ms ({t / steps * 1e6:.2f} us/step)")
            res[prec] = dict(t=t, info=sim.info)

    host = cpu_info()
    cpu, errs, gerr = None, {}, {}
    if not args.no_oracle:
        import oracle
        threads = oracle.threads()
        o = oracle.Oracle(prob)
        sched = moving_rows(prob) if kind == "moving" else None
        t0 = time.perf_counter()
        ref = o.run(osteps, pt_schedule=sched)
        tc = time.perf_counter() - t0
        cpu = dict(value=E * osteps / tc, unit="element-updates/s", cores=threads, kind="oracle",
                   sample=f"{osteps} steps of the same workload ({args.workload}), FP64 C "
                          f"oracle with an OpenMP element loop on {threads} threads, {tc:.2f} s",
                   host=host)
        if kind == "standin":
            # the paper's timing study ran one thread: the oracle on one thread too
            oracle.set_threads(1)
            t0 = time.perf_counter()
            o.run(osteps)
            t1c = time.perf_counter() - t0
            oracle.set_threads(threads)
            cpu["one_thread"] = dict(value=E * osteps / t1c, ms_per_step=t1c / osteps * 1e3,
                                     seconds=t1c)
            cpu["ms_per_step"] = tc / osteps * 1e3
            log(f"oracle {osteps} steps: {threads} threads {tc:.2f} s, one thread {t1c:.2f} s")
        for prec in res:
            with Simulation(prob, prec=prec, **kw) as sim:
                if sched is not None:
                    sim.set_point_schedule(sched)
                sim.set_temperature()
                sim.step(osteps)
                errs[prec] = oracle.err_max(sim.temperature(), ref)
        log(f"oracle {osteps} steps {tc:.2f} s; err_max {errs}")
    # error after the workload's full step count, against the stored oracle run
    for prec in ([] if args.no_golden else res):
        g = golden_error(args.workload,
                         lambda ce: Simulation(prob, prec=prec, check_every=ce, **kw), steps)
        if g is not None:
            gerr[prec] = g
    if gerr:
        log(f"full-horizon err_max {({k: v['err_max'] for k, v in gerr.items()})}")

    import hashlib
    src_sha = hashlib.sha1(b"".join(open(f, "rb").read() for f in TRAFFIC_SRC)).hexdigest()
    r32 = res["fp32c"]
    t = r32["t"]
    info = r32["info"]
    K = info["fuse_steps"]
    resident = bool(info["resident"])
    # a point-load schedule adds one row of record powers a step
    sched_b = info["n_bnd_nodes"] * 4 if kind == "moving" else 0
    if resident:
        # one launch runs all the timed steps: the tile data is loaded once, then
        # every step moves only the tagged halo exchange
        launches = 1
        alg = info["algorithmic_bytes_per_launch"] + steps * (info["exchange_bytes_per_step"]
                                                              + sched_b)
        moved = info["moved_bytes_per_launch"] + steps * (info["exchange_bytes_per_step"]
                                                          + info["reread_bytes_per_step"]
                                                          + sched_b)
        kernel = "k_resident"
    else:
        launches = -(-steps // K)
        alg = info["algorithmic_bytes_per_launch"]
        moved = info["moved_bytes_per_launch"]
        kernel = "k_step1" if K == 1 else "k_step"
    achieved = alg / (t / launches) / 1e9
    traffic = None
    tr = TRAFFIC.get(args.workload)
    shape_now = (info["n_tiles"], info["block_threads"], K, int(resident))
    if tr and tr[0] == src_sha and tr[1] == kernel and tuple(tr[2]) == shape_now:
        traffic = tr[3] + (steps * tr[4] if resident else 0.0)
    cfg = {"workload": f"{args.workload}: {desc} ({E} elements, {N} nodes)",
           "elements": E, "nodes": N, "precision": "fp32c",
           "graph_steps": args.graph_steps,
           "steps_per_launch": steps if resident else K, "resident": resident,
           "tiles": info["n_tiles"], "block_threads": info["block_threads"],
           "autotuned": tuned is not None}
    if kind == "adjoint":
        cfg["ckpt_every"] = prob["meta"]["ckpt_every"]
        cfg["keep_states"] = False
    line = {
        "metric": METRIC,
        "value": E * steps / t,
        "unit": "element-updates/s",
        "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": t / steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32-compensated",
        "data": "synthetic (seeded)",
        "config": cfg,
        "hbm_gbs_algorithmic": achieved,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
                     "kernel": kernel, "us_per_launch": t / launches * 1e6,
                     "bytes_per_launch_algorithmic": alg,
                     "bytes_per_launch_moved": moved},
        "cpu_baseline": cpu,
    }
    if kind == "moving":
        with Simulation(prob, prec="fp32c", **kw) as sim:
            n1 = min(steps, 1000)
            t1 = timed_moving_host(sim, n1, prob, min(args.warmup, 200))
        line["host_driven"] = {"us_per_step": t1 / n1 * 1e6, "steps": n1,
                               "how": "fed_set_bc from device rows, then one step, per call",
                               "schedule_speedup": (t1 / n1) / (t / steps)}
        log(f"host-driven moving source: {t1 / n1 * 1e6:.2f} us/step")
    if resident and kind in ("steps", "moving", "standin"):
        # the per-step working set of the method (every element operator and
        # node state, once) processed per step, for comparison with the
        # streaming kernel that moves it from memory every step
        line["working_set_gbs_per_step"] = info["algorithmic_bytes_per_launch"] * steps / t / 1e9
        # the one-step-per-launch kernel on the same problem, same run
        kw1 = {k: v for k, v in kw.items() if k != "resident"}
        with Simulation(prob, prec="fp32c", **kw1) as sim:
            if kind == "moving":
                sim.set_point_schedule(moving_rows(prob))
            n1 = min(steps, 2000)
            t1 = timed_steps(sim, n1, min(args.warmup, 200), args.graph_steps)
            i1 = sim.info
        a1 = i1["algorithmic_bytes_per_launch"] / (t1 / n1) / 1e9
        line["streaming_kernel"] = {"kernel": "k_step1", "us_per_step": t1 / n1 * 1e6,
                                    "steps": n1, "tiles": i1["n_tiles"],
                                    "roofline_achieved_gbs": a1,
                                    "roofline_frac": a1 / PEAK_HBM_GBS,
                                    "resident_speedup": (t1 / n1) / (t / steps)}
        log(f"streaming k_step1: {t1 / n1 * 1e6:.2f} us/step")
    if kind == "adjoint":
        line["roofline"] = None   # forward + adjoint mix, no single dominant kernel rate
        line["note"] = ("value counts forward steps; time includes the adjoint pass with "
                        "every checkpoint segment recomputed")
        line["adjoint"] = {p: {k: v for k, v in r.items() if k not in ("t", "info")}
                           for p, r in res.items()}
    if kind == "standin":
        ms = PAPER_STANDIN[args.workload]
        line["paper"] = {"ms_per_step": ms, "element_updates_per_s": 40021 / (ms * 1e-3),
                         "how": "the paper's single-thread C++ on 40,021 tetrahedra, Intel "
                                "i7-6700 at 3.40 GHz (Sec. 4.6); context, not a target"}
    if "fp64" in res:
        t64 = res["fp64"]["t"]
        i64 = res["fp64"]["info"]
        if i64["resident"]:
            b64 = i64["algorithmic_bytes_per_launch"] + steps * (i64["exchange_bytes_per_step"]
                                                                 + 2 * sched_b)
            l64 = 1
        else:
            b64 = i64["algorithmic_bytes_per_launch"]
            l64 = -(-steps // i64["fuse_steps"])
        line["fp64"] = {"value": E * steps / t64, "ms_per_step": t64 / steps * 1e3,
                        "hbm_gbs_algorithmic": b64 / (t64 / l64) / 1e9,
                        "speedup_fp32c_over_fp64": t64 / t}
    if errs:
        line["err_max_vs_oracle"] = errs
        line["err_steps"] = osteps
    if gerr:
        line["err_full_horizon"] = gerr
    print(json.dumps(line), flush=True)
    # every context is closed (with-blocks above); drain the device and hand
    # torch's cached blocks back before the interpreter and the HIP runtime
    # shut down
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


if __name__ == "__main__":
    main()
