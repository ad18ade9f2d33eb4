"""Autotuner for the launch shape of the step kernel.

Times a set of launch shapes - (tile_nodes, block_threads, fuse_steps) with
one kernel launch per K steps, and resident stepping (one launch for all the
steps, tiles held in registers) where the mesh fits the GPU's resident
workgroups - on the actual problem and returns the fastest.  Results are
cached in a JSON file keyed by element type, precision, problem size (rounded
to a power of two) and GPU architecture, so a repeated run of a similar
problem skips the search.  Every candidate gives bitwise-identical
temperatures (the nodal sums run in ascending element order whatever the
tiling), so the choice affects speed only.
"""
from __future__ import annotations

import json
import math
import os

DEFAULT_CANDIDATES = [dict(tile_nodes=t, block_threads=b, fuse_steps=k)
                      for k in (1, 2) for t in (256, 512, 1024) for b in (256, 512)] + \
                     [dict(resident=True, block_threads=b) for b in (1024, 512)]
# meshes whose set-up takes seconds: the shapes that won on smaller meshes
LARGE_CANDIDATES = [dict(tile_nodes=t, block_threads=b, fuse_steps=1)
                    for t, b in ((512, 256), (1024, 256), (1024, 512), (256, 256))]
LARGE_ELEMS = 2_000_000
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "fedfem", "autotune.json")


def _arch():
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def cache_key(prob, prec):
    E = prob["conn"].shape[1]
    n_inst = 1 if prob["node_instance"] is None else int(prob["node_instance"].max()) + 1
    return f"{prob['elem']}-{prec}-E2^{round(math.log2(max(E, 1)))}-inst{min(n_inst, 2)}-{_arch()}"


def time_candidate(prob, prec, cand, steps=200, graph_steps=100, reps=2):
    """Microseconds per step of one candidate (best of reps)."""
    import torch
    from .sim import Simulation
    with Simulation(prob, prec=prec, **cand) as s:
        s.set_temperature()
        s.step(graph_steps, graph_steps=graph_steps)
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            s.step(steps, graph_steps=graph_steps)
            b.record()
            torch.cuda.synchronize()
            best = min(best, a.elapsed_time(b) * 1e3 / steps)
    return best


def autotune(prob, prec="fp32c", candidates=None, steps=200, cache=DEFAULT_CACHE, refresh=False,
             log=None):
    """Best launch shape for this problem: dict(tile_nodes, block_threads,
    fuse_steps, us_per_step, key, from_cache)."""
    key = cache_key(prob, prec)
    table = {}
    if cache and os.path.exists(cache):
        with open(cache) as fh:
            table = json.load(fh)
    if not refresh and key in table:
        return dict(table[key], key=key, from_cache=True)
    best = None
    if candidates is None:
        candidates = LARGE_CANDIDATES if prob["conn"].shape[1] > LARGE_ELEMS else DEFAULT_CANDIDATES
    for cand in candidates:
        try:
            us = time_candidate(prob, prec, cand, steps=steps)
        except Exception as exc:  # a shape the mesh cannot take (e.g. LDS) is skipped
            if log:
                log(f"autotune {cand}: skipped ({exc})")
            continue
        if log:
            log(f"autotune {cand}: {us:.2f} us/step")
        if best is None or us < best["us_per_step"]:
            best = dict(cand, us_per_step=us)
    if best is None:
        raise RuntimeError("no candidate launch shape worked")
    table[key] = best
    if cache:
        os.makedirs(os.path.dirname(cache), exist_ok=True)
        with open(cache + ".tmp", "w") as fh:
            json.dump(table, fh, indent=1, sort_keys=True)
        os.replace(cache + ".tmp", cache)
    return dict(best, key=key, from_cache=False)


def launch_kwargs(tuned):
    return {k: tuned[k] for k in ("tile_nodes", "block_threads", "fuse_steps", "resident")
            if k in tuned}
