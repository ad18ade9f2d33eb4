"""Parity at each workload's full step count, in the launch shape the
benchmark times: the GPU temperatures after all the steps against the FP64
oracle's, stored at 4,098 seeded nodes by tests/golden/make_golden.py (which
calls only the oracle; err_max = max over those nodes of |T - T_ref| over
max |T_ref| of the whole field).  Bar: 1e-5 compensated FP32, 1e-12 FP64.
Plain FP32's error is printed beside them (no bar: it is what the
compensated state exists to avoid).  The runs must also stay inside the
range their stability bound was derived for (the health check)."""
from __future__ import annotations

import os

import numpy as np
import pytest

from tests.golden import make_golden as G
from workloads import problems as P

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32c": 1e-5}

# workload -> (problem builder, launch shape of the benchmark, precisions)
CASES = {
    "nonlinear_hex64": (lambda: P.cube_nonlinear_hex(64, 10000), dict(resident=True),
                        ("fp32c", "fp64", "fp32")),
    "aniso_tet128": (lambda: P.cube_aniso_tet(128, 2000),
                     dict(tile_nodes=1024, block_threads=512), ("fp32c", "fp64")),
    "batched_hex256": (lambda: P.batched_hex(256, nsteps=5000),
                       dict(tile_nodes=1024, block_threads=512), ("fp32c", "fp64")),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_full_horizon(name):
    from paper_1909_03355_amd import Simulation
    build, shape, precs = CASES[name]
    steps = G.WORKLOADS[name][1]
    if not os.path.exists(G.path_of(name, steps)):
        pytest.skip(f"no stored oracle run for {name} (python tests/golden/make_golden.py {name})")
    head, ids, ref = G.read(name, steps)
    p = build()
    scale = float(head["max_abs"])
    for prec in precs:
        with Simulation(p, prec=prec, **shape) as s:
            s.set_temperature()
            s.step(steps, graph_steps=100)
            h = s.health()
            lo, hi = s.temperature_range()
            T = s.temperature()
        err = float(np.max(np.abs(T[ids] - ref)) / scale)
        print(f"{name} {prec} after {steps} steps: err_max {err:.3e} over {ids.size} nodes; "
              f"T in [{lo:.4f}, {hi:.4f}]", flush=True)
        assert h["first_bad_step"] == -1
        assert p["T_lo"] <= lo and hi <= p["T_hi"]
        if prec in TOL:
            assert err <= TOL[prec], (prec, err)
