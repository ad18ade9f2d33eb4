"""Full-size runs of the large workloads against the oracle (sampled steps),
batched-versus-solo bitwise equality, and the autotuner."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from oracle import Oracle
from workloads import problems as P

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32c": 1e-5}


def _run(p, prec, nsteps, **kw):
    from paper_1909_03355_amd import Simulation
    with Simulation(p, prec=prec, **kw) as s:
        s.set_temperature()
        s.step(nsteps, graph_steps=10)
        return s.temperature(), s.dt_crit.copy(), s.dt.copy()


def _instance(p, i):
    """Instance i of a batched problem as a problem of its own."""
    ns, ne = p["meta"]["node_start"], p["meta"]["elem_start"]
    n0, n1, e0, e1 = ns[i], ns[i + 1], ne[i], ne[i + 1]
    fmask = np.all((p["faces"] >= n0) & (p["faces"] < n1), axis=1)
    q = dict(p)
    q.update(x=p["x"][n0:n1], y=p["y"][n0:n1], z=p["z"][n0:n1],
             conn=(p["conn"][:, e0:e1] - n0).astype(np.int32),
             materials=[p["materials"][i]], elem_material=None, node_instance=None,
             faces=(p["faces"][fmask] - n0).astype(np.int32),
             face_h=p["face_h"][fmask], face_Ta=p["face_Ta"][fmask],
             face_eps=p["face_eps"][fmask], face_q=p["face_q"][fmask], T0=p["T0"][n0:n1])
    return q, n0, n1


# the launch shapes bench.py times these workloads in
BENCH_SHAPE = dict(tile_nodes=1024, block_threads=512)


def test_batched_full_size():
    p = P.batched_hex(nsteps=20)
    o = Oracle(p)
    ref = o.run(20)
    for prec in ("fp64", "fp32c"):
        T, dtc, dt = _run(p, prec, 20, **BENCH_SHAPE)
        np.testing.assert_allclose(dtc, o.dt_crit, rtol=1e-12)
        np.testing.assert_allclose(dt, o.dt_inst, rtol=1e-12)
        err = oracle.err_max(T, ref)
        print(f"batched_hex256 {prec}: err_max {err:.2e}", flush=True)
        assert err <= TOL[prec]
        if prec == "fp32c":
            # every instance alone gives the same bits as inside the batch
            for i in (0, 77, 255):
                q, n0, n1 = _instance(p, i)
                Ti, _, _ = _run(q, prec, 20)
                assert np.array_equal(Ti, T[n0:n1]), i
            # the default launch shape gives the same bits
            assert np.array_equal(_run(p, prec, 20)[0], T)


def test_aniso_tet_full_size():
    p = P.cube_aniso_tet(nsteps=4)
    o = Oracle(p)
    ref = o.run(4)
    for prec in ("fp64", "fp32c"):
        T, dtc, _ = _run(p, prec, 4, **BENCH_SHAPE)
        assert abs(dtc[0] / o.dt_crit - 1) < 1e-12
        err = oracle.err_max(T, ref)
        print(f"aniso_tet128 {prec}: err_max {err:.2e}", flush=True)
        assert err <= TOL[prec]


def test_autotuner(tmp_path):
    from paper_1909_03355_amd.autotune import autotune, launch_kwargs
    p = P.cube_nonlinear_hex(12, 60)
    cands = [dict(tile_nodes=64, block_threads=128, fuse_steps=1),
             dict(tile_nodes=256, block_threads=256, fuse_steps=1),
             dict(tile_nodes=128, block_threads=256, fuse_steps=2)]
    cache = str(tmp_path / "tune.json")
    best = autotune(p, "fp32c", candidates=cands, steps=50, cache=cache)
    assert not best["from_cache"] and best["us_per_step"] > 0
    again = autotune(p, "fp32c", candidates=cands, steps=50, cache=cache)
    assert again["from_cache"] and launch_kwargs(again) == launch_kwargs(best)
    T1, _, _ = _run(p, "fp32c", 60, **launch_kwargs(best))
    T2, _, _ = _run(p, "fp32c", 60, **launch_kwargs(cands[0]))
    assert np.array_equal(T1, T2)


def test_tables_hex64_full_size():
    """The tabulated-D(T), c(T) workload at 64^3, resident, 200 steps: against
    the oracle, and bitwise against one step per launch."""
    p = P.cube_nonlinear_hex_tables(64, 200)
    ref = Oracle(p).run(200)
    for prec in ("fp64", "fp32c"):
        T, _, _ = _run(p, prec, 200, resident=True)
        err = oracle.err_max(T, ref)
        print(f"tables_hex64 {prec}: err_max {err:.2e}", flush=True)
        assert err <= TOL[prec]
        assert np.array_equal(T, _run(p, prec, 200)[0])


def test_meanhex_hex64_full_size():
    """The uniform-gradient hexahedron on the distorted 64^3 mesh, 100 steps,
    in the launch shape bench.py times (resident), against the oracle, and
    bitwise equal to one step per launch.  In FP32 this launch keeps the
    operators of the elements that run after the halo wait in LDS, so it
    re-reads less than every operator each step; FP64 re-reads them all."""
    from paper_1909_03355_amd import Simulation
    p = P.cube_nonlinear_hex_mean(64, 100)
    ref = Oracle(p).run(100)
    for prec in ("fp64", "fp32c"):
        T, dtc, _ = _run(p, prec, 100, resident=True)
        err = oracle.err_max(T, ref)
        print(f"meanhex_hex64 {prec}: err_max {err:.2e}", flush=True)
        assert err <= TOL[prec]
        assert np.array_equal(T, _run(p, prec, 100)[0])
        with Simulation(p, prec=prec, resident=True) as s:
            i = s.info
        full = 27 * (8 if prec == "fp64" else 4) * i["n_elems_expanded"]
        print(f"meanhex_hex64 {prec}: re-read {i['reread_bytes_per_step'] / 1e6:.2f} of "
              f"{full / 1e6:.2f} MB a step", flush=True)
        if prec == "fp32c":
            assert 0 < i["reread_bytes_per_step"] < 0.8 * full
        else:
            assert i["reread_bytes_per_step"] == full


def test_meanhg_hex64_full_size():
    """Hourglass control on the distorted 64^3 mesh, 100 steps, in the launch
    shape bench.py times (resident): the critical step and the temperatures
    against the oracle, bitwise equal to one step per launch."""
    p = P.cube_nonlinear_hex_mean_hg(64, 100)
    o = Oracle(p)
    ref = o.run(100)
    for prec in ("fp64", "fp32c"):
        T, dtc, _ = _run(p, prec, 100, resident=True)
        assert abs(dtc[0] / o.dt_crit - 1) < 1e-12
        err = oracle.err_max(T, ref)
        print(f"meanhg_hex64 {prec}: err_max {err:.2e}", flush=True)
        assert err <= TOL[prec]
        assert np.array_equal(T, _run(p, prec, 100)[0])


def test_nonlinear_adjoint_hex64():
    """The adjoint through D(T), c(T) and radiation at 64^3 (200 steps,
    checkpoints every 50, resident forward and adjoint): FP32C gradients
    against the FP64 oracle adjoint (max error / max |g| <= 1e-4)."""
    from paper_1909_03355_amd import Simulation
    p = P.nonlinear_adjoint_hex(64, 200, ckpt_every=50)
    sens = p["meta"]["sensors"]
    o = Oracle(p)
    hist = o.run(200, history=True)
    lam = np.zeros(hist[-1].size)
    lam[sens] = 2.0 * (hist[-1][sens] - 60.0) / sens.size
    ref = o.adjoint(hist, lam)
    del hist
    with Simulation(p, prec="fp32c", resident=True) as s:
        s.checkpoint_every(50)
        s.set_temperature()
        s.step(200)
        T = s.temperature()
        lam_gpu = np.zeros(T.size)
        lam_gpu[sens] = 2.0 * (T[sens] - 60.0) / sens.size
        g = s.backward(lam_gpu)
        assert s.info["resident_adjoint"] == 1
    rel = lambda a, b: float(np.max(np.abs(a - b)) / np.max(np.abs(b)))
    errs = {"logk": rel(g["logk"], ref["g_logk"]), "c": rel(g["c"], ref["g_c"]),
            "h": rel(g["h"], ref["g_h"]), "T0": rel(g["T0"], ref["lam0"])}
    print("nladjoint_hex64 fp32c", {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    for k, v in errs.items():
        assert v <= 1e-4, (k, v)


def test_moving_source_hex64_full_size():
    """The moving-source workload at 64^3 in the launch shape bench.py times
    (resident, a point-load schedule moving a 2 W source one node a step),
    200 steps (the 65-row path wraps three times): against the oracle, and
    bitwise against one step per launch."""
    from paper_1909_03355_amd import Simulation
    p = P.moving_source_hex(64, 200)
    n = p["pt_nodes"].size
    W = np.diag(np.full(n, p["meta"]["source_power"]))
    ref = Oracle(p).run(200, pt_schedule=W)
    for prec in ("fp64", "fp32c"):
        out = []
        for kw in (dict(resident=True), dict()):
            with Simulation(p, prec=prec, **kw) as s:
                s.set_point_schedule(W)
                s.set_temperature()
                s.step(200)
                out.append(s.temperature())
        err = oracle.err_max(out[0], ref)
        print(f"moving_source_hex64 {prec}: err_max {err:.2e}", flush=True)
        assert err <= TOL[prec]
        assert np.array_equal(out[0], out[1])
