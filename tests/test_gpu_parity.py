"""Parity of the HIP path with the FP64 oracle, through the C ABI.

Tolerances (the parity norm is err_max = max|T - T_ref| / max|T_ref|):
  FP64 on the GPU     <= 1e-12
  FP32 compensated    <= 1e-5
Edge cases: single element, tiny tiles (many ragged tiles), batched
instances, Dirichlet / convection / radiation / flux / point loads, and
bitwise determinism across tilings, graph replay and repeated runs.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from oracle import Oracle
from tests import helpers as H
from workloads import mesh as M, problems as P

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32c": 1e-5}


def _sim(p, prec, **kw):
    from paper_1909_03355_amd import Simulation
    return Simulation(p, prec=prec, **kw)


def _gpu_run(p, prec, nsteps, graph_steps=None, **kw):
    with _sim(p, prec, **kw) as s:
        s.set_temperature()
        s.step(nsteps, graph_steps=graph_steps)
        return s.temperature(), s


def _check(p, nsteps, precs=("fp64", "fp32c"), **kw):
    o = Oracle(p)
    ref = o.run(nsteps)
    out = {}
    for prec in precs:
        T, s = _gpu_run(p, prec, nsteps, **kw)
        np.testing.assert_allclose(s.dt_crit, np.atleast_1d(o.dt_crit), rtol=1e-12)
        err = oracle.err_max(T, ref)
        print(f"{p['name']} {prec} steps={nsteps} err_max={err:.3e} rms={oracle.err_rms(T, ref):.3e}",
              flush=True)
        assert err <= TOL[prec], (prec, err)
        out[prec] = T
    return ref, out


def test_plain_cube_fp64_and_fp32c():
    _check(P.cube_plain(10, 1000), 1000)


def test_plain_cube_tets():
    _check(P.cube_plain(6, 200, elem="tet4"), 200)


def test_nonlinear_hex_small():
    _check(P.cube_nonlinear_hex(8, 300), 300)


def test_nonlinear_hex_ragged_tiles():
    # 9^3 = 729 nodes in tiles of at most 37: many tiles of uneven size
    _check(P.cube_nonlinear_hex(8, 100), 100, tile_nodes=37)


def test_aniso_tet_small():
    _check(P.cube_aniso_tet(6, 200), 200)


def test_batched_small():
    p = P.batched_hex(n_inst=6, lo=2, hi=7, nsteps=150)
    ref, out = _check(p, 150)


def test_adjoint_workload_forward_small():
    _check(P.adjoint_hex(8, 100, n_sensors=16), 100)


def test_paper_standin_td():
    p = P.paper_standin(n=6, td=True, nsteps=100)
    _check(p, 100)


def test_single_element_all_bcs():
    for elem in ("hex8", "tet4"):
        X = H.distorted_hex(3) if elem == "hex8" else H.random_tet(3)
        p = H.single_element(elem, X, H.aniso_material(rho=1000.0, c0=900.0))
        nfn = 4 if elem == "hex8" else 3
        faces = M.boundary_faces(dict(elem=elem, conn=p["conn"]))
        P.set_faces(p, faces, h=20.0, Ta=5.0, eps=0.5, q=100.0)
        p["pt_nodes"], p["pt_W"] = np.array([1], np.int32), np.array([0.3])
        p["T0"] = np.linspace(20, 60, X.shape[0])
        p["dt"], p["T_lo"], p["T_hi"] = None, 0.0, 100.0
        _check(p, 50)


def test_dirichlet_and_points_tet():
    p = P.paper_standin(n=5, td=False, nsteps=50)
    _check(p, 50)


def test_tilings_are_bitwise_identical():
    """Every nodal sum runs in ascending element order whatever the tiling."""
    p = P.cube_nonlinear_hex(8, 50)
    base, _ = _gpu_run(p, "fp32c", 50)
    for tn in (23, 64, 300):
        T, _ = _gpu_run(p, "fp32c", 50, tile_nodes=tn)
        assert np.array_equal(T, base), tn
    T, _ = _gpu_run(p, "fp32c", 50, block_threads=64)
    assert np.array_equal(T, base)


@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
def test_fused_steps_are_bitwise_identical(prec):
    """A launch that advances K steps (K element rings of halo per tile) gives
    exactly the single-step result; step counts not divisible by K end with a
    shorter launch."""
    for p in (P.cube_nonlinear_hex(8, 37), P.cube_aniso_tet(5, 37)):
        base, _ = _gpu_run(p, prec, 37, fuse_steps=1)
        for K in (2, 3, 4):
            T, s = _gpu_run(p, prec, 37, fuse_steps=K)
            assert s.info["fuse_steps"] == K
            assert np.array_equal(T, base), (p["name"], K)
        T, _ = _gpu_run(p, prec, 37, fuse_steps=3, graph_steps=12, tile_nodes=50)
        assert np.array_equal(T, base)


def test_graph_and_repeat_bitwise():
    p = P.cube_nonlinear_hex(8, 90)
    a, _ = _gpu_run(p, "fp32c", 90)
    b, _ = _gpu_run(p, "fp32c", 90, graph_steps=20)
    c, _ = _gpu_run(p, "fp32c", 90, graph_steps=20)
    assert np.array_equal(a, b) and np.array_equal(b, c)


def test_state_resume_bitwise():
    p = P.cube_nonlinear_hex(6, 40)
    full, _ = _gpu_run(p, "fp32c", 40)
    with _sim(p, "fp32c") as s:
        s.set_temperature()
        s.step(20)
        hi, lo, st = s.get_state()
    with _sim(p, "fp32c") as s2:
        s2.set_state(hi, lo, st)
        s2.step(20)
        assert s2.steps_taken == 40
        assert np.array_equal(s2.temperature(), full)


def test_errors():
    from paper_1909_03355_amd import FedError
    from paper_1909_03355_amd import _lib as L
    p = P.cube_plain(4, 10)
    o = Oracle(p)
    with pytest.raises(FedError) as ei:
        _sim(dict(p, dt=1.05 * o.dt_crit), "fp64")
    assert ei.value.code == L.FED_E_UNSTABLE
    # inverted hexahedron: swap two layers of local nodes
    q = dict(p, conn=p["conn"][[4, 5, 6, 7, 0, 1, 2, 3]].copy())
    with pytest.raises(FedError) as ei:
        _sim(q, "fp32c")
    assert ei.value.code == L.FED_E_MESH
    # step before set_temperature
    with _sim(p, "fp32c") as s:
        with pytest.raises(FedError) as ei:
            s.step(1)
        assert ei.value.code == L.FED_E_STATE


def test_health_check_fires_when_unstable():
    from paper_1909_03355_amd import FedError
    from paper_1909_03355_amd import _lib as L
    n = 8
    p, m = H.box_problem("hex8", n, side=1.0)
    p["T0"] = ((-1.0) ** np.rint(m["x"] * n)) * 1.0
    p["T_lo"], p["T_hi"] = -2.0, 2.0
    o = Oracle(p)
    p["dt"] = 1.2 * o.dt_crit
    with _sim(p, "fp32c", allow_unstable=True) as s:
        s.set_temperature()
        s.step(200)
        with pytest.raises(FedError) as ei:
            s.temperature()
        assert ei.value.code == L.FED_E_UNSTABLE


def test_nonlinear_hex64_full_size_sampled_steps():
    """Full 64^3 workload, 200 steps, in the launch configuration the
    benchmark uses (default tiles, graph replay)."""
    p = P.cube_nonlinear_hex(64, 200)
    o = Oracle(p)
    ref = o.run(200)
    for prec in ("fp64", "fp32c"):
        T, s = _gpu_run(p, prec, 200, graph_steps=100)
        err = oracle.err_max(T, ref)
        print(f"hex64 {prec} 200 steps err_max={err:.3e}", flush=True)
        assert err <= TOL[prec]
