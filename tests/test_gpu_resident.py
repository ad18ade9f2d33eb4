"""Resident stepping (one launch for all the steps of a call, each tile's
elements and nodes held in registers, halo temperatures exchanged through
step-tagged words in memory; FP32 hexahedral tiles place their nodes in LDS
in caller order) against the one-step-per-launch kernel (bitwise: same
element loads, same ordered nodal sums, same update) and the FP64 oracle
(err_max <= 1e-12 FP64, <= 1e-5 compensated FP32)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from oracle import Oracle
from tests import helpers as H
from workloads import problems as P

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32c": 1e-5}


def _sim(p, prec, **kw):
    from paper_1909_03355_amd import Simulation
    return Simulation(p, prec=prec, **kw)


def _run(p, prec, nsteps, graph_steps=None, **kw):
    with _sim(p, prec, **kw) as s:
        s.set_temperature()
        s.step(nsteps, graph_steps=graph_steps)
        return s.temperature(), dict(s.info)


CASES = {
    "nonlinear_hex12": lambda n: P.cube_nonlinear_hex(12, n),
    "aniso_tet6": lambda n: P.cube_aniso_tet(6, n),
    "batched6": lambda n: P.batched_hex(n_inst=6, lo=2, hi=7, nsteps=n),
    "standin_td_dirichlet_points": lambda n: P.paper_standin(n=6, td=True, nsteps=n),
    "plain_hex10": lambda n: P.cube_plain(10, n),
}


@pytest.mark.parametrize("prec", ["fp32c", "fp64", "fp32"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_resident_bitwise_equals_launch_per_step(case, prec):
    p = CASES[case](61)
    print(f"resident {case} {prec}", flush=True)
    base, _ = _run(p, prec, 61)
    # default resident tiles (one per CU), and small tiles with 4 workgroups per CU
    for kw in (dict(), dict(tile_nodes=40, block_threads=256)):
        T, info = _run(p, prec, 61, resident=True, **kw)
        assert info["resident"] == 1 and info["exchange_bytes_per_step"] > 0
        assert np.array_equal(T, base), kw


def test_resident_split_calls_graph_and_resume():
    """Odd and even step counts per call (the final buffer alternates), a graph
    request (served by resident launches), zero steps, and an exact resume."""
    p = P.cube_nonlinear_hex(10, 50)
    base, _ = _run(p, "fp32c", 50)
    with _sim(p, "fp32c", resident=True) as s:
        s.set_temperature()
        s.step(17)
        s.step(0)
        s.step(3, graph_steps=2)
        hi, lo, st = s.get_state()
        s.step(20, graph_steps=10)
        s.step(10)
        assert s.steps_taken == 50
        assert np.array_equal(s.temperature(), base)
    with _sim(p, "fp32c", resident=True) as s:
        s.set_state(hi, lo, st)
        s.step(30)
        assert np.array_equal(s.temperature(), base)


ADJ_CASES = {
    "adjoint_hex8": lambda: P.adjoint_hex(8, 40, n_sensors=16),
    "nonlinear_hex8": lambda: P.cube_nonlinear_hex(8, 40),
    "nonlinear_radiation_dirichlet": lambda: H.nonlinear_adjoint_problem("hex8"),
    "tables_two_materials": lambda: H.table_laws(H.two_material_problem("hex8", 6)),
}


def _backward(p, prec, res, nsteps=40, ck=15, **kw):
    with _sim(p, prec, resident=res, **kw) as s:
        s.checkpoint_every(ck)
        s.set_temperature()
        s.step(nsteps)
        T = s.temperature()
        g = np.random.default_rng(5).standard_normal(T.size) * 1e-3
        return T, s.backward(g), dict(s.info)


@pytest.mark.parametrize("prec", ["fp32c", "fp64", "fp32"])
@pytest.mark.parametrize("case", sorted(ADJ_CASES))
def test_resident_adjoint_bitwise(case, prec):
    """fed_backward on a resident context (each segment recomputed in one
    launch and its adjoint steps run in one resident launch) against the
    one-step-per-launch adjoint on the same tiles: bitwise equal multipliers
    and derivatives; segments of 15, 15 and 10 steps."""
    p = ADJ_CASES[case]()
    print(f"resident adjoint {case} {prec}", flush=True)
    for kw in (dict(), dict(tile_nodes=40, block_threads=256)):
        T0, g0, _ = _backward(p, prec, False, **kw)
        T1, g1, info = _backward(p, prec, True, **kw)
        assert info["resident_adjoint"] == 1, kw
        assert np.array_equal(T0, T1)
        for k in g0:
            assert np.array_equal(g0[k], g1[k]), (kw, k)


def test_resident_adjoint_not_offered_for_tetrahedra():
    """Tetrahedral resident contexts recompute resident and run the adjoint
    one step per launch; still bitwise equal."""
    p = P.cube_aniso_tet(4, 20)
    T0, g0, _ = _backward(p, "fp32c", False, nsteps=20, ck=8)
    T1, g1, info = _backward(p, "fp32c", True, nsteps=20, ck=8)
    assert info["resident"] == 1 and info["resident_adjoint"] == 0
    assert np.array_equal(T0, T1)
    for k in g0:
        assert np.array_equal(g0[k], g1[k]), k


def test_resident_rejects_meshes_that_do_not_fit():
    from paper_1909_03355_amd import FedError
    from paper_1909_03355_amd import _lib as L
    p = P.cube_nonlinear_hex(12, 10)
    # one tile of 2197 nodes exceeds the registers of 256 threads
    with pytest.raises(FedError) as ei:
        _sim(p, "fp32c", resident=True, tile_nodes=4000, block_threads=256)
    assert ei.value.code == L.FED_E_MESH
    # K > 1 is not available in resident stepping
    with pytest.raises(FedError) as ei:
        _sim(p, "fp32c", resident=True, fuse_steps=2)
    assert ei.value.code == L.FED_E_ARG


def test_resident_hex64_full_size():
    """The 64^3 workload, 200 steps, resident with the default tiles: bitwise
    equal to the one-step kernel and within tolerance of the oracle."""
    p = P.cube_nonlinear_hex(64, 200)
    ref = Oracle(p).run(200)
    for prec in ("fp64", "fp32c"):
        T, info = _run(p, prec, 200, resident=True)
        err = oracle.err_max(T, ref)
        print(f"hex64 resident {prec}: tiles {info['n_tiles']} err_max {err:.3e}", flush=True)
        assert err <= TOL[prec]
        base, _ = _run(p, prec, 200, graph_steps=100)
        assert np.array_equal(T, base)


def test_resident_wait_failure_is_reported():
    """Failure path of the bounded halo waits: with every wait looking for a
    tag no word carries, each gives up after 64 polls, the launch still ends,
    and the readout reports FED_E_HIP; normal waits and a new initial state
    then step exactly as a fresh context does."""
    from paper_1909_03355_amd import FedError
    p = P.cube_nonlinear_hex(8, 20)
    with _sim(p, "fp32c", resident=True) as s:
        s.test_waits(spin_limit=64, never_match=True)
        s.set_temperature()
        s.step(5)
        with pytest.raises(FedError, match="FED_E_HIP"):
            s.temperature()
        s.test_waits(0, False)
        s.set_temperature()
        s.step(20)
        T = s.temperature()
    with _sim(p, "fp32c", resident=True) as s:
        s.set_temperature()
        s.step(20)
        assert np.array_equal(s.temperature(), T)
    with _sim(p, "fp32c") as s:
        with pytest.raises(FedError, match="FED_E_STATE"):
            s.test_waits(64, True)


@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
def test_kept_states_give_the_same_gradients(prec):
    """fed_keep_states: the backward pass over the states the forward launches
    kept equals, bit for bit, the one that recomputes every checkpoint
    segment (also across a partial last segment and a split step call)."""
    from paper_1909_03355_amd import FedError, Simulation
    p = P.nonlinear_adjoint_hex(8, 45, n_sensors=30, ckpt_every=10)
    sens = p["meta"]["sensors"]
    out = []
    for keep in (False, True):
        with Simulation(p, prec=prec, resident=True) as s:
            s.checkpoint_every(10)
            if keep:
                s.keep_states()
            s.set_temperature()
            s.step(17)
            s.step(28)
            T = s.temperature()
            lam = np.zeros(T.size)
            lam[sens] = 2.0 * (T[sens] - 60.0) / sens.size
            g = s.backward(lam)
            out.append((T, g))
    (Ta, ga), (Tb, gb) = out
    assert np.array_equal(Ta, Tb)
    for k in ("logk", "c", "h", "T0"):
        assert np.array_equal(ga[k], gb[k]), k
    with Simulation(p, prec=prec) as s:
        s.checkpoint_every(10)
        with pytest.raises(FedError, match="FED_E_STATE"):
            s.keep_states()
