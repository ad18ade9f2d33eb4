"""The in-run health check (fed_options.check_margin / check_every /
energy_tol, fed_health_get): the stability bound of Sec. 3.4 (Eq. 29) holds
for temperatures in [T_lo, T_hi], so every step's temperatures are checked
against that window; the first step that leaves it is latched and reported
as FED_E_UNSTABLE: exactly the step the oracle leaves the window in the
one-step and fused kernels, and the first of the resident kernel's checks
(every 32 steps, over the extremes of every step) that covers it.  The energy balance of the explicit update is checked every
check_every steps: its residual is at rounding level for FP64 and compensated
FP32 and visibly larger for plain FP32, whose state cannot hold increments
far below ulp(T)."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import Oracle
from workloads import problems as P

pytestmark = pytest.mark.gpu

SHAPES = {
    "one_step": dict(tile_nodes=40),
    "fused": dict(tile_nodes=40, fuse_steps=2, block_threads=256),
    "resident": dict(resident=True),
}


def _leaving_problem():
    """A finite run that leaves its window: the workload's flux patch on a
    16^3 mesh with T_hi lowered to 500 C (the flux heats the patch past it at
    step 36, well clear of the threshold, without the run going unstable: dt
    stays 0.9 of the bound, and the run levels off near 555 C)."""
    p = P.cube_nonlinear_hex(16, 200)
    p["T_lo"], p["T_hi"] = -40.0, 500.0
    return p


def _first_out(p, nsteps, margin=0.0):
    o = Oracle(p)
    H = o.run(nsteps, history=True)
    out = (H.max(axis=1) > p["T_hi"] + margin) | (H.min(axis=1) < p["T_lo"] - margin)
    idx = np.nonzero(out)[0]
    assert np.all(np.isfinite(H))
    return (int(idx[0]) if idx.size else -1), H


@pytest.mark.parametrize("shape", sorted(SHAPES))
@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_window_reports_the_first_step_outside(shape, prec):
    from paper_1909_03355_amd import FedError, Simulation
    from paper_1909_03355_amd import _lib as L
    p = _leaving_problem()
    n_out, H = _first_out(p, 200)
    assert 5 < n_out < 150, n_out
    with Simulation(p, prec=prec, check_margin=0.0, **SHAPES[shape]) as s:
        s.set_temperature()
        s.step(n_out - 1, graph_steps=10 if shape == "one_step" else None)
        s.temperature()                      # still inside: no error
        assert s.health()["first_bad_step"] == -1
        s.step(200 - (n_out - 1), graph_steps=10 if shape == "one_step" else None)
        with pytest.raises(FedError) as ei:
            s.temperature()
        assert ei.value.code == L.FED_E_UNSTABLE
        h = s.health()
        print(f"{shape} {prec}: oracle leaves [{p['T_lo']}, {p['T_hi']}] at step {n_out}, "
              f"GPU reports step {h['first_bad_step']}", flush=True)
        expect = n_out
        if shape == "resident":
            # resident launches compare the extremes of every step every 32
            # steps (and at the launch's end): the check that covers step n_out
            l0 = n_out - 1                      # steps before the second launch
            expect = l0 + min(-(-(n_out - l0) // 32) * 32, 200 - l0)
        assert h["first_bad_step"] == expect


def test_margin_and_set_range():
    from paper_1909_03355_amd import FedError, Simulation
    from paper_1909_03355_amd import _lib as L
    p = _leaving_problem()
    n_out, H = _first_out(p, 200)
    hi = float(H.max()) - p["T_hi"] + 1.0
    with Simulation(p, prec="fp32c", check_margin=hi) as s:
        s.set_temperature()
        s.step(200)
        s.temperature()
        h = s.health()
        assert h["first_bad_step"] == -1 and h["window_hi"] == p["T_hi"] + hi
    with Simulation(p, prec="fp32c", resident=True, check_margin=0.0) as s:
        s.set_temperature()
        s.step(200)
        with pytest.raises(FedError) as ei:
            s.temperature()
        assert ei.value.code == L.FED_E_UNSTABLE
        # the range the run needs: the record clears, the step is re-checked
        s.set_range(-40.0, float(H.max()) + 1.0)
        T = s.temperature()
        assert s.health()["first_bad_step"] == -1
        assert np.all(np.isfinite(T))


def test_unstable_step_is_flagged_before_it_is_not_finite():
    """dt above the bound on workload 1 (constant properties, where the
    element bound is sharp): the high modes grow; the window, [T_lo, T_hi]
    since the step exceeds the bound, fires long before the values overflow."""
    from paper_1909_03355_amd import FedError, Simulation
    from paper_1909_03355_amd import _lib as L
    p = P.cube_plain(8, 100)
    p["dt"] = 1.5 * float(Oracle(p).dt_crit)
    with Simulation(p, prec="fp32c", allow_unstable=True, tile_nodes=40) as s:
        h = s.health()
        assert (h["window_lo"], h["window_hi"]) == (p["T_lo"], p["T_hi"])
        s.set_temperature()
        s.step(60)
        with pytest.raises(FedError) as ei:
            T = s.temperature()
        assert ei.value.code == L.FED_E_UNSTABLE
        h = s.health()
        print(f"unstable step: left the window at step {h['first_bad_step']}", flush=True)
        assert 0 < h["first_bad_step"] <= 60


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_derived_window_is_where_the_step_stays_stable(prec):
    """By default the window is the widest [T_lo - m, T_hi + m] over which the
    step in use stays within the bound: at its edges the oracle's bound over
    the window equals the step (the window is as wide as it may be and no
    wider)."""
    from paper_1909_03355_amd import Simulation
    p = P.cube_nonlinear_hex(16, 10)
    with Simulation(p, prec=prec) as s:
        h = s.health()
        dt = float(s.dt[0])
    lo, hi = h["window_lo"], h["window_hi"]
    m = p["T_lo"] - lo
    print(f"{prec}: [T_lo, T_hi] = [{p['T_lo']}, {p['T_hi']}], window [{lo:.6g}, {hi:.6g}]",
          flush=True)
    assert m > 0 and abs((hi - p["T_hi"]) - m) < 1e-9 * (1 + m)
    edge = float(Oracle(dict(p, T_lo=lo, T_hi=hi)).dt_crit)
    assert abs(edge - dt) <= 1e-6 * dt
    wider = float(Oracle(dict(p, T_lo=lo - 0.01 * m, T_hi=hi + 0.01 * m)).dt_crit)
    assert wider < dt
    # constant properties without radiation: the bound does not depend on T
    q = P.cube_plain(6, 10)
    with Simulation(q, prec=prec) as s:
        h = s.health()
    assert h["window_lo"] == -np.inf and h["window_hi"] == np.inf


@pytest.mark.parametrize("shape", ["one_step", "resident"])
def test_energy_balance(shape):
    """Energy checks every 25 steps on a run with radiation, convection, a
    flux patch and a Dirichlet face: the residual is at rounding level in
    FP64 and compensated FP32; plain FP32 loses increments below ulp(T)."""
    from paper_1909_03355_amd import FedError, Simulation
    from paper_1909_03355_amd import _lib as L
    p = P.cube_nonlinear_hex(12, 100)
    p["T_lo"], p["T_hi"] = -40.0, 1000.0
    z = p["z"]
    top = np.nonzero(np.isclose(z, z.max()))[0]
    p["dir_nodes"] = top.astype(np.int32)
    p["dir_T"] = np.full(top.size, 30.0)
    res = {}
    for prec in ("fp64", "fp32c", "fp32"):
        with Simulation(p, prec=prec, check_every=25, **SHAPES[shape]) as s:
            s.set_temperature()
            s.step(100)
            s.temperature()
            h = s.health()
            assert h["energy_checks"] == 4
            assert h["energy_step"] in (25, 50, 75, 100)
            res[prec] = h["energy_residual"]
    print(f"{shape}: energy residuals {res}", flush=True)
    assert res["fp64"] < 1e-12
    assert res["fp32c"] < 1e-5
    assert res["fp32"] > 10 * res["fp32c"]
    # a tolerance below the residual turns it into an error
    with Simulation(p, prec="fp32", check_every=25, energy_tol=res["fp32"] / 2,
                    **SHAPES[shape]) as s:
        s.set_temperature()
        s.step(100)
        with pytest.raises(FedError) as ei:
            s.temperature()
        assert ei.value.code == L.FED_E_UNSTABLE


def test_energy_checks_in_graph_replays_and_kept_states():
    from paper_1909_03355_amd import Simulation
    p = P.cube_nonlinear_hex(12, 100)
    p["T_lo"], p["T_hi"] = -40.0, 1000.0
    with Simulation(p, prec="fp32c", check_every=10, tile_nodes=40) as s:
        s.set_temperature()
        s.step(100, graph_steps=20)        # five replays, one check each
        T = s.temperature()
        h = s.health()
        assert h["energy_checks"] == 5 and h["energy_residual"] < 1e-5
    with Simulation(p, prec="fp32c", tile_nodes=40) as s:
        s.set_temperature()
        s.step(100, graph_steps=20)
        assert np.array_equal(s.temperature(), T)   # the checks change nothing
    # kept states of a resident context: the check steps' states are kept too
    g = {}
    for ce in (0, 7):
        with Simulation(p, prec="fp32c", resident=True, check_every=ce) as s:
            s.checkpoint_every(20)
            s.keep_states(True)
            s.set_temperature()
            s.step(100)
            Tk = s.temperature()
            g[ce] = (Tk, s.backward(np.ones_like(Tk))["logk"])
    assert np.array_equal(g[0][0], g[7][0]) and np.array_equal(g[0][1], g[7][1])
