"""Material laws beyond one shared linear k(T): materials with different
(s0, s1) k(T) laws, and shared piecewise-linear multiplier tables for D(T) and
c(T), against the oracle (err_max <= 1e-12 FP64, <= 1e-5 compensated FP32;
gradients 1e-10 / 1e-4), and bitwise across launch shapes, resident stepping
included."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from oracle import Oracle
from tests import helpers as H

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32c": 1e-5}
GTOL = {"fp64": 1e-10, "fp32c": 1e-4}


def _run(p, prec, nsteps, **kw):
    from paper_1909_03355_amd import Simulation
    with Simulation(p, prec=prec, **kw) as s:
        s.set_temperature()
        s.step(nsteps, graph_steps=10)
        return s.temperature()


CASES = {
    "two_material_hex": lambda: H.two_material_problem("hex8"),
    "two_material_tet": lambda: H.two_material_problem("tet4", 4),
    "tables_hex": lambda: H.table_laws(H.two_material_problem("hex8")),
    "tables_tet": lambda: H.table_laws(H.two_material_problem("tet4", 4)),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_laws_match_oracle(case):
    p = CASES[case]()
    nsteps = 80
    o = Oracle(p)
    ref = o.run(nsteps)
    for key in ("k_table", "c_table"):           # the run crosses table kinks
        if key in p:
            Tt = p[key][0]
            assert np.any((Tt > ref.min()) & (Tt < ref.max())), key
    for prec in ("fp64", "fp32c"):
        T = _run(p, prec, nsteps)
        err = oracle.err_max(T, ref)
        print(f"{case} {prec}: err_max {err:.2e}", flush=True)
        assert err <= TOL[prec]
        # other launch shapes give the same bits, resident stepping included
        assert np.array_equal(_run(p, prec, nsteps, fuse_steps=2, tile_nodes=60), T)
        assert np.array_equal(_run(p, prec, nsteps, resident=True), T)


@pytest.mark.parametrize("case", ["two_material_hex", "tables_hex", "tables_tet"])
def test_laws_adjoint_matches_oracle(case):
    from paper_1909_03355_amd import Simulation
    p = CASES[case]()
    nsteps = 40
    o = Oracle(p)
    hist = o.run(nsteps, history=True)
    sens = np.arange(0, o.N, 5)
    lam = np.zeros(o.N)
    lam[sens] = 2.0 * (hist[-1][sens] - 50.0) / sens.size
    ref = o.adjoint(hist, lam)
    rel = lambda a, b: float(np.max(np.abs(a - b)) / np.max(np.abs(b)))
    for prec in ("fp64", "fp32c"):
        grads = []
        for kw in (dict(), dict(resident=True)):
            with Simulation(p, prec=prec, **kw) as s:
                s.checkpoint_every(16)
                s.set_temperature()
                s.step(nsteps)
                grads.append(s.backward(lam))
        g = grads[0]
        errs = {"logk": rel(g["logk"], ref["g_logk"]), "c": rel(g["c"], ref["g_c"]),
                "h": rel(g["h"], ref["g_h"]), "T0": rel(g["T0"], ref["lam0"])}
        print(case, prec, {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
        for k, v in errs.items():
            assert v <= GTOL[prec], (prec, k, v)
        # a resident context (its recompute and, where offered, its adjoint
        # launch) gives the same derivatives bit for bit
        for k in g:
            assert np.array_equal(grads[1][k], g[k]), k
