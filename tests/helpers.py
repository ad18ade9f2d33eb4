"""Small problem builders shared by the tests (inputs only, no method math)."""
from __future__ import annotations

import numpy as np

from workloads import mesh as M, problems as P

GOLDEN = __import__("os").path.join(__import__("os").path.dirname(__file__), "golden")


def single_element(elem, X, mat=None):
    """One element with node coordinates X (ne x 3)."""
    ne = X.shape[0]
    conn = np.arange(ne, dtype=np.int32)[:, None].copy()
    m = dict(elem=elem, x=X[:, 0].copy(), y=X[:, 1].copy(), z=X[:, 2].copy(), conn=conn)
    p = P._base(m, "single")
    p["materials"] = [mat or P.material(rho=1.0, c0=1.0, k=[1.0])]
    p["dt"] = 1e-9
    return p


def distorted_hex(seed=0, amp=0.15):
    """A non-affine hexahedron: unit cube corners jittered."""
    g = np.random.default_rng(seed)
    X = (M.HEX_SIGNS.astype(float) + 1.0) / 2.0
    return X + amp * g.uniform(-1, 1, size=X.shape)


def random_tet(seed=0):
    g = np.random.default_rng(seed)
    X = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float)
    return X + 0.2 * g.uniform(-1, 1, size=X.shape)


def aniso_material(rho=1.0, c0=1.0):
    return P.material(rho=rho, c0=c0, k=[3.0, 2.0, 1.5, 0.4, -0.3, 0.2])


def D_of(mat, s=1.0):
    k = mat["k"]
    return s * np.array([[k[0], k[3], k[5]], [k[3], k[1], k[4]], [k[5], k[4], k[2]]])


def box_problem(elem, n, side=1.0, mat=None, nsteps=1):
    m = M.box_hex(n, n, n, side, side, side) if elem == "hex8" else \
        M.box_tet_kuhn(n, n, n, side, side, side)
    p = P._base(m, f"box_{elem}_{n}")
    p["materials"] = [mat or P.material(rho=1000.0, c0=1000.0, k=[1.0])]
    p["nsteps"] = nsteps
    return p, m


def nonlinear_adjoint_problem(elem):
    """Box with D(T) = Dk (1 + 0.005 T), c(T) = c0 + 2 T, radiation on the top,
    convection on five sides, a Dirichlet side, a point load, per-element k
    factors and a fixed dt at half the critical step."""
    n = 3
    kk = [1.0] if elem == "hex8" else [3.0, 2.0, 1.5, 0.4, -0.3, 0.2]
    mat = P.material(1000.0, 900.0, kk, c1=2.0, s0=1.0, s1=0.005)
    p, m = box_problem(elem, n, side=0.1, mat=mat)
    g = np.random.default_rng(12)
    p["elem_kscale"] = np.exp(0.4 * g.standard_normal(p["conn"].shape[1]))
    if elem == "hex8":
        faces, sides = M.box_side_faces(m)
    else:
        faces = M.boundary_faces(m)
        c = np.stack([m["x"][faces].mean(1), m["y"][faces].mean(1), m["z"][faces].mean(1)], 1)
        sides = np.where(np.isclose(c[:, 0], 0.0), 0, np.where(np.isclose(c[:, 2], 0.1), 5, 1))
    keep = sides != 0
    faces, sides = faces[keep], sides[keep]
    top = sides == 5
    P.set_faces(p, faces, h=g.uniform(5, 30, faces.shape[0]), Ta=20.0,
                eps=np.where(top, 0.8, 0.0), q=np.where(top, 0.0, 500.0))
    left = np.nonzero(np.isclose(m["x"], 0.0))[0].astype(np.int32)
    p["dir_nodes"], p["dir_T"] = left, np.full(left.size, 40.0)
    p["pt_nodes"], p["pt_W"] = np.array([m["x"].size - 1], np.int32), np.array([2.0])
    p["T0"] = g.uniform(150, 300, m["x"].size)
    p["T_lo"], p["T_hi"] = 0.0, 400.0
    from oracle import Oracle
    p["dt"] = 0.5 * Oracle(p).dt_crit
    return p


def two_material_problem(elem="hex8", n=6):
    """Box of two materials with different k(T) laws (s0, s1), c(T) laws and
    densities, split at x = side/2; convection, radiation on the top face, a
    flux on the bottom, random T0."""
    side = 0.1
    m = M.box_hex(n, n, n, side, side, side) if elem == "hex8" else \
        M.box_tet_kuhn(n, n, n, side, side, side)
    p = P._base(m, f"two_material_{elem}")
    p["materials"] = [P.material(2700.0, 880.0, [200.0, 180.0, 150.0], c1=0.4, s0=1.0, s1=-4e-4),
                      P.material(7800.0, 460.0, [40.0], c1=0.25, s0=0.8, s1=2e-3)]
    cx = m["x"][m["conn"]].mean(axis=0)
    p["elem_material"] = (cx > side / 2).astype(np.int32)
    faces = M.boundary_faces(m)
    cz = m["z"][faces].mean(axis=1)
    top, bottom = np.isclose(cz, side), np.isclose(cz, 0.0)
    P.set_faces(p, faces, h=12.0, Ta=25.0, eps=np.where(top, 0.7, 0.0),
                q=np.where(bottom, 4e4, 0.0))
    p["T0"] = np.random.default_rng(31).uniform(20.0, 80.0, m["x"].size)
    p["T_lo"], p["T_hi"] = 0.0, 400.0
    return p


def table_laws(p):
    """The same problem with kinked multiplier tables for D and c instead of
    linear laws (materials with s0 = 1, s1 = 0, c1 = 0)."""
    q = dict(p)
    q["materials"] = [dict(m, s0=1.0, s1=0.0, c1=0.0) for m in p["materials"]]
    q["elem_material"] = p["elem_material"]
    q["k_table"] = (np.array([0.0, 40.0, 55.0, 120.0, 400.0]),
                    np.array([1.0, 1.3, 0.9, 1.6, 2.0]))
    q["c_table"] = (np.array([10.0, 35.0, 60.0, 90.0]), np.array([0.8, 1.1, 1.4, 1.2]))
    return q
