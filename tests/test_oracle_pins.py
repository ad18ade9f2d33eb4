"""Pins of the FP64 oracle against things other than itself: brute force on
tiny inputs (finite differences of the interpolant, dense assembly), closed
forms (1-D FTCS reduction, Fourier series, 7-point Laplacian, critical step),
invariants (energy balance, constants, hourglass modes) and the paper's patch
tests (Sec. 4.1, geometry of Fig. 2(c)).  CPU only."""
from __future__ import annotations

import os

import numpy as np
import pytest

import oracle
from oracle import Oracle
from tests import helpers as H
from workloads import mesh as M, problems as P

SIG = 5.67e-8


# ----------------------------------------------------------------------------
# brute force: the element load from finite differences of the interpolant
def _trilinear(V, xi):
    N = np.prod(1.0 + M.HEX_SIGNS * np.asarray(xi), axis=1) / 8.0
    return N @ V


def hex_energy(X, T, D):
    """8 det J(0) gradT(0)^T D gradT(0), with J and the natural gradient of T
    at the centre taken by central differences of the trilinear interpolant
    (exact for a trilinear map)."""
    h = 0.25
    J = np.zeros((3, 3))
    gxi = np.zeros(3)
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        J[:, j] = (_trilinear(X, e) - _trilinear(X, -e)) / (2 * h)
        gxi[j] = (_trilinear(T[:, None], e) - _trilinear(T[:, None], -e))[0] / (2 * h)
    g = np.linalg.solve(J.T, gxi)
    return 8.0 * np.linalg.det(J) * g @ D @ g


def tet_energy(X, T, D):
    """V gradT^T D gradT with the plane through the four values solved
    directly and V from the determinant of the edge vectors."""
    A = np.hstack([X, np.ones((4, 1))])
    coef = np.linalg.solve(A, T)
    g = coef[:3]
    V = abs(np.linalg.det(X[1:] - X[0])) / 6.0
    return V * g @ D @ g


def fd_load(energy, X, T, D):
    """F = d/dT (1/2 T^T K T): central differences of an exact quadratic."""
    F = np.zeros(T.size)
    for a in range(T.size):
        d = np.zeros(T.size)
        d[a] = 0.5
        F[a] = (energy(X, T + d, D) - energy(X, T - d, D)) / (4 * 0.5)
    return F


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("elem", ["hex8", "tet4"])
def test_element_load_bruteforce(elem, seed):
    mat = H.aniso_material()
    X = H.distorted_hex(seed) if elem == "hex8" else H.random_tet(seed)
    p = H.single_element(elem, X, mat)
    o = Oracle(p)
    T = np.random.default_rng(seed + 10).uniform(-5, 5, X.shape[0])
    F, _ = o.loads(T)
    energy = hex_energy if elem == "hex8" else tet_energy
    D = H.D_of(mat)
    Fb = fd_load(energy, X, T, D)
    assert np.max(np.abs(F - Fb)) <= 1e-11 * np.max(np.abs(Fb))
    # the quadratic form itself, and symmetry / constants in the null space
    assert abs(T @ F - energy(X, T, D)) <= 1e-11 * abs(energy(X, T, D))
    F1, _ = o.loads(np.full(X.shape[0], 3.7))
    assert np.max(np.abs(F1)) < 1e-12


def _dense_step(p, T, cfun, sfun, dt):
    """One explicit step assembled densely from brute-force element matrices:
    K_e from the polarised quadratic form, lumped capacity from independent
    volumes, convection from face areas of the axis-aligned box."""
    X = np.stack([p["x"], p["y"], p["z"]], axis=1)
    N = X.shape[0]
    conn = p["conn"]
    ne = conn.shape[0]
    energy = hex_energy if ne == 8 else tet_energy
    mat = p["materials"][0]
    K = np.zeros((N, N))
    Cap = np.zeros(N)
    for e in range(conn.shape[1]):
        idx = conn[:, e]
        Xe = X[idx]
        D = H.D_of(mat, sfun(T[idx].mean()))
        Ke = np.zeros((ne, ne))
        for a in range(ne):
            for b in range(ne):
                ea, eb = np.eye(ne)[a], np.eye(ne)[b]
                Ke[a, b] = (energy(Xe, ea + eb, D) - energy(Xe, ea - eb, D)) / 4.0
        K[np.ix_(idx, idx)] += Ke
        if ne == 8:
            vol = np.prod(Xe.max(0) - Xe.min(0))
        else:
            vol = abs(np.linalg.det(Xe[1:] - Xe[0])) / 6.0
        Cap[idx] += mat["rho"] * vol / ne * cfun(T[idx])
    Q = np.zeros(N)
    for f, fa in enumerate(p["faces"]):
        Xf = X[fa]
        if fa.size == 4:
            area = np.linalg.norm(np.cross(Xf[1] - Xf[0], Xf[3] - Xf[0]))
        else:
            area = 0.5 * np.linalg.norm(np.cross(Xf[1] - Xf[0], Xf[2] - Xf[0]))
        for k in fa:
            Q[k] += area / fa.size * (-p["face_h"][f] * (T[k] - p["face_Ta"][f])
                                      - SIG * p["face_eps"][f] * ((T[k] - p["Tz"]) ** 4
                                                                   - (p["face_Ta"][f] - p["Tz"]) ** 4)
                                      + p["face_q"][f])
    return T + dt * (Q - K @ T) / Cap


@pytest.mark.parametrize("elem", ["hex8", "tet4"])
def test_one_step_dense(elem):
    mat = P.material(rho=900.0, c0=800.0, c1=1.5, k=[3.0, 2.0, 1.5, 0.4, -0.3, 0.2],
                     s0=1.0, s1=0.004)
    p, m = H.box_problem(elem, 2, side=0.1, mat=mat)
    faces, sides = M.box_side_faces(m)
    P.set_faces(p, faces, h=np.where(sides % 2 == 0, 12.0, 7.0), Ta=15.0,
                eps=np.where(sides == 5, 0.7, 0.0), q=np.where(sides == 4, 500.0, 0.0))
    p["T0"] = np.random.default_rng(3).uniform(20, 60, m["x"].size)
    p["T_lo"], p["T_hi"] = 0.0, 100.0
    o = Oracle(p)
    T1 = o.run(1)
    ref = _dense_step(p, o.initial(), lambda T: 800.0 + 1.5 * T,
                      lambda Tb: 1.0 + 0.004 * Tb, o.dt[0])
    assert np.max(np.abs(T1 - ref)) <= 1e-12 * np.max(np.abs(ref))


# ----------------------------------------------------------------------------
# geometry closed forms
def test_areas_and_mass_totals():
    for elem in ("hex8", "tet4"):
        p, m = H.box_problem(elem, 3, side=0.2)
        faces, _ = M.box_side_faces(m)
        P.set_faces(p, faces)
        o = Oracle(p)
        assert abs(o.farea.sum() - 6 * 0.04) < 1e-15
        assert abs(o.V.sum() - 0.008) < 1e-16
        _, Cap = o.loads(np.zeros(o.N))
        assert abs(Cap.sum() - 1000.0 * 1000.0 * 0.008) < 1e-8


def test_patch_volumes():
    """The 16-node patch of Fig. 2(c) tiles the unit cube: exact element
    volumes add to 1 for both meshes.  For the distorted hexahedra the one-point
    weight 8 det J(0) does not (the reason the mass uses the exact volume)."""
    x, y, z = M.patch_nodes(os.path.join(H.GOLDEN, "patch_nodes.txt"))
    for mesh in (M.patch_hex(x, y, z), M.patch_tet(x, y, z)):
        p = P._base(mesh, "patch")
        p["materials"] = [P.material(1.0, 1.0, [1.0])]
        o = Oracle(p)
        assert o.n_bad == 0
        assert abs(o.V.sum() - 1.0) < 1e-13
    oh = Oracle(dict(P._base(M.patch_hex(x, y, z), "ph"), materials=[P.material(1, 1, [1])]))
    assert abs(oh.W.sum() - 1.0) > 1e-3
    # mass conservation (Sec. 3.1): the lumped capacity of the distorted
    # patch adds up to rho c times the cube's volume
    ph = dict(P._base(M.patch_hex(x, y, z), "ph"), materials=[P.material(700.0, 900.0, [1])])
    _, Cap = Oracle(ph).loads(np.zeros(16))
    assert abs(Cap.sum() - 700.0 * 900.0) < 1e-9


# ----------------------------------------------------------------------------
# patch tests (Sec. 4.1): a linear field imposed on the boundary is reproduced
def _relax(o, T, tol=1e-12, chunk=2000, maxit=200):
    for _ in range(maxit):
        Tn = o.run(chunk, T0=T, apply_initial=False)
        if np.max(np.abs(Tn - T)) < tol:
            return Tn
        T = Tn
    return T


def _linear_patch(p, bnodes, lin):
    p["dir_nodes"] = bnodes.astype(np.int32)
    p["dir_T"] = lin[bnodes]
    p["T0"] = np.zeros(lin.size)
    o = Oracle(p)
    return o, _relax(o, o.initial())


def test_patch_tet_paper_geometry():
    x, y, z = M.patch_nodes(os.path.join(H.GOLDEN, "patch_nodes.txt"))
    mesh = M.patch_tet(x, y, z)
    p = P._base(mesh, "patch_tet")
    p["materials"] = [P.material(1.0, 1.0, [1.0])]
    lin = 200 * x + 100 * y + 200 * z          # the field of Sec. 4.1
    o, T = _linear_patch(p, np.arange(8), lin)
    assert np.max(np.abs(T - lin)) < 1e-9


@pytest.mark.parametrize("elem", ["hex8", "tet4"])
def test_patch_anisotropic_affine_grid(elem):
    """Linear fields solve div(D grad T) = 0 for any constant D, so both
    element types must reproduce them on an affinely mapped grid."""
    n = 3
    m = M.box_hex(n, n, n) if elem == "hex8" else M.box_tet_kuhn(n, n, n)
    A = np.array([[1.0, 0.3, 0.1], [0.0, 0.9, 0.2], [0.1, 0.0, 1.1]])
    X = np.stack([m["x"], m["y"], m["z"]], 1) @ A.T
    m = dict(m, x=X[:, 0].copy(), y=X[:, 1].copy(), z=X[:, 2].copy())
    p = P._base(m, "affine")
    p["materials"] = [H.aniso_material()]
    lin = 200 * m["x"] + 100 * m["y"] + 200 * m["z"] + 7.0
    o, T = _linear_patch(p, M.boundary_nodes(m), lin)
    assert np.max(np.abs(T - lin)) < 1e-8


def test_patch_distorted_hex_known_result():
    """Recorded known result: with the literal one-point centre-B hexahedron
    (Eq. 17) the distorted 7-element patch does NOT reproduce the linear field
    exactly: the interior rows of K T_lin are not zero."""
    x, y, z = M.patch_nodes(os.path.join(H.GOLDEN, "patch_nodes.txt"))
    p = P._base(M.patch_hex(x, y, z), "patch_hex")
    p["materials"] = [P.material(1.0, 1.0, [1.0])]
    o = Oracle(p)
    lin = 200 * x + 100 * y + 200 * z
    F, _ = o.loads(lin)
    assert np.max(np.abs(F[8:])) > 1.0


# ----------------------------------------------------------------------------
# uniform-gradient (element-mean) hexahedron
def _mean_gradient_numpy(X, order=4):
    """(1/V) integral of the gradient operator over a trilinear hexahedron by
    an order-4 Gauss rule, with J from the interpolant's derivatives at each
    point (independent of the oracle's 2x2x2 rule); returns (Bbar 3x8, V)."""
    xg, wg = np.polynomial.legendre.leggauss(order)
    S = M.HEX_SIGNS.astype(float)
    acc, vol = np.zeros((3, 8)), 0.0
    for a_, wa in zip(xg, wg):
        for b_, wb in zip(xg, wg):
            for c_, wc in zip(xg, wg):
                p = np.array([a_, b_, c_])
                dN = np.empty((8, 3))
                for j in range(3):
                    others = [k for k in range(3) if k != j]
                    dN[:, j] = S[:, j] * np.prod(1.0 + S[:, others] * p[others], axis=1) / 8.0
                J = X.T @ dN
                d = np.linalg.det(J)
                acc += wa * wb * wc * d * np.linalg.solve(J.T, dN.T)
                vol += wa * wb * wc * d
    return acc / vol, vol


def test_mean_gradient_hex_against_higher_order_quadrature():
    """The oracle's element-mean gradient (exact 2x2x2 rule) equals an
    order-4 Gauss integration of the gradient operator on distorted
    hexahedra, and satisfies sum_a b_a = 0, sum_a b_a x_a^T = I."""
    for seed in range(4):
        X = H.distorted_hex(seed, amp=0.2)
        p = H.single_element("hex8", X)
        p["hex_gradient"] = "mean"
        o = Oracle(p)
        Bref, Vref = _mean_gradient_numpy(X)
        B = o.B.reshape(3, 8)
        assert np.max(np.abs(B - Bref)) < 1e-12 * np.max(np.abs(Bref))
        assert abs(o.V[0] - Vref) < 1e-13 and abs(o.W[0] - Vref) < 1e-13
        assert np.max(np.abs(B.sum(1))) < 1e-12
        assert np.max(np.abs(B @ X - np.eye(3))) < 1e-12


def test_mean_gradient_equals_centre_on_affine_grids():
    """On parallelepipeds the gradient is constant, so the mean-gradient run
    equals the centre-point run of Eq. 17 to rounding."""
    n = 4
    m = M.box_hex(n, n, n, 0.1, 0.1, 0.1)
    A = np.array([[1.0, 0.3, 0.1], [0.0, 0.9, 0.2], [0.1, 0.0, 1.1]])
    X = np.stack([m["x"], m["y"], m["z"]], 1) @ A.T
    m = dict(m, x=X[:, 0].copy(), y=X[:, 1].copy(), z=X[:, 2].copy())
    p = P._base(m, "affine_mean")
    p["materials"] = [H.aniso_material(rho=1000.0, c0=900.0)]
    p["T0"] = np.random.default_rng(2).uniform(0, 100, X.shape[0])
    a = Oracle(p).run(50)
    b = Oracle(dict(p, hex_gradient="mean")).run(50)
    assert np.max(np.abs(a - b)) < 1e-11 * np.max(np.abs(a))


def test_patch_distorted_hex_mean_gradient():
    """Sec. 4.1's patch test on the distorted 7-hexahedron patch of Fig. 2(c),
    which the centre-point hexahedron fails: the mean-gradient hexahedron
    reproduces the linear field."""
    x, y, z = M.patch_nodes(os.path.join(H.GOLDEN, "patch_nodes.txt"))
    p = P._base(M.patch_hex(x, y, z), "patch_hex_mean")
    p["materials"] = [P.material(1.0, 1.0, [1.0])]
    p["hex_gradient"] = "mean"
    lin = 200 * x + 100 * y + 200 * z
    F, _ = Oracle(p).loads(lin)
    assert np.max(np.abs(F[8:])) < 1e-10
    o, T = _linear_patch(p, np.arange(8), lin)
    assert np.max(np.abs(T - lin)) < 1e-9


def _hg_cube(eps, h=0.5, k=2.0):
    X = (M.HEX_SIGNS.astype(float) + 1.0) / 2.0 * h
    p = H.single_element("hex8", X, P.material(rho=3.0, c0=5.0, k=[k]))
    p["hex_gradient"] = "mean"
    p["hourglass"] = eps
    return p


def test_hourglass_cube_closed_form():
    """Hourglass control on a cube of side h: gamma_alpha = h_alpha / 8 and
    kappa = 1.5 eps k h, so a pure hourglass field h_alpha gets the load
    kappa h_alpha / 8, a linear field gets nothing from the term, and the
    element's largest eigenvalue is max(k h / 2, kappa / 8) (the ranges of
    the mean-gradient and hourglass parts are orthogonal on a cube), which
    fixes the critical step 2 (rho c V / 8) / lambda."""
    h, k = 0.5, 2.0
    S = M.HEX_SIGNS.astype(float)
    pats = [S[:, 1] * S[:, 2], S[:, 2] * S[:, 0], S[:, 0] * S[:, 1], S[:, 0] * S[:, 1] * S[:, 2]]
    X = (S + 1.0) / 2.0 * h
    lin = 3.0 * X[:, 0] - 2.0 * X[:, 1] + X[:, 2]
    F0, _ = Oracle(_hg_cube(0.0, h, k)).loads(lin)
    for eps in (0.5, 4.0):
        o = Oracle(_hg_cube(eps, h, k))
        kap = 1.5 * eps * k * h
        for hp in pats:
            F, _ = o.loads(hp)
            assert np.max(np.abs(F - kap * hp / 8.0)) < 1e-12 * kap
        F, _ = o.loads(lin)
        assert np.max(np.abs(F - F0)) < 1e-12 * np.max(np.abs(F0))
        lam = max(k * h / 2.0, kap / 8.0)
        dt = 2.0 * (3.0 * 5.0 * h ** 3 / 8.0) / lam
        assert abs(o.dt_crit - dt) < 1e-12 * dt


def test_hourglass_mode_decays_only_with_control():
    """The checkerboard (-1)^(i+j+k) is a pure hourglass field in every
    hexahedron of a box grid: the uniform-gradient element leaves it fixed,
    the hourglass term damps it (every step lowers its amplitude)."""
    n = 4
    k, j, i = np.meshgrid(np.arange(n + 1), np.arange(n + 1), np.arange(n + 1), indexing="ij")
    for eps in (0.0, 0.3):
        p, m = H.box_problem("hex8", n, side=1.0)
        p["hex_gradient"] = "mean"
        p["hourglass"] = eps
        p["T0"] = ((-1.0) ** (i + j + k)).ravel() * 5.0
        hist = Oracle(p).run(20, history=True)
        amp = np.max(np.abs(hist), axis=1)
        if eps == 0.0:
            assert np.max(np.abs(hist[-1] - p["T0"])) < 1e-12
        else:
            assert np.all(np.diff(amp) < 0) and amp[-1] < 0.9 * amp[0]


def test_hourglass_keeps_the_distorted_patch_test():
    """gamma vanishes on linear fields on any hexahedron: with the hourglass
    term on, the distorted patch of Fig. 2(c) still reproduces the linear
    field exactly."""
    x, y, z = M.patch_nodes(os.path.join(H.GOLDEN, "patch_nodes.txt"))
    p = P._base(M.patch_hex(x, y, z), "patch_hex_hg")
    p["materials"] = [P.material(1.0, 1.0, [1.0])]
    p["hex_gradient"] = "mean"
    p["hourglass"] = 0.5
    lin = 200 * x + 100 * y + 200 * z
    F, _ = Oracle(p).loads(lin)
    assert np.max(np.abs(F[8:])) < 1e-10
    o, T = _linear_patch(p, np.arange(8), lin)
    assert np.max(np.abs(T - lin)) < 1e-9


# ----------------------------------------------------------------------------
# workload 1 reduces to 1-D FTCS at every step (exact identity)
def test_cube_plain_equals_ftcs():
    p = P.cube_plain(10, 1000)
    o = Oracle(p)
    assert abs(o.dt_crit - 5000.0) < 1e-9          # rho c h^2 / (2 k)
    hist = o.run(1000, history=True)
    r = o.dt[0] * 1.0 / (1000.0 * 1000.0) / 0.01
    u = np.zeros(11)
    u[10] = 100.0
    lev = np.rint(p["z"] * 10).astype(int)
    worst = 0.0
    for n in range(1, 1001):
        un = u.copy()
        un[0] = u[0] + r * 2 * (u[1] - u[0])      # insulated: mirror node
        un[1:10] = u[1:10] + r * (u[:9] - 2 * u[1:10] + u[2:11])
        u = un
        if n in (1, 10, 100, 1000):
            worst = max(worst, np.max(np.abs(hist[n] - u[lev])))
    assert worst < 1e-11


def fourier(z, at, terms=400):
    m = np.arange(terms)[:, None]
    lam = (2 * m + 1) * np.pi / 2
    s = ((-1.0) ** m / (2 * m + 1)) * np.cos(lam * z[None, :]) * np.exp(-lam ** 2 * at)
    return 100.0 - (400.0 / np.pi) * s.sum(0)


def test_fourier_convergence():
    """Continuum check: T = 100 - (400/pi) sum (-1)^m/(2m+1) cos(..) exp(..)
    at alpha t = 0.45 with r = 0.45 fixed; the error falls ~4x per halving."""
    errs = []
    for n in (10, 20, 40):
        m = M.box_hex(1, 1, n, 1.0 / n, 1.0 / n, 1.0)
        p = P._base(m, "col")
        p["materials"] = [P.material(1000.0, 1000.0, [1.0])]
        top = np.nonzero(np.isclose(m["z"], 1.0))[0].astype(np.int32)
        p["dir_nodes"], p["dir_T"] = top, np.full(top.size, 100.0)
        o = Oracle(p)
        steps = n * n                               # alpha t = steps r h^2 = 0.45
        T = o.run(steps)
        alpha_t = steps * o.dt[0] * 1e-6
        assert abs(alpha_t - 0.45) < 1e-12
        errs.append(np.max(np.abs(T - fourier(m["z"], alpha_t))))
    assert errs[0] < 0.3
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5


# ----------------------------------------------------------------------------
# invariants
def test_energy_balance_nonlinear():
    """Insulated, nonlinear c(T) and D(T), point sources: the heat stored in a
    step, sum_k C_k(T^n) (T^{n+1}_k - T^n_k), equals dt * sum of the inputs."""
    mat = P.material(rho=1000.0, c0=1000.0, c1=2.0, k=[1.0, 2.0, 0.5], s0=1.0, s1=0.005)
    for elem in ("hex8", "tet4"):
        p, m = H.box_problem(elem, 4, side=0.1, mat=mat)
        g = np.random.default_rng(5)
        p["T0"] = g.uniform(20, 80, m["x"].size)
        p["pt_nodes"] = np.array([3, 17, 40], np.int32)
        p["pt_W"] = np.array([2.0, 1.0, 0.5])
        p["T_lo"], p["T_hi"] = 0.0, 200.0
        o = Oracle(p)
        T0 = o.initial()
        T1 = o.run(1)
        n_inc = np.bincount(m["conn"].ravel(), minlength=m["x"].size)
        vol = 0.1 ** 3 / m["conn"].shape[1]
        Cap = 1000.0 * vol / m["conn"].shape[0] * n_inc * (1000.0 + 2.0 * T0)
        stored = np.sum(Cap * (T1 - T0))
        assert abs(stored - o.dt[0] * 3.5) < 1e-10 * abs(stored)


def test_point_schedule_energy_and_location():
    """Scheduled point loads (row (step0 + n) mod n_rows at step n), insulated
    box with nonlinear c(T) and D(T): every step stores dt times the total of
    its own row (rows with distinct totals, the table wrapping twice, two
    values of step0), and the first two steps from a uniform field raise only
    the nodes their rows load, by dt W / C (the second row's node is not a
    neighbour of the first's, so no conduction reaches it yet)."""
    mat = P.material(rho=1000.0, c0=1000.0, c1=2.0, k=[1.0, 2.0, 0.5], s0=1.0, s1=0.005)
    p, m = H.box_problem("hex8", 4, side=0.1, mat=mat)
    nodes = np.array([3, 17, 40, 77], np.int32)      # (3,0,0) (2,3,0) (0,3,1) (2,0,3)
    p["pt_nodes"], p["pt_W"] = nodes, np.zeros(4)
    p["T_lo"], p["T_hi"] = 0.0, 200.0
    W = np.array([[2.0, 0.0, 0.0, 0.0], [0.0, 3.0, 0.0, 0.0], [0.0, 0.0, 1.0, 3.0]])
    n_inc = np.bincount(m["conn"].ravel(), minlength=m["x"].size)
    cap = 1000.0 * 0.1 ** 3 / m["conn"].shape[1] / 8 * n_inc
    for step0 in (0, 2):
        p["T0"] = np.random.default_rng(6).uniform(20, 80, m["x"].size)
        o = Oracle(p)
        hist = o.run(7, history=True, pt_schedule=W, step0=step0)
        for n in range(7):
            stored = np.sum(cap * (1000.0 + 2.0 * hist[n]) * (hist[n + 1] - hist[n]))
            total = W[(step0 + n) % 3].sum()
            assert abs(stored - o.dt[0] * total) < 1e-10 * abs(stored)
    p["T0"] = np.full(m["x"].size, 30.0)
    o = Oracle(p)
    hist = o.run(2, history=True, pt_schedule=W)
    C30 = cap * (1000.0 + 2.0 * 30.0)
    d1 = hist[1] - hist[0]
    assert np.max(np.abs(np.delete(d1, 3))) < 1e-12
    assert abs(d1[3] - o.dt[0] * 2.0 / C30[3]) < 1e-12 * d1[3]
    d2 = hist[2] - hist[1]
    assert abs(d2[17] - o.dt[0] * 3.0 / C30[17]) < 1e-12 * d2[17]
    # a one-row schedule is the fixed loads of that row
    p["pt_W"] = W[2]
    assert np.array_equal(Oracle(p).run(3), Oracle(p).run(3, pt_schedule=W[2:]))


def test_constant_field_is_fixed_point():
    mat = P.material(rho=1000.0, c0=1000.0, c1=2.0, k=[1.0, 2.0, 0.5], s0=1.0, s1=0.005)
    for elem in ("hex8", "tet4"):
        p, m = H.box_problem(elem, 3, side=0.1, mat=mat)
        p["T0"] = np.full(m["x"].size, 42.0)
        p["T_lo"], p["T_hi"] = 0.0, 100.0
        T1 = Oracle(p).run(3)
        assert np.max(np.abs(T1 - 42.0)) < 1e-11


def test_hourglass_mode_is_fixed_point():
    """(-1)^(i+j+k) has zero centre gradient in every hexahedron (Eq. 17
    integrates at the centre only), so it is not damped at all."""
    p, m = H.box_problem("hex8", 4, side=1.0)
    n = 4
    k, j, i = np.meshgrid(np.arange(n + 1), np.arange(n + 1), np.arange(n + 1), indexing="ij")
    p["T0"] = ((-1.0) ** (i + j + k)).ravel() * 5.0
    T1 = Oracle(p).run(5)
    assert np.max(np.abs(T1 - p["T0"])) < 1e-12


def test_kuhn_tets_give_seven_point_laplacian():
    """Isotropic Kuhn tetrahedra on a regular grid: every interior row of K is
    k h (6, -1 x 6) and the lumped mass is rho c h^3, i.e. one explicit step
    is the 7-point finite-difference Laplacian update."""
    n, side = 4, 0.4
    h = side / n
    p, m = H.box_problem("tet4", n, side=side, mat=P.material(1000.0, 1000.0, [2.0]))
    g = np.random.default_rng(9)
    T = g.uniform(0, 10, m["x"].size)
    p["T0"] = T
    o = Oracle(p)
    T1 = o.run(1)
    Tg = T.reshape(n + 1, n + 1, n + 1)
    lap = (Tg[2:, 1:-1, 1:-1] + Tg[:-2, 1:-1, 1:-1] + Tg[1:-1, 2:, 1:-1] + Tg[1:-1, :-2, 1:-1]
           + Tg[1:-1, 1:-1, 2:] + Tg[1:-1, 1:-1, :-2] - 6 * Tg[1:-1, 1:-1, 1:-1])
    expect = Tg[1:-1, 1:-1, 1:-1] + o.dt[0] * 2.0 * h * lap / (1000.0 * 1000.0 * h ** 3)
    got = T1.reshape(n + 1, n + 1, n + 1)[1:-1, 1:-1, 1:-1]
    assert np.max(np.abs(got - expect)) < 1e-12


def test_critical_step_is_sharp():
    """Eq. 29: the x-checkerboard is the fastest mode of the one-point
    hexahedral grid; 1.01 dt_crit amplifies it, 0.99 dt_crit damps it."""
    n = 8
    amps = []
    for f in (0.99, 1.01):
        p, m = H.box_problem("hex8", n, side=1.0)
        p["T0"] = ((-1.0) ** np.rint(m["x"] * n)) * 1.0
        o = Oracle(p)
        p["dt"] = f * o.dt_crit
        o = Oracle(p)
        amps.append(np.max(np.abs(o.run(400))))
    assert amps[0] < 0.5 and amps[1] > 2.0


def test_single_hex_boundary_recursion():
    """One hexahedron with convection and radiation on all faces and a uniform
    temperature: F = 0, every node carries area 3 a^2 / 4 and capacity
    rho c a^3 / 8, so all nodes follow the scalar explicit-Euler recursion."""
    a, h, eps, Ta, rho, c = 0.05, 25.0, 0.6, 10.0, 2000.0, 500.0
    m = M.box_hex(1, 1, 1, a, a, a)
    p = P._base(m, "one")
    p["materials"] = [P.material(rho, c, [5.0])]
    faces, _ = M.box_side_faces(m)
    P.set_faces(p, faces, h=h, Ta=Ta, eps=eps)
    p["T0"] = np.full(8, 300.0)
    p["T_lo"], p["T_hi"] = 0.0, 300.0
    o = Oracle(p)
    T = 300.0
    A, Cap = 3 * a * a / 4, rho * c * a ** 3 / 8
    for _ in range(50):
        T = T + o.dt[0] / Cap * A * (-h * (T - Ta) - SIG * eps * ((T + 273.15) ** 4 - (Ta + 273.15) ** 4))
    assert np.max(np.abs(o.run(50) - T)) < 1e-11 * T


@pytest.mark.parametrize("s1,c1", [(0.004, 2.0), (-0.0006, -0.5), (-0.0006, 2.0), (0.004, -0.5)])
def test_critical_step_closed_form_with_boundary_and_range(s1, c1):
    """Eq. 29 with the element bound and the boundary rate of Sec. 2 (Eq. 4,
    7), in closed form for one cube of side a, k(T) = k (s0 + s1 T),
    c(T) = c0 + c1 T, convection and radiation on all six faces.  The
    one-point hexahedron's K_e = (k a / 16) sum_i s_i s_i^T has largest
    eigenvalue k a / 2; each node carries capacity rho c a^3 / 8 and area
    3 a^2 / 4, so
        lambda_e = 4 k s_max / (rho c_min a^2),
        lambda_k = (h + 4 sigma eps (T_hi - Tz)^3) 6 / (rho c_min a),
    with s_max and c_min the extremes over [T_lo, T_hi]: at T_hi or T_lo
    depending on the signs of the slopes."""
    a, k, rho, c0, h, eps, Ta = 0.02, 10.0, 2500.0, 700.0, 80.0, 0.9, 15.0
    T_lo, T_hi, Tz = 10.0, 900.0, -273.15
    m = M.box_hex(1, 1, 1, a, a, a)
    p = P._base(m, "one_dt")
    p["materials"] = [P.material(rho, c0, [k], c1=c1, s0=1.0, s1=s1)]
    faces, _ = M.box_side_faces(m)
    P.set_faces(p, faces, h=h, Ta=Ta, eps=eps)
    p["T_lo"], p["T_hi"], p["Tz"] = T_lo, T_hi, Tz
    s_max = max(1.0 + s1 * T_lo, 1.0 + s1 * T_hi)
    c_min = min(c0 + c1 * T_lo, c0 + c1 * T_hi)
    lam_e = 4.0 * k * s_max / (rho * c_min * a * a)
    lam_k = (h + 4.0 * SIG * eps * (T_hi - Tz) ** 3) * 6.0 / (rho * c_min * a)
    assert 0.1 * lam_e < lam_k < 10.0 * lam_e      # both terms matter
    assert Oracle(p).dt_crit == pytest.approx(2.0 / (lam_e + lam_k), rel=1e-12)


def test_twisted_quad_face_area():
    """Face areas of bilinear quadrilaterals: on a hexahedron whose top face
    is twisted (one corner lifted by 0.6 of the side), the 2x2 Gauss rule of
    |x_u x x_v| is within 2e-4 of a 40x40 Gauss-Legendre reference (a rule
    with misplaced points, or the centre point alone, misses by >= 2e-3); the
    planar faces are exact against the diagonal cross-product area."""
    m = M.box_hex(1, 1, 1, 1.0, 1.0, 1.0)
    top = np.nonzero((m["x"] > 0.5) & (m["y"] > 0.5) & (m["z"] > 0.5))[0]
    m["z"] = m["z"].copy()
    m["z"][top] = 1.6
    p = P._base(m, "twist")
    p["materials"] = [P.material(1000.0, 1000.0, [1.0])]
    faces, _ = M.box_side_faces(m)
    P.set_faces(p, faces, h=1.0, Ta=0.0)
    o = Oracle(p)
    X = np.stack([m["x"], m["y"], m["z"]], 1)
    su, sv = np.array([-1.0, 1.0, 1.0, -1.0]), np.array([-1.0, -1.0, 1.0, 1.0])
    x, w = np.polynomial.legendre.leggauss(40)
    n_twisted = 0
    for f, fa in enumerate(faces):
        Xf = X[fa]
        planar = abs(np.dot(np.cross(Xf[1] - Xf[0], Xf[3] - Xf[0]), Xf[2] - Xf[0])) < 1e-14
        if planar:
            ref = 0.5 * np.linalg.norm(np.cross(Xf[2] - Xf[0], Xf[3] - Xf[1]))
            assert o.farea[f] == pytest.approx(ref, rel=1e-13)
            continue
        n_twisted += 1
        ref = 0.0
        for u, wu in zip(x, w):
            for v, wv in zip(x, w):
                xu = (su * (1 + sv * v) / 4) @ Xf
                xv = (sv * (1 + su * u) / 4) @ Xf
                ref += wu * wv * np.linalg.norm(np.cross(xu, xv))
        assert abs(o.farea[f] - ref) <= 2e-4 * ref
    assert n_twisted == 1


# ----------------------------------------------------------------------------
# piecewise-linear property tables (shared multipliers of D and c)
def _table_problem(elem="hex8"):
    p = H.nonlinear_adjoint_problem(elem)
    p["materials"] = [dict(m, s0=1.0, s1=0.0, c1=0.0) for m in p["materials"]]
    return p


def test_tables_equal_to_linear_laws_reproduce_them():
    """A two-point k table on s0 + s1 T and a c table on 1 + (c1/c0) T, both
    spanning the temperatures, give the linear-law run to rounding."""
    lin = H.nonlinear_adjoint_problem("hex8")
    m = lin["materials"][0]
    Tt = np.array([-500.0, 1500.0])
    tab = dict(_table_problem(), k_table=(Tt, m["s0"] + m["s1"] * Tt),
               c_table=(Tt, 1.0 + m["c1"] / m["c0"] * Tt))
    a, b = Oracle(lin).run(40), Oracle(tab).run(40)
    assert np.max(np.abs(a - b)) < 1e-11 * np.max(np.abs(a))


def test_table_segment_selection_and_clamping():
    """Temperatures inside one segment of a kinked table follow that segment's
    linear law; a table lying entirely below the temperatures acts as its last
    value (clamped), one above them as its first."""
    p = _table_problem()
    o = Oracle(p)
    assert o.initial().min() >= 40.0      # T0 in [150, 300], Dirichlet side 40
    Tt = np.array([-100.0, 20.0, 1000.0, 2000.0])
    f = np.array([0.4, 1.0, 1.0 + 0.004 * 980.0, 9.0])   # slope 0.004 on [20, 1000]
    seg = Oracle(dict(p, materials=[dict(p["materials"][0], s0=1.0 - 0.004 * 20.0, s1=0.004)]))
    got = Oracle(dict(p, k_table=(Tt, f))).run(30)
    ref = seg.run(30)
    assert 20.0 < ref.min() and ref.max() < 1000.0   # the run stays in the [20, 1000] segment
    assert np.max(np.abs(got - ref)) < 1e-11 * np.max(np.abs(ref))
    for Tt2, f2, s in ((np.array([-50.0, 0.0]), np.array([5.0, 2.5]), 2.5),
                       (np.array([5000.0, 6000.0]), np.array([0.7, 3.0]), 0.7)):
        got = Oracle(dict(p, k_table=(Tt2, f2), c_table=(Tt2, f2))).run(30)
        const = dict(p, materials=[dict(p["materials"][0], s0=s, c0=p["materials"][0]["c0"] * s)])
        ref = Oracle(const).run(30)
        assert np.max(np.abs(got - ref)) < 1e-11 * np.max(np.abs(ref))


@pytest.mark.parametrize("elem", ["hex8", "tet4"])
def test_k_table_nodal_average_on_an_element_straddling_a_kink(elem):
    """Sec. 4.2.2: the conductivity of an element is the average of the table
    evaluated at each of its nodes from the node's own temperature.  One
    element whose nodes sit on both sides of a sharp kink: the oracle's load
    equals s_e K0 T with s_e = mean(np.interp(T_a)) and K0 from the
    brute-force quadratic form, and differs from the table read at the mean
    temperature by far more than rounding (so the pin tells the rules apart)."""
    mat = H.aniso_material()
    X = H.distorted_hex(4) if elem == "hex8" else H.random_tet(4)
    ne = X.shape[0]
    p = H.single_element(elem, X, mat)
    Tt, f = np.array([0.0, 50.0, 60.0, 200.0]), np.array([1.0, 1.2, 4.0, 4.5])
    p["k_table"] = (Tt, f)
    T = np.where(np.arange(ne) % 2 == 0, 20.0, 95.0) + np.arange(ne)
    F, _ = Oracle(p).loads(T)
    energy = hex_energy if elem == "hex8" else tet_energy
    K0 = np.zeros((ne, ne))
    for a in range(ne):
        for b in range(ne):
            ea, eb = np.eye(ne)[a], np.eye(ne)[b]
            K0[a, b] = (energy(X, ea + eb, H.D_of(mat)) - energy(X, ea - eb, H.D_of(mat))) / 4.0
    s_nodal = np.mean(np.interp(T, Tt, f))
    s_mean = np.interp(T.mean(), Tt, f)
    ref = s_nodal * (K0 @ T)
    assert np.max(np.abs(F - ref)) <= 1e-10 * np.max(np.abs(ref))
    assert abs(s_nodal - s_mean) > 0.2 * s_nodal


def test_k_table_nodal_average_adjoint_on_a_kink():
    """The derivative of the nodal average with respect to T_a is the table's
    slope at T_a over n_e: one distorted hexahedron straddling a kink, dL/dT0
    of a one-step run against central differences."""
    mat = H.aniso_material(rho=1000.0, c0=1000.0)
    X = H.distorted_hex(5)
    p = H.single_element("hex8", X, mat)
    p["k_table"] = (np.array([0.0, 50.0, 60.0, 200.0]), np.array([1.0, 1.2, 4.0, 4.5]))
    p["T0"] = np.array([20.0, 95.0, 22.0, 93.0, 30.0, 85.0, 25.0, 90.0])
    p["dt"] = 50.0
    w = np.linspace(0.5, 1.5, 8)
    o = Oracle(p)
    hist = o.run(1, history=True)
    g = o.adjoint(hist, w.copy())
    for k in range(8):
        Ls = []
        for d in (1e-4, -1e-4):
            T0 = p["T0"].copy()
            T0[k] += d
            Ls.append(w @ Oracle(dict(p, T0=T0)).run(1))
        fd = (Ls[0] - Ls[1]) / 2e-4
        assert abs(fd - g["lam0"][k]) <= 1e-7 * max(abs(fd), 1.0)


def test_c_table_single_hex_recursion():
    """One hexahedron, uniform temperature, convection on all faces: every node
    follows T' = T - dt A h (T - Ta) / (rho c0 fc(T) a^3 / 8) with fc
    interpolated independently by numpy."""
    a, h, Ta, rho, c0 = 0.05, 40.0, 10.0, 2000.0, 500.0
    m = M.box_hex(1, 1, 1, a, a, a)
    p = P._base(m, "one_ctab")
    p["materials"] = [P.material(rho, c0, [5.0])]
    faces, _ = M.box_side_faces(m)
    P.set_faces(p, faces, h=h, Ta=Ta)
    Tt, f = np.array([0.0, 100.0, 200.0, 320.0]), np.array([1.0, 1.6, 1.1, 2.0])
    p["c_table"] = (Tt, f)
    p["T0"] = np.full(8, 300.0)
    p["T_lo"], p["T_hi"] = 0.0, 300.0
    o = Oracle(p)
    T = 300.0
    A = 3 * a * a / 4
    for _ in range(200):
        T = T + o.dt[0] * A * (-h * (T - Ta)) / (rho * c0 * np.interp(T, Tt, f) * a ** 3 / 8)
    assert T < 200.0                       # the run crosses two kinks
    assert np.max(np.abs(o.run(200) - T)) < 1e-11 * T


def test_table_adjoint_matches_finite_differences():
    """Kinked k and c tables: the adjoint's table slopes against central
    differences of the forward run (log k, c0, h and T0)."""
    p = _table_problem("hex8")
    p["k_table"] = (np.array([0.0, 120.0, 220.0, 400.0]), np.array([0.8, 1.5, 1.2, 2.2]))
    p["c_table"] = (np.array([0.0, 160.0, 260.0, 400.0]), np.array([1.0, 1.8, 1.3, 1.9]))
    p["dt"] = 0.5 * Oracle(p).dt_crit
    nsteps = 30
    o = Oracle(p)
    sens = np.arange(1, o.N, 3)
    sens = sens[~np.isin(sens, o.dir_nodes)]
    target = np.full(sens.size, 100.0)
    hist = o.run(nsteps, history=True)
    lam = np.zeros(o.N)
    lam[sens] = hist[-1][sens] - target
    g = o.adjoint(hist, lam)
    theta = np.log(p["elem_kscale"])
    for e in (3, int(np.argmax(np.abs(g["g_logk"])))):
        Ls = []
        for d in (1e-4, -1e-4):
            th = theta.copy()
            th[e] += d
            Ls.append(_loss(dict(p, elem_kscale=np.exp(th)), sens, target, nsteps)[0])
        fd = (Ls[0] - Ls[1]) / 2e-4
        assert abs(fd - g["g_logk"][e]) <= 2e-6 * max(abs(fd), 1e-3 * np.abs(g["g_logk"]).max())
    for k in (o.N // 2, o.N - 1):
        Ls = []
        for d in (1e-3, -1e-3):
            T0 = p["T0"].copy()
            T0[k] += d
            Ls.append(_loss(dict(p, T0=T0), sens, target, nsteps)[0])
        fd = (Ls[0] - Ls[1]) / 2e-3
        assert abs(fd - g["lam0"][k]) <= 2e-6 * max(abs(fd), 1e-3 * np.abs(g["lam0"]).max())
    e = int(np.argmax(np.abs(g["g_c"])))
    m0 = p["materials"][0]
    base = dict(p, materials=[dict(m0) for _ in range(o.E)],
                elem_material=np.arange(o.E, dtype=np.int32))
    Ls = []
    for d in (1e-3, -1e-3):
        mm = [dict(m0) for _ in range(o.E)]
        mm[e]["c0"] = m0["c0"] * (1 + d)
        Ls.append(_loss(dict(base, materials=mm), sens, target, nsteps)[0])
    fd = (Ls[0] - Ls[1]) / (2e-3 * m0["c0"])
    assert abs(fd - g["g_c"][e]) <= 2e-6 * abs(fd)


# ----------------------------------------------------------------------------
# adjoint
def _adjoint_problem():
    n = 4
    p, m = H.box_problem("hex8", n, side=0.1, mat=P.material(1000.0, 1000.0, [1.0]))
    g = np.random.default_rng(11)
    p["elem_kscale"] = np.exp(0.5 * g.standard_normal(n ** 3))
    faces, sides = M.box_side_faces(m)
    P.set_faces(p, faces[sides != 0], h=15.0, Ta=20.0)
    bottom = np.nonzero(np.isclose(m["x"], 0.0))[0].astype(np.int32)
    p["dir_nodes"], p["dir_T"] = bottom, np.full(bottom.size, 50.0)
    p["T0"] = g.uniform(80, 100, m["x"].size)
    p["dt"] = 2.0
    return p, m


def _loss(p, sens, target, nsteps):
    T = Oracle(p).run(nsteps)
    return 0.5 * np.sum((T[sens] - target) ** 2), T


def test_adjoint_matches_finite_differences():
    p, m = _adjoint_problem()
    nsteps = 30
    sens = np.array([5, 40, 77, 100, 120])
    target = np.full(sens.size, 60.0)
    o = Oracle(p)
    hist = o.run(nsteps, history=True)
    lam = np.zeros(o.N)
    lam[sens] = hist[-1][sens] - target
    g = o.adjoint(hist, lam)
    eps = 1e-4
    theta = np.log(p["elem_kscale"])
    for e in (0, 13, 37, 63):
        th = theta.copy()
        th[e] += eps
        Lp, _ = _loss(dict(p, elem_kscale=np.exp(th)), sens, target, nsteps)
        th[e] -= 2 * eps
        Lm, _ = _loss(dict(p, elem_kscale=np.exp(th)), sens, target, nsteps)
        fd = (Lp - Lm) / (2 * eps)
        assert abs(fd - g["g_logk"][e]) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(g["g_logk"]).max())
    # heat capacity (per element, via per-element materials) and h (per face),
    # each at the entry with the largest gradient so the differences are not
    # lost in the rounding of the loss
    eps = 1e-3
    e = int(np.argmax(np.abs(g["g_c"])))
    mats = [P.material(1000.0, 1000.0, [1.0]) for _ in range(o.E)]
    base = dict(p, materials=mats, elem_material=np.arange(o.E, dtype=np.int32))
    Ls = []
    for d in (eps, -eps):
        mm = [dict(x) for x in mats]
        mm[e]["c0"] = 1000.0 * (1 + d)
        Ls.append(_loss(dict(base, materials=mm), sens, target, nsteps)[0])
    fd_c = (Ls[0] - Ls[1]) / (2 * eps * 1000.0)
    assert abs(fd_c - g["g_c"][e]) <= 1e-6 * abs(fd_c)
    f = int(np.argmax(np.abs(g["g_h"])))
    Ls = []
    for d in (eps, -eps):
        hh = p["face_h"].copy()
        hh[f] *= (1 + d)
        Ls.append(_loss(dict(p, face_h=hh), sens, target, nsteps)[0])
    fd_h = (Ls[0] - Ls[1]) / (2 * eps * 15.0)
    assert abs(fd_h - g["g_h"][f]) <= 1e-6 * abs(fd_h)


def test_hourglass_adjoint_matches_finite_differences():
    """The hourglass term enters the adjoint (its load, and log k through
    kappa): central differences of the oracle's forward run on the nonlinear
    problem with the uniform-gradient hexahedron and hourglass control."""
    p = dict(H.nonlinear_adjoint_problem("hex8"), hex_gradient="mean", hourglass=0.5)
    p["dt"] = 0.5 * Oracle(dict(p, dt=None)).dt_crit
    nsteps = 30
    o = Oracle(p)
    sens = np.arange(1, o.N, 3)
    sens = sens[~np.isin(sens, o.dir_nodes)]
    target = np.full(sens.size, 100.0)
    hist = o.run(nsteps, history=True)
    lam = np.zeros(o.N)
    lam[sens] = hist[-1][sens] - target
    g = o.adjoint(hist, lam)
    theta = np.log(p["elem_kscale"])
    for e in (0, o.E - 1, int(np.argmax(np.abs(g["g_logk"])))):
        Ls = []
        for d in (1e-4, -1e-4):
            th = theta.copy()
            th[e] += d
            Ls.append(_loss(dict(p, elem_kscale=np.exp(th)), sens, target, nsteps)[0])
        fd = (Ls[0] - Ls[1]) / 2e-4
        assert abs(fd - g["g_logk"][e]) <= 2e-6 * max(abs(fd), 1e-3 * np.abs(g["g_logk"]).max())
    k = o.N // 2 + 1
    assert k not in set(o.dir_nodes)
    Ls = []
    for d in (1e-3, -1e-3):
        T0 = o.initial().copy()
        T0[k] += d
        Ls.append(0.5 * np.sum((o.run(nsteps, T0=T0, apply_initial=False)[sens] - target) ** 2))
    fd = (Ls[0] - Ls[1]) / 2e-3
    assert abs(fd - g["lam0"][k]) <= 2e-6 * max(abs(fd), 1e-3 * np.abs(g["lam0"]).max())


def test_adjoint_transpose_identity():
    """<w, J v> = <J^T w, v> for the one-step Jacobian J (the step is affine
    in T for a T-independent problem, so J v is a difference of two steps)."""
    p, m = _adjoint_problem()
    o = Oracle(p)
    g = np.random.default_rng(4)
    T = o.initial()
    v = g.standard_normal(o.N)
    v[o.dir_nodes] = 0.0
    w = g.standard_normal(o.N)
    Jv = o.run(1, T0=T + v, apply_initial=False) - o.run(1, T0=T, apply_initial=False)
    hist = o.run(1, T0=T, apply_initial=False, history=True)
    JTw = o.adjoint(hist, w)["lam0"]
    assert abs(w @ Jv - JTw @ v) < 1e-12 * abs(w @ Jv)


@pytest.mark.parametrize("elem", ["hex8", "tet4"])
def test_nonlinear_adjoint_matches_finite_differences(elem):
    """Every Jacobian term of the nonlinear step (k(Tbar), c(T), radiation)
    enters the gradients: central differences of the oracle's own forward run
    against its adjoint, for log k, c0, h and T0."""
    p = H.nonlinear_adjoint_problem(elem)
    nsteps = 40
    o = Oracle(p)
    sens = np.arange(1, o.N, 3)
    sens = sens[~np.isin(sens, o.dir_nodes)]
    target = np.full(sens.size, 100.0)
    hist = o.run(nsteps, history=True)
    lam = np.zeros(o.N)
    lam[sens] = hist[-1][sens] - target
    g = o.adjoint(hist, lam)

    def close(fd, ad, scale):
        assert abs(fd - ad) <= 2e-6 * max(abs(fd), 1e-3 * scale), (fd, ad)

    eps = 1e-4
    theta = np.log(p["elem_kscale"])
    for e in (0, 7, o.E - 1, int(np.argmax(np.abs(g["g_logk"])))):
        Ls = []
        for d in (eps, -eps):
            th = theta.copy()
            th[e] += d
            Ls.append(_loss(dict(p, elem_kscale=np.exp(th)), sens, target, nsteps)[0])
        close((Ls[0] - Ls[1]) / (2 * eps), g["g_logk"][e], np.abs(g["g_logk"]).max())
    # c0 of one element (per-element materials with the same c1 and D(T))
    e = int(np.argmax(np.abs(g["g_c"])))
    m0 = p["materials"][0]
    mats = [dict(m0) for _ in range(o.E)]
    base = dict(p, materials=mats, elem_material=np.arange(o.E, dtype=np.int32))
    Ls = []
    for d in (1e-3, -1e-3):
        mm = [dict(x) for x in mats]
        mm[e]["c0"] = m0["c0"] * (1 + d)
        Ls.append(_loss(dict(base, materials=mm), sens, target, nsteps)[0])
    close((Ls[0] - Ls[1]) / (2e-3 * m0["c0"]), g["g_c"][e], np.abs(g["g_c"]).max())
    # h of the face with the largest derivative (a radiating one among them)
    for f in (int(np.argmax(np.abs(g["g_h"]))), int(np.nonzero(p["face_eps"] > 0)[0][0])):
        Ls = []
        for d in (1e-3, -1e-3):
            hh = p["face_h"].copy()
            hh[f] *= (1 + d)
            Ls.append(_loss(dict(p, face_h=hh), sens, target, nsteps)[0])
        close((Ls[0] - Ls[1]) / (2e-3 * p["face_h"][f]), g["g_h"][f], np.abs(g["g_h"]).max())
    # initial temperatures of free nodes (one under radiation)
    rad_nodes = np.unique(p["faces"][p["face_eps"] > 0])
    free = [k for k in (int(rad_nodes[-1]), o.N // 2, o.N - 1) if k not in set(o.dir_nodes)]
    for k in free:
        Ls = []
        for d in (1e-3, -1e-3):
            T0 = p["T0"].copy()
            T0[k] += d
            Ls.append(_loss(dict(p, T0=T0), sens, target, nsteps)[0])
        close((Ls[0] - Ls[1]) / 2e-3, g["lam0"][k], np.abs(g["lam0"]).max())
    assert np.all(g["lam0"][o.dir_nodes] == 0.0)


def test_nonlinear_adjoint_transpose_identity():
    """<w, J v> = <J^T w, v> for the Jacobian J of one nonlinear step, with J v
    from a central difference of the step (error O(eps^2))."""
    p = H.nonlinear_adjoint_problem("hex8")
    o = Oracle(p)
    g = np.random.default_rng(5)
    T = o.initial()
    v = g.standard_normal(o.N)
    v[o.dir_nodes] = 0.0
    w = g.standard_normal(o.N)
    eps = 1e-3
    Jv = (o.run(1, T0=T + eps * v, apply_initial=False)
          - o.run(1, T0=T - eps * v, apply_initial=False)) / (2 * eps)
    hist = o.run(1, T0=T, apply_initial=False, history=True)
    JTw = o.adjoint(hist, w)["lam0"]
    assert abs(w @ Jv - JTw @ v) < 1e-8 * np.abs(w) @ np.abs(Jv)


def test_error_norms():
    a = np.array([1.0, 2.0, -4.0])
    b = np.array([1.0, 2.5, -4.0])
    assert oracle.err_max(b, a) == 0.5 / 4.0
    assert abs(oracle.err_rms(b, a) - np.sqrt(0.25 / 21.0)) < 1e-16
