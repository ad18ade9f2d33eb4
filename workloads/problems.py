"""Problem definitions: the benchmark workloads and small variants of them.

A *problem* is a plain dict of numpy arrays and scalars that fully describes
one run of the explicit scheme (mesh, materials, boundary conditions, initial
temperatures, time-step rule, step count).  Both the oracle and the GPU
library consume the same dict; nothing in here evaluates the method.

Keys
----
elem            'hex8' | 'tet4'
x, y, z         float64[N] node coordinates (m)
conn            int32[n_e, E] connectivity (structure of arrays)
materials       list of dict(rho, c0, c1, k[6], s0, s1):
                    c(T) = c0 + c1 T                     (J/(kg K))
                    D(T) = Dk * (s0 + s1 T),  Dk = [xx, yy, zz, xy, yz, xz]
elem_material   int32[E] or None (None: material 0 everywhere)
elem_k          float64[6, E] or None: per-element Dk replacing the material's
elem_kscale     float64[E] or None: per-element factor on D (e.g. exp(log k))
dir_nodes       int32[]   Dirichlet nodes; dir_T float64[] their temperatures
faces           int32[F, 3|4] boundary faces; face_h, face_Ta, face_eps,
                face_q float64[F]: convection coefficient (W/(m^2 K)), ambient
                temperature (C), emissivity, and applied flux into the body
                (W/m^2) of every face
pt_nodes/pt_W   concentrated nodal heat inputs (W)
T0              float64[N] initial temperatures (C)
dt              float or None.  None: dt = safety * dt_crit, with dt_crit the
                stability bound evaluated over the temperature range
                [T_lo, T_hi]; with node_instance given, one dt per instance.
Tz              absolute zero in C (-273.15)
node_instance   int32[N] or None: independent instances of a batched mesh
nsteps          number of explicit steps
hex_gradient    optional 'centre' (default) | 'mean': the hexahedron's gradient
                at its centre or averaged over it (uniform gradient)
hourglass       optional float >= 0 (default 0): hourglass control strength of
                the uniform-gradient hexahedron
"""
from __future__ import annotations

import numpy as np

from . import fields, mesh as M

TZ = -273.15
SIGMA_SB = 5.67e-8    # Stefan-Boltzmann constant, Sec. 2 (radiation condition)


def material(rho, c0, k, c1=0.0, s0=1.0, s1=0.0):
    k = list(k)
    if len(k) == 1:
        k = [k[0], k[0], k[0], 0.0, 0.0, 0.0]
    elif len(k) == 3:
        k = [k[0], k[1], k[2], 0.0, 0.0, 0.0]
    assert len(k) == 6
    return dict(rho=float(rho), c0=float(c0), c1=float(c1),
                k=[float(v) for v in k], s0=float(s0), s1=float(s1))


def _base(m, name):
    n = m["x"].size
    e = m["conn"].shape[1]
    return dict(name=name, elem=m["elem"], x=m["x"], y=m["y"], z=m["z"],
                conn=np.ascontiguousarray(m["conn"], dtype=np.int32),
                materials=[], elem_material=None, elem_k=None, elem_kscale=None,
                dir_nodes=np.zeros(0, np.int32), dir_T=np.zeros(0),
                faces=None, face_h=None, face_Ta=None, face_eps=None, face_q=None,
                pt_nodes=np.zeros(0, np.int32), pt_W=np.zeros(0),
                T0=np.zeros(n), dt=None, safety=0.9, T_lo=0.0, T_hi=100.0,
                Tz=TZ, node_instance=None, nsteps=1, meta=dict(n_nodes=n, n_elems=e))


def set_faces(p, faces, h=0.0, Ta=0.0, eps=0.0, q=0.0):
    nf = faces.shape[0]
    p["faces"] = np.ascontiguousarray(faces, dtype=np.int32)
    for key, val in (("face_h", h), ("face_Ta", Ta), ("face_eps", eps), ("face_q", q)):
        arr = np.asarray(val, dtype=np.float64)
        p[key] = np.broadcast_to(arr, (nf,)).copy()
    return p


# --------------------------------------------------------------------------
# Workload 1: plain FED-FEM, FP64, 10^3 hexahedra on the unit cube, T=100 on
# z=1, other faces insulated, dt = 0.9 dt_crit, 1000 steps.
def cube_plain(n=10, nsteps=1000, elem="hex8"):
    m = M.box_hex(n, n, n) if elem == "hex8" else M.box_tet_kuhn(n, n, n)
    p = _base(m, f"plain_{elem}_{n}")
    p["materials"] = [material(rho=1000.0, c0=1000.0, k=[1.0])]
    top = np.nonzero(np.isclose(m["z"], 1.0))[0].astype(np.int32)
    p["dir_nodes"] = top
    p["dir_T"] = np.full(top.size, 100.0)
    p["T_lo"], p["T_hi"] = 0.0, 100.0
    p["nsteps"] = nsteps
    return p


# --------------------------------------------------------------------------
# Workload 2: nonlinear hexahedra.  0.1 m cube, n^3 hexahedra, orthotropic
# D(T) = diag(1, 2, 0.5) (1 + 0.005 T), c(T) = 1000 + 2 T, rho = 1000,
# T0 ~ U[20, 25] per node, convection h = 10 to 20 C on all faces, radiation
# eps = 0.8 to 20 C on the top face, 1e5 W/m^2 on the central bottom patch
# (the central (n/8)^2 faces, 12.5 mm square at n = 64).
def cube_nonlinear_hex(n=64, nsteps=10000, seed=1909_0002):
    side = 0.1
    m = M.box_hex(n, n, n, side, side, side)
    p = _base(m, f"nonlinear_hex_{n}")
    p["materials"] = [material(rho=1000.0, c0=1000.0, c1=2.0, k=[1.0, 2.0, 0.5],
                               s0=1.0, s1=0.005)]
    faces, sides = M.box_side_faces(m)
    nf = faces.shape[0]
    h = np.full(nf, 10.0)
    Ta = np.full(nf, 20.0)
    eps = np.where(sides == 5, 0.8, 0.0)
    q = np.zeros(nf)
    # bottom side: faces enumerated with x fastest, then y
    bottom = np.nonzero(sides == 4)[0]
    fi = np.arange(bottom.size)
    u, v = fi % n, fi // n
    half = max(n // 16, 1)
    lo, hi = n // 2 - half, n // 2 + half
    patch = bottom[(u >= lo) & (u < hi) & (v >= lo) & (v < hi)]
    q[patch] = 1.0e5
    set_faces(p, faces, h=h, Ta=Ta, eps=eps, q=q)
    g = fields.rng(seed)
    p["T0"] = fields.uniform(g, 20.0, 25.0, m["x"].size)
    # [20, 1000] C holds the run at 64^3 (20.85..392.5 C over 10,000 steps);
    # coarser meshes take larger steps (dt ~ h^2) and the flux patch makes the
    # explicit step overshoot below 20 C in the first steps (down to -20 C at
    # 8^3), so their range starts at -40 C
    p["T_lo"], p["T_hi"] = (20.0 if n >= 64 else -40.0), 1000.0
    p["nsteps"] = nsteps
    p["meta"].update(seed=seed, flux_faces=int(patch.size))
    return p


# --------------------------------------------------------------------------
# Variants of workload 2 that exercise the follow-up features at full size:
# the temperature dependence of D and c as piecewise-linear tables, the
# uniform-gradient hexahedron on a distorted mesh, the forward model of a
# sensor loss for the nonlinear adjoint, and a point source that moves
# across the top face one node per step.
def cube_nonlinear_hex_tables(n=64, nsteps=10000):
    """Workload 2 with D and c scaled by tabulated multipliers of T (clamped
    beyond the ends): D rises 0.5% per C up to 400 C and flattens above; c
    has a latent-heat-like bump around 500 C."""
    p = cube_nonlinear_hex(n, nsteps)
    p["name"] = f"nonlinear_hex_tables_{n}"
    p["materials"] = [dict(m, s0=1.0, s1=0.0, c1=0.0) for m in p["materials"]]
    p["k_table"] = (np.array([0.0, 400.0, 700.0, 1000.0]), np.array([1.0, 3.0, 3.6, 4.0]))
    p["c_table"] = (np.array([0.0, 400.0, 500.0, 600.0, 1000.0]),
                    np.array([1.0, 1.8, 2.6, 2.2, 3.0]))
    return p


def cube_nonlinear_hex_mean(n=64, nsteps=10000, amp=0.25, seed=1909_0006):
    """Workload 2 on a distorted mesh (interior nodes moved by up to amp times
    the spacing) with the uniform-gradient hexahedron."""
    p = cube_nonlinear_hex(n, nsteps)
    mj = M.jitter_interior(dict(elem=p["elem"], x=p["x"], y=p["y"], z=p["z"], conn=p["conn"]),
                           amp, seed)
    p.update(x=mj["x"], y=mj["y"], z=mj["z"], name=f"nonlinear_hex_mean_{n}")
    p["hex_gradient"] = "mean"
    p["meta"].update(jitter=amp, jitter_seed=seed)
    return p


def cube_nonlinear_hex_mean_hg(n=64, nsteps=10000, eps=0.3):
    """The distorted uniform-gradient workload with hourglass control of
    strength eps."""
    p = cube_nonlinear_hex_mean(n, nsteps)
    p["name"] = f"nonlinear_hex_mean_hg_{n}"
    p["hourglass"] = eps
    p["meta"].update(hourglass=eps)
    return p


def nonlinear_adjoint_hex(n=64, nsteps=2000, n_sensors=512, ckpt_every=100, seed=1909_0007):
    """Workload 2 as the forward model of a mean-square sensor loss (seeded
    sensor nodes), for the adjoint through k(T), c(T) and radiation."""
    p = cube_nonlinear_hex(n, nsteps)
    g = fields.rng(seed)
    p["name"] = f"nonlinear_adjoint_hex_{n}"
    p["meta"].update(sensors=np.sort(g.choice(p["x"].size, n_sensors, replace=False)),
                     ckpt_every=ckpt_every)
    return p


def moving_source_hex(n=64, nsteps=2000, power=2.0):
    """Workload 2 with a point source of the given power on the line y = side/2
    of the top face, listed node by node; the source moves one node a step.
    At 64^3 a 2 W source heats the node under it to about 380 C and the
    explicit step's overshoot next to it cools a node below 20 C (to about
    -26 C), so the range the stability bound covers is [-40, 1000] C (50 W
    would drive the step unstable)."""
    p = cube_nonlinear_hex(n, nsteps)
    p["T_lo"] = -40.0
    top = np.isclose(p["z"], p["z"].max())
    mid = np.isclose(p["y"], 0.5 * (p["y"].min() + p["y"].max()))
    line = np.nonzero(top & mid)[0]
    line = line[np.argsort(p["x"][line])].astype(np.int32)
    p["name"] = f"moving_source_hex_{n}"
    p["pt_nodes"], p["pt_W"] = line, np.zeros(line.size)
    p["meta"].update(source_power=power)
    return p


# --------------------------------------------------------------------------
# Workload 3: large anisotropic tetrahedral mesh.  n^3 grid on a 0.1 m cube,
# every cell split into 6 Kuhn tetrahedra; per-element SPD conductivity
# R diag(lam) R^T with Haar-random R and lam log-uniform in [0.5, 5];
# c(T) = 1000 + 2 T; rho = 1000; convection h = 10 to 20 C on all faces;
# T0 ~ U[20, 25]; 2000 steps.
def cube_aniso_tet(n=128, nsteps=2000, seed=1909_0003):
    side = 0.1
    m = M.box_tet_kuhn(n, n, n, side, side, side)
    p = _base(m, f"aniso_tet_{n}")
    p["materials"] = [material(rho=1000.0, c0=1000.0, c1=2.0, k=[1.0])]
    g = fields.rng(seed)
    p["elem_k"] = fields.spd_tensors(g, m["conn"].shape[1], 0.5, 5.0)
    faces, _ = M.box_side_faces(m)
    set_faces(p, faces, h=10.0, Ta=20.0)
    p["T0"] = fields.uniform(g, 20.0, 25.0, m["x"].size)
    p["T_lo"], p["T_hi"] = 15.0, 30.0
    p["nsteps"] = nsteps
    p["meta"].update(seed=seed)
    return p


# --------------------------------------------------------------------------
# Workload 4: batched scenarios.  n_inst independent hexahedral boxes of side
# 0.1 m with per-axis cell counts uniform in {lo..hi}; per instance k0 in
# [0.5, 5] (isotropic, constant), c in [500, 4000] (constant), h in [5, 50],
# eps in [0, 0.9], uniform T0 in [0, 40]; convection and radiation to 20 C on
# all faces; rho = 1000; one dt = 0.9 dt_crit per instance.
def batched_hex(n_inst=256, lo=8, hi=48, nsteps=5000, seed=1909_0004):
    g = fields.rng(seed)
    dims = g.integers(lo, hi + 1, size=(n_inst, 3))
    k0 = g.uniform(0.5, 5.0, n_inst)
    c = g.uniform(500.0, 4000.0, n_inst)
    hc = g.uniform(5.0, 50.0, n_inst)
    eps = g.uniform(0.0, 0.9, n_inst)
    t0 = g.uniform(0.0, 40.0, n_inst)
    side = 0.1
    meshes, faces_all, fi_inst = [], [], []
    for i in range(n_inst):
        nx, ny, nz = (int(v) for v in dims[i])
        meshes.append(M.box_hex(nx, ny, nz, side, side, side))
    # instances stay at the origin: consumers keep them apart by node_instance,
    # and large offsets would cost digits in the element edge vectors
    big = M.concatenate(meshes)
    for i, mi in enumerate(meshes):
        f, _ = M.box_side_faces(mi)
        faces_all.append(f.astype(np.int64) + big["node_start"][i])
        fi_inst.append(np.full(f.shape[0], i))
    faces = np.concatenate(faces_all).astype(np.int32)
    fi_inst = np.concatenate(fi_inst)
    p = _base(big, f"batched_hex_{n_inst}")
    p["materials"] = [material(rho=1000.0, c0=c[i], k=[k0[i]]) for i in range(n_inst)]
    p["elem_material"] = big["elem_instance"].copy()
    set_faces(p, faces, h=hc[fi_inst], Ta=20.0, eps=eps[fi_inst])
    p["T0"] = t0[big["node_instance"]]
    p["node_instance"] = big["node_instance"].copy()
    p["T_lo"], p["T_hi"] = 0.0, 40.0
    p["nsteps"] = nsteps
    p["meta"].update(seed=seed, dims=dims, node_start=big["node_start"],
                     elem_start=big["elem_start"])
    return p


# --------------------------------------------------------------------------
# Workload 5: adjoint.  n^3 hexahedra on a 0.1 m cube with per-element
# log-conductivity theta = Gaussian random field (mean log 1 = 0, sigma 0.5,
# correlation length 0.1 * side), k_e = exp(theta_e) isotropic; rho = 1000,
# c = 1000; T0 = 100; convection h = 15 to 20 C on all faces; fixed
# dt = 0.1 s (below dt_crit for both fields); loss = mean over n_sensors
# seeded nodes of (T - T*)^2 with T* a run with theta from target_seed.
def adjoint_hex(n=48, nsteps=2000, seed=1909_0005, target_seed=1909_0055,
                n_sensors=512, dt=0.1, ckpt_every=100):
    side = 0.1
    m = M.box_hex(n, n, n, side, side, side)
    p = _base(m, f"adjoint_hex_{n}")
    p["materials"] = [material(rho=1000.0, c0=1000.0, k=[1.0])]
    g = fields.rng(seed)
    corr = 0.1 * n          # 0.1 * side, in cells
    theta = fields.gaussian_random_field(g, (n, n, n), corr, mean=0.0, sigma=0.5)
    gt = fields.rng(target_seed)
    theta_t = fields.gaussian_random_field(gt, (n, n, n), corr, mean=0.0, sigma=0.5)
    p["elem_kscale"] = np.exp(theta)
    faces, _ = M.box_side_faces(m)
    set_faces(p, faces, h=15.0, Ta=20.0)
    p["T0"] = np.full(m["x"].size, 100.0)
    p["dt"] = dt
    p["T_lo"], p["T_hi"] = 20.0, 100.0
    p["nsteps"] = nsteps
    gs = fields.rng(seed + 1)
    p["meta"].update(seed=seed, theta=theta, theta_target=theta_t,
                     sensors=fields.pick(gs, m["x"].size, min(n_sensors, m["x"].size)),
                     ckpt_every=ckpt_every)
    return p


# --------------------------------------------------------------------------
# Paper-sized stand-in for the timing study (Sec. 4.6): a 0.1 m cube of
# 19^3 cells x 6 Kuhn tetrahedra (41,154 elements / 8,000 nodes, close to the
# paper's 40,021 / 7,872), k = 200, rho = 1000, c = 2000, dt = 0.005 s,
# 2000 steps, back face at 37 C, 0.2 W on every node of the front, top and
# two side faces (Sec. 4.2.1).  td=True uses the temperature-dependent
# properties of Sec. 4.2.2: k and c rising 6 and 20 per C from 200 and 2000
# at 37 C (k 200 -> 2000 and c 2000 -> 8000 over 37 -> 337 C).
def paper_standin(n=19, td=False, nsteps=2000):
    side = 0.1
    m = M.box_tet_kuhn(n, n, n, side, side, side)
    p = _base(m, f"paper_standin_{'td' if td else 'ti'}")
    if td:
        # k(T) = 200 + 6 (T - 37), c(T) = 2000 + 20 (T - 37)
        p["materials"] = [material(rho=1000.0, c0=2000.0 - 20.0 * 37.0, c1=20.0,
                                   k=[1.0], s0=200.0 - 6.0 * 37.0, s1=6.0)]
    else:
        p["materials"] = [material(rho=1000.0, c0=2000.0, k=[200.0])]
    x, y, z = m["x"], m["y"], m["z"]
    back = np.nonzero(np.isclose(y, side))[0]
    p["dir_nodes"] = back.astype(np.int32)
    p["dir_T"] = np.full(back.size, 37.0)
    loaded = np.isclose(y, 0.0) | np.isclose(z, side) | np.isclose(x, 0.0) | np.isclose(x, side)
    loaded &= ~np.isclose(y, side)
    pts = np.nonzero(loaded)[0].astype(np.int32)
    p["pt_nodes"] = pts
    p["pt_W"] = np.full(pts.size, 0.2)
    p["T0"] = np.full(x.size, 37.0)
    p["dt"] = 0.005
    # the run stays within 37..41 C over 2000 steps; [37, 100] bounds the
    # stability check (with the TD laws, dt_crit over 37..337 C would be
    # 0.0041 s, below the paper's 0.005 s, and 0.014 s over 37..100 C)
    p["T_lo"], p["T_hi"] = 37.0, 100.0
    p["nsteps"] = nsteps
    return p


WORKLOADS = {
    "plain_fp64_cube10": cube_plain,
    "nonlinear_hex64": cube_nonlinear_hex,
    "aniso_tet128": cube_aniso_tet,
    "batched_hex256": batched_hex,
    "adjoint_hex48": adjoint_hex,
}
