"""FP64 CPU oracle for FED-FEM (arXiv 1909.03355).

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's CPU
baseline may import this package.  The product (the GPU library and its
Python binding) never calls it, and it shares no code with them; the only
thing both sides use is the seeded input module ``workloads``.

The stepping loop lives in ``fedfem_oracle.c`` (plain C, FP64); this module
expands the problem description into per-element arrays, calls the C code,
and evaluates the critical time step with numpy's symmetric eigensolver.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

SIGMA_SB = 5.67e-8   # Stefan-Boltzmann constant (Sec. 2, radiation condition)

_d = C.POINTER(C.c_double)
_i32 = C.POINTER(C.c_int32)
_i8 = C.POINTER(C.c_int8)


class _Problem(C.Structure):
    _fields_ = [("ne", C.c_int32), ("nfn", C.c_int32),
                ("N", C.c_int64), ("E", C.c_int64), ("nf", C.c_int64),
                ("npt", C.c_int64), ("ndir", C.c_int64),
                ("conn", _i32), ("B", _d), ("W", _d), ("V", _d),
                ("rho", _d), ("c0", _d), ("c1", _d), ("s0", _d), ("s1", _d), ("Dk", _d),
                ("faces", _i32), ("farea", _d), ("fh", _d), ("fTa", _d), ("feps", _d),
                ("fq", _d), ("pt_nodes", _i32), ("pt_W", _d),
                ("dir_nodes", _i32), ("dir_T", _d), ("dt", _d),
                ("Tz", C.c_double), ("sigma", C.c_double),
                ("nkt", C.c_int32), ("nct", C.c_int32),
                ("kt_T", _d), ("kt_f", _d), ("ct_T", _d), ("ct_f", _d),
                ("hg_G", _d), ("hg_k", _d)]


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = C.CDLL(path)
        L.orc_geometry.restype = C.c_int64
        L.orc_geometry.argtypes = [C.c_int, C.c_int64, _d, _d, _d, _i32, _d, _d, _d, _d]
        L.orc_geometry_mean.restype = C.c_int64
        L.orc_geometry_mean.argtypes = [C.c_int64, _d, _d, _d, _i32, _d, _d, _d, _d]
        L.orc_hourglass.argtypes = [C.c_int64, _d, _d, _d, _i32, _d, _d, _d, C.c_double, _d, _d]
        L.orc_face_areas.restype = None
        L.orc_face_areas.argtypes = [C.c_int, C.c_int64, _d, _d, _d, _i32, _d]
        P = C.POINTER(_Problem)
        L.orc_loads.argtypes = [P, _d, _d, _d, _d]
        L.orc_surface.argtypes = [P, _d, _d]
        L.orc_run.argtypes = [P, _d, C.c_int64, _d, _d, _d, _d, _d, _d]
        L.orc_run_sched.argtypes = [P, _d, C.c_int64, C.c_int64, C.c_int64, _d, _d, _d, _d, _d,
                                    _d, _d]
        L.orc_threads.restype = C.c_int
        L.orc_threads.argtypes = []
        L.orc_set_threads.restype = None
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_adjoint.restype = C.c_int
        L.orc_adjoint.argtypes = [P, _d, C.c_int64, _i8, _d, _d, _d, _d]
        _LIB = L
    return _LIB


def _p(a, t=_d):
    return a.ctypes.data_as(t) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Oracle:
    """The explicit scheme of Sec. 3 on one problem (see ``workloads.problems``)."""

    def __init__(self, prob):
        self.prob = prob
        L = lib()
        self.ne = 8 if prob["elem"] == "hex8" else 4
        x, y, z = _f64(prob["x"]), _f64(prob["y"]), _f64(prob["z"])
        conn = np.ascontiguousarray(prob["conn"], dtype=np.int32)
        self.N, self.E = x.size, conn.shape[1]
        self.x, self.y, self.z, self.conn = x, y, z, conn
        # ---- pre-computation (Sec. 3.5 (i)) -------------------------------
        self.B = np.zeros(self.E * 3 * self.ne)
        self.W = np.zeros(self.E)
        self.V = np.zeros(self.E)
        self.detJ0 = np.zeros(self.E)
        # hexahedra: centre-point B (Eq. 17), or the element-mean gradient
        # ("hex_gradient": "mean", the uniform-gradient hexahedron)
        self.hex_gradient = prob.get("hex_gradient", "centre")
        if self.ne == 8 and self.hex_gradient == "mean":
            self.n_bad = L.orc_geometry_mean(self.E, _p(x), _p(y), _p(z), _p(conn, _i32),
                                             _p(self.B), _p(self.W), _p(self.V), _p(self.detJ0))
        else:
            self.n_bad = L.orc_geometry(self.ne, self.E, _p(x), _p(y), _p(z), _p(conn, _i32),
                                        _p(self.B), _p(self.W), _p(self.V), _p(self.detJ0))
        mats = prob["materials"]
        mid = prob["elem_material"]
        mid = np.zeros(self.E, np.int64) if mid is None else np.asarray(mid, np.int64)
        tab = lambda key: np.array([m[key] for m in mats], dtype=np.float64)[mid]
        self.rho, self.c0, self.c1 = tab("rho"), tab("c0"), tab("c1")
        self.s0, self.s1 = tab("s0"), tab("s1")
        if prob["elem_k"] is not None:
            Dk = _f64(prob["elem_k"]).copy()
        else:
            Dk = np.array([m["k"] for m in mats], dtype=np.float64)[mid].T.copy()
        if prob["elem_kscale"] is not None:
            Dk = Dk * _f64(prob["elem_kscale"])[None, :]
        self.Dk = np.ascontiguousarray(Dk)
        # optional hourglass control of the uniform-gradient hexahedron
        # ("hourglass": eps > 0; the term is described at orc_hourglass)
        self.hourglass = float(prob.get("hourglass", 0.0) or 0.0)
        self.hg_G = self.hg_k = None
        if self.hourglass > 0:
            if not (self.ne == 8 and self.hex_gradient == "mean"):
                raise ValueError("hourglass control needs the uniform-gradient hexahedron")
            self.hg_G, self.hg_k = np.zeros(self.E * 32), np.zeros(self.E)
            L.orc_hourglass(self.E, _p(x), _p(y), _p(z), _p(conn, _i32), _p(self.B), _p(self.V),
                            _p(self.Dk), self.hourglass, _p(self.hg_G), _p(self.hg_k))
        # optional shared multiplier tables: D_e = Dk mean_a fk(T_a), c(T) = c0 fc(T)
        kt, ct = prob.get("k_table"), prob.get("c_table")
        self.kt = None if kt is None else (_f64(kt[0]), _f64(kt[1]))
        self.ct = None if ct is None else (_f64(ct[0]), _f64(ct[1]))
        # boundary faces
        if prob["faces"] is not None and prob["faces"].shape[0] > 0:
            self.faces = np.ascontiguousarray(prob["faces"], dtype=np.int32)
            self.nfn = self.faces.shape[1]
            self.farea = np.zeros(self.faces.shape[0])
            L.orc_face_areas(self.nfn, self.faces.shape[0], _p(x), _p(y), _p(z),
                             _p(self.faces, _i32), _p(self.farea))
            self.fh, self.fTa = _f64(prob["face_h"]), _f64(prob["face_Ta"])
            self.feps, self.fq = _f64(prob["face_eps"]), _f64(prob["face_q"])
        else:
            self.faces = np.zeros((0, 4), np.int32)
            self.nfn = 4
            self.farea = self.fh = self.fTa = self.feps = self.fq = np.zeros(0)
        self.pt_nodes = np.ascontiguousarray(prob["pt_nodes"], dtype=np.int32)
        self.pt_W = _f64(prob["pt_W"])
        self.dir_nodes = np.ascontiguousarray(prob["dir_nodes"], dtype=np.int32)
        self.dir_T = _f64(prob["dir_T"])
        self.is_dir = np.zeros(self.N, np.int8)
        self.is_dir[self.dir_nodes] = 1
        # ---- time step (Sec. 3.4) -----------------------------------------
        self.dt_crit = self.critical_dt()
        if prob["dt"] is not None:
            dt = np.broadcast_to(np.asarray(prob["dt"], dtype=np.float64),
                                 np.shape(self.dt_crit)).copy()
        else:
            dt = prob["safety"] * np.asarray(self.dt_crit, dtype=np.float64)
        self.dt_inst = dt
        inst = prob["node_instance"]
        if inst is None:
            self.dt = np.full(self.N, float(dt))
        else:
            self.dt = _f64(np.asarray(dt)[np.asarray(inst)])
        self.Tz = float(prob["Tz"])
        self._work = None
        self._build_struct()

    # ------------------------------------------------------------------
    def _build_struct(self):
        s = _Problem()
        s.ne, s.nfn = self.ne, self.nfn
        s.N, s.E, s.nf = self.N, self.E, self.faces.shape[0]
        s.npt, s.ndir = self.pt_nodes.size, self.dir_nodes.size
        s.conn = _p(self.conn, _i32)
        s.B, s.W, s.V = _p(self.B), _p(self.W), _p(self.V)
        s.rho, s.c0, s.c1 = _p(self.rho), _p(self.c0), _p(self.c1)
        s.s0, s.s1, s.Dk = _p(self.s0), _p(self.s1), _p(self.Dk)
        s.faces = _p(self.faces, _i32)
        s.farea, s.fh, s.fTa = _p(self.farea), _p(self.fh), _p(self.fTa)
        s.feps, s.fq = _p(self.feps), _p(self.fq)
        s.pt_nodes, s.pt_W = _p(self.pt_nodes, _i32), _p(self.pt_W)
        s.dir_nodes, s.dir_T = _p(self.dir_nodes, _i32), _p(self.dir_T)
        s.dt = _p(self.dt)
        s.Tz, s.sigma = self.Tz, SIGMA_SB
        s.nkt = 0 if self.kt is None else self.kt[0].size
        s.nct = 0 if self.ct is None else self.ct[0].size
        if self.kt is not None:
            s.kt_T, s.kt_f = _p(self.kt[0]), _p(self.kt[1])
        if self.ct is not None:
            s.ct_T, s.ct_f = _p(self.ct[0]), _p(self.ct[1])
        if self.hg_k is not None:
            s.hg_G, s.hg_k = _p(self.hg_G), _p(self.hg_k)
        self._s = s

    def _buffers(self):
        if self._work is None:
            self._work = dict(Fe=np.zeros(self.E * self.ne), F=np.zeros(self.N),
                              C=np.zeros(self.N), Q=np.zeros(self.N), Tn=np.zeros(self.N))
        return self._work

    # ------------------------------------------------------------------
    def element_matrices(self, scale=None, lo=0, hi=None):
        """K_e = W B^T D B for elements [lo, hi) with D = Dk * scale
        (scale defaults to s0 + s1 * 0), plus the hourglass term when on."""
        hi = self.E if hi is None else hi
        ne = self.ne
        B = self.B.reshape(self.E, 3, ne)[lo:hi]
        Dk = self.Dk[:, lo:hi]
        sc = self.s0[lo:hi] if scale is None else np.asarray(scale)[lo:hi]
        D = np.zeros((hi - lo, 3, 3))
        for (i, j), r in zip([(0, 0), (1, 1), (2, 2), (0, 1), (1, 2), (0, 2)], range(6)):
            D[:, i, j] = Dk[r] * sc
            D[:, j, i] = Dk[r] * sc
        K = self.W[lo:hi, None, None] * np.einsum("eia,eij,ejb->eab", B, D, B)
        if self.hg_k is not None:
            G = self.hg_G.reshape(self.E, 4, 8)[lo:hi]
            K = K + (sc * self.hg_k[lo:hi])[:, None, None] * np.einsum("eqa,eqb->eab", G, G)
        return K

    def critical_dt(self):
        """Stability bound dt_crit = 2 / lambda_max (Eq. 29), with lambda_max
        bounded element by element (Irons' element-eigenvalue bound, valid
        because both the lumped mass and K are sums of element PSD parts):
            lambda_e = lambda_max(K_e(T_hi)) / (rho_e c_e(T_lo) V_e / n_e)
            lambda_k = (h A_k + 4 sigma eps A_k (T_hi - Tz)^3) / C_k(T_lo)
            dt_crit  = 2 / (max_e lambda_e + max_k lambda_k)
        The temperature extremes of c and D are taken over [T_lo, T_hi].
        With node_instance set, one dt_crit per instance."""
        p = self.prob
        Tlo, Thi = float(p["T_lo"]), float(p["T_hi"])
        smax = np.maximum(self.s0 + self.s1 * Tlo, self.s0 + self.s1 * Thi)
        smin = np.minimum(self.s0 + self.s1 * Tlo, self.s0 + self.s1 * Thi)
        cmin = np.minimum(self.c0 + self.c1 * Tlo, self.c0 + self.c1 * Thi)
        # a piecewise-linear table takes its extremes at the ends of the range
        # or at breakpoints inside it
        def extremes(tab):
            Tt, f = tab
            pts = np.concatenate([[Tlo, Thi], Tt[(Tt > Tlo) & (Tt < Thi)]])
            v = np.interp(pts, Tt, f)
            return v.min(), v.max()
        if self.kt is not None:
            lo_, hi_ = extremes(self.kt)
            smax, smin = np.full(self.E, hi_), np.full(self.E, lo_)
        if self.ct is not None:
            cmin = self.c0 * extremes(self.ct)[0]
        if np.any(smin <= 0) or np.any(cmin <= 0):
            raise ValueError("conductivity or heat capacity not positive on [T_lo, T_hi]")
        lam_e = np.zeros(self.E)
        chunk = 1 << 19
        for lo in range(0, self.E, chunk):
            hi = min(self.E, lo + chunk)
            K = self.element_matrices(smax, lo, hi)
            lam_e[lo:hi] = np.linalg.eigvalsh(K)[:, -1] / (
                self.rho[lo:hi] * cmin[lo:hi] * self.V[lo:hi] / self.ne)
        Cmin = np.zeros(self.N)
        np.add.at(Cmin, self.conn.ravel(),
                  np.tile(self.rho * cmin * self.V / self.ne, self.ne))
        lam_b = np.zeros(self.N)
        if self.faces.shape[0]:
            share = self.farea / self.nfn
            coef = share * (self.fh + 4.0 * SIGMA_SB * self.feps * (Thi - float(p["Tz"])) ** 3)
            np.add.at(lam_b, self.faces.ravel(), np.repeat(coef, self.nfn))
        lam_b = lam_b / Cmin
        inst = p["node_instance"]
        if inst is None:
            return 2.0 / (lam_e.max() + lam_b.max())
        inst = np.asarray(inst)
        ninst = int(inst.max()) + 1
        einst = inst[self.conn[0]]
        le = np.zeros(ninst)
        np.maximum.at(le, einst, lam_e)
        lb = np.zeros(ninst)
        np.maximum.at(lb, inst, lam_b)
        return 2.0 / (le + lb)

    # ------------------------------------------------------------------
    def initial(self, T0=None):
        """T at t = 0 with the essential condition applied (Sec. 3.5 (ii))."""
        T = _f64(self.prob["T0"] if T0 is None else T0).copy()
        T[self.dir_nodes] = self.dir_T
        return T

    def loads(self, T):
        """(F, C): conductive nodal load K(T) T and lumped capacity at T."""
        w = self._buffers()
        T = _f64(T)
        F, Cc = np.zeros(self.N), np.zeros(self.N)
        lib().orc_loads(C.byref(self._s), _p(T), _p(w["Fe"]), _p(F), _p(Cc))
        return F, Cc

    def surface(self, T):
        """Q: surface and concentrated heat input into every node at T."""
        T = _f64(T)
        Q = np.zeros(self.N)
        lib().orc_surface(C.byref(self._s), _p(T), _p(Q))
        return Q

    def run(self, nsteps=None, T0=None, history=False, apply_initial=True, pt_schedule=None,
            step0=0):
        """T after nsteps explicit steps (or the (nsteps+1, N) history).

        With ``pt_schedule`` (n_rows x n_pt) step n of the run takes the
        concentrated loads of row (step0 + n) mod n_rows instead of pt_W."""
        nsteps = self.prob["nsteps"] if nsteps is None else int(nsteps)
        T = self.initial(T0) if apply_initial else _f64(T0).copy()
        w = self._buffers()
        hist = np.zeros((nsteps + 1, self.N)) if history else None
        if pt_schedule is None:
            lib().orc_run(C.byref(self._s), _p(T), nsteps, _p(w["Fe"]), _p(w["F"]),
                          _p(w["C"]), _p(w["Q"]), _p(w["Tn"]), _p(hist))
        else:
            Ws = _f64(pt_schedule)
            if Ws.ndim != 2 or Ws.shape[1] != self.pt_nodes.size or Ws.shape[0] < 1:
                raise ValueError("pt_schedule must be (n_rows >= 1, n_pt)")
            lib().orc_run_sched(C.byref(self._s), _p(T), nsteps, int(step0), Ws.shape[0],
                                _p(Ws), _p(w["Fe"]), _p(w["F"]), _p(w["C"]), _p(w["Q"]),
                                _p(w["Tn"]), _p(hist))
        return hist if history else T

    def adjoint(self, hist, lam_final):
        """Exact discrete adjoint of ``run`` (the transpose of its recursion,
        including the temperature dependence of D, c and radiation).

        Returns dict(g_logk[E], g_c[E], g_h[F], lam0[N]) for a loss whose
        gradient with respect to the final temperatures is ``lam_final``:
        derivatives with respect to the log of the per-element conductivity
        factors, the per-element heat capacities c0, the per-face convection
        coefficients and the initial temperatures (0 on Dirichlet nodes).
        """
        nsteps = hist.shape[0] - 1
        hist = np.ascontiguousarray(hist, dtype=np.float64)
        lam = _f64(lam_final).copy()
        g_logk, g_c = np.zeros(self.E), np.zeros(self.E)
        g_h = np.zeros(self.faces.shape[0])
        rc = lib().orc_adjoint(C.byref(self._s), _p(hist), nsteps, _p(self.is_dir, _i8),
                               _p(lam), _p(g_logk), _p(g_c), _p(g_h))
        if rc != 0:
            raise MemoryError("oracle adjoint: out of memory")
        return dict(g_logk=g_logk, g_c=g_c, g_h=g_h, lam0=lam)


def threads():
    """Threads the oracle's element loop uses (OpenMP)."""
    return int(lib().orc_threads())


def set_threads(n):
    """Sets the oracle's OpenMP thread count (n >= 1)."""
    lib().orc_set_threads(int(n))


def err_max(T, Tref):
    """max_k |T_k - Tref_k| / max_k |Tref_k|  (the parity norm)."""
    T, Tref = np.asarray(T, np.float64), np.asarray(Tref, np.float64)
    return float(np.max(np.abs(T - Tref)) / max(np.max(np.abs(Tref)), 1e-300))


def err_rms(T, Tref):
    """Eq. 30: sqrt(sum (Tref - T)^2 / sum Tref^2)."""
    T, Tref = np.asarray(T, np.float64), np.asarray(Tref, np.float64)
    return float(np.sqrt(np.sum((Tref - T) ** 2) / np.sum(Tref ** 2)))
