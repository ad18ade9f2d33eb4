"""Python front end of the FED-FEM GPU library.

``Simulation`` marshals a problem description (the dict layout documented in
``workloads.problems``) into the C ABI and exposes the three stages of the
method: pre-computation (construction), initialisation
(``set_temperature``) and time stepping (``step``).  PyTorch is used only for
device memory and the current HIP stream.
"""
from __future__ import annotations

import atexit
import ctypes as C
import weakref

import numpy as np

from . import _lib as L

PRECISIONS = {"fp32c": L.FED_FP32C, "fp64": L.FED_FP64, "fp32": L.FED_FP32}

# contexts still open; closed before the interpreter tears torch and the HIP
# runtime down, so no context outlives the allocator that owns its memory
_LIVE = weakref.WeakSet()


@atexit.register
def _close_all():
    for s in list(_LIVE):
        try:
            s.close()
        except Exception:
            pass


def torch_allocator(stream):
    """(dev_alloc, dev_free) hooks that take a context's device memory from
    torch's caching allocator on `stream` (a raw hipStream_t or None for the
    current stream), so torch owns and accounts for it."""
    import torch
    dev = torch.cuda.current_device()
    st = None if stream is None else int(stream.value or 0)

    def alloc(nbytes, _ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), dev, st)
        except RuntimeError:
            return None  # the library reports FED_E_HIP (out of memory)

    def free(ptr, _ctx):
        torch.cuda.caching_allocator_delete(ptr)

    return L.DEV_ALLOC(alloc), L.DEV_FREE(free)


def _ptr(a, t=C.c_double):
    return None if a is None else a.ctypes.data_as(C.POINTER(t))


def current_stream():
    """hipStream_t of torch's current stream (None = default stream)."""
    try:
        import torch
        if torch.cuda.is_available():
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    except ImportError:
        pass
    return None


class Simulation:
    def __init__(self, prob, prec="fp32c", tile_nodes=0, block_threads=0, fuse_steps=0,
                 allow_unstable=False, stream=None, resident=False, allocator="torch",
                 check_margin=None, check_every=0, energy_tol=0.0):
        """allocator: "torch" takes the device memory from torch's caching
        allocator (the default when torch sees a GPU), "hip" lets the library
        call hipMalloc.  check_margin, check_every, energy_tol: the in-run
        health check (fed_options in include/fedfem.h); check_margin None: the
        window the stability bound allows, a number: [T_lo - m, T_hi + m]."""
        lib = L.lib()
        self._ctx = None
        self.run_id = 0    # counts set_temperature / set_state / set_params calls
        self.prec = prec
        self.prob = prob
        f64 = lambda a: np.ascontiguousarray(a, dtype=np.float64)
        i32 = lambda a: np.ascontiguousarray(a, dtype=np.int32)
        keep = []   # arrays referenced by the ctypes structs until fed_create returns
        x, y, z = f64(prob["x"]), f64(prob["y"]), f64(prob["z"])
        conn = i32(prob["conn"])
        keep += [x, y, z, conn]
        self.N, self.E = x.size, conn.shape[1]
        mesh = L.fed_mesh(L.FED_HEX8 if prob["elem"] == "hex8" else L.FED_TET4, self.N, self.E,
                          _ptr(x), _ptr(y), _ptr(z), _ptr(conn, C.c_int32))
        mats_in = prob["materials"]
        arr = (L.fed_material * len(mats_in))()
        for i, m in enumerate(mats_in):
            arr[i].rho, arr[i].c0, arr[i].c1 = m["rho"], m["c0"], m["c1"]
            for r in range(6):
                arr[i].k[r] = m["k"][r]
            arr[i].s0, arr[i].s1 = m["s0"], m["s1"]
        emat = None if prob["elem_material"] is None else i32(prob["elem_material"])
        ek = None if prob["elem_k"] is None else f64(prob["elem_k"])
        ks = None if prob["elem_kscale"] is None else f64(prob["elem_kscale"])
        keep += [emat, ek, ks]
        # optional multiplier tables (T points, values) of D and c
        tabs = []
        for key in ("k_table", "c_table"):
            tb = prob.get(key)
            tb = (None, None) if tb is None else (f64(tb[0]), f64(tb[1]))
            keep += list(tb)
            tabs.append(tb)
        (kT, kf), (cT, cf) = tabs
        mats = L.fed_materials(len(mats_in), arr, _ptr(emat, C.c_int32), _ptr(ek), _ptr(ks),
                               0 if kT is None else kT.size, _ptr(kT), _ptr(kf),
                               0 if cT is None else cT.size, _ptr(cT), _ptr(cf))
        dn, dT = i32(prob["dir_nodes"]), f64(prob["dir_T"])
        keep += [dn, dT]
        faces = prob["faces"]
        if faces is not None and faces.shape[0] > 0:
            faces = i32(faces)
            fh, fTa, feps, fq = (f64(prob[k]) for k in ("face_h", "face_Ta", "face_eps", "face_q"))
            nf, nfn = faces.shape
        else:
            faces = fh = fTa = feps = fq = None
            nf, nfn = 0, 4
        keep += [faces, fh, fTa, feps, fq]
        pn, pW = i32(prob["pt_nodes"]), f64(prob["pt_W"])
        keep += [pn, pW]
        bcs = L.fed_bcs(dn.size, _ptr(dn, C.c_int32), _ptr(dT), nf, nfn, _ptr(faces, C.c_int32),
                        _ptr(fh), _ptr(fTa), _ptr(feps), _ptr(fq), pn.size, _ptr(pn, C.c_int32),
                        _ptr(pW), float(prob["Tz"]))
        inst = None if prob["node_instance"] is None else i32(prob["node_instance"])
        keep.append(inst)
        dt = 0.0 if prob["dt"] is None else float(prob["dt"])
        opt = L.fed_options(PRECISIONS[prec], dt, float(prob["safety"]), float(prob["T_lo"]),
                            float(prob["T_hi"]), int(bool(allow_unstable)),
                            _ptr(inst, C.c_int32), int(tile_nodes), int(block_threads),
                            int(fuse_steps), int(bool(resident)),
                            1 if prob.get("hex_gradient", "centre") == "mean" else 0,
                            float(prob.get("hourglass", 0.0) or 0.0))
        self.stream = current_stream() if stream is None else stream
        if allocator not in ("torch", "hip"):
            raise ValueError("allocator must be 'torch' or 'hip'")
        self._hooks = None
        if allocator == "torch":
            try:
                import torch
                if torch.cuda.is_available():
                    self._hooks = torch_allocator(self.stream)
            except ImportError:
                pass
        if self._hooks is not None:
            # the callbacks live as long as the context (self._hooks)
            opt.dev_alloc, opt.dev_free = self._hooks
        opt.check_window = 0 if check_margin is None else 1
        opt.check_margin = 0.0 if check_margin is None else float(check_margin)
        opt.check_every = int(check_every)
        opt.energy_tol = float(energy_tol)
        self.allocator = "torch" if self._hooks is not None else "hip"
        ctx = C.c_void_p()
        L.check(lib.fed_create(C.byref(mesh), C.byref(mats), C.byref(bcs), C.byref(opt),
                               self.stream, C.byref(ctx)))
        self._ctx = ctx
        _LIVE.add(self)
        info = L.fed_info()
        L.check(lib.fed_info_get(ctx, C.byref(info)))
        self.info = {k: getattr(info, k) for k, _ in L.fed_info._fields_}
        n = self.info["n_instances"]
        self.dt_crit, self.dt = np.zeros(n), np.zeros(n)
        L.check(lib.fed_dt(ctx, _ptr(self.dt_crit), _ptr(self.dt), n))

    # ------------------------------------------------------------------
    def _c(self):
        if self._ctx is None:
            raise RuntimeError("simulation closed")
        return self._ctx

    def set_temperature(self, T=None):
        """Initialisation (Sec. 3.5 (ii)): T0 (caller order, FP64 numpy array or
        CUDA tensor; default the problem's T0) with the Dirichlet values applied."""
        T = self.prob["T0"] if T is None else T
        self.run_id += 1   # a new run: steps, checkpoints and states start over
        if hasattr(T, "is_cuda") and T.is_cuda:
            import torch
            assert T.dtype == torch.float64 and T.is_contiguous() and T.numel() == self.N
            L.check(L.lib().fed_set_temperature(self._c(), C.c_void_p(T.data_ptr()), 1, self.stream))
        else:
            Th = np.ascontiguousarray(T, dtype=np.float64)
            assert Th.size == self.N
            L.check(L.lib().fed_set_temperature(self._c(), Th.ctypes.data_as(C.c_void_p), 0,
                                                self.stream))

    def step(self, n, graph_steps=None):
        """Enqueue n explicit steps (asynchronous)."""
        if graph_steps:
            L.check(L.lib().fed_step_graph(self._c(), int(n), int(graph_steps), self.stream))
        else:
            L.check(L.lib().fed_step(self._c(), int(n), self.stream))

    def temperature(self, out=None):
        """Current temperatures (FP64, caller order).  Synchronises; raises
        FedError(FED_E_UNSTABLE) if the health check fired."""
        if out is not None:
            L.check(L.lib().fed_get_temperature(self._c(), C.c_void_p(out.data_ptr()), 1,
                                                self.stream))
            return out
        T = np.empty(self.N)
        L.check(L.lib().fed_get_temperature(self._c(), T.ctypes.data_as(C.c_void_p), 0,
                                            self.stream))
        return T

    def health(self):
        """The in-run health record (synchronises): steps, first_bad_step (-1
        if none), the window, energy_residual, energy_step, energy_checks."""
        h = L.fed_health()
        L.check(L.lib().fed_health_get(self._c(), C.byref(h), self.stream))
        return {k: getattr(h, k) for k, _ in L.fed_health._fields_}

    @property
    def device_bytes(self):
        """Device memory the context holds now (bytes)."""
        info = L.fed_info()
        L.check(L.lib().fed_info_get(self._c(), C.byref(info)))
        return info.device_bytes

    @property
    def steps_taken(self):
        v = C.c_int64()
        L.check(L.lib().fed_steps_taken(self._c(), C.byref(v)))
        return v.value

    def get_state(self):
        dt = np.float64 if self.prec == "fp64" else np.float32
        hi, lo = np.empty(self.N, dt), np.empty(self.N, np.float32)
        st = C.c_int64()
        L.check(L.lib().fed_get_state(self._c(), hi.ctypes.data_as(C.c_void_p),
                                      lo.ctypes.data_as(C.c_void_p), C.byref(st), self.stream))
        return hi, lo, st.value

    def set_state(self, hi, lo, step):
        self.run_id += 1
        dt = np.float64 if self.prec == "fp64" else np.float32
        hi = np.ascontiguousarray(hi, dtype=dt)
        lo = np.ascontiguousarray(lo, dtype=np.float32)
        L.check(L.lib().fed_set_state(self._c(), hi.ctypes.data_as(C.c_void_p),
                                      lo.ctypes.data_as(C.c_void_p), int(step), self.stream))

    # ---- adjoint -------------------------------------------------------
    def checkpoint_every(self, every):
        """Keep the state every `every` steps for the adjoint (before
        set_temperature; 0 turns it off)."""
        L.check(L.lib().fed_checkpoint_every(self._c(), int(every)))

    @staticmethod
    def _arg(a):
        """(pointer, on_device, keep-alive) for an FP64 array or CUDA tensor."""
        if a is None:
            return None, None, None
        if hasattr(a, "is_cuda") and a.is_cuda:
            import torch
            t = a.detach().to(torch.float64).contiguous()
            return C.c_void_p(t.data_ptr()), 1, t
        h = np.ascontiguousarray(a, dtype=np.float64)
        return h.ctypes.data_as(C.c_void_p), 0, h

    def set_params(self, kscale=None, elem_c=None, face_h=None):
        """Replace per-element conductivity factors, per-element heat capacities
        and per-face convection coefficients; re-derives the precomputed arrays."""
        self.run_id += 1   # the parameters of the adjoint change
        args = [self._arg(a) for a in (kscale, elem_c, face_h)]
        dev = {d for _, d, _ in args if d is not None}
        if len(dev) > 1:
            raise ValueError("pass all parameters on the host or all on the device")
        on_dev = dev.pop() if dev else 0
        L.check(L.lib().fed_set_params(self._c(), args[0][0], args[1][0], args[2][0], on_dev,
                                       self.stream))

    def set_bc(self, face_Ta=None, face_q=None, pt_W=None):
        """Time-varying boundary conditions: replace the per-face ambient
        temperatures, heat fluxes and concentrated loads for the steps that
        follow (numpy arrays, validated; or CUDA tensors, asynchronous)."""
        args = [self._arg(a) for a in (face_Ta, face_q, pt_W)]
        dev = {d for _, d, _ in args if d is not None}
        if len(dev) > 1:
            raise ValueError("pass all arrays on the host or all on the device")
        on_dev = dev.pop() if dev else 0
        L.check(L.lib().fed_set_bc(self._c(), args[0][0], args[1][0], args[2][0], on_dev,
                                   self.stream))
        self._keep_bc = args  # device tensors stay alive until the copies have run

    def set_point_schedule(self, W):
        """Per-step concentrated loads: W is (n_rows, n_pt) (numpy, validated,
        or a CUDA tensor); step n since set_temperature applies row n mod
        n_rows.  None removes the schedule."""
        if W is None:
            L.check(L.lib().fed_set_point_schedule(self._c(), None, 0, 0, self.stream))
            self._keep_sched = None
            return
        if len(W.shape) != 2:
            raise ValueError("W must be (n_rows, n_pt)")
        ptr, on_dev, keep = self._arg(W)
        L.check(L.lib().fed_set_point_schedule(self._c(), ptr, int(W.shape[0]), on_dev,
                                               self.stream))
        self._keep_sched = keep  # a device tensor stays alive until the copy has run

    def keep_states(self, on=True):
        """Keep every forward state for the adjoint instead of recomputing the
        checkpoint segments (resident contexts; after checkpoint_every)."""
        L.check(L.lib().fed_keep_states(self._c(), int(bool(on))))

    def test_waits(self, spin_limit=0, never_match=False):
        """Test hook of resident stepping's failure path (see fed_test_waits)."""
        L.check(L.lib().fed_test_waits(self._c(), int(spin_limit), int(bool(never_match))))

    def temperature_range(self):
        """(min, max) of the current temperatures (synchronises)."""
        lo, hi = C.c_double(), C.c_double()
        L.check(L.lib().fed_temperature_range(self._c(), C.byref(lo), C.byref(hi), self.stream))
        return lo.value, hi.value

    def set_range(self, T_lo, T_hi):
        """Re-derive the stability bound for [T_lo, T_hi] (raises FedError with
        FED_E_UNSTABLE if the time step in use exceeds it)."""
        try:
            L.check(L.lib().fed_set_range(self._c(), float(T_lo), float(T_hi), self.stream))
        finally:
            self._refresh_dt()

    def _refresh_dt(self):
        n = self.info["n_instances"]
        L.check(L.lib().fed_dt(self._c(), _ptr(self.dt_crit), _ptr(self.dt), n))

    def backward(self, dL_dT):
        """Discrete adjoint of the steps taken: returns dict(logk, c, h, T0) of
        dL/dlog k_e, dL/dc_e, dL/dh_f and dL/dT0 (numpy, or CUDA tensors when
        dL_dT is a CUDA tensor)."""
        nf = 0 if self.prob["faces"] is None else self.prob["faces"].shape[0]
        if hasattr(dL_dT, "is_cuda") and dL_dT.is_cuda:
            import torch
            g = dL_dT.detach().to(torch.float64).contiguous()
            out = {k: torch.zeros(n, dtype=torch.float64, device=g.device)
                   for k, n in (("logk", self.E), ("c", self.E), ("h", max(nf, 1)), ("T0", self.N))}
            ptr = lambda t: C.c_void_p(t.data_ptr())
            L.check(L.lib().fed_backward(self._c(), ptr(g), ptr(out["logk"]), ptr(out["c"]),
                                         ptr(out["h"]) if nf else None, ptr(out["T0"]), 1,
                                         self.stream))
            out["h"] = out["h"][:nf]
            return out
        g = np.ascontiguousarray(dL_dT, dtype=np.float64)
        out = {"logk": np.zeros(self.E), "c": np.zeros(self.E), "h": np.zeros(nf),
               "T0": np.zeros(self.N)}
        ptr = lambda a: a.ctypes.data_as(C.c_void_p)
        L.check(L.lib().fed_backward(self._c(), ptr(g), ptr(out["logk"]), ptr(out["c"]),
                                     ptr(out["h"]) if nf else None, ptr(out["T0"]), 0, self.stream))
        return out

    def close(self):
        if getattr(self, "_ctx", None) is not None:
            L.lib().fed_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
