"""ctypes binding of libfedfem.so (the C ABI in include/fedfem.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  Importing this module raises if the library is missing; there
is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfedfem.so")

FED_OK, FED_E_ARG, FED_E_MESH, FED_E_UNSTABLE, FED_E_HIP, FED_E_STATE, FED_E_NOMEM = \
    0, -1, -2, -3, -4, -5, -6
FED_TET4, FED_HEX8 = 4, 8
FED_FP32C, FED_FP64, FED_FP32 = 0, 1, 2

STATUS_NAMES = {0: "FED_OK", -1: "FED_E_ARG", -2: "FED_E_MESH", -3: "FED_E_UNSTABLE",
                -4: "FED_E_HIP", -5: "FED_E_STATE", -6: "FED_E_NOMEM"}

_d = C.POINTER(C.c_double)
_i32 = C.POINTER(C.c_int32)


class fed_mesh(C.Structure):
    _fields_ = [("elem", C.c_int32), ("n_nodes", C.c_int64), ("n_elems", C.c_int64),
                ("x", _d), ("y", _d), ("z", _d), ("conn", _i32)]


class fed_material(C.Structure):
    _fields_ = [("rho", C.c_double), ("c0", C.c_double), ("c1", C.c_double),
                ("k", C.c_double * 6), ("s0", C.c_double), ("s1", C.c_double)]


class fed_materials(C.Structure):
    _fields_ = [("n_materials", C.c_int32), ("materials", C.POINTER(fed_material)),
                ("elem_material", _i32), ("elem_k", _d), ("elem_kscale", _d),
                ("n_ktab", C.c_int32), ("ktab_T", _d), ("ktab_f", _d),
                ("n_ctab", C.c_int32), ("ctab_T", _d), ("ctab_f", _d)]


class fed_bcs(C.Structure):
    _fields_ = [("n_dir", C.c_int64), ("dir_nodes", _i32), ("dir_T", _d),
                ("n_faces", C.c_int64), ("face_nodes", C.c_int32), ("faces", _i32),
                ("face_h", _d), ("face_Ta", _d), ("face_eps", _d), ("face_q", _d),
                ("n_pt", C.c_int64), ("pt_nodes", _i32), ("pt_W", _d), ("Tz", C.c_double)]


# device-memory hooks of fed_options: dev_alloc(bytes, alloc_ctx) -> pointer or
# NULL, dev_free(pointer, alloc_ctx)
DEV_ALLOC = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
DEV_FREE = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class fed_options(C.Structure):
    _fields_ = [("prec", C.c_int32), ("dt", C.c_double), ("safety", C.c_double),
                ("T_lo", C.c_double), ("T_hi", C.c_double), ("allow_unstable", C.c_int32),
                ("node_instance", _i32), ("tile_nodes", C.c_int32),
                ("block_threads", C.c_int32), ("fuse_steps", C.c_int32),
                ("resident", C.c_int32), ("hex_gradient", C.c_int32),
                ("hourglass", C.c_double),
                ("dev_alloc", DEV_ALLOC), ("dev_free", DEV_FREE), ("alloc_ctx", C.c_void_p),
                ("check_window", C.c_int32), ("check_margin", C.c_double),
                ("check_every", C.c_int32),
                ("energy_tol", C.c_double)]


class fed_health(C.Structure):
    _fields_ = [("steps", C.c_int64), ("first_bad_step", C.c_int64),
                ("window_lo", C.c_double), ("window_hi", C.c_double),
                ("energy_residual", C.c_double), ("energy_step", C.c_int64),
                ("energy_checks", C.c_int64)]


class fed_info(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("n_elems", C.c_int64), ("n_instances", C.c_int64),
                ("n_tiles", C.c_int64), ("n_elems_expanded", C.c_int64),
                ("n_halo", C.c_int64), ("n_bnd_nodes", C.c_int64),
                ("elem", C.c_int32), ("prec", C.c_int32), ("block_threads", C.c_int32),
                ("lds_bytes", C.c_int32), ("fuse_steps", C.c_int32), ("resident", C.c_int32),
                ("algorithmic_bytes_per_launch", C.c_double),
                ("moved_bytes_per_launch", C.c_double),
                ("exchange_bytes_per_step", C.c_double),
                ("resident_adjoint", C.c_int32), ("reserved_", C.c_int32),
                ("device_bytes", C.c_int64), ("reread_bytes_per_step", C.c_double)]


# name -> (restype, argtypes) of every symbol the header declares
SIGNATURES = {
    "fed_create": (C.c_int, [C.POINTER(fed_mesh), C.POINTER(fed_materials), C.POINTER(fed_bcs),
                             C.POINTER(fed_options), C.c_void_p, C.POINTER(C.c_void_p)]),
    "fed_dt": (C.c_int, [C.c_void_p, _d, _d, C.c_int64]),
    "fed_info_get": (C.c_int, [C.c_void_p, C.POINTER(fed_info)]),
    "fed_set_temperature": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]),
    "fed_step": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p]),
    "fed_step_graph": (C.c_int, [C.c_void_p, C.c_int64, C.c_int32, C.c_void_p]),
    "fed_get_temperature": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]),
    "fed_steps_taken": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64)]),
    "fed_health_get": (C.c_int, [C.c_void_p, C.POINTER(fed_health), C.c_void_p]),
    "fed_get_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_int64),
                                C.c_void_p]),
    "fed_set_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]),
    "fed_checkpoint_every": (C.c_int, [C.c_void_p, C.c_int64]),
    "fed_set_params": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                 C.c_void_p]),
    "fed_set_bc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                             C.c_void_p]),
    "fed_set_point_schedule": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int32,
                                         C.c_void_p]),
    "fed_test_waits": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32]),
    "fed_keep_states": (C.c_int, [C.c_void_p, C.c_int32]),
    "fed_temperature_range": (C.c_int, [C.c_void_p, _d, _d, C.c_void_p]),
    "fed_set_range": (C.c_int, [C.c_void_p, C.c_double, C.c_double, C.c_void_p]),
    "fed_backward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                               C.c_void_p, C.c_int32, C.c_void_p]),
    "fed_backward_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                       C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]),
    "fed_destroy": (None, [C.c_void_p]),
    "fed_last_error": (C.c_char_p, []),
}

_LIB = None


class FedError(RuntimeError):
    def __init__(self, code, msg):
        self.code = code
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")


def lib():
    """The loaded library; raises if it has not been built."""
    global _LIB
    if _LIB is None:
        # torch ships its own HIP runtime and loads it by file name; importing it
        # first lets that runtime (same soname) satisfy this library's dependency,
        # so the process holds one HIP runtime and torch tensors/streams are ours.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1909_03355_amd.build` (no CPU fallback exists)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


def check(rc):
    if rc != FED_OK:
        raise FedError(rc, lib().fed_last_error().decode())
    return rc
