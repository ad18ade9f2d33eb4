"""MI355X-native FED-FEM: the per-time-step hot path of the fast explicit
dynamics finite element algorithm for transient heat transfer (Zhang &
Chauhan, arXiv 1909.03355) as hand-written HIP kernels behind a C ABI.

The compute lives in ``libfedfem.so``; this package only marshals
arguments.  There is no CPU fallback: if the library is missing, using it
raises.
"""
from ._lib import FedError, lib  # noqa: F401
from .sim import Simulation  # noqa: F401
