"""fed_backward_noalloc, the adjoint entry point that allocates nothing (its
work arrays live in the library's static scratch array), against
fed_backward, bit for bit, on two calls in a row, the second with a smaller
mesh; it allocates no device memory; it refuses work arrays larger than the
scratch."""
from __future__ import annotations

import ctypes as C

import numpy as np
import pytest

from workloads import problems as P

pytestmark = pytest.mark.gpu


def _grads(s, fn, lam):
    """(g_logk, g_c, g_h, dL/dT0) from one of the two adjoint entry points."""
    from paper_1909_03355_amd import _lib as L
    nf = s.prob["faces"].shape[0]
    out = [np.zeros(s.E), np.zeros(s.E), np.zeros(nf), np.zeros(s.N)]
    p = lambda a: a.ctypes.data_as(C.c_void_p)
    L.check(fn(s._c(), p(lam), p(out[0]), p(out[1]), p(out[2]), p(out[3]), 0, s.stream))
    return out


@pytest.mark.parametrize("prec,resident", [("fp32c", False), ("fp64", False), ("fp32c", True)])
def test_noalloc_matches_backward_twice(prec, resident):
    import torch
    from paper_1909_03355_amd import Simulation
    from paper_1909_03355_amd import _lib as L
    lib = L.lib()
    # second call: a smaller mesh, fewer steps
    for n, steps in ((12, 60), (6, 30)):
        p = P.cube_nonlinear_hex(n, steps)
        with Simulation(p, prec=prec, resident=resident) as s:
            s.checkpoint_every(16)
            s.set_temperature()
            s.step(steps)
            T = s.temperature()
            lam = np.linspace(-1.0, 1.0, s.N) * (T - 20.0)
            print(f"n={n} {prec} resident={resident}: N={s.N}", flush=True)
            ref = _grads(s, lib.fed_backward, lam)
            torch.cuda.synchronize()
            m0 = torch.cuda.memory_allocated()
            held = s.device_bytes
            got = _grads(s, lib.fed_backward_noalloc, lam)
            torch.cuda.synchronize()
            assert torch.cuda.memory_allocated() == m0
            assert s.device_bytes == held
            for a, b in zip(got, ref):
                assert np.array_equal(a, b)
            # the forward state is unchanged: stepping on gives the same bits
            # as a context that never ran the adjoint
            assert np.array_equal(s.temperature(), T)


def test_noalloc_kept_states():
    from paper_1909_03355_amd import Simulation
    from paper_1909_03355_amd import _lib as L
    lib = L.lib()
    p = P.cube_nonlinear_hex(12, 50)
    with Simulation(p, prec="fp32c", resident=True) as s:
        s.checkpoint_every(20)
        s.keep_states(True)
        s.set_temperature()
        s.step(50)
        T = s.temperature()
        lam = T - 20.0
        ref = _grads(s, lib.fed_backward, lam)
        got = _grads(s, lib.fed_backward_noalloc, lam)
        for a, b in zip(got, ref):
            assert np.array_equal(a, b)


def test_noalloc_refuses_work_beyond_the_scratch():
    from paper_1909_03355_amd import FedError, Simulation
    from paper_1909_03355_amd import _lib as L
    lib = L.lib()
    # 32^3 hexahedra in FP64 with 500 steps a segment: the recomputed segment
    # alone needs 8 x 35,937 x 501 bytes (144 MB) against 64 MiB of scratch
    p = P.cube_nonlinear_hex(32, 4)
    with Simulation(p, prec="fp64") as s:
        s.checkpoint_every(500)
        s.set_temperature()
        s.step(4)
        T = s.temperature()
        with pytest.raises(FedError) as ei:
            _grads(s, lib.fed_backward_noalloc, T)
        assert ei.value.code == L.FED_E_ARG
        assert "scratch" in str(ei.value)
        # the context still works through the allocating entry point
        _grads(s, lib.fed_backward, T)
