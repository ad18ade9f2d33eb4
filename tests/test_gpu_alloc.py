"""Device memory from the caller's allocator (fed_options.dev_alloc/dev_free):
the Python front end hands the library torch's caching allocator, so torch
owns and accounts for every buffer of a context; results are bitwise those of
a context whose memory comes from hipMalloc; closing the context gives the
memory back; a lone hook is refused."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from workloads import problems as P

pytestmark = pytest.mark.gpu


def _run(p, prec, allocator, nsteps=60, ckpt=0):
    from paper_1909_03355_amd import Simulation
    with Simulation(p, prec=prec, allocator=allocator, tile_nodes=40) as s:
        if ckpt:
            s.checkpoint_every(ckpt)
        s.set_temperature()
        s.step(nsteps)
        T = s.temperature()
        return T, s.device_bytes


@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
def test_torch_allocator_owns_the_context(prec):
    import torch
    from paper_1909_03355_amd import Simulation
    p = P.cube_nonlinear_hex(8, 60)
    torch.cuda.synchronize()
    m0 = torch.cuda.memory_allocated()
    s = Simulation(p, prec=prec, allocator="torch", tile_nodes=40)
    assert s.allocator == "torch"
    held = s.device_bytes
    grown = torch.cuda.memory_allocated() - m0
    print(f"{prec}: context holds {held} B, torch's allocator grew by {grown} B", flush=True)
    assert held > 0
    # every buffer is a torch block (rounded up to 512 B); the temporaries of
    # fed_create have been given back
    assert held <= grown <= held + 512 * 128
    # checkpoints taken later come from the same allocator
    s.checkpoint_every(20)
    s.set_temperature()
    s.step(60)
    T = s.temperature()
    assert s.device_bytes > held
    assert torch.cuda.memory_allocated() - m0 >= s.device_bytes
    s.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == m0
    # parity unchanged: the same bits as with hipMalloc, within the oracle tolerance
    T_hip, held_hip = _run(p, prec, "hip", ckpt=20)
    assert np.array_equal(T, T_hip)
    ref = oracle.Oracle(p).run(60)
    assert oracle.err_max(T, ref) <= (1e-12 if prec == "fp64" else 1e-5)


def test_resident_and_adjoint_with_torch_allocator():
    import torch
    from paper_1909_03355_amd import Simulation
    p = P.cube_nonlinear_hex(12, 40)
    g = {}
    for alloc in ("torch", "hip"):
        with Simulation(p, prec="fp32c", allocator=alloc, resident=True) as s:
            s.checkpoint_every(10)
            s.set_temperature()
            s.step(40)
            T = s.temperature()
            g[alloc] = (T, s.backward(np.ones_like(T))["logk"])
        torch.cuda.synchronize()
    assert np.array_equal(g["torch"][0], g["hip"][0])
    assert np.array_equal(g["torch"][1], g["hip"][1])


def test_lone_hook_is_refused():
    from paper_1909_03355_amd import FedError, Simulation
    from paper_1909_03355_amd import _lib as L
    p = P.cube_nonlinear_hex(4, 10)
    # a context built through the binding but with dev_free left NULL
    import paper_1909_03355_amd.sim as S
    real = S.torch_allocator

    def half(stream):
        a, _ = real(stream)
        return a, L.DEV_FREE()
    S.torch_allocator = half
    try:
        with pytest.raises(FedError) as ei:
            Simulation(p, prec="fp32c", allocator="torch")
        assert ei.value.code == L.FED_E_ARG
        assert "together" in str(ei.value)
    finally:
        S.torch_allocator = real
