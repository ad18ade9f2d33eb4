"""torch.autograd front end of the library's forward steps and adjoint.

``FEDFunction.apply(log_k, elem_c, face_h, T0, sim, nsteps)`` runs nsteps
explicit steps from T0 with per-element conductivity factors exp(log_k),
per-element heat capacities elem_c and per-face convection coefficients
face_h (each may be None to keep the problem's values) and returns the final
temperatures as a CUDA float64 tensor.  Its backward is the library's
hand-written discrete adjoint (fed_backward): checkpoints every ``sim``'s
checkpoint interval (set with ``sim.checkpoint_every`` before the call),
each segment recomputed from its checkpoint or, after ``sim.keep_states()``
on a resident context, read from the states the forward kept; FP64 gradient
accumulators.  The adjoint differentiates through D(T), c(T), radiation,
property tables and the uniform-gradient hexahedron (with or without
hourglass control).  Torch provides tensors and the stream only.
"""
from __future__ import annotations

import torch


class FEDFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, log_k, elem_c, face_h, T0, sim, nsteps):
        sim.set_params(kscale=None if log_k is None else torch.exp(log_k.detach().double()),
                       elem_c=None if elem_c is None else elem_c.detach().double(),
                       face_h=None if face_h is None else face_h.detach().double())
        sim.set_temperature(T0.detach().double().contiguous())
        sim.step(int(nsteps))
        out = torch.empty(sim.N, dtype=torch.float64, device=T0.device)
        sim.temperature(out=out)
        ctx.sim = sim
        ctx.run = sim.run_id
        ctx.has = (log_k is not None, elem_c is not None, face_h is not None)
        return out

    @staticmethod
    def backward(ctx, gT):
        if ctx.sim.run_id != ctx.run:
            # the context's checkpoints and parameters belong to a later run
            raise RuntimeError("FEDFunction.backward: the simulation has started another run "
                               "since this output was computed; use one Simulation per "
                               "differentiated run")
        g = ctx.sim.backward(gT.contiguous())
        hk, hc, hh = ctx.has
        return (g["logk"] if hk else None, g["c"] if hc else None, g["h"] if hh else None,
                g["T0"], None, None)


def run(sim, nsteps, T0, log_k=None, elem_c=None, face_h=None):
    """Differentiable final temperatures; see FEDFunction."""
    return FEDFunction.apply(log_k, elem_c, face_h, T0, sim, nsteps)
