"""Receiver traces as a differentiable function of the per-element wave
speed and density.

``receiver_traces(solver, c, rho, U0, nsteps, dt)`` runs the time-stepped
solve on the device and returns the pressure at the solver's receivers after
every step, a (nsteps, nrec) float64 tensor.  Its backward is the discrete
adjoint of the whole solve: the incoming gradient of the traces becomes the
receivers' adjoint sources, forward states are recomputed from the
checkpoints the forward kept (wdg_adjoint_record; if the solver has run
something else since, wdg_adjoint_gradient redoes the forward sweep), and the
gradient with respect to c and rho comes back per element.  Only argument
marshalling happens here.
"""
from __future__ import annotations

import numpy as np
import torch

from .wdg import Solver


def _host(x) -> np.ndarray:
    return np.ascontiguousarray(x.detach().to("cpu", torch.float64).numpy())


class ReceiverTraces(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c, rho, solver: Solver, U0: np.ndarray, t0: float, nsteps: int, dt: float,
                checkpoint_every: int):
        cm, rm = _host(c), _host(rho)
        solver.set_material(cm, rm)
        solver.set_fields(U0)
        solver.time = t0
        solver.adjoint_record(checkpoint_every, nsteps)
        solver.step(nsteps, dt)
        traces = solver.read_receivers()
        ctx.solver = solver
        ctx.record_id = solver.record_id
        ctx.setup = (cm, rm, U0, t0, int(nsteps), float(dt), int(checkpoint_every))
        ctx.like = (c.dtype, c.device, rho.dtype, rho.device)
        return torch.as_tensor(traces, dtype=torch.float64)

    @staticmethod
    def backward(ctx, grad_traces):
        cm, rm, U0, t0, nsteps, dt, every = ctx.setup
        s = ctx.solver
        w = _host(grad_traces)
        if s.record_id == ctx.record_id and s.recorded_steps() == nsteps:
            # the checkpoints of this forward are still held by the solver
            gc, gr = s.adjoint_gradient_recorded(w)
        else:
            s.set_material(cm, rm)
            s.set_fields(U0)
            s.time = t0
            gc, gr = s.adjoint_gradient(nsteps, dt, w, every)
        cdt, cdev, rdt, rdev = ctx.like
        return (torch.as_tensor(gc, dtype=cdt, device=cdev), torch.as_tensor(gr, dtype=rdt, device=rdev),
                None, None, None, None, None, None)


def receiver_traces(solver: Solver, c, rho, U0, nsteps: int, dt: float, t0: float = 0.0,
                    checkpoint_every: int = 50):
    """Traces (nsteps, nrec) of the solve from fields U0 at time t0 with
    material (c, rho); differentiable with respect to c and rho."""
    return ReceiverTraces.apply(c, rho, solver, U0, t0, nsteps, dt, checkpoint_every)
