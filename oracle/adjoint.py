"""Receiver-misfit gradient with respect to per-element wave speed and
density (oracle, FP64; test infrastructure only).

The fully discrete forward map is the DG semi-discretisation of ``dg`` with
the LSRK(5,4) steps of ``lsrk`` and a Ricker point source; receivers sample
the pressure after every step.  The misfit is

    J(c, rho) = 1/2 sum_n sum_r (p_r(t_{n+1}) - d_{n,r})^2 .

Its exact gradient is taken by complex-step differentiation of the whole
discrete solve: with the material of element k perturbed by i h (h tiny),
Im J / h is dJ/dtheta_k to rounding, since every operation of the solve is
analytic in (c, rho) (kappa = rho c^2, Z = rho c, the upwind penalties, the
source vector) and no difference of nearby values is formed.  This is the
derivative of the discrete map, i.e. what a discrete adjoint computes.
"""
from __future__ import annotations

import numpy as np

from . import dg, lsrk


def solve_traces(mesh: dg.Mesh, N: int, U0: np.ndarray, dt: float, nsteps: int, src, rec: np.ndarray):
    """Receiver traces (nsteps, nrec) of the forward solve; complex material allowed."""
    ops = dg.build_operators(mesh, N)
    source = dg.make_point_source(mesh, N, *src) if src is not None else None
    rel, rows = dg.make_receivers(mesh, N, rec)
    cplx = np.iscomplexobj(mesh.c) or np.iscomplexobj(mesh.rho)
    U = np.array(U0, dtype=np.complex128 if cplx else np.float64, copy=True)
    res = np.zeros_like(U)

    def f(t, U):
        out = dg.rhs(ops, U)
        if source is not None:
            out[source.elem, 0] += source.value(t) * source.vec
        return out

    traces = []
    for n in range(nsteps):
        lsrk.step(f, n * dt, U, res, dt)
        traces.append(np.einsum("rj,rj->r", rows, U[rel, 0]))
    return np.array(traces)


def misfit(traces: np.ndarray, data: np.ndarray) -> float:
    return 0.5 * float(np.sum((traces - data) ** 2))


def gradient_complex_step(mesh: dg.Mesh, N: int, U0, dt: float, nsteps: int, src, rec, data, elems=None,
                          h: float = 1e-30):
    """(J, dJ/dc, dJ/drho) for the elements ``elems`` (default all)."""
    elems = np.arange(mesh.K) if elems is None else np.asarray(elems)
    J = misfit(solve_traces(mesh, N, U0, dt, nsteps, src, rec), data)
    gc = np.zeros(len(elems))
    gr = np.zeros(len(elems))
    for i, k in enumerate(elems):
        for which, out in (("c", gc), ("rho", gr)):
            c = mesh.c.astype(np.complex128)
            rho = mesh.rho.astype(np.complex128)
            (c if which == "c" else rho)[k] += 1j * h
            m = dg.Mesh(mesh.verts, mesh.wedges, c, rho, mesh.bc, mesh.flux, tets=mesh.tets)
            tr = solve_traces(m, N, U0, dt, nsteps, src, rec)
            out[i] = float(np.sum((tr.real - data) * tr.imag)) / h
    return J, gc, gr
