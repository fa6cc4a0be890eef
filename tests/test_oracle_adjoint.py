"""Pins of the oracle's misfit gradient (complex-step derivative of the
fully discrete solve) against central finite differences and basic
invariants."""
import numpy as np
import pytest

from oracle import adjoint, dg
from paper_1607_03399_amd import inputs


def _problem(flux="upwind", bc="rigid", hybrid=False):
    m = inputs.layered_config(2, 2, 0.3, seed=4)  # 16 wedges, banded c and rho
    if hybrid:
        v, w, t, c, rho = inputs.split_columns(m, [3])
        mesh = dg.Mesh(v, w, c, rho, bc, flux, tets=t)
    else:
        mesh = dg.Mesh(m.verts, m.wedges, m.c, m.rho, bc, flux)
    N = 2
    x = dg.node_coords(mesh, N)
    mask = dg.node_mask(mesh, N)
    U0 = np.zeros((mesh.K, 4, x.shape[1]))
    U0[:, 0] = inputs.gaussian_pulse(x, width=0.25) * mask
    dt = dg.stable_dt(mesh, N, 0.5)
    src = ([0.3, 0.6, 0.4], 4.0, 0.15, 1.0)
    rec = np.array([[0.7, 0.3, 0.8], [0.2, 0.2, 0.3]])
    return mesh, N, U0, dt, src, rec


@pytest.mark.parametrize("flux,hybrid", [("upwind", False), ("central", False), ("upwind", True)])
def test_gradient_matches_central_differences(flux, hybrid):
    mesh, N, U0, dt, src, rec = _problem(flux=flux, hybrid=hybrid)
    nsteps = 12
    base = adjoint.solve_traces(mesh, N, U0, dt, nsteps, src, rec)
    data = 0.9 * base + 0.01  # a misfit with non-zero residuals
    elems = [0, 5, mesh.K - 1]
    J, gc, gr = adjoint.gradient_complex_step(mesh, N, U0, dt, nsteps, src, rec, data, elems=elems)
    assert J > 0
    for i, k in enumerate(elems):
        for which, g in (("c", gc[i]), ("rho", gr[i])):
            vals = []
            for sgn in (1, -1):
                c, rho = mesh.c.copy(), mesh.rho.copy()
                arr = c if which == "c" else rho
                eps = 1e-5 * arr[k]
                arr[k] += sgn * eps
                m = dg.Mesh(mesh.verts, mesh.wedges, c, rho, mesh.bc, mesh.flux, tets=mesh.tets)
                vals.append(adjoint.misfit(adjoint.solve_traces(m, N, U0, dt, nsteps, src, rec), data))
            fd = (vals[0] - vals[1]) / (2 * eps)
            assert abs(fd - g) <= 1e-6 * max(abs(g), 1e-3 * abs(J))


def test_gradient_vanishes_at_the_data_and_is_linear():
    mesh, N, U0, dt, src, rec = _problem()
    nsteps = 8
    data = adjoint.solve_traces(mesh, N, U0, dt, nsteps, src, rec)
    J, gc, gr = adjoint.gradient_complex_step(mesh, N, U0, dt, nsteps, src, rec, data, elems=[1, 2])
    # (the complex solve's real part differs from the real solve by rounding only)
    assert J == 0.0 and np.abs(gc).max() < 1e-14 and np.abs(gr).max() < 1e-14
    # directional derivative along v equals the sum of the per-element ones
    data = data * 1.1
    elems = [1, 2, 7]
    J, gc, gr = adjoint.gradient_complex_step(mesh, N, U0, dt, nsteps, src, rec, data, elems=elems)
    v = np.array([0.3, -1.0, 0.5])
    c = mesh.c.astype(complex)
    c[elems] += 1e-30j * v
    m = dg.Mesh(mesh.verts, mesh.wedges, c, mesh.rho, mesh.bc, mesh.flux)
    tr = adjoint.solve_traces(m, N, U0, dt, nsteps, src, rec)
    d = float(np.sum((tr.real - data) * tr.imag)) / 1e-30
    assert abs(d - np.dot(v, gc)) <= 1e-12 * max(abs(d), 1e-300)
