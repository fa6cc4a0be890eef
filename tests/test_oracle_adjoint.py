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


def test_stage_mass_terms_sum_by_parts():
    """The reverse sweep on the device pairs each stage's forward residual
    with b_s times the adjoint state the stage reads instead of pairing the
    stage right-hand side with the stage's adjoint vector.  Over one
    low-storage Runge-Kutta step the two sums agree because the first stage
    discards the residual (a_1 = 0), res_s = a_s res_{s-1} + dt R_s, and the
    sweep's recurrence sig_s = a_{s+1} sig_{s+1} + b_s U~_s (sig_6 = 0)."""
    from oracle import lsrk

    a, b = lsrk.A, lsrk.B
    assert a[0] == 0.0
    rng = np.random.default_rng(5)
    n, dt = 37, 0.013
    R = rng.standard_normal((5, n))  # stage right-hand sides
    Ua = rng.standard_normal((5, n))  # adjoint state read by each reverse stage
    res = np.zeros((5, n))
    prev = rng.standard_normal(n)  # last step's residual, discarded by stage 1
    for s in range(5):
        prev = a[s] * prev + dt * R[s]
        res[s] = prev
    sig = np.zeros((6, n))
    for s in range(4, -1, -1):
        sig[s] = (a[s + 1] * sig[s + 1] if s < 4 else 0.0) + b[s] * Ua[s]
    lhs = sum(sig[s] @ (dt * R[s]) for s in range(5))
    rhs = sum(b[s] * (Ua[s] @ res[s]) for s in range(5))
    assert abs(lhs - rhs) <= 1e-13 * (abs(lhs) + 1.0)
    # a plausible slip, pairing each residual with sig_s itself, does not agree
    wrong = sum(sig[s] @ res[s] for s in range(5))
    assert abs(wrong - lhs) > 1e-3 * abs(lhs)
