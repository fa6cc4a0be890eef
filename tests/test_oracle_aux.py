"""Pins of the oracle's auxiliary pieces: sources, receivers, point location,
energy, node coordinates and the subset (sampled) RHS mode."""
import numpy as np

from oracle import dg
from paper_1607_03399_amd import inputs


def _mesh(m, bc="rigid", flux="upwind"):
    return dg.Mesh(m.verts, m.wedges, m.c, m.rho, bc, flux)


def test_ricker_closed_form():
    f0, t0 = 10.0, 0.1
    assert abs(dg.ricker(t0, f0, t0, 2.5) - 2.5) < 1e-15
    tz = t0 + 1.0 / (np.pi * f0 * np.sqrt(2.0))  # zero crossings of 1 - 2 a
    assert abs(dg.ricker(tz, f0, t0)) < 1e-15
    assert abs(dg.ricker(2 * t0 - 0.123, f0, t0) - dg.ricker(0.123, f0, t0)) < 1e-15


def test_point_location_and_receivers_exact_for_polynomials():
    m = inputs.layered_config(3, 3, 0.3, seed=2)
    mesh = _mesh(m)
    N = 3
    x = dg.node_coords(mesh, N)
    pts = np.array([[0.1, 0.2, 0.3], [0.77, 0.41, 0.93], [0.5, 0.12, 0.05]])
    el, rows = dg.make_receivers(mesh, N, pts)
    f = lambda X: 1 + X[..., 0] ** 2 * X[..., 1] - 2 * X[..., 2] ** 3 + X[..., 0] * X[..., 2]
    vals = np.einsum("rj,rj->r", rows, f(x[el]))
    np.testing.assert_allclose(vals, f(pts), atol=1e-12)


def test_source_vector_injects_unit_mass():
    """(1/kappa) 1^T M (kappa M^-1 l(xs)) = sum_i l_i(xs) = 1: the source adds
    s(t) to d/dt int p/kappa, as int delta = 1 requires."""
    m = inputs.layered_config(3, 3, 0.3, seed=2)
    mesh = _mesh(m)
    N = 2
    src = dg.make_point_source(mesh, N, [0.4, 0.6, 0.55], 10.0, 0.1)
    ops = dg.build_operators(mesh, N, elems=[src.elem])
    Np = ops.M.shape[1]
    assert abs(np.ones(Np) @ ops.M[0] @ src.vec / ops.kappa[0] - 1.0) < 1e-12


def test_energy_of_constant_state():
    m = inputs.layered_config(2, 2, 0.3, seed=1)
    mesh = _mesh(m)
    N = 2
    ops = dg.build_operators(mesh, N)
    Np = ops.M.shape[1]
    U = np.zeros((mesh.K, 4, Np))
    U[:, 0] = 1.0
    U[:, 3] = 2.0
    vol = np.einsum("i,kij,j->k", np.ones(Np), ops.M, np.ones(Np))
    kappa = m.rho * m.c ** 2
    expect = 0.5 * np.sum(vol / kappa + m.rho * vol * 4.0)
    assert abs(dg.energy(ops, U) - expect) < 1e-12 * expect
    assert abs(vol.sum() - 1.0) < 1e-12  # unit cube


def test_node_coordinates_flat_wedge_are_affine_images():
    X = inputs.random_vertical_wedges(1, seed=3)[0]
    X[:3, 2] = 0.0
    X[3:, 2] = 2.0
    mesh = dg.Mesh(X, np.arange(6)[None], np.ones(1), np.ones(1))
    N = 2
    from oracle import basis as B
    W = B.Wedge(N)
    x = dg.node_coords(mesh, N)[0]
    l1, l2, l3 = -(W.r + W.s) / 2, (1 + W.r) / 2, (1 + W.s) / 2
    xy = l1[:, None] * X[0, :2] + l2[:, None] * X[1, :2] + l3[:, None] * X[2, :2]
    np.testing.assert_allclose(x[:, :2], xy, atol=1e-15)
    np.testing.assert_allclose(x[:, 2], 1.0 + W.t, atol=1e-15)


def test_subset_rhs_equals_full_rhs():
    m = inputs.layered_config(3, 4, 0.3, seed=5)
    mesh = _mesh(m)
    N = 2
    full = dg.build_operators(mesh, N)
    sub = np.array([0, 5, 17, 40, 71])
    part = dg.build_operators(mesh, N, elems=sub)
    U = np.random.default_rng(0).standard_normal((mesh.K, 4, full.M.shape[1]))
    np.testing.assert_allclose(dg.rhs(part, U), dg.rhs(full, U)[sub], rtol=1e-13, atol=1e-13)
