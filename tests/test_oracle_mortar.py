"""Pins of the oracle's nonconforming wedge/tetrahedron faces.

When whole columns of prisms are split into tetrahedra, a wedge next to a
split column faces two triangular tetrahedron faces with one
quadrilateral.  The oracle integrates the flux on the common refinement (the
two triangles), in the wedge face's (edge, vertical) coordinates: Gauss in
the vertical on each side of the diagonal (exact) times a converged Gauss
rule along the edge.  Checked: the rule's convergence, exactness on global
polynomials (no spurious jumps), the semi-discrete energy identity with the
mortar jumps, stable spectra, conservation and convergence rates.
"""
import numpy as np
import pytest

from oracle import basis as B
from oracle import dg, lsrk
from oracle import geometry as G
from paper_1607_03399_amd import inputs


def _split(nx=3, layers=3, cols=(4, 9), seed=1, bc="rigid", flux="upwind"):
    m = inputs.layered_config(nx, layers, 0.3, seed=seed)
    v, w, t, c, rho = inputs.split_columns(m, list(cols))
    return dg.Mesh(v, w, c, rho, bc, flux, tets=t)


def test_column_split_structure():
    m = inputs.layered_config(3, 3, 0.3, seed=1)
    mesh = _split()
    assert mesh.nw == m.K - 2 * 3 and mesh.nt == 2 * 3 * 3
    nbr, _ = dg.face_connectivity(mesh)
    mortars = dg.mortar_faces(mesh, nbr)
    # two interior columns, three lateral faces each, three layers
    assert len(mortars) == 18
    assert (nbr == -3).sum() == 18 * 3
    for (k, f, diag, ((t0, f0), (t1, f1))) in mortars:
        assert k < mesh.nw and f >= 2 and t0 >= mesh.nw and t1 >= mesh.nw
        quad = set(mesh.wedges[k][list(B.Wedge.face_verts[f])])
        tri0 = set(mesh.tets[t0 - mesh.nw][list(B.Tet.face_verts[f0])])
        tri1 = set(mesh.tets[t1 - mesh.nw][list(B.Tet.face_verts[f1])])
        assert tri0 | tri1 == quad and len(tri0 & tri1) == 2


def test_mortar_rule_converged_and_area():
    """The mortar points cover each quadrilateral exactly once: the weights of
    its two regions add up to the face area (two planar triangles); and 24
    points along the edge agree with 48 to rounding for a rational integrand
    with the worst height ratio of the test meshes."""
    mesh = _split()
    ops = dg.build_operators(mesh, 2)
    regs = ops.extra["mortars"]
    nbr, _ = dg.face_connectivity(mesh)
    mortars = dg.mortar_faces(mesh, nbr)
    assert len(regs) == 2 * len(mortars)
    for (k, f, diag, tets) in mortars:
        X = mesh.verts[mesh.wedges[k][list(B.Wedge.face_verts[f])]]
        area = 0.5 * np.linalg.norm(np.cross(X[1] - X[0], X[2] - X[0])) + \
            0.5 * np.linalg.norm(np.cross(X[2] - X[0], X[3] - X[0]))
        w = sum(r["wJ"].sum() for r in regs if r["k"] == k and r["f"] == f)
        assert abs(w - area) < 1e-13 * area
    xg, wg = B.gauss_nodes_weights(24)
    xh, wh = B.gauss_nodes_weights(48)
    h = lambda x: 1.0 + 0.6 * x  # vertical edge lengths 0.4 and 1.6: poles at x = -5/3
    f = lambda x: (1 + x) ** 5 / h(x) ** 7
    assert abs(np.dot(wg, f(xg)) - np.dot(wh, f(xh))) < 1e-13 * abs(np.dot(wh, f(xh)))


@pytest.mark.parametrize("N", [1, 2, 3])
def test_global_polynomials_have_no_jumps(N):
    """p and u of degree <= N in x, y, z are represented exactly on both kinds
    of element, so every flux vanishes and the right-hand side is the exact
    -kappa div u, -grad p / rho, also next to the split columns."""
    mesh = _split(flux="upwind")
    mesh.c[:] = 1.5
    mesh.rho[:] = 2.0
    ops = dg.build_operators(mesh, N)
    x = dg.node_coords(mesh, N)
    mask = dg.node_mask(mesh, N)
    X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
    U = np.zeros((mesh.K, 4, x.shape[1]))
    U[:, 0] = X ** N + Y * Z ** (N - 1) - 0.5 * Z
    U[:, 1] = Y ** N - X
    U[:, 2] = Z ** N + X * Y * (N > 1)
    U[:, 3] = X ** (N - 1) * Y + Z
    U *= mask[:, None, :]
    kap, rho = 1.5 ** 2 * 2.0, 2.0
    # d/dx (Y^N - X) = -1; d/dy (Z^N + XY) = X (N > 1); d/dz (X^(N-1) Y + Z) = 1
    div = -1.0 + X * (N > 1) + 1.0
    gp = [N * X ** (N - 1), Z ** (N - 1), (N - 1) * Y * Z ** max(N - 2, 0) - 0.5]
    R = dg.rhs(ops, U)
    # the rigid-wall mirror state is not a polynomial continuation: check elements off the walls
    nbr = ops.nbr
    inner = np.all((nbr >= 0) | (nbr == -2) | (nbr == -3), axis=1)
    assert inner.sum() > 0
    np.testing.assert_allclose(R[inner, 0][mask[inner]], (-kap * div)[inner][mask[inner]], atol=1e-9)
    for d in range(3):
        np.testing.assert_allclose(R[inner, d + 1][mask[inner]], (-gp[d] / rho)[inner][mask[inner]], atol=1e-9)


@pytest.mark.parametrize("bc", ["rigid", "dirichlet"])
@pytest.mark.parametrize("flux", ["upwind", "central"])
def test_mortar_energy_identity(bc, flux):
    mesh = _split(bc=bc, flux=flux)
    N = 2
    ops = dg.build_operators(mesh, N)
    mask = dg.node_mask(mesh, N)
    U = np.random.default_rng(0).standard_normal((mesh.K, 4, mask.shape[1])) * mask[:, None, :]
    R = dg.rhs(ops, U)
    lhs = dg.energy_rate(ops, U, R)
    jumps = dg.energy_rate_from_jumps(ops, U)
    scale = dg.energy(ops, U)
    if flux == "central":
        assert abs(lhs) < 1e-12 * scale
    else:
        assert jumps < 0 and abs(lhs - jumps) < 1e-12 * scale


def test_mortar_spectrum_stable_and_conservative():
    m = inputs.layered_config(2, 2, 0.3, seed=3)
    v, w, t, c, rho = inputs.split_columns(m, [2])
    for flux in ("upwind", "central"):
        mesh = dg.Mesh(v, w, c, rho, "dirichlet", flux, tets=t)
        N = 2
        ops = dg.build_operators(mesh, N)
        mask = dg.node_mask(mesh, N)
        idx = np.nonzero(np.broadcast_to(mask[:, None, :], (mesh.K, 4, mask.shape[1])).ravel())[0]
        E = np.zeros((len(idx), mesh.K * 4 * mask.shape[1]))
        E[np.arange(len(idx)), idx] = 1.0
        A = dg.rhs(ops, E.reshape(len(idx), mesh.K, 4, -1)).reshape(len(idx), -1)[:, idx].T
        lam = np.linalg.eigvals(A)
        rA = np.abs(lam).max()
        assert lam.real.max() <= 1e-10 * rA
        if flux == "central":
            assert np.abs(lam.real).max() <= 1e-10 * rA
    mesh = _split(bc="rigid")
    ops = dg.build_operators(mesh, 2)
    mask = dg.node_mask(mesh, 2)
    U = np.random.default_rng(2).standard_normal((mesh.K, 4, mask.shape[1])) * mask[:, None, :]
    inv = lambda U: float(np.sum(np.einsum("ki,kij,kj->k", mask.astype(float), ops.M, U[:, 0]) / ops.kappa))
    I0 = inv(U)
    res = np.zeros_like(U)
    dt = dg.stable_dt(mesh, 2, 0.5)
    for s in range(5):
        res = lsrk.A[s] * res + dt * dg.rhs(ops, U)
        U = U + lsrk.B[s] * res
    assert abs(inv(U) - I0) < 1e-12 * max(1.0, abs(I0))


def test_mortar_convergence():
    """Standing mode (Dirichlet) on [-1,1]^3 with a quarter of the columns
    split into tetrahedra: rate >= N + 1/2 (N = 2)."""
    N = 2
    errs = []
    for n in (2, 4):
        m = inputs.cube_mesh(n, z_jitter=0.2, seed=n)
        cols = np.random.default_rng(n).choice(2 * n * n, max(1, n * n // 2), replace=False)
        v, w, t, c, rho = inputs.split_columns(m, cols)
        mesh = dg.Mesh(v, w, c, rho, "dirichlet", "upwind", tets=t)
        ops = dg.build_operators(mesh, N)
        x = dg.node_coords(mesh, N)
        mask = dg.node_mask(mesh, N)
        U0 = inputs.standing_mode_dirichlet(x, 0.0) * mask[:, None, :]
        T = 0.4
        dt = dg.stable_dt(mesh, N, 0.5)
        ns = int(np.ceil(T / dt))
        U, _ = lsrk.integrate(lambda t_, U: dg.rhs(ops, U), U0, T / ns, ns)
        err = 0.0
        for kind, ref in enumerate(dg.references(N, mesh)):
            ids = np.nonzero(mesh.kinds() == kind)[0]
            R, S, Tq, W = ref.volume_quadrature()
            Bv, _ = ref.eval(R, S, Tq)
            Xv = dg._vertices(mesh, kind, ids)
            xq, Jm = G.map_points(ref.kind, Xv, np.stack([R, S, Tq], 1))
            ex = inputs.standing_mode_dirichlet(xq, T)[:, 0, :]
            ph = np.einsum("qj,kj->kq", Bv, U[ids, 0, :ref.Np])
            err += np.sum(W * np.linalg.det(Jm) * (ph - ex) ** 2)
        errs.append(np.sqrt(err))
    assert np.log2(errs[0] / errs[1]) >= N + 0.5
