"""Pins of the oracle's tetrahedra and of mixed wedge/tetrahedron meshes.

Tetrahedra join wedges through triangular faces (Sec. 3.1: the wedge's
triangle nodes are the tetrahedron's face nodes).  Checked here: Warp & Blend
tetrahedron nodes (faces equal the triangle nodes, edges GLL, symmetry),
collapsed quadrature against closed forms, exact derivatives on affine
tetrahedra, and on hybrid meshes the energy identity, stable spectra,
conservation and convergence.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import basis as B
from oracle import dg, lsrk
from oracle import geometry as G
from paper_1607_03399_amd import inputs


def _bary(r, s, t):
    return np.stack([-(1 + r + s + t) / 2, (1 + r) / 2, (1 + s) / 2, (1 + t) / 2], 1)


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5])
def test_tet_nodes_structure(N):
    r, s, t = B.tet_nodes(N)
    assert len(r) == (N + 1) * (N + 2) * (N + 3) // 6
    lam = _bary(r, s, t)
    assert lam.min() > -1e-14
    tri_r, tri_s = B.tri_nodes(N)
    tri_lam = np.stack([-(tri_r + tri_s) / 2, (1 + tri_r) / 2, (1 + tri_s) / 2], 1)
    gll, _ = B.gll_nodes_weights(N)
    for face in itertools.combinations(range(4), 3):
        opp = ({0, 1, 2, 3} - set(face)).pop()
        on = lam[:, opp] < 1e-12
        assert on.sum() == (N + 1) * (N + 2) // 2
        fl = lam[on][:, list(face)]
        # same point set as the triangle nodes, in the face's barycentrics
        d = np.abs(fl[:, None, :] - tri_lam[None, :, :]).max(axis=2).min(axis=1)
        assert d.max() < 1e-14
    for a, b in itertools.combinations(range(4), 2):
        others = [v for v in range(4) if v not in (a, b)]
        on = (lam[:, others] < 1e-12).all(axis=1)
        x = np.sort(lam[on, b] - lam[on, a])
        np.testing.assert_allclose(x, gll, atol=1e-14)
    # invariance under every relabelling of the vertices
    for perm in itertools.permutations(range(4)):
        lp = lam[:, list(perm)]
        d = np.abs(lp[:, None, :] - lam[None, :, :]).max(axis=2).min(axis=1)
        assert d.max() < 1e-13


def test_tet_nodes_low_order_lattice():
    r, s, t = B.tet_nodes(2)
    lam = _bary(r, s, t)
    assert np.allclose(lam * 2, np.round(lam * 2), atol=1e-14)


def _tet_monomial(a, b, c):
    """int over the bi-unit tet of (1+r)^a (1+s)^b (1+t)^c."""
    return 2.0 ** (a + b + c + 3) * math.factorial(a) * math.factorial(b) * math.factorial(c) / math.factorial(a + b + c + 3)


@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_tet_quadrature_exactness(n):
    r, s, t, w = B.tet_quadrature(n)
    deg = 2 * n - 3
    for a in range(deg + 1):
        for b in range(deg + 1 - a):
            for c in range(deg + 1 - a - b):
                q = np.sum(w * (1 + r) ** a * (1 + s) ** b * (1 + t) ** c)
                assert abs(q - _tet_monomial(a, b, c)) < 1e-13 * max(1.0, _tet_monomial(a, b, c))


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_tet_basis_and_derivatives(N):
    T = B.Tet(N)
    v, g = T.eval(T.r, T.s, T.t)
    np.testing.assert_allclose(v, np.eye(T.Np), atol=1e-11)
    f = T.r ** (N - 1) * T.t + T.s ** N - 2 * T.r * T.s * (N > 1)
    fr = (N - 1) * T.r ** max(N - 2, 0) * T.t - 2 * T.s * (N > 1)
    ft = T.r ** (N - 1)
    np.testing.assert_allclose(g[..., 0] @ f, fr, atol=1e-10)
    np.testing.assert_allclose(g[..., 2] @ f, ft, atol=1e-10)


def _hybrid(nx=3, layers=4, tet_layers=2, seed=1, bc="rigid", flux="upwind"):
    m = inputs.layered_config(nx, layers, 0.3, seed=seed)
    v, w, t, c, rho = inputs.split_layers(m, tet_layers)
    return dg.Mesh(v, w, c, rho, bc, flux, tets=t)


def test_split_prisms_are_conforming_and_fill_the_prism():
    m = inputs.layered_config(3, 2, 0.3, seed=2)
    v, w, t, c, rho = inputs.split_layers(m, 2)
    assert len(w) == 0 and len(t) == 3 * m.K
    # volumes add up to the prism volumes
    X = v[t]
    vol = np.einsum("kd,kd->k", np.cross(X[:, 1] - X[:, 0], X[:, 2] - X[:, 0]), X[:, 3] - X[:, 0]) / 6
    assert np.all(vol > 0)
    P = v[m.wedges]
    e1, e2 = P[:, 1, :2] - P[:, 0, :2], P[:, 2, :2] - P[:, 0, :2]
    area = 0.5 * np.abs(e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0])
    pvol = area * (P[:, 3:, 2] - P[:, :3, 2]).mean(axis=1)
    assert abs(vol.sum() - pvol.sum()) < 1e-12
    # every interior face is shared by exactly two elements
    mesh = dg.Mesh(v, w, c, rho, tets=t)
    nbr, _ = dg.face_connectivity(mesh)
    assert (nbr[:, :4] == -1).sum() == 2 * 18 + 4 * 3 * 2 * 2  # top/bottom triangles + split side quads


@pytest.mark.parametrize("N", [1, 2, 3])
def test_tet_derivative_exact_on_affine_elements(N):
    mesh = _hybrid()
    ops = dg.build_operators(mesh, N)
    x = dg.node_coords(mesh, N)
    mask = dg.node_mask(mesh, N)
    X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
    f = X ** N + Y ** (N - 1) * Z - 0.5 * Z ** N
    fx = N * X ** (N - 1)
    fy = (N - 1) * Y ** max(N - 2, 0) * Z if N > 1 else 0 * X
    fz = Y ** (N - 1) - 0.5 * N * Z ** (N - 1)
    for d, ref in enumerate((fx, fy, fz)):
        D = np.einsum("kij,kjl,kl->ki", ops.Minv, ops.S[d], f * mask)
        np.testing.assert_allclose(D[mask], ref[mask], atol=1e-10)


@pytest.mark.parametrize("bc", ["rigid", "dirichlet"])
@pytest.mark.parametrize("flux", ["upwind", "central"])
def test_hybrid_energy_identity(bc, flux):
    mesh = _hybrid(bc=bc, flux=flux)
    N = 2
    ops = dg.build_operators(mesh, N)
    mask = dg.node_mask(mesh, N)
    U = np.random.default_rng(0).standard_normal((mesh.K, 4, mask.shape[1])) * mask[:, None, :]
    R = dg.rhs(ops, U)
    # padding entries of tetrahedra stay exactly zero
    assert np.abs(R * ~mask[:, None, :]).max() == 0.0
    lhs = dg.energy_rate(ops, U, R)
    rhs_ = dg.energy_rate_from_jumps(ops, U)
    scale = dg.energy(ops, U)
    if flux == "central":
        assert abs(lhs) < 1e-12 * scale
    else:
        assert abs(lhs - rhs_) < 1e-12 * scale and rhs_ < 0


def test_hybrid_spectrum_stable_and_conservative():
    mesh = _hybrid(nx=2, layers=2, tet_layers=1, bc="dirichlet")
    N = 2
    ops = dg.build_operators(mesh, N)
    mask = dg.node_mask(mesh, N)
    idx = np.nonzero(np.broadcast_to(mask[:, None, :], (mesh.K, 4, mask.shape[1])).ravel())[0]
    n = len(idx)
    E = np.zeros((n, mesh.K * 4 * mask.shape[1]))
    E[np.arange(n), idx] = 1.0
    A = dg.rhs(ops, E.reshape(n, mesh.K, 4, -1)).reshape(n, -1)[:, idx].T
    lam = np.linalg.eigvals(A)
    assert lam.real.max() <= 1e-10 * np.abs(lam).max()
    # rigid walls: pressure integral conserved
    mesh = _hybrid(bc="rigid")
    ops = dg.build_operators(mesh, N)
    mask = dg.node_mask(mesh, N)
    U = np.random.default_rng(1).standard_normal((mesh.K, 4, mask.shape[1])) * mask[:, None, :]
    one = mask.astype(float)

    def inv(U):
        return float(np.sum(np.einsum("ki,kij,kj->k", one, ops.M, U[:, 0]) / ops.kappa))

    I0 = inv(U)
    res = np.zeros_like(U)
    dt = dg.stable_dt(mesh, N, 0.5)
    for s in range(5):
        res = lsrk.A[s] * res + dt * dg.rhs(ops, U)
        U = U + lsrk.B[s] * res
    assert abs(inv(U) - I0) < 1e-12 * max(1.0, abs(I0))


def test_hybrid_convergence():
    """Standing mode (Dirichlet) on [-1,1]^3 with the lower half split into
    tetrahedra: rate >= N + 1/2 (N = 2)."""
    N = 2
    errs = []
    for n in (2, 4):
        m = inputs.cube_mesh(n, z_jitter=0.2, seed=n)
        v, w, t, c, rho = inputs.split_layers(m, n // 2)
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
    rate = np.log2(errs[0] / errs[1])
    assert rate >= N + 0.5
