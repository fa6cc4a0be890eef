"""Host-side tests of libwdg (no GPU): exported symbols, reference operators
against the oracle's independent construction, mesh validation error codes,
the state machine, node coordinates, point location and the time step."""
import os
import re

import numpy as np
import pytest

from oracle import basis as OB
from oracle import dg
from paper_1607_03399_amd import inputs
from paper_1607_03399_amd import wdg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.skipif(not os.path.exists(wdg.LIB_PATH), reason="libwdg.so not built")


def test_library_exports_every_declared_symbol():
    with open(os.path.join(ROOT, "include", "wdg.h")) as fh:
        text = fh.read()
    declared = set(re.findall(r"\b(wdg_[a-z_]+)\s*\(", text))
    assert len(declared) >= 20
    lib = wdg.load_library()
    for name in declared:
        assert hasattr(lib, name), name


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5])
def test_reference_operators_match_oracle(N):
    W = OB.Wedge(N)
    NT = W.Np_tri
    r = wdg.reference_operator(N, "r")
    s = wdg.reference_operator(N, "s")
    np.testing.assert_allclose(r, W.tri.r, atol=1e-14)
    np.testing.assert_allclose(s, W.tri.s, atol=1e-14)
    np.testing.assert_allclose(wdg.reference_operator(N, "t"), W.tgll, atol=1e-15)
    L, Lr, Ls = W.tri.eval(W.tri.r, W.tri.s)
    np.testing.assert_allclose(wdg.reference_operator(N, "Dr").reshape(NT, NT), Lr, atol=1e-11)
    np.testing.assert_allclose(wdg.reference_operator(N, "Ds").reshape(NT, NT), Ls, atol=1e-11)
    Dt = OB.lagrange1d_deriv(W.tgll, W.tgll)
    np.testing.assert_allclose(wdg.reference_operator(N, "Dt").reshape(N + 1, N + 1), Dt, atol=1e-12)
    rq, sq, wq = OB.tri_quadrature(N + 2)
    Lq, _, _ = W.tri.eval(rq, sq)
    Mtri = Lq.T @ (wq[:, None] * Lq)
    np.testing.assert_allclose(wdg.reference_operator(N, "Mtri").reshape(NT, NT), Mtri, atol=1e-13)
    lam = [-(rq + sq) / 2, (1 + rq) / 2, (1 + sq) / 2]
    for v in range(3):
        Mv = Lq.T @ ((wq * lam[v])[:, None] * Lq)
        np.testing.assert_allclose(wdg.reference_operator(N, f"Mv{v}").reshape(NT, NT), Mv, atol=1e-13)
    tg, wg = OB.gauss_nodes_weights(N + 2)
    l1 = OB.lagrange1d(W.tgll, tg)
    M1 = l1.T @ (wg[:, None] * l1)
    np.testing.assert_allclose(wdg.reference_operator(N, "M1").reshape(N + 1, N + 1), M1, atol=1e-14)
    e0 = np.zeros(N + 1)
    e0[0] = 1
    np.testing.assert_allclose(wdg.reference_operator(N, "g0"), np.linalg.solve(M1, e0), atol=1e-11)
    # edge lift pieces: (Mtri)^-1 int_edge l_i l_q (1 -+ xi)/2
    vref = np.array([[-1, -1], [1, -1], [-1, 1]], float)
    for e in range(3):
        a, b = vref[e], vref[(e + 1) % 3]
        pts = a[None] * (1 - tg[:, None]) / 2 + b[None] * (1 + tg[:, None]) / 2
        Le, _, _ = W.tri.eval(pts[:, 0], pts[:, 1])
        Ta = Le.T @ ((wg * (1 - tg) / 2)[:, None] * l1)
        Tb = Le.T @ ((wg * (1 + tg) / 2)[:, None] * l1)
        np.testing.assert_allclose(wdg.reference_operator(N, f"Ea{e}").reshape(NT, N + 1), np.linalg.solve(Mtri, Ta),
                                   atol=1e-11)
        np.testing.assert_allclose(wdg.reference_operator(N, f"Eb{e}").reshape(NT, N + 1), np.linalg.solve(Mtri, Tb),
                                   atol=1e-11)
        # edge node lists run from the first to the second vertex through the GLL points
        ids = wdg.reference_operator(N, f"edge{e}").astype(int)
        np.testing.assert_allclose(np.stack([r[ids], s[ids]], 1), pts_gll(a, b, W.tgll), atol=1e-14)


def pts_gll(a, b, t):
    return a[None] * (1 - t[:, None]) / 2 + b[None] * (1 + t[:, None]) / 2


def _host_solver(N=2):
    return wdg.Solver(N, 64, device=-1)


def test_node_coordinates_match_oracle():
    m = inputs.cfg1_mesh()
    for N in (1, 2, 3):
        s = _host_solver(N)
        s.set_mesh(m.verts, m.wedges)
        x = s.node_coords()
        xo = dg.node_coords(dg.Mesh(m.verts, m.wedges, m.c, m.rho), N)
        np.testing.assert_allclose(x, xo, atol=1e-14)
        s.close()


def test_stable_dt_matches_oracle_reading():
    m = inputs.layered_config(4, 5, 0.3, seed=3)
    for N in (1, 3):
        s = _host_solver(N)
        s.set_mesh(m.verts, m.wedges)
        s.set_material(m.c, m.rho)
        dt = s.stable_dt(0.5)
        ref = dg.stable_dt(dg.Mesh(m.verts, m.wedges, m.c, m.rho), N, 0.5)
        assert abs(dt - ref) < 1e-12 * ref
        s.close()


def _expect(code, fn, *a):
    with pytest.raises(wdg.WdgError) as ei:
        fn(*a)
    assert ei.value.name == code, str(ei.value)


def _one_wedge():
    v = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 0, 1], [0, 1, 1]], float)
    return v, np.arange(6)[None, :]


def test_validation_error_codes():
    v, w = _one_wedge()
    s = _host_solver()
    s.set_mesh(v, w)  # valid
    bad = v.copy()
    bad[3, 0] += 1e-3
    _expect("WDG_ERR_NOT_VERTICAL", s.set_mesh, bad, w)
    cw = w[:, [0, 2, 1, 3, 5, 4]]
    _expect("WDG_ERR_ORIENTATION", s.set_mesh, v, cw)
    inv = v.copy()
    inv[5, 2] = -0.5  # top vertex below its bottom partner
    _expect("WDG_ERR_JACOBIAN", s.set_mesh, inv, w)
    flat = v.copy()
    flat[3:, 2] = 0.0
    _expect("WDG_ERR_JACOBIAN", s.set_mesh, flat, w)
    degenerate = v.copy()
    degenerate[2, :2] = degenerate[5, :2] = [2.0, 0.0]
    _expect("WDG_ERR_JACOBIAN", s.set_mesh, degenerate, w)
    _expect("WDG_ERR_ARG", s.set_mesh, v, np.array([[0, 1, 2, 3, 4, 9]]))
    # a tetrahedron on the bottom triangle and one vertex of the top: its
    # triangles cut across the wedge's quadrilateral faces
    _expect("WDG_ERR_NONCONFORMING", s.set_mesh, v, w, np.array([[0, 1, 2, 3]]))
    vt = np.vstack([v, [[0.3, 0.3, -1.0]]])
    s.set_mesh(vt, w, np.array([[0, 2, 1, 6]]))  # tetrahedron below the wedge (valid)
    _expect("WDG_ERR_ORIENTATION", s.set_mesh, vt, w, np.array([[0, 1, 2, 6]]))
    _expect("WDG_ERR_ARG", s.set_mesh, vt, w, np.array([[0, 1, 2, 7]]))
    flat_t = np.vstack([v, [[0.3, 0.3, 0.0]]])
    _expect("WDG_ERR_JACOBIAN", s.set_mesh, flat_t, w, np.array([[0, 2, 1, 6]]))
    # three wedges on one triangle face
    v2 = np.vstack([v, v[3:] + [0, 0, 1], v[:3] - [0, 0, 1]])
    w3 = np.array([[0, 1, 2, 3, 4, 5], [3, 4, 5, 6, 7, 8], [9, 10, 11, 3, 4, 5]])
    _expect("WDG_ERR_NONCONFORMING", s.set_mesh, v2, w3)
    s.close()


def test_cfg3_literal_amplitude_inverts_a_layer():
    """0.05 sin sin interfaces with 24 layers (layer thickness 1/24) invert
    the first layer; the mesh is rejected."""
    L = 24

    def z(k, x, y):
        if k in (0, L):
            return np.full_like(x, k / L)
        return k / L + 0.05 * np.sin(2 * np.pi * x) * np.sin(2 * np.pi * y)

    v, w = inputs.layered_mesh(8, 8, L, z)
    s = _host_solver()
    _expect("WDG_ERR_JACOBIAN", s.set_mesh, v, w)
    s.close()


def test_state_machine_and_arguments():
    v, w = _one_wedge()
    s = _host_solver()
    _expect("WDG_ERR_STATE", s.set_material, 1.0, 1.0)
    _expect("WDG_ERR_STATE", s.num_nodes)
    s.set_mesh(v, w)
    assert s.num_nodes() == 18
    _expect("WDG_ERR_STATE", s.set_fields, np.zeros((1, 4, 18)))
    _expect("WDG_ERR_ARG", s.set_material, -1.0, 1.0)
    s.set_material(1.0, 1.0)
    _expect("WDG_ERR_STATE", s.set_fields, np.zeros((1, 4, 18)))  # host-only contexts hold no fields
    _expect("WDG_ERR_STATE", s.step, 1, 0.1)
    _expect("WDG_ERR_ARG", s.stable_dt, -1.0)
    _expect("WDG_ERR_OUTSIDE", s.add_ricker_source, [5.0, 5.0, 5.0], 10.0, 0.1)
    assert s.add_ricker_source([0.2, 0.2, 0.5], 10.0, 0.1) == 0
    _expect("WDG_ERR_OUTSIDE", s.set_receivers, [[0.9, 0.9, 0.5]])  # outside the triangle
    s.set_receivers([[0.1, 0.1, 0.1]])
    with pytest.raises(wdg.WdgError):
        wdg.Solver(7, 32, -1)
    with pytest.raises(wdg.WdgError):
        wdg.Solver(3, 16, -1)
    s.close()


def test_no_device_is_an_error_not_a_fallback():
    """A device context on a machine without a GPU fails at set_mesh with
    WDG_ERR_HIP; there is no CPU path."""
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    v, w = _one_wedge()
    s = wdg.Solver(2, 64, 0)
    _expect("WDG_ERR_HIP", s.set_mesh, v, w)
    s.close()


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5])
def test_tet_reference_operators_match_oracle(N):
    """Tetrahedron nodes, derivative, mass and lift matrices of the library's
    own construction against the oracle's (nodes: same Warp & Blend reading;
    operators: the oracle's Vandermonde derivatives and quadrature)."""
    T = OB.Tet(N)
    Np, NT = T.Np, (N + 1) * (N + 2) // 2
    for name, ref in (("tet_r", T.r), ("tet_s", T.s), ("tet_t", T.t)):
        np.testing.assert_allclose(wdg.reference_operator(N, name), ref, atol=1e-13)
    _, G = T.eval(T.r, T.s, T.t)
    for d, name in enumerate(("tet_Dr", "tet_Ds", "tet_Dt")):
        np.testing.assert_allclose(wdg.reference_operator(N, name).reshape(Np, Np), G[..., d], atol=1e-10)
    r, s, t, w = OB.tet_quadrature(N + 2)
    Bq, _ = T.eval(r, s, t)
    M = np.einsum("q,qi,qj->ij", w, Bq, Bq)
    np.testing.assert_allclose(wdg.reference_operator(N, "tet_M").reshape(Np, Np), M, atol=1e-12)
    tri = OB.Triangle(N)
    E = np.zeros((Np, 4 * NT))
    for f, (xi, wf, _, _) in enumerate(T.face_rules()):
        Bf, _ = T.eval(xi[:, 0], xi[:, 1], xi[:, 2])
        ra, sa, _ = OB.tri_quadrature(N + 2)
        Lt, _, _ = tri.eval(ra, sa)
        E[:, f * NT:(f + 1) * NT] = np.einsum("q,qi,qm->im", wf, Bf, Lt)
    LIFT = np.linalg.solve(M, E)
    np.testing.assert_allclose(wdg.reference_operator(N, "tet_LIFT").reshape(Np, 4 * NT), LIFT, atol=1e-10)
    # face node lists: the triangle nodes mapped through the face's vertices, in order
    tr, ts = OB.tri_nodes(N)
    lam = np.stack([-(tr + ts) / 2, (1 + tr) / 2, (1 + ts) / 2], 1)
    X = np.stack([T.r, T.s, T.t], 1)
    for f, fv in enumerate(T.face_verts):
        ids = wdg.reference_operator(N, f"tet_face{f}").astype(int)
        P = lam @ T.ref_verts[list(fv)]
        np.testing.assert_allclose(X[ids], P, atol=1e-13)


def _hybrid_mesh(nx=3, layers=4, tet_layers=2, seed=1):
    m = inputs.layered_config(nx, layers, 0.3, seed=seed)
    return inputs.split_layers(m, tet_layers)


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_hybrid_node_coordinates_and_dt_match_oracle(N):
    v, w, t, c, rho = _hybrid_mesh()
    s = _host_solver(N)
    s.set_mesh(v, w, t)
    assert s.num_nodes() == len(w) * s.Np + len(t) * s.Npt
    om = dg.Mesh(v, w, c, rho, tets=t)
    np.testing.assert_allclose(s.node_coords(), dg.node_coords(om, N), atol=1e-14)
    s.set_material(c, rho)
    dt = s.stable_dt(0.5)
    ref = dg.stable_dt(om, N, 0.5)
    assert abs(dt - ref) < 1e-12 * ref
    s.close()


def test_tetrahedra_only_mesh_is_accepted():
    v, w, t, c, rho = _hybrid_mesh(nx=2, layers=2, tet_layers=2)
    assert len(w) == 0
    s = _host_solver(2)
    s.set_mesh(v, w, t)
    om = dg.Mesh(v, w, c, rho, tets=t)
    np.testing.assert_allclose(s.node_coords(), dg.node_coords(om, 2)[:, :s.Npt], atol=1e-14)
    s.close()


def test_column_split_mesh_host_side():
    """Columns split into tetrahedra: wedge quadrilaterals against two
    tetrahedron triangles are accepted (coupled on the common refinement);
    node coordinates and time step as the oracle's."""
    m = inputs.layered_config(3, 3, 0.3, seed=1)
    v, w, t, c, rho = inputs.split_columns(m, [4, 9])
    s = _host_solver(2)
    s.set_mesh(v, w, t)
    om = dg.Mesh(v, w, c, rho, tets=t)
    np.testing.assert_allclose(s.node_coords(), dg.node_coords(om, 2), atol=1e-14)
    s.set_material(c, rho)
    assert abs(s.stable_dt(0.5) - dg.stable_dt(om, 2, 0.5)) < 1e-12 * s.stable_dt(0.5)
    # one triangle of a split quadrilateral missing: not conforming
    _expect("WDG_ERR_NONCONFORMING", s.set_mesh, v, w, t[1:])
    s.close()


def test_adjoint_gradient_argument_checks():
    """Order and argument checks of wdg_adjoint_gradient (no device work)."""
    m = inputs.layered_config(2, 2, 0.3, seed=4)
    s = wdg.Solver(2, 64, device=-1)
    s.set_mesh(m.verts, m.wedges)
    s.set_material(m.c, m.rho)
    s.set_receivers([[0.5, 0.5, 0.5]])
    with pytest.raises(wdg.WdgError) as e:  # a host-only context holds no fields
        s.adjoint_gradient(3, 1e-3, np.zeros((3, 1)))
    assert e.value.name == "WDG_ERR_STATE"
    with pytest.raises(ValueError):
        s.adjoint_gradient(3, 1e-3, np.zeros((2, 1)))
    s.close()


def test_wedge_block_arguments():
    """Elements per block of the node-lane kernel: only the compiled shapes of
    the context's order and precision (none below order 4 or in FP64)."""
    for N, bits, shapes in ((4, 32, (8, 17, 12, 4)), (5, 32, (12, 9, 6, 3))):
        s = wdg.Solver(N, bits, device=-1)
        for e in shapes:
            s.set_wedge_block(e)
        s.set_wedge_block(0)
        for e in (1, 5, 9 if N == 4 else 8, 64, -1):
            _expect("WDG_ERR_ARG", s.set_wedge_block, e)
        s.close()
    for N, bits in ((3, 32), (4, 64)):
        s = wdg.Solver(N, bits, device=-1)
        s.set_wedge_block(0)
        _expect("WDG_ERR_ARG", s.set_wedge_block, 8)
        s.close()
