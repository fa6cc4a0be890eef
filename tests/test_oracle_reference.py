"""Pins of the oracle's reference elements against textbook facts.

Everything here is checked against closed forms, published values or
structural facts that a transcription mistake (wrong node, wrong weight,
transposed derivative) would break.
"""
import math

import numpy as np
import pytest

from oracle import basis as B


# Published GLL rules (Abramowitz & Stegun 25.4.32): nodes, weights
GLL_TABLE = {
    1: ([-1.0, 1.0], [1.0, 1.0]),
    2: ([-1.0, 0.0, 1.0], [1 / 3, 4 / 3, 1 / 3]),
    3: ([-1.0, -1 / math.sqrt(5), 1 / math.sqrt(5), 1.0], [1 / 6, 5 / 6, 5 / 6, 1 / 6]),
    4: ([-1.0, -math.sqrt(3 / 7), 0.0, math.sqrt(3 / 7), 1.0], [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10]),
}


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_gll_matches_published_rules(N):
    x, w = B.gll_nodes_weights(N)
    xr, wr = GLL_TABLE[N]
    np.testing.assert_allclose(x, xr, atol=1e-15)
    np.testing.assert_allclose(w, wr, atol=1e-15)


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5])
def test_gll_exact_to_degree_2N_minus_1(N):
    x, w = B.gll_nodes_weights(N)
    assert abs(w.sum() - 2.0) < 1e-14
    for k in range(2 * N):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.sum(w * x ** k) - exact) < 1e-14
    # degree 2N is NOT integrated exactly (this is the aliasing of mass lumping)
    assert abs(np.sum(w * x ** (2 * N)) - 2.0 / (2 * N + 1)) > 1e-3


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5])
def test_1d_derivative_exact(N):
    x, _ = B.gll_nodes_weights(N)
    D = B.lagrange1d_deriv(x, x)
    for k in range(N + 1):
        np.testing.assert_allclose(D @ x ** k, k * x ** max(k - 1, 0) if k else 0 * x, atol=1e-12)


def _tri_monomial_integral(a, b):
    """int over the bi-unit triangle of (1+r)^a (1+s)^b = 2^(a+b+2) a! b! / (a+b+2)!."""
    return 2.0 ** (a + b + 2) * math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6, 7])
def test_duffy_rule_exactness(n):
    r, s, w = B.tri_quadrature(n)
    deg = 2 * n - 2
    for a in range(deg + 1):
        for b in range(deg + 1 - a):
            q = np.sum(w * (1 + r) ** a * (1 + s) ** b)
            assert abs(q - _tri_monomial_integral(a, b)) < 1e-13 * max(1, _tri_monomial_integral(a, b))


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5])
def test_triangle_nodes_structure(N):
    r, s = B.tri_nodes(N)
    assert len(r) == (N + 1) * (N + 2) // 2
    xg, _ = B.gll_nodes_weights(N)
    # vertices are nodes
    for v in [(-1, -1), (1, -1), (-1, 1)]:
        assert np.min(np.hypot(r - v[0], s - v[1])) < 1e-15
    # every edge carries exactly the N+1 GLL points (alpha = 0 warp & blend)
    e1 = np.sort(r[np.abs(s + 1) < 1e-13])
    e3 = np.sort(s[np.abs(r + 1) < 1e-13])
    e2 = np.sort(r[np.abs(r + s) < 1e-13])
    for e in (e1, e2, e3):
        np.testing.assert_allclose(e, xg, atol=1e-15)
    # invariance of the node set under the vertex rotation V1->V2->V3->V1 and
    # under the reflection r <-> s
    l1, l2, l3 = -(r + s) / 2, (1 + r) / 2, (1 + s) / 2
    rr, ss = 2 * l1 - 1, 2 * l2 - 1  # rotated barycentric roles
    for (a, b) in ((rr, ss), (s, r)):
        d = np.hypot(a[:, None] - r[None, :], b[:, None] - s[None, :]).min(axis=1)
        assert d.max() < 1e-14
    # all nodes inside
    assert np.all(r >= -1 - 1e-15) and np.all(s >= -1 - 1e-15) and np.all(r + s <= 1e-15)


def test_triangle_nodes_low_order_closed_forms():
    # N <= 2: GLL = equispaced, so the warp vanishes: lattice points
    r, s = B.tri_nodes(2)
    lattice = {(-1, -1), (0, -1), (1, -1), (-1, 0), (0, 0), (-1, 1)}
    got = {(round(a, 14), round(b, 14)) for a, b in zip(r, s)}
    assert got == {(float(a), float(b)) for a, b in lattice}
    # N = 3: the single interior node is the centroid by symmetry
    r, s = B.tri_nodes(3)
    interior = (r > -1 + 1e-12) & (s > -1 + 1e-12) & (r + s < -1e-12)
    assert interior.sum() == 1
    np.testing.assert_allclose([r[interior][0], s[interior][0]], [-1 / 3, -1 / 3], atol=1e-15)


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5])
def test_triangle_lagrange_basis(N):
    T = B.Triangle(N)
    L, Lr, Ls = T.eval(T.r, T.s)
    np.testing.assert_allclose(L, np.eye(T.Np), atol=1e-12)
    # nodal derivative matrices differentiate P^N exactly
    for a in range(N + 1):
        for b in range(N + 1 - a):
            f = T.r ** a * T.s ** b
            fr = a * T.r ** max(a - 1, 0) * T.s ** b
            fs = b * T.r ** a * T.s ** max(b - 1, 0)
            np.testing.assert_allclose(Lr @ f, fr, atol=1e-11)
            np.testing.assert_allclose(Ls @ f, fs, atol=1e-11)
    # mass matrix: integrates interpolants exactly
    rq, sq, wq = B.tri_quadrature(N + 2)
    Lq, _, _ = T.eval(rq, sq)
    Mh = Lq.T @ (wq[:, None] * Lq)
    assert abs(np.ones(T.Np) @ Mh @ np.ones(T.Np) - 2.0) < 1e-13
    f = (1 + T.r) ** N
    assert abs(np.ones(T.Np) @ Mh @ f - _tri_monomial_integral(N, 0)) < 1e-12


@pytest.mark.parametrize("N", [1, 2, 3])
def test_wedge_basis_tensor_product(N):
    W = B.Wedge(N)
    v, g = W.eval(W.r, W.s, W.t)
    np.testing.assert_allclose(v, np.eye(W.Np), atol=1e-12)
    assert W.Np == (N + 1) ** 2 * (N + 2) // 2
    # gradient of x^a y^b z^c on the reference wedge (identity map)
    rng = np.random.default_rng(0)
    pts = rng.uniform(-1, 0, (7, 2))
    tp = rng.uniform(-1, 1, 7)
    vq, gq = W.eval(pts[:, 0], pts[:, 1], tp)
    f = W.r ** (N - 1) * W.s + W.t ** N
    np.testing.assert_allclose(vq @ f, pts[:, 0] ** (N - 1) * pts[:, 1] + tp ** N, atol=1e-12)
    np.testing.assert_allclose(gq[..., 2] @ f, N * tp ** (N - 1), atol=1e-11)
    np.testing.assert_allclose(gq[..., 1] @ f, pts[:, 0] ** (N - 1), atol=1e-11)
