"""Reference elements for the oracle (FP64, NumPy).

Reference domains (bi-unit everywhere, the reading taken for the mixed
[0,1] / [-1,1] notation of Sec. 3):

* interval  t in [-1, 1]
* triangle  T = {(r, s): r >= -1, s >= -1, r + s <= 0}, vertices
  V1 = (-1,-1), V2 = (1,-1), V3 = (-1,1)
* wedge     T x [-1, 1]

Nodal sets (Sec. 3.1): triangle nodes are the Warp & Blend points of
Warburton (2006) with the blending parameter alpha = 0; vertical nodes are
the N+1 Gauss-Legendre-Lobatto points; wedge nodes are their tensor
product, node n = j * Np_tri + i for triangle node i and GLL node j.

Lagrange bases are obtained by inverting a Vandermonde matrix of a plain
polynomial basis of the right space: products of Legendre polynomials
P_a(r) P_b(s), a + b <= N, span P^N on the triangle (Sec. 3, definition of
P^N(T)); P_a(t), a <= N, spans P^N on the interval.
"""
from __future__ import annotations

import math

import numpy as np
from numpy.polynomial import legendre as npleg

# ---------------------------------------------------------------------------
# 1D
# ---------------------------------------------------------------------------


def gll_nodes_weights(N: int):
    """Gauss-Legendre-Lobatto nodes and weights on [-1, 1] (N+1 points).

    Interior nodes are the roots of P_N'; the weights are 2 / (N(N+1) P_N(x)^2).
    """
    if N < 1:
        raise ValueError("GLL needs N >= 1")
    cN = np.zeros(N + 1)
    cN[N] = 1.0
    interior = np.sort(np.real(npleg.legroots(npleg.legder(cN)))) if N > 1 else np.zeros(0)
    x = np.concatenate([[-1.0], interior, [1.0]])
    # polish interior roots with Newton on P_N'
    if N > 1:
        d1 = npleg.legder(cN)
        d2 = npleg.legder(cN, 2)
        for _ in range(4):
            xi = x[1:-1]
            x[1:-1] = xi - npleg.legval(xi, d1) / npleg.legval(xi, d2)
    PN = npleg.legval(x, cN)
    w = 2.0 / (N * (N + 1) * PN ** 2)
    return x, w


def gauss_nodes_weights(n: int):
    """n-point Gauss-Legendre rule on [-1, 1] (exact to degree 2n-1)."""
    return npleg.leggauss(n)


def lagrange1d(nodes: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Values l_j(x_q) of the Lagrange polynomials on ``nodes``; shape (len(x), len(nodes))."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    out = np.ones((len(x), n))
    for j in range(n):
        for m in range(n):
            if m != j:
                out[:, j] *= (x - nodes[m]) / (nodes[j] - nodes[m])
    return out


def lagrange1d_deriv(nodes: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Derivatives l_j'(x_q) by the product rule; shape (len(x), len(nodes))."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    out = np.zeros((len(x), n))
    for j in range(n):
        for k in range(n):
            if k == j:
                continue
            term = np.full(len(x), 1.0 / (nodes[j] - nodes[k]))
            for m in range(n):
                if m != j and m != k:
                    term *= (x - nodes[m]) / (nodes[j] - nodes[m])
            out[:, j] += term
    return out


# ---------------------------------------------------------------------------
# Triangle
# ---------------------------------------------------------------------------

# equilateral triangle used by the Warp & Blend construction (side 2)
_EQ_VERTS = np.array([[-1.0, -1.0 / math.sqrt(3.0)],
                      [1.0, -1.0 / math.sqrt(3.0)],
                      [0.0, 2.0 / math.sqrt(3.0)]])
_BIUNIT_VERTS = np.array([[-1.0, -1.0], [1.0, -1.0], [-1.0, 1.0]])


def _warp_1d(N: int, x: np.ndarray) -> np.ndarray:
    """Scaled 1D warp: (interpolant of GLL - equispaced shift) / (1 - x^2).

    The interpolant (degree N, through the equispaced points) maps the
    equispaced points of [-1,1] to the GLL points.  Division by 1 - x^2 is the
    edge-blending normalisation of Warburton (2006); it is zero at x = +-1.
    """
    xeq = np.linspace(-1.0, 1.0, N + 1)
    xgll, _ = gll_nodes_weights(N)
    shift = lagrange1d(xeq, x) @ (xgll - xeq)
    out = np.zeros_like(x)
    inside = np.abs(x) < 1.0 - 1e-10
    out[inside] = shift[inside] / (1.0 - x[inside] ** 2)
    return out


def tri_nodes(N: int):
    """Warp & Blend nodes (alpha = 0) on the bi-unit triangle.

    Node ordering: lattice index (a, b), a + b <= N, barycentrics
    lambda2 = a/N, lambda3 = b/N, with b the outer loop.
    Returns (r, s) arrays of length (N+1)(N+2)/2.
    """
    lam = []
    for b in range(N + 1):
        for a in range(N + 1 - b):
            l2 = a / N
            l3 = b / N
            lam.append((1.0 - l2 - l3, l2, l3))
    lam = np.array(lam)
    X = lam @ _EQ_VERTS  # equispaced points in the equilateral triangle
    # edge-by-edge displacement: blend 4 la lb, warp along the edge direction
    for (A, B) in ((0, 1), (1, 2), (2, 0)):
        d = _EQ_VERTS[B] - _EQ_VERTS[A]
        d = d / np.linalg.norm(d)
        w = 4.0 * lam[:, A] * lam[:, B] * _warp_1d(N, lam[:, B] - lam[:, A])
        X = X + w[:, None] * d[None, :]
    # affine map equilateral -> bi-unit through barycentric coordinates
    T = np.vstack([_EQ_VERTS.T, np.ones(3)])  # 3x3
    bary = np.linalg.solve(T, np.vstack([X.T, np.ones(len(X))]))  # (3, n)
    rs = bary.T @ _BIUNIT_VERTS
    return rs[:, 0].copy(), rs[:, 1].copy()


def tri_modes(N: int):
    """Exponent pairs (a, b), a + b <= N, of the Legendre-product basis."""
    return [(a, b) for a in range(N + 1) for b in range(N + 1 - a)]


def _leg(n: int, x: np.ndarray):
    c = np.zeros(n + 1)
    c[n] = 1.0
    return npleg.legval(x, c), npleg.legval(x, npleg.legder(c)) if n > 0 else np.zeros_like(x)


def tri_poly_basis(N: int, r: np.ndarray, s: np.ndarray):
    """P_a(r) P_b(s) and its r-, s-derivatives at points; each (npts, Np_tri)."""
    r = np.atleast_1d(r).astype(np.float64)
    s = np.atleast_1d(s).astype(np.float64)
    modes = tri_modes(N)
    P = np.zeros((len(r), len(modes)))
    Pr = np.zeros_like(P)
    Ps = np.zeros_like(P)
    for m, (a, b) in enumerate(modes):
        la, dla = _leg(a, r)
        lb, dlb = _leg(b, s)
        P[:, m] = la * lb
        Pr[:, m] = dla * lb
        Ps[:, m] = la * dlb
    return P, Pr, Ps


class Triangle:
    """Nodal P^N triangle: nodes, Lagrange values and derivatives at points."""

    def __init__(self, N: int):
        self.N = N
        self.r, self.s = tri_nodes(N)
        self.Np = len(self.r)
        V, _, _ = tri_poly_basis(N, self.r, self.s)
        self.Vinv = np.linalg.inv(V)

    def eval(self, r, s):
        """Lagrange basis at points: (values, d/dr, d/ds), each (npts, Np)."""
        P, Pr, Ps = tri_poly_basis(self.N, r, s)
        return P @ self.Vinv, Pr @ self.Vinv, Ps @ self.Vinv


def tri_quadrature(n: int):
    """Collapsed-coordinate (Duffy) rule on the bi-unit triangle.

    Gauss-Legendre in (a, b) on [-1,1]^2 with r = (1+a)(1-b)/2 - 1, s = b and
    Jacobian (1-b)/2.  With n points per direction it integrates polynomials
    of total degree 2n - 2 exactly.  Returns (r, s, w); sum(w) = 2.
    """
    x, w = gauss_nodes_weights(n)
    A, B = np.meshgrid(x, x, indexing="ij")
    WA, WB = np.meshgrid(w, w, indexing="ij")
    r = (1.0 + A) * (1.0 - B) / 2.0 - 1.0
    s = B
    ww = WA * WB * (1.0 - B) / 2.0
    return r.ravel(), s.ravel(), ww.ravel()


# ---------------------------------------------------------------------------
# Wedge
# ---------------------------------------------------------------------------


class Wedge:
    """Nodal wedge: triangle Lagrange (x) GLL Lagrange (Sec. 3.1).

    Basis function n = j * Np_tri + i is l^tri_i(r, s) l^1D_j(t).
    """

    kind = "wedge"
    nfaces = 5
    # local vertex ids of the faces: bottom, top, quads on edges v1v2, v2v3, v3v1
    face_verts = [(0, 1, 2), (3, 4, 5), (0, 1, 4, 3), (1, 2, 5, 4), (2, 0, 3, 5)]
    ref_verts = np.array([[-1, -1, -1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1], [1, -1, 1], [-1, 1, 1]], float)

    def __init__(self, N: int):
        self.N = N
        self.tri = Triangle(N)
        self.tgll, self.wgll = gll_nodes_weights(N)
        self.Nq = N + 1
        self.Np_tri = self.tri.Np
        self.Np = self.Np_tri * self.Nq
        j, i = np.divmod(np.arange(self.Np), self.Np_tri)
        self.node_i = i
        self.node_j = j
        self.r = self.tri.r[i]
        self.s = self.tri.s[i]
        self.t = self.tgll[j]

    def eval(self, r, s, t):
        """Values (npts, Np) and reference gradients (npts, Np, 3)."""
        L, Lr, Ls = self.tri.eval(r, s)
        T = lagrange1d(self.tgll, t)
        Tt = lagrange1d_deriv(self.tgll, t)
        i, j = self.node_i, self.node_j
        val = L[:, i] * T[:, j]
        grad = np.stack([Lr[:, i] * T[:, j], Ls[:, i] * T[:, j], L[:, i] * Tt[:, j]], axis=-1)
        return val, grad

    def volume_quadrature(self, lumped: bool = False):
        """Tensor rule: Duffy triangle (N+2)^2 points x Gauss N+2 in t.

        Exact for every volume integrand of the method on vertically mapped
        wedges (degree <= 2N+1 in (r, s), <= 2N in t).  ``lumped=True``
        replaces the t-rule by the (N+1)-point GLL rule, i.e. mass lumping in
        the extruded direction (Sec. 4.1).
        """
        rq, sq, wq = tri_quadrature(self.N + 2)
        if lumped:
            tq, wt = self.tgll, self.wgll
        else:
            tq, wt = gauss_nodes_weights(self.N + 2)
        R = np.repeat(rq, len(tq))
        S = np.repeat(sq, len(tq))
        T = np.tile(tq, len(rq))
        W = np.repeat(wq, len(tq)) * np.tile(wt, len(rq))
        return R, S, T, W


# ---------------------------------------------------------------------------
# Tetrahedron
# ---------------------------------------------------------------------------

# equilateral tetrahedron (edge length 2) used by the 3D Warp & Blend construction
_EQ_TET = np.array([[-1.0, -1.0 / math.sqrt(3.0), -1.0 / math.sqrt(6.0)],
                    [1.0, -1.0 / math.sqrt(3.0), -1.0 / math.sqrt(6.0)],
                    [0.0, 2.0 / math.sqrt(3.0), -1.0 / math.sqrt(6.0)],
                    [0.0, 0.0, 3.0 / math.sqrt(6.0)]])
_BIUNIT_TET = np.array([[-1.0, -1.0, -1.0], [1.0, -1.0, -1.0], [-1.0, 1.0, -1.0], [-1.0, -1.0, 1.0]])
# faces of the tetrahedron: (opposite vertex, the three face vertices)
_TET_FACES = [(3, (0, 1, 2)), (2, (0, 1, 3)), (0, (1, 2, 3)), (1, (0, 2, 3))]


def tet_nodes(N: int):
    """Warp & Blend nodes (alpha = 0) on the bi-unit tetrahedron.

    Equispaced lattice (a, b, c), a+b+c <= N, barycentrics lambda2 = a/N,
    lambda3 = b/N, lambda4 = c/N (c outer, then b, then a).  Every face adds
    its 2D warp (the triangle construction of ``tri_nodes`` evaluated with the
    face's barycentrics), weighted by the face blend
        beta = l_b l_c l_d / ((l_b + l_a/2)(l_c + l_a/2)(l_d + l_a/2)),
    l_a the barycentric of the opposite vertex; beta = 1 on the face.  Nodes on
    an edge get the 1D GLL warp of that edge only.  Face nodes therefore equal
    the triangle nodes and edge nodes the GLL points.
    """
    lam = []
    for c in range(N + 1):
        for b in range(N + 1 - c):
            for a in range(N + 1 - b - c):
                lam.append((1.0 - (a + b + c) / N, a / N, b / N, c / N))
    lam = np.array(lam)
    X = lam @ _EQ_TET
    tol = 1e-10
    nonzero = (lam > tol).sum(axis=1)
    shift = np.zeros_like(X)
    for a, (b, c, d) in _TET_FACES:
        w = np.zeros_like(X)
        for (u, v) in ((b, c), (c, d), (d, b)):
            e = _EQ_TET[v] - _EQ_TET[u]
            e = e / np.linalg.norm(e)
            amt = 4.0 * lam[:, u] * lam[:, v] * _warp_1d(N, lam[:, v] - lam[:, u])
            w += amt[:, None] * e[None, :]
        la, lb, lc, ld = lam[:, a], lam[:, b], lam[:, c], lam[:, d]
        denom = (lb + 0.5 * la) * (lc + 0.5 * la) * (ld + 0.5 * la)
        beta = np.where(denom > tol, lb * lc * ld / np.where(denom > tol, denom, 1.0), 0.0)
        shift += beta[:, None] * w
        # edge nodes of this face: exactly the edge warp
        on_edge = (la < tol) & (nonzero == 2)
        shift[on_edge] = w[on_edge]
    X = X + shift
    T = np.vstack([_EQ_TET.T, np.ones(4)])
    bary = np.linalg.solve(T, np.vstack([X.T, np.ones(len(X))]))
    rst = bary.T @ _BIUNIT_TET
    return rst[:, 0].copy(), rst[:, 1].copy(), rst[:, 2].copy()


def tet_modes(N: int):
    return [(a, b, c) for a in range(N + 1) for b in range(N + 1 - a) for c in range(N + 1 - a - b)]


def tet_poly_basis(N: int, r, s, t):
    """P_a(r) P_b(s) P_c(t), a+b+c <= N, and its gradient at points."""
    r, s, t = (np.atleast_1d(x).astype(np.float64) for x in (r, s, t))
    modes = tet_modes(N)
    P = np.zeros((len(r), len(modes)))
    G = np.zeros((len(r), len(modes), 3))
    for m, (a, b, c) in enumerate(modes):
        la, dla = _leg(a, r)
        lb, dlb = _leg(b, s)
        lc, dlc = _leg(c, t)
        P[:, m] = la * lb * lc
        G[:, m, 0] = dla * lb * lc
        G[:, m, 1] = la * dlb * lc
        G[:, m, 2] = la * lb * dlc
    return P, G


def tet_quadrature(n: int):
    """Collapsed-coordinate rule on the bi-unit tetrahedron, n Gauss points per
    direction: r = (1+a)(1-b)(1-c)/4 - 1, s = (1+b)(1-c)/2 - 1, t = c, Jacobian
    (1-b)/2 ((1-c)/2)^2; exact to total degree 2n - 3.  sum(w) = 4/3."""
    x, w = gauss_nodes_weights(n)
    A, Bq, Cq = np.meshgrid(x, x, x, indexing="ij")
    WA, WB, WC = np.meshgrid(w, w, w, indexing="ij")
    r = (1 + A) * (1 - Bq) * (1 - Cq) / 4 - 1
    s = (1 + Bq) * (1 - Cq) / 2 - 1
    t = Cq
    ww = WA * WB * WC * (1 - Bq) / 2 * ((1 - Cq) / 2) ** 2
    return r.ravel(), s.ravel(), t.ravel(), ww.ravel()


class Tet:
    """Nodal P^N tetrahedron (Warp & Blend nodes, alpha = 0)."""

    kind = "tet"
    nfaces = 4
    # local vertex ids of the faces: bottom (t=-1), front (s=-1), slanted, left (r=-1)
    face_verts = [(0, 1, 2), (0, 1, 3), (1, 2, 3), (0, 2, 3)]
    ref_verts = _BIUNIT_TET

    def __init__(self, N: int):
        self.N = N
        self.r, self.s, self.t = tet_nodes(N)
        self.Np = len(self.r)
        V, _ = tet_poly_basis(N, self.r, self.s, self.t)
        self.Vinv = np.linalg.inv(V)

    def eval(self, r, s, t):
        P, G = tet_poly_basis(self.N, r, s, t)
        return P @ self.Vinv, np.einsum("qmd,mj->qjd", G, self.Vinv)

    def volume_quadrature(self, lumped: bool = False):
        return tet_quadrature(self.N + 2)

    def face_rules(self, lumped: bool = False):
        """(xi (nq,3), w (nq,), dxi/da, dxi/db) for every face; the reference
        triangle (a, b) maps through the face's vertices by barycentrics."""
        ra, sa, wa = tri_quadrature(self.N + 2)
        l1, l2, l3 = -(ra + sa) / 2, (1 + ra) / 2, (1 + sa) / 2
        rules = []
        for fv in self.face_verts:
            P, Q, R = (self.ref_verts[v] for v in fv)
            xi = l1[:, None] * P + l2[:, None] * Q + l3[:, None] * R
            rules.append((xi, wa, (Q - P) / 2, (R - P) / 2))
        return rules


def _wedge_face_rules(self, lumped: bool = False):
    """(xi (nq,3), w (nq,), dxi/da, dxi/db) for the five wedge faces.

    Triangles: Duffy rule with N+2 points per direction at t = -1 / +1.
    Quadrilaterals: Gauss (N+2) along the edge times Gauss (N+2) in t (GLL
    N+1 in t when lumped); edge parameter u in [-1,1] from the edge's first
    vertex to its second.
    """
    N = self.N
    ra, sa, wa = tri_quadrature(N + 2)
    xg, wg = gauss_nodes_weights(N + 2)
    xt, wt = gll_nodes_weights(N) if lumped else (xg, wg)
    U, T = np.meshgrid(xg, xt, indexing="ij")
    WU, WT = np.meshgrid(wg, wt, indexing="ij")
    u, t, wq = U.ravel(), T.ravel(), (WU * WT).ravel()
    one = np.ones_like(ra)
    return [
        (np.stack([ra, sa, -one], 1), wa, np.array([1.0, 0, 0]), np.array([0, 1.0, 0])),
        (np.stack([ra, sa, one], 1), wa, np.array([1.0, 0, 0]), np.array([0, 1.0, 0])),
        (np.stack([u, -np.ones_like(u), t], 1), wq, np.array([1.0, 0, 0]), np.array([0, 0, 1.0])),
        (np.stack([-u, u, t], 1), wq, np.array([-1.0, 1.0, 0]), np.array([0, 0, 1.0])),
        (np.stack([-np.ones_like(u), -u, t], 1), wq, np.array([0, -1.0, 0]), np.array([0, 0, 1.0])),
    ]


Wedge.face_rules = _wedge_face_rules
