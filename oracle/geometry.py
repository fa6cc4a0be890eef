"""Element geometry for the oracle: vertex maps, Jacobians, inverse maps.

Wedges (Sec. 3.2): x = Phi(r,s,t) = sum_i nu_i v_i(r,s,t) with the six
low-order vertex functions of the paper, rewritten for the bi-unit
reference wedge with triangle barycentrics
    lambda1 = -(r+s)/2, lambda2 = (1+r)/2, lambda3 = (1+s)/2
and vertical hat functions (1-t)/2 (bottom), (1+t)/2 (top):
    v1 = lambda1 (1-t)/2, v2 = lambda2 (1-t)/2, v3 = lambda3 (1-t)/2,
    v4 = lambda1 (1+t)/2, v5 = lambda2 (1+t)/2, v6 = lambda3 (1+t)/2.
Vertex pairs (1,4), (2,5), (3,6) share (r, s).

Tetrahedra: affine map through the four barycentrics of the bi-unit
reference tet with vertices (-1,-1,-1), (1,-1,-1), (-1,1,-1), (-1,-1,1).

Nothing here assumes a wedge is vertically mapped: the Jacobian matrix,
its determinant and inverse are the general 3x3 ones at every point, and
the inverse map is found by Newton iteration.
"""
from __future__ import annotations

import numpy as np


def wedge_vertex_functions(xi: np.ndarray):
    """Values (npts, 6) and reference gradients (npts, 6, 3) of v1..v6."""
    r, s, t = xi[:, 0], xi[:, 1], xi[:, 2]
    l1 = -(r + s) / 2.0
    l2 = (1.0 + r) / 2.0
    l3 = (1.0 + s) / 2.0
    lo = (1.0 - t) / 2.0
    hi = (1.0 + t) / 2.0
    v = np.stack([l1 * lo, l2 * lo, l3 * lo, l1 * hi, l2 * hi, l3 * hi], axis=1)
    dl = np.array([[-0.5, -0.5], [0.5, 0.0], [0.0, 0.5]])  # d lambda_v / d(r, s)
    g = np.zeros((len(r), 6, 3))
    for v_ in range(3):
        g[:, v_, 0] = dl[v_, 0] * lo
        g[:, v_, 1] = dl[v_, 1] * lo
        g[:, v_ + 3, 0] = dl[v_, 0] * hi
        g[:, v_ + 3, 1] = dl[v_, 1] * hi
    g[:, 0, 2] = -l1 / 2.0
    g[:, 1, 2] = -l2 / 2.0
    g[:, 2, 2] = -l3 / 2.0
    g[:, 3, 2] = l1 / 2.0
    g[:, 4, 2] = l2 / 2.0
    g[:, 5, 2] = l3 / 2.0
    return v, g


def tet_vertex_functions(xi: np.ndarray):
    """Barycentrics (npts, 4) of the bi-unit tet and their gradients (npts, 4, 3)."""
    r, s, t = xi[:, 0], xi[:, 1], xi[:, 2]
    v = np.stack([-(1.0 + r + s + t) / 2.0, (1.0 + r) / 2.0, (1.0 + s) / 2.0, (1.0 + t) / 2.0], axis=1)
    g = np.zeros((len(r), 4, 3))
    g[:, 0, :] = -0.5
    g[:, 1, 0] = 0.5
    g[:, 2, 1] = 0.5
    g[:, 3, 2] = 0.5
    return v, g


def vertex_functions(kind: str, xi: np.ndarray):
    if kind == "wedge":
        return wedge_vertex_functions(xi)
    if kind == "tet":
        return tet_vertex_functions(xi)
    raise ValueError(kind)


def map_points(kind: str, X: np.ndarray, xi: np.ndarray):
    """Physical points and Jacobian matrices.

    X: (K, nv, 3) vertex coordinates, xi: (npts, 3) reference points.
    Returns x (K, npts, 3) and Jm (K, npts, 3, 3) with Jm[..., d, c] = dx_d/dxi_c.
    """
    v, g = vertex_functions(kind, xi)
    x = np.einsum("qi,kid->kqd", v, X)
    Jm = np.einsum("qic,kid->kqdc", g, X)
    return x, Jm


def map_points_paired(kind: str, X: np.ndarray, xi: np.ndarray):
    """As map_points but one reference point per element: X (m, nv, 3), xi (m, 3)."""
    v, g = vertex_functions(kind, xi)
    x = np.einsum("mi,mid->md", v, X)
    Jm = np.einsum("mic,mid->mdc", g, X)
    return x, Jm


def inverse_map(kind: str, X: np.ndarray, x: np.ndarray, tol: float = 1e-15, maxit: int = 60):
    """Reference coordinates of physical points by Newton iteration.

    X: (m, nv, 3) vertices of the element holding each point, x: (m, 3).
    """
    m = x.shape[0]
    xi = np.zeros((m, 3))
    if kind == "tet":
        xi[:] = -0.5
    else:
        xi[:, 0] = -1.0 / 3.0
        xi[:, 1] = -1.0 / 3.0
    for _ in range(maxit):
        xm, Jm = map_points_paired(kind, X, xi)
        dxi = np.linalg.solve(Jm, (xm - x)[..., None])[..., 0]
        xi = xi - dxi
        if np.abs(dxi).max() < 1e-12:
            break
    # quadratic convergence: one more step reaches rounding level
    xm, Jm = map_points_paired(kind, X, xi)
    xi = xi - np.linalg.solve(Jm, (xm - x)[..., None])[..., 0]
    return xi
