"""Plain DG semi-discretisation of first-order acoustics (oracle, FP64).

Follows Sec. 2 of the paper directly:

* PDE (Sec. 2):  p_t / kappa + div u = 0,  rho u_t + grad p = 0, rho and
  kappa = rho c^2 constant per element.
* Strong DG form (eq. ``form``): for every test function l_i of element k
      int (1/kappa) p_t l_i = - int (div u) l_i
                              + int_dk 1/2 (tau_p [p] - n.[u]) l_i
      int rho u_t l_i       = - int (grad p) l_i
                              + int_dk 1/2 (tau_u [u].n - [p]) n l_i
  with [q] = q+ - q-, tau_p = 1/{rho c}, tau_u = {rho c} (upwind) or
  tau = 0 (central flux, Sec. 4.1).
* Boundary mirror states: Dirichlet p = 0 via p+ = -p-, u+ = u- (Sec. 2);
  rigid wall via p+ = p-, u+ = u- - 2 (n.u-) n (reading for the layered
  test configurations, which ask for rigid walls).
* Matrix form (Sec. 2.1): M^k dU/dt = ... with M^k and S^k_{x,y,z} the
  exact integrals, inverted densely.

Every element matrix is built by quadrature over the *physical* element
through the general 3x3 Jacobian at each point; face integrals use
quadrature on each face with the neighbour trace evaluated at the physical
quadrature point through the neighbour's inverse map.  No node maps,
orientation codes or Kronecker factorisations are used.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import basis as B
from . import geometry as G

# ---------------------------------------------------------------------------
# Mesh description
# ---------------------------------------------------------------------------

# local faces of the wedge: vertex ids and reference parametrisation
WEDGE_FACE_VERTS = [(0, 1, 2), (3, 4, 5), (0, 1, 4, 3), (1, 2, 5, 4), (2, 0, 3, 5)]


@dataclass
class Mesh:
    """Wedge mesh: vertices (nv,3), wedges (nw,6) with v1..v3 the bottom
    triangle and v4..v6 above them, per-element wave speed c and density rho.
    bc in {'dirichlet', 'rigid'}, flux in {'upwind', 'central'}."""

    verts: np.ndarray
    wedges: np.ndarray
    c: np.ndarray
    rho: np.ndarray
    bc: str = "rigid"
    flux: str = "upwind"

    @property
    def K(self) -> int:
        return len(self.wedges)


def face_connectivity(mesh: Mesh):
    """Neighbour element and neighbour local face for every (element, face).

    Faces are matched by their sets of global vertex ids.  Returns
    nbr (K, 5) int64 (-1 on the boundary) and nbr_face (K, 5).
    """
    K = mesh.K
    keys = np.full((K, 5, 4), -1, dtype=np.int64)
    for f, fv in enumerate(WEDGE_FACE_VERTS):
        ids = np.sort(mesh.wedges[:, list(fv)], axis=1)
        keys[:, f, 4 - len(fv):] = ids
    flat = keys.reshape(-1, 4)
    order = np.lexsort(flat.T[::-1])
    sk = flat[order]
    same = np.all(sk[1:] == sk[:-1], axis=1)
    nbr = np.full(K * 5, -1, dtype=np.int64)
    a = order[:-1][same]
    b = order[1:][same]
    nbr[a] = b // 5
    nbr[b] = a // 5
    nbr_face = np.full(K * 5, -1, dtype=np.int64)
    nbr_face[a] = b % 5
    nbr_face[b] = a % 5
    # a face shared by more than two elements is not a valid conforming mesh
    if np.any(same[1:] & same[:-1]):
        raise ValueError("face shared by more than two elements")
    return nbr.reshape(K, 5), nbr_face.reshape(K, 5)


# ---------------------------------------------------------------------------
# Face quadrature on the reference wedge
# ---------------------------------------------------------------------------


def wedge_face_rules(N: int, lumped: bool = False):
    """Reference face rules for the five wedge faces.

    Returns a list of (xi (nq,3), w (nq,), dxi_da (3,), dxi_db (3,)): points
    in volume reference coordinates, face weights, and the constant
    derivatives of the face parametrisation.  Triangles use the Duffy rule
    with N+2 points per direction; quads Gauss (N+2) along the edge times
    Gauss (N+2) in t (GLL N+1 in t when lumped).
    """
    ra, sa, wa = B.tri_quadrature(N + 2)
    xg, wg = B.gauss_nodes_weights(N + 2)
    if lumped:
        xt, wt = B.gll_nodes_weights(N)
    else:
        xt, wt = xg, wg
    U, T = np.meshgrid(xg, xt, indexing="ij")
    WU, WT = np.meshgrid(wg, wt, indexing="ij")
    u, t, wq = U.ravel(), T.ravel(), (WU * WT).ravel()
    rules = []
    rules.append((np.stack([ra, sa, -np.ones_like(ra)], 1), wa, np.array([1.0, 0, 0]), np.array([0, 1.0, 0])))
    rules.append((np.stack([ra, sa, np.ones_like(ra)], 1), wa, np.array([1.0, 0, 0]), np.array([0, 1.0, 0])))
    rules.append((np.stack([u, -np.ones_like(u), t], 1), wq, np.array([1.0, 0, 0]), np.array([0, 0, 1.0])))
    rules.append((np.stack([-u, u, t], 1), wq, np.array([-1.0, 1.0, 0]), np.array([0, 0, 1.0])))
    rules.append((np.stack([-np.ones_like(u), -u, t], 1), wq, np.array([0, -1.0, 0]), np.array([0, 0, 1.0])))
    return rules


# ---------------------------------------------------------------------------
# Dense element operators
# ---------------------------------------------------------------------------


@dataclass
class Operators:
    """Dense per-element operators for a subset ``elems`` of the mesh."""

    N: int
    elems: np.ndarray
    M: np.ndarray          # (K, Np, Np)
    Minv: np.ndarray       # (K, Np, Np)
    S: np.ndarray          # (3, K, Np, Np)  (S_d)_ij = int l_i d_d l_j
    Pown: list             # per face (nq, Np)
    wJ: list               # per face (K, nq)   weight * surface Jacobian
    n: list                # per face (K, nq, 3) outward unit normal
    nbr: np.ndarray        # (K, 5) global neighbour id, -1 on the boundary
    Pnbr: list             # per face (K, nq, Np) neighbour basis at the points
    tau_p: np.ndarray      # (K, 5)
    tau_u: np.ndarray      # (K, 5)
    kappa: np.ndarray      # (K,)
    rho: np.ndarray        # (K,)
    bc: str
    extra: dict = field(default_factory=dict)


def element_vertices(mesh: Mesh, elems: np.ndarray) -> np.ndarray:
    return mesh.verts[mesh.wedges[elems]]


def build_operators(mesh: Mesh, N: int, elems=None, lumped: bool = False, chunk: int = 256) -> Operators:
    """Build the dense operators of the elements ``elems`` (default: all)."""
    K_all = mesh.K
    elems = np.arange(K_all) if elems is None else np.asarray(elems, dtype=np.int64)
    ref = B.Wedge(N)
    Np = ref.Np
    R, S_, T, W = ref.volume_quadrature(lumped)
    xi_v = np.stack([R, S_, T], 1)
    Bv, Bg = ref.eval(R, S_, T)
    rules = wedge_face_rules(N, lumped)
    Pown = [ref.eval(*rule[0].T)[0] for rule in rules]

    nbr_all, _ = face_connectivity(mesh)
    kappa_all = mesh.rho * mesh.c ** 2
    Z_all = mesh.rho * mesh.c

    K = len(elems)
    M = np.zeros((K, Np, Np))
    Sd = np.zeros((3, K, Np, Np))
    wJ = [np.zeros((K, len(r[1]))) for r in rules]
    nn = [np.zeros((K, len(r[1]), 3)) for r in rules]
    Pnbr = [np.zeros((K, len(r[1]), Np)) for r in rules]
    for c0 in range(0, K, chunk):
        ids = elems[c0:c0 + chunk]
        sl = slice(c0, c0 + len(ids))
        X = element_vertices(mesh, ids)
        # volume: general Jacobian at every quadrature point
        _, Jm = G.map_points("wedge", X, xi_v)
        detJ = np.linalg.det(Jm)
        if np.any(detJ <= 0):
            raise ValueError("non-positive Jacobian")
        Jinv = np.linalg.inv(Jm)  # Jinv[..., c, d] = d xi_c / d x_d
        Gp = np.einsum("qjc,kqcd->kqjd", Bg, Jinv)
        wdet = W[None, :] * detJ
        M[sl] = np.einsum("kq,qi,qj->kij", wdet, Bv, Bv)
        for d in range(3):
            Sd[d, sl] = np.einsum("kq,qi,kqj->kij", wdet, Bv, Gp[..., d])
        centroid = X.mean(axis=1)
        for f, (xi_f, w_f, da, db) in enumerate(rules):
            xq, Jf = G.map_points("wedge", X, xi_f)
            t1 = np.einsum("kqdc,c->kqd", Jf, da)
            t2 = np.einsum("kqdc,c->kqd", Jf, db)
            cr = np.cross(t1, t2)
            area = np.linalg.norm(cr, axis=-1)
            nvec = cr / area[..., None]
            sign = np.sign(np.einsum("kqd,kqd->k", xq - centroid[:, None, :], nvec))
            nn[f][sl] = nvec * sign[:, None, None]
            wJ[f][sl] = w_f[None, :] * area
            nb = nbr_all[ids, f]
            inner = np.nonzero(nb >= 0)[0]
            if len(inner):
                nq = len(w_f)
                Xn = element_vertices(mesh, nb[inner])
                Xrep = np.repeat(Xn, nq, axis=0)
                xi_n = G.inverse_map("wedge", Xrep, xq[inner].reshape(-1, 3))
                vals, _ = ref.eval(xi_n[:, 0], xi_n[:, 1], xi_n[:, 2])
                Pnbr[f][c0 + inner] = vals.reshape(len(inner), nq, Np)
    nbr = nbr_all[elems]
    Zm = Z_all[elems][:, None] * np.ones((1, 5))
    Zp = np.where(nbr >= 0, Z_all[np.maximum(nbr, 0)], Zm)
    if mesh.flux == "upwind":
        tau_p = 2.0 / (Zm + Zp)
        tau_u = (Zm + Zp) / 2.0
    elif mesh.flux == "central":
        tau_p = np.zeros_like(Zm)
        tau_u = np.zeros_like(Zm)
    else:
        raise ValueError(mesh.flux)
    Minv = np.linalg.inv(M)
    return Operators(N=N, elems=elems, M=M, Minv=Minv, S=Sd, Pown=Pown, wJ=wJ, n=nn, nbr=nbr,
                     Pnbr=Pnbr, tau_p=tau_p, tau_u=tau_u, kappa=kappa_all[elems], rho=mesh.rho[elems],
                     bc=mesh.bc)


# ---------------------------------------------------------------------------
# Right-hand side
# ---------------------------------------------------------------------------


def face_traces(ops: Operators, U: np.ndarray, f: int):
    """Own and neighbour traces (p-, u-, p+, u+) at the quadrature points of face f.

    U: (..., K_all, 4, Np) full state; traces are for ops.elems.
    """
    Uk = U[..., ops.elems, :, :]
    P = ops.Pown[f]
    pm = np.einsum("qj,...kj->...kq", P, Uk[..., 0, :])
    um = np.einsum("qj,...kdj->...kdq", P, Uk[..., 1:4, :])
    nb = ops.nbr[:, f]
    Un = U[..., np.maximum(nb, 0), :, :]
    pp = np.einsum("kqj,...kj->...kq", ops.Pnbr[f], Un[..., 0, :])
    up = np.einsum("kqj,...kdj->...kdq", ops.Pnbr[f], Un[..., 1:4, :])
    n = ops.n[f]  # (K, nq, 3)
    bnd = (nb < 0)[:, None]
    if ops.bc == "dirichlet":
        pp = np.where(bnd, -pm, pp)
        up = np.where(bnd[:, None, :], um, up)
    elif ops.bc == "rigid":
        pp = np.where(bnd, pm, pp)
        unm = np.einsum("...kdq,kqd->...kq", um, n)
        mirror = um - 2.0 * unm[..., None, :] * np.moveaxis(n, -1, -2)
        up = np.where(bnd[:, None, :], mirror, up)
    else:
        raise ValueError(ops.bc)
    return pm, um, pp, up


def rhs(ops: Operators, U: np.ndarray) -> np.ndarray:
    """dU/dt for the elements ops.elems given the full state U (..., K_all, 4, Np)."""
    Uk = U[..., ops.elems, :, :]
    p = Uk[..., 0, :]
    vol = np.zeros_like(Uk)
    for d in range(3):
        vol[..., 0, :] -= np.einsum("kij,...kj->...ki", ops.S[d], Uk[..., d + 1, :])
        vol[..., d + 1, :] = -np.einsum("kij,...kj->...ki", ops.S[d], p)
    surf = np.zeros_like(Uk)
    for f in range(5):
        pm, um, pp, up = face_traces(ops, U, f)
        n = ops.n[f]
        jp = pp - pm
        jun = np.einsum("...kdq,kqd->...kq", up - um, n)
        Fp = 0.5 * (ops.tau_p[:, f, None] * jp - jun)
        Fu = 0.5 * (ops.tau_u[:, f, None] * jun - jp)
        P = ops.Pown[f]
        surf[..., 0, :] += np.einsum("qj,...kq->...kj", P, ops.wJ[f] * Fp)
        for d in range(3):
            surf[..., d + 1, :] += np.einsum("qj,...kq->...kj", P, ops.wJ[f] * n[..., d] * Fu)
    out = np.einsum("kij,...kfj->...kfi", ops.Minv, vol + surf)
    out[..., 0, :] *= ops.kappa[:, None]
    out[..., 1:, :] *= (1.0 / ops.rho)[:, None, None]
    return out


def energy(ops: Operators, U: np.ndarray) -> float:
    """E = 1/2 sum_k (p^T M p / kappa + rho u^T M u) (integrand of eq. ``estab``)."""
    Uk = U[ops.elems]
    MU = np.einsum("kij,kfj->kfi", ops.M, Uk)
    e = np.einsum("kfi,kfi->kf", Uk, MU)
    return 0.5 * float(np.sum(e[:, 0] / ops.kappa + ops.rho * e[:, 1:].sum(axis=1)))


def energy_rate_from_jumps(ops: Operators, U: np.ndarray) -> float:
    """Face-dissipation side of the energy identity, computed from traces only.

    Each interior face contributes -1/2 int (tau_p [p]^2 + tau_u [u_n]^2);
    it is visited from both sides, hence the factor 1/4 per visit.  A
    Dirichlet face contributes -int tau_p (p-)^2, a rigid face
    -int tau_u (u_n-)^2 (mirror states inserted in the same flux).
    Requires ops built for all elements.
    """
    total = 0.0
    for f in range(5):
        pm, um, pp, up = face_traces(ops, U, f)
        n = ops.n[f]
        jp = pp - pm
        jun = np.einsum("kdq,kqd->kq", up - um, n)
        integrand = ops.tau_p[:, f, None] * jp ** 2 + ops.tau_u[:, f, None] * jun ** 2
        # boundary faces: the mirror states give [p] = -2 p- (Dirichlet) or
        # [u_n] = -2 u_n- (rigid), so -tau (.)^2 is again -1/4 of the jump form
        total += float(np.sum(-0.25 * ops.wJ[f] * integrand))
    return total


def energy_rate(ops: Operators, U: np.ndarray, dUdt: np.ndarray) -> float:
    """dE/dt = sum_k (p^T M p_t / kappa + rho u^T M u_t)."""
    Uk = U[ops.elems]
    MU = np.einsum("kij,kfj->kfi", ops.M, dUdt)
    e = np.einsum("kfi,kfi->kf", Uk, MU)
    return float(np.sum(e[:, 0] / ops.kappa + ops.rho * e[:, 1:].sum(axis=1)))


# ---------------------------------------------------------------------------
# Nodes, interpolation, point location
# ---------------------------------------------------------------------------


def node_coords(mesh: Mesh, N: int) -> np.ndarray:
    """Physical node coordinates (K, Np, 3)."""
    ref = B.Wedge(N)
    xi = np.stack([ref.r, ref.s, ref.t], 1)
    x, _ = G.map_points("wedge", mesh.verts[mesh.wedges], xi)
    return x


def locate(mesh: Mesh, x: np.ndarray, tol: float = 1e-12):
    """Lowest-index element containing point x and its reference coordinates."""
    x = np.asarray(x, float)
    X = mesh.verts[mesh.wedges]
    # only elements whose bounding box holds the point can contain it
    pad = 1e-9 * (np.abs(X).max() + 1.0)
    cand = np.nonzero(np.all((X.min(axis=1) - pad <= x) & (x <= X.max(axis=1) + pad), axis=1))[0]
    if len(cand) == 0:
        raise ValueError("point outside the mesh")
    xi = G.inverse_map("wedge", X[cand], np.repeat(x[None, :], len(cand), axis=0))
    r, s, t = xi[:, 0], xi[:, 1], xi[:, 2]
    inside = (r >= -1 - tol) & (s >= -1 - tol) & (r + s <= tol) & (np.abs(t) <= 1 + tol)
    hits = np.nonzero(inside)[0]
    if len(hits) == 0:
        raise ValueError("point outside the mesh")
    return int(cand[hits[0]]), xi[hits[0]]


def point_basis(N: int, xi: np.ndarray) -> np.ndarray:
    """Wedge Lagrange basis values at one reference point (Np,)."""
    ref = B.Wedge(N)
    v, _ = ref.eval(np.array([xi[0]]), np.array([xi[1]]), np.array([xi[2]]))
    return v[0]


def ricker(t, f0: float, t0: float, amp: float = 1.0):
    """Ricker wavelet amp (1 - 2 pi^2 f0^2 (t-t0)^2) exp(-pi^2 f0^2 (t-t0)^2)."""
    a = (np.pi * f0 * (np.asarray(t) - t0)) ** 2
    return amp * (1.0 - 2.0 * a) * np.exp(-a)


@dataclass
class PointSource:
    """Source s(t) delta(x - xs) in the pressure equation:
    rhs_p += kappa s(t) M^-1 l(xs) on the element holding xs."""

    elem: int
    vec: np.ndarray  # kappa M^-1 l(xs), (Np,)
    f0: float
    t0: float
    amp: float

    def value(self, t: float) -> float:
        return float(ricker(t, self.f0, self.t0, self.amp))


def make_point_source(mesh: Mesh, N: int, xs, f0: float, t0: float, amp: float = 1.0) -> PointSource:
    k, xi = locate(mesh, xs)
    ops = build_operators(mesh, N, elems=[k])
    lvec = point_basis(N, xi)
    vec = ops.kappa[0] * (ops.Minv[0] @ lvec)
    return PointSource(k, vec, f0, t0, amp)


def make_receivers(mesh: Mesh, N: int, xr: np.ndarray):
    """(elements, basis rows) sampling p at receiver points."""
    elems, rows = [], []
    for x in np.atleast_2d(xr):
        k, xi = locate(mesh, x)
        elems.append(k)
        rows.append(point_basis(N, xi))
    return np.array(elems), np.array(rows)


# ---------------------------------------------------------------------------
# Time step (reading of "trace and Markov inequalities", Sec. 6)
# ---------------------------------------------------------------------------


def stable_dt(mesh: Mesh, N: int, cfl: float) -> float:
    """dt = cfl / max_k [ c_k (N+1)(N+3)/3 max_f max J_f / min J ].

    The paper takes the step from trace and Markov inequality constants
    without printing the formula (Sec. 6); this reading uses the 3D trace
    constant (N+1)(N+3)/3 and the face-to-volume Jacobian ratio.

    J is the volume Jacobian (bi-unit reference), J_f the face Jacobian; both
    are linear on vertically mapped wedges, so their extremes are taken over
    the reference vertices.
    """
    X = mesh.verts[mesh.wedges]
    vref = np.array([[-1, -1, -1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1], [1, -1, 1], [-1, 1, 1]], float)
    _, Jm = G.map_points("wedge", X, vref)
    Jmin = np.linalg.det(Jm).min(axis=1)
    rules = wedge_face_rules(N)
    Jfmax = np.zeros(mesh.K)
    face_ref_verts = [vref[list(fv)] for fv in WEDGE_FACE_VERTS]
    for f, (_, _, da, db) in enumerate(rules):
        _, Jf = G.map_points("wedge", X, face_ref_verts[f])
        t1 = np.einsum("kqdc,c->kqd", Jf, da)
        t2 = np.einsum("kqdc,c->kqd", Jf, db)
        Jfmax = np.maximum(Jfmax, np.linalg.norm(np.cross(t1, t2), axis=-1).max(axis=1))
    rate = mesh.c * ((N + 1) * (N + 3) / 3.0) * Jfmax / Jmin
    return cfl / float(rate.max())
