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

Meshes mix wedges (elements 0..nw-1) and tetrahedra (nw..nw+nt-1), joined
through triangular faces (Sec. 3.1).  Where a wedge's quadrilateral face is
covered by two triangular tetrahedron faces instead (columns of prisms split
into tetrahedra next to unsplit columns), the flux is integrated on the
common refinement, the two triangles, with quadrature exact in the vertical
coordinate and converged along the edge (``mortar_faces``).  Nodal arrays are (K, 4, Np) with Np
the largest element size; a tetrahedron uses its first Np_tet entries and
the rest stay zero (see ``node_mask``).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import basis as B
from . import geometry as G

NFACE = 5  # face slots per element (tetrahedra leave the last one empty)


@dataclass
class Mesh:
    """Vertices (nv,3); wedges (nw,6) with v1..v3 the bottom triangle and
    v4..v6 above them; tetrahedra (nt,4); per-element wave speed c and
    density rho (wedges first).  bc in {'dirichlet','rigid'}, flux in
    {'upwind','central'}."""

    verts: np.ndarray
    wedges: np.ndarray
    c: np.ndarray
    rho: np.ndarray
    bc: str = "rigid"
    flux: str = "upwind"
    tets: np.ndarray = None

    @property
    def nw(self) -> int:
        return len(self.wedges)

    @property
    def nt(self) -> int:
        return 0 if self.tets is None else len(self.tets)

    @property
    def K(self) -> int:
        return self.nw + self.nt

    def kinds(self) -> np.ndarray:
        """0 for wedges, 1 for tetrahedra."""
        return np.concatenate([np.zeros(self.nw, int), np.ones(self.nt, int)])


def references(N: int, mesh: Mesh):
    refs = [B.Wedge(N)]
    if mesh is not None and mesh.nt:
        refs.append(B.Tet(N))
    return refs


def node_mask(mesh: Mesh, N: int) -> np.ndarray:
    """(K, Np) True on the nodes an element actually has."""
    refs = references(N, mesh)
    Np = max(r.Np for r in refs)
    mask = np.zeros((mesh.K, Np), bool)
    for kind, ref in enumerate(refs):
        mask[mesh.kinds() == kind, :ref.Np] = True
    return mask


def _vertices(mesh: Mesh, kind: int, ids: np.ndarray) -> np.ndarray:
    if kind == 0:
        return mesh.verts[mesh.wedges[ids]]
    return mesh.verts[mesh.tets[np.asarray(ids) - mesh.nw]]


def face_connectivity(mesh: Mesh):
    """Neighbour element and its local face for every (element, face slot).

    Faces are matched by their sets of global vertex ids.  Returns nbr (K, 5)
    (-1 on the boundary, -2 for the empty fifth slot of a tetrahedron) and
    nbr_face (K, 5).
    """
    K = mesh.K
    keys = np.full((K, NFACE, 4), -1, dtype=np.int64)
    present = np.zeros((K, NFACE), bool)
    kinds = mesh.kinds()
    for kind, ref in enumerate([B.Wedge, B.Tet][: 2 if mesh.nt else 1]):
        ids = np.nonzero(kinds == kind)[0]
        conn = mesh.wedges if kind == 0 else mesh.tets
        for f, fv in enumerate(ref.face_verts):
            v = np.sort(conn[:, list(fv)], axis=1)
            keys[ids, f, 4 - len(fv):] = v
            present[ids, f] = True
    flat = keys.reshape(-1, 4)
    slot_ok = present.reshape(-1)
    cand = np.nonzero(slot_ok)[0]
    order = cand[np.lexsort(flat[cand].T[::-1])]
    sk = flat[order]
    same = np.all(sk[1:] == sk[:-1], axis=1)
    if np.any(same[1:] & same[:-1]):
        raise ValueError("face shared by more than two elements")
    nbr = np.full(K * NFACE, -1, dtype=np.int64)
    nbr_face = np.full(K * NFACE, -1, dtype=np.int64)
    a = order[:-1][same]
    b = order[1:][same]
    nbr[a] = b // NFACE
    nbr[b] = a // NFACE
    nbr_face[a] = b % NFACE
    nbr_face[b] = a % NFACE
    nbr[~slot_ok] = -2
    return nbr.reshape(K, NFACE), nbr_face.reshape(K, NFACE)


def mortar_faces(mesh: Mesh, nbr: np.ndarray):
    """Wedge quadrilateral faces covered by two triangular tetrahedron faces.

    The quadrilateral of wedge face f (corners A0, A1 on the bottom edge from
    its first to its second vertex, A2, A3 above them) is split along A0-A2
    (diagonal 0) or A1-A3 (diagonal 1).  Returns a list of
    (wedge, face, diagonal, ((tet, tet_face) below the diagonal,
    (tet, tet_face) above it)); ``nbr`` is marked -3 on every face involved.
    """
    if not mesh.nt:
        return []
    open_tri = {}
    kinds = mesh.kinds()
    for k in np.nonzero((kinds == 1) & np.any(nbr[:, :4] == -1, axis=1))[0]:
        for f, fv in enumerate(B.Tet.face_verts):
            if nbr[k, f] == -1:
                open_tri[tuple(sorted(mesh.tets[k - mesh.nw][list(fv)]))] = (k, f)
    out = []
    for k in range(mesh.nw):
        for f in range(2, 5):
            if nbr[k, f] != -1:
                continue
            A = mesh.wedges[k][list(B.Wedge.face_verts[f])]  # A0 A1 A2 A3
            for diag, (lo, hi) in enumerate((((0, 1, 2), (0, 2, 3)), ((0, 1, 3), (1, 2, 3)))):
                kl = tuple(sorted(A[list(lo)]))
                kh = tuple(sorted(A[list(hi)]))
                if kl in open_tri and kh in open_tri:
                    tl, th = open_tri.pop(kl), open_tri.pop(kh)
                    out.append((k, f, diag, (tl, th)))
                    nbr[k, f] = -3
                    nbr[tl[0], tl[1]] = -3
                    nbr[th[0], th[1]] = -3
                    break
    return out


def _mortar_rule(N: int):
    """Rule on the quadrilateral face in (edge parameter xi, vertical t):
    Gauss in xi (24 points: the integrand is rational along the edge, with
    poles far outside [-1,1] while the wedge has positive height) times
    Gauss in t on each side of the diagonal (N+3 points: exact, the
    integrands are polynomials of degree <= 2N in t at fixed xi)."""
    xg, wg = B.gauss_nodes_weights(24)
    tg, wt = B.gauss_nodes_weights(N + 3)
    return xg, wg, tg, wt


def build_mortars(mesh: Mesh, N: int, refs, elems: np.ndarray):
    """Quadrature data of every mortar region touching ``elems``: own wedge and
    tetrahedron basis values at the points of the common refinement."""
    nbr, _ = face_connectivity(mesh)
    mortars = mortar_faces(mesh, nbr)
    if not mortars:
        return None
    xg, wg, tg, wt = _mortar_rule(N)
    W, T = refs[0], refs[1]
    pos = -np.ones(mesh.K, dtype=np.int64)
    pos[elems] = np.arange(len(elems))
    Z = mesh.rho * mesh.c
    regions = []
    for (k, f, diag, tets) in mortars:
        X = mesh.verts[mesh.wedges[k]]
        e = f - 2
        a, b = e, (e + 1) % 3
        zb = X[a, 2] * (1 - xg) / 2 + X[b, 2] * (1 + xg) / 2
        zt = X[a + 3, 2] * (1 - xg) / 2 + X[b + 3, 2] * (1 + xg) / 2
        if diag == 0:
            zd = X[a, 2] * (1 - xg) / 2 + X[b + 3, 2] * (1 + xg) / 2
        else:
            zd = X[b, 2] * (1 + xg) / 2 + X[a + 3, 2] * (1 - xg) / 2
        td = (2 * zd - zb - zt) / (zt - zb)
        centroid = X.mean(axis=0)
        for side, (t_el, t_face) in enumerate(tets):
            if pos[k] < 0 and pos[t_el] < 0:
                continue
            lo = -1.0 if side == 0 else td
            hi = td if side == 0 else 1.0
            T_ = (lo + hi)[:, None] / 2 + ((hi - lo)[:, None] / 2) * tg[None, :]   # (nxi, nt)
            w = wg[:, None] * wt[None, :] * (hi - lo)[:, None] / 2
            xi_e = np.repeat(xg, len(tg))
            tt = T_.ravel()
            if e == 0:
                rs = np.stack([xi_e, -np.ones_like(xi_e)], 1)
                da = np.array([1.0, 0, 0])
            elif e == 1:
                rs = np.stack([-xi_e, xi_e], 1)
                da = np.array([-1.0, 1.0, 0])
            else:
                rs = np.stack([-np.ones_like(xi_e), -xi_e], 1)
                da = np.array([0, -1.0, 0])
            xi = np.concatenate([rs, tt[:, None]], 1)
            xq, Jq = G.map_points("wedge", X[None], xi)
            xq, Jq = xq[0], Jq[0]
            t1 = Jq @ da
            t2 = Jq @ np.array([0, 0, 1.0])
            cr = np.cross(t1, t2)
            area = np.linalg.norm(cr, axis=-1)
            n = cr[0] / area[0]
            if np.dot(xq[0] - centroid, n) < 0:
                n = -n
            wJ = w.ravel() * area
            Pw, _ = W.eval(xi[:, 0], xi[:, 1], xi[:, 2])
            Xt = mesh.verts[mesh.tets[t_el - mesh.nw]]
            xt = G.inverse_map("tet", np.repeat(Xt[None], len(xq), axis=0), xq)
            Pt, _ = T.eval(xt[:, 0], xt[:, 1], xt[:, 2])
            Zs = Z[k] + Z[t_el]
            if mesh.flux == "upwind":
                tp, tu = 2.0 / Zs, Zs / 2.0
            else:
                tp = tu = 0.0
            regions.append(dict(k=k, f=f, t=t_el, pk=pos[k], pt=pos[t_el], Pw=Pw, Pt=Pt, wJ=wJ, n=n,
                                tau_p=tp, tau_u=tu))
    return regions


def _mortar_fluxes(reg, U):
    """Traces and fluxes of one mortar region seen from the wedge."""
    Uw = U[..., reg["k"], :, :]
    Ut = U[..., reg["t"], :, :]
    Pw, Pt, n = reg["Pw"], reg["Pt"], reg["n"]
    pm = np.einsum("qj,...j->...q", Pw, Uw[..., 0, :Pw.shape[1]])
    um = np.einsum("qj,...dj->...dq", Pw, Uw[..., 1:4, :Pw.shape[1]])
    pp = np.einsum("qj,...j->...q", Pt, Ut[..., 0, :Pt.shape[1]])
    up = np.einsum("qj,...dj->...dq", Pt, Ut[..., 1:4, :Pt.shape[1]])
    jp = pp - pm
    jun = np.einsum("...dq,d->...q", up - um, n)
    return jp, jun


def _add_mortars(ops, U, surf):
    for reg in ops.extra.get("mortars") or []:
        jp, jun = _mortar_fluxes(reg, U)
        tp, tu, n, wJ = reg["tau_p"], reg["tau_u"], reg["n"], reg["wJ"]
        if reg["pk"] >= 0:
            Fp = 0.5 * (tp * jp - jun)
            Fu = 0.5 * (tu * jun - jp)
            Pw = reg["Pw"]
            nw_ = Pw.shape[1]
            surf[..., reg["pk"], 0, :nw_] += np.einsum("qj,...q->...j", Pw, wJ * Fp)
            for d in range(3):
                surf[..., reg["pk"], d + 1, :nw_] += np.einsum("qj,...q->...j", Pw, wJ * n[d] * Fu)
        if reg["pt"] >= 0:
            # seen from the tetrahedron: normal -n, jumps [p]' = -[p], [u.n]' = [u.n]
            Fp = 0.5 * (-tp * jp - jun)
            Fu = 0.5 * (tu * jun + jp)
            Pt = reg["Pt"]
            nt_ = Pt.shape[1]
            surf[..., reg["pt"], 0, :nt_] += np.einsum("qj,...q->...j", Pt, wJ * Fp)
            for d in range(3):
                surf[..., reg["pt"], d + 1, :nt_] -= np.einsum("qj,...q->...j", Pt, wJ * n[d] * Fu)


# ---------------------------------------------------------------------------
# Dense element operators
# ---------------------------------------------------------------------------


@dataclass
class Operators:
    """Dense per-element operators for a subset ``elems`` of the mesh.

    Nodal dimension Np is the largest element size (zero padding)."""

    N: int
    elems: np.ndarray
    M: np.ndarray          # (K, Np, Np), zero padding
    Minv: np.ndarray       # (K, Np, Np), zero padding
    S: np.ndarray          # (3, K, Np, Np)  (S_d)_ij = int l_i d_d l_j
    Pown: list             # per face slot (K, nq, Np) own basis at the face points
    wJ: list               # per face slot (K, nq) weight * surface Jacobian (0: no face)
    n: list                # per face slot (K, nq, 3) outward unit normal
    nbr: np.ndarray        # (K, 5) global neighbour id, -1 boundary, -2 no face
    Pnbr: list             # per face slot (K, nq, Np) neighbour basis at the points
    tau_p: np.ndarray      # (K, 5)
    tau_u: np.ndarray      # (K, 5)
    kappa: np.ndarray      # (K,)
    rho: np.ndarray        # (K,)
    bc: str
    extra: dict = field(default_factory=dict)


def build_operators(mesh: Mesh, N: int, elems=None, lumped: bool = False, chunk: int = 256) -> Operators:
    """Build the dense operators of the elements ``elems`` (default: all)."""
    elems = np.arange(mesh.K) if elems is None else np.asarray(elems, dtype=np.int64)
    refs = references(N, mesh)
    Np = max(r.Np for r in refs)
    kinds_all = mesh.kinds()
    rules = [r.face_rules(lumped) for r in refs]
    nq = max(len(rule[1]) for rr in rules for rule in rr)

    nbr_all, _ = face_connectivity(mesh)
    mortar_faces(mesh, nbr_all)  # marks the faces integrated on the common refinement (-3)
    kappa_all = mesh.rho * mesh.c ** 2
    Z_all = mesh.rho * mesh.c

    K = len(elems)
    M = np.zeros((K, Np, Np))
    Minv = np.zeros((K, Np, Np))
    Sd = np.zeros((3, K, Np, Np))
    Pown = [np.zeros((K, nq, Np)) for _ in range(NFACE)]
    wJ = [np.zeros((K, nq)) for _ in range(NFACE)]
    nn = [np.zeros((K, nq, 3)) for _ in range(NFACE)]
    Pnbr = [np.zeros((K, nq, Np)) for _ in range(NFACE)]
    for kind, ref in enumerate(refs):
        sel = np.nonzero(kinds_all[elems] == kind)[0]
        if len(sel) == 0:
            continue
        n_k = ref.Np
        R, S_, T, W = ref.volume_quadrature(lumped)
        xi_v = np.stack([R, S_, T], 1)
        Bv, Bg = ref.eval(R, S_, T)
        own_face = [ref.eval(*rule[0].T)[0] for rule in rules[kind]]
        for c0 in range(0, len(sel), chunk):
            loc = sel[c0:c0 + chunk]
            ids = elems[loc]
            X = _vertices(mesh, kind, ids)
            # volume: general Jacobian at every quadrature point
            _, Jm = G.map_points(ref.kind, X, xi_v)
            detJ = np.linalg.det(Jm)
            if np.any(detJ <= 0):
                raise ValueError("non-positive Jacobian")
            Jinv = np.linalg.inv(Jm)  # Jinv[..., c, d] = d xi_c / d x_d
            Gp = np.einsum("qjc,kqcd->kqjd", Bg, Jinv)
            wdet = W[None, :] * detJ
            Mk = np.einsum("kq,qi,qj->kij", wdet, Bv, Bv)
            M[loc, :n_k, :n_k] = Mk
            Minv[loc, :n_k, :n_k] = np.linalg.inv(Mk)
            for d in range(3):
                Sd[d, loc, :n_k, :n_k] = np.einsum("kq,qi,kqj->kij", wdet, Bv, Gp[..., d])
            centroid = X.mean(axis=1)
            for f, (xi_f, w_f, da, db) in enumerate(rules[kind]):
                m_f = len(w_f)
                Pown[f][loc, :m_f, :n_k] = own_face[f][None]
                xq, Jf = G.map_points(ref.kind, X, xi_f)
                t1 = np.einsum("kqdc,c->kqd", Jf, da)
                t2 = np.einsum("kqdc,c->kqd", Jf, db)
                cr = np.cross(t1, t2)
                area = np.linalg.norm(cr, axis=-1)
                nvec = cr / area[..., None]
                sign = np.sign(np.einsum("kqd,kqd->k", xq - centroid[:, None, :], nvec))
                nn[f][loc, :m_f] = nvec * sign[:, None, None]
                wJ[f][loc, :m_f] = w_f[None, :] * area * (nbr_all[ids, f] != -3)[:, None]
                nb = nbr_all[ids, f]
                for nkind, nref in enumerate(refs):
                    inner = np.nonzero((nb >= 0) & (kinds_all[np.maximum(nb, 0)] == nkind))[0]
                    if len(inner) == 0:
                        continue
                    Xn = _vertices(mesh, nkind, nb[inner])
                    Xrep = np.repeat(Xn, m_f, axis=0)
                    xi_n = G.inverse_map(nref.kind, Xrep, xq[inner].reshape(-1, 3))
                    vals, _ = nref.eval(xi_n[:, 0], xi_n[:, 1], xi_n[:, 2])
                    Pnbr[f][loc[inner], :m_f, :nref.Np] = vals.reshape(len(inner), m_f, nref.Np)
    nbr = nbr_all[elems]
    Zm = Z_all[elems][:, None] * np.ones((1, NFACE))
    Zp = np.where(nbr >= 0, Z_all[np.maximum(nbr, 0)], Zm)
    if mesh.flux == "upwind":
        tau_p = 2.0 / (Zm + Zp)
        tau_u = (Zm + Zp) / 2.0
    elif mesh.flux == "central":
        tau_p = np.zeros_like(Zm)
        tau_u = np.zeros_like(Zm)
    else:
        raise ValueError(mesh.flux)
    ops = Operators(N=N, elems=elems, M=M, Minv=Minv, S=Sd, Pown=Pown, wJ=wJ, n=nn, nbr=nbr,
                    Pnbr=Pnbr, tau_p=tau_p, tau_u=tau_u, kappa=kappa_all[elems], rho=mesh.rho[elems],
                    bc=mesh.bc)
    ops.extra["mortars"] = build_mortars(mesh, N, refs, elems)
    return ops


# ---------------------------------------------------------------------------
# Right-hand side
# ---------------------------------------------------------------------------


def face_traces(ops: Operators, U: np.ndarray, f: int):
    """Own and neighbour traces (p-, u-, p+, u+) at the quadrature points of face f.

    U: (..., K_all, 4, Np) full state; traces are for ops.elems.
    """
    Uk = U[..., ops.elems, :, :]
    P = ops.Pown[f]
    pm = np.einsum("kqj,...kj->...kq", P, Uk[..., 0, :])
    um = np.einsum("kqj,...kdj->...kdq", P, Uk[..., 1:4, :])
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
    for f in range(NFACE):
        pm, um, pp, up = face_traces(ops, U, f)
        n = ops.n[f]
        jp = pp - pm
        jun = np.einsum("...kdq,kqd->...kq", up - um, n)
        Fp = 0.5 * (ops.tau_p[:, f, None] * jp - jun)
        Fu = 0.5 * (ops.tau_u[:, f, None] * jun - jp)
        P = ops.Pown[f]
        surf[..., 0, :] += np.einsum("kqj,...kq->...kj", P, ops.wJ[f] * Fp)
        for d in range(3):
            surf[..., d + 1, :] += np.einsum("kqj,...kq->...kj", P, ops.wJ[f] * n[..., d] * Fu)
    _add_mortars(ops, U, surf)
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
    for f in range(NFACE):
        pm, um, pp, up = face_traces(ops, U, f)
        n = ops.n[f]
        jp = pp - pm
        jun = np.einsum("kdq,kqd->kq", up - um, n)
        integrand = ops.tau_p[:, f, None] * jp ** 2 + ops.tau_u[:, f, None] * jun ** 2
        # boundary faces: the mirror states give [p] = -2 p- (Dirichlet) or
        # [u_n] = -2 u_n- (rigid), so -tau (.)^2 is again -1/4 of the jump form
        total += float(np.sum(-0.25 * ops.wJ[f] * integrand))
    # faces on a common refinement are visited once: -1/2 of the jump form
    for reg in ops.extra.get("mortars") or []:
        jp, jun = _mortar_fluxes(reg, U)
        total += float(np.sum(-0.5 * reg["wJ"] * (reg["tau_p"] * jp ** 2 + reg["tau_u"] * jun ** 2)))
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
    """Physical node coordinates (K, Np, 3); padding entries are zero."""
    refs = references(N, mesh)
    Np = max(r.Np for r in refs)
    out = np.zeros((mesh.K, Np, 3))
    kinds = mesh.kinds()
    for kind, ref in enumerate(refs):
        ids = np.nonzero(kinds == kind)[0]
        if len(ids) == 0:
            continue
        xi = np.stack([ref.r, ref.s, ref.t], 1)
        x, _ = G.map_points(ref.kind, _vertices(mesh, kind, ids), xi)
        out[ids, :ref.Np] = x
    return out


def _inside(kind: int, xi: np.ndarray, tol: float) -> np.ndarray:
    r, s, t = xi[:, 0], xi[:, 1], xi[:, 2]
    if kind == 0:
        return (r >= -1 - tol) & (s >= -1 - tol) & (r + s <= tol) & (np.abs(t) <= 1 + tol)
    return (r >= -1 - tol) & (s >= -1 - tol) & (t >= -1 - tol) & (r + s + t <= -1 + tol)


def locate(mesh: Mesh, x: np.ndarray, tol: float = 1e-12):
    """Lowest-index element containing point x and its reference coordinates."""
    x = np.asarray(x, float)
    kinds = mesh.kinds()
    best = None
    for kind in range(2 if mesh.nt else 1):
        ids = np.nonzero(kinds == kind)[0]
        X = _vertices(mesh, kind, ids)
        # only elements whose bounding box holds the point can contain it
        pad = 1e-9 * (np.abs(X).max() + 1.0)
        cand = np.nonzero(np.all((X.min(axis=1) - pad <= x) & (x <= X.max(axis=1) + pad), axis=1))[0]
        if len(cand) == 0:
            continue
        xi = G.inverse_map(["wedge", "tet"][kind], X[cand], np.repeat(x[None, :], len(cand), axis=0))
        hits = np.nonzero(_inside(kind, xi, tol))[0]
        if len(hits) and (best is None or ids[cand[hits[0]]] < best[0]):
            best = (int(ids[cand[hits[0]]]), xi[hits[0]])
    if best is None:
        raise ValueError("point outside the mesh")
    return best


def point_basis(N: int, xi: np.ndarray, mesh: Mesh = None, elem: int = 0) -> np.ndarray:
    """Lagrange basis of the element's kind at one reference point (Np_max,)."""
    refs = references(N, mesh)
    kind = 0 if mesh is None else int(mesh.kinds()[elem])
    ref = refs[kind]
    v, _ = ref.eval(np.array([xi[0]]), np.array([xi[1]]), np.array([xi[2]]))
    out = np.zeros(max(r.Np for r in refs))
    out[:ref.Np] = v[0]
    return out


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
    lvec = point_basis(N, xi, mesh, k)
    vec = ops.kappa[0] * (ops.Minv[0] @ lvec)
    return PointSource(k, vec, f0, t0, amp)


def make_receivers(mesh: Mesh, N: int, xr: np.ndarray):
    """(elements, basis rows) sampling p at receiver points."""
    elems, rows = [], []
    for x in np.atleast_2d(xr):
        k, xi = locate(mesh, x)
        elems.append(k)
        rows.append(point_basis(N, xi, mesh, k))
    return np.array(elems), np.array(rows)


# ---------------------------------------------------------------------------
# Time step (reading of "trace and Markov inequalities", Sec. 6)
# ---------------------------------------------------------------------------


def stable_dt(mesh: Mesh, N: int, cfl: float) -> float:
    """dt = cfl / max_k [ c_k (N+1)(N+3)/3 max_f max J_f / min J ].

    The paper takes the step from trace and Markov inequality constants
    without printing the formula (Sec. 6); this reading uses the 3D trace
    constant (N+1)(N+3)/3 and the face-to-volume Jacobian ratio.  J and J_f
    are linear on vertically mapped wedges (constant on tetrahedra), so their
    extremes are taken over the reference vertices.
    """
    refs = references(N, mesh)
    kinds = mesh.kinds()
    ratio = np.zeros(mesh.K)
    for kind, ref in enumerate(refs):
        ids = np.nonzero(kinds == kind)[0]
        if len(ids) == 0:
            continue
        X = _vertices(mesh, kind, ids)
        _, Jm = G.map_points(ref.kind, X, ref.ref_verts)
        Jmin = np.linalg.det(Jm).min(axis=1)
        Jfmax = np.zeros(len(ids))
        for f, (_, _, da, db) in enumerate(ref.face_rules()):
            _, Jf = G.map_points(ref.kind, X, ref.ref_verts[list(ref.face_verts[f])])
            t1 = np.einsum("kqdc,c->kqd", Jf, da)
            t2 = np.einsum("kqdc,c->kqd", Jf, db)
            Jfmax = np.maximum(Jfmax, np.linalg.norm(np.cross(t1, t2), axis=-1).max(axis=1))
        ratio[ids] = Jfmax / Jmin
    rate = mesh.c * ((N + 1) * (N + 3) / 3.0) * ratio
    return cfl / float(rate.max())
