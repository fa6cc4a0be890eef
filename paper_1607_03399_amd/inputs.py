"""Seeded synthetic inputs: layered wedge meshes, materials, initial states.

This module is shared by the tests, the benchmark and the oracle-side test
code.  It holds no arithmetic of the DG method itself: it only produces
vertex coordinates, connectivity, per-element material values and point
evaluations of closed-form initial data.

Meshes follow the layered construction of Sec. 5 of the paper: a surface
triangulation of a rectangle is extruded into layers whose interfaces are
given surfaces z_k(x, y); every wedge has its bottom triangle (v1, v2, v3,
counter-clockwise seen from above) on interface k and its top triangle
(v4, v5, v6) directly above on interface k+1, so every wedge is vertically
mapped.  Squares of the base grid are split along the (i,j)->(i+1,j+1)
diagonal.  Elements are numbered column by column (element = column *
layers + layer) with columns in Morton (Z-curve) order of their base
squares, which keeps face neighbours close in memory.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class WedgeMesh:
    verts: np.ndarray      # (nv, 3) float64
    wedges: np.ndarray     # (nw, 6) int64
    c: np.ndarray          # (nw,) wave speed
    rho: np.ndarray        # (nw,) density
    layers: int
    name: str = ""

    @property
    def K(self) -> int:
        return len(self.wedges)


def _morton_key(i: np.ndarray, j: np.ndarray) -> np.ndarray:
    key = np.zeros_like(i, dtype=np.int64)
    for b in range(16):
        key |= ((i >> b) & 1) << (2 * b)
        key |= ((j >> b) & 1) << (2 * b + 1)
    return key


def layered_mesh(nx: int, ny: int, layers: int, zfun, x0=0.0, x1=1.0, y0=0.0, y1=1.0,
                 xy_jitter: float = 0.0, seed: int = 0, order: str = "morton") -> tuple:
    """Vertices and wedges of an extruded, layered mesh.

    zfun(k, x, y) gives the height of interface k = 0..layers at base vertex
    (x, y).  ``xy_jitter`` (fraction of the cell size) moves interior base
    vertices horizontally, which keeps every wedge vertically mapped.
    Returns verts (nv,3), wedges (nw,6).
    """
    xs = np.linspace(x0, x1, nx + 1)
    ys = np.linspace(y0, y1, ny + 1)
    X, Y = np.meshgrid(xs, ys, indexing="ij")  # (nx+1, ny+1)
    if xy_jitter > 0:
        rng = np.random.default_rng(seed + 7919)
        dx = (x1 - x0) / nx
        dy = (y1 - y0) / ny
        jx = rng.uniform(-1, 1, X.shape) * xy_jitter * dx
        jy = rng.uniform(-1, 1, Y.shape) * xy_jitter * dy
        interior = np.zeros(X.shape, bool)
        interior[1:-1, 1:-1] = True
        X = X + np.where(interior, jx, 0.0)
        Y = Y + np.where(interior, jy, 0.0)
    nvl = (nx + 1) * (ny + 1)
    verts = np.zeros(((layers + 1) * nvl, 3))
    for k in range(layers + 1):
        Z = np.asarray(zfun(k, X, Y), dtype=np.float64) * np.ones_like(X)
        sl = slice(k * nvl, (k + 1) * nvl)
        verts[sl, 0] = X.ravel()
        verts[sl, 1] = Y.ravel()
        verts[sl, 2] = Z.ravel()

    def vid(i, j):
        return i * (ny + 1) + j

    I, J = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    I = I.ravel()
    J = J.ravel()
    if order == "morton":
        perm = np.argsort(_morton_key(I, J), kind="stable")
    else:
        perm = np.arange(len(I))
    I = I[perm]
    J = J[perm]
    a = vid(I, J)
    b = vid(I + 1, J)
    c = vid(I + 1, J + 1)
    d = vid(I, J + 1)
    tris = np.empty((2 * len(I), 3), dtype=np.int64)
    tris[0::2] = np.stack([a, b, c], 1)
    tris[1::2] = np.stack([a, c, d], 1)
    nt = len(tris)
    wedges = np.empty((nt * layers, 6), dtype=np.int64)
    for l in range(layers):
        wedges[l::layers, 0:3] = tris + l * nvl
        wedges[l::layers, 3:6] = tris + (l + 1) * nvl
    return verts, wedges


# ---------------------------------------------------------------------------
# Named configurations
# ---------------------------------------------------------------------------


def cfg1_mesh() -> WedgeMesh:
    """Unit cube, 4x4 base (32 triangles) x 4 layers = 128 wedges.

    Interior interfaces z_k = k/4 + 0.05 sin(2 pi x) sin(2 pi y), k = 1..3;
    the walls z = 0 and z = 1 stay flat.  c = rho = 1.
    """
    L = 4

    def z(k, x, y):
        if k in (0, L):
            return np.full_like(x, k / L)
        return k / L + 0.05 * np.sin(2 * np.pi * x) * np.sin(2 * np.pi * y)

    v, w = layered_mesh(4, 4, L, z)
    K = len(w)
    return WedgeMesh(v, w, np.ones(K), np.ones(K), L, "cfg1")


def smooth_interfaces(layers: int, amplitude: float, seed: int = 0):
    """Random smooth interfaces z_k = k/L + amplitude * dz * g_k(x, y).

    g_k = sum_{m,n=1..3} a cos(2 pi m x + phi) cos(2 pi n y + psi), a ~ N(0,1),
    phases ~ U[0, 2 pi), normalised so that max |g_k| over the base vertices
    is 1; k = 1..L-1, walls flat.  Returns zfun for ``layered_mesh``.
    """
    rng = np.random.default_rng(seed)
    coef = []
    for _ in range(1, layers):
        a = rng.standard_normal((3, 3))
        phi = rng.uniform(0.0, 2 * np.pi, (3, 3))
        psi = rng.uniform(0.0, 2 * np.pi, (3, 3))
        coef.append((a, phi, psi))
    dz = 1.0 / layers

    def g(k, x, y):
        a, phi, psi = coef[k - 1]
        out = np.zeros_like(x)
        for m in range(3):
            for n in range(3):
                out += a[m, n] * np.cos(2 * np.pi * (m + 1) * x + phi[m, n]) * np.cos(2 * np.pi * (n + 1) * y + psi[m, n])
        return out

    def z(k, x, y):
        if k in (0, layers):
            return np.full_like(x, k / layers)
        gk = g(k, x, y)
        return k / layers + amplitude * dz * gk / np.abs(gk).max()

    return z


def banded_material(layers: int):
    """Per-layer c in {2.5, 1.5, 1.0} (bottom third, middle third, top) and
    rho = 2 in the lower half, 1 above.  Returns (c[l], rho[l])."""
    l = np.arange(layers)
    c = np.where(l < layers // 3, 2.5, np.where(l < (2 * layers) // 3, 1.5, 1.0))
    rho = np.where(l < layers / 2, 2.0, 1.0)
    return c, rho


def layered_config(nx: int, layers: int, amplitude: float = 0.3, seed: int = 0, name: str = "") -> WedgeMesh:
    """nx x nx base on the unit square, ``layers`` layers with random smooth
    interfaces and banded per-layer material."""
    v, w = layered_mesh(nx, nx, layers, smooth_interfaces(layers, amplitude, seed))
    cl, rl = banded_material(layers)
    lay = np.arange(len(w)) % layers
    return WedgeMesh(v, w, cl[lay], rl[lay], layers, name)


def cfg2_mesh() -> WedgeMesh:
    """64x64 base (8192 triangles) x 32 layers = 262144 wedges, N = 3."""
    return layered_config(64, 32, 0.3, 0, "cfg2")


def cfg5_mesh() -> WedgeMesh:
    """128x128 base x 16 layers = 524288 wedges, N = 3 (forward solve)."""
    return layered_config(128, 16, 0.3, 0, "cfg5")


def adjoint_problem(mesh: WedgeMesh, nrec: int = 16, seed: int = 0, amplitude: float = 0.1, width: float = 0.1):
    """Inputs of the receiver-misfit gradient workload on ``mesh`` (a window of
    a few hundredths of a second at the time steps of a 128 x 128 x 16 mesh):
    a Ricker source at the centre (f0 = 60, t0 = 0.02, so that it fires inside
    the window), ``nrec`` seeded receivers 0.01 to 0.04 from it, and the wave
    speed c (1 + amplitude exp(-|x_e - x_a|^2 / width^2)) per element (x_e:
    element centroid, x_a: a seeded centre within 0.03 of the source) that
    synthesises the data.  Returns (receivers (nrec, 3), source
    (xyz, f0, t0, amp), c_true)."""
    rng = np.random.default_rng(seed)
    xs = np.array([0.5, 0.5, 0.5])
    d = rng.standard_normal((nrec, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rec = xs + d * rng.uniform(0.01, 0.04, (nrec, 1))
    xa = xs + rng.uniform(-0.03, 0.03, 3)
    cent = mesh.verts[mesh.wedges].mean(axis=1)
    bump = np.exp(-np.sum((cent - xa) ** 2, axis=1) / width ** 2)
    return rec, (xs, 60.0, 0.02, 1.0), mesh.c * (1.0 + amplitude * bump)


def batch_problems(n: int = 48, seed: int = 0, kmin: int = 1000, kmax: int = 60000):
    """Independent problems of the batched workload: sizes log-uniform in
    [kmin, kmax] wedges (nx x nx base, 4 to 16 layers, random smooth
    interfaces), orders drawn from {2, 3, 4, 5}, seeded per-layer wave speed
    in [1, 3] and density in [1, 2.5], and a Ricker source position inside.
    Returns a list of (N, WedgeMesh, source xyz)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        target = float(np.exp(rng.uniform(np.log(kmin), np.log(kmax))))
        layers = int(rng.integers(4, 17))
        nx = max(2, int(round(np.sqrt(target / (2 * layers)))))
        N = int(rng.choice([2, 3, 4, 5]))
        v, w = layered_mesh(nx, nx, layers, smooth_interfaces(layers, 0.3, seed * 1000 + i))
        cl = rng.uniform(1.0, 3.0, layers)
        rl = rng.uniform(1.0, 2.5, layers)
        lay = np.arange(len(w)) % layers
        mesh = WedgeMesh(v, w, cl[lay], rl[lay], layers, f"batch{i}")
        out.append((N, mesh, rng.uniform(0.2, 0.8, 3)))
    return out


def cfg3_hybrid_mesh(tet_layers: int = 5):
    """32x32 base (2048 triangles) x 24 layers with random smooth interfaces;
    the lowest ``tet_layers`` layers split into tetrahedra (3 per prism):
    38912 wedges + 30720 tetrahedra at the default, N = 4.  Returns
    (verts, wedges, tets, c, rho) as ``split_layers``."""
    return split_layers(layered_config(32, 24, 0.3, 0, "cfg3"), tet_layers)


def cube_mesh(n: int, lo: float = -1.0, hi: float = 1.0, z_jitter: float = 0.0, xy_jitter: float = 0.0,
              seed: int = 0) -> WedgeMesh:
    """[lo,hi]^3 with n x n base squares and n layers (mesh size h = (hi-lo)/n).

    ``z_jitter`` moves interior interface heights randomly by up to that
    fraction of the layer thickness (vertically perturbed wedges); the walls
    stay flat.
    """
    rng = np.random.default_rng(seed)
    dz = (hi - lo) / n
    jit = rng.uniform(-1, 1, (n + 1, n + 1, n + 1)) * z_jitter * dz

    def z(k, x, y):
        base = lo + k * dz
        if k in (0, n) or z_jitter == 0:
            return np.full_like(x, base)
        return base + jit[k, : x.shape[0], : x.shape[1]]

    v, w = layered_mesh(n, n, n, z, lo, hi, lo, hi, xy_jitter=xy_jitter, seed=seed)
    K = len(w)
    return WedgeMesh(v, w, np.ones(K), np.ones(K), n, f"cube{n}")


def random_vertical_wedges(K: int, seed: int = 0):
    """K independent random vertically mapped wedges (vertex arrays (K, 6, 3))."""
    rng = np.random.default_rng(seed)
    out = np.zeros((K, 6, 3))
    for k in range(K):
        while True:
            p = rng.uniform(-1, 1, (3, 2))
            area = 0.5 * ((p[1, 0] - p[0, 0]) * (p[2, 1] - p[0, 1]) - (p[2, 0] - p[0, 0]) * (p[1, 1] - p[0, 1]))
            if abs(area) > 0.2:
                break
        if area < 0:
            p = p[[0, 2, 1]]
        zb = rng.uniform(-0.5, 0.0, 3)
        zt = rng.uniform(0.4, 1.0, 3)
        out[k, :3, :2] = p
        out[k, 3:, :2] = p
        out[k, :3, 2] = zb
        out[k, 3:, 2] = zt
    return out


def gaussian_pulse(x: np.ndarray, centre=(0.5, 0.5, 0.5), width: float = 0.1) -> np.ndarray:
    """exp(-|x - centre|^2 / width^2) at points x (..., 3)."""
    d = x - np.asarray(centre)
    return np.exp(-np.sum(d * d, axis=-1) / width ** 2)


def standing_mode_dirichlet(x: np.ndarray, t: float):
    """Exact mode on [-1,1]^3 with p = 0 on the walls, rho = c = 1 (Sec. 6.1):
    p = cos(pi x/2) cos(pi y/2) cos(pi z/2) cos(sqrt(3) pi t / 2)."""
    w = np.sqrt(3.0) * np.pi / 2.0
    cx, cy, cz = (np.cos(np.pi * x[..., d] / 2) for d in range(3))
    sx, sy, sz = (np.sin(np.pi * x[..., d] / 2) for d in range(3))
    p = cx * cy * cz * np.cos(w * t)
    k = np.sin(w * t) / np.sqrt(3.0)
    return np.stack([p, sx * cy * cz * k, cx * sy * cz * k, cx * cy * sz * k], axis=-2)


def standing_mode_rigid(x: np.ndarray, t: float):
    """Exact mode on [0,1]^3 with rigid walls, rho = c = 1:
    p = cos(pi x) cos(pi y) cos(pi z) cos(sqrt(3) pi t)."""
    w = np.sqrt(3.0) * np.pi
    cx, cy, cz = (np.cos(np.pi * x[..., d]) for d in range(3))
    sx, sy, sz = (np.sin(np.pi * x[..., d]) for d in range(3))
    p = cx * cy * cz * np.cos(w * t)
    k = np.sin(w * t) / np.sqrt(3.0)
    return np.stack([p, sx * cy * cz * k, cx * sy * cz * k, cx * cy * sz * k], axis=-2)


# ---------------------------------------------------------------------------
# Hybrid wedge / tetrahedron meshes
# ---------------------------------------------------------------------------


def prism_to_tets(prism, verts):
    """Split a prism (a, b, c bottom; d, e, f above them) into 3 tetrahedra.

    Each quadrilateral face is cut along the diagonal through its lowest
    global vertex id, so neighbouring split prisms share their diagonals
    (the standard conforming rule for prisms).  The prism is first relabelled
    so that its lowest vertex id is a; the diagonal of the face opposite a then
    decides the split.  Tetrahedra are returned positively oriented.
    """
    a, b, c, d, e, f = (int(v) for v in prism)
    # rotations (and the bottom/top flip) that keep the prism structure
    labels = [(a, b, c, d, e, f), (b, c, a, e, f, d), (c, a, b, f, d, e),
              (d, f, e, a, c, b), (e, d, f, b, a, c), (f, e, d, c, b, a)]
    a, b, c, d, e, f = min(labels, key=lambda L: L[0])
    if min(b, f) < min(c, e):
        tets = [(a, b, c, f), (a, b, f, e), (a, e, f, d)]
    else:
        tets = [(a, b, c, e), (a, e, c, f), (a, e, f, d)]
    out = []
    for t in tets:
        p = verts[list(t)]
        vol = np.dot(np.cross(p[1] - p[0], p[2] - p[0]), p[3] - p[0])
        out.append(t if vol > 0 else (t[0], t[2], t[1], t[3]))
    return out


def split_layers(mesh: WedgeMesh, tet_layers: int):
    """Hybrid mesh: the wedges of the lowest ``tet_layers`` layers become 3
    tetrahedra each; wedges and tetrahedra meet only across triangular faces.
    Returns (verts, wedges, tets, c, rho) with material per element (wedges
    first, then tetrahedra in the order of the split wedges)."""
    lay = np.arange(mesh.K) % mesh.layers
    split = lay < tet_layers
    tets, tc, tr = [], [], []
    for k in np.nonzero(split)[0]:
        for t in prism_to_tets(mesh.wedges[k], mesh.verts):
            tets.append(t)
            tc.append(mesh.c[k])
            tr.append(mesh.rho[k])
    keep = ~split
    wedges = mesh.wedges[keep]
    c = np.concatenate([mesh.c[keep], np.array(tc)])
    rho = np.concatenate([mesh.rho[keep], np.array(tr)])
    return mesh.verts, wedges, np.array(tets, dtype=np.int64).reshape(-1, 4), c, rho


def split_columns(mesh: WedgeMesh, columns):
    """Hybrid mesh: every wedge of the given base columns (element =
    column x layers + layer) becomes 3 tetrahedra.  The quadrilateral faces
    between a split and an unsplit column are then covered by two triangular
    tetrahedron faces each (nonconforming: a wedge quadrilateral against two
    triangles).  Returns (verts, wedges, tets, c, rho) as ``split_layers``."""
    col = np.arange(mesh.K) // mesh.layers
    split = np.isin(col, np.asarray(columns))
    tets, tc, tr = [], [], []
    for k in np.nonzero(split)[0]:
        for t in prism_to_tets(mesh.wedges[k], mesh.verts):
            tets.append(t)
            tc.append(mesh.c[k])
            tr.append(mesh.rho[k])
    keep = ~split
    wedges = mesh.wedges[keep]
    c = np.concatenate([mesh.c[keep], np.array(tc)])
    rho = np.concatenate([mesh.rho[keep], np.array(tr)])
    return mesh.verts, wedges, np.array(tets, dtype=np.int64).reshape(-1, 4), c, rho


def cfg3_columns_mesh(fraction: float = 0.2, seed: int = 0):
    """32x32 base (2048 triangles) x 24 layers with random smooth interfaces and
    banded material; a seeded random ``fraction`` of the columns split into
    tetrahedra (410 columns at 20 %: 39312 wedges + 29520 tetrahedra), N = 4."""
    m = layered_config(32, 24, 0.3, seed, "cfg3")
    ncol = m.K // m.layers
    cols = np.random.default_rng(seed).choice(ncol, int(round(fraction * ncol)), replace=False)
    return split_columns(m, cols)
