"""Parity of the hybrid wedge/tetrahedron path (through the C ABI) with the
FP64 oracle.  Meshes: layered wedge meshes whose lowest layers are split into
conforming tetrahedra (three per prism), so that tetrahedra meet wedges at
triangular faces.  Tolerances as for wedges: relative L2 over all nodal
values, FP64 1e-12, FP32 1e-5."""
import itertools
import sys

import numpy as np
import pytest

from oracle import dg, lsrk
from paper_1607_03399_amd import inputs
from paper_1607_03399_amd import wdg
from parity import TET_KERNELS as KERNELS, TOL, check, tet_chunk

pytestmark = pytest.mark.gpu
# even permutations of four vertices keep a tetrahedron's orientation
EVEN = [p for p in itertools.permutations(range(4))
        if sum(1 for i in range(4) for j in range(i + 1, 4) if p[i] > p[j]) % 2 == 0]


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _hybrid(nx=3, layers=4, tet_layers=2, seed=1, permute=None):
    m = inputs.layered_config(nx, layers, 0.3, seed=seed)
    v, w, t, c, rho = inputs.split_layers(m, tet_layers)
    if permute is not None:
        rng = np.random.default_rng(permute)
        w = w.copy()
        for k in range(len(w)):
            r = rng.integers(3)
            w[k] = np.concatenate([np.roll(w[k, :3], -r), np.roll(w[k, 3:], -r)])
        t = np.array([t[k][list(EVEN[rng.integers(len(EVEN))])] for k in range(len(t))]).reshape(-1, 4)
    return v, w, t, c, rho


def _solver(mesh, N, bits, bc="rigid", flux="upwind", kernel="mfma"):
    v, w, t, c, rho = mesh
    s = wdg.Solver(N, bits, device=0)
    s.set_mesh(v, w, t)
    s.set_material(c, rho)
    s.set_boundary(bc)
    s.set_flux(flux)
    s.set_tet_kernel(kernel)
    return s


def _omesh(mesh, bc="rigid", flux="upwind"):
    v, w, t, c, rho = mesh
    return dg.Mesh(v, w, c, rho, bc, flux, tets=t)


def _compare_rhs(mesh, N, bits, bc, flux, seed):
    """Largest relative L2 error of the library's right-hand side of a random
    state over both tetrahedron kernels; the per-element bound is asserted
    here."""
    om = _omesh(mesh, bc, flux)
    mask = dg.node_mask(om, N)
    U = np.random.default_rng(seed).standard_normal((om.K, 4, mask.shape[1])) * mask[:, None, :]
    ref = dg.rhs(dg.build_operators(om, N), U)
    worst = 0.0
    for kernel in KERNELS:
        s = _solver(mesh, N, bits, bc, flux, kernel)
        got = s.eval_rhs(U[:, :, :s.NPmax])
        s.close()
        err = check(got, ref[:, :, :got.shape[2]], TOL[bits], f"hybrid N={N} {bits} {bc} {flux} {kernel}")[0]
        worst = max(worst, err)
    return worst


@pytest.mark.parametrize("bits", [64, 32])
@pytest.mark.parametrize("N", [1, 2, 3, 4, 5])
def test_hybrid_rhs_parity(N, bits):
    mesh = _hybrid(seed=N)
    for bc, flux in (("rigid", "upwind"), ("dirichlet", "central")):
        _say("hybrid rhs", N, bits, bc, flux)
        err = _compare_rhs(mesh, N, bits, bc, flux, 20 + N)
        _say("   rel err", err)
        assert err <= TOL[bits]


@pytest.mark.parametrize("bits", [64, 32])
def test_hybrid_rhs_parity_permuted_vertices(bits):
    """Rotated wedge vertex lists and even permutations of every tetrahedron's
    vertices: wedge/tetrahedron and tetrahedron/tetrahedron faces meet through
    all six vertex permutations."""
    for N in (2, 4):
        mesh = _hybrid(nx=4, layers=4, tet_layers=2, seed=7, permute=N)
        _say("hybrid permuted", N, bits)
        assert _compare_rhs(mesh, N, bits, "rigid", "upwind", 5) <= TOL[bits]


@pytest.mark.parametrize("bits", [64, 32])
def test_tetrahedra_only_and_ragged(bits):
    """All elements tetrahedra; and tetrahedron counts that leave ragged chunks."""
    for nx, layers, tl in ((2, 2, 2), (3, 3, 1), (5, 2, 1)):
        mesh = _hybrid(nx=nx, layers=layers, tet_layers=tl, seed=nx)
        _say("tets", nx, layers, tl, bits, len(mesh[1]), len(mesh[2]))
        for N in (1, 3):
            assert _compare_rhs(mesh, N, bits, "dirichlet", "upwind", nx + N) <= TOL[bits]


def _run(mesh, N, bits, U0, dt, nsteps, src, rec, tet_blocks=0, kernel="mfma", overlap=False):
    s = _solver(mesh, N, bits, kernel=kernel)
    s.set_tet_blocks(tet_blocks)
    s.set_overlap(overlap)
    s.add_ricker_source(*src)
    s.set_receivers(rec)
    s.set_fields(U0[:, :, :s.NPmax])
    s.step(nsteps, dt)
    out = s.get_fields()
    tr = s.read_receivers()
    E = s.energy()
    s.close()
    return out, tr, E


def _run_oracle(mesh, N, U0, dt, nsteps, src, rec):
    om = _omesh(mesh)
    ops = dg.build_operators(om, N)
    source = dg.make_point_source(om, N, *src)
    rel_el, rows = dg.make_receivers(om, N, rec)
    tr = []

    def f(t, U):
        out = dg.rhs(ops, U)
        out[source.elem, 0] += source.value(t) * source.vec
        return out

    def after(n, t, U):
        tr.append(np.einsum("rj,rj->r", rows, U[rel_el, 0]))

    U, _ = lsrk.integrate(f, U0, dt, nsteps, after_step=after)
    return U, np.array(tr), dg.energy(ops, U)


@pytest.mark.parametrize("looped,kernel", [(False, "mfma"), (True, "mfma"), (True, "valu")])
@pytest.mark.parametrize("N,bits,nsteps", [(2, 64, 100), (4, 32, 100)])
def test_hybrid_time_integration(N, bits, nsteps, looped, kernel):
    """Gaussian pulse plus a Ricker source inside the tetrahedral layer,
    receivers in both kinds of element: fields, traces and energy.  Looped:
    the tetrahedron kernel's persistent blocks are capped at a third of its
    chunks, so that every block loops over at least three chunks (next-chunk
    prefetch included) in every stage."""
    mesh = _hybrid(nx=3, layers=4, tet_layers=2, seed=3)
    om = _omesh(mesh)
    x = dg.node_coords(om, N)
    mask = dg.node_mask(om, N)
    U0 = np.zeros((om.K, 4, x.shape[1]))
    U0[:, 0] = inputs.gaussian_pulse(x, width=0.2) * mask
    dt = dg.stable_dt(om, N, 0.5)
    src = ([0.45, 0.55, 0.2], 5.0, 0.2, 1.0)
    rec = np.array([[0.5, 0.5, 0.8], [0.3, 0.6, 0.15], [0.7, 0.2, 0.3]])
    kinds = om.kinds()
    assert kinds[dg.locate(om, np.array(src[0]))[0]] == 1
    assert {int(kinds[dg.locate(om, r)[0]]) for r in rec} == {0, 1}
    _say("hybrid steps library", N, bits, kernel)
    nchunks = -(-len(mesh[2]) // tet_chunk(N, kernel))
    tet_blocks = max(1, nchunks // 3) if looped else 0
    assert not looped or nchunks >= 3 * tet_blocks
    got, gtr, gE = _run(mesh, N, bits, U0, dt, nsteps, src, rec, tet_blocks, kernel)
    _say("hybrid steps oracle", N, bits)
    ref, rtr, rE = _run_oracle(mesh, N, U0, dt, nsteps, src, rec)
    ref = ref[:, :, :got.shape[2]]
    tol = TOL[bits]
    err, emax = check(got, ref, tol, f"hybrid steps N={N} {bits} blocks={tet_blocks} {kernel}")
    _say("   rel err", err, "worst element", emax)
    assert np.abs(gtr - rtr).max() <= tol * np.abs(rtr).max()
    assert abs(gE - rE) <= tol * rE


@pytest.mark.parametrize("columns", [False, True])
@pytest.mark.parametrize("N,bits", [(2, 64), (4, 32)])
def test_overlap_matches_serial_order(N, bits, columns):
    """The tetrahedron kernel on the context's second stream beside the wedge
    kernel ends 30 steps in bitwise the same fields, receiver traces and energy
    as all kernels in order on one stream (the default); on a conforming
    hybrid mesh and on one with mortar faces (split columns)."""
    if columns:
        m = inputs.layered_config(3, 3, 0.3, seed=1)
        mesh = inputs.split_columns(m, [4, 9])
    else:
        mesh = _hybrid(nx=3, layers=4, tet_layers=2, seed=3)
    om = _omesh(mesh)
    x = dg.node_coords(om, N)
    mask = dg.node_mask(om, N)
    U0 = np.zeros((om.K, 4, x.shape[1]))
    U0[:, 0] = inputs.gaussian_pulse(x, width=0.2) * mask
    dt = dg.stable_dt(om, N, 0.5)
    src = ([0.45, 0.55, 0.2], 5.0, 0.2, 1.0)
    rec = np.array([[0.5, 0.5, 0.8], [0.3, 0.6, 0.15]])
    _say("overlap A/B", N, bits, "columns" if columns else "layers")
    a = _run(mesh, N, bits, U0, dt, 30, src, rec, overlap=True)
    b = _run(mesh, N, bits, U0, dt, 30, src, rec, overlap=False)
    assert np.array_equal(a[0], b[0])
    assert np.array_equal(a[1], b[1])
    assert a[2] == b[2]
