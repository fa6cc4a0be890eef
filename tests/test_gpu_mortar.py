"""Parity of the nonconforming hybrid path (through the C ABI) with the FP64
oracle: columns of prisms split into tetrahedra, so that wedge
quadrilaterals meet two tetrahedron triangles and are coupled on that common
refinement (mortar kernel).  Tolerances: relative L2 over all nodal values,
FP64 1e-12, FP32 1e-5."""
import itertools
import sys

import numpy as np
import pytest

from oracle import dg, lsrk
from paper_1607_03399_amd import inputs
from paper_1607_03399_amd import wdg
from parity import TET_KERNELS as KERNELS, TOL, check, tet_chunk

pytestmark = pytest.mark.gpu
EVEN = [p for p in itertools.permutations(range(4))
        if sum(1 for i in range(4) for j in range(i + 1, 4) if p[i] > p[j]) % 2 == 0]


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _columns(nx=3, layers=3, cols=(4, 9), seed=1, permute=None):
    m = inputs.layered_config(nx, layers, 0.3, seed=seed)
    v, w, t, c, rho = inputs.split_columns(m, list(cols))
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
    """Largest relative L2 error over both tetrahedron kernels (matrix cores,
    vector units); the per-element bound is asserted here."""
    om = _omesh(mesh, bc, flux)
    mask = dg.node_mask(om, N)
    U = np.random.default_rng(seed).standard_normal((om.K, 4, mask.shape[1])) * mask[:, None, :]
    ref = dg.rhs(dg.build_operators(om, N), U)
    worst = 0.0
    for kernel in KERNELS:
        s = _solver(mesh, N, bits, bc, flux, kernel)
        got = s.eval_rhs(U[:, :, :s.NPmax])
        s.close()
        err = check(got, ref[:, :, :got.shape[2]], TOL[bits], f"mortar N={N} {bits} {bc} {flux} {kernel}")[0]
        worst = max(worst, err)
    return worst


@pytest.mark.parametrize("bits", [64, 32])
@pytest.mark.parametrize("N", [1, 2, 3, 4, 5])
def test_mortar_rhs_parity(N, bits):
    mesh = _columns(seed=N)
    for bc, flux in (("rigid", "upwind"), ("dirichlet", "central")):
        _say("mortar rhs", N, bits, bc, flux)
        err = _compare_rhs(mesh, N, bits, bc, flux, 40 + N)
        _say("   rel err", err)
        assert err <= TOL[bits]


@pytest.mark.parametrize("bits", [64, 32])
def test_mortar_rhs_parity_permuted_and_ragged(bits):
    """Rotated wedge vertex lists, permuted tetrahedra, several split columns
    (some next to each other, some on the walls) and element counts that leave
    ragged chunks."""
    for N, nx, layers, cols in ((2, 4, 4, (3, 10, 11, 17, 30)), (4, 5, 3, (0, 7, 8, 21, 33, 49))):
        mesh = _columns(nx=nx, layers=layers, cols=cols, seed=nx, permute=N)
        _say("mortar permuted", N, bits, len(mesh[1]), len(mesh[2]))
        assert _compare_rhs(mesh, N, bits, "rigid", "upwind", 9) <= TOL[bits]


@pytest.mark.parametrize("looped,kernel", [(False, "mfma"), (True, "mfma"), (True, "valu")])
@pytest.mark.parametrize("N,bits", [(2, 64), (4, 32)])
def test_mortar_time_integration(N, bits, looped, kernel):
    """Gaussian pulse and a Ricker source inside a split column, receivers in
    wedges and tetrahedra: fields, traces and energy after 100 steps.  Seven
    of the 18 columns are split (63 tetrahedra).  Looped: the tetrahedron
    kernel's persistent blocks are capped at a third of its chunks, so that
    every block loops over at least three chunks in every stage."""
    mesh = _columns(nx=3, layers=3, cols=(1, 4, 6, 9, 11, 14, 16), seed=3)
    om = _omesh(mesh)
    x = dg.node_coords(om, N)
    mask = dg.node_mask(om, N)
    U0 = np.zeros((om.K, 4, x.shape[1]))
    U0[:, 0] = inputs.gaussian_pulse(x, width=0.2) * mask
    dt = dg.stable_dt(om, N, 0.5)
    kinds = om.kinds()
    # a point in the first tetrahedron's interior, and receivers of both kinds
    xs = dg.node_coords(om, 1)[om.nw, :4].mean(axis=0)
    assert kinds[dg.locate(om, xs)[0]] == 1
    rec = np.array([[0.5, 0.5, 0.8], xs + [0.01, 0.0, 0.02], [0.8, 0.15, 0.3]])
    src = (xs, 5.0, 0.2, 1.0)
    s = _solver(mesh, N, bits, kernel=kernel)
    nchunks = -(-s.Kt // tet_chunk(N, kernel))
    tet_blocks = max(1, nchunks // 3) if looped else 0
    assert not looped or nchunks >= 3 * tet_blocks
    s.set_tet_blocks(tet_blocks)
    s.add_ricker_source(*src)
    s.set_receivers(rec)
    s.set_fields(U0[:, :, :s.NPmax])
    s.step(100, dt)
    got = s.get_fields()
    gtr = s.read_receivers()
    gE = s.energy()
    s.close()
    ops = dg.build_operators(om, N)
    source = dg.make_point_source(om, N, *src)
    rel_el, rows = dg.make_receivers(om, N, rec)
    tr = []

    def f(t, U):
        out = dg.rhs(ops, U)
        out[source.elem, 0] += source.value(t) * source.vec
        return out

    ref, _ = lsrk.integrate(f, U0, dt, 100,
                            after_step=lambda n, t, U: tr.append(np.einsum("rj,rj->r", rows, U[rel_el, 0])))
    rE = dg.energy(ops, ref)
    tol = TOL[bits]
    err, emax = check(got, ref[:, :, :got.shape[2]], tol, f"mortar steps N={N} {bits} blocks={tet_blocks} {kernel}")
    _say("mortar steps", N, bits, kernel, "rel err", err, "worst element", emax)
    rtr = np.array(tr)
    assert np.abs(gtr - rtr).max() <= tol * np.abs(rtr).max()
    assert abs(gE - rE) <= tol * rE
