"""The column-split hybrid configuration at full size (32 x 32 base x 24
layers, 20 % of the columns split into tetrahedra: 39 312 wedges + 29 520
tetrahedra, N = 4; Sec. 5 hybrid meshes, Sec. 3.1 tetrahedra sharing the
triangle face nodes), through the C ABI, against the FP64 oracle on sampled
elements, element by element, with both tetrahedron kernels (operator
products on the matrix cores, and per-node dot products).

The sample holds wedges and tetrahedra on both sides of mortar faces (a wedge
quadrilateral against two tetrahedron triangles), tetrahedra spread over the
whole range (the persistent tetrahedron kernels reach the later ones in their
second and later passes over the chunks), and the first and last elements of
each kind.  The right-hand side is also evaluated with the kernel capped at
64 blocks (tens of chunks per block) and must not change by a single bit."""
import sys

import numpy as np
import pytest

from oracle import dg
from paper_1607_03399_amd import inputs
from paper_1607_03399_amd import wdg
from parity import TET_KERNELS, TOL, check, tet_chunk

pytestmark = pytest.mark.gpu

N = 4


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _sample(om, rng):
    nw, nt = om.nw, om.nt
    nbr, _ = dg.face_connectivity(om)
    mort = dg.mortar_faces(om, nbr)
    assert len(mort) > 1000
    pick = rng.choice(len(mort), 12, replace=False)
    mort_el = []
    for i in pick:
        k, f, diag, tets = mort[i]
        mort_el += [k, tets[0][0], tets[1][0]]
    # three tetrahedra from each eighth of the range (all passes of the persistent blocks)
    edges = np.linspace(0, nt, 9).astype(np.int64)
    tets = [nw + rng.integers(edges[b], edges[b + 1], 3) for b in range(8)]
    fixed = [0, nw - 1, nw, nw + nt // 2, om.K - 1]
    return np.unique(np.concatenate([mort_el, rng.integers(0, nw, 12), *tets, fixed]).astype(np.int64))


@pytest.mark.parametrize("bits", [32, 64])
def test_cfg3_full_size_sampled_rhs(bits):
    v, w, t, c, rho = inputs.cfg3_columns_mesh()
    om = dg.Mesh(v, w, c, rho, "rigid", "upwind", tets=t)
    assert (om.nw, om.nt) == (39312, 29520)
    rng = np.random.default_rng(31 + bits)
    mask = dg.node_mask(om, N)
    U = rng.standard_normal((om.K, 4, mask.shape[1])) * mask[:, None, :]
    if bits == 32:
        U = U.astype(np.float32).astype(np.float64)
    s = wdg.Solver(N, bits, device=0)
    s.set_mesh(v, w, t)
    s.set_material(c, rho)
    got = {}
    for kernel in TET_KERNELS:
        _say("cfg3 library", bits, kernel)
        assert -(-om.nt // tet_chunk(N, kernel)) >= 64 * 20
        s.set_tet_kernel(kernel)
        s.set_tet_blocks(0)
        got[kernel] = s.eval_rhs(U[:, :, :s.NPmax])
        s.set_tet_blocks(64)
        assert np.array_equal(got[kernel], s.eval_rhs(U[:, :, :s.NPmax]))
    s.close()
    sample = _sample(om, rng)
    _say("cfg3 oracle on", len(sample), "elements")
    ops = dg.build_operators(om, N, elems=sample)
    full = dg.rhs(ops, U)
    for kernel in TET_KERNELS:
        ref = full[:, :, :got[kernel].shape[2]]
        err, emax = check(got[kernel][sample], ref, TOL[bits], f"cfg3 sampled rhs {bits} {kernel}")
        _say("   sampled rel err", kernel, err, "worst element", emax)
