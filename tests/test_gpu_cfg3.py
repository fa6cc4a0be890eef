"""The column-split hybrid configuration at full size (32 x 32 base x 24
layers, 20 % of the columns split into tetrahedra: 39 312 wedges + 29 520
tetrahedra, N = 4; Sec. 5 hybrid meshes, Sec. 3.1 tetrahedra sharing the
triangle face nodes), through the C ABI, against the FP64 oracle on sampled
elements, element by element.

The sample holds wedges and tetrahedra on both sides of mortar faces (a wedge
quadrilateral against two tetrahedron triangles), tetrahedra that the
persistent tetrahedron kernel reaches in its second and third pass over the
chunks (2048 blocks of 7 tetrahedra at N = 4: local index >= 14 336 and
>= 28 672), and the first and last elements of each kind.  The right-hand
side is also evaluated with the kernel capped at 64 blocks (about 66 chunks
per block) and must not change by a single bit."""
import sys

import numpy as np
import pytest

from oracle import dg
from paper_1607_03399_amd import inputs
from paper_1607_03399_amd import wdg
from parity import TOL, check

pytestmark = pytest.mark.gpu

N = 4
EPB_TET = 256 // 35  # tetrahedra per chunk of the tetrahedron kernel at N = 4


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
    chunk_start = 2048 * EPB_TET
    assert nt > 2 * chunk_start
    tets = [nw + chunk_start + rng.integers(0, chunk_start, 8), nw + 2 * chunk_start + rng.integers(0, nt - 2 * chunk_start, 8),
            nw + rng.integers(0, chunk_start, 8)]
    fixed = [0, nw - 1, nw, nw + chunk_start, nw + 2 * chunk_start, om.K - 1]
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
    _say("cfg3 library", bits)
    s = wdg.Solver(N, bits, device=0)
    s.set_mesh(v, w, t)
    s.set_material(c, rho)
    got = s.eval_rhs(U[:, :, :s.NPmax])
    s.set_tet_blocks(64)
    got64 = s.eval_rhs(U[:, :, :s.NPmax])
    s.close()
    assert np.array_equal(got, got64)
    sample = _sample(om, rng)
    _say("cfg3 oracle on", len(sample), "elements")
    ops = dg.build_operators(om, N, elems=sample)
    ref = dg.rhs(ops, U)[:, :, :got.shape[2]]
    err, emax = check(got[sample], ref, TOL[bits], f"cfg3 sampled rhs {bits}")
    _say("   sampled rel err", err, "worst element", emax)
