"""The allocation-free right-hand side (wdg_eval_rhs_noalloc) against
wdg_eval_rhs through the C ABI: two calls in a row on one GPU, the second on a
smaller mesh (the library's fixed staging array keeps the first call's
contents), in both precisions, a hybrid mesh with mortar faces among them.
Both entry points run the same stage kernels on the same converted input, so
the results must agree bit for bit; a mesh whose staging exceeds the array is
rejected before anything reaches the GPU."""
import sys

import numpy as np
import pytest

from paper_1607_03399_amd import inputs
from paper_1607_03399_amd import wdg

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _solver(N, bits, mesh_fn):
    v, w, t, c, rho = mesh_fn()
    s = wdg.Solver(N, bits, device=0)
    s.set_mesh(v, w, t)
    s.set_material(c, rho)
    s.set_boundary("rigid")
    s.set_flux("upwind")
    return s


def _hybrid():
    return inputs.split_columns(inputs.layered_config(6, 4, 0.3, seed=3), [2, 7, 11, 20, 33])


def _small():
    m = inputs.layered_config(3, 3, 0.3, seed=5)
    return m.verts, m.wedges, np.zeros((0, 4), np.int64), m.c, m.rho


def _state(s, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((s.K, 4, s.NPmax)) * s.mask[:, None, :]


@pytest.mark.parametrize("bits", [32, 64])
def test_noalloc_rhs_equals_eval_rhs_twice_second_smaller(bits):
    N = 3
    s1 = _solver(N, bits, _hybrid)
    s2 = _solver(N, bits, _small)
    assert s2.K < s1.K
    s1.add_ricker_source([0.4, 0.45, 0.5], 10.0, 0.05, 1.0)
    for s, seed, t in ((s1, 1, 0.03), (s2, 2, 0.0)):
        _say("noalloc", bits, "K", s.K)
        U = _state(s, seed)
        got = s.eval_rhs_noalloc(U, t)
        ref = s.eval_rhs(U, t)
        assert np.array_equal(got, ref), float(np.abs(got - ref).max())
        assert np.abs(ref).max() > 0
    s1.close()
    s2.close()


def test_noalloc_rejects_oversized_mesh():
    nmax = wdg.eval_rhs_noalloc_max_nodes(64)
    assert nmax == ((32 << 20) - 512) // 96
    m = inputs.layered_config(20, 12, 0.3, seed=1)  # 9 600 wedges x 40 nodes > nmax in FP64
    s = wdg.Solver(3, 64, device=0)
    s.set_mesh(m.verts, m.wedges)
    s.set_material(m.c, m.rho)
    assert s.K * s.Np > nmax
    with pytest.raises(wdg.WdgError) as e:
        s.eval_rhs_noalloc(np.zeros((s.K, 4, s.NPmax)))
    assert e.value.code == -1
    s.close()
