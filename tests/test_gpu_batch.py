"""Batched launch of independent problems (through the C ABI): the fields
after batch steps equal those of each problem stepped alone (the same stage
arithmetic), for meshes of different orders, sizes, materials, sources and
time steps; one problem of every order also against the FP64 oracle."""
import sys

import numpy as np
import pytest

from oracle import dg, lsrk
from paper_1607_03399_amd import inputs
from paper_1607_03399_amd import wdg
from parity import TOL, check

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _problem(N, nx, layers, seed, bits, src):
    m = inputs.layered_config(nx, layers, 0.3, seed=seed)
    s = wdg.Solver(N, bits, device=0)
    s.set_mesh(m.verts, m.wedges)
    s.set_material(m.c, m.rho)
    s.set_boundary("rigid" if seed % 2 else "dirichlet")
    s.set_flux("upwind" if seed % 3 else "central")
    s.add_ricker_source(src, 8.0, 0.05, 1.0)
    x = s.node_coords()
    U = np.zeros((s.K, 4, s.NPmax))
    U[:, 0] = inputs.gaussian_pulse(x, centre=src, width=0.2)
    s.set_fields(U)
    return m, s, U, s.stable_dt(0.5) * (0.8 + 0.05 * seed)


SPECS = [(2, 3, 2, 1, [0.4, 0.5, 0.5]), (3, 4, 3, 2, [0.5, 0.3, 0.6]), (4, 2, 3, 3, [0.6, 0.6, 0.4]),
         (5, 2, 2, 4, [0.3, 0.4, 0.5]), (3, 5, 2, 5, [0.5, 0.5, 0.5]), (2, 7, 3, 6, [0.7, 0.2, 0.3])]


@pytest.mark.parametrize("bits", [32, 64])
@pytest.mark.parametrize("autotune,concurrent", [(True, True), (False, True), (True, False)])
def test_batch_equals_single_problem_steps(bits, autotune, concurrent):
    batch = wdg.Batch(bits, device=0)
    batch.set_concurrent(concurrent)
    probs = []
    for (N, nx, layers, seed, src) in SPECS:
        m, s, U, dt = _problem(N, nx, layers, seed, bits, src)
        batch.add(s, dt)
        probs.append((N, nx, layers, seed, src, s, U, dt))
    batch.prepare(autotune=autotune)
    for N in sorted({p[0] for p in probs}):
        _say("batch config N", N, batch.config(N), batch.trials(N))
        if autotune:
            # the single-problem kernel's family: the node-lane kernel (orders
            # 4 and 5 in FP32) at four block sizes, else the level-lane one at
            # two register budgets
            tr = batch.trials(N)
            node = N >= 4 and bits == 32
            assert len(tr) == (4 if node else 2) and {t[0] for t in tr} == {"node" if node else "level"}
            e, w, us = batch.config(N)
            best = min(tr, key=lambda t: t[3])
            assert (e, w) == best[1:3] and us == best[3]
        else:
            assert batch.trials(N) == []
    batch.step(7)
    batch.step(5)  # a second call continues from the state the first left
    for (N, nx, layers, seed, src, s, U, dt) in probs:
        got = s.get_fields()
        assert abs(s.time - 12 * dt) <= 1e-12 * 12 * dt
        assert s.time == (0.0 + 7 * dt) + 5 * dt
        m, r, U2, dt2 = _problem(N, nx, layers, seed, bits, src)
        assert dt2 == dt
        r.step(7, dt)
        r.step(5, dt)
        ref = r.get_fields()
        r.close()
        _say("problem", N, nx, layers, "max abs diff", float(np.abs(got - ref).max()))
        assert np.array_equal(got, ref)
    batch.close()
    for p in probs:
        p[5].close()


ORACLE_SPECS = [(2, 2, 2, 7, [0.4, 0.5, 0.5]), (3, 3, 2, 8, [0.5, 0.5, 0.5]), (4, 2, 3, 9, [0.6, 0.4, 0.5]),
                (5, 2, 2, 10, [0.5, 0.6, 0.4])]


@pytest.mark.parametrize("bits", [64, 32])
def test_batch_matches_oracle(bits):
    """One problem of each order N = 2..5 in one batch (autotuned), each
    against the FP64 oracle after 20 steps, element by element."""
    batch = wdg.Batch(bits, device=0)
    probs = []
    for (N, nx, layers, seed, src) in ORACLE_SPECS:
        m, s, U, dt = _problem(N, nx, layers, seed, bits, src)
        batch.add(s, dt)
        probs.append((N, seed, src, m, s, U, dt))
    batch.prepare()
    batch.step(20)
    for (N, seed, src, m, s, U, dt) in probs:
        got = s.get_fields()
        om = dg.Mesh(m.verts, m.wedges, m.c, m.rho, "rigid" if seed % 2 else "dirichlet",
                     "upwind" if seed % 3 else "central")
        ops = dg.build_operators(om, N)
        source = dg.make_point_source(om, N, src, 8.0, 0.05, 1.0)

        def f(t, V):
            out = dg.rhs(ops, V)
            out[source.elem, 0] += source.value(t) * source.vec
            return out

        ref, _ = lsrk.integrate(f, U[:, :, :ops.M.shape[1]], dt, 20)
        err, emax = check(got[:, :, :ref.shape[2]], ref, TOL[bits], f"batch N={N} {bits}")
        _say("batch vs oracle N", N, bits, "rel err", err, "worst element", emax)
    batch.close()
    for p in probs:
        p[4].close()


def test_batch_rejects_hybrid_and_late_adds():
    batch = wdg.Batch(64, device=0)
    v, w, t, c, rho = inputs.split_columns(inputs.layered_config(2, 2, 0.3, seed=4), [1])
    h = wdg.Solver(2, 64, device=0)
    h.set_mesh(v, w, t)
    h.set_material(c, rho)
    h.set_fields(np.zeros((h.K, 4, h.NPmax)))
    with pytest.raises(wdg.WdgError) as e:
        batch.add(h, 1e-3)
    assert e.value.name == "WDG_ERR_UNSUPPORTED"
    m, s, U, dt = _problem(2, 2, 2, 1, 64, [0.5, 0.5, 0.5])
    batch.add(s, dt)
    batch.prepare(autotune=False)
    m2, s2, U2, dt2 = _problem(2, 2, 2, 2, 64, [0.5, 0.5, 0.5])
    with pytest.raises(wdg.WdgError) as e:
        batch.add(s2, dt2)
    assert e.value.name == "WDG_ERR_STATE"
    batch.close()
    for q in (h, s, s2):
        q.close()
