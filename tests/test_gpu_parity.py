"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances (relative Euclidean L2 over all four fields' nodal values):
FP64 1e-12, FP32 1e-5, for single right-hand sides and after 100 steps.
"""
import os
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


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _solver(m, N, bits, bc="rigid", flux="upwind", wedge="auto"):
    s = wdg.Solver(N, bits, device=0)
    s.set_mesh(m.verts, m.wedges)
    s.set_material(m.c, m.rho)
    s.set_boundary(bc)
    s.set_flux(flux)
    s.set_wedge_kernel(wedge)
    return s


def _wedge_kernels(N, bits):
    """Wedge stage kernels of an order: the level-lane kernel runs at every
    order, the node-lane kernel at orders 4 and 5 in FP32."""
    return ("level", "node") if N >= 4 and bits == 32 else ("auto",)


def _omesh(m, bc="rigid", flux="upwind"):
    return dg.Mesh(m.verts, m.wedges, m.c, m.rho, bc, flux)


def _rotated(m, seed=0):
    """Same mesh with every wedge's vertex list rotated by a random amount
    (v1,v2,v3 -> v2,v3,v1 etc., tops alike): neighbouring wedges then see
    each other's faces through nontrivial vertex permutations."""
    rng = np.random.default_rng(seed)
    w = m.wedges.copy()
    for k in range(len(w)):
        r = rng.integers(3)
        b = np.roll(w[k, :3], -r)
        t = np.roll(w[k, 3:], -r)
        w[k] = np.concatenate([b, t])
    return inputs.WedgeMesh(m.verts, w, m.c, m.rho, m.layers, m.name + "-rot")


def test_element_data_matches_oracle():
    """Setup kernel (FP64 on the device): geometric factors and L^{tri,k}."""
    m = inputs.layered_config(3, 3, 0.3, seed=1)
    # orders 4 and 5 store L^{tri,k} itself, column by column
    for N, bits, tol in ((2, 64, 1e-12), (3, 32, 2e-6), (4, 32, 2e-6), (5, 64, 1e-11)):
        _say("element data", N, bits)
        s = _solver(m, N, bits)
        geo, lift = s.element_data()
        om = _omesh(m)
        ops = dg.build_operators(om, N)
        NT = (N + 1) * (N + 2) // 2
        from oracle import basis as OB
        W = OB.Wedge(N)
        rq, sq, wq = OB.tri_quadrature(N + 2)
        Lq, _, _ = W.tri.eval(rq, sq)
        Mhat = Lq.T @ (wq[:, None] * Lq)
        tg, wg = OB.gauss_nodes_weights(N + 2)
        l1 = OB.lagrange1d(W.tgll, tg)
        m100 = float((l1[:, 0] * wg) @ l1[:, 0])  # M^1D[0, 0]
        for k in range(m.K):
            # M^k = M^1D (x) M^{tri,k} (pinned in the oracle tests): leading block / M^1D[0,0]
            Mtk = ops.M[k][:NT, :NT] / m100
            Lref = np.linalg.solve(Mtk, Mhat)
            assert np.abs(lift[k] - Lref).max() <= tol * np.abs(Lref).max()
            # face normals and Jacobians against the oracle's face quadrature
            for f, sl in ((0, 12), (1, 16)):
                np.testing.assert_allclose(geo[k, sl], ops.wJ[f][k].sum() / 2.0, rtol=tol)
                np.testing.assert_allclose(geo[k, sl + 1:sl + 4], ops.n[f][k][0], atol=tol)
            for e in range(3):
                np.testing.assert_allclose(geo[k, 22 + 4 * e:24 + 4 * e], ops.n[2 + e][k][0][:2], atol=tol)
                area = ops.wJ[2 + e][k].sum()
                np.testing.assert_allclose(2.0 * (geo[k, 20 + 4 * e] + geo[k, 21 + 4 * e]), area, rtol=tol)
        s.close()


@pytest.mark.parametrize("bits", [64, 32])
@pytest.mark.parametrize("N", [1, 2, 3, 4, 5])
def test_rhs_parity(N, bits):
    m = inputs.layered_config(3, 3, 0.3, seed=N)  # 54 wedges, curved, banded c and rho
    for bc, flux in (("rigid", "upwind"), ("dirichlet", "central")):
        ops = dg.build_operators(_omesh(m, bc, flux), N)
        rng = np.random.default_rng(10 + N)
        U = rng.standard_normal((m.K, 4, ops.M.shape[1]))
        ref = dg.rhs(ops, U)
        for wedge in _wedge_kernels(N, bits):
            _say("rhs", N, bits, bc, flux, wedge)
            s = _solver(m, N, bits, bc, flux, wedge)
            got = s.eval_rhs(U)
            err, emax = check(got, ref, TOL[bits], f"rhs N={N} {bits} {bc} {flux} {wedge}")
            _say("   rel err", err, "worst element", emax)
            s.close()


@pytest.mark.parametrize("bits", [64, 32])
@pytest.mark.parametrize("N", [3, 4, 5])
def test_rhs_parity_permuted_vertices_and_ragged_sizes(N, bits):
    """Nontrivial face permutations; element counts that leave a ragged last
    workgroup (16 or 15 wedges per block at N = 3; 12 per block of the
    node-lane kernel at N = 4, 9 at N = 5, 4 of the level-lane kernel at
    N = 5 in FP64); a single element with only boundary faces."""
    for K_cut in (1, 7, 65, 131):
        base = _rotated(inputs.layered_config(4, 5, 0.3, seed=3), seed=K_cut)
        w = base.wedges[:K_cut]
        used = np.unique(w)
        remap = -np.ones(len(base.verts), dtype=np.int64)
        remap[used] = np.arange(len(used))
        m = inputs.WedgeMesh(base.verts[used], remap[w], base.c[:K_cut], base.rho[:K_cut], base.layers)
        _say("ragged", N, bits, K_cut)
        s = _solver(m, N, bits)
        U = np.random.default_rng(K_cut).standard_normal((m.K, 4, s.Np))
        got = s.eval_rhs(U)
        ref = dg.rhs(dg.build_operators(_omesh(m), N), U)
        check(got, ref, TOL[bits], f"ragged K={K_cut}")
        s.close()


def _run_library(m, N, bits, U0, dt, nsteps, bc="rigid", src=None, rec=None):
    s = _solver(m, N, bits, bc)
    if src is not None:
        s.add_ricker_source(*src)
    if rec is not None:
        s.set_receivers(rec)
    s.set_fields(U0)
    s.step(nsteps, dt)
    out = s.get_fields()
    traces = s.read_receivers() if rec is not None else None
    E = s.energy()
    s.close()
    return out, traces, E


def _run_oracle(m, N, U0, dt, nsteps, bc="rigid", src=None, rec=None):
    om = _omesh(m, bc)
    ops = dg.build_operators(om, N)
    source = dg.make_point_source(om, N, *src) if src is not None else None
    rel_el, rows = dg.make_receivers(om, N, np.atleast_2d(rec)) if rec is not None else (None, None)
    tr = []

    def f(t, U):
        out = dg.rhs(ops, U)
        if source is not None:
            out[source.elem, 0] += source.value(t) * source.vec
        return out

    def after(n, t, U):
        if rec is not None:
            tr.append(np.einsum("rj,rj->r", rows, U[rel_el, 0]))

    U, _ = lsrk.integrate(f, U0, dt, nsteps, after_step=after)
    return U, (np.array(tr) if rec is not None else None), dg.energy(ops, U)


def test_cfg1_100_steps_fp64():
    """cfg1 (128 wedges, N=2, FP64, rigid, Gaussian pulse, CFL 0.5) after
    100 steps, with a Ricker source and receivers as well."""
    m = inputs.cfg1_mesh()
    N = 2
    x = dg.node_coords(_omesh(m), N)
    U0 = np.zeros((m.K, 4, x.shape[1]))
    U0[:, 0] = inputs.gaussian_pulse(x)
    dt = dg.stable_dt(_omesh(m), N, 0.5)
    src = ([0.3, 0.6, 0.45], 5.0, 0.2, 1.0)
    rec = np.array([[0.5, 0.5, 0.5], [0.2, 0.7, 0.9], [0.81, 0.33, 0.12]])
    _say("cfg1 library")
    got, gtr, gE = _run_library(m, N, 64, U0, dt, 100, src=src, rec=rec)
    _say("cfg1 oracle")
    ref, rtr, rE = _run_oracle(m, N, U0, dt, 100, src=src, rec=rec)
    check(got, ref, 1e-12, "cfg1 100 steps")
    assert gtr.shape == (100, 3)
    assert np.abs(gtr - rtr).max() <= 1e-12 * np.abs(rtr).max()
    assert abs(gE - rE) <= 1e-12 * rE


def test_fp32_100_steps_n3():
    m = inputs.layered_config(6, 4, 0.3, seed=5)  # 288 wedges, banded c, rho
    N = 3
    om = _omesh(m)
    x = dg.node_coords(om, N)
    U0 = np.zeros((m.K, 4, x.shape[1]))
    U0[:, 0] = inputs.gaussian_pulse(x, width=0.2)
    U0[:, 3] = 0.5 * inputs.gaussian_pulse(x, centre=(0.4, 0.6, 0.5), width=0.25)
    dt = dg.stable_dt(om, N, 0.5)
    _say("fp32 library")
    got, _, _ = _run_library(m, N, 32, U0, dt, 100)
    _say("fp32 oracle")
    ref, _, _ = _run_oracle(m, N, U0, dt, 100)
    err, emax = check(got, ref, 1e-5, "fp32 100 steps")
    _say("   rel err", err, "worst element", emax)


@pytest.mark.parametrize("N", [4, 5])
def test_fp32_100_steps_high_order(N):
    """FP32 at orders 4 and 5 (the node-lane wedge kernel, the default there)
    after 100 steps with a Ricker source and receivers, against the FP64
    oracle: fields element by element, traces and energy at the FP32
    tolerance."""
    m = inputs.layered_config(3, 3, 0.3, seed=11)  # 54 wedges, curved, banded c and rho
    om = _omesh(m)
    x = dg.node_coords(om, N)
    U0 = np.zeros((m.K, 4, x.shape[1]))
    U0[:, 0] = inputs.gaussian_pulse(x, width=0.25)
    U0[:, 2] = 0.5 * inputs.gaussian_pulse(x, centre=(0.6, 0.4, 0.5), width=0.3)
    dt = dg.stable_dt(om, N, 0.5)
    src = ([0.4, 0.45, 0.55], 5.0, 0.2, 1.0)
    rec = np.array([[0.5, 0.5, 0.5], [0.25, 0.7, 0.8]])
    _say("fp32 high order library", N)
    got, gtr, gE = _run_library(m, N, 32, U0, dt, 100, src=src, rec=rec)
    _say("fp32 high order oracle", N)
    ref, rtr, rE = _run_oracle(m, N, U0, dt, 100, src=src, rec=rec)
    err, emax = check(got, ref, 1e-5, f"fp32 100 steps N={N}")
    _say("   rel err", err, "worst element", emax)
    assert np.abs(gtr - rtr).max() <= 1e-5 * np.abs(rtr).max()
    assert abs(gE - rE) <= 1e-5 * rE


def test_cfg2_full_size_100_steps_fp32_against_fp64():
    """cfg2 at full size (262144 wedges, N=3): 100 FP32 steps against 100 FP64
    steps of the device path (the FP64 path is held to the oracle at 1e-12 on
    the smaller meshes above), element by element at the FP32 tolerance, and
    the upwind scheme's energy does not increase over any 10 of the steps in
    either precision.  Over the whole run FP64 dissipates 4.3e-9 of the energy;
    FP32 rounding moves the energy by up to 7e-9 per 10 steps (measured alike
    with the stored inverse triangular mass and with the factored one), so the
    sign of the FP32 total is rounding: FP64 must decrease, FP32 must stay
    within twice FP32's unit roundoff of the start."""
    m = inputs.cfg2_mesh()
    N = 3
    out = {}
    for bits in (64, 32):
        _say("cfg2 100 steps", bits)
        s = _solver(m, N, bits)
        U0 = np.zeros((m.K, 4, 40))
        U0[:, 0] = inputs.gaussian_pulse(s.node_coords(), width=0.2)
        s.set_fields(U0)
        dt = s.stable_dt(0.5) if bits == 64 else out[64][1]
        E = [s.energy()]
        for _ in range(10):
            s.step(10, dt)
            E.append(s.energy())
        F = s.get_fields()
        s.close()
        assert np.all(np.isfinite(F))
        assert all(E[k + 1] <= E[k] * (1 + 1e-6) for k in range(10)), E
        if bits == 64:
            assert E[-1] < E[0]
        else:
            assert E[-1] <= E[0] * (1 + 2.0 ** -23), E
        out[bits] = (F, dt)
    err, emax = check(out[32][0], out[64][0], 1e-5, "cfg2 100 steps FP32 vs FP64")
    _say("   rel err", err, "worst element", emax)


def test_dirichlet_steps_fp64_and_energy_decay():
    m = inputs.cube_mesh(2, z_jitter=0.3, seed=2)
    N = 3
    om = _omesh(m, "dirichlet")
    x = dg.node_coords(om, N)
    U0 = inputs.standing_mode_dirichlet(x, 0.0)
    dt = dg.stable_dt(om, N, 0.5)
    got, _, gE = _run_library(m, N, 64, U0, dt, 40, bc="dirichlet")
    ref, _, rE = _run_oracle(m, N, U0, dt, 40, bc="dirichlet")
    check(got, ref, 1e-12, "dirichlet 40 steps")
    assert abs(gE - rE) <= 1e-12 * rE


def test_determinism_bitwise():
    m = inputs.layered_config(5, 4, 0.3, seed=7)
    N = 3
    U0 = np.random.default_rng(0).standard_normal((m.K, 4, 40))
    outs = []
    for _ in range(2):
        s = _solver(m, N, 32)
        s.set_fields(U0)
        s.step(10, 1e-3)
        outs.append(s.get_fields())
        s.close()
    assert np.array_equal(outs[0], outs[1])


def test_checkpoint_resume():
    m = inputs.layered_config(4, 3, 0.3, seed=8)
    N = 2
    U0 = np.random.default_rng(1).standard_normal((m.K, 4, 18))
    s = _solver(m, N, 64)
    s.set_fields(U0)
    s.step(20, 2e-3)
    full = s.get_fields()
    s.set_fields(U0)
    s.time = 0.0
    s.step(10, 2e-3)
    mid, t = s.get_fields(), s.time
    s.close()
    s2 = _solver(m, N, 64)
    s2.set_fields(mid)
    s2.time = t
    s2.step(10, 2e-3)
    assert _rel(s2.get_fields(), full) <= 1e-14
    s2.close()


def test_torch_bound_state_and_stream():
    import torch

    m = inputs.layered_config(4, 3, 0.3, seed=9)
    N = 3
    U0 = np.random.default_rng(2).standard_normal((m.K, 4, 40))
    s = _solver(m, N, 32)
    s.set_fields(U0)
    st = torch.cuda.Stream()
    s.bind_torch(stream=st)
    s.step(5, 1e-3)
    a = s.get_fields()
    s.close()
    s = _solver(m, N, 32)
    s.set_fields(U0)
    s.step(5, 1e-3)
    b = s.get_fields()
    s.close()
    assert np.array_equal(a, b)


def test_cfg2_full_size_sampled_rhs_and_energy():
    """cfg2 at full size (262144 wedges, N=3, FP32): the right-hand side of a
    random state on 48 sampled elements against the oracle, element by
    element; then 5 steps of the upwind scheme do not increase the energy."""
    m = inputs.cfg2_mesh()
    N = 3
    _say("cfg2 setup")
    s = _solver(m, N, 32)
    rng = np.random.default_rng(4)
    U = rng.standard_normal((m.K, 4, 40)).astype(np.float32).astype(np.float64)
    got = s.eval_rhs(U)
    sample = np.sort(rng.choice(m.K, 48, replace=False))
    sample[0] = 0
    sample[-1] = m.K - 1
    _say("cfg2 oracle sample")
    ops = dg.build_operators(_omesh(m), N, elems=sample)
    ref = dg.rhs(ops, U)
    err, emax = check(got[sample], ref, 1e-5, "cfg2 sampled rhs")
    _say("   sampled rel err", err, "worst element", emax)
    U0 = np.zeros_like(U)
    U0[:, 0] = inputs.gaussian_pulse(s.node_coords(), width=0.1)
    s.set_fields(U0)
    E0 = s.energy()
    dt = s.stable_dt(0.5)
    s.step(5, dt)
    E1 = s.energy()
    F = s.get_fields()
    assert np.all(np.isfinite(F))
    assert E1 <= E0 * (1 + 1e-5)
    s.close()


@pytest.mark.parametrize("N", [4, 5])
def test_node_kernel_block_shapes_bitwise(N):
    """Every elements-per-block shape of the node-lane kernel (FP32) gives
    bitwise the same right-hand side and 5-step fields on a 131-wedge mesh
    with permuted vertices (a ragged last block for every shape), and the
    default shape matches the oracle."""
    base = _rotated(inputs.layered_config(4, 5, 0.3, seed=3), seed=131)
    w = base.wedges[:131]
    used = np.unique(w)
    remap = -np.ones(len(base.verts), dtype=np.int64)
    remap[used] = np.arange(len(used))
    m = inputs.WedgeMesh(base.verts[used], remap[w], base.c[:131], base.rho[:131], base.layers)
    ops = dg.build_operators(_omesh(m), N)
    U = np.random.default_rng(40 + N).standard_normal((m.K, 4, ops.M.shape[1]))
    shapes = (8, 17, 12, 4) if N == 4 else (12, 9, 6, 3)
    outs = []
    for e in (0,) + shapes:
        _say("block shape", N, e)
        s = _solver(m, N, 32, wedge="node")
        s.set_wedge_block(e)
        r = s.eval_rhs(U)
        s.set_fields(U)
        dt = s.stable_dt(0.5)
        s.step(5, dt)
        outs.append((r, s.get_fields()))
        s.close()
    check(outs[0][0], dg.rhs(ops, U), TOL[32], f"node kernel N={N} default shape")
    for r, f in outs[1:]:
        assert np.array_equal(r, outs[0][0])
        assert np.array_equal(f, outs[0][1])
