"""Discrete adjoint of the time-stepped solve (through the C ABI and the
torch.autograd.Function) against the FP64 oracle's exact discrete derivative
(complex step of the whole solve) and against central finite differences of
the device's own forward solve."""
import sys

import numpy as np
import pytest

from oracle import adjoint, dg
from paper_1607_03399_amd import inputs
from paper_1607_03399_amd import wdg

pytestmark = pytest.mark.gpu

# FP64: both sides compute the same derivative of the same discrete map, so
# they differ by rounding of long sums only.  FP32: the forward and adjoint
# states carry single-precision rounding over every stage.
TOL = {64: 1e-12, 32: 1e-5}


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


def _problem(nx=2, layers=2, seed=4, N=2, width=0.25):
    m = inputs.layered_config(nx, layers, 0.3, seed=seed)
    x = dg.node_coords(dg.Mesh(m.verts, m.wedges, m.c, m.rho, "rigid", "upwind"), N)
    U0 = np.zeros((m.K, 4, x.shape[1]))
    U0[:, 0] = inputs.gaussian_pulse(x, width=width)
    src = ([0.3, 0.6, 0.4], 4.0, 0.15, 1.0)
    rec = np.array([[0.7, 0.3, 0.8], [0.2, 0.2, 0.3], [0.55, 0.45, 0.5]])
    return m, N, U0, src, rec


def _solver(m, N, bits, bc, flux, src, rec, c=None, rho=None):
    s = wdg.Solver(N, bits, device=0)
    s.set_mesh(m.verts, m.wedges)
    s.set_material(m.c if c is None else c, m.rho if rho is None else rho)
    s.set_boundary(bc)
    s.set_flux(flux)
    s.add_ricker_source(*src)
    s.set_receivers(rec)
    return s


@pytest.mark.parametrize("bits", [64, 32])
@pytest.mark.parametrize("flux,bc", [("upwind", "rigid"), ("central", "rigid"), ("upwind", "dirichlet")])
def test_gradient_matches_oracle(flux, bc, bits):
    m, N, U0, src, rec = _problem()
    om = dg.Mesh(m.verts, m.wedges, m.c, m.rho, bc, flux)
    dt = dg.stable_dt(om, N, 0.5)
    nsteps = 12
    base = adjoint.solve_traces(om, N, U0, dt, nsteps, src, rec)
    data = 0.9 * base + 0.01
    elems = np.random.default_rng(7).choice(m.K, 8, replace=False)
    _say("adjoint vs oracle", flux, bc, bits, "elements", elems)
    J, gc_ref, gr_ref = adjoint.gradient_complex_step(om, N, U0, dt, nsteps, src, rec, data, elems=elems)
    s = _solver(m, N, bits, bc, flux, src, rec)
    s.set_fields(U0)
    gc, gr = s.adjoint_gradient(nsteps, dt, base - data, checkpoint_every=5)
    s.close()
    ec, er = _rel(gc[elems], gc_ref), _rel(gr[elems], gr_ref)
    _say("   rel err c", ec, "rho", er)
    assert ec <= TOL[bits] and er <= TOL[bits]


@pytest.mark.parametrize("bits", [64, 32])
@pytest.mark.parametrize("N", [4, 5])
def test_gradient_matches_oracle_high_order(N, bits):
    """Orders 4 and 5 (in FP32 the forward recomputation runs the node-lane
    kernel, writing each stage's residual out of place): the self-contained
    gradient, and the recorded forward that fills the last segment itself,
    against the oracle's complex-step derivative, and bitwise equal."""
    m, _, U0, src, rec = _problem(N=N)
    om = dg.Mesh(m.verts, m.wedges, m.c, m.rho, "rigid", "upwind")
    dt = dg.stable_dt(om, N, 0.5)
    nsteps, every = 7, 3
    base = adjoint.solve_traces(om, N, U0, dt, nsteps, src, rec)
    data = 0.9 * base + 0.01
    elems = np.random.default_rng(7).choice(m.K, 4, replace=False)
    _say("adjoint vs oracle N", N, "bits", bits, "elements", elems)
    J, gc_ref, gr_ref = adjoint.gradient_complex_step(om, N, U0, dt, nsteps, src, rec, data, elems=elems)
    s = _solver(m, N, bits, "rigid", "upwind", src, rec)
    s.set_fields(U0)
    gc, gr = s.adjoint_gradient(nsteps, dt, base - data, checkpoint_every=every)
    s.adjoint_record(every, nsteps)
    s.step(nsteps, dt)
    g2 = s.adjoint_gradient_recorded(base - data)
    s.close()
    ec, er = _rel(gc[elems], gc_ref), _rel(gr[elems], gr_ref)
    _say("   rel err c", ec, "rho", er)
    assert ec <= TOL[bits] and er <= TOL[bits]
    assert np.array_equal(g2[0], gc) and np.array_equal(g2[1], gr)


def test_checkpoint_interval_does_not_change_the_gradient():
    m, N, U0, src, rec = _problem()
    s = _solver(m, N, 64, "rigid", "upwind", src, rec)
    s.set_fields(U0)
    dt = s.stable_dt(0.5)
    w = np.random.default_rng(3).standard_normal((13, len(rec)))
    out = [s.adjoint_gradient(13, dt, w, checkpoint_every=ce) for ce in (1, 4, 13, 50)]
    U_after = s.get_fields()
    s.close()
    for gc, gr in out[1:]:
        assert np.array_equal(gc, out[0][0]) and np.array_equal(gr, out[0][1])
    assert np.array_equal(U_after[:, :, :U0.shape[2]], U0)  # the state is unchanged


def test_recorded_forward_and_memory_modes_give_the_same_gradient():
    """Checkpoints kept by the forward steps (recording) and both memory modes
    of the reverse sweep (segment stage store / per-step recomputation) give
    bitwise the same gradient as the self-contained call."""
    m, N, U0, src, rec = _problem()
    s = _solver(m, N, 64, "rigid", "upwind", src, rec)
    s.set_fields(U0)
    dt = s.stable_dt(0.5)
    w = np.random.default_rng(9).standard_normal((11, len(rec)))
    ref = s.adjoint_gradient(11, dt, w, checkpoint_every=4)
    s.set_adjoint_memory_limit(1)  # forces per-step recomputation
    low = s.adjoint_gradient(11, dt, w, checkpoint_every=4)
    s.set_adjoint_memory_limit(0)
    s.adjoint_record(4, 11)
    s.step(6, dt)
    s.step(5, dt)
    U_end = s.get_fields()
    assert s.recorded_steps() == 11
    rec_g = s.adjoint_gradient_recorded(w)
    assert np.array_equal(s.get_fields(), U_end)
    for a in (low, rec_g):
        assert np.array_equal(a[0], ref[0]) and np.array_equal(a[1], ref[1])
    # the recording ends with a step of another size, and with set_fields
    s.step(1, 0.5 * dt)
    with pytest.raises(wdg.WdgError) as e:
        s.adjoint_gradient_recorded(np.zeros((12, len(rec))))
    assert e.value.name == "WDG_ERR_STATE"
    s.set_fields(U0)
    s.time = 0.0
    s.adjoint_record(4, 8)
    s.step(8, dt)
    assert s.recorded_steps() == 8
    s.step(1, dt)  # beyond max_steps
    assert s.recorded_steps() == 0
    # a source added after the recording ends it (the recorded forward had none)
    s.set_fields(U0)
    s.time = 0.0
    s.adjoint_record(4, 8)
    s.step(3, dt)
    assert s.recorded_steps() == 3
    s.add_ricker_source([0.5, 0.5, 0.5], 4.0, 0.1, 1.0)
    assert s.recorded_steps() == 0
    s.close()


@pytest.mark.parametrize("bits", [64, 32])
@pytest.mark.parametrize("nsteps,every,split", [(11, 4, (6, 5)), (12, 4, (5, 7)), (5, 1, (2, 3)), (11, 13, (11,))])
def test_recorded_forward_keeps_the_last_segment(bits, nsteps, every, split):
    """With the reverse sweep's store kept from an earlier gradient call, the
    recorded forward writes its segments' stage data into it and the sweep
    skips recomputing the last segment: the final state, the receiver traces
    and the gradient are bitwise those of the plain forward and of the
    self-contained call; a second gradient of the same recording, and one
    after further recorded steps, recompute everything and agree too."""
    m, N, U0, src, rec = _problem()
    s = _solver(m, N, bits, "rigid", "upwind", src, rec)
    s.set_fields(U0)
    dt = s.stable_dt(0.5)
    rng = np.random.default_rng(17)
    w = rng.standard_normal((nsteps, len(rec)))
    w2 = rng.standard_normal((nsteps + 3, len(rec)))
    _say(f"bits={bits} nsteps={nsteps} every={every} split={split}")
    ref = s.adjoint_gradient(nsteps, dt, w, checkpoint_every=every)  # keeps the store
    ref2 = s.adjoint_gradient(nsteps + 3, dt, w2, checkpoint_every=every)
    s.step(nsteps, dt)
    U_plain, tr_plain = s.get_fields(), s.read_receivers()
    s.set_fields(U0)
    s.time = 0.0
    s.adjoint_record(every, nsteps + 3)
    for k in split:
        s.step(k, dt)
    assert s.recorded_steps() == nsteps
    assert np.array_equal(s.get_fields(), U_plain)
    assert np.array_equal(s.read_receivers(), tr_plain)
    for _ in range(2):
        g = s.adjoint_gradient_recorded(w)
        assert np.array_equal(g[0], ref[0]) and np.array_equal(g[1], ref[1])
    s.step(3, dt)
    g = s.adjoint_gradient_recorded(w2)
    assert np.array_equal(g[0], ref2[0]) and np.array_equal(g[1], ref2[1])
    s.close()


def test_gradient_matches_central_differences():
    """Device-only check on a larger mesh (N=3): the adjoint gradient of the
    misfit against central differences of the device's own forward solve."""
    m, N, U0, src, rec = _problem(nx=4, layers=4, seed=11, N=3, width=0.2)
    nsteps = 30

    def misfit(c, rho, data=None):
        s = _solver(m, N, 64, "rigid", "upwind", src, rec, c, rho)
        s.set_fields(U0)
        dt = s.stable_dt(0.5)
        s.step(nsteps, dt)
        tr = s.read_receivers()
        s.close()
        return tr, dt

    base, dt = misfit(m.c, m.rho)
    data = 1.05 * base - 0.002
    s = _solver(m, N, 64, "rigid", "upwind", src, rec)
    s.set_fields(U0)
    gc, gr = s.adjoint_gradient(nsteps, dt, base - data)
    s.close()
    J = lambda tr: 0.5 * float(np.sum((tr - data) ** 2))
    J0 = J(base)
    elems = np.random.default_rng(5).choice(m.K, 8, replace=False)
    for k in elems:
        for which, g in (("c", gc[k]), ("rho", gr[k])):
            vals = []
            for sgn in (1, -1):
                c, rho = m.c.copy(), m.rho.copy()
                arr = c if which == "c" else rho
                eps = 1e-4 * arr[k]
                arr[k] += sgn * eps
                s = _solver(m, N, 64, "rigid", "upwind", src, rec, c, rho)
                s.set_fields(U0)
                s.step(nsteps, dt)
                vals.append(J(s.read_receivers()))
                s.close()
            fd = (vals[0] - vals[1]) / (2 * eps)
            _say("fd", k, which, fd, g)
            # truncation O(eps^2) relative; rounding of J (1e-14 J) over 2 eps
            assert abs(fd - g) <= 1e-6 * abs(g) + 1e-14 * J0 / eps


def test_autograd_function():
    torch = pytest.importorskip("torch")
    from paper_1607_03399_amd.autograd import receiver_traces

    m, N, U0, src, rec = _problem()
    s = _solver(m, N, 64, "rigid", "upwind", src, rec)
    dt = s.stable_dt(0.5)
    nsteps = 10
    om = dg.Mesh(m.verts, m.wedges, m.c, m.rho, "rigid", "upwind")
    data = 0.8 * adjoint.solve_traces(om, N, U0, dt, nsteps, src, rec)
    c = torch.tensor(m.c, dtype=torch.float64, requires_grad=True)
    rho = torch.tensor(m.rho, dtype=torch.float64, requires_grad=True)
    tr = receiver_traces(s, c, rho, U0, nsteps, dt, checkpoint_every=3)
    loss = 0.5 * ((tr - torch.as_tensor(data)) ** 2).sum()
    loss.backward()
    elems = [0, 6, 13]
    J, gc_ref, gr_ref = adjoint.gradient_complex_step(om, N, U0, dt, nsteps, src, rec, data, elems=elems)
    s.close()
    assert abs(loss.item() - J) <= 1e-12 * J
    assert _rel(c.grad.numpy()[elems], gc_ref) <= TOL[64]
    assert _rel(rho.grad.numpy()[elems], gr_ref) <= TOL[64]


def test_unsupported_configurations():
    m, N, U0, src, rec = _problem()
    s = _solver(m, N, 64, "rigid", "upwind", src, rec)
    s.set_fields(U0)
    dt = s.stable_dt(0.5)
    with pytest.raises(ValueError):
        s.adjoint_gradient(4, dt, np.zeros((3, len(rec))))
    s.set_mass("lumped")
    with pytest.raises(wdg.WdgError) as e:
        s.adjoint_gradient(4, dt, np.zeros((4, len(rec))))
    assert e.value.code == -11
    s.close()
    v, w, t, c, rho = inputs.split_columns(inputs.layered_config(2, 2, 0.3, seed=4), [1])
    s = wdg.Solver(2, 64, device=0)
    s.set_mesh(v, w, t)
    s.set_material(c, rho)
    s.set_receivers(rec)
    s.set_fields(np.zeros((s.K, 4, s.NPmax)))
    with pytest.raises(wdg.WdgError) as e:
        s.adjoint_gradient(4, dt, np.zeros((4, len(rec))))
    assert e.value.code == -11
    s.close()


def test_cfg5_gradient_central_differences_and_fp32():
    """The receiver-misfit gradient at full size (128 x 128 x 16 = 524 288
    wedges, N = 3; 16 receivers, data from a 10 % Gaussian anomaly in c; 100
    steps, checkpoints every 50), on 8 seeded elements within 0.05 of the
    source: the FP64 adjoint against central differences of the FP64 device
    forward (one context, material reset between solves), and the FP32
    adjoint against the FP64 adjoint with the same misfit weights."""
    m = inputs.cfg5_mesh()
    rec, src, c_true = inputs.adjoint_problem(m)
    nsteps, every = 100, 50
    cent = m.verts[m.wedges].mean(axis=1)
    near = np.nonzero(np.linalg.norm(cent - np.asarray(src[0]), axis=1) < 0.05)[0]
    elems = np.sort(np.random.default_rng(12).choice(near, 8, replace=False))

    def solver(bits):
        s = wdg.Solver(3, bits, device=0)
        s.set_mesh(m.verts, m.wedges)
        s.set_boundary("rigid")
        s.set_flux("upwind")
        s.add_ricker_source(*src)
        s.set_receivers(rec)
        s.set_material(m.c, m.rho)
        return s

    s = solver(64)
    dt = s.stable_dt(0.5)
    U0 = np.zeros((s.K, 4, s.NPmax))
    U0[:, 0] = inputs.gaussian_pulse(s.node_coords(), width=0.2)

    def traces(c, rho):
        s.set_material(c, rho)
        s.set_fields(U0)
        s.time = 0.0
        s.step(nsteps, dt)
        return s.read_receivers()

    _say("cfg5 data")
    data = traces(c_true, m.rho)
    base = traces(m.c, m.rho)
    w = base - data
    J = lambda tr: 0.5 * float(np.sum((tr - data) ** 2))
    J0 = J(base)
    assert J0 > 0
    s.set_material(m.c, m.rho)
    s.set_fields(U0)
    s.time = 0.0
    gc, gr = s.adjoint_gradient(nsteps, dt, w, every)
    _say("cfg5 J", J0, "elements", elems)
    for k in elems:
        for which, g in (("c", gc[k]), ("rho", gr[k])):
            vals = []
            for sgn in (1, -1):
                c, rho = m.c.copy(), m.rho.copy()
                arr = c if which == "c" else rho
                eps = 1e-3 * arr[k]
                arr[k] += sgn * eps
                vals.append(J(traces(c, rho)))
            fd = (vals[0] - vals[1]) / (2 * eps)
            _say("   fd", k, which, fd, "adjoint", g, "rel", abs(fd - g) / abs(g))
            # truncation (eps / value)^2 ~ 1e-6 relative; rounding of the FP64
            # forward (~1e-15 J) over 2 eps
            assert abs(fd - g) <= 1e-5 * abs(g) + 1e-13 * J0 / eps
    s.close()
    s32 = solver(32)
    s32.set_fields(U0)
    gc32, gr32 = s32.adjoint_gradient(nsteps, dt, w, every)
    s32.close()
    ec, er = _rel(gc32[elems], gc[elems]), _rel(gr32[elems], gr[elems])
    eall = max(_rel(gc32, gc), _rel(gr32, gr))
    # largest error of one element against the largest gradient entry
    emax = max(np.abs(gc32 - gc).max() / np.abs(gc).max(), np.abs(gr32 - gr).max() / np.abs(gr).max())
    _say("cfg5 FP32 vs FP64 adjoint: sampled c", ec, "rho", er, "all elements", eall, "worst element", emax)
    # Over all elements the FP32 gradient meets the FP32 bound (about 2e-7
    # measured), and so does every element against the gradient's scale
    # (about 2e-7).  The 8 elements next to the source carry gradients three
    # orders below the largest ones, where the rounding of the FP32 forward and
    # adjoint fields (not the accumulation: FP64 accumulators gave the same
    # per-element errors to three digits) leaves about 6e-5 relative: bound 2e-4.
    assert eall <= TOL[32] and emax <= TOL[32]
    assert ec <= 2e-4 and er <= 2e-4
