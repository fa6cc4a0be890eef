#!/usr/bin/env python3
"""Throughput of the wedge DG solver on one MI355X.

Workload (default): 64 x 64 base squares (8192 triangles) x 32 layers =
262144 vertically mapped wedges with random smooth interfaces, N = 3
(40 nodes per wedge), FP32, banded per-layer wave speed and density, rigid
walls, upwind flux, Ricker point source at the centre, initial Gaussian
pressure pulse (width 0.2), 200 steps of the five-stage low-storage
Runge-Kutta scheme.  Inputs are synthetic (seeded).

Prints one JSON line: DG node-updates per second per Runge-Kutta stage
(elements x nodes x 5 x steps / wall time); the HBM-roofline fraction of the
dominant stage kernel (its algorithmic bytes per launch, as the hot-path
scope table counts them, over its average duration from HIP events on the
solver stream) beside a measured device-copy rate; further forward legs
(the column-split hybrid mesh with wedge, tetrahedron and mortar kernels,
524288 wedges, orders 4 and 5, FP64); the adjoint leg (receiver-misfit
gradient on 524288 wedges: gradient time over forward time); the batched
leg (48 independent problems of mixed orders and sizes: one batch against
the problems one by one); and the FP64 CPU oracle timed on bounded samples,
one process and all cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0


def tet_stage_bytes(N: int, bits: int, reads_res: bool) -> int:
    """Algorithmic HBM bytes of one stage for one tetrahedron: state, residual
    as for wedges (4 fields x Np_tet), geometry and material record (32
    values), connectivity (8 int32); reference operators are read once per
    block and counted as cache hits."""
    NP = (N + 1) * (N + 2) * (N + 3) // 6
    ts = bits // 8
    return 4 * NP * ts * (3 + int(reads_res)) + 32 * ts + 8 * 4


def stage_bytes(N: int, bits: int, reads_res: bool) -> int:
    """Algorithmic HBM bytes of one stage for one wedge.

    State U read and U' written, residual written (and read after the first
    stage): 4 fields x Np values each; per-element geometry and material
    record (40 values), triangular operator (N <= 3: none, the stage factors
    M^{tri,k} from the record's vertex weights; N >= 4: L^{tri,k}, Np_tri^2
    values padded to a multiple of 4) and connectivity (8 int32).  Neighbour
    traces are counted as cache hits.  At N = 3 in FP32 this is 2752 B (2112 B
    in the first stage).
    """
    NT = (N + 1) * (N + 2) // 2
    NP = NT * (N + 1)
    ts = bits // 8
    LS = 0 if N <= 3 else (NT * NT + 3) // 4 * 4
    state = 4 * NP * ts
    return state * (3 + int(reads_res)) + 40 * ts + LS * ts + 8 * 4


def table_stage_bytes(N: int, bits: int) -> int:
    """Algorithmic HBM bytes of one stage for one wedge as the hot-path scope
    table counts them (the roofline's reference figure): state read, residual
    read and written, state written (4 fields x Np values each, the residual
    read counted in every stage), about 41 geometry and material values, five
    neighbour ids and the packed face codes (28 B), and L^{tri,k} stored whole
    (Np_tri^2 values).  N = 3 FP32: 3152 B; N = 2/4/5: 1488/5892/10020 B;
    FP64 N = 3: 6276 B."""
    NT = (N + 1) * (N + 2) // 2
    NP = NT * (N + 1)
    ts = bits // 8
    return 16 * NP * ts + 41 * ts + 28 + NT * NT * ts


def mortar_bytes(N: int, bits: int) -> int:
    """Algorithmic HBM bytes of one stage for one mortar face (a wedge
    quadrilateral against two tetrahedron triangles): both packed coupling
    matrices, the gathered face nodes ((N+1)^2 wedge + 2 Np_tri tetrahedron
    4-vectors), the outputs (wedge pre-lift contributions [p, u][Nq][Np_tri
    padded to 4] and both tetrahedron-face fluxes [p, u][Np_tri]), the integer
    record (8 int32) and the six FP64 geometry values the kernel reads."""
    NT = (N + 1) * (N + 2) // 2
    Nq = N + 1
    ts = bits // 8
    n = Nq * Nq + NT
    core = (n * (n + 1) + 3) // 4 * 4
    ntp = (NT + 3) // 4 * 4
    return core * ts + (Nq * Nq + 2 * NT) * 4 * ts + (2 * Nq * ntp + 4 * NT) * ts + 32 + 48


TRAFFIC_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "wedge_stage_cfg2_traffic.json")
# sources the wedge stage kernel is compiled from (its traffic record is tied to them)
KERNEL_SOURCES = [os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1607_03399_amd", "csrc", f)
                  for f in ("wedge_stage.hip", "device_common.hpp", "kernels.hpp")]


def measured_traffic(config: str):
    """HBM bytes per stage launch from the committed FETCH_SIZE / WRITE_SIZE
    counter runs, or None when the kernel source has changed since."""
    import hashlib

    if config != "cfg2" or not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as f:
        rec = json.load(f)
    h = hashlib.sha256()
    for path in KERNEL_SOURCES:
        with open(path, "rb") as f:
            h.update(f.read())
    sha = h.hexdigest()
    if rec.get("kernel_sha256") != sha:
        return None
    return float(rec["bytes_per_launch"])


def _oracle_stages(block: int, sample: int, seconds: float, dt: float, N: int, config: str):
    """The FP64 oracle on wedges [block * sample, (block + 1) * sample) of the
    workload mesh (whole columns): untimed setup, then Runge-Kutta stages
    (right-hand side + update) until ``seconds`` have elapsed.  Returns
    (elements, nodes per element, stages, wall seconds, CPU seconds)."""
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    from oracle import dg, lsrk
    from paper_1607_03399_amd import inputs

    mesh = inputs.cfg2_mesh() if config == "cfg2" else inputs.cfg5_mesh()
    om = dg.Mesh(mesh.verts, mesh.wedges, mesh.c, mesh.rho, "rigid", "upwind")
    elems = np.arange(block * sample, min((block + 1) * sample, mesh.K))
    ops = dg.build_operators(om, N, elems=elems)
    NP = ops.M.shape[1]
    rng = np.random.default_rng(block)
    U = rng.standard_normal((mesh.K, 4, NP))
    res = np.zeros((len(elems), 4, NP))
    stages = 0
    c0 = time.process_time()
    t0 = time.perf_counter()
    while True:
        s = stages % 5
        res *= lsrk.A[s]
        res += dt * dg.rhs(ops, U)
        U[elems] += lsrk.B[s] * res
        stages += 1
        if time.perf_counter() - t0 >= seconds and s == 4:
            break
    return len(elems), NP, stages, time.perf_counter() - t0, time.process_time() - c0


def _host_cpu():
    """Core count available to this process and the processor as lscpu names it."""
    ncpu = len(os.sched_getaffinity(0))
    info = {}
    try:
        import subprocess

        out = subprocess.run(["lscpu"], stdout=subprocess.PIPE, stderr=subprocess.DEVNULL, text=True, timeout=10).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core", "CPU(s)",
                             "CPU max MHz"):
                info[k.strip()] = v.strip()
    except Exception:
        pass
    return ncpu, info


def cpu_baseline(config: str, N: int, dt: float, seconds: float, sample: int, workers: int):
    """The FP64 oracle as it stands, on the host of the GPU machine: one process on the
    first ``sample`` wedges (whole columns), then ``workers`` processes at
    once, each on its own block of ``sample`` wedges, for the same time
    (every process single-threaded: the oracle's einsums run on one core).
    The worker processes are started fresh (spawn), not forked from this
    process, which holds a GPU context."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor

    ncpu, info = _host_cpu()
    ne, NP, stages, wall, cpu = _oracle_stages(0, sample, seconds, dt, N, config)
    one = ne * NP * stages / wall
    out = {
        "value": one,
        "unit": "node-updates/s",
        "cores": max(1, int(round(cpu / wall))),
        "kind": "oracle",
        "sample": f"first {ne} wedges (whole columns) of the same mesh, {stages} stages, {wall:.1f} s wall, "
                  "single process",
        "nproc": ncpu,
        "lscpu": info,
    }
    if workers > 1:
        env_keys = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")
        saved = {k: os.environ.get(k) for k in env_keys}
        for k in env_keys:
            os.environ[k] = "1"
        try:
            with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
                futs = [ex.submit(_oracle_stages, b, sample, seconds, dt, N, config) for b in range(workers)]
                rs = [f.result() for f in futs]
        finally:
            for k, v in saved.items():
                if v is None:
                    os.environ.pop(k, None)
                else:
                    os.environ[k] = v
        total = sum(r[0] * r[1] * r[2] / r[3] for r in rs)
        out["all_cores"] = {
            "value": total,
            "unit": "node-updates/s",
            "cores": workers,
            "sample": f"{workers} processes, each on its own block of {sample} wedges (whole columns), "
                      f"{min(r[2] for r in rs)}-{max(r[2] for r in rs)} stages in about {seconds:.0f} s each",
        }
    return out


def initial_state(s):
    """Gaussian pressure pulse (width 0.2) at the centre, zero velocity: every
    node carries a non-zero value, so the timing does not depend on the
    hardware moving all-zero data faster."""
    from paper_1607_03399_amd import inputs

    U = np.zeros((s.K, 4, s.NPmax))
    U[:, 0] = inputs.gaussian_pulse(s.node_coords(), width=0.2) * s.mask
    return U


def adjoint_benchmark(steps: int, every: int):
    """Receiver-misfit gradient on 128 x 128 x 16 = 524288 wedges, N = 3,
    FP32: 16 seeded receivers record p for ``steps`` steps; the data come from
    a wave speed with a seeded 10 % Gaussian anomaly; the gradient with respect
    to every element's c and rho by the discrete adjoint with checkpoints every
    ``every`` steps.  After an untimed warm-up pass (allocations), times the
    forward solve (which keeps the checkpoints) and the gradient call (reverse
    sweep, recomputing the forward segment by segment from the checkpoints)
    on the same GPU."""
    from paper_1607_03399_amd import inputs
    from paper_1607_03399_amd import wdg

    mesh = inputs.cfg5_mesh()
    rec, src, c_true = inputs.adjoint_problem(mesh)
    s = wdg.Solver(3, 32, device=0)
    s.set_mesh(mesh.verts, mesh.wedges)
    s.set_boundary("rigid")
    s.set_flux("upwind")
    s.add_ricker_source(*src)
    s.set_receivers(rec)
    s.set_material(mesh.c, mesh.rho)
    dt = s.stable_dt(0.5)
    U0 = initial_state(s)
    # data: the solve with the anomaly (setup, untimed)
    s.set_material(c_true, mesh.rho)
    s.set_fields(U0)
    s.time = 0.0
    s.step(steps, dt)
    data = s.read_receivers()
    s.set_material(mesh.c, mesh.rho)
    # warm-up pass (untimed): kernels, the checkpoint buffers and the reverse
    # sweep's state buffers are allocated here and kept by the solver, as in
    # repeated gradient evaluations (a fresh allocation of ~170 GB can take
    # seconds on this driver once other large buffers have been freed)
    s.set_fields(U0)
    s.time = 0.0
    s.adjoint_record(every, steps)
    s.step(steps, dt)
    s.adjoint_gradient_recorded(s.read_receivers() - data)
    s.synchronize()
    s.set_fields(U0)
    s.time = 0.0
    # forward solve keeping its checkpoints (the forward of the autograd Function)
    t0 = time.perf_counter()
    s.adjoint_record(every, steps)
    s.step(steps, dt)
    s.synchronize()
    fwd = time.perf_counter() - t0
    traces = s.read_receivers()
    w = traces - data
    t0 = time.perf_counter()
    gc, gr = s.adjoint_gradient_recorded(w)
    adj = time.perf_counter() - t0
    s.close()
    if not (np.all(np.isfinite(gc)) and np.all(np.isfinite(gr))):
        raise RuntimeError("non-finite gradient")
    return {
        "workload": "cfg5 adjoint: 128x128x16 = 524288 wedges, N=3, FP32, Ricker source (f0=60) at the centre, "
                    f"16 seeded receivers 0.01-0.04 from it, {steps} steps, misfit against data from a seeded "
                    "10% Gaussian anomaly in c, "
                    f"gradient w.r.t. per-element c and rho, checkpoints every {every} steps",
        "steps": steps,
        "checkpoint_every": every,
        "forward_s": fwd,
        "adjoint_s": adj,
        "adjoint_fwd_ratio": adj / fwd,
        "misfit": 0.5 * float(np.sum(w ** 2)),
        "grad_c_norm": float(np.linalg.norm(gc)),
        "grad_rho_norm": float(np.linalg.norm(gr)),
    }


def batch_benchmark(steps: int):
    """48 independent problems (1k-60k wedges, N in {2,3,4,5}, own material,
    source and time step), FP32: ``steps`` steps of each problem one after the
    other (plain form), then all of them together as one batch (autotuned,
    graph-replayed; setup untimed).  Both runs start from the same state and
    must end in bitwise the same fields."""
    from paper_1607_03399_amd import inputs
    from paper_1607_03399_amd import wdg

    specs = inputs.batch_problems()
    solvers, dts, U0s = [], [], []
    for N, mesh, xs in specs:
        s = wdg.Solver(N, 32, device=0)
        s.set_mesh(mesh.verts, mesh.wedges)
        s.set_material(mesh.c, mesh.rho)
        s.set_boundary("rigid")
        s.set_flux("upwind")
        s.add_ricker_source(xs, 10.0, 0.1, 1.0)
        U = np.zeros((s.K, 4, s.NPmax))
        U[:, 0] = inputs.gaussian_pulse(s.node_coords(), centre=xs, width=0.2)
        solvers.append(s)
        dts.append(s.stable_dt(0.5))
        U0s.append(U)

    def reset():
        for s, U in zip(solvers, U0s):
            s.set_fields(U)
            s.time = 0.0

    reset()
    for s, dt in zip(solvers, dts):  # warm up every order's kernels
        s.step(1, dt)
    reset()
    for s in solvers:
        s.synchronize()
    t0 = time.perf_counter()
    for s, dt in zip(solvers, dts):
        s.step(steps, dt)
    for s in solvers:
        s.synchronize()
    seq = time.perf_counter() - t0
    seq_fields = [s.get_fields() for s in solvers]
    reset()
    batch = wdg.Batch(32, device=0)
    for s, dt in zip(solvers, dts):
        batch.add(s, dt)
    batch.prepare(autotune=True)
    batch.step(1)  # first call captures the graph
    reset()
    t0 = time.perf_counter()
    batch.step(steps)
    bat = time.perf_counter() - t0
    same = all(np.array_equal(s.get_fields(), f) for s, f in zip(solvers, seq_fields))
    # the same batch with the orders of a stage one after another on one stream
    batch.set_concurrent(False)
    reset()
    batch.step(1)  # captures that graph
    reset()
    t0 = time.perf_counter()
    batch.step(steps)
    bat1 = time.perf_counter() - t0
    same = same and all(np.array_equal(s.get_fields(), f) for s, f in zip(solvers, seq_fields))
    orders = sorted({N for N, _, _ in specs})
    tuned = {str(N): {"elements_per_block": batch.config(N)[0], "waves_per_simd": batch.config(N)[1],
                      "tuned_stage_us": batch.config(N)[2],
                      "candidates": [{"kernel": k + "-lane", "elements_per_block": e, "waves_per_simd": w,
                                      "median_stage_us": us} for k, e, w, us in batch.trials(N)]} for N in orders}
    nodes = sum(s.K * s.Np for s in solvers)
    batch.close()
    for s in solvers:
        s.close()
    if not same:
        raise RuntimeError("batched fields differ from the plain solves")
    return {
        "workload": "cfg4 batched: 48 seeded problems, 1k-60k wedges (log-uniform), N in {2,3,4,5}, per-layer "
                    f"c in [1,3] and rho in [1,2.5], own Ricker source and time step each, FP32, {steps} steps",
        "problems": len(specs),
        "elements": int(sum(s.K for s in solvers)),
        "nodes": int(nodes),
        "steps": steps,
        "sequential_s": seq,
        "batched_s": bat,
        "batched_one_stream_s": bat1,
        "speedup": seq / bat,
        "batched_node_updates_per_s": nodes * 5 * steps / bat,
        "sequential_node_updates_per_s": nodes * 5 * steps / seq,
        "identical_fields": same,
        "tuned": tuned,
    }


def copy_bandwidth(nbytes: int = 512 << 20, reps: int = 10) -> float:
    """Device-to-device copy of nbytes (read + write) timed with events."""
    import torch

    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        y.copy_(x)
    b.record()
    torch.cuda.synchronize()
    sec = a.elapsed_time(b) / 1e3 / reps
    del x, y
    return 2 * nbytes / sec / 1e9


CONFIGS = {
    "cfg2": "262144 wedges (64x64 base x 32 layers), N=3",
    "cfg5": "524288 wedges (128x128 base x 16 layers), N=3",
    "cfg3": "hybrid: 39312 wedges + 29520 tetrahedra (20% of 32x32x24 columns split), N=4",
    "cfg3-layers": "hybrid: 38912 wedges + 30720 tetrahedra (lowest 5 of 24 layers split), N=4",
    "order4": "73728 wedges (48x48 base x 16 layers), N=4",
    "order5": "73728 wedges (48x48 base x 16 layers), N=5",
}


def workload(config: str):
    """(N, verts, wedges, tets, c, rho, wedge mesh or None, description) of a configuration."""
    from paper_1607_03399_amd import inputs

    if config == "cfg3":
        verts, wedges, tets, c, rho = inputs.cfg3_columns_mesh()
        return 4, verts, wedges, tets, c, rho, None, (
            "cfg3: 32x32 base x 24 layers, a seeded 20% of the columns split into 3 tetrahedra per prism "
            f"(nonconforming faces on the common refinement): {len(wedges)} wedges + {len(tets)} tetrahedra, "
            "N=4 (75/35 nodes), banded c and rho, rigid walls, upwind flux, Ricker source f0=10, initial "
            "Gaussian pulse (width 0.2), LSRK(5,4), CFL 0.5")
    if config == "cfg3-layers":
        verts, wedges, tets, c, rho = inputs.cfg3_hybrid_mesh()
        return 4, verts, wedges, tets, c, rho, None, (
            "cfg3 (layer-split variant): 32x32 base x 24 layers, lowest 5 layers split into 3 tetrahedra per "
            f"prism: {len(wedges)} wedges + {len(tets)} tetrahedra, N=4 (75/35 nodes), banded c and rho, "
            "rigid walls, upwind flux, Ricker source f0=10, initial Gaussian pulse (width 0.2), LSRK(5,4), "
            "CFL 0.5")
    if config in ("order4", "order5"):
        N = int(config[-1])
        mesh = inputs.layered_config(48, 16, 0.3, 0, config)
        dims = "48x48x16"
    else:
        N = 3
        mesh = inputs.cfg2_mesh() if config == "cfg2" else inputs.cfg5_mesh()
        dims = "64x64x32" if config == "cfg2" else "128x128x16"
    desc = (f"{config}: layered vertically mapped wedges, {mesh.K} elements ({dims}), N={N} "
            f"({(N + 1) ** 2 * (N + 2) // 2} nodes/wedge), banded c and rho, rigid walls, upwind flux, Ricker "
            "source f0=10, initial Gaussian pulse (width 0.2), LSRK(5,4), CFL 0.5")
    return N, mesh.verts, mesh.wedges, np.zeros((0, 4), np.int64), mesh.c, mesh.rho, mesh, desc


def forward_leg(config: str, bits: int, steps: int, warmup: int, layer_march: str = "off", tet_kernel: str = "mfma",
                wedge_kernel: str = "auto"):
    """Time ``steps`` steps of a configuration (after ``warmup`` steps) on a
    torch-bound state and stream; per-kernel averages from HIP events on that
    stream.  Returns (result dict, time step, wedge mesh or None)."""
    import torch

    from paper_1607_03399_amd import wdg

    N, verts, wedges, tets, c, rho, mesh, desc = workload(config)
    Kw, Kt = len(wedges), len(tets)
    s = wdg.Solver(N, bits, device=0)
    s.set_mesh(verts, wedges, tets)
    s.set_material(c, rho)
    s.set_boundary("rigid")
    s.set_flux("upwind")
    s.set_layer_march(layer_march)
    s.set_tet_kernel(tet_kernel)
    s.set_wedge_kernel(wedge_kernel)
    s.add_ricker_source([0.5, 0.5, 0.5], 10.0, 0.1, 1.0)
    s.set_fields(initial_state(s))
    s.bind_torch()
    dt = s.stable_dt(0.5)
    s.step(warmup, dt)
    s.synchronize()
    torch.cuda.synchronize()
    def timed_pass():
        t0 = time.perf_counter()
        s.step(steps, dt)
        s.synchronize()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    wall_plain = wall_overlap = None
    if Kw and Kt:
        # hybrid: the step as it runs, without per-kernel events (an event
        # between two kernels adds a gap), then with the tetrahedron kernel
        # on the second stream beside the wedge kernel
        wall_plain = timed_pass()
        s.set_overlap(True)
        wall_overlap = timed_pass()
        s.set_overlap(False)
    # per-kernel HIP events (kernels in order on the solver stream)
    s.kernel_timing(True)
    t0 = time.perf_counter()
    s.step(steps, dt)
    s.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    w_ms, t_ms, m_ms, nlaunch = s.read_kernel_timing_split()
    s.kernel_timing(False)
    U = s.get_fields()
    nmort = s.mortar_count() if Kt else 0
    s.close()
    if not np.all(np.isfinite(U)):
        raise RuntimeError("non-finite fields")
    assert nlaunch == 5 * steps, (nlaunch, 5 * steps)
    NPw = (N + 1) ** 2 * (N + 2) // 2
    NPt = (N + 1) * (N + 2) * (N + 3) // 6
    nodes = Kw * NPw + Kt * NPt
    kernels = {}
    if Kw:
        avg = w_ms * 1e3 / nlaunch
        rec_bytes = Kw * (stage_bytes(N, bits, False) + 4 * stage_bytes(N, bits, True)) / 5
        node = N >= 4 and bits == 32 and wedge_kernel in ("node", "auto")
        kernels["wedge_stage"] = {"avg_us": avg, "variant": "node-lane" if node else "level-lane",
                                  "bytes_per_launch": Kw * table_stage_bytes(N, bits),
                                  "GBs": Kw * table_stage_bytes(N, bits) / avg / 1e3,
                                  "record_bytes_per_launch": rec_bytes, "record_GBs": rec_bytes / avg / 1e3}
    if Kt:
        avg = t_ms * 1e3 / nlaunch
        tb = Kt * (tet_stage_bytes(N, bits, False) + 4 * tet_stage_bytes(N, bits, True)) / 5
        kernels["tet_stage"] = {"avg_us": avg, "bytes_per_launch": tb, "GBs": tb / avg / 1e3, "variant": tet_kernel}
    if nmort:
        avg = m_ms * 1e3 / nlaunch
        mb = nmort * mortar_bytes(N, bits)
        kernels["mortar_kernel"] = {"avg_us": avg, "mortars": nmort, "bytes_per_launch": mb, "GBs": mb / avg / 1e3}
    leg = {
        "workload": desc,
        "precision": bits,
        "elements": Kw + Kt,
        "wedges": Kw,
        "tetrahedra": Kt,
        "order": N,
        "nodes": nodes,
        "dt": dt,
        "steps": steps,
        "ms_per_step": (wall_plain if wall_plain is not None else wall) * 1e3 / steps,
        "node_updates_per_s": nodes * 5 * steps / (wall_plain if wall_plain is not None else wall),
        "kernels": kernels,
    }
    if wall_plain is not None:
        leg["ms_per_step_with_kernel_events"] = wall * 1e3 / steps
        leg["ms_per_step_tet_beside_wedge"] = wall_overlap * 1e3 / steps
    return leg, dt, mesh


def ab_passes(kind: str, config: str, steps: int, warmup: int, reps: int = 3):
    """Alternate two settings on one solver and print one JSON line per timed
    pass: 'wedge-kernel' (level-lane vs node-lane wedge kernel, per-kernel HIP
    events) or 'overlap' (hybrid meshes: the three kernels in order vs the
    tetrahedron kernel beside the wedge kernel, wall time per step without
    events)."""
    import torch

    from paper_1607_03399_amd import wdg

    N, verts, wedges, tets, c, rho, mesh, desc = workload(config)
    s = wdg.Solver(N, 32, device=0)
    s.set_mesh(verts, wedges, tets)
    s.set_material(c, rho)
    s.set_boundary("rigid")
    s.set_flux("upwind")
    s.add_ricker_source([0.5, 0.5, 0.5], 10.0, 0.1, 1.0)
    s.set_fields(initial_state(s))
    s.bind_torch()
    dt = s.stable_dt(0.5)
    s.step(warmup, dt)
    s.synchronize()
    settings = ("level", "node") if kind == "wedge-kernel" else (False, True)
    for rep in range(reps):
        for v in settings:
            if kind == "wedge-kernel":
                s.set_wedge_kernel(v)
            else:
                s.set_overlap(v)
            s.step(2, dt)
            s.synchronize()
            torch.cuda.synchronize()
            if kind == "wedge-kernel":
                s.kernel_timing(True)
            t0 = time.perf_counter()
            s.step(steps, dt)
            s.synchronize()
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            line = {"ab": kind, "config": config, "setting": v, "pass": rep, "ms_per_step": wall * 1e3 / steps}
            if kind == "wedge-kernel":
                w_ms, t_ms, m_ms, n = s.read_kernel_timing_split()
                s.kernel_timing(False)
                line["wedge_stage_us"] = w_ms * 1e3 / n
            print(json.dumps(line), flush=True)
    s.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="cfg2", choices=sorted(CONFIGS),
                    help=("; ".join(f"{k}: {v}" for k, v in CONFIGS.items()) + " (default cfg2)").replace("%", "%%"))
    ap.add_argument("--precision", type=int, default=32, choices=[32, 64])
    ap.add_argument("--layer-march", default="off", choices=["off", "chunk", "column"],
                    help="layer marching of the level-lane wedge kernel: vertical neighbours inside a chunk from "
                         "LDS (chunk), and one block marching each column segment (column)")
    ap.add_argument("--tet-kernel", default="mfma", choices=["mfma", "valu"],
                    help="tetrahedron operator products on the matrix cores (default) or as per-node dot products")
    ap.add_argument("--wedge-kernel", default="auto", choices=["auto", "level", "node"],
                    help="wedge stage kernel: auto (one lane per triangle node in FP32 at orders 4 and 5, else one "
                         "lane per GLL level), level (one lane per GLL level) or node (one lane per triangle node at "
                         "orders 4 and 5 in FP32)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--cpu-sample", type=int, default=1024)
    ap.add_argument("--cpu-workers", type=int, default=0,
                    help="processes of the all-core oracle figure (default: the host's cores, at most 16)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the adjoint leg (cfg2 runs the cfg5 receiver-misfit gradient after the forward bench)")
    ap.add_argument("--adjoint-steps", type=int, default=500)
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched leg (cfg2 runs the cfg4 48-problem batch after the forward bench)")
    ap.add_argument("--batch-steps", type=int, default=300)
    ap.add_argument("--no-legs", action="store_true",
                    help="skip the other forward configurations (cfg2 runs cfg3 with both tetrahedron kernels, "
                         "cfg5, order 4 and 5 and FP64 cfg2 for 20 steps each)")
    ap.add_argument("--leg-steps", type=int, default=40)
    ap.add_argument("--no-copy-calibration", action="store_true",
                    help="skip the plain 512 MiB device copy (the measured HBM reference of the roofline)")
    ap.add_argument("--ab", choices=["wedge-kernel", "overlap"],
                    help="instead of the bench line: alternate the two wedge kernels (FP32, orders 4 and 5) or the "
                         "in-order and side-by-side hybrid stage on the chosen --config, three times each, and print "
                         "one JSON line per pass of --steps steps")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        if int(os.environ.get("RANK", "0")) == 0:
            print(json.dumps({"error": "this solver runs on one GPU; --gpus must be 1 (the library does not "
                                       "shard a mesh across GPUs)", "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    import torch  # noqa: F401  (device memory and streams of the bound state)

    if args.ab:
        ab_passes(args.ab, args.config, args.steps, args.warmup)
        return

    copy_gbs = None if args.no_copy_calibration else copy_bandwidth()
    bits = args.precision
    main_leg, dt, mesh = forward_leg(args.config, bits, args.steps, args.warmup, args.layer_march, args.tet_kernel,
                                     args.wedge_kernel)
    kernels = main_leg["kernels"]
    dominant = max(kernels, key=lambda k: kernels[k]["avg_us"])
    achieved = kernels[dominant]["GBs"]
    N = main_leg["order"]
    out = {
        "metric": f"DG node-updates/s per RK stage ({'wedge' if not main_leg['tetrahedra'] else 'wedge+tet'} "
                  f"N={N}, FP{bits})",
        "value": main_leg["node_updates_per_s"],
        "unit": "node-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_leg["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if bits == 32 else "f64",
        "data": "synthetic",
        "config": {k: main_leg[k] for k in ("workload", "elements", "wedges", "tetrahedra", "order", "nodes", "dt",
                                            "kernels")},
        "roofline": {
            "bound": "hbm",
            "kernel": dominant,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(args.config) if bits == 32 else None,
            "bytes_per_launch": kernels[dominant]["bytes_per_launch"],
            "measured_copy_GBs": copy_gbs,
            "frac_of_copy": achieved / copy_gbs if copy_gbs else None,
        },
    }
    if dominant == "wedge_stage":
        out["roofline"]["record_frac"] = kernels[dominant]["record_GBs"] / HBM_PEAK_GBS
    default_run = args.config == "cfg2" and bits == 32
    if default_run and not args.no_legs:
        legs = {}
        for name, cfg, b, tk, wk in (("cfg3", "cfg3", 32, "mfma", "auto"), ("cfg3_tet_valu", "cfg3", 32, "valu", "auto"),
                                     ("cfg3_wedge_level", "cfg3", 32, "mfma", "level"),
                                     ("cfg5_forward", "cfg5", 32, "mfma", "auto"), ("order4", "order4", 32, "mfma", "auto"),
                                     ("order4_wedge_level", "order4", 32, "mfma", "level"),
                                     ("order5", "order5", 32, "mfma", "auto"),
                                     ("order5_wedge_level", "order5", 32, "mfma", "level"),
                                     ("cfg2_fp64", "cfg2", 64, "mfma", "auto")):
            legs[name], _, _ = forward_leg(cfg, b, args.leg_steps, 10, tet_kernel=tk, wedge_kernel=wk)
        # layer marching (the paper's future work) against the gathers, same kernel
        for name, mode in (("cfg2_chunk_march", "chunk"), ("cfg2_column_march", "column")):
            legs[name], _, _ = forward_leg("cfg2", 32, args.leg_steps, 10, layer_march=mode)
        out["legs"] = legs
    if default_run and not args.no_adjoint:
        out["adjoint"] = adjoint_benchmark(args.adjoint_steps, 50)
    if default_run and not args.no_batch:
        out["batched"] = batch_benchmark(args.batch_steps)
    if not args.no_cpu_baseline and mesh is not None and args.config in ("cfg2", "cfg5"):
        workers = args.cpu_workers or min(16, len(os.sched_getaffinity(0)))
        out["cpu_baseline"] = cpu_baseline(args.config, N, dt, args.cpu_seconds, args.cpu_sample, workers)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
