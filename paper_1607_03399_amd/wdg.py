"""Thin ctypes binding of libwdg (C ABI in include/wdg.h).

Only argument marshalling lives here: every step of the solver runs in the
HIP library.  Arrays of nodal values use the layout (K, 4, Np) with fields
(p, u_x, u_y, u_z) and node n = j * Np_tri + i inside an element.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwdg.so")

OK = 0
ERRORS = {
    -1: "WDG_ERR_ARG", -2: "WDG_ERR_STATE", -3: "WDG_ERR_NOT_VERTICAL", -4: "WDG_ERR_JACOBIAN",
    -5: "WDG_ERR_ORIENTATION", -6: "WDG_ERR_NONCONFORMING", -7: "WDG_ERR_OUTSIDE", -8: "WDG_ERR_HIP",
    -9: "WDG_ERR_OOM", -10: "WDG_ERR_UNSTABLE", -11: "WDG_ERR_UNSUPPORTED",
}
BC = {"dirichlet": 0, "rigid": 1}
FLUX = {"upwind": 0, "central": 1}
MASS = {"exact": 0, "lumped": 1}

_lib = None
_dp = C.POINTER(C.c_double)
_i64p = C.POINTER(C.c_int64)


class WdgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code
        self.name = ERRORS.get(code, str(code))


def load_library() -> C.CDLL:
    """Load libwdg.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1607_03399_amd.build`")
    # torch ships its own HIP runtime under the same soname; loading torch first
    # makes the library and torch share that one runtime (streams, memory)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    sig = {
        "wdg_create": (C.c_int, [C.c_int, C.c_int, C.c_int, C.POINTER(vp)]),
        "wdg_destroy": (C.c_int, [vp]),
        "wdg_last_error": (C.c_char_p, [vp]),
        "wdg_set_mesh": (C.c_int, [vp, C.c_int64, _dp, C.c_int64, _i64p, C.c_int64, _i64p]),
        "wdg_set_material": (C.c_int, [vp, _dp, _dp]),
        "wdg_set_boundary": (C.c_int, [vp, C.c_int]),
        "wdg_set_flux": (C.c_int, [vp, C.c_int]),
        "wdg_set_mass": (C.c_int, [vp, C.c_int]),
        "wdg_set_layer_march": (C.c_int, [vp, C.c_int]),
        "wdg_set_tet_blocks": (C.c_int, [vp, C.c_int]),
        "wdg_set_overlap": (C.c_int, [vp, C.c_int]),
        "wdg_set_wedge_block": (C.c_int, [vp, C.c_int]),
        "wdg_set_tet_kernel": (C.c_int, [vp, C.c_int]),
        "wdg_set_wedge_kernel": (C.c_int, [vp, C.c_int]),
        "wdg_num_nodes": (C.c_int, [vp, _i64p]),
        "wdg_get_node_coords": (C.c_int, [vp, _dp]),
        "wdg_set_fields": (C.c_int, [vp, _dp, _dp, _dp, _dp]),
        "wdg_get_fields": (C.c_int, [vp, _dp, _dp, _dp, _dp]),
        "wdg_bind_device_state": (C.c_int, [vp, vp, vp, vp]),
        "wdg_add_ricker_source": (C.c_int, [vp, _dp, C.c_double, C.c_double, C.c_double, C.POINTER(C.c_int)]),
        "wdg_set_receivers": (C.c_int, [vp, C.c_int64, _dp]),
        "wdg_read_receivers": (C.c_int, [vp, _dp, _i64p]),
        "wdg_stable_dt": (C.c_int, [vp, C.c_double, _dp]),
        "wdg_step": (C.c_int, [vp, C.c_int64, C.c_double]),
        "wdg_get_time": (C.c_int, [vp, _dp]),
        "wdg_set_time": (C.c_int, [vp, C.c_double]),
        "wdg_synchronize": (C.c_int, [vp]),
        "wdg_eval_rhs": (C.c_int, [vp, C.c_double, _dp, _dp]),
        "wdg_eval_rhs_noalloc": (C.c_int, [vp, C.c_double, _dp, _dp]),
        "wdg_eval_rhs_noalloc_max_nodes": (C.c_int, [C.c_int, _i64p]),
        "wdg_energy": (C.c_int, [vp, _dp]),
        "wdg_adjoint_gradient": (C.c_int, [vp, C.c_int64, C.c_double, _dp, C.c_int64, _dp, _dp]),
        "wdg_adjoint_record": (C.c_int, [vp, C.c_int64, C.c_int64]),
        "wdg_adjoint_gradient_recorded": (C.c_int, [vp, _dp, _dp, _dp, _i64p]),
        "wdg_set_adjoint_memory_limit": (C.c_int, [vp, C.c_int64]),
        "wdg_get_element_data": (C.c_int, [vp, _dp, _dp]),
        "wdg_mortar_couplings": (C.c_int, [vp, C.c_int64, C.POINTER(C.c_int64), _dp, C.POINTER(C.c_int64)]),
        "wdg_kernel_timing": (C.c_int, [vp, C.c_int]),
        "wdg_read_kernel_timing": (C.c_int, [vp, _dp, _i64p]),
        "wdg_read_kernel_timing_split": (C.c_int, [vp, _dp, _i64p]),
        "wdg_reference_operator": (C.c_int, [C.c_int, C.c_char_p, _dp, C.c_int64, _i64p]),
        "wdg_batch_create": (C.c_int, [C.c_int, C.c_int, C.POINTER(vp)]),
        "wdg_batch_destroy": (C.c_int, [vp]),
        "wdg_batch_last_error": (C.c_char_p, [vp]),
        "wdg_batch_add": (C.c_int, [vp, vp, C.c_double, C.POINTER(C.c_int)]),
        "wdg_batch_prepare": (C.c_int, [vp, C.c_int]),
        "wdg_batch_step": (C.c_int, [vp, C.c_int64]),
        "wdg_batch_config": (C.c_int, [vp, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), _dp]),
        "wdg_batch_set_concurrent": (C.c_int, [vp, C.c_int]),
        "wdg_batch_trials": (C.c_int, [vp, C.c_int, C.c_int64, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                       C.POINTER(C.c_int), _dp, _i64p]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _ptr(a: np.ndarray, ctype=C.c_double):
    return a.ctypes.data_as(C.POINTER(ctype))


def reference_operator(N: int, name: str) -> np.ndarray:
    """Host-built reference operator of the library (see wdg_reference_operator)."""
    lib = load_library()
    n = C.c_int64()
    rc = lib.wdg_reference_operator(N, name.encode(), None, 0, C.byref(n))
    if rc:
        raise WdgError(rc, f"reference operator {name}")
    out = np.zeros(n.value)
    lib.wdg_reference_operator(N, name.encode(), _ptr(out), n.value, C.byref(n))
    return out


def eval_rhs_noalloc_max_nodes(precision: int) -> int:
    """Largest node count wdg_eval_rhs_noalloc stages in its fixed device array."""
    lib = load_library()
    n = C.c_int64()
    rc = lib.wdg_eval_rhs_noalloc_max_nodes(int(precision), C.byref(n))
    if rc:
        raise WdgError(rc, "eval_rhs_noalloc_max_nodes")
    return n.value


class Solver:
    """One solver context (one device, one polynomial order, one precision)."""

    def __init__(self, N: int, precision: int = 32, device: int = 0):
        self._lib = load_library()
        self.N = N
        self.precision = precision
        self.NT = (N + 1) * (N + 2) // 2
        self.Np = self.NT * (N + 1)
        self.K = 0
        h = C.c_void_p()
        rc = self._lib.wdg_create(N, precision, device, C.byref(h))
        if rc:
            raise WdgError(rc, "wdg_create")
        self._h = h
        self._bound = None

    # -- plumbing ----------------------------------------------------------
    def _check(self, rc: int, what: str):
        if rc:
            msg = self._lib.wdg_last_error(self._h)
            raise WdgError(rc, f"{what}: {msg.decode() if msg else ''}")

    def close(self):
        if getattr(self, "_h", None):
            self._lib.wdg_destroy(self._h)
            self._h = None
        self._bound = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- setup -------------------------------------------------------------
    def set_mesh(self, verts, wedges, tets=None):
        v = np.ascontiguousarray(verts, dtype=np.float64)
        w = np.ascontiguousarray(wedges, dtype=np.int64)
        t = np.ascontiguousarray(np.zeros((0, 4)) if tets is None else tets, dtype=np.int64)
        self._check(self._lib.wdg_set_mesh(self._h, len(v), _ptr(v), len(w), _ptr(w, C.c_int64), len(t),
                                           _ptr(t, C.c_int64)), "set_mesh")
        self.Kw, self.Kt = len(w), len(t)
        self.K = self.Kw + self.Kt
        self.Npt = (self.N + 1) * (self.N + 2) * (self.N + 3) // 6
        # element-major arrays are padded to the largest element: (K, ..., NPmax);
        # mask[k, i] marks the nodes element k has (wedges first, then tetrahedra)
        self.NPmax = self.Np if self.Kw else self.Npt
        self.mask = np.zeros((self.K, self.NPmax), dtype=bool)
        self.mask[:self.Kw, :self.Np] = True
        self.mask[self.Kw:, :self.Npt] = True

    def set_material(self, c, rho):
        c = np.ascontiguousarray(np.broadcast_to(c, (self.K,)), dtype=np.float64)
        r = np.ascontiguousarray(np.broadcast_to(rho, (self.K,)), dtype=np.float64)
        self._check(self._lib.wdg_set_material(self._h, _ptr(c), _ptr(r)), "set_material")

    def set_boundary(self, bc: str):
        self._check(self._lib.wdg_set_boundary(self._h, BC[bc]), "set_boundary")

    def set_flux(self, flux: str):
        self._check(self._lib.wdg_set_flux(self._h, FLUX[flux]), "set_flux")

    def set_layer_march(self, mode):
        """False/'off', True/'chunk' (vertical neighbours inside a chunk from LDS) or 'column'
        (one block marches each column, carrying a chunk's top level to the next)."""
        code = {False: 0, True: 1, "off": 0, "chunk": 1, "column": 2}[mode]
        self._check(self._lib.wdg_set_layer_march(self._h, code), "set_layer_march")

    def set_wedge_block(self, elements: int):
        """Elements per block of the node-lane wedge kernel (0: default; orders 4 and 5 in FP32)."""
        self._check(self._lib.wdg_set_wedge_block(self._h, int(elements)), "set_wedge_block")

    def set_overlap(self, enable: bool):
        """Hybrid stages: run the tetrahedron kernel on a second stream beside the wedge kernel
        (True) or all kernels in order on the solver stream (False, the default)."""
        self._check(self._lib.wdg_set_overlap(self._h, int(bool(enable))), "set_overlap")

    def set_tet_blocks(self, blocks: int):
        """Cap on the persistent blocks of the tetrahedron kernel (0: default)."""
        self._check(self._lib.wdg_set_tet_blocks(self._h, int(blocks)), "set_tet_blocks")

    def set_tet_kernel(self, variant: str):
        """'mfma' (default: operator products on the matrix cores) or 'valu' (per-node dot products)."""
        self._check(self._lib.wdg_set_tet_kernel(self._h, {"mfma": 0, "valu": 1}[variant]), "set_tet_kernel")

    def set_wedge_kernel(self, variant: str):
        """'auto' (default: one lane per triangle node in FP32 at orders 4 and 5, else one lane per
        GLL level),
        'level' (one lane per GLL level) or 'node' (one lane per triangle node wherever it exists)."""
        self._check(self._lib.wdg_set_wedge_kernel(self._h, {"auto": 0, "level": 1, "node": 2}[variant]),
                    "set_wedge_kernel")

    def set_mass(self, mass: str):
        """'exact' (default, energy stable) or 'lumped' (Gauss-Lobatto in t, for comparison)."""
        self._check(self._lib.wdg_set_mass(self._h, MASS[mass]), "set_mass")

    def num_nodes(self) -> int:
        n = C.c_int64()
        self._check(self._lib.wdg_num_nodes(self._h, C.byref(n)), "num_nodes")
        return n.value

    def node_coords(self) -> np.ndarray:
        """(K, NPmax, 3) node coordinates, zero on padding."""
        out = np.zeros((self.num_nodes(), 3))
        self._check(self._lib.wdg_get_node_coords(self._h, _ptr(out)), "get_node_coords")
        X = np.zeros((self.K, self.NPmax, 3))
        X[self.mask] = out
        return X

    def _flatten(self, U) -> np.ndarray:
        """(K, 4, NPmax) -> (4, nodes) in the library's node order."""
        U = np.asarray(U, dtype=np.float64).reshape(self.K, 4, self.NPmax)
        return np.ascontiguousarray(np.stack([U[:, f, :][self.mask] for f in range(4)]))

    def _unflatten(self, F) -> np.ndarray:
        U = np.zeros((self.K, 4, self.NPmax))
        for f in range(4):
            U[:, f, :][self.mask] = F[f]
        return U

    # -- state -------------------------------------------------------------
    def set_fields(self, U):
        """U: (K, 4, NPmax) nodal values of (p, u_x, u_y, u_z); padding ignored."""
        F = self._flatten(U)
        self._check(self._lib.wdg_set_fields(self._h, *[_ptr(F[i]) for i in range(4)]), "set_fields")

    def get_fields(self) -> np.ndarray:
        F = np.zeros((4, self.num_nodes()))
        self._check(self._lib.wdg_get_fields(self._h, *[_ptr(F[i]) for i in range(4)]), "get_fields")
        return self._unflatten(F)

    def bind_torch(self, device=None, stream=None):
        """Allocate the state as torch tensors on the current HIP device and run
        every launch on the given (or current) torch stream."""
        import torch

        dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        dtype = torch.float32 if self.precision == 32 else torch.float64
        n = self.num_nodes() * 4
        U = torch.empty(2 * n, dtype=dtype, device=dev)
        res = torch.empty(n, dtype=dtype, device=dev)
        st = torch.cuda.current_stream(dev) if stream is None else stream
        self._check(self._lib.wdg_bind_device_state(self._h, C.c_void_p(U.data_ptr()), C.c_void_p(res.data_ptr()),
                                                    C.c_void_p(st.cuda_stream)), "bind_device_state")
        self._bound = (U, res, st)
        return self._bound

    def set_stream(self, stream):
        self._check(self._lib.wdg_bind_device_state(self._h, None, None, C.c_void_p(stream.cuda_stream)),
                    "bind_device_state")

    # -- sources and receivers --------------------------------------------
    def add_ricker_source(self, xyz, f0: float, t0: float, amp: float = 1.0) -> int:
        x = np.ascontiguousarray(xyz, dtype=np.float64)
        sid = C.c_int()
        self._check(self._lib.wdg_add_ricker_source(self._h, _ptr(x), f0, t0, amp, C.byref(sid)), "add_ricker_source")
        return sid.value

    def set_receivers(self, xyz):
        x = np.ascontiguousarray(np.atleast_2d(xyz), dtype=np.float64)
        self._nrec = len(x)
        self._check(self._lib.wdg_set_receivers(self._h, len(x), _ptr(x)), "set_receivers")

    def read_receivers(self) -> np.ndarray:
        n = C.c_int64()
        self._check(self._lib.wdg_read_receivers(self._h, None, C.byref(n)), "read_receivers")
        out = np.zeros((n.value, getattr(self, "_nrec", 0)))
        if out.size:
            self._check(self._lib.wdg_read_receivers(self._h, _ptr(out), C.byref(n)), "read_receivers")
        return out

    # -- stepping ----------------------------------------------------------
    def stable_dt(self, cfl: float) -> float:
        dt = C.c_double()
        self._check(self._lib.wdg_stable_dt(self._h, cfl, C.byref(dt)), "stable_dt")
        return dt.value

    def step(self, nsteps: int, dt: float):
        self._check(self._lib.wdg_step(self._h, int(nsteps), float(dt)), "step")

    @property
    def time(self) -> float:
        t = C.c_double()
        self._check(self._lib.wdg_get_time(self._h, C.byref(t)), "get_time")
        return t.value

    @time.setter
    def time(self, t: float):
        self._check(self._lib.wdg_set_time(self._h, float(t)), "set_time")

    def synchronize(self):
        self._check(self._lib.wdg_synchronize(self._h), "synchronize")

    def eval_rhs(self, U, t: float = 0.0) -> np.ndarray:
        inp = self._flatten(U)  # field blocks
        out = np.zeros_like(inp)
        self._check(self._lib.wdg_eval_rhs(self._h, float(t), _ptr(inp), _ptr(out)), "eval_rhs")
        return self._unflatten(out)

    def eval_rhs_noalloc(self, U, t: float = 0.0) -> np.ndarray:
        """eval_rhs staged through the library's fixed device array (no device allocation)."""
        inp = self._flatten(U)
        out = np.zeros_like(inp)
        self._check(self._lib.wdg_eval_rhs_noalloc(self._h, float(t), _ptr(inp), _ptr(out)), "eval_rhs_noalloc")
        return self._unflatten(out)

    def energy(self) -> float:
        E = C.c_double()
        self._check(self._lib.wdg_energy(self._h, C.byref(E)), "energy")
        return E.value

    def adjoint_gradient(self, nsteps: int, dt: float, weights, checkpoint_every: int = 50):
        """(dF/dc, dF/drho) per element of F = sum_{n,r} weights[n, r] p_r(after step n)
        for the solve that ``step(nsteps, dt)`` would run from the current state
        (discrete adjoint; see wdg_adjoint_gradient).  The state is unchanged."""
        w = np.ascontiguousarray(weights, dtype=np.float64)
        if w.shape != (int(nsteps), getattr(self, "_nrec", 0)):
            raise ValueError(f"weights must be (nsteps, nrec) = ({nsteps}, {getattr(self, '_nrec', 0)})")
        gc = np.zeros(self.K)
        gr = np.zeros(self.K)
        self._check(self._lib.wdg_adjoint_gradient(self._h, int(nsteps), float(dt), _ptr(w), int(checkpoint_every),
                                                   _ptr(gc), _ptr(gr)), "adjoint_gradient")
        return gc, gr

    def adjoint_record(self, checkpoint_every: int, max_steps: int):
        """Keep checkpoints of the following ``step`` calls for adjoint_gradient_recorded."""
        self._check(self._lib.wdg_adjoint_record(self._h, int(checkpoint_every), int(max_steps)), "adjoint_record")
        self.record_id = getattr(self, "record_id", 0) + 1

    def recorded_steps(self) -> int:
        """Steps of the current forward recording (0: none)."""
        n = C.c_int64(0)
        self._lib.wdg_adjoint_gradient_recorded(self._h, None, None, None, C.byref(n))
        return n.value

    def adjoint_gradient_recorded(self, weights):
        """(dF/dc, dF/drho) of F = sum weights[n, r] p_r(after recorded step n) for
        the solve recorded since adjoint_record (no forward sweep)."""
        n = C.c_int64()
        gc = np.zeros(self.K)
        gr = np.zeros(self.K)
        w = np.ascontiguousarray(weights, dtype=np.float64)
        if w.ndim != 2 or w.shape[1] != getattr(self, "_nrec", 0):
            raise ValueError("weights must be (recorded steps, nrec)")
        # probe: the number of recorded steps (the call itself fails on the null arrays)
        self._lib.wdg_adjoint_gradient_recorded(self._h, None, None, None, C.byref(n))
        if n.value and w.shape[0] != n.value:
            raise ValueError(f"weights must have {n.value} rows (recorded steps)")
        self._check(self._lib.wdg_adjoint_gradient_recorded(self._h, _ptr(w), _ptr(gc), _ptr(gr), C.byref(n)),
                    "adjoint_gradient_recorded")
        return gc, gr

    def set_adjoint_memory_limit(self, nbytes: int):
        self._check(self._lib.wdg_set_adjoint_memory_limit(self._h, int(nbytes)), "set_adjoint_memory_limit")

    def kernel_timing(self, enable: bool):
        self._check(self._lib.wdg_kernel_timing(self._h, int(bool(enable))), "kernel_timing")

    def read_kernel_timing(self):
        """(summed stage-kernel milliseconds, number of timed launches)."""
        ms = C.c_double()
        n = C.c_int64()
        self._check(self._lib.wdg_read_kernel_timing(self._h, C.byref(ms), C.byref(n)), "read_kernel_timing")
        return ms.value, n.value

    def read_kernel_timing_split(self):
        """(wedge, tetrahedron, mortar kernel milliseconds, number of timed stages)."""
        ms = np.zeros(3)
        n = C.c_int64()
        self._check(self._lib.wdg_read_kernel_timing_split(self._h, _ptr(ms), C.byref(n)), "read_kernel_timing_split")
        return float(ms[0]), float(ms[1]), float(ms[2]), n.value

    def mortar_count(self) -> int:
        """Number of mortar faces (wedge quadrilaterals covered by two tetrahedron triangles)."""
        cnt = C.c_int64()
        self._check(self._lib.wdg_mortar_couplings(self._h, 0, None, None, C.byref(cnt)), "mortar_couplings")
        return cnt.value

    def mortar_couplings(self):
        """(faces (nmort, 7) int64, couplings (nmort, 2, n (n+1)/2)) of the mortar
        faces, integrated on the host (see wdg_mortar_couplings)."""
        cnt = C.c_int64()
        self._check(self._lib.wdg_mortar_couplings(self._h, 0, None, None, C.byref(cnt)), "mortar_couplings")
        nm = cnt.value
        n = (self.N + 1) ** 2 + self.NT
        faces = np.zeros((nm, 7), dtype=np.int64)
        cp = np.zeros((nm, 2, n * (n + 1) // 2))
        fp = faces.ctypes.data_as(C.POINTER(C.c_int64))
        self._check(self._lib.wdg_mortar_couplings(self._h, nm, fp, _ptr(cp), C.byref(cnt)), "mortar_couplings")
        return faces, cp

    def element_data(self):
        """(geo (Kw,40), lift (Kw,Np_tri,Np_tri)) of the wedges, built by the device setup kernel."""
        geo = np.zeros((self.Kw, 40))
        lift = np.zeros((self.Kw, self.NT, self.NT))
        self._check(self._lib.wdg_get_element_data(self._h, _ptr(geo), _ptr(lift)), "get_element_data")
        return geo, lift


class Batch:
    """Many independent problems (Solver objects on one device and precision)
    advanced together: one launch per polynomial order and stage, one step
    replayed as a HIP graph (see wdg_batch_* in wdg.h)."""

    def __init__(self, precision: int = 32, device: int = 0):
        self._lib = load_library()
        h = C.c_void_p()
        rc = self._lib.wdg_batch_create(device, precision, C.byref(h))
        if rc:
            raise WdgError(rc, "wdg_batch_create")
        self._h = h
        self.problems = []

    def _check(self, rc: int, what: str):
        if rc:
            msg = self._lib.wdg_batch_last_error(self._h)
            raise WdgError(rc, f"{what}: {msg.decode() if msg else ''}")

    def add(self, solver: Solver, dt: float) -> int:
        idx = C.c_int()
        self._check(self._lib.wdg_batch_add(self._h, solver._h, float(dt), C.byref(idx)), "batch_add")
        self.problems.append(solver)
        return idx.value

    def prepare(self, autotune: bool = True):
        self._check(self._lib.wdg_batch_prepare(self._h, int(bool(autotune))), "batch_prepare")

    def step(self, nsteps: int):
        self._check(self._lib.wdg_batch_step(self._h, int(nsteps)), "batch_step")

    def set_concurrent(self, enable: bool):
        """Orders of a stage on their own streams at once (default), or one
        after another on the batch's stream (wdg_batch_set_concurrent)."""
        self._check(self._lib.wdg_batch_set_concurrent(self._h, int(bool(enable))), "batch_set_concurrent")

    def config(self, N: int):
        """(elements per block, waves per SIMD chosen by the autotuner, tuned stage microseconds)."""
        e = C.c_int()
        w = C.c_int()
        us = C.c_double()
        self._check(self._lib.wdg_batch_config(self._h, int(N), C.byref(e), C.byref(w), C.byref(us)), "batch_config")
        return e.value, w.value, us.value

    def trials(self, N: int):
        """The autotuner's candidates of order N: [(kernel 'level' or 'node', elements per block,
        waves per SIMD, median stage us)]."""
        n = C.c_int64()
        self._check(self._lib.wdg_batch_trials(self._h, int(N), 0, None, None, None, None, C.byref(n)),
                    "batch_trials")
        k = n.value
        kk = (C.c_int * max(k, 1))()
        e = (C.c_int * max(k, 1))()
        w = (C.c_int * max(k, 1))()
        us = np.zeros(max(k, 1))
        self._check(self._lib.wdg_batch_trials(self._h, int(N), k, kk, e, w, _ptr(us), C.byref(n)), "batch_trials")
        return [("node" if kk[i] == 2 else "level", int(e[i]), int(w[i]), float(us[i])) for i in range(k)]

    def close(self):
        if getattr(self, "_h", None):
            self._lib.wdg_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
