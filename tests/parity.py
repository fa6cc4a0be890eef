"""Comparison helpers of the GPU parity tests.

``rel`` is the relative Euclidean L2 error over all nodal values of all four
fields, the measure the tolerances (FP64 1e-12, FP32 1e-5) are stated in.
``elem_rel`` is the largest error of a single element against the same
scale (the root-mean-square element norm of the reference), so that one
wrong element cannot hide in the global norm: ``check`` requires it to stay
within ten times the tolerance.  Arrays are element-major: (K, ...).
"""
import numpy as np

TOL = {64: 1e-12, 32: 1e-5}
# tetrahedron stage kernels: operator products on the matrix cores / as per-node dot products
TET_KERNELS = ("mfma", "valu")


def tet_chunk(N: int, kernel: str) -> int:
    """Tetrahedra per chunk (the unit a persistent block loops over) of the
    tetrahedron stage kernel."""
    if kernel == "valu":
        return 256 // ((N + 1) * (N + 2) * (N + 3) // 6)
    return 16 if N <= 2 else 8
ELEM_FACTOR = 10.0


def rel(a, b) -> float:
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def elem_rel(a, b) -> float:
    a = np.asarray(a).reshape(len(a), -1)
    b = np.asarray(b).reshape(len(b), -1)
    d = np.sqrt(((a - b) ** 2).sum(axis=1))
    scale = np.sqrt(np.mean((b ** 2).sum(axis=1)))
    return float(d.max() / scale)


def check(got, ref, tol, what="") -> tuple:
    """Assert the global and the per-element bound; returns both errors."""
    e, m = rel(got, ref), elem_rel(got, ref)
    assert e <= tol, f"{what}: relative L2 error {e:.3e} > {tol:.1e}"
    assert m <= ELEM_FACTOR * tol, f"{what}: worst element {m:.3e} > {ELEM_FACTOR * tol:.1e}"
    return e, m
