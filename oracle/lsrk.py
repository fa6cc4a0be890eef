"""Five-stage fourth-order low-storage Runge-Kutta (oracle).

The paper advances in time with a multirate Adams-Bashforth scheme and
notes that any standard explicit scheme may be used (Sec. 6.2).  The solver
here uses the 2N-storage LSRK(5,4) of Carpenter & Kennedy (1994):
for stage s = 1..5
    res = a_s res + dt f(t + c_s dt, U)
    U   = U + b_s res
"""
from __future__ import annotations

import numpy as np

A = np.array([0.0,
              -567301805773.0 / 1357537059087.0,
              -2404267990393.0 / 2016746695238.0,
              -3550918686646.0 / 2091501179385.0,
              -1275806237668.0 / 842570457699.0])
B = np.array([1432997174477.0 / 9575080441755.0,
              5161836677717.0 / 13612068292357.0,
              1720146321549.0 / 2090206949498.0,
              3134564353537.0 / 4481467310338.0,
              2277821191437.0 / 14882151754819.0])
C = np.array([0.0,
              1432997174477.0 / 9575080441755.0,
              2526269341429.0 / 6820363962896.0,
              2006345519317.0 / 3224310063776.0,
              2802321613138.0 / 2924317926251.0])


def step(f, t: float, U: np.ndarray, res: np.ndarray, dt: float):
    """One step; f(t, U) -> dU/dt.  Updates U and res in place."""
    for s in range(5):
        res *= A[s]
        res += dt * f(t + C[s] * dt, U)
        U += B[s] * res
    return U, res


def integrate(f, U0: np.ndarray, dt: float, nsteps: int, t0: float = 0.0, after_step=None):
    """Run nsteps; after_step(n, t, U) is called after each completed step."""
    U = np.array(U0, dtype=np.float64, copy=True)
    res = np.zeros_like(U)
    t = t0
    for n in range(nsteps):
        step(f, t, U, res, dt)
        t = t0 + (n + 1) * dt
        if after_step is not None:
            after_step(n, t, U)
    return U, t
