"""FP64 reference of the explicit Runge-Kutta step (Sec. 7.1) on MPS (test
infrastructure only).

dy/dt = H y with H an MPO.  The classical fourth-order step
    k1 = H y, k2 = H (y + dt/2 k1), k3 = H (y + dt/2 k2), k4 = H (y + dt k3),
    y' = y + dt/6 (k1 + 2 k2 + 2 k3 + k4)
is written with every stage as an apply or a compressed linear combination
(H is linear, so H(y + a k) = H y + a H k), each compressed by the two-site
sweep of the oracle (`oracle.mps.apply_simplify`, `oracle.mps.combine`).
"""

from __future__ import annotations

from oracle import mps as om


def rk4_step(mpo, y, dt: float, max_bond: int, tol: float, sweeps: int = 2):
    k1 = om.apply_simplify(mpo, y, max_bond, tol, sweeps).mps
    k2 = om.combine([(1.0, mpo, y), (0.5 * dt, mpo, k1)], max_bond, tol, sweeps).mps
    k3 = om.combine([(1.0, mpo, y), (0.5 * dt, mpo, k2)], max_bond, tol, sweeps).mps
    k4 = om.combine([(1.0, mpo, y), (dt, mpo, k3)], max_bond, tol, sweeps).mps
    return om.combine([(1.0, None, y), (dt / 6.0, None, k1), (dt / 3.0, None, k2), (dt / 3.0, None, k3),
                       (dt / 6.0, None, k4)], max_bond, tol, sweeps).mps


def dense_rk4(H, v, dt: float, steps: int):
    """The same scheme on a dense vector with a dense matrix H."""
    y = v.copy()
    for _ in range(steps):
        k1 = H @ y
        k2 = H @ (y + 0.5 * dt * k1)
        k3 = H @ (y + 0.5 * dt * k2)
        k4 = H @ (y + dt * k3)
        y = y + dt / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
    return y
