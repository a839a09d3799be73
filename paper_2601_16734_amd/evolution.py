"""Explicit time steppers built on apply + compression (Sec. 7.1).

dy/dt = H y with H an MPO (e.g. the finite-difference Laplacian of Sec. 5.1
for the diffusion equation).  Every stage is an apply or the compression of a
linear combination (smps_mpo_apply / smps_combine); this module only strings
the library calls together, all arithmetic runs in the library.
"""

from __future__ import annotations

from . import binding as B


def euler_step(ctx: B.Context, H: B.MPO, y: B.MPS, dt: float, st: B.Strategy) -> B.MPS:
    """y + dt H y."""
    out, _ = ctx.combine([(1.0, None, y), (dt, H, y)], st)
    return out


def rk4_step(ctx: B.Context, H: B.MPO, y: B.MPS, dt: float, st: B.Strategy) -> B.MPS:
    """Classical fourth-order Runge-Kutta step, with the stages written as
    compressions of linear combinations (H is linear, so H(y + a k) = Hy + a Hk):
        k1 = H y
        k2 = H y + dt/2 H k1
        k3 = H y + dt/2 H k2
        k4 = H y + dt   H k3
        y' = y + dt/6 (k1 + 2 k2 + 2 k3 + k4)."""
    k1, _ = ctx.mpo_apply(H, y, st)
    k2, _ = ctx.combine([(1.0, H, y), (0.5 * dt, H, k1)], st)
    k3, _ = ctx.combine([(1.0, H, y), (0.5 * dt, H, k2)], st)
    k4, _ = ctx.combine([(1.0, H, y), (dt, H, k3)], st)
    out, _ = ctx.combine([(1.0, None, y), (dt / 6.0, None, k1), (dt / 3.0, None, k2), (dt / 3.0, None, k3),
                          (dt / 6.0, None, k4)], st)
    for k in (k1, k2, k3, k4):
        k.destroy()
    return out
