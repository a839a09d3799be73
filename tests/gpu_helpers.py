"""Comparison helpers for GPU-vs-oracle parity tests (host side)."""

import numpy as np

from oracle import mps as om


def cross_fidelity_loss(a, b) -> float:
    """1 - |<a,b>| / (||a|| ||b||) from host site tensors (oracle scalar product)."""
    ab = om.scprod(a, b)
    aa = om.scprod(a, a)
    bb = om.scprod(b, b)
    return float(1.0 - abs(ab) / np.sqrt(aa * bb))


def rel_norm_err(a_norm: float, b_norm: float) -> float:
    return abs(a_norm - b_norm) / abs(b_norm)


def isometry_residual_right(t) -> float:
    a, s, b = t.shape
    M = t.reshape(a, s * b)
    return float(np.abs(M @ M.T - np.eye(a)).max())
