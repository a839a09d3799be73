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


def error_bound_slack(ref) -> float:
    """Allowance for the accumulated error bound sum_k sqrt(delta_k) (Sec. 2.3)
    beyond its relative agreement: at a step whose two-site tensor is
    numerically rank-deficient the discarded weight is rounding noise, which
    the Gram-matrix split resolves to about 1e-18 ||theta||^2 (singular values
    to about eps ||theta|| times the condition number of the kept part) where
    LAPACK on theta resolves it to eps^2 ||theta||^2; sqrt of that noise is
    summed over the steps."""
    return float(sum(1e-9 * np.sqrt(n2 + d) for n2, d in zip(ref.norms2, ref.deltas)))
