"""FP64 reference of the randomized factorization and of its Gaussian sketch
(test infrastructure only).

The paper's only randomized method is its sketching-based function encoding
(Sec. 4.6, sketching methods); the randomized SVD used
here to cut the cost of the two-site split is the range finder with subspace
iteration of Halko, Martinsson & Tropp (SIAM Rev. 53(2), 2011, Alg. 4.4 and
Sec. 5.1), written for the row space of X (nvec x len):

    Y = G X                         G: k x nvec standard Gaussian
    P = orth(Y);  repeat q times:  P = orth((P X^T) X)
    B = P X^T = W diag(s) Z^T       small SVD
    Q = W[:, :r]^T P                r from the truncation rule

with q = 0 (POWER_ITERS): the device orthonormalises through Gram matrices,
which square the condition number, and a power step would square it again.

with ||X||_F^2 - sum_{j<r} s_j^2 as the (exact) discarded weight.  The step
is accepted when that weight is within the tolerance (relative-norm rule) and
r <= k - p/2 (p = oversampling); otherwise the caller falls back to the exact
SVD.

Gaussians come from the counter-based generator Philox4x64-10 (Salmon,
Moraes, Dror & Shaw, SC'11): entry n of the k x nvec matrix (row-major) uses
block n // 4 with counter (n // 4, step, 0, 0) and key SKETCH_KEY; the four
64-bit outputs give uniforms u = ((x >> 11) + 1/2) 2^-53 and two Box-Muller
pairs (u0, u1) -> (rho cos, rho sin), (u2, u3) -> (rho cos, rho sin),
rho = sqrt(-2 ln u_first), angle = 2 pi u_second.  Lane n % 4 picks the value.
"""

from __future__ import annotations

import numpy as np

from oracle.mps import REL_NORM2, REL_SV, svd_desc

PHILOX_M = (0xD2E7470EE14C6C93, 0xCA5A826395121157)
PHILOX_W = (0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B)
SKETCH_KEY = (0x0260116734000001, 0x00000000005EE95D)
OVERSAMPLE = 16
POWER_ITERS = 0
# the learned rank is raised by this factor before oversampling (a sketch
# below the rank is refused and redone exactly; one above it costs columns)
PREDICT_MARGIN = 1.25
M64 = (1 << 64) - 1


def philox4x64_10_scalar(ctr, key):
    """Philox4x64 with 10 rounds on Python integers (one block)."""
    x = [int(c) & M64 for c in ctr]
    k = [int(c) & M64 for c in key]
    for rnd in range(10):
        if rnd:
            k = [(k[0] + PHILOX_W[0]) & M64, (k[1] + PHILOX_W[1]) & M64]
        p0 = PHILOX_M[0] * x[0]
        p1 = PHILOX_M[1] * x[2]
        x = [(p1 >> 64) ^ x[1] ^ k[0], p1 & M64, (p0 >> 64) ^ x[3] ^ k[1], p0 & M64]
    return x


def _mulhilo(a, b):
    """Full 64 x 64 -> 128-bit products of uint64 arrays, as (hi, lo)."""
    m32 = np.uint64(0xFFFFFFFF)
    s32 = np.uint64(32)
    a_lo, a_hi = a & m32, a >> s32
    b_lo, b_hi = b & m32, b >> s32
    t = a_lo * b_lo
    u = a_hi * b_lo + (t >> s32)
    v = a_lo * b_hi + (u & m32)
    hi = a_hi * b_hi + (u >> s32) + (v >> s32)
    return hi, a * b


def philox4x64_10(c0, c1, c2, c3, key):
    """Vectorised Philox4x64-10 over uint64 counter arrays."""
    with np.errstate(over="ignore"):
        x = [np.asarray(c, dtype=np.uint64).copy() for c in (c0, c1, c2, c3)]
        k0, k1 = np.uint64(key[0]), np.uint64(key[1])
        M0, M1 = np.uint64(PHILOX_M[0]), np.uint64(PHILOX_M[1])
        for rnd in range(10):
            if rnd:
                k0 = k0 + np.uint64(PHILOX_W[0])
                k1 = k1 + np.uint64(PHILOX_W[1])
            hi0, lo0 = _mulhilo(np.broadcast_to(M0, x[0].shape), x[0])
            hi1, lo1 = _mulhilo(np.broadcast_to(M1, x[2].shape), x[2])
            x = [hi1 ^ x[1] ^ k0, lo1, hi0 ^ x[3] ^ k1, lo0]
    return x


def uniforms(x):
    return ((x >> np.uint64(11)).astype(np.float64) + 0.5) * 2.0 ** -53


def gaussians(step: int, n: int, key=SKETCH_KEY) -> np.ndarray:
    """The first n values of the sketch stream of factorization step `step`."""
    nb = (n + 3) // 4
    b = np.arange(nb, dtype=np.uint64)
    z = np.zeros(nb, dtype=np.uint64)
    out = philox4x64_10(b, np.full(nb, step, dtype=np.uint64), z, z, key)
    u = [uniforms(o) for o in out]
    rho0 = np.sqrt(-2.0 * np.log(u[0]))
    rho1 = np.sqrt(-2.0 * np.log(u[2]))
    a0 = 2.0 * np.pi * u[1]
    a1 = 2.0 * np.pi * u[3]
    g = np.stack([rho0 * np.cos(a0), rho0 * np.sin(a0), rho1 * np.cos(a1), rho1 * np.sin(a1)], axis=1)
    return g.reshape(-1)[:n]


def orth_rows(Y, floor_eps: float = 2.0 ** -52):
    """Orthonormal basis (rows) of the row space of Y, dropping directions
    with singular value at most floor_eps * max(m, n) * ||Y||_F."""
    if Y.size == 0:
        return Y[:0]
    _, s, Vt = svd_desc(Y)
    f = floor_eps * max(Y.shape) * np.sqrt(np.sum(Y * Y))
    return Vt[s > f]


def rank_with_total(s, total: float, tol: float, max_rank: int, mode: int):
    """Truncation rule on approximate singular values when the exact total
    weight is known: the weight missed by s is counted in every tail.
    Returns (r, discarded weight)."""
    s = np.asarray(s, dtype=np.float64)
    n = len(s)
    sq = s * s
    missed = max(0.0, total - float(np.sum(sq[::-1])))
    tails = np.zeros(n + 1)
    acc = 0.0
    for j in range(n - 1, -1, -1):
        acc += sq[j]
        tails[j] = acc
    if mode == REL_NORM2:
        thr = tol * total
        r = n
        for cand in range(1, n + 1):
            if missed + tails[cand] <= thr:
                r = cand
                break
    elif mode == REL_SV:
        r = int(np.sum(s > tol * s[0])) if n else 0
    else:
        raise ValueError(mode)
    r = max(1, min(r, max_rank, n))
    return r, missed + tails[r]


def rsvd_rows(X, k: int, tol: float, max_rank: int, mode: int, step: int,
              oversample: int = OVERSAMPLE, power: int = POWER_ITERS):
    """Randomized truncated factorization of the row space of X (see the
    module docstring).  Returns (Q r x len, s, r, delta, accepted)."""
    X = np.asarray(X, dtype=np.float64)
    nvec, _ = X.shape
    G = gaussians(step, k * nvec).reshape(k, nvec)
    P = orth_rows(G @ X)
    for _ in range(power):
        P = orth_rows((P @ X.T) @ X)
    Bm = P @ X.T
    W, s, _ = svd_desc(Bm)
    total = float(np.sum(X * X))
    r, delta = rank_with_total(s, total, tol, max_rank, mode)
    Q = W[:, :r].T @ P
    ok = r <= k - oversample // 2
    if mode == REL_NORM2:
        ok = ok and delta <= tol * total
    return Q, s, r, float(delta), bool(ok)


class SketchedSplit:
    """Split hook for oracle.mps.apply_simplify that follows the randomized
    factorization schedule.  The first left-to-right pass is exact.  Later
    steps predict the rank r_hat from the bond's previous split: the kept
    rank there (predictor None) or ceil(1.25 exp(predictor(features))) clipped to
    [1, min(max_bond, m, n)]; r_hat at that cap means the exact SVD.  With
    fixed=True there is no estimate: r_hat = min(max_bond, m, n).  A sketch
    k = r_hat + p of at least min(m, n) rows means the exact SVD.  kinds[step] records
    0 / +k accepted / -k replaced by the exact SVD."""

    def __init__(self, max_bond: int, tol: float, mode: int = REL_NORM2, predictor=None, fixed: bool = False):
        self.max_bond, self.tol, self.mode, self.predictor = max_bond, tol, mode, predictor
        self.fixed = fixed
        self.kinds = []

    def sketch_size(self, prev, nv, ln):
        lim = min(nv, ln, self.max_bond)
        if self.fixed:  # no rank estimate: the sketch covers the cap
            k = lim + OVERSAMPLE
            return k if k < min(nv, ln) else 0
        spectrum, rank = prev
        if self.predictor is None:
            rhat = min(lim, rank)
        else:
            from oracle.mlp import features
            lr = min(30.0, max(0.0, float(self.predictor(features(spectrum)))))
            rhat = int(min(lim, np.ceil(PREDICT_MARGIN * np.exp(lr))))
        rhat = max(1, rhat)
        if rhat >= lim:
            return 0
        k = rhat + OVERSAMPLE
        return k if k < min(nv, ln) else 0

    def __call__(self, th, bond, direction, sweep, step, prev):
        if sweep == 0 and direction > 0:
            self.kinds.append(0)
            return None
        a, s, t, c = th.shape
        M = th.reshape(a * s, t * c)
        X = M.T if direction > 0 else M
        k = self.sketch_size(prev, *X.shape)
        if k == 0:
            self.kinds.append(0)
            return None
        Q, sv, r, delta, ok = rsvd_rows(X, k, self.tol, self.max_bond, self.mode, step)
        if not ok:
            self.kinds.append(-k)
            return None
        self.kinds.append(k)
        if direction > 0:
            return Q.T.reshape(a, s, r), (Q @ M).reshape(r, t, c), r, delta, sv
        return (M @ Q.T).reshape(a, s, r), Q.reshape(r, t, c), r, delta, sv
