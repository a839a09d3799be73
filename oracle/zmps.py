"""FP64 complex oracle of apply + compression (test infrastructure only).

The same method as `oracle.mps` route F (Sec. 2.3 Eq. simplification,
Sec. 2.4.2, Sec. 2.5) for complex MPS and MPO: the tensors are complex128 and
the environments contract the conjugate of the compressed state (the bra), so
that the local problem's minimiser is the projection
    theta = sum L[k] A_k B_k A_{k+1} B_{k+1} R[k+2]
with L, R built from conj(psi).  The split is the complex truncated SVD
(U S V^H) with the real truncation rule of `oracle.mps` on the singular
values; the sweep order, the guess (the input state, right-canonicalised by
QR) and the result (centre at site 0, not normalised) are those of route F.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg

from oracle.mps import REL_NORM2, chain, tail_sums, truncation_rank


def right_canonical(mps):
    """Right isometries on sites 1..L-1 by the QR factorisation of each site's
    transposed matrix, the triangular factor carried into the site on its left."""
    out = [np.array(A, dtype=np.complex128, copy=True) for A in mps]
    for k in range(len(out) - 1, 0, -1):
        a, s, b = out[k].shape
        q, r = np.linalg.qr(out[k].reshape(a, s * b).T)  # M^T = Q R, M = R^T Q^T
        m = q.shape[1]
        out[k] = q.T.reshape(m, s, b)
        out[k - 1] = np.einsum("xsa,ma->xsm", out[k - 1], r)
    return out


def scprod(a, b) -> complex:
    """<a, b> = sum conj(a) b by the transfer-matrix sweep (Sec. 2.4.4)."""
    E = np.ones((1, 1), dtype=np.complex128)
    for A, B in zip(a, b):
        E = chain("ab,asc,bsd->cd", E, np.conj(A), B)
    return complex(E[0, 0])


def norm_from_center(mps, center: int) -> float:
    return float(np.sqrt(np.sum(np.abs(mps[center]) ** 2)))


def _split(theta, a, s, t, c, tol, max_bond, mode, direction):
    M = theta.reshape(a * s, t * c)
    try:
        U, S, Vh = scipy.linalg.svd(M, full_matrices=False, lapack_driver="gesdd")
    except np.linalg.LinAlgError:
        U, S, Vh = scipy.linalg.svd(M, full_matrices=False, lapack_driver="gesvd")
    r = truncation_rank(S, tol, max_bond, mode)
    delta = float(tail_sums(S)[r])
    if direction > 0:
        return U[:, :r].reshape(a, s, r), (S[:r, None] * Vh[:r]).reshape(r, t, c), r, delta
    return (U[:, :r] * S[None, :r]).reshape(a, s, r), Vh[:r].reshape(r, t, c), r, delta


def apply_simplify(mpo, mps, max_bond: int, tol: float, sweeps: int = 4, mode: int = REL_NORM2):
    """Returns (state with centre at site 0, its norm, per-step discarded weights)."""
    L = len(mps)
    A = [np.asarray(x, dtype=np.complex128) for x in mps]
    B = [np.asarray(x, dtype=np.complex128) for x in mpo]
    psi = right_canonical(A)
    one = np.ones((1, 1, 1), dtype=np.complex128)
    Lenv = [None] * (L + 1)
    Renv = [None] * (L + 1)
    Lenv[0] = one
    Renv[L] = one

    def grow_left(E, P, Bk, Ak):
        return chain("abx,asc,bspd,xpy->cdy", E, np.conj(P), Bk, Ak)

    def grow_right(E, P, Bk, Ak):
        return chain("cdy,asc,bspd,xpy->abx", E, np.conj(P), Bk, Ak)

    if L == 1:
        psi[0] = np.einsum("bspd,xpy->bxsdy", B[0], A[0]).reshape(1, B[0].shape[1], 1)
        return psi, norm_from_center(psi, 0), []
    for k in range(L - 1, 0, -1):
        Renv[k] = grow_right(Renv[k + 1], psi[k], B[k], A[k])
    deltas = []
    for _ in range(sweeps):
        for direction, bonds in ((+1, range(0, L - 1)), (-1, range(L - 2, -1, -1))):
            for k in bonds:
                th = chain("abx,xpy,bspe,yqz,etqf,cfz->astc",
                           Lenv[k], A[k], B[k], A[k + 1], B[k + 1], Renv[k + 2])
                a, s, t, c = th.shape
                psi[k], psi[k + 1], r, delta = _split(th, a, s, t, c, tol, max_bond, mode, direction)
                deltas.append(delta)
                if direction > 0:
                    Lenv[k + 1] = grow_left(Lenv[k], psi[k], B[k], A[k])
                else:
                    Renv[k + 1] = grow_right(Renv[k + 2], psi[k + 1], B[k + 1], A[k + 1])
    return psi, norm_from_center(psi, 0), deltas
