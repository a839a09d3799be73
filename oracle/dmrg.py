"""FP64 reference of two-site DMRG (Sec. 3.1.1) for real symmetric MPOs
(test infrastructure only).

With the state in mixed canonical form around the pair (k, k+1), the norm
form of the pair is the identity and the local problem is H_k a = E a with
    (H_k a)[a', s', t', c'] = sum L[k][a', b, a] W_k[b, s', s, b']
                                  W_{k+1}[b', t', t, b''] R[k+2][c', b'', c] a[a, s, t, c],
L and R the three-layer environments of <psi | H | psi>.  The lowest
eigenvector of the dense H_k (LAPACK `eigh`) replaces the pair, which is
split by the truncated SVD of route F's split and the centre moves on;
sweeps go left to right then right to left.  The guess is right-
canonicalised and normalised first.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg

from oracle.mps import REL_NORM2, _split, chain, norm_from_center, right_canonical


def dmrg(mpo, guess, max_bond: int, tol: float, sweeps: int = 4, mode: int = REL_NORM2):
    """Returns (energy after the last step, state canonical at site 0, energies per step)."""
    L = len(guess)
    W = [np.asarray(x, dtype=np.float64) for x in mpo]
    psi = right_canonical([np.asarray(x, dtype=np.float64) for x in guess])
    psi[0] = psi[0] / norm_from_center(psi, 0)
    one = np.ones((1, 1, 1))
    Lenv = [None] * (L + 1)
    Renv = [None] * (L + 1)
    Lenv[0] = one
    Renv[L] = one

    def grow_left(E, P, Wk):
        return chain("abx,asc,bspd,xpy->cdy", E, P, Wk, P)

    def grow_right(E, P, Wk):
        return chain("cdy,asc,bspd,xpy->abx", E, P, Wk, P)

    for k in range(L - 1, 0, -1):
        Renv[k] = grow_right(Renv[k + 1], psi[k], W[k])
    energies = []
    E = float("nan")
    for _ in range(sweeps):
        for direction, bonds in ((+1, range(0, L - 1)), (-1, range(L - 2, -1, -1))):
            for k in bonds:
                a, s = psi[k].shape[0], psi[k].shape[1]
                t, c = psi[k + 1].shape[1], psi[k + 1].shape[2]
                Heff = chain("xby,bspe,etqf,wfz->xstwypqz", Lenv[k], W[k], W[k + 1], Renv[k + 2])
                # rows (a', s', t', c'), columns (a, s, t, c)
                Hm = Heff.reshape(a * s * t * c, a * s * t * c)
                Hm = 0.5 * (Hm + Hm.T)
                vals, vecs = scipy.linalg.eigh(Hm)
                E = float(vals[0])
                energies.append(E)
                th = vecs[:, 0].reshape(a, s, t, c)
                left, right, r, delta, S = _split(th, a, s, t, c, tol, max_bond, mode, direction)
                psi[k], psi[k + 1] = left, right
                if direction > 0:
                    Lenv[k + 1] = grow_left(Lenv[k], psi[k], W[k])
                else:
                    Renv[k + 1] = grow_right(Renv[k + 2], psi[k + 1], W[k + 1])
    return E, psi, energies


def xx_chain_ground_energy(J: float, L: int) -> float:
    """Closed form for H = J sum_i (X_i X_{i+1} + Y_i Y_{i+1}), open chain:
    by the Jordan-Wigner map the model is free fermions with hopping 2J,
    single-particle energies 4 J cos(k pi / (L + 1)), k = 1..L, and the ground
    state fills every negative level."""
    eps = 4.0 * J * np.cos(np.arange(1, L + 1) * np.pi / (L + 1))
    return float(np.sum(eps[eps < 0]))


def tfim_ground_energy(L: int, J: float = 1.0, h: float = 1.0) -> float:
    """Closed form for H = -J sum Z_i Z_{i+1} - h sum X_i, open chain
    (Lieb, Schultz & Mattis 1961; Pfeuty 1970).  With Majorana operators
    a_i, b_i of the Jordan-Wigner fermions, X_i = -i a_i b_i and
    Z_i Z_{i+1} = -i b_i a_{i+1}, so H = (i/4) gamma^T A gamma with A real
    antisymmetric and tridiagonal along (a_1, b_1, a_2, ..., b_L), its
    off-diagonal entries alternating 2h (within a site) and 2J (between sites).
    The ground energy is -1/4 of the sum of the absolute eigenvalues of iA;
    on this path graph a diagonal sign change maps A to the symmetric
    tridiagonal matrix with the same off-diagonal magnitudes, so those are its
    absolute eigenvalues."""
    off = np.empty(2 * L - 1)
    off[0::2] = 2.0 * h
    off[1::2] = 2.0 * J
    ev = scipy.linalg.eigh_tridiagonal(np.zeros(2 * L), off, eigvals_only=True)
    return float(-0.25 * np.sum(np.abs(ev)))
