"""FP64 oracle of the MPS-BLAS pieces on the apply + compression path.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper passages followed:
  * Sec. 2.1 / 2.2 -- MPS and MPO tensor layouts, open boundaries.
  * Sec. 2.3 -- canonical form (left/right isometries around a centre k),
    truncation by maximum bond and tolerance, the variational problem
    Eq. (simplification), the accumulated error bound kept with the state.
  * Sec. 2.4.2, Eq. (MPO-times-MPS) -- exact product tensors C with the
    combined index gamma = beta * chi_A + alpha (alpha fastest).
  * Sec. 2.4.4 -- scalar product by a transfer-matrix sweep; the norm of a
    canonical MPS from its centre tensor alone.
  * Sec. 2.5, Eqs. (single-site-linear), (single-site-quadratic) -- the
    two-site reduction with cached left/right environments, and the sweep
    (left-to-right then right-to-left) of local quadratic problems.

Readings where the paper is silent (each is listed in the design notes):
  * truncation rule REL_NORM2 (default): the smallest r >= 1 whose discarded
    tail sum_{j>=r} s_j^2 (summed smallest first) is <= tol * sum_j s_j^2,
    then r <- min(r, max_bond).  REL_SV keeps s_j > tol * s_0 (at least one).
  * initial guess: the input MPS itself, brought to right-canonical form by QR.
  * a sweep is one left-to-right pass over bonds 0..L-2 followed by one
    right-to-left pass over bonds L-2..0; the result has its centre at site 0
    and is not normalised.
  * error bound: sum over steps of sqrt(discarded weight of the step).
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg

REL_NORM2 = 0
REL_SV = 1


def chain(spec: str, *ops):
    """np.einsum(spec, *ops) evaluated by contracting the operands pairwise from
    left to right (each pair through BLAS); the order of the operands in the
    spec is the order of contraction."""
    ins, out = spec.split("->")
    terms = ins.split(",")
    cur, cur_t = ops[0], terms[0]
    for i in range(1, len(ops)):
        nxt = terms[i]
        later = set("".join(terms[i + 1:])) | set(out)
        keep = "".join(ch for ch in dict.fromkeys(cur_t + nxt) if ch in later)
        cur = np.einsum(f"{cur_t},{nxt}->{keep}", cur, ops[i], optimize=True)
        cur_t = keep
    return np.einsum(f"{cur_t}->{out}", cur)


# ---------------------------------------------------------------------------
# Scalar product and norm (Sec. 2.4.4)
# ---------------------------------------------------------------------------

def scprod(a, b) -> float:
    """<a, b> by the transfer-matrix sweep E_{k+1} = sum E_k a_k b_k, O(L chi^3 d)."""
    E = np.ones((1, 1))
    for A, B in zip(a, b):
        E = chain("ab,asc,bsd->cd", E, A.conj(), B)
    return float(E[0, 0].real) if np.isrealobj(E) else E[0, 0]


def norm_from_center(mps, center: int) -> float:
    """For a canonical MPS the squared norm is the squared Frobenius norm of
    the centre tensor (Sec. 2.4.4)."""
    return float(np.sqrt(np.sum(np.abs(mps[center]) ** 2)))


# ---------------------------------------------------------------------------
# Canonical form (Sec. 2.3)
# ---------------------------------------------------------------------------

def is_left_isometry(A, atol=1e-12) -> bool:
    a, s, b = A.shape
    M = A.reshape(a * s, b)
    return bool(np.allclose(M.T @ M, np.eye(b), atol=atol))


def is_right_isometry(A, atol=1e-12) -> bool:
    a, s, b = A.shape
    M = A.reshape(a, s * b)
    return bool(np.allclose(M @ M.T, np.eye(a), atol=atol))


def right_canonical(mps):
    """Move the isometry centre to site 0: for k = L-1..1 write the site as
    M = (chi_l) x (d chi_r), take the QR factorisation of M^T = Q R so that
    M = R^T Q^T, keep Q^T as a right isometry and absorb R^T into site k-1."""
    out = [np.array(A, dtype=np.float64, copy=True) for A in mps]
    for k in range(len(out) - 1, 0, -1):
        a, s, b = out[k].shape
        q, r = np.linalg.qr(out[k].reshape(a, s * b).T)  # (s b, m), (m, a)
        m = q.shape[1]
        out[k] = q.T.reshape(m, s, b)
        out[k - 1] = np.einsum("xsa,ma->xsm", out[k - 1], r)
    return out


# ---------------------------------------------------------------------------
# Truncation (Sec. 2.3)
# ---------------------------------------------------------------------------

def tail_sums(s) -> np.ndarray:
    """t[r] = sum_{j>=r} s_j^2 accumulated from the smallest value upwards;
    t has len(s)+1 entries and t[len(s)] = 0."""
    sq = np.asarray(s, dtype=np.float64) ** 2
    t = np.zeros(len(sq) + 1)
    acc = 0.0
    for j in range(len(sq) - 1, -1, -1):
        acc = acc + sq[j]
        t[j] = acc
    return t


def truncation_rank(s, tol: float, max_bond: int, mode: int = REL_NORM2) -> int:
    """Kept rank for descending singular values s."""
    n = len(s)
    if n == 0:
        return 0
    if mode == REL_NORM2:
        t = tail_sums(s)
        thr = tol * t[0]
        r = n
        for cand in range(1, n + 1):
            if t[cand] <= thr:
                r = cand
                break
    elif mode == REL_SV:
        r = int(np.sum(np.asarray(s) > tol * s[0]))
    else:
        raise ValueError(mode)
    r = max(1, r)
    return min(r, int(max_bond))


def svd_desc(M):
    """SVD with descending singular values; gesdd, falling back to gesvd."""
    try:
        return scipy.linalg.svd(M, full_matrices=False, lapack_driver="gesdd")
    except np.linalg.LinAlgError:
        return scipy.linalg.svd(M, full_matrices=False, lapack_driver="gesvd")


# ---------------------------------------------------------------------------
# Exact MPO x MPS (Sec. 2.4.2, Eq. MPO-times-MPS)
# ---------------------------------------------------------------------------

def mpo_times_mps(mpo, mps):
    """C[gamma, j, gamma'] = sum_i B[beta, j, i, beta'] A[alpha, i, alpha'],
    gamma = beta * chi_A + alpha (alpha is the fastest running index)."""
    out = []
    for B, A in zip(mpo, mps):
        Dl, J, I, Dr = B.shape
        al, _, ar = A.shape
        C = np.einsum("bjic,xiy->bxjcy", B, A)  # (beta, alpha, j, beta', alpha')
        out.append(C.reshape(Dl * al, J, Dr * ar))
    return out


# ---------------------------------------------------------------------------
# Two-site variational sweep (Sec. 2.3 Eq. simplification; Sec. 2.5)
# ---------------------------------------------------------------------------

@dataclass
class SweepResult:
    mps: list                # compressed MPS, centre at site 0
    norm: float              # Frobenius norm of the centre tensor
    ranks: list              # final bond dimensions, len L+1
    deltas: list = field(default_factory=list)     # discarded weight per step
    norms2: list = field(default_factory=list)     # ||psi||^2 after each step
    spectra: list = field(default_factory=list)    # (sweep, direction, bond, s)
    step_ranks: list = field(default_factory=list)  # kept rank of each step
    error_bound: float = 0.0

    @property
    def total_discarded(self) -> float:
        return float(np.sum(self.deltas))


def _split(theta, a, s, t, c, tol, max_bond, mode, direction):
    """Factor the two-site tensor as a truncated SVD; returns the new pair,
    the kept rank, the discarded weight and the singular values."""
    U, S, Vt = svd_desc(theta.reshape(a * s, t * c))
    r = truncation_rank(S, tol, max_bond, mode)
    delta = tail_sums(S)[r]
    if direction > 0:   # centre moves right: left site is an isometry
        left = U[:, :r].reshape(a, s, r)
        right = (S[:r, None] * Vt[:r]).reshape(r, t, c)
    else:               # centre moves left: right site is an isometry
        left = (U[:, :r] * S[None, :r]).reshape(a, s, r)
        right = Vt[:r].reshape(r, t, c)
    return left, right, r, float(delta), S


def apply_simplify(mpo, mps, max_bond: int, tol: float, sweeps: int = 4,
                   mode: int = REL_NORM2, guess=None, split_hook=None, max_steps=None) -> SweepResult:
    """Route F: compress U v with three-layer environments <psi | U | v>.

    L[k][a, b, x] contracts sites < k of psi (a), U (b) and v (x);
    R[k][a, b, x] contracts sites >= k.  With psi in mixed canonical form
    around the pair (k, k+1), the quadratic term of the local problem is the
    identity and its minimiser is the projection
        theta[a,s,t,c] = sum L[k][a,b,x] A_k[x,p,y] B_k[b,s,p,b']
                             A_{k+1}[y,q,z] B_{k+1}[b',t,q,b''] R[k+2][c,b'',z],
    which is split by a truncated SVD and the centre moved on.

    split_hook (optional) may replace the exact split of a step: it is called
    as split_hook(theta, bond, direction, sweep, step, previous) with previous
    = (spectrum, kept rank) of the bond's last split, or None, and returns
    None (exact split) or (left, right, r, delta, s).

    max_steps (optional) stops after that many two-site steps, leaving the
    per-step log of those steps (the state is then not a finished result).
    """
    L = len(mps)
    A = [np.asarray(x, dtype=np.float64) for x in mps]
    B = [np.asarray(x, dtype=np.float64) for x in mpo]
    psi = right_canonical(A if guess is None else guess)
    one = np.ones((1, 1, 1))
    Lenv = [None] * (L + 1)
    Renv = [None] * (L + 1)
    Lenv[0] = one
    Renv[L] = one

    def grow_left(E, P, Bk, Ak):
        return chain("abx,asc,bspd,xpy->cdy", E, P, Bk, Ak)

    def grow_right(E, P, Bk, Ak):
        return chain("cdy,asc,bspd,xpy->abx", E, P, Bk, Ak)

    for k in range(L - 1, 0, -1):
        Renv[k] = grow_right(Renv[k + 1], psi[k], B[k], A[k])

    res = SweepResult(mps=psi, norm=0.0, ranks=[])
    if L == 1:
        theta = np.einsum("bspd,xpy->bxsdy", B[0], A[0]).reshape(1, B[0].shape[1], 1)
        psi[0] = theta
        res.norm = norm_from_center(psi, 0)
        res.ranks = [1, 1]
        return res

    def theta_at(k):
        return chain("abx,xpy,bspe,yqz,etqf,cfz->astc",
                     Lenv[k], A[k], B[k], A[k + 1], B[k + 1], Renv[k + 2])

    last_spectrum = {}
    step = 0
    for sw in range(sweeps):
        for direction, bonds in ((+1, range(0, L - 1)), (-1, range(L - 2, -1, -1))):
            for k in bonds:
                th = theta_at(k)
                a, s, t, c = th.shape
                got = None
                if split_hook is not None:
                    got = split_hook(th, k, direction, sw, step, last_spectrum.get(k))
                if got is None:
                    got = _split(th, a, s, t, c, tol, max_bond, mode, direction)
                left, right, r, delta, S = got
                last_spectrum[k] = (S, r)
                step += 1
                res.step_ranks.append(r)
                psi[k], psi[k + 1] = left, right
                res.deltas.append(delta)
                res.norms2.append(float(np.sum(S[:r] ** 2)))
                res.spectra.append((sw, direction, k, S))
                if max_steps is not None and step >= max_steps:
                    res.mps = psi
                    res.norm = float("nan")
                    return res
                if direction > 0:
                    Lenv[k + 1] = grow_left(Lenv[k], psi[k], B[k], A[k])
                else:
                    Renv[k + 1] = grow_right(Renv[k + 2], psi[k + 1], B[k + 1], A[k + 1])
    res.mps = psi
    res.norm = norm_from_center(psi, 0)
    res.ranks = [1] + [p.shape[2] for p in psi]
    res.error_bound = float(np.sum(np.sqrt(res.deltas)))
    return res


def apply_simplify_explicit(mpo, mps, max_bond: int, tol: float, sweeps: int = 4,
                            mode: int = REL_NORM2) -> SweepResult:
    """Route C: first form the exact product C (Eq. MPO-times-MPS), then
    compress it with two-layer environments <psi | C> (Eq. single-site-linear).
    Same guess, same sweep order and the same split as route F."""
    L = len(mps)
    C = mpo_times_mps(mpo, mps)
    psi = right_canonical([np.asarray(x, dtype=np.float64) for x in mps])
    Lenv = [None] * (L + 1)
    Renv = [None] * (L + 1)
    Lenv[0] = np.ones((1, 1))
    Renv[L] = np.ones((1, 1))
    for k in range(L - 1, 0, -1):
        Renv[k] = chain("cg,asc,hsg->ah", Renv[k + 1], psi[k], C[k])
    res = SweepResult(mps=psi, norm=0.0, ranks=[])
    for sw in range(sweeps):
        for direction, bonds in ((+1, range(0, L - 1)), (-1, range(L - 2, -1, -1))):
            for k in bonds:
                th = chain("ag,gsh,hti,ci->astc", Lenv[k], C[k], C[k + 1], Renv[k + 2])
                a, s, t, c = th.shape
                left, right, r, delta, S = _split(th, a, s, t, c, tol, max_bond, mode, direction)
                psi[k], psi[k + 1] = left, right
                res.deltas.append(delta)
                res.norms2.append(float(np.sum(S[:r] ** 2)))
                if direction > 0:
                    Lenv[k + 1] = chain("ag,asc,gsh->ch", Lenv[k], psi[k], C[k])
                else:
                    Renv[k + 1] = chain("cg,asc,hsg->ah", Renv[k + 2], psi[k + 1], C[k + 1])
    res.mps = psi
    res.norm = norm_from_center(psi, 0)
    res.ranks = [1] + [p.shape[2] for p in psi]
    res.error_bound = float(np.sum(np.sqrt(res.deltas)))
    return res


def combine(terms, max_bond: int, tol: float, sweeps: int = 4, mode: int = REL_NORM2) -> SweepResult:
    """Compression of a linear combination (Sec. 2.4.1, Eq. mps-sum-opt):
    psi ~ sum_l w_l U_l v_l, terms = [(w_l, mpo_l or None, mps_l)], by the
    two-site sweep of route F with one set of three-layer environments per
    term; the local minimiser is the sum of the terms' projections,
    theta = sum_l w_l theta_l.  The guess is the first term's state."""
    L = len(terms[0][2])
    T = []
    for w, mpo, mps in terms:
        A = [np.asarray(x, dtype=np.float64) for x in mps]
        if mpo is None:
            B = [np.eye(a.shape[1]).reshape(1, a.shape[1], a.shape[1], 1) for a in A]
        else:
            B = [np.asarray(x, dtype=np.float64) for x in mpo]
        T.append((float(w), B, A))
    psi = right_canonical(T[0][2])
    one = np.ones((1, 1, 1))
    Lenv = [[None] * (L + 1) for _ in T]
    Renv = [[None] * (L + 1) for _ in T]
    for i in range(len(T)):
        Lenv[i][0] = one
        Renv[i][L] = one

    def grow_left(E, P, Bk, Ak):
        return chain("abx,asc,bspd,xpy->cdy", E, P, Bk, Ak)

    def grow_right(E, P, Bk, Ak):
        return chain("cdy,asc,bspd,xpy->abx", E, P, Bk, Ak)

    for i, (_, B, A) in enumerate(T):
        for k in range(L - 1, 0, -1):
            Renv[i][k] = grow_right(Renv[i][k + 1], psi[k], B[k], A[k])
    res = SweepResult(mps=psi, norm=0.0, ranks=[])
    if L == 1:
        psi[0] = sum(w * np.einsum("bspd,xpy->bxsdy", B[0], A[0]).reshape(1, B[0].shape[1], 1)
                     for w, B, A in T)
        res.norm = norm_from_center(psi, 0)
        res.ranks = [1, 1]
        return res
    for sw in range(sweeps):
        for direction, bonds in ((+1, range(0, L - 1)), (-1, range(L - 2, -1, -1))):
            for k in bonds:
                th = sum(w * chain("abx,xpy,bspe,yqz,etqf,cfz->astc", Lenv[i][k], A[k], B[k], A[k + 1],
                                   B[k + 1], Renv[i][k + 2])
                         for i, (w, B, A) in enumerate(T))
                a, s, t, c = th.shape
                left, right, r, delta, S = _split(th, a, s, t, c, tol, max_bond, mode, direction)
                psi[k], psi[k + 1] = left, right
                res.deltas.append(delta)
                res.norms2.append(float(np.sum(S[:r] ** 2)))
                res.step_ranks.append(r)
                for i, (_, B, A) in enumerate(T):
                    if direction > 0:
                        Lenv[i][k + 1] = grow_left(Lenv[i][k], psi[k], B[k], A[k])
                    else:
                        Renv[i][k + 1] = grow_right(Renv[i][k + 2], psi[k + 1], B[k + 1], A[k + 1])
    res.mps = psi
    res.norm = norm_from_center(psi, 0)
    res.ranks = [1] + [p.shape[2] for p in psi]
    res.error_bound = float(np.sum(np.sqrt(res.deltas)))
    return res


def simplify(mps, max_bond: int, tol: float, sweeps: int = 4, mode: int = REL_NORM2) -> SweepResult:
    """Compression of a single MPS (Eq. simplification with phi = v): the same
    sweep with the identity operator (bond 1)."""
    d = [A.shape[1] for A in mps]
    ident = [np.eye(x).reshape(1, x, x, 1) for x in d]
    return apply_simplify(ident, mps, max_bond, tol, sweeps, mode)


# ---------------------------------------------------------------------------
# TT-SVD of a dense vector (Oseledets 2011), used as a quality reference
# ---------------------------------------------------------------------------

def tt_svd(vec, dims, max_bond: int):
    """Sequential truncated SVDs of the unfoldings, left to right."""
    out = []
    rest = np.asarray(vec, dtype=np.float64).reshape(1, -1)
    r = 1
    for k, d in enumerate(dims[:-1]):
        M = rest.reshape(r * d, -1)
        U, S, Vt = svd_desc(M)
        keep = min(max_bond, int(np.sum(S > 0)) or 1)
        out.append(U[:, :keep].reshape(r, d, keep))
        rest = S[:keep, None] * Vt[:keep]
        r = keep
    out.append(rest.reshape(r, dims[-1], 1))
    return out


def unfolding_tail_bound(vec, dims, max_bond: int) -> float:
    """Lower bound on ||w - vec||^2 over MPS w with bonds <= max_bond: for every
    cut, the weight beyond the first max_bond singular values of that
    unfolding (Eckart-Young); return the largest over cuts."""
    best = 0.0
    v = np.asarray(vec)  # real or complex
    left = 1
    for k in range(len(dims) - 1):
        left *= dims[k]
        S = np.linalg.svd(v.reshape(left, -1), compute_uv=False)
        best = max(best, float(np.sum(S[max_bond:] ** 2)))
    return best
