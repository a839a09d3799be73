"""Seeded synthetic inputs for MPO-times-MPS apply + compression workloads.

This module only *draws* or *writes down* input tensors: random MPS/MPO site
tensors, and the closed-form operators and states the paper builds by
construction (finite-difference shift / Laplacian MPOs of Sec. 5.1, the
bond-2 sine and bond-1 exponential states of Sec. 4.2, nearest-neighbour
XXZ-type and transverse-field Ising Hamiltonian MPOs).  It contains none of the compression arithmetic:
no contraction, no factorization, no truncation.  Both the CPU oracle and the
GPU library consume exactly the arrays produced here.

Conventions (Sec. 2.1 and 2.2):
  * MPS site tensor  A[k] has shape (chi_l, d, chi_r), C order, open ends
    (chi_0 = chi_L = 1).
  * MPO site tensor  B[k] has shape (D_l, d_out, d_in, D_r).
  * Binary quantization is most-significant digit first (Eq. binary), so
    site 0 carries the most significant bit.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_ROOT = 260116734


def rng_for(config: int, rep: int = 0) -> np.random.Generator:
    """Generator for (config, repetition); one stream per workload."""
    return np.random.default_rng(np.random.SeedSequence([SEED_ROOT, int(config), int(rep)]))


def bond_caps(L: int, d: int, chi: int) -> list[int]:
    """Bond dimensions min(chi, d^k, d^(L-k)) for k = 0..L (open ends are 1)."""
    out = []
    for k in range(L + 1):
        out.append(int(min(chi, d ** min(k, 64), d ** min(L - k, 64))))
    return out


def random_mps(rng: np.random.Generator, L: int, d: int, chi: int, *, variance: str = "inv_chi",
               dtype=np.float64) -> list[np.ndarray]:
    """Random MPS with bonds at the cap profile and i.i.d. Gaussian entries.

    variance:
      "unit"     -> N(0, 1)
      "inv_chi"  -> N(0, 1/chi) times a per-site constant (chi / (d*chi_r))^(1/2)
                    that keeps the expected squared norm at 1 (otherwise it
                    grows like d^L and a 100-site chain would sit near 1e30).
    Tensors are drawn site by site in C order.
    """
    bonds = bond_caps(L, d, chi)
    out = []
    for k in range(L):
        shape = (bonds[k], d, bonds[k + 1])
        x = rng.standard_normal(shape)
        if variance == "inv_chi":
            x *= math.sqrt(1.0 / (d * bonds[k + 1]))
        elif variance != "unit":
            raise ValueError(variance)
        out.append(np.ascontiguousarray(x.astype(dtype)))
    return out


def random_mpo(rng: np.random.Generator, L: int, d: int, D: int, dtype=np.float64) -> list[np.ndarray]:
    """Random MPO with bond D (1 at the ends), entries N(0, 1/D) scaled by 1/sqrt(d)
    so that the operator has O(1) gain per site."""
    out = []
    for k in range(L):
        dl = 1 if k == 0 else D
        dr = 1 if k == L - 1 else D
        x = rng.standard_normal((dl, d, d, dr)) * math.sqrt(1.0 / (D * d))
        out.append(np.ascontiguousarray(x.astype(dtype)))
    return out


# ---------------------------------------------------------------------------
# Closed-form operators (Sec. 5.1: finite differences through shift operators)
# ---------------------------------------------------------------------------

def _carry_tensor(carries: list[int]) -> np.ndarray:
    """Local adder tensor T[c_out, o, p, c_in] for binary digits.

    The shift (D_m v)_i = v_{i+m} has matrix elements U[o_idx, p_idx] = 1 iff
    p_idx = o_idx + m.  Adding m to the output index digit by digit, from the
    least significant site towards the most significant one, needs one carry
    state per bond: the input digit is p = (o + c_in) mod 2 and the carry passed
    to the more significant neighbour is floor((o + c_in) / 2).
    """
    idx = {c: j for j, c in enumerate(carries)}
    T = np.zeros((len(carries), 2, 2, len(carries)))
    for c_in in carries:
        for o in (0, 1):
            s = o + c_in
            p = s % 2
            c_out = s // 2  # floor division: -1 // 2 == -1
            if c_out in idx:
                T[idx[c_out], o, p, idx[c_in]] = 1.0
    return T


def weighted_shifts_mpo(n: int, weights: dict[int, float], periodic: bool = False) -> list[np.ndarray]:
    """MPO of sum_m w_m D_m on n binary sites, m in {-1, 0, +1}.

    Bond dimension = number of carry values needed.  The least significant
    site injects the initial carry m with weight w_m; the most significant
    site keeps only carry 0 (open boundary: displaced indices that leave
    [0, 2^n) give 0) or sums all carries (periodic: index arithmetic mod 2^n).
    """
    carries = [0]
    for m in sorted(weights):
        if m not in carries:
            carries.append(m)
    if any(m not in (-1, 0, 1) for m in weights):
        raise ValueError("only unit shifts are needed here")
    T = _carry_tensor(carries)
    wR = np.array([weights.get(c, 0.0) for c in carries])
    left = np.zeros(len(carries))
    if periodic:
        left[:] = 1.0
    else:
        left[carries.index(0)] = 1.0
    out = []
    for k in range(n):
        t = T.copy()
        if k == n - 1:
            t = np.einsum("aopc,c->aop", t, wR)[..., None]
        if k == 0:
            t = np.einsum("a,aopc->opc", left, t)[None]
        out.append(np.ascontiguousarray(t))
    return out


def laplacian_mpo(n: int, periodic: bool = False, dx: float = 1.0) -> list[np.ndarray]:
    """(D_{+1} + D_{-1} - 2 I) / dx^2 as a bond-3 MPO (Sec. 5.1)."""
    mpo = weighted_shifts_mpo(n, {1: 1.0, -1: 1.0, 0: -2.0}, periodic)
    mpo[0] = mpo[0] / (dx * dx)
    return mpo


def shift_mpo(n: int, m: int = 1, periodic: bool = False) -> list[np.ndarray]:
    """Single displacement D_m (bond 2 for m = +-1)."""
    return weighted_shifts_mpo(n, {m: 1.0}, periodic)


def identity_mpo(L: int, d: int) -> list[np.ndarray]:
    return [np.eye(d).reshape(1, d, d, 1).copy() for _ in range(L)]


# ---------------------------------------------------------------------------
# XXZ-type nearest-neighbour Hamiltonian, D = 5
# ---------------------------------------------------------------------------

def xxz_mpo(Jxy: np.ndarray, Jz: np.ndarray) -> list[np.ndarray]:
    """H = sum_i Jxy_i (X_i X_{i+1} + Y_i Y_{i+1}) + Jz_i Z_i Z_{i+1}, open chain.

    Uses XX + YY = 2 (s+ s- + s- s+) with s+ = [[0,1],[0,0]], so every
    entry is real.  Bond i couples sites i and i+1 (len(Jxy) = L - 1).
    """
    L = len(Jxy) + 1
    I = np.eye(2)
    sp = np.array([[0.0, 1.0], [0.0, 0.0]])
    sm = sp.T.copy()
    Z = np.diag([1.0, -1.0])
    out = []
    for k in range(L):
        W = np.zeros((5, 2, 2, 5))
        W[0, :, :, 0] = I
        W[4, :, :, 4] = I
        W[0, :, :, 1] = sp
        W[0, :, :, 2] = sm
        W[0, :, :, 3] = Z
        if k > 0:
            W[1, :, :, 4] = 2.0 * Jxy[k - 1] * sm
            W[2, :, :, 4] = 2.0 * Jxy[k - 1] * sp
            W[3, :, :, 4] = Jz[k - 1] * Z
        if k == 0:
            W = W[0:1]
        if k == L - 1:
            W = W[..., 4:5]
        out.append(np.ascontiguousarray(W))
    return out


# ---------------------------------------------------------------------------
# Closed-form states (Sec. 4.2: sums of exponentials)
# ---------------------------------------------------------------------------

def tfim_mpo(L: int, J: float = 1.0, h: float = 1.0) -> list[np.ndarray]:
    """Transverse-field Ising chain of the DMRG example (Sec. 10.1), open ends:
    H = -J sum_i Z_i Z_{i+1} - h sum_i X_i (Pauli matrices), written as the
    D = 3 operator with rows/columns (done, pending Z, start).  The example's
    formula is J = h = 1; its code listing uses Z/2 and X/2 with unit
    prefactors, i.e. J = 1/4, h = 1/2."""
    I = np.eye(2)
    Z = np.diag([1.0, -1.0])
    X = np.array([[0.0, 1.0], [1.0, 0.0]])
    out = []
    for k in range(L):
        W = np.zeros((3, 2, 2, 3))
        W[0, :, :, 0] = I
        W[0, :, :, 1] = Z
        W[0, :, :, 2] = -h * X
        W[1, :, :, 2] = -J * Z
        W[2, :, :, 2] = I
        if k == 0:
            W = W[0:1]
        if k == L - 1:
            W = W[..., 2:3]
        out.append(np.ascontiguousarray(W))
    return out


def gaussian_grid(n: int, a: float = -0.5, b: float = 0.5, sigma: float = 0.1) -> np.ndarray:
    """exp(-x^2 / (2 sigma^2)) sampled at x_i = a + i (b - a) / 2^n, i < 2^n: the
    initial condition of the diffusion example (Sec. 10.3)."""
    x = a + (b - a) / 2 ** n * np.arange(2 ** n)
    return np.exp(-0.5 * (x / sigma) ** 2)


def placement_mps(vec: np.ndarray, n: int) -> list[np.ndarray]:
    """An exact MPS of a length-2^n vector (binary digits, most significant
    first) built by index placement only: sites left of m = n // 2 copy the
    digits seen so far into the bond (bond 2^k), sites right of m carry the
    remaining digits from the right, and site m holds the entries of vec as a
    (2^m, 2, 2^(n-1-m)) block.  Bond dimensions 2^min(k, n-k) at most; no
    arithmetic is done on the values."""
    vec = np.asarray(vec, dtype=np.float64)
    assert vec.shape == (2 ** n,)
    m = n // 2
    out = []
    for k in range(n):
        if k < m:
            A = np.zeros((2 ** k, 2, 2 ** (k + 1)))
            for l in range(2 ** k):
                for s in range(2):
                    A[l, s, 2 * l + s] = 1.0
        elif k == m:
            A = vec.reshape(2 ** m, 2, 2 ** (n - 1 - m)).copy()
        else:
            r = 2 ** (n - 1 - k)
            A = np.zeros((2 * r, 2, r))
            for s in range(2):
                for q in range(r):
                    A[s * r + q, s, q] = 1.0
        out.append(A)
    return out


def sine_mps(n: int, a: float, dx: float) -> list[np.ndarray]:
    """Bond-2 MPS of v_i = sin(a + i dx), i MSB-first on n sites."""
    th = [dx * 2.0 ** (n - 1 - k) for k in range(n)]
    if n == 1:
        return [np.array([math.sin(a), math.sin(a + th[0])]).reshape(1, 2, 1)]
    out = []
    for k in range(n):
        if k == 0:
            t = np.zeros((1, 2, 2))
            for s in (0, 1):
                t[0, s] = [math.cos(a + th[0] * s), math.sin(a + th[0] * s)]
        elif k == n - 1:
            t = np.zeros((2, 2, 1))
            for s in (0, 1):
                t[:, s, 0] = [math.sin(th[k] * s), math.cos(th[k] * s)]
        else:
            t = np.zeros((2, 2, 2))
            for s in (0, 1):
                c, sn = math.cos(th[k] * s), math.sin(th[k] * s)
                t[:, s, :] = [[c, sn], [-sn, c]]
        out.append(t)
    return out


def exp_mps(n: int, kappa: float, a: float, dx: float) -> list[np.ndarray]:
    """Bond-1 MPS of v_i = exp(kappa (a + i dx))."""
    out = []
    for k in range(n):
        th = dx * 2.0 ** (n - 1 - k)
        t = np.array([1.0, math.exp(kappa * th)]).reshape(1, 2, 1)
        if k == 0:
            t = t * math.exp(kappa * a)
        out.append(t)
    return out


def decaying_spectrum_mps(rng: np.random.Generator, L: int, d: int, chi: int,
                          tau_range=(10.0, 100.0)) -> tuple[list[np.ndarray], np.ndarray]:
    """MPS whose bond spectra decay like exp(-j / tau_k), tau_k ~ U[tau_range].

    Site k = Q_k diag(exp(-j / tau_{k+1})): Q_k is a random left isometry of
    shape (chi_l * d, chi_r) drawn as the orthonormal factor of a Gaussian
    matrix, so the state is left-canonical and the singular values across
    bond k+1 are approximately the prescribed decay.
    """
    bonds = bond_caps(L, d, chi)
    taus = rng.uniform(tau_range[0], tau_range[1], size=L + 1)
    out = []
    for k in range(L):
        cl, cr = bonds[k], bonds[k + 1]
        g = rng.standard_normal((cl * d, cr))
        q, r = np.linalg.qr(g)
        q = q * np.sign(np.diag(r))[None, :]
        lam = np.exp(-np.arange(cr) / taus[k + 1])
        t = (q * lam[None, :]).reshape(cl, d, cr)
        out.append(np.ascontiguousarray(t))
    return out, taus


# ---------------------------------------------------------------------------
# Workload descriptions
# ---------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    mps: list
    mpo: list
    max_bond: int
    tol: float
    sweeps: int = 4
    meta: dict = field(default_factory=dict)


def workload_laplacian_small(rep: int = 0, max_bond: int = 16, tol: float = 1e-12) -> Workload:
    """n=10, d=2, chi=8 MPS with N(0,1) entries; bond-3 open Laplacian;
    compress to tol 1e-12 and max bond 16.  (The normalisation of the state
    is a norm computation and is left to the caller.)"""
    rng = rng_for(1, rep)
    mps = random_mps(rng, 10, 2, 8, variance="unit")
    return Workload("laplacian_n10_chi8", mps, laplacian_mpo(10), max_bond, tol)


def workload_random_mpo(rep: int = 0, L: int = 20, chi: int = 64, D: int = 8) -> Workload:
    """n=20, d=2, chi=64 MPS, N(0,1/chi); random MPO D=8; chi<=64, tol 1e-10, 4 sweeps."""
    rng = rng_for(2, rep)
    mps = random_mps(rng, L, 2, chi, variance="inv_chi")
    mpo = random_mpo(rng, L, 2, D)
    return Workload(f"random_mpo_n{L}_chi{chi}_D{D}", mps, mpo, chi, 1e-10)


def workload_xxz(rep: int = 0, L: int = 100, chi: int = 256) -> Workload:
    """L=100, d=2, chi=256 random MPS; XXZ-type MPO D=5, couplings U[0.5,1.5]."""
    rng = rng_for(3, rep)
    mps = random_mps(rng, L, 2, chi, variance="inv_chi")
    Jxy = rng.uniform(0.5, 1.5, size=L - 1)
    Jz = rng.uniform(0.5, 1.5, size=L - 1)
    return Workload(f"xxz_L{L}_chi{chi}_D5", mps, xxz_mpo(Jxy, Jz), chi, 1e-10,
                    meta={"Jxy": Jxy, "Jz": Jz})


def workload_batch(rep: int = 0, count: int = 512, n_range=(8, 30), chis=(4, 8, 16, 32, 64, 128)) -> list[Workload]:
    """Batch of QTT MPS: n ~ U{8..30}, chi ~ U{4,8,...,128}, float32 N(0,1/chi)
    entries; each gets either the bond-3 Laplacian or the bond-2 shift D_{+1}."""
    rng = rng_for(4, rep)
    out = []
    for i in range(count):
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        chi = int(rng.choice(chis))
        mps = random_mps(rng, n, 2, chi, variance="inv_chi", dtype=np.float32)
        which = int(rng.integers(0, 2))
        mpo = laplacian_mpo(n) if which == 0 else shift_mpo(n, 1)
        out.append(Workload(f"batch{i}_n{n}_chi{chi}_{'lap' if which == 0 else 'shift'}",
                            mps, mpo, chi, 1e-10, meta={"n": n, "chi": chi, "op": which}))
    return out


def workload_decaying(rep: int = 0, L: int = 64, chi: int = 512, D: int = 8) -> Workload:
    """L=64, d=2, chi=512 MPS with spectra ~ exp(-j/tau), tau ~ U[10,100]; random MPO D=8."""
    rng = rng_for(5, rep)
    mps, taus = decaying_spectrum_mps(rng, L, 2, chi)
    mpo = random_mpo(rng, L, 2, D)
    return Workload(f"decaying_L{L}_chi{chi}_D{D}", mps, mpo, chi, 1e-10, meta={"taus": taus})


def product_mpo(rng: np.random.Generator, L: int, d: int, spread: float = 0.3) -> list[np.ndarray]:
    """Bond-1 MPO of independent local operators I + spread * N(0,1) (a product
    operator: it rescales the bond spectra of a state but does not flatten them)."""
    out = []
    for _ in range(L):
        m = np.eye(d) + spread * rng.standard_normal((d, d))
        out.append(np.ascontiguousarray(m.reshape(1, d, d, 1)))
    return out


def workload_decaying_tol(rep: int = 0, L: int = 32, chi: int = 512, tau_range=(20.0, 40.0)) -> Workload:
    """Tolerance-bound variant of the decaying-spectrum workload: L=32, d=2,
    chi=512 MPS with spectra ~ exp(-j/tau), tau ~ U[20,40] per bond, under a
    product operator; at tol 1e-10 the kept ranks (about 11.5 tau) fall below
    the cap of 512, so the tolerance, not the cap, decides them."""
    rng = rng_for(6, rep)
    mps, taus = decaying_spectrum_mps(rng, L, 2, chi, tau_range=tau_range)
    mpo = product_mpo(rng, L, 2)
    return Workload(f"decaying_tol_L{L}_chi{chi}", mps, mpo, chi, 1e-10, sweeps=2, meta={"taus": taus})


# ---- rank-predictor inputs -------------------------------------------------------
def mlp_params(rng: np.random.Generator, n: int = 6337, scale: float = 0.2) -> np.ndarray:
    """Random FP32 parameter vector for the 32-64-64-1 rank predictor."""
    return (rng.standard_normal(n) * scale).astype(np.float32)


def mlp_inputs(rng: np.random.Generator, n: int, floor: float = 1e-30):
    """n synthetic log-spectrum feature rows (32 descending values starting at
    0, floored at log(floor)) and log-rank labels in [0, log 512]."""
    steps = rng.exponential(rng.uniform(0.05, 2.0, size=(n, 1)), size=(n, 32))
    steps[:, 0] = 0.0
    X = np.maximum(-np.cumsum(steps, axis=1), math.log(floor)).astype(np.float32)
    y = rng.uniform(0.0, math.log(512.0), size=n).astype(np.float32)
    return X, y
