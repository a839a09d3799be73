"""Dense brute-force views of MPS and MPO (oracle; test infrastructure only).

Sec. 2.1, Eq. (general-MPS): v_{s1..sL} = A^(1)s1 A^(2)s2 ... A^(L)sL with open
ends (first and last bond of dimension one).  Eq. (quantization)/(binary):
the flat index is i = sum_k s_k prod_{j>k} d_j, most significant digit first.
Sec. 2.2, Eq. (MPO): U^{j1..jL}_{i1..iL} = B^(1)j1 i1 ... B^(L)jL iL with tensors
stored as B[n][beta_{n-1}, j_n (output), i_n (input), beta_n].
"""

from __future__ import annotations

import itertools

import numpy as np


def flat_index(digits, dims) -> int:
    """Eq. (quantization): i = sum_k s_k prod_{j>k} d_j (most significant first)."""
    i = 0
    for s, d in zip(digits, dims):
        i = i * d + int(s)
    return i


def mps_entry(mps, digits) -> float:
    """One amplitude as the explicit product of L matrices (Eq. general-MPS)."""
    m = np.ones((1, 1))
    for A, s in zip(mps, digits):
        m = m @ A[:, s, :]
    return float(m[0, 0])


def mps_to_dense_bruteforce(mps) -> np.ndarray:
    """Every amplitude by the explicit matrix product (tiny chains only)."""
    dims = [A.shape[1] for A in mps]
    out = np.zeros(int(np.prod(dims)))
    for digits in itertools.product(*[range(d) for d in dims]):
        out[flat_index(digits, dims)] = mps_entry(mps, digits)
    return out


def mps_to_dense(mps) -> np.ndarray:
    """Same definition, with the matrix product vectorised over the digits
    already absorbed (left to right, so the first site is most significant)."""
    acc = np.ones((1, 1))  # (flat index so far, bond)
    for A in mps:
        acc = np.einsum("ia,asb->isb", acc, A).reshape(-1, A.shape[2])
    return acc.reshape(-1)


def mpo_entry(mpo, out_digits, in_digits) -> float:
    m = np.ones((1, 1))
    for B, j, i in zip(mpo, out_digits, in_digits):
        m = m @ B[:, j, i, :]
    return float(m[0, 0])


def mpo_to_dense(mpo) -> np.ndarray:
    """Matrix U[j, i] with j the output (row) and i the input (column) index."""
    acc = np.ones((1, 1, 1))  # (out so far, in so far, bond)
    for B in mpo:
        acc = np.einsum("jia,aqpb->jqipb", acc, B)
        J, Q, I, P, Bd = acc.shape
        acc = acc.reshape(J * Q, I * P, Bd)
    return acc[:, :, 0]


def mpo_to_dense_bruteforce(mpo) -> np.ndarray:
    dout = [B.shape[1] for B in mpo]
    din = [B.shape[2] for B in mpo]
    U = np.zeros((int(np.prod(dout)), int(np.prod(din))))
    for jd in itertools.product(*[range(d) for d in dout]):
        for idg in itertools.product(*[range(d) for d in din]):
            U[flat_index(jd, dout), flat_index(idg, din)] = mpo_entry(mpo, jd, idg)
    return U
