"""Pins of the FP64 oracle against facts that do not come from the oracle itself:
brute-force definitions, closed forms, textbook theorems and library routines
on special cases.  CPU only."""

import math

import numpy as np
import pytest

import synth
from oracle import dense, mps as om


def rand_mps(rng, dims, bonds):
    return [rng.standard_normal((bonds[k], dims[k], bonds[k + 1])) for k in range(len(dims))]


def rand_mpo(rng, dout, din, bonds):
    return [rng.standard_normal((bonds[k], dout[k], din[k], bonds[k + 1])) for k in range(len(dout))]


# ---------------------------------------------------------------- dense views

def test_mps_dense_matches_explicit_products_mixed_dims():
    rng = np.random.default_rng(1)
    m = rand_mps(rng, [2, 3, 2, 4], [1, 2, 3, 2, 1])
    np.testing.assert_allclose(dense.mps_to_dense(m), dense.mps_to_dense_bruteforce(m), rtol=1e-14, atol=1e-14)


def test_product_state_is_kronecker_msb_first():
    rng = np.random.default_rng(2)
    vecs = [rng.standard_normal(d) for d in (2, 3, 2)]
    m = [v.reshape(1, -1, 1) for v in vecs]
    ref = np.kron(np.kron(vecs[0], vecs[1]), vecs[2])
    np.testing.assert_allclose(dense.mps_to_dense(m), ref, rtol=1e-14)
    # digit (1, 2, 0) -> flat index 1*6 + 2*2 + 0 = 10
    assert dense.flat_index((1, 2, 0), (2, 3, 2)) == 10


def test_mpo_dense_matches_bruteforce_and_kron():
    rng = np.random.default_rng(3)
    U = rand_mpo(rng, [2, 2, 3], [2, 3, 2], [1, 2, 2, 1])
    np.testing.assert_allclose(dense.mpo_to_dense(U), dense.mpo_to_dense_bruteforce(U), rtol=1e-13, atol=1e-13)
    mats = [rng.standard_normal((2, 3)), rng.standard_normal((3, 2))]
    prod = [M.reshape(1, *M.shape, 1) for M in mats]
    np.testing.assert_allclose(dense.mpo_to_dense(prod), np.kron(mats[0], mats[1]), rtol=1e-14)


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("n", [1, 2, 3, 6])
def test_laplacian_open_is_tridiagonal(n):
    N = 2 ** n
    ref = -2.0 * np.eye(N) + np.eye(N, k=1) + np.eye(N, k=-1)
    np.testing.assert_array_equal(dense.mpo_to_dense(synth.laplacian_mpo(n)), ref)
    assert max(B.shape[0] for B in synth.laplacian_mpo(n)) <= 3


@pytest.mark.parametrize("n", [2, 3, 5])
def test_laplacian_periodic_has_corners(n):
    N = 2 ** n
    ref = -2.0 * np.eye(N) + np.eye(N, k=1) + np.eye(N, k=-1)
    ref[0, N - 1] += 1.0
    ref[N - 1, 0] += 1.0
    np.testing.assert_array_equal(dense.mpo_to_dense(synth.laplacian_mpo(n, periodic=True)), ref)


@pytest.mark.parametrize("n", [1, 3, 5])
def test_shifts(n):
    N = 2 ** n
    v = np.arange(N, dtype=float) + 1.0
    Dp = dense.mpo_to_dense(synth.shift_mpo(n, +1))
    Dm = dense.mpo_to_dense(synth.shift_mpo(n, -1))
    # (D_m v)_i = v_{i+m} inside the grid, 0 outside (open boundary)
    ref_p = np.append(v[1:], 0.0)
    ref_m = np.insert(v[:-1], 0, 0.0)
    np.testing.assert_array_equal(Dp @ v, ref_p)
    np.testing.assert_array_equal(Dm @ v, ref_m)
    assert all(B.shape[3] <= 2 for B in synth.shift_mpo(n, +1))


def test_xxz_mpo_is_pauli_sum():
    L = 5
    rng = np.random.default_rng(4)
    Jxy = rng.uniform(0.5, 1.5, L - 1)
    Jz = rng.uniform(0.5, 1.5, L - 1)
    X = np.array([[0, 1], [1, 0]], dtype=complex)
    Y = np.array([[0, -1j], [1j, 0]])
    Z = np.array([[1, 0], [0, -1]], dtype=complex)

    def op(o, i):
        m = np.array([[1.0 + 0j]])
        for k in range(L):
            m = np.kron(m, o if k == i else np.eye(2))
        return m

    H = np.zeros((2 ** L, 2 ** L), dtype=complex)
    for i in range(L - 1):
        H += Jxy[i] * (op(X, i) @ op(X, i + 1) + op(Y, i) @ op(Y, i + 1)) + Jz[i] * op(Z, i) @ op(Z, i + 1)
    assert np.abs(H.imag).max() == 0
    np.testing.assert_allclose(dense.mpo_to_dense(synth.xxz_mpo(Jxy, Jz)), H.real, atol=1e-14)


@pytest.mark.parametrize("n", [1, 2, 7])
def test_sine_and_exp_states(n):
    a, dx = 0.3, 2 * math.pi / 2 ** n
    x = a + dx * np.arange(2 ** n)
    np.testing.assert_allclose(dense.mps_to_dense(synth.sine_mps(n, a, dx)), np.sin(x), atol=1e-13)
    np.testing.assert_allclose(dense.mps_to_dense(synth.exp_mps(n, 0.7, a, dx)), np.exp(0.7 * x), rtol=1e-13)


def test_laplacian_on_sine_discrete_identity():
    n = 8
    a, dx = 0.1, 0.05
    v = dense.mps_to_dense(synth.sine_mps(n, a, dx))
    w = dense.mpo_to_dense(synth.laplacian_mpo(n)) @ v
    x = a + dx * np.arange(2 ** n)
    np.testing.assert_allclose(w[1:-1], 2 * (math.cos(dx) - 1) * np.sin(x[1:-1]), atol=1e-13)
    # boundary rows lose one neighbour
    assert abs(w[0] - (np.sin(x[1]) - 2 * np.sin(x[0]))) < 1e-13


# ---------------------------------------------------------------- scalar product, norm, canonical form

def test_scprod_matches_dense_dot():
    rng = np.random.default_rng(5)
    dims = [2] * 7
    bonds = [1, 2, 4, 5, 5, 4, 2, 1]
    a, b = rand_mps(rng, dims, bonds), rand_mps(rng, dims, bonds)
    ref = float(dense.mps_to_dense(a) @ dense.mps_to_dense(b))
    assert abs(om.scprod(a, b) - ref) <= 1e-12 * abs(ref) + 1e-13


def test_right_canonical_isometries_and_norm():
    rng = np.random.default_rng(6)
    dims = [2] * 8
    bonds = [1, 2, 4, 8, 8, 8, 4, 2, 1]
    m = rand_mps(rng, dims, bonds)
    c = om.right_canonical(m)
    for k in range(1, 8):
        assert om.is_right_isometry(c[k], atol=1e-13)
    v0, v1 = dense.mps_to_dense(m), dense.mps_to_dense(c)
    np.testing.assert_allclose(v1, v0, rtol=1e-12, atol=1e-12 * np.abs(v0).max())
    assert abs(om.norm_from_center(c, 0) - np.linalg.norm(v0)) <= 1e-13 * np.linalg.norm(v0)


# ---------------------------------------------------------------- truncation rule

def test_truncation_rank_rel_norm2_hand_values():
    s = np.array([4.0, 2.0, 1.0, 0.5])      # squares 16, 4, 1, .25; total 21.25
    # tails: t1 = 5.25, t2 = 1.25, t3 = .25, t4 = 0
    assert om.truncation_rank(s, 0.0, 10) == 4
    assert om.truncation_rank(s, 0.25 / 21.25, 10) == 3
    assert om.truncation_rank(s, 0.25 / 21.25 * 0.999, 10) == 4
    assert om.truncation_rank(s, 1.25 / 21.25, 10) == 2
    assert om.truncation_rank(s, 5.25 / 21.25, 10) == 1
    assert om.truncation_rank(s, 1.0, 10) == 1
    assert om.truncation_rank(s, 0.0, 2) == 2
    assert om.truncation_rank(np.zeros(3), 1e-10, 5) == 1


def test_truncation_rank_rel_sv():
    s = np.array([1.0, 0.5, 1e-3, 1e-9])
    assert om.truncation_rank(s, 1e-2, 10, om.REL_SV) == 2
    assert om.truncation_rank(s, 1e-6, 10, om.REL_SV) == 3
    assert om.truncation_rank(s, 1e-6, 2, om.REL_SV) == 2


def test_tail_sum_order_is_smallest_first():
    s = np.array([1.0, 1e-8, 1e-8])
    t = om.tail_sums(s)
    assert t[1] == (1e-8) ** 2 + (1e-8) ** 2
    assert t[3] == 0.0


def test_eckart_young_discarded_weight():
    """With the state canonical around the pair, truncating the two-site SVD
    changes the vector by exactly the discarded squared singular values."""
    rng = np.random.default_rng(7)
    dims = [2] * 8
    m = om.right_canonical(rand_mps(rng, dims, [1, 2, 4, 8, 8, 8, 4, 2, 1]))
    v = dense.mps_to_dense(m)
    th = np.einsum("asb,btc->astc", m[0], m[1])
    a, s, t, c = th.shape
    U, S, Vt = np.linalg.svd(th.reshape(a * s, t * c), full_matrices=False)
    r = 1
    w = list(m)
    w[0] = U[:, :r].reshape(a, s, r)
    w[1] = (S[:r, None] * Vt[:r]).reshape(r, t, c)
    dist2 = float(np.sum((dense.mps_to_dense(w) - v) ** 2))
    assert abs(dist2 - float(np.sum(S[r:] ** 2))) <= 1e-12 * float(np.sum(S ** 2))


# ---------------------------------------------------------------- exact product and the sweep

def test_mpo_times_mps_is_dense_product():
    rng = np.random.default_rng(8)
    v = rand_mps(rng, [2] * 6, [1, 2, 3, 3, 3, 2, 1])
    U = rand_mpo(rng, [2] * 6, [2] * 6, [1, 3, 2, 3, 2, 3, 1])
    C = om.mpo_times_mps(U, v)
    ref = dense.mpo_to_dense(U) @ dense.mps_to_dense(v)
    np.testing.assert_allclose(dense.mps_to_dense(C), ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
    assert C[2].shape == (2 * 3, 2, 3 * 3)


def test_apply_exact_when_unconstrained_random_nonsymmetric_mpo():
    rng = np.random.default_rng(9)
    v = rand_mps(rng, [2] * 8, synth.bond_caps(8, 2, 4))
    U = rand_mpo(rng, [2] * 8, [2] * 8, [1] + [3] * 7 + [1])
    res = om.apply_simplify(U, v, max_bond=64, tol=0.0, sweeps=2)
    ref = dense.mpo_to_dense(U) @ dense.mps_to_dense(v)
    got = dense.mps_to_dense(res.mps)
    assert np.linalg.norm(got - ref) <= 1e-11 * np.linalg.norm(ref)
    assert abs(res.norm - np.linalg.norm(ref)) <= 1e-12 * np.linalg.norm(ref)
    for k in range(1, 8):
        assert om.is_right_isometry(res.mps[k], atol=1e-12)


def test_laplacian_exact_variant():
    w = synth.workload_laplacian_small(max_bond=32, tol=0.0)
    v = w.mps
    res = om.apply_simplify(w.mpo, v, w.max_bond, w.tol, sweeps=4)
    ref = dense.mpo_to_dense(w.mpo) @ dense.mps_to_dense(v)
    assert np.linalg.norm(dense.mps_to_dense(res.mps) - ref) <= 1e-12 * np.linalg.norm(ref)


def test_identity_mpo_and_simplify_reproduce_state():
    rng = np.random.default_rng(10)
    v = rand_mps(rng, [2] * 7, synth.bond_caps(7, 2, 4))
    res = om.simplify(v, max_bond=16, tol=0.0, sweeps=1)
    ref = dense.mps_to_dense(v)
    got = dense.mps_to_dense(res.mps)
    assert abs(got @ ref / (np.linalg.norm(got) * np.linalg.norm(ref)) - 1) < 1e-14
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


def test_routes_fused_and_explicit_agree_truncated():
    w = synth.workload_laplacian_small()
    f = om.apply_simplify(w.mpo, w.mps, w.max_bond, w.tol, sweeps=4)
    c = om.apply_simplify_explicit(w.mpo, w.mps, w.max_bond, w.tol, sweeps=4)
    assert f.ranks == c.ranks
    assert abs(f.norm - c.norm) <= 1e-12 * f.norm
    gf, gc = dense.mps_to_dense(f.mps), dense.mps_to_dense(c.mps)
    assert 1 - abs(gf @ gc) / (np.linalg.norm(gf) * np.linalg.norm(gc)) < 1e-12


def test_routes_agree_random_mpo_small():
    w = synth.workload_random_mpo(L=10, chi=8, D=4)
    f = om.apply_simplify(w.mpo, w.mps, 8, 1e-10, sweeps=3)
    c = om.apply_simplify_explicit(w.mpo, w.mps, 8, 1e-10, sweeps=3)
    assert f.ranks == c.ranks
    assert abs(f.norm - c.norm) <= 1e-11 * f.norm
    assert abs(om.scprod(f.mps, c.mps) / (f.norm * c.norm) - 1) < 1e-10


def test_projection_invariant_and_bounds_on_truncated_laplacian():
    """Truncated SVD of the projected pair is an orthogonal projection, so
    <psi, U v> = ||psi||^2 and ||U v - psi||^2 = ||U v||^2 - ||psi||^2; the
    distance is bounded below by the largest unfolding tail (Eckart-Young)."""
    w = synth.workload_laplacian_small()
    res = om.apply_simplify(w.mpo, w.mps, w.max_bond, w.tol, sweeps=4)
    uv = dense.mpo_to_dense(w.mpo) @ dense.mps_to_dense(w.mps)
    psi = dense.mps_to_dense(res.mps)
    scale = uv @ uv
    assert abs(psi @ uv - psi @ psi) <= 1e-12 * scale
    dist2 = float(np.sum((uv - psi) ** 2))
    assert abs(dist2 - (scale - psi @ psi)) <= 1e-12 * scale
    assert dist2 >= om.unfolding_tail_bound(uv, [2] * 10, w.max_bond) * (1 - 1e-10)
    # ||psi||^2 after every step never decreases by more than rounding
    n2 = np.array(res.norms2)
    assert np.all(np.diff(n2) >= -1e-12 * scale)
    # the accumulated bound (sum of sqrt of discarded weights) dominates the true distance
    assert math.sqrt(dist2) <= res.error_bound * (1 + 1e-9) + 1e-12 * math.sqrt(scale)
    # the shifted copies of a bond-8 state need only a few extra bond states, so the
    # cap of 16 does not bind and tolerance alone sets the ranks here
    assert max(res.ranks) <= 16


def test_tt_svd_reference_quality():
    w = synth.workload_laplacian_small()
    uv = dense.mpo_to_dense(w.mpo) @ dense.mps_to_dense(w.mps)
    tt = om.tt_svd(uv, [2] * 10, 16)
    tt_err = float(np.sum((dense.mps_to_dense(tt) - uv) ** 2))
    res = om.apply_simplify(w.mpo, w.mps, w.max_bond, w.tol, sweeps=4)
    var_err = float(np.sum((dense.mps_to_dense(res.mps) - uv) ** 2))
    lb = om.unfolding_tail_bound(uv, [2] * 10, 16)
    assert lb * (1 - 1e-10) <= tt_err
    assert lb * (1 - 1e-10) <= var_err
    # the variational optimum is never worse than twice the quasi-optimal TT-SVD error here
    assert var_err <= 2 * tt_err


# ---------------------------------------------------------------- rank-predictor network (oracle side)

def test_bf16_rounding_hand_values():
    from oracle import mlp
    x = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -2.5, 0.1], dtype=np.float32)
    r = mlp.bf16_round(x)
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: even mantissa wins (1); 1 + 3*2^-8 rounds up to 1 + 2^-6
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == np.float32(1.0 + 2.0 ** -6) and r[3] == -2.5
    assert abs(r[4] - 0.1) < 0.1 * 2.0 ** -8 and (r.view(np.uint32) & 0xFFFF == 0).all()


def test_mlp_backward_matches_finite_differences():
    from oracle import mlp
    rng = np.random.default_rng(3)
    p = rng.standard_normal(mlp.N_PARAMS) * 0.2
    X = rng.standard_normal((6, 32))
    y = rng.standard_normal(6) * 2
    L, g = mlp.loss_and_grad(p, X, y, quantize=False)
    h = 1e-6
    idx = rng.choice(mlp.N_PARAMS, 60, replace=False)
    idx = np.concatenate([idx, [mlp.N_PARAMS - 1, 2048, 2048 + 64 + 4095]])
    for i in idx:
        e = np.zeros(mlp.N_PARAMS)
        e[i] = h
        fd = (mlp.loss_and_grad(p + e, X, y, quantize=False)[0] - mlp.loss_and_grad(p - e, X, y, quantize=False)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), i


def test_mlp_loss_asymmetry_and_features():
    from oracle import mlp
    p = np.zeros(mlp.N_PARAMS)
    X = np.zeros((2, 32))
    # output is b3 = 0: label 0.5 -> under-prediction (x4), label -0.5 -> over-prediction
    Lu, _ = mlp.loss_and_grad(p, X[:1], [0.5])
    Lo, _ = mlp.loss_and_grad(p, X[:1], [-0.5])
    assert abs(Lu - 4 * 0.125) < 1e-15 and abs(Lo - 0.125) < 1e-15
    L3, _ = mlp.loss_and_grad(p, X[:1], [3.0])
    assert abs(L3 - 4 * 2.5) < 1e-15  # linear branch beyond the Huber threshold
    f = mlp.features([2.0, 1.0, 0.0])
    assert f[0] == 0.0 and abs(f[1] - np.log(0.5)) < 1e-15 and f[2] == np.log(1e-30) and f[31] == np.log(1e-30)


def test_adam_constant_gradient_moves_by_lr_per_step():
    """With a constant gradient the bias-corrected moments equal g and g^2 at
    every step, so Adam moves each coordinate by lr * g / (|g| + eps)."""
    from oracle.mlp import adam_step
    g = np.array([1.0, -2.0, 0.0, 1e-3])
    p = np.array([0.5, 0.5, 0.5, 0.5])
    m = np.zeros(4)
    v = np.zeros(4)
    lr = 1e-2
    for t in range(1, 6):
        p_new, m, v = adam_step(p, g, m, v, t, lr)
        np.testing.assert_allclose(p - p_new, lr * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-18)
        p = p_new
