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


def test_tt_svd_full_rank_reconstructs_a_random_vector():
    # bonds up to 2^5 = 32 cover every unfolding of a 10-qubit vector exactly
    rng = np.random.default_rng(41)
    v = rng.standard_normal(2 ** 10)
    tt = om.tt_svd(v, [2] * 10, 32)
    assert [t.shape[2] for t in tt[:-1]] == [2, 4, 8, 16, 32, 16, 8, 4, 2]
    np.testing.assert_allclose(dense.mps_to_dense(tt), v, rtol=0, atol=1e-14 * np.abs(v).max())
    # every site but the last is a left isometry (Sec. 2.3 canonical form)
    for t in tt[:-1]:
        M = t.reshape(-1, t.shape[2])
        assert np.abs(M.T @ M - np.eye(M.shape[1])).max() <= 1e-13


def _basis_superposition(coeffs, patterns):
    v = np.zeros(2 ** len(patterns[0]))
    for c, p in zip(coeffs, patterns):
        v[int(p, 2)] += c  # MSB first (Eq. binary)
    return v


def test_tt_svd_and_unfolding_bound_on_hand_built_spectra():
    # v = sum_j c_j |b_j> over four orthogonal product states.  For cuts 2..8
    # the prefixes and suffixes of the four patterns are all distinct, so the
    # Schmidt values there are exactly |c_j|; at cuts 1 and 9 two patterns
    # share each prefix (suffix) and the rank is 2.  Keeping 2 (3) states the
    # smallest weight beyond the cap is c_2^2 + c_3^2 (c_3^2) -- by hand.
    c = np.array([0.8, 0.5, 0.3, 0.1])
    pats = ["0000000000", "1111111111", "0101010101", "1010101010"]
    v = _basis_superposition(c, pats)
    assert om.unfolding_tail_bound(v, [2] * 10, 2) == pytest.approx(0.3 ** 2 + 0.1 ** 2, rel=1e-14)
    assert om.unfolding_tail_bound(v, [2] * 10, 3) == pytest.approx(0.1 ** 2, rel=1e-12)
    assert om.unfolding_tail_bound(v, [2] * 10, 4) <= 1e-28
    # TT-SVD truncates only at cut 2, where the kept singular vectors are the
    # basis states of the two largest terms: the approximation is exactly
    # c_0 |b_0> + c_1 |b_1> and the error meets the bound (Eckart-Young)
    tt2 = om.tt_svd(v, [2] * 10, 2)
    np.testing.assert_allclose(dense.mps_to_dense(tt2), _basis_superposition(c[:2], pats[:2]), atol=1e-15)
    err2 = float(np.sum((dense.mps_to_dense(tt2) - v) ** 2))
    assert err2 == pytest.approx(0.3 ** 2 + 0.1 ** 2, rel=1e-13)
    err3 = float(np.sum((dense.mps_to_dense(om.tt_svd(v, [2] * 10, 3)) - v) ** 2))
    assert err3 == pytest.approx(0.1 ** 2, rel=1e-12)


def test_tt_svd_error_is_the_tail_at_the_only_truncated_cut():
    # a 10-qubit vector with prescribed Schmidt values s_j = 2^-j/2 at the
    # middle cut (random orthonormal factors on both halves): caps of 16 < 20
    # < 32 truncate that cut only, so TT-SVD's error and the unfolding bound
    # both equal sum_{j >= 20} s_j^2 exactly
    rng = np.random.default_rng(7)
    s = 2.0 ** (-np.arange(32) / 2.0)
    U, _ = np.linalg.qr(rng.standard_normal((32, 32)))
    W, _ = np.linalg.qr(rng.standard_normal((32, 32)))
    v = (U * s[None, :]) @ W.T
    v = v.reshape(-1)
    tail = float(np.sum(s[20:] ** 2))
    tt = om.tt_svd(v, [2] * 10, 20)
    err = float(np.sum((dense.mps_to_dense(tt) - v) ** 2))
    assert err == pytest.approx(tail, rel=1e-9)
    assert om.unfolding_tail_bound(v, [2] * 10, 20) == pytest.approx(tail, rel=1e-9)
    # a dropped tail term or a shifted cut would miss by s_19^2 or s_20^2
    assert abs(err - tail) < 1e-3 * s[20] ** 2


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


# ---- randomized factorization (oracle/rsvd.py) ---------------------------------

def test_philox_matches_numpy_bit_generator():
    """Philox4x64-10 pinned to numpy's independent implementation (which
    advances the counter before producing a block)."""
    from oracle import rsvd
    for ctr, key in [((0, 0, 0, 0), (0, 0)), ((5, 3, 0, 0), (7, 9)), ((2**64 - 2, 1, 2, 3), (2**63, 12345))]:
        bg = np.random.Philox(counter=np.array(ctr, dtype=np.uint64), key=np.array(key, dtype=np.uint64))
        raw = [int(x) for x in bg.random_raw(4)]
        nxt = (ctr[0] + 1) % 2**64
        assert rsvd.philox4x64_10_scalar((nxt,) + tuple(ctr[1:]), key) == raw
        v = rsvd.philox4x64_10(np.array([nxt], dtype=np.uint64), np.array([ctr[1]], dtype=np.uint64),
                               np.array([ctr[2]], dtype=np.uint64), np.array([ctr[3]], dtype=np.uint64), key)
        assert [int(x[0]) for x in v] == raw


def test_sketch_gaussians_moments():
    from oracle import rsvd
    g = rsvd.gaussians(3, 400_000)
    assert abs(g.mean()) < 6e-3 and abs(g.var() - 1.0) < 1e-2
    assert abs(np.mean(np.abs(g) < 1.0) - 0.682689) < 4e-3
    assert abs(np.mean(g ** 4) - 3.0) < 5e-2
    # different steps give different streams, the same step the same one
    assert not np.allclose(rsvd.gaussians(4, 64), rsvd.gaussians(3, 64))
    assert np.array_equal(rsvd.gaussians(3, 64), g[:64])


def test_rank_with_total_hand_values():
    from oracle import rsvd
    from oracle.mps import REL_NORM2
    # s^2 = 9, 4, 1, missed weight 0.5, total 14.5, threshold 1.6:
    # tails with the missed weight: r=1 -> 5.5, r=2 -> 1.5 (fits), so r = 2
    r, d = rsvd.rank_with_total([3.0, 2.0, 1.0], 14.5, 1.6 / 14.5, 10, REL_NORM2)
    assert r == 2 and abs(d - 1.5) < 1e-15
    # the missed weight alone above the threshold: keep everything
    r, d = rsvd.rank_with_total([3.0, 2.0, 1.0], 20.0, 0.1, 10, REL_NORM2)
    assert r == 3 and abs(d - 6.0) < 1e-12


def test_rsvd_equals_exact_svd_when_sketch_covers_rank():
    from oracle import rsvd
    from oracle.mps import REL_NORM2, svd_desc
    rng = np.random.default_rng(21)
    for rank, (m, n) in [(8, (60, 90)), (5, (120, 40)), (12, (64, 64))]:
        X = rng.standard_normal((m, rank)) @ np.diag(np.geomspace(10, 0.1, rank)) @ rng.standard_normal((rank, n))
        Q, s, r, delta, ok = rsvd.rsvd_rows(X, rank + 16, 1e-12, 100, REL_NORM2, step=7)
        _, S, Vt = svd_desc(X)
        assert ok and r == rank
        np.testing.assert_allclose(s[:rank], S[:rank], rtol=1e-12)
        # same row space: equal projectors
        assert np.max(np.abs(Q.T @ Q - Vt[:rank].T @ Vt[:rank])) < 1e-10
        assert np.max(np.abs(Q @ Q.T - np.eye(rank))) < 1e-12


def test_rsvd_discarded_weight_is_the_projection_error():
    """delta = ||X||^2 - sum_{j<r} s_j^2 must equal ||X - X Q^T Q||_F^2 for the
    returned Q, also when the sketch misses part of the spectrum."""
    from oracle import rsvd
    from oracle.mps import REL_NORM2, REL_SV
    rng = np.random.default_rng(8)
    U, _ = np.linalg.qr(rng.standard_normal((80, 80)))
    V, _ = np.linalg.qr(rng.standard_normal((100, 80)))
    X = U @ np.diag(np.exp(-np.arange(80) / 6.0)) @ V.T
    for k, mode, tol in [(30, REL_NORM2, 1e-8), (20, REL_NORM2, 1e-12), (24, REL_SV, 1e-3)]:
        Q, s, r, delta, ok = rsvd.rsvd_rows(X, k, tol, 100, mode, step=1)
        err = np.sum((X - X @ Q.T @ Q) ** 2)
        assert abs(err - delta) <= 1e-12 * np.sum(X * X) + 1e-6 * err
    # the sketch of 20 cannot reach a 1e-12 relative tail here: rejected
    assert not rsvd.rsvd_rows(X, 20, 1e-12, 100, REL_NORM2, step=1)[4]


def _decaying_identity_case(L=16, chi=64, taus=(3.0, 6.0), seed=4):
    rng = np.random.default_rng(seed)
    mps, _ = synth.decaying_spectrum_mps(rng, L, 2, chi, tau_range=taus)
    return mps, synth.identity_mpo(L, 2)


def test_sketched_sweep_matches_exact_sweep_when_sketches_are_accepted():
    """Compressing a state with fast-decaying spectra (tolerance-bound ranks
    of about 25 on 50 x 50 two-site matrices): accepted randomized splits must
    reproduce the exact sweep to rounding."""
    from oracle import rsvd
    from oracle.mps import apply_simplify
    mps, mpo = _decaying_identity_case()
    L = len(mps)
    exact = apply_simplify(mpo, mps, 64, 1e-10, sweeps=2)
    # the cap-sized sketch needs a cap below the matrix size: 32 (ranks stay
    # ~25; only the bulk matrices, 49 or more on both sides, are sketched)
    capped = apply_simplify(mpo, mps, 32, 1e-10, sweeps=2)
    # (a constant prediction sized so that the margin brings the sketch to 25 + oversampling)
    for cap, ref, kw, least in ((64, exact, {"predictor": lambda f: np.log(24.5 / rsvd.PREDICT_MARGIN)}, 10),
                                (64, exact, {"predictor": None}, 10), (32, capped, {"fixed": True}, 6)):
        hook = rsvd.SketchedSplit(cap, 1e-10, **kw)
        got = apply_simplify(mpo, mps, cap, 1e-10, sweeps=2, split_hook=hook)
        assert hook.kinds[:L - 1] == [0] * (L - 1)
        assert sum(k > 0 for k in hook.kinds) >= least
        assert got.ranks == ref.ranks
        assert abs(got.norm - ref.norm) < 1e-12 * ref.norm
        f = om.scprod(got.mps, ref.mps) / (got.norm * ref.norm)
        assert abs(1 - f) < 1e-12


# ---- linear combinations (Sec. 2.4.1, Eq. mps-sum-opt) --------------------------

def _small_terms(seed, L=6, chi=3, D=2, n=3):
    rng = np.random.default_rng(seed)
    terms = []
    for i in range(n):
        mps = synth.random_mps(rng, L, 2, chi)
        mpo = None if i == 1 else synth.random_mpo(rng, L, 2, D)
        terms.append((float(rng.uniform(-2, 2)), mpo, mps))
    return terms


def test_combination_without_truncation_is_the_dense_sum():
    terms = _small_terms(40)
    res = om.combine(terms, max_bond=64, tol=0.0, sweeps=2)
    want = sum(w * (dense.mpo_to_dense(m) @ dense.mps_to_dense(v) if m is not None else dense.mps_to_dense(v))
               for w, m, v in terms)
    got = dense.mps_to_dense(res.mps)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))


def test_combination_of_one_term_is_the_apply():
    rng = np.random.default_rng(41)
    mps = synth.random_mps(rng, 8, 2, 6)
    mpo = synth.random_mpo(rng, 8, 2, 3)
    a = om.combine([(1.0, mpo, mps)], max_bond=5, tol=1e-10, sweeps=2)
    b = om.apply_simplify(mpo, mps, 5, 1e-10, sweeps=2)
    assert a.ranks == b.ranks
    assert abs(a.norm - b.norm) <= 1e-12 * b.norm
    np.testing.assert_allclose(a.deltas, b.deltas, rtol=1e-9, atol=1e-15)


def test_combination_is_linear_in_the_weights():
    rng = np.random.default_rng(42)
    mps = synth.random_mps(rng, 7, 2, 5)
    mpo = synth.random_mpo(rng, 7, 2, 2)
    a = om.combine([(0.3, mpo, mps), (1.2, mpo, mps)], max_bond=4, tol=1e-10, sweeps=2)
    b = om.combine([(1.5, mpo, mps)], max_bond=4, tol=1e-10, sweeps=2)
    assert a.ranks == b.ranks
    f = om.scprod(a.mps, b.mps) / (a.norm * b.norm)
    assert abs(1 - f) <= 1e-12 and abs(a.norm - b.norm) <= 1e-12 * b.norm


# ---- two-site DMRG (Sec. 3.1.1) -----------------------------------------------

def test_dmrg_xx_chain_matches_free_fermions():
    from oracle import dmrg as od
    L = 8
    H = synth.xxz_mpo(np.ones(L - 1), np.zeros(L - 1))
    guess = synth.random_mps(np.random.default_rng(60), L, 2, 4)
    E, psi, _ = od.dmrg(H, guess, max_bond=16, tol=0.0, sweeps=4)
    assert abs(E - od.xx_chain_ground_energy(1.0, L)) <= 1e-10 * abs(E)


def test_dmrg_matches_dense_ground_state():
    from oracle import dmrg as od
    L = 8
    rng = np.random.default_rng(61)
    H = synth.xxz_mpo(rng.uniform(0.5, 1.5, L - 1), rng.uniform(0.5, 1.5, L - 1))
    guess = synth.random_mps(rng, L, 2, 3)
    E, psi, energies = od.dmrg(H, guess, max_bond=16, tol=0.0, sweeps=4)
    Hd = dense.mpo_to_dense(H)
    e0 = np.linalg.eigvalsh(Hd)[0]
    assert abs(E - e0) <= 1e-10 * abs(e0)
    v = dense.mps_to_dense(psi)
    assert abs(np.linalg.norm(v) - 1.0) <= 1e-12
    assert np.linalg.norm(Hd @ v - E * v) <= 1e-8 * abs(E)
    # the energy never rises along the sweep (variational, nothing truncated)
    assert all(b <= a + 1e-10 * abs(a) for a, b in zip(energies, energies[1:]))


def test_tfim_closed_form_matches_dense_spectrum():
    # the free-fermion formula against dense diagonalisation, and its two
    # one-term limits (-h X per site; -J ZZ per bond) done by hand
    from oracle import dmrg as od
    for L, J, h in [(1, 1.0, 1.0), (3, 1.0, 1.0), (6, 0.25, 0.5), (9, 1.0, 0.3), (10, 0.7, 1.9)]:
        e0 = np.linalg.eigvalsh(dense.mpo_to_dense(synth.tfim_mpo(L, J, h)))[0]
        assert abs(od.tfim_ground_energy(L, J, h) - e0) <= 1e-12 * abs(e0)
    assert abs(od.tfim_ground_energy(7, 0.0, 1.3) - (-7 * 1.3)) <= 1e-12
    assert abs(od.tfim_ground_energy(7, 0.8, 0.0) - (-6 * 0.8)) <= 1e-12


def test_dmrg_tfim_matches_closed_form():
    from oracle import dmrg as od
    L = 10
    H = synth.tfim_mpo(L, 1.0, 1.0)
    guess = synth.random_mps(np.random.default_rng(67), L, 2, 2)
    E, _, _ = od.dmrg(H, guess, max_bond=32, tol=0.0, sweeps=3)
    assert abs(E - od.tfim_ground_energy(L)) <= 1e-11 * abs(E)


# ---- diffusion workload inputs and the RK4 step (Sec. 7.1, Sec. 10.3) ---------

def test_placement_mps_reproduces_the_vector_exactly():
    rng = np.random.default_rng(80)
    for n in range(1, 8):
        v = rng.standard_normal(2 ** n)
        mps = synth.placement_mps(v, n)
        assert [t.shape[0] for t in mps][0] == 1 and mps[-1].shape[2] == 1
        np.testing.assert_array_equal(dense.mps_to_dense(mps), v)


def test_oracle_rk4_amplifies_a_laplacian_eigenvector_by_the_rk4_factor():
    # v_i = sin((i + 1) dx), dx = pi / (N + 1), is an eigenvector of the open
    # second-difference operator with eigenvalue -4 sin^2(dx / 2); one RK4 step
    # multiplies it by 1 + z + z^2/2 + z^3/6 + z^4/24, z = lambda dt
    from oracle import evolution as oe
    n = 6
    N = 2 ** n
    dx = np.pi / (N + 1)
    y0 = synth.sine_mps(n, dx, dx)
    lam = -4.0 * np.sin(dx / 2) ** 2
    dt = 0.3
    z = lam * dt
    R = 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24
    H = synth.laplacian_mpo(n)
    y = y0
    for _ in range(2):
        y = oe.rk4_step(H, y, dt, max_bond=8, tol=0.0, sweeps=2)
    want = R ** 2 * dense.mps_to_dense(y0)
    assert np.max(np.abs(dense.mps_to_dense(y) - want)) <= 1e-12 * np.max(np.abs(want))
    got_dense = oe.dense_rk4(dense.mpo_to_dense(H), dense.mps_to_dense(y0), dt, 2)
    assert np.max(np.abs(got_dense - want)) <= 1e-12 * np.max(np.abs(want))


# ---- complex arithmetic (apply + compression of complex MPS / MPO) -------------

def _zrand_mps(rng, L, d, chi):
    return [a + 1j * b for a, b in zip(synth.random_mps(rng, L, d, chi), synth.random_mps(rng, L, d, chi))]


def _zrand_mpo(rng, L, d, D):
    return [a + 1j * b for a, b in zip(synth.random_mpo(rng, L, d, D), synth.random_mpo(rng, L, d, D))]


def test_complex_apply_without_truncation_is_the_dense_product():
    from oracle import zmps
    rng = np.random.default_rng(90)
    v, U = _zrand_mps(rng, 6, 2, 3), _zrand_mpo(rng, 6, 2, 2)
    psi, nrm, _ = zmps.apply_simplify(U, v, max_bond=64, tol=0.0, sweeps=2)
    want = dense.mpo_to_dense(U) @ dense.mps_to_dense(v)
    got = dense.mps_to_dense(psi)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))
    assert abs(nrm - np.linalg.norm(want)) <= 1e-12 * np.linalg.norm(want)
    # the transfer-matrix scalar product against the dense one
    assert abs(zmps.scprod(psi, v) - np.vdot(got, dense.mps_to_dense(v))) <= 1e-12 * abs(np.vdot(got, got)) ** 0.5 * \
        np.linalg.norm(dense.mps_to_dense(v))


def test_complex_oracle_reduces_to_the_real_one_on_real_input():
    from oracle import zmps
    rng = np.random.default_rng(91)
    v, U = synth.random_mps(rng, 8, 2, 6), synth.random_mpo(rng, 8, 2, 3)
    psi, nrm, deltas = zmps.apply_simplify(U, v, max_bond=5, tol=1e-10, sweeps=2)
    ref = om.apply_simplify(U, v, max_bond=5, tol=1e-10, sweeps=2)
    assert abs(nrm - ref.norm) <= 1e-12 * ref.norm
    assert np.max(np.abs(np.asarray(deltas) - np.asarray(ref.deltas))) <= 1e-12 * ref.norm ** 2
    ov = abs(np.vdot(dense.mps_to_dense(psi), dense.mps_to_dense(ref.mps)))
    assert abs(ov / (nrm * ref.norm) - 1.0) <= 1e-12


def test_complex_compression_is_phase_covariant_and_optimal_when_truncated():
    # U -> e^{i phi} U multiplies the compressed result by e^{i phi}; and the
    # compressed state never beats the best rank-limited approximation
    # (distance >= the Eckart-Young bound of the dense product)
    from oracle import zmps
    rng = np.random.default_rng(92)
    v, U = _zrand_mps(rng, 8, 2, 4), _zrand_mpo(rng, 8, 2, 3)
    psi, nrm, _ = zmps.apply_simplify(U, v, max_bond=6, tol=0.0, sweeps=3)
    ph = np.exp(0.7j)
    Up = [U[0] * ph] + U[1:]
    psi2, nrm2, _ = zmps.apply_simplify(Up, v, max_bond=6, tol=0.0, sweeps=3)
    a, b = dense.mps_to_dense(psi), dense.mps_to_dense(psi2)
    assert abs(nrm2 - nrm) <= 1e-12 * nrm
    assert np.max(np.abs(b - ph * a)) <= 1e-10 * np.max(np.abs(a))
    w = dense.mpo_to_dense(U) @ dense.mps_to_dense(v)
    dist2 = np.linalg.norm(w - a) ** 2
    bound = om.unfolding_tail_bound(w, [2] * 8, 6)
    assert dist2 >= bound * (1 - 1e-9)
    # the variational result is the projection: |<psi, Uv>| = |psi|^2
    assert abs(abs(np.vdot(a, w)) - nrm ** 2) <= 1e-10 * nrm ** 2
