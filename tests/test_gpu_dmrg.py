"""Two-site DMRG ground-state search on the GPU (Sec. 3.1.1) against the
free-fermion closed form of the XX chain, dense diagonalisation, and the FP64
oracle's DMRG (dense local eigensolver)."""

import numpy as np
import pytest

import synth
from oracle import dense
from oracle import dmrg as od
from paper_2601_16734_amd import binding as B

pytestmark = pytest.mark.gpu


def test_xx_chain_energy_matches_free_fermions(ctx):
    L = 8
    H = synth.xxz_mpo(np.ones(L - 1), np.zeros(L - 1))
    guess = synth.random_mps(np.random.default_rng(60), L, 2, 4)
    psi, E = ctx.dmrg(ctx.mpo_create(H), ctx.mps_create(guess), B.strategy(16, 0.0, sweeps=6))
    exact = od.xx_chain_ground_energy(1.0, L)
    print("xx L=8", E, exact, flush=True)
    assert abs(E - exact) <= 1e-10 * abs(exact)


def test_random_couplings_match_dense_ground_state_and_oracle(ctx):
    L = 8
    rng = np.random.default_rng(61)
    H = synth.xxz_mpo(rng.uniform(0.5, 1.5, L - 1), rng.uniform(0.5, 1.5, L - 1))
    guess = synth.random_mps(rng, L, 2, 3)
    psi, E = ctx.dmrg(ctx.mpo_create(H), ctx.mps_create(guess), B.strategy(16, 0.0, sweeps=6))
    Hd = dense.mpo_to_dense(H)
    e0 = np.linalg.eigvalsh(Hd)[0]
    E_or, psi_or, _ = od.dmrg(H, guess, max_bond=16, tol=0.0, sweeps=4)
    print("xxz L=8", E, e0, E_or, flush=True)
    assert abs(E - e0) <= 1e-10 * abs(e0)
    assert abs(E - E_or) <= 1e-10 * abs(e0)
    sites = psi.read()
    v = dense.mps_to_dense(sites)
    assert abs(np.linalg.norm(v) - 1.0) <= 1e-12
    assert np.linalg.norm(Hd @ v - E * v) <= 1e-7 * abs(E)
    # same state as the oracle's up to a sign (the ground state is non-degenerate here)
    w = dense.mps_to_dense(psi_or)
    assert abs(abs(v @ w) - 1.0) <= 1e-10
    # returned canonical at site 0: sites 1.. are right isometries
    for t in sites[1:]:
        m = t.reshape(t.shape[0], -1)
        assert np.max(np.abs(m @ m.T - np.eye(m.shape[0]))) <= 1e-12


def test_truncated_search_is_variational_and_matches_oracle(ctx):
    L = 10
    H = synth.xxz_mpo(np.ones(L - 1), 0.5 * np.ones(L - 1))
    guess = synth.random_mps(np.random.default_rng(62), L, 2, 2)
    st = B.strategy(6, 0.0, sweeps=6)
    psi, E = ctx.dmrg(ctx.mpo_create(H), ctx.mps_create(guess), st)
    e0 = np.linalg.eigvalsh(dense.mpo_to_dense(H))[0]
    E_or, _, _ = od.dmrg(H, guess, max_bond=6, tol=0.0, sweeps=6)
    print("xxz L=10 chi=6", E, E_or, e0, flush=True)
    assert psi.shape()[1][1:-1] == [min(6, 2 ** min(k, L - k)) for k in range(1, L)]
    assert E >= e0 - 1e-10 * abs(e0)
    assert abs(E - e0) <= 1e-3 * abs(e0)
    assert abs(E - E_or) <= 1e-8 * abs(e0)


def test_longer_chain_against_closed_form(ctx):
    L = 24
    H = synth.xxz_mpo(np.ones(L - 1), np.zeros(L - 1))
    guess = synth.random_mps(np.random.default_rng(63), L, 2, 8)
    psi, E = ctx.dmrg(ctx.mpo_create(H), ctx.mps_create(guess), B.strategy(48, 1e-14, sweeps=5), krylov_dim=32)
    exact = od.xx_chain_ground_energy(1.0, L)
    print("xx L=24 chi=48", E, exact, flush=True)
    assert E >= exact - 1e-9 * abs(exact)
    assert abs(E - exact) <= 1e-7 * abs(exact)
    assert abs(ctx.norm(psi) - 1.0) <= 1e-12


@pytest.mark.parametrize("L", [16, 64])
def test_critical_ising_chain_at_the_benchmark_tolerance(ctx, L):
    # -sum ZZ - sum X at the benchmark's relative tolerance eps^2 / (n - 1),
    # eps = 1e-6, bond left free (cap 256), early exit on the energy
    H = synth.tfim_mpo(L, 1.0, 1.0)
    guess = synth.random_mps(np.random.default_rng(70), L, 2, 4)
    st = B.strategy(256, 1e-12 / (L - 1), sweeps=8, sweep_tol=1e-13)
    psi, E = ctx.dmrg(ctx.mpo_create(H), ctx.mps_create(guess), st)
    exact = od.tfim_ground_energy(L, 1.0, 1.0)
    info = ctx.last_info()
    print("tfim", L, E, exact, (E - exact) / abs(exact), max(psi.shape()[1]), info["sweeps_done"], flush=True)
    assert E >= exact - 1e-11 * abs(exact)
    assert abs(E - exact) <= 1e-10 * abs(exact)
    assert info["sweeps_done"] < 8


def test_ising_chain_of_the_code_listing(ctx):
    # Z/2 and X/2 with unit prefactors: J = 1/4, h = 1/2
    L = 10
    H = synth.tfim_mpo(L, 0.25, 0.5)
    guess = synth.random_mps(np.random.default_rng(71), L, 2, 2)
    psi, E = ctx.dmrg(ctx.mpo_create(H), ctx.mps_create(guess), B.strategy(32, 0.0, sweeps=4))
    exact = od.tfim_ground_energy(L, 0.25, 0.5)
    assert abs(E - exact) <= 1e-12 * abs(exact)


def test_bad_arguments_are_rejected(ctx):
    H = ctx.mpo_create(synth.xxz_mpo(np.ones(3), np.zeros(3)))
    v = ctx.mps_create(synth.random_mps(np.random.default_rng(64), 4, 2, 2))
    short = ctx.mps_create(synth.random_mps(np.random.default_rng(65), 3, 2, 2))
    with pytest.raises(B.SmpsError) as e:
        ctx.dmrg(H, short, B.strategy(8, 0.0))
    assert e.value.code == B.EINVAL
    with pytest.raises(B.SmpsError) as e:
        ctx.dmrg(H, v, B.strategy(8, 0.0), krylov_dim=1)
    assert e.value.code == B.EINVAL
    with pytest.raises(B.SmpsError) as e:
        ctx.dmrg(H, v, B.strategy(8, 0.0, precision="fp32"))
    assert e.value.code == B.EUNSUPPORTED
    zero = ctx.mps_create([np.zeros_like(t) for t in synth.random_mps(np.random.default_rng(66), 4, 2, 2)])
    with pytest.raises(B.SmpsError) as e:
        ctx.dmrg(H, zero, B.strategy(8, 0.0))
    assert e.value.code == B.EINVAL
