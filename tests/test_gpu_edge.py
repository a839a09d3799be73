"""Edge cases of the apply + compression path against the FP64 oracle: a
single site, rank-1 truncation, the zero state, physical dimensions other
than 2 (also mixed along the chain), the singular-value truncation rule, the
early stop on the sweep tolerance, and the size limit."""

import math

import numpy as np
import pytest

import synth
from oracle import mps as om
from paper_2601_16734_amd import binding as B
from tests.gpu_helpers import cross_fidelity_loss, rel_norm_err

pytestmark = pytest.mark.gpu


def rand_mps(rng, phys, bonds):
    return [rng.standard_normal((bonds[k], phys[k], bonds[k + 1])) / math.sqrt(phys[k] * bonds[k + 1])
            for k in range(len(phys))]


def rand_mpo(rng, phys, bonds):
    return [rng.standard_normal((bonds[k], phys[k], phys[k], bonds[k + 1])) / math.sqrt(phys[k] * bonds[k + 1])
            for k in range(len(phys))]


def gpu_apply(ctx, mpo, mps, st):
    out, err = ctx.mpo_apply(ctx.mpo_create(mpo), ctx.mps_create(mps), st)
    return out.read(), ctx.last_info()


def test_single_site(ctx):
    rng = np.random.default_rng(0)
    mps = rand_mps(rng, [3], [1, 1])
    mpo = rand_mpo(rng, [3], [1, 1])
    got, info = gpu_apply(ctx, mpo, mps, B.strategy(4, 1e-12))
    ref = om.apply_simplify(mpo, mps, 4, 1e-12)
    assert info["steps"] == 0
    np.testing.assert_allclose(got[0], ref.mps[0], rtol=0, atol=1e-14)


def test_rank_one_truncation(ctx):
    w = synth.workload_random_mpo(2, L=8, chi=6, D=3)
    got, info = gpu_apply(ctx, w.mpo, w.mps, B.strategy(1, 0.0, sweeps=2))
    ref = om.apply_simplify(w.mpo, w.mps, 1, 0.0, sweeps=2)
    assert [1] + [t.shape[2] for t in got] == ref.ranks == [1] * 9
    assert rel_norm_err(info["norm"], ref.norm) <= 1e-10
    assert cross_fidelity_loss(got, ref.mps) <= 1e-10


def test_zero_state(ctx):
    rng = np.random.default_rng(1)
    mps = [np.zeros_like(t) for t in rand_mps(rng, [2] * 6, [1, 2, 4, 4, 4, 2, 1])]
    mpo = rand_mpo(rng, [2] * 6, [1, 2, 2, 2, 2, 2, 1])
    got, info = gpu_apply(ctx, mpo, mps, B.strategy(4, 1e-10, sweeps=2))
    assert info["norm"] == 0.0 and info["discarded"] == 0.0
    assert all(np.all(np.isfinite(t)) for t in got)
    assert np.all(got[0] == 0.0)


@pytest.mark.parametrize("phys", [[3] * 7, [2, 3, 4, 2, 3, 2]])
def test_other_physical_dimensions(ctx, phys):
    rng = np.random.default_rng(len(phys))
    L = len(phys)
    bonds = [1] + [min(6, int(np.prod(phys[:k])), int(np.prod(phys[k:]))) for k in range(1, L)] + [1]
    mps = rand_mps(rng, phys, bonds)
    mpo = rand_mpo(rng, phys, [1] + [3] * (L - 1) + [1])
    st = B.strategy(8, 1e-10, sweeps=3)
    got, info = gpu_apply(ctx, mpo, mps, st)
    ref = om.apply_simplify(mpo, mps, 8, 1e-10, sweeps=3)
    assert [1] + [t.shape[2] for t in got] == ref.ranks
    assert rel_norm_err(info["norm"], ref.norm) <= 1e-10
    assert cross_fidelity_loss(got, ref.mps) <= 1e-10


def test_singular_value_rule(ctx):
    w = synth.workload_random_mpo(3, L=10, chi=16, D=4)
    st = B.strategy(32, 1e-2, sweeps=2, trunc_mode=B.TRUNC_REL_SV)
    got, info = gpu_apply(ctx, w.mpo, w.mps, st)
    ref = om.apply_simplify(w.mpo, w.mps, 32, 1e-2, sweeps=2, mode=om.REL_SV)
    assert [1] + [t.shape[2] for t in got] == ref.ranks
    assert rel_norm_err(info["norm"], ref.norm) <= 1e-10
    assert cross_fidelity_loss(got, ref.mps) <= 1e-10
    deltas, _, _ = ctx.last_log()
    np.testing.assert_allclose(deltas, ref.deltas, rtol=1e-8, atol=1e-12 * ref.norm ** 2)


def test_sweep_tolerance_stops_early(ctx):
    w = synth.workload_laplacian_small()
    st = B.strategy(w.max_bond, w.tol, sweeps=8, sweep_tol=1e-9)
    got, info = gpu_apply(ctx, w.mpo, w.mps, st)
    assert 2 <= info["sweeps_done"] < 8
    assert info["steps"] == info["sweeps_done"] * 2 * (len(w.mps) - 1)
    ref = om.apply_simplify(w.mpo, w.mps, w.max_bond, w.tol, sweeps=info["sweeps_done"])
    assert rel_norm_err(info["norm"], ref.norm) <= 1e-12
    assert cross_fidelity_loss(got, ref.mps) <= 1e-12


def test_two_site_size_limit(ctx):
    rng = np.random.default_rng(2)
    L = 24
    bonds = [1] + [min(1100, 2 ** k, 2 ** (L - k)) for k in range(1, L)] + [1]
    mps = [np.zeros((bonds[k], 2, bonds[k + 1])) for k in range(L)]
    mpo = synth.identity_mpo(L, 2)
    with pytest.raises(B.SmpsError) as e:
        ctx.mpo_apply(ctx.mpo_create(mpo), ctx.mps_create(mps), B.strategy(1100, 1e-10))
    assert e.value.code == B.EUNSUPPORTED
