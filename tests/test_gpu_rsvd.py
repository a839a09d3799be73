"""GPU parity of the randomized two-site factorization (sketch sized by the
rank predictor or by the previous rank, exact SVD as fallback) against the
oracle's randomized schedule, plus the forced-fallback identity."""

import math

import numpy as np
import pytest

import synth
from oracle import mps as om
from oracle import rsvd as orsvd
from paper_2601_16734_amd import binding as B
from tests.gpu_helpers import cross_fidelity_loss, rel_norm_err

pytestmark = pytest.mark.gpu

N_PARAMS = 6337


def constant_predictor(ctx, rank_hat: float):
    """Predictor whose output is log(rank_hat) for every input (all weights 0)."""
    p = np.zeros(N_PARAMS, dtype=np.float32)
    p[-1] = np.float32(math.log(rank_hat))
    ctx.rank_mlp_set(p)
    return lambda f: float(p[-1])


def decaying_case(L, chi, taus, D, seed=4):
    rng = np.random.default_rng(seed)
    mps, _ = synth.decaying_spectrum_mps(rng, L, 2, chi, tau_range=taus)
    mpo = synth.identity_mpo(L, 2) if D == 1 else synth.random_mpo(rng, L, 2, D)
    return mps, mpo


def run(ctx, mps, mpo, max_bond, tol, sweeps, fact):
    st = B.strategy(max_bond, tol, sweeps=sweeps, factorization=fact)
    out, err = ctx.mpo_apply(ctx.mpo_create(mpo), ctx.mps_create(mps), st)
    return out.read(), ctx.last_info(), ctx.last_factor_log(), ctx.last_log()


@pytest.mark.parametrize("fact", [B.FACT_RSVD_MLP, B.FACT_RSVD_PREV, B.FACT_RSVD_FIXED])
def test_randomized_schedule_matches_oracle(ctx, fact):
    mps, mpo = decaying_case(16, 64, (3.0, 6.0), 1)
    # a prediction that the sizing margin raises to 25 (+ oversampling)
    pred = constant_predictor(ctx, 24.5 / orsvd.PREDICT_MARGIN)
    # the cap-sized sketch needs a cap below the bulk matrix size (ranks stay ~25)
    fixed = fact == B.FACT_RSVD_FIXED
    cap, least = (32, 6) if fixed else (64, 10)
    hook = orsvd.SketchedSplit(cap, 1e-10, predictor=pred if fact == B.FACT_RSVD_MLP else None, fixed=fixed)
    ref = om.apply_simplify(mpo, mps, cap, 1e-10, sweeps=2, split_hook=hook)
    got, info, kinds, (deltas, ranks, _) = run(ctx, mps, mpo, cap, 1e-10, 2, fact)
    assert list(kinds) == hook.kinds
    assert info["rsvd_accepted"] == sum(k > 0 for k in hook.kinds) >= least
    assert info["rsvd_fallbacks"] == 0
    assert [1] + [t.shape[2] for t in got] == ref.ranks
    assert rel_norm_err(info["norm"], ref.norm) <= 1e-10
    assert cross_fidelity_loss(got, ref.mps) <= 1e-10
    # the logged discarded weight of every step, randomized ones included
    scale = ref.norm ** 2
    assert np.max(np.abs(deltas - np.array(ref.deltas))) <= 1e-10 * scale


def test_fallback_when_rank_is_underpredicted_matches_exact(ctx):
    """Predicted rank 1 (sketch 18 after the margin) on bonds of rank ~25: every randomized step
    is rejected and replaced by the exact SVD.  The exact mode factorizes the
    steps whose needed side is the shorter one with accumulated rotations (the
    randomized modes keep one orientation), so the two agree to rounding, with
    the same ranks and discarded weights."""
    mps, mpo = decaying_case(16, 64, (3.0, 6.0), 1)
    constant_predictor(ctx, 1.0)
    got, info, kinds, (deltas, ranks, _) = run(ctx, mps, mpo, 64, 1e-10, 2, B.FACT_RSVD_MLP)
    ref, info0, kinds0, (deltas0, ranks0, _) = run(ctx, mps, mpo, 64, 1e-10, 2, B.FACT_SVD)
    assert info["rsvd_accepted"] == 0 and info["rsvd_fallbacks"] >= 10
    assert all(k <= 0 for k in kinds) and all(k == 0 for k in kinds0)
    assert list(ranks) == list(ranks0)
    assert [t.shape for t in got] == [t.shape for t in ref]
    assert np.max(np.abs(np.asarray(deltas) - np.asarray(deltas0))) <= 1e-12 * info0["norm"] ** 2
    assert rel_norm_err(info["norm"], info0["norm"]) <= 1e-12
    assert cross_fidelity_loss(got, ref) <= 1e-12


def test_rejections_match_oracle_with_random_operator(ctx):
    mps, mpo = decaying_case(14, 32, (3.0, 6.0), 2)
    # sized to 19 (+ oversampling) after the margin: below the ranks the random operator produces
    pred = constant_predictor(ctx, 18.5 / orsvd.PREDICT_MARGIN)
    hook = orsvd.SketchedSplit(32, 1e-10, predictor=pred)
    ref = om.apply_simplify(mpo, mps, 32, 1e-10, sweeps=2, split_hook=hook)
    got, info, kinds, _ = run(ctx, mps, mpo, 32, 1e-10, 2, B.FACT_RSVD_MLP)
    assert list(kinds) == hook.kinds
    assert info["rsvd_fallbacks"] == sum(k < 0 for k in hook.kinds) > 0
    assert rel_norm_err(info["norm"], ref.norm) <= 1e-10
    assert cross_fidelity_loss(got, ref.mps) <= 1e-10


def test_randomized_needs_a_predictor_and_the_single_path():
    fresh = B.Context(0)
    mps, mpo = decaying_case(6, 8, (3.0, 6.0), 1)
    U, v = fresh.mpo_create(mpo), fresh.mps_create(mps)
    with pytest.raises(B.SmpsError) as e:
        fresh.mpo_apply(U, v, B.strategy(8, 1e-10, factorization=B.FACT_RSVD_MLP))
    assert e.value.code == B.EINVAL
    with pytest.raises(B.SmpsError) as e:
        fresh.mpo_apply_batched([U], [v], B.strategy(8, 1e-10, factorization=B.FACT_RSVD_PREV))
    assert e.value.code == B.EUNSUPPORTED
    # the previous-rank sizing needs no predictor
    out, _ = fresh.mpo_apply(U, v, B.strategy(8, 1e-10, factorization=B.FACT_RSVD_PREV))
    assert out.shape()[1][0] == 1
