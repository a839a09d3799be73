"""The trained rank predictor in use: training on spectra that the sweeps
themselves produce, then the randomized factorization it sizes, against the
exact factorization and against sizing by the previous rank.

Correctness is asserted (every mode reproduces the exact result within the
oracle tolerance, fallbacks included); the gain (accepted steps, wall time)
is measured and printed, since it depends on the workload and is not a
parity property."""

import json
import time

import numpy as np
import pytest

import synth
from oracle import mps as om
from paper_2601_16734_amd import binding as B
from paper_2601_16734_amd import rank_training as RT
from tests.gpu_helpers import cross_fidelity_loss, rel_norm_err

pytestmark = pytest.mark.gpu


def decaying(rep, L=16, chi=64, taus=(3.0, 6.0)):
    rng = np.random.default_rng(4 + 1000 * rep)
    mps, _ = synth.decaying_spectrum_mps(rng, L, 2, chi, tau_range=taus)
    return synth.identity_mpo(L, 2), mps


def timed_apply(ctx, mpo, mps, chi, fact, sweeps=2):
    import torch
    U, v = ctx.mpo_create(mpo), ctx.mps_create(mps)
    st = B.strategy(chi, 1e-10, sweeps=sweeps, factorization=fact)
    torch.cuda.synchronize()
    t = time.perf_counter()
    out, _ = ctx.mpo_apply(U, v, st)
    torch.cuda.synchronize()
    return time.perf_counter() - t, out.read(), ctx.last_info()


def test_trained_predictor_sizes_accepted_sketches(ctx):
    # training data: small instances of the three exact workloads, plus two
    # seeds of the decaying-spectrum family (the evaluation uses another seed)
    probs = []
    for rep in range(4):
        w = synth.workload_laplacian_small(rep)
        probs.append((w.mpo, w.mps, w.max_bond, w.tol))
    w = synth.workload_random_mpo(0, L=12, chi=32, D=4)
    probs.append((w.mpo, w.mps, w.max_bond, w.tol))
    w = synth.workload_xxz(0, L=16, chi=32)
    probs.append((w.mpo, w.mps, w.max_bond, w.tol))
    F0, Y0 = RT.collect_pairs(ctx, probs, sweeps=4)
    F1, Y1 = RT.collect_pairs(ctx, [(*decaying(r), 64, 1e-10) for r in (1, 2)], sweeps=2)
    assert len(Y0) > 100 and len(Y1) > 20
    F, Y = np.concatenate([F0, F1]), np.concatenate([Y0, Y1])
    ctx.rank_mlp_init(0)
    l0, _ = ctx.rank_mlp_grad(F, Y)
    loss = RT.train_predictor(ctx, F, Y, epochs=150)
    assert np.isfinite(loss) and loss < 0.5 * l0

    mpo, mps = decaying(0)
    ref = om.apply_simplify(mpo, mps, 64, 1e-10, sweeps=2)
    report = {}
    for name, fact in [("exact", B.FACT_SVD), ("predictor", B.FACT_RSVD_MLP), ("previous_rank", B.FACT_RSVD_PREV),
                       ("fixed_sketch", B.FACT_RSVD_FIXED)]:
        timed_apply(ctx, mpo, mps, 64, fact)  # first call sizes the workspace
        dt, got, info = timed_apply(ctx, mpo, mps, 64, fact)
        assert rel_norm_err(info["norm"], ref.norm) <= 1e-10, name
        assert cross_fidelity_loss(got, ref.mps) <= 1e-10, name
        report[name] = {"seconds": dt, "accepted": info["rsvd_accepted"], "fallbacks": info["rsvd_fallbacks"]}
    assert report["predictor"]["accepted"] > 0
    print(json.dumps({"rank_predictor_gain": report}))
