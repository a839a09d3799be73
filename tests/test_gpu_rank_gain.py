"""The trained rank predictor in use on tolerance-bound spectra (L=32,
chi=512, decaying bond spectra under a product operator, 2 sweeps): trained
on spectra that exact sweeps produce (small exact workloads and two other
seeds of the same family), then the randomized factorization it sizes
against the exact factorization and against sizing by the previous rank.

Asserted: every mode reproduces the oracle's run (tests/golden) within the
randomized bar; the predictor's sketches are accepted with few fallbacks;
the predictor-sized run is faster than the previous-rank-sized one.  The
ratio to the exact path is measured and held within a bound (on these sizes
the randomized split does not beat the warm-started one-sided Jacobi SVD)."""

import json
import os
import time

import numpy as np
import pytest

import synth
from paper_2601_16734_amd import binding as B
from paper_2601_16734_amd import rank_training as RT

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def train(ctx):
    probs = [(w.mpo, w.mps, w.max_bond, w.tol) for w in
             [synth.workload_laplacian_small(r) for r in range(4)] +
             [synth.workload_random_mpo(0, L=12, chi=32, D=4), synth.workload_xxz(0, L=16, chi=32)]]
    F0, Y0 = RT.collect_pairs(ctx, probs, sweeps=4)
    tr = [synth.workload_decaying_tol(r) for r in (1, 2)]
    F1, Y1 = RT.collect_pairs(ctx, [(w.mpo, w.mps, w.max_bond, w.tol) for w in tr], sweeps=2)
    assert len(Y0) > 100 and len(Y1) > 50
    F, Y = np.concatenate([F0, F1]), np.concatenate([Y0, Y1])
    ctx.rank_mlp_init(0)
    l0, _ = ctx.rank_mlp_grad(F, Y)
    loss = RT.train_predictor(ctx, F, Y, epochs=150)
    assert np.isfinite(loss) and loss < 0.5 * l0
    return len(Y), loss


def test_trained_predictor_gain_on_tolerance_bound_spectra(ctx):
    import torch
    pairs, loss = train(ctx)
    with open(os.path.join(HERE, "golden", "decaying_tol_L32_chi512_s2.json")) as f:
        g = json.load(f)
    w = synth.workload_decaying_tol(0)
    U, v = ctx.mpo_create(w.mpo), ctx.mps_create(w.mps)
    report = {}
    for name, fact in [("exact", B.FACT_SVD), ("predictor", B.FACT_RSVD_MLP), ("previous_rank", B.FACT_RSVD_PREV)]:
        st = B.strategy(w.max_bond, w.tol, sweeps=g["sweeps"], factorization=fact)
        o, _ = ctx.mpo_apply(U, v, st)  # sizes the workspace
        o.destroy()
        times = []
        for _ in range(2):
            torch.cuda.synchronize()
            t = time.perf_counter()
            o, _ = ctx.mpo_apply(U, v, st)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t)
            info = ctx.last_info()
            bonds = o.shape()[1]
            o.destroy()
        assert abs(info["norm"] - g["norm"]) <= 1e-8 * g["norm"], name
        assert np.max(np.abs(np.array(bonds) - np.array(g["ranks"]))) <= 16, name
        report[name] = {"seconds": min(times), "accepted": info["rsvd_accepted"],
                        "fallbacks": info["rsvd_fallbacks"]}
    U.destroy()
    v.destroy()
    p, prev, ex = report["predictor"], report["previous_rank"], report["exact"]
    print(json.dumps({"training_pairs": pairs, "loss": loss, "rank_predictor_gain": report,
                      "predictor_over_previous_rank": prev["seconds"] / p["seconds"],
                      "predictor_over_exact": ex["seconds"] / p["seconds"]}))
    # measured: predictor 1.13x the previous-rank sizing (48 accepted, no
    # fallback, against 15 accepted and 42 fallbacks), 0.89x the exact split;
    # the bounds leave a few per cent for box-to-box variation
    assert p["accepted"] >= 20 and p["fallbacks"] <= p["accepted"] // 10
    assert p["seconds"] <= 0.95 * prev["seconds"]
    assert p["seconds"] <= 1.2 * ex["seconds"]
