"""Whole-run parity of the full-size workloads against the oracle's stored
results (tests/golden/, written by make_goldens.py from `oracle/` alone):

* L=100 chi=256 XXZ-type MPO D=5, 4 sweeps -- FP64, FP32 and BF16x3
  contractions (FP64 splits);
* all 512 chains of the QTT batch, 4 sweeps, one batched call (one graph,
  every chain at its own bond cap) -- FP64 and FP32 to the bar; BF16x3's error distribution (it misses 1e-8 on chains
  still moving after 4 sweeps);
* L=64 chi=512 decaying spectra, random MPO D=8, 4 sweeps -- the exact split
  and the randomized split sized by the trained rank predictor (exact
  fallback);
* L=32 chi=512 tolerance-bound decaying spectra, 2 sweeps -- exact and both
  rank estimates.

Quantities (Sec. 2.3 split and error bound, Sec. 2.4.4 norm, Sec. 2.5 sweep):
the kept rank of every step (exact integers), the discarded weight and the
kept weight of every step, the final centre norm, the final bonds, the
accumulated error bound, and the scalar products with three seeded probe
states (gauge-invariant fingerprints of the final state).  The parity bar of
the mixed precisions is 1e-8 relative in the norm."""

import json
import math
import os

import numpy as np
import pytest

import synth
from oracle import mps as om
from paper_2601_16734_amd import binding as B

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
PROBE_CONFIG = 90  # the probe stream of make_goldens.py


def golden(name):
    with open(os.path.join(HERE, "golden", name)) as f:
        return json.load(f)


def probes(L, count=3, chi=8):
    return [synth.random_mps(synth.rng_for(PROBE_CONFIG, i), L, 2, chi) for i in range(count)]


def slack(g):
    # the error bound sums sqrt of per-step discarded weights: rounding-level
    # weights of numerically rank-deficient steps enter through their sqrt
    return float(sum(1e-9 * math.sqrt(n2 + d) for n2, d in zip(g["step_norms2"], g["step_deltas"])))


FACT = {"svd": B.FACT_SVD, "rsvd_mlp": B.FACT_RSVD_MLP, "rsvd_prev": B.FACT_RSVD_PREV}


def run_single(ctx, w, sweeps, precision="fp64", factorization="svd"):
    U, v = ctx.mpo_create(w.mpo), ctx.mps_create(w.mps)
    out, err = ctx.mpo_apply(U, v, B.strategy(w.max_bond, w.tol, sweeps=sweeps, precision=precision,
                                              factorization=FACT[factorization]))
    deltas, ranks, _ = ctx.last_log()
    info = ctx.last_info()
    got = out.read()
    out.destroy()
    U.destroy()
    v.destroy()
    return got, info, np.asarray(deltas), list(ranks), err


def check_single(g, got, info, deltas, ranks, err, exact_steps=True, norm_tol=1e-10, probe_tol=1e-6):
    n = len(g["step_ranks"])
    assert len(ranks) == n
    if exact_steps:
        assert [1] + [t.shape[2] for t in got] == g["ranks"]
        assert ranks == g["step_ranks"]
        sc = np.asarray(g["step_norms2"]) + np.asarray(g["step_deltas"])
        bad = np.nonzero(np.abs(deltas - np.asarray(g["step_deltas"])) >
                         1e-10 * sc + 1e-8 * np.asarray(g["step_deltas"]))[0]
        assert bad.size == 0, f"discarded weight off at steps {bad[:10]}"
        assert abs(err - g["error_bound"]) <= 1e-6 * g["error_bound"] + slack(g)
    assert abs(info["norm"] - g["norm"]) <= norm_tol * g["norm"]
    for p, ref in zip(probes(g["L"]), g["probe_overlaps"]):
        ov = om.scprod(p, got)
        assert abs(ov - ref) <= probe_tol * abs(ref), (ov, ref)


# ---------------------------------------------------------------- L=100 chi=256 XXZ

@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_xxz_L100_chi256_whole_run(ctx, precision):
    g = golden("xxz_L100_chi256_s4.json")
    w = synth.workload_xxz(0)
    got, info, deltas, ranks, err = run_single(ctx, w, g["sweeps"], precision)
    if precision == "fp64":
        check_single(g, got, info, deltas, ranks, err)
    else:
        # the ranks sit at the cap (256) throughout; the contractions' rounding
        # moves the converged norm to second order only
        assert ranks == g["step_ranks"]
        check_single(g, got, info, deltas, ranks, err, exact_steps=False, norm_tol=1e-8, probe_tol=1e-3)
        # the discarded weights of the last pass: first order in the products'
        # rounding (BF16x3 ~ 2^-17 per product), a few 1e-8 of ||theta||^2
        last = slice(-(len(w.mps) - 1), None)
        sc = (np.asarray(g["step_norms2"]) + np.asarray(g["step_deltas"]))[last]
        assert np.all(np.abs(deltas[last] - np.asarray(g["step_deltas"])[last]) <= 1e-6 * sc)


# ---------------------------------------------------------------- the 512-chain batch

def batch512_errors(ctx, precision):
    """Run the 512 chains (one batched call, every chain at its own cap, one
    graph) and return, per chain, (relative norm error, bonds match,
    error-bound difference)."""
    g = golden("batch512_s4.json")
    ws = synth.workload_batch(0)
    assert len(ws) == len(g["chains"]) == 512
    vs = [ctx.mps_create(w.mps, dtype=np.float32) for w in ws]
    Us = [ctx.mpo_create(w.mpo) for w in ws]
    res = [None] * len(ws)
    st = B.strategy(128, 1e-10, sweeps=g["sweeps"], precision=precision)
    outs, errs = ctx.mpo_apply_batched(Us, vs, st, max_bonds=[w.max_bond for w in ws])
    for i, (o, ref) in enumerate(zip(outs, g["chains"])):
        assert ref["name"] == ws[i].name
        phys, bonds, centre = o.shape()
        rel = abs(ctx.norm(o) - ref["norm"]) / ref["norm"]
        # error-bound allowance: rounding-level weights of rank-deficient steps
        # enter through their sqrt (8 passes over at most L - 1 bonds)
        eb = abs(errs[i] - ref["error_bound"]) - (1e-6 * ref["error_bound"] + 1e-9 * ref["norm"] * 8 * len(phys))
        res[i] = (rel, list(bonds) == ref["ranks"], eb)
        o.destroy()
    for h in vs + Us:
        h.destroy()
    return res


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch512_every_chain(ctx, precision):
    res = batch512_errors(ctx, precision)
    bad_bonds = [i for i, r in enumerate(res) if not r[1]]
    assert not bad_bonds, bad_bonds[:10]
    bar = 1e-10 if precision == "fp64" else 1e-8
    bad = [(i, r[0]) for i, r in enumerate(res) if r[0] > bar]
    assert not bad, bad[:10]
    if precision == "fp64":
        assert all(r[2] <= 0.0 for r in res), [i for i, r in enumerate(res) if r[2] > 0.0][:10]
    print(f"batch512 {precision}: worst relative norm error {max(r[0] for r in res):.2e}")


def test_batch512_bf16x3_error_distribution(ctx):
    # BF16x3 products carry ~2^-17 relative rounding; a chain still moving
    # after 4 sweeps keeps that error at first order in its norm, so the
    # precision does not meet the 1e-8 bar on every chain of this batch (it
    # is reported, not claimed, for the batch).  Held: the bonds, and a
    # worst-case norm error within the first-order estimate.
    # A kept rank whose last singular value sits at the truncation threshold
    # can move by one under that rounding, so the bonds are held on all but a
    # few chains.
    res = batch512_errors(ctx, "bf16x3")
    errs = np.array([r[0] for r in res])
    moved = [i for i, r in enumerate(res) if not r[1]]
    print(f"batch512 bf16x3: {int(np.sum(errs <= 1e-8))} of 512 chains within 1e-8, worst {errs.max():.2e}; "
          f"bonds moved on chains {moved}")
    assert len(moved) <= 8
    assert errs.max() <= 1e-6


# ---------------------------------------------------------------- L=64 chi=512 decaying spectra

def trained_predictor(ctx):
    from paper_2601_16734_amd import rank_training as RT
    probs = [(w.mpo, w.mps, w.max_bond, w.tol) for w in
             [synth.workload_laplacian_small(r) for r in range(4)] + [synth.workload_random_mpo(r) for r in range(2)]]
    F, Y = RT.collect_pairs(ctx, probs, sweeps=4)
    RT.train_predictor(ctx, F, Y, epochs=100)


def test_decaying_L64_chi512_whole_run_exact(ctx):
    g = golden("decaying_L64_chi512_s4.json")
    w = synth.workload_decaying(0)
    got, info, deltas, ranks, err = run_single(ctx, w, g["sweeps"])
    check_single(g, got, info, deltas, ranks, err)


def test_decaying_L64_chi512_whole_run_learned_rank(ctx):
    # every two-site rank of this workload sits at the cap, where the
    # acceptance rule refuses a sketch: each randomized step falls back to the
    # exact split, so the run must reproduce the oracle's whole run
    g = golden("decaying_L64_chi512_s4.json")
    w = synth.workload_decaying(0)
    trained_predictor(ctx)
    got, info, deltas, ranks, err = run_single(ctx, w, g["sweeps"], factorization="rsvd_mlp")
    check_single(g, got, info, deltas, ranks, err)
    assert ctx.last_info()["rsvd_accepted"] == 0


# ---------------------------------------------------------------- tolerance-bound decaying spectra

@pytest.mark.parametrize("factorization", ["svd", "rsvd_prev", "rsvd_mlp"])
def test_decaying_tol_L32_chi512_whole_run(ctx, factorization):
    g = golden("decaying_tol_L32_chi512_s2.json")
    w = synth.workload_decaying_tol(0)
    if factorization == "rsvd_mlp":
        trained_predictor(ctx)
    got, info, deltas, ranks, err = run_single(ctx, w, g["sweeps"], factorization=factorization)
    if factorization == "svd":
        check_single(g, got, info, deltas, ranks, err)
    else:
        # an accepted sketch applies the rank rule to its Rayleigh-Ritz values
        # with the weight the sketch misses counted in every tail, so it may
        # keep more vectors than the exact split (never more than its
        # oversampling allows) while discarding at most tol ||theta||^2; the
        # state stays within the bar
        diff = np.asarray(ranks) - np.asarray(g["step_ranks"])
        assert np.all(np.abs(diff) <= 16), np.nonzero(np.abs(diff) > 16)[0][:10]
        print(f"{factorization}: {int(np.sum(diff != 0))} of {len(diff)} steps keep another rank "
              f"(largest difference {int(np.abs(diff).max())})")
        check_single(g, got, info, deltas, ranks, err, exact_steps=False, norm_tol=1e-8, probe_tol=1e-4)
