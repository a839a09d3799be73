"""Full-size workloads (L=100 chi=256 XXZ; L=64 chi=512 decaying spectra):
the oracle cannot finish a whole run in test time, so parity is checked on
the outputs it can compute one by one -- the rank and discarded weight of
the first steps of the sweep -- and on properties that hold at any size:
isometric sites, the centre norm against the scalar product, and mixed
against FP64 precision."""

import math

import numpy as np
import pytest

import synth
from oracle import mps as om
from paper_2601_16734_amd import binding as B

pytestmark = pytest.mark.gpu

SAMPLED_STEPS = 12


def isometry_residual(t):
    a, s, b = t.shape
    M = t.reshape(a, s * b)
    return float(np.abs(M @ M.T - np.eye(a)).max())


def run(ctx, w, sweeps, precision="fp64"):
    out, err = ctx.mpo_apply(ctx.mpo_create(w.mpo), ctx.mps_create(w.mps),
                             B.strategy(w.max_bond, w.tol, sweeps=sweeps, precision=precision))
    deltas, ranks, _ = ctx.last_log()
    return out, ctx.last_info(), deltas, ranks


def check_first_steps(w, sweeps, deltas, ranks):
    ref = om.apply_simplify(w.mpo, w.mps, w.max_bond, w.tol, sweeps=sweeps, max_steps=SAMPLED_STEPS)
    assert list(ranks[:SAMPLED_STEPS]) == ref.step_ranks
    for k in range(SAMPLED_STEPS):
        scale = ref.norms2[k] + ref.deltas[k]  # ||theta||^2 of the step
        assert abs(deltas[k] - ref.deltas[k]) <= 1e-10 * scale + 1e-8 * ref.deltas[k], k


def check_state(ctx, out, info, sites=None):
    psi = out.read()
    idx = range(1, len(psi)) if sites is None else sites
    for k in idx:
        assert isometry_residual(psi[k]) <= 1e-10, k
    nn = math.sqrt(ctx.scprod(out, out))
    assert abs(nn - info["norm"]) <= 1e-12 * info["norm"]


def test_xxz_L100_chi256_sampled_parity_and_mixed_precision(ctx):
    # the configured 4 sweeps: before convergence the compressed norm moves
    # with the rounding of the contractions to first order (FP32 after 2
    # sweeps: 2.3e-8 from FP64), after it only to second order
    w = synth.workload_xxz(0)
    out, info, deltas, ranks = run(ctx, w, sweeps=4)
    check_first_steps(w, 4, deltas, ranks)
    check_state(ctx, out, info)
    out32, info32, _, _ = run(ctx, w, sweeps=4, precision="fp32")
    assert abs(info32["norm"] - info["norm"]) <= 1e-8 * info["norm"]
    f = ctx.scprod(out, out32) / (info["norm"] * info32["norm"])
    assert abs(1.0 - f) <= 1e-8


def test_decaying_L64_chi512_sampled_parity(ctx):
    w = synth.workload_decaying(0)
    out, info, deltas, ranks = run(ctx, w, sweeps=1)
    check_first_steps(w, 1, deltas, ranks)
    check_state(ctx, out, info, sites=[1, 2, 16, 31, 32, 48, 62, 63])


def test_blocked_factorizations_vs_whole_oracle(ctx):
    # L=18 chi=256: the bulk two-site tensors are 512 x 512 and their edges
    # 256 x 512, beyond one workgroup's LDS; their rows (256 and 512 long)
    # take the blocked path with 16-lane and whole-wave pair groups.  Small
    # enough for the whole oracle run.
    rng = np.random.default_rng(140)
    mps = synth.random_mps(rng, 18, 2, 256)
    mpo = synth.random_mpo(rng, 18, 2, 2)
    ref = om.apply_simplify(mpo, mps, 256, 1e-10, sweeps=2)
    out, err = ctx.mpo_apply(ctx.mpo_create(mpo), ctx.mps_create(mps), B.strategy(256, 1e-10, sweeps=2))
    info = ctx.last_info()
    got = out.read()
    assert [1] + [t.shape[2] for t in got] == ref.ranks
    assert abs(info["norm"] - ref.norm) <= 1e-10 * ref.norm
    ab = om.scprod(got, ref.mps)
    assert 1.0 - abs(ab) / math.sqrt(om.scprod(got, got) * om.scprod(ref.mps, ref.mps)) <= 1e-10
    assert abs(err - ref.error_bound) <= 1e-6 * ref.error_bound + 1e-12
    check_state(ctx, out, info)


def test_round_kernel_rows_beyond_1024_vs_whole_oracle(ctx):
    # L=3, d=40, chi=40, bond cap 24: the two-site tensors are 40 x 1600 and
    # 1600 x 40.  The splits whose vectors are the 40 rows of 1600 elements
    # (left-to-right at the second bond, right-to-left at the first) take the
    # global-memory round kernel (rows beyond 1024 elements, one wave per
    # pair, one launch per round); the others (1600 vectors of 40 elements)
    # the blocked path.  The cap truncates every step.
    rng = np.random.default_rng(141)
    mps = synth.random_mps(rng, 3, 40, 40)
    mpo = synth.random_mpo(rng, 3, 40, 2)
    ref = om.apply_simplify(mpo, mps, 24, 1e-12, sweeps=2)
    out, err = ctx.mpo_apply(ctx.mpo_create(mpo), ctx.mps_create(mps), B.strategy(24, 1e-12, sweeps=2))
    info = ctx.last_info()
    deltas, ranks, _ = ctx.last_log()
    got = out.read()
    assert [1] + [t.shape[2] for t in got] == ref.ranks == [1, 24, 24, 1]
    assert list(ranks) == ref.step_ranks
    for k in range(len(ref.deltas)):
        scale = ref.norms2[k] + ref.deltas[k]
        assert abs(deltas[k] - ref.deltas[k]) <= 1e-10 * scale, k
    assert abs(info["norm"] - ref.norm) <= 1e-12 * ref.norm
    ab = om.scprod(got, ref.mps)
    assert 1.0 - abs(ab) / math.sqrt(om.scprod(got, got) * om.scprod(ref.mps, ref.mps)) <= 1e-12
    assert abs(err - ref.error_bound) <= 1e-6 * ref.error_bound + 1e-12
    check_state(ctx, out, info)
