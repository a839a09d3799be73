"""Observability of the single-problem sweep: per-phase kernel timing (HIP
events around every launch when profiling is on) partitions the launches as
documented and changes no result; the same input run twice gives the same
bits."""

import pytest

import synth
from paper_2601_16734_amd import binding as B

pytestmark = pytest.mark.gpu


def test_phase_timers_partition_the_launches(ctx):
    w = synth.workload_random_mpo(0, L=12, chi=32, D=4)
    U, v = ctx.mpo_create(w.mpo), ctx.mps_create(w.mps)
    st = B.strategy(32, 1e-10, sweeps=2)
    ref, _ = ctx.mpo_apply(U, v, st)
    ref_norm = ctx.last_info()["norm"]
    steps = ctx.last_info()["steps"]
    ctx.set_profiling(True)
    try:
        out, _ = ctx.mpo_apply(U, v, st)
        t = {c: ctx.kernel_time(c) for c in range(7)}
    finally:
        ctx.set_profiling(False)
    assert ctx.last_info()["norm"] == ref_norm  # timing changes nothing
    assert steps == 2 * 2 * (12 - 1)
    # one two-site product per step; one split per step plus the L - 1 of the
    # guess's canonical form
    assert t[4][1] == steps
    assert t[0][1] == steps + 12 - 1
    assert 0 < t[2][1] <= t[0][1] and t[2][0] <= t[0][0]
    for c in (3, 5):
        assert t[c][1] >= steps
    # phases 3-5 are contractions (category 1); the rest of 1 lies outside the steps
    assert t[3][1] + t[4][1] + t[5][1] < t[1][1]
    assert t[3][0] + t[4][0] + t[5][0] <= t[1][0] * (1 + 1e-9)
    assert t[6][1] > 0
    assert all(t[c][0] > 0 for c in range(7))
    for h in (out, ref, U, v):
        h.destroy()


@pytest.mark.parametrize("precision", ["fp64", "bf16x3"])
def test_single_path_is_deterministic(ctx, precision):
    # the same input twice gives the same bits: every reduction on the path
    # (dot products, norms, tail sums, GEMM k order) has a fixed order
    import numpy as np
    w = synth.workload_random_mpo(0)
    U, v = ctx.mpo_create(w.mpo), ctx.mps_create(w.mps)
    st = B.strategy(w.max_bond, w.tol, sweeps=2, precision=precision)
    runs = []
    for _ in range(2):
        out, err = ctx.mpo_apply(U, v, st)
        deltas, ranks, _ = ctx.last_log()
        runs.append((out.read(), err, np.array(deltas), list(ranks)))
        out.destroy()
    (a, ea, da, ra), (b, eb, db, rb) = runs
    assert ea == eb and ra == rb
    np.testing.assert_array_equal(da, db)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)
    U.destroy()
    v.destroy()
