"""GEMM tile autotuner: tuning every product shape of an apply, the table's
save/load round trip, and that the chosen tiles never change result bits
(single and batched paths)."""

import numpy as np
import pytest

import synth
from paper_2601_16734_amd import binding as B

pytestmark = pytest.mark.gpu


def apply_read(ctx, w, precision):
    out, _ = ctx.mpo_apply(ctx.mpo_create(w.mpo), ctx.mps_create(w.mps),
                           B.strategy(w.max_bond, w.tol, sweeps=2, precision=precision))
    return out.read(), ctx.last_info()["norm"]


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_tuned_tiles_give_identical_results(ctx, precision):
    w = synth.workload_random_mpo(1, L=10, chi=32, D=4)
    ctx.autotune_clear()
    ref, nref = apply_read(ctx, w, precision)
    U, v = ctx.mpo_create(w.mpo), ctx.mps_create(w.mps)
    tuned = ctx.autotune_apply(U, v, B.strategy(w.max_bond, w.tol, sweeps=2, precision=precision), reps=3)
    assert tuned > 0 and ctx.autotune_entries() >= tuned
    got, ngot = apply_read(ctx, w, precision)
    assert ngot == nref
    for a, b in zip(got, ref):
        np.testing.assert_array_equal(a, b)
    ctx.autotune_clear()


def test_each_tile_and_the_table_roundtrip(ctx, tmp_path):
    ctx.autotune_clear()
    tiles = {ctx.autotune_gemm("fp64", M, N, K, reps=3) for (M, N, K) in [(128, 128, 512), (64, 512, 64), (512, 512, 32)]}
    assert tiles <= {0, 1, 2, 3}
    n = ctx.autotune_entries()
    assert n == 3
    path = tmp_path / "tiles.json"
    ctx.autotune_save(path)
    ctx.autotune_clear()
    assert ctx.autotune_entries() == 0
    ctx.autotune_load(path)
    assert ctx.autotune_entries() == n
    bad = tmp_path / "bad.json"
    bad.write_text('[\n  {"precision": 0, "tile": 9}\n]\n')
    with pytest.raises(B.SmpsError):
        ctx.autotune_load(bad)
    ctx.autotune_clear()


def test_batched_results_unchanged_by_tuning(ctx):
    rng = np.random.default_rng(3)
    ws = [(synth.laplacian_mpo(L), synth.random_mps(rng, L, 2, 16)) for L in (6, 9, 12)]
    st = B.strategy(16, 1e-10, sweeps=2)
    Us = [ctx.mpo_create(m) for m, _ in ws]
    vs = [ctx.mps_create(s) for _, s in ws]
    ctx.autotune_clear()
    ref, _ = ctx.mpo_apply_batched(Us, vs, st)
    ref = [o.read() for o in ref]
    for U, v in zip(Us, vs):
        ctx.autotune_apply(U, v, st, reps=2)
    got, _ = ctx.mpo_apply_batched(Us, vs, st)
    for o, r in zip(got, ref):
        for a, b in zip(o.read(), r):
            np.testing.assert_array_equal(a, b)
    ctx.autotune_clear()
