"""GPU parity of the batched (lockstep, graph-captured) apply + compression:
every problem of a batch against the single-problem path and the FP64 oracle."""

import math

import numpy as np
import pytest

import synth
from oracle import mps as om
from paper_2601_16734_amd import binding as B
from tests.gpu_helpers import cross_fidelity_loss, rel_norm_err

pytestmark = pytest.mark.gpu


def small_batch():
    rng = np.random.default_rng(77)
    out = []
    for i in range(10):
        L = int(rng.integers(3, 13))
        chi = int(rng.choice([2, 4, 8, 16]))
        mps = synth.random_mps(rng, L, 2, chi)
        kind = i % 3
        if kind == 0:
            mpo = synth.laplacian_mpo(L)
        elif kind == 1:
            mpo = synth.shift_mpo(L, 1)
        else:
            mpo = synth.random_mpo(rng, L, 2, int(rng.integers(1, 5)))
        out.append(synth.Workload(f"b{i}", mps, mpo, chi, 1e-10))
    return out


def upload(ctx, ws):
    vs = [ctx.mps_create(w.mps) for w in ws]
    Us = [ctx.mpo_create(w.mpo) for w in ws]
    return vs, Us


def test_batched_equals_single_and_oracle(ctx):
    ws = small_batch()
    vs, Us = upload(ctx, ws)
    st = B.strategy(16, 1e-10, sweeps=3)
    outs, errs = ctx.mpo_apply_batched(Us, vs, st)
    for i, w in enumerate(ws):
        one, err1 = ctx.mpo_apply(Us[i], vs[i], B.strategy(w.max_bond, 1e-10, sweeps=3))
        st_i = B.strategy(w.max_bond, 1e-10, sweeps=3)
        got = outs[i].read()
        single = one.read()
        ref = om.apply_simplify(w.mpo, w.mps, 16, 1e-10, sweeps=3)
        # the batch used max_bond 16 for all; compare with the oracle at 16
        assert [1] + [t.shape[2] for t in got] == ref.ranks, i
        assert rel_norm_err(ctx.norm(outs[i]), ref.norm) <= 1e-10, i
        assert cross_fidelity_loss(got, ref.mps) <= 1e-10, i
        assert abs(errs[i] - ref.error_bound) <= 1e-6 * ref.error_bound + 1e-12, i
        del st_i, single


def test_batched_matches_single_bitwise_on_lds_path(ctx):
    # batched launches use the one-sided Jacobi split; so does the single path here
    ws = small_batch()
    vs, Us = upload(ctx, ws)
    st = B.strategy(16, 1e-10, sweeps=2)
    outs, errs = ctx.mpo_apply_batched(Us, vs, st)
    ctx.set_split("jacobi")
    try:
        for i in range(len(ws)):
            one, err1 = ctx.mpo_apply(Us[i], vs[i], st)
            a, b = outs[i].read(), one.read()
            assert [t.shape for t in a] == [t.shape for t in b]
            for x, y in zip(a, b):
                np.testing.assert_array_equal(x, y)
            assert errs[i] == err1
    finally:
        ctx.set_split("auto")


def test_batched_graph_replay_is_deterministic(ctx):
    ws = small_batch()
    vs, Us = upload(ctx, ws)
    st = B.strategy(16, 1e-10, sweeps=2)
    first, e1 = ctx.mpo_apply_batched(Us, vs, st)
    a = [o.read() for o in first]
    for _ in range(2):
        again, e2 = ctx.mpo_apply_batched(Us, vs, st)
        assert e1 == e2
        for x, o in zip(a, again):
            for s1, s2 in zip(x, o.read()):
                np.testing.assert_array_equal(s1, s2)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_batched_mixed_precision_vs_oracle(ctx, precision):
    ws = small_batch()
    vs, Us = upload(ctx, ws)
    outs, errs = ctx.mpo_apply_batched(Us, vs, B.strategy(16, 1e-10, sweeps=3, precision=precision))
    for i, w in enumerate(ws):
        ref = om.apply_simplify(w.mpo, w.mps, 16, 1e-10, sweeps=3)
        got = outs[i].read()
        assert rel_norm_err(ctx.norm(outs[i]), ref.norm) <= 1e-8, (precision, i)
        assert cross_fidelity_loss(got, ref.mps) <= 1e-8, (precision, i)


@pytest.fixture(scope="module")
def qtt_sample():
    """The first 16 problems of the 512-problem QTT batch (n in [8, 30], chi in
    {4, ..., 128}, FP32 inputs, Laplacian or shift), including a chi = 128
    chain whose two-site tensors exceed the LDS and take the blocked path."""
    return synth.workload_batch(count=16)


def test_qtt_batch_sample_vs_oracle(ctx, qtt_sample):
    ws = qtt_sample
    vs = [ctx.mps_create(w.mps, dtype=np.float32) for w in ws]
    Us = [ctx.mpo_create(w.mpo) for w in ws]
    # each problem keeps its own chi as the bond cap: batch problems by cap
    by_cap = {}
    for i, w in enumerate(ws):
        by_cap.setdefault(w.max_bond, []).append(i)
    for cap, idx in sorted(by_cap.items()):
        outs, errs = ctx.mpo_apply_batched([Us[i] for i in idx], [vs[i] for i in idx], B.strategy(cap, 1e-10))
        for o, i in zip(outs, idx):
            w = ws[i]
            mps64 = [t.astype(np.float64) for t in w.mps]
            ref = om.apply_simplify(w.mpo, mps64, cap, 1e-10, sweeps=4)
            got = o.read()
            ne, fl = rel_norm_err(ctx.norm(o), ref.norm), cross_fidelity_loss(got, ref.mps)
            print(f"problem {i} n={w.meta['n']} chi={cap}: norm err {ne:.2e} fidelity loss {fl:.2e}")
            assert ne <= 1e-8 and fl <= 1e-8, i


def test_single_blocked_path_vs_oracle(ctx, qtt_sample):
    w = [x for x in qtt_sample if x.meta["chi"] == 128][0]
    v = ctx.mps_create(w.mps, dtype=np.float32)
    U = ctx.mpo_create(w.mpo)
    out, err = ctx.mpo_apply(U, v, B.strategy(128, 1e-10))
    ref = om.apply_simplify(w.mpo, [t.astype(np.float64) for t in w.mps], 128, 1e-10, sweeps=4)
    got = out.read()
    assert rel_norm_err(ctx.last_info()["norm"], ref.norm) <= 1e-8
    assert cross_fidelity_loss(got, ref.mps) <= 1e-8


def test_batched_refuses_a_graph_beyond_its_kernel_limit(ctx):
    # every step adds a bounded number of kernels (the blocked factorization
    # runs all its sweeps in one persistent launch), so only a very long chain
    # reaches the graph limit: L = 1000 with 4 sweeps, refused before capture
    L = 1000
    phys, bonds = [2] * L, synth.bond_caps(L, 2, 8)
    v = ctx.mps_zeros(phys, bonds)
    U = ctx.mpo_zeros(phys, phys, [1] + [2] * (L - 1) + [1])
    st = B.strategy(8, 1e-10, sweeps=4)
    with pytest.raises(B.SmpsError) as e:
        ctx.plan_apply_batched([U], [v], st)
    assert e.value.code == B.EUNSUPPORTED and e.value.info["graph_kernels"] > 100000
    with pytest.raises(B.SmpsError) as e:
        ctx.mpo_apply_batched([U], [v], st)
    assert e.value.code == B.EUNSUPPORTED
    assert "limit" in str(e.value)
    v.destroy()
    U.destroy()


def test_l100_chi256_chain_in_a_batch_matches_the_oracle_run(ctx):
    # the chain whose batched capture once held 2.2e5 kernels: its 512 x 512
    # two-site tensors take the persistent blocked factorization; the batch
    # also holds a short chain of the QTT batch.  Against the oracle's whole
    # run (tests/golden, 4 sweeps, FP64): bonds, norm, error bound, probes.
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "xxz_L100_chi256_s4.json")))
    w = synth.workload_xxz(0)
    small = synth.workload_batch(0)[0]
    vs, Us = upload(ctx, [w, small])
    plan = ctx.plan_apply_batched(Us, vs, B.strategy(256, 1e-10, sweeps=4))
    assert plan["graph_kernels"] < 100000
    outs, errs = ctx.mpo_apply_batched(Us, vs, B.strategy(256, 1e-10, sweeps=4))
    got = outs[0].read()
    assert [1] + [t.shape[2] for t in got] == g["ranks"]
    assert rel_norm_err(ctx.norm(outs[0]), g["norm"]) <= 1e-10
    slack = sum(1e-9 * np.sqrt(n2 + d) for n2, d in zip(g["step_norms2"], g["step_deltas"]))
    assert abs(errs[0] - g["error_bound"]) <= 1e-6 * g["error_bound"] + slack
    probes = [synth.random_mps(synth.rng_for(90, i), 100, 2, 8) for i in range(3)]
    for p, ref in zip(probes, g["probe_overlaps"]):
        assert abs(om.scprod(p, got) - ref) <= 1e-6 * abs(ref)
    # the short chain (max bond 256 here, above its own chi): its oracle run
    ref = om.apply_simplify([np.asarray(x, np.float64) for x in small.mpo],
                            [np.asarray(x, np.float64) for x in small.mps], 256, 1e-10, sweeps=4)
    assert rel_norm_err(ctx.norm(outs[1]), ref.norm) <= 1e-10
    assert [1] + [t.shape[2] for t in outs[1].read()] == ref.ranks


def test_batched_blocked_launch_with_long_and_short_rows(ctx):
    # chi = 256 and chi = 128 chains in one batch: at the bulk steps their
    # blocked factorizations share a launch shaped for the longer (512) rows,
    # the shorter rows zero padded; each result must match its oracle run
    rng = np.random.default_rng(141)
    ws = []
    for chi in (256, 128):
        mps = synth.random_mps(rng, 16, 2, chi)
        mpo = synth.random_mpo(rng, 16, 2, 2)
        ws.append(synth.Workload(f"chi{chi}", mps, mpo, 256, 1e-10))
    vs, Us = upload(ctx, ws)
    outs, errs = ctx.mpo_apply_batched(Us, vs, B.strategy(256, 1e-10, sweeps=1))
    for i, w in enumerate(ws):
        ref = om.apply_simplify(w.mpo, w.mps, 256, 1e-10, sweeps=1)
        got = outs[i].read()
        assert [1] + [t.shape[2] for t in got] == ref.ranks, i
        assert rel_norm_err(ctx.norm(outs[i]), ref.norm) <= 1e-10, i
        assert cross_fidelity_loss(got, ref.mps) <= 1e-10, i
