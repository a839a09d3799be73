"""Workspace limit and planning on a device context: a limit below what
the apply needs is refused with SMPS_ENOMEM before any device work, and the
host-side plan of a device context equals a planning context's (the path
decisions depend on the gfx950 LDS budget only)."""

import pytest

import synth
from paper_2601_16734_amd import binding as B

pytestmark = pytest.mark.gpu


def test_workspace_limit_on_a_device_context(ctx):
    w = synth.workload_random_mpo(0, L=12, chi=32, D=4)
    U, v = ctx.mpo_create(w.mpo), ctx.mps_create(w.mps)
    st = B.strategy(32, 1e-10, sweeps=2)
    need = ctx.plan_apply(U, v, st)["workspace_bytes"]
    try:
        ctx.set_workspace_limit(need - 1)
        with pytest.raises(B.SmpsError) as e:
            ctx.mpo_apply(U, v, st)
        assert e.value.code == B.ENOMEM
        assert ctx.workspace_bytes() <= need - 1
        ctx.set_workspace_limit(need)
        out, _ = ctx.mpo_apply(U, v, st)
        assert ctx.workspace_bytes() == need  # the arena's headroom is cut at the limit
        ref = ctx.norm(out)
        out.destroy()
    finally:
        ctx.set_workspace_limit(0)
    out, _ = ctx.mpo_apply(U, v, st)
    assert ctx.norm(out) == ref
    for h in (out, U, v):
        h.destroy()


def test_device_plan_equals_the_planning_context_plan(ctx):
    p = B.Context.planning()
    try:
        for L, chi, D in [(20, 64, 8), (100, 256, 5), (24, 128, 3)]:
            phys, bonds = [2] * L, synth.bond_caps(L, 2, chi)
            ob = [1] + [D] * (L - 1) + [1]
            st = B.strategy(chi, 1e-10, sweeps=4)
            a = ctx.plan_apply(ctx.mpo_zeros(phys, phys, ob), ctx.mps_zeros(phys, bonds), st)
            b = p.plan_apply(p.mpo_zeros(phys, phys, ob), p.mps_zeros(phys, bonds), st)
            assert a == b, (L, chi, a, b)
            if chi <= 128:
                a = ctx.plan_apply_batched([ctx.mpo_zeros(phys, phys, ob)], [ctx.mps_zeros(phys, bonds)], st)
                b = p.plan_apply_batched([p.mpo_zeros(phys, phys, ob)], [p.mps_zeros(phys, bonds)], st)
                assert a == b, (L, chi, a, b)
    finally:
        p.close()


def test_destroyed_handle_is_refused_on_a_device_context(ctx):
    w = synth.workload_laplacian_small(0)
    U, v = ctx.mpo_create(w.mpo), ctx.mps_create(w.mps)
    raw = v.h
    v.destroy()
    v.h = raw
    with pytest.raises(B.SmpsError) as e:
        ctx.mpo_apply(U, v, B.strategy(8, 1e-10))
    assert e.value.code == B.EINVAL
    v.h = None
    U.destroy()
