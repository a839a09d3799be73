"""Operator utilities on the GPU (Sec. 2.4.1-2.4.3): transpose, product from
the right, a list of operators applied in turn, and operator compression."""

import numpy as np
import pytest

import synth
from oracle import dense
from oracle import mps as om
from paper_2601_16734_amd import binding as B

pytestmark = pytest.mark.gpu


def joined(mpos, weights):
    """Block sum of MPOs (the sum operator, bond = sum of bonds), built site by site."""
    L = len(mpos[0])
    out = []
    for k in range(L):
        blocks = [m[k] for m in mpos]
        if k == 0:
            out.append(np.concatenate([w * b for w, b in zip(weights, blocks)], axis=3))
        elif k == L - 1:
            out.append(np.concatenate(blocks, axis=0))
        else:
            Dl = sum(b.shape[0] for b in blocks)
            Dr = sum(b.shape[3] for b in blocks)
            d = blocks[0].shape[1]
            t = np.zeros((Dl, d, d, Dr))
            i = j = 0
            for b in blocks:
                t[i:i + b.shape[0], :, :, j:j + b.shape[3]] = b
                i += b.shape[0]
                j += b.shape[3]
            out.append(t)
    return out


def test_transpose_exchanges_site_indices(ctx):
    rng = np.random.default_rng(0)
    mpo = synth.random_mpo(rng, 5, 3, 4)
    T = ctx.mpo_transpose(ctx.mpo_create(mpo)).read()
    for a, b in zip(T, mpo):
        np.testing.assert_array_equal(a, np.transpose(b, (0, 2, 1, 3)))


def test_apply_from_the_right_is_the_transposed_product(ctx):
    rng = np.random.default_rng(1)
    mps = synth.random_mps(rng, 6, 2, 4)
    mpo = synth.random_mpo(rng, 6, 2, 3)
    out, _ = ctx.mpo_apply_right(ctx.mps_create(mps), ctx.mpo_create(mpo), B.strategy(64, 0.0, sweeps=2))
    want = dense.mpo_to_dense(mpo).T @ dense.mps_to_dense(mps)
    got = dense.mps_to_dense(out.read())
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))


def test_operator_list_applied_in_turn(ctx):
    rng = np.random.default_rng(2)
    mps = synth.random_mps(rng, 10, 2, 8)
    U1 = synth.random_mpo(rng, 10, 2, 3)
    U2 = synth.laplacian_mpo(10)
    st = B.strategy(8, 1e-10, sweeps=2)
    out, _ = ctx.mpo_list_apply([ctx.mpo_create(U1), ctx.mpo_create(U2)], ctx.mps_create(mps), st)
    r1 = om.apply_simplify(U1, mps, 8, 1e-10, sweeps=2)
    r2 = om.apply_simplify(U2, r1.mps, 8, 1e-10, sweeps=2)
    got = out.read()
    assert [1] + [t.shape[2] for t in got] == r2.ranks
    f = om.scprod(got, r2.mps) / np.sqrt(om.scprod(got, got) * om.scprod(r2.mps, r2.mps))
    assert abs(1 - f) <= 1e-10


def test_operator_compression(ctx):
    n = 8
    lap = synth.laplacian_mpo(n)
    redundant = joined([lap, lap], [0.25, 0.75])  # bond 6, equal to the Laplacian (bond 3)
    U, _ = ctx.mpo_simplify(ctx.mpo_create(redundant), B.strategy(16, 1e-14, sweeps=2))
    pout, pin, bonds = U.shape()
    assert pout == [2] * n and pin == [2] * n
    assert max(bonds) <= 3
    got = dense.mpo_to_dense(U.read())
    want = dense.mpo_to_dense(lap)
    assert np.max(np.abs(got - want)) <= 1e-12
