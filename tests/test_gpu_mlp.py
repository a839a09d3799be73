"""GPU parity of the rank predictor's hand-written kernels (forward, backward,
Adam) against the FP64 oracle network, on synthetic inputs and weights."""

import numpy as np
import pytest

import synth
from oracle import mlp as om

pytestmark = pytest.mark.gpu


def _away_from_kinks(params, X, y, margin=1e-3):
    """Rows whose pre-activations and loss residual stay clear of the ReLU and
    Huber kinks, where FP32 and FP64 may legitimately take different branches."""
    _, (Xd, z1, h1, z2, h2, _, _) = om.forward(params, X)
    pred = om.forward(params, X)[0]
    e = pred - y
    ok = (np.abs(z1).min(1) > margin) & (np.abs(z2).min(1) > margin)
    ok &= (np.abs(e) > margin) & (np.abs(np.abs(e) - om.HUBER_DELTA) > margin)
    return ok


def _setup(ctx, seed, n):
    rng = np.random.default_rng(seed)
    params = synth.mlp_params(rng)
    X, y = synth.mlp_inputs(rng, n)
    ok = _away_from_kinks(params.astype(np.float64), X, y)
    X, y = X[ok], y[ok]
    ctx.rank_mlp_set(params)
    return params, X, y


def test_mlp_forward_matches_oracle(ctx):
    params, X, y = _setup(ctx, 11, 300)
    got = ctx.rank_mlp_predict(X)
    ref = om.forward(params.astype(np.float64), X)[0]
    scale = np.abs(ref).max()
    assert np.max(np.abs(got - ref)) <= 2e-5 * scale


@pytest.mark.parametrize("n", [1, 31, 32, 33, 257])
def test_mlp_gradient_matches_oracle(ctx, n):
    params, X, y = _setup(ctx, 100 + n, n + 40)
    X, y = X[:n], y[:n]
    loss, grad = ctx.rank_mlp_grad(X, y)
    rloss, rgrad = om.loss_and_grad(params.astype(np.float64), X, y)
    assert abs(loss - rloss) <= 2e-5 * max(1.0, abs(rloss))
    o = 0
    for shape in om.SIZES:
        k = int(np.prod(shape))
        g, r = grad[o:o + k], rgrad[o:o + k]
        assert np.max(np.abs(g - r)) <= 5e-5 * max(np.abs(r).max(), 1e-6), shape
        o += k


def test_mlp_one_adam_step_matches_oracle(ctx):
    params, X, y = _setup(ctx, 7, 140)
    n = len(y)
    lr = 1e-3
    ctx.rank_mlp_train(X, y, epochs=1, batch=n, lr=lr)
    got = ctx.rank_mlp_get()
    _, g = om.loss_and_grad(params.astype(np.float64), X, y)
    ref, _, _ = om.adam_step(params.astype(np.float64), g, np.zeros_like(g), np.zeros_like(g), 1, lr)
    # a coordinate moves by about lr * sign(g); near-zero gradients are FP32-noise dominated
    big = np.abs(g) > 1e-3 * np.abs(g).max()
    assert np.max(np.abs(got - ref)[big]) <= 1e-6
    assert np.max(np.abs(got - ref)) <= 1.01 * lr + 1e-6


def test_mlp_training_reduces_loss(ctx):
    """Labels from a fixed smooth rule of the spectrum: the network must fit them."""
    rng = np.random.default_rng(5)
    X, _ = synth.mlp_inputs(rng, 2048)
    # number of values above 1e-5 of the largest (a rank-like target)
    y = np.log(np.maximum(1.0, (X > np.log(1e-5)).sum(1))).astype(np.float32)
    ctx.rank_mlp_init(3)
    l0, _ = ctx.rank_mlp_grad(X, y)
    last = ctx.rank_mlp_train(X, y, epochs=40, batch=256, lr=1e-3)
    l1, _ = ctx.rank_mlp_grad(X, y)
    assert np.isfinite(last) and l1 < 0.2 * l0, (l0, l1, last)
