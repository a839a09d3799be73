"""Explicit Runge-Kutta steps of the diffusion equation dy/dt = Laplacian(y)
(Sec. 7.1, Laplacian of Sec. 5.1), each stage an apply or the compression of
a linear combination on the GPU: against the closed form for an eigenvector
of the open Laplacian and against dense RK4 for a generic state."""

import math

import numpy as np
import pytest

import synth
from oracle import dense
from oracle import mps as om
from paper_2601_16734_amd import binding as B
from paper_2601_16734_amd import evolution as EV

pytestmark = pytest.mark.gpu


def rk4_factor(z):
    return 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24


def test_rk4_on_an_eigenvector_matches_the_closed_form(ctx):
    n = 10
    N = 2 ** n
    dx = math.pi / (N + 1)
    y0 = synth.sine_mps(n, dx, dx)  # v_i = sin((i + 1) dx) vanishes at i = -1 and i = N
    lam = -4.0 * math.sin(dx / 2) ** 2
    H = ctx.mpo_create(synth.laplacian_mpo(n))
    st = B.strategy(8, 1e-14, sweeps=2)
    y = ctx.mps_create(y0)
    dt = 0.4
    for _ in range(3):
        y = EV.rk4_step(ctx, H, y, dt, st)
    want = rk4_factor(lam * dt) ** 3 * dense.mps_to_dense(y0)
    got = dense.mps_to_dense(y.read())
    assert np.max(np.abs(got - want)) <= 1e-11 * np.max(np.abs(want))


def test_rk4_matches_dense_rk4(ctx):
    n = 8
    N = 2 ** n
    x = np.arange(N)
    vec = np.exp(-((x - 90.0) / 20.0) ** 2) + 0.5 * np.sin(0.07 * x)
    y0 = om.tt_svd(vec, [2] * n, 64)
    Lap = dense.mpo_to_dense(synth.laplacian_mpo(n))
    dt = 0.2
    want = vec.copy()
    for _ in range(4):
        k1 = Lap @ want
        k2 = Lap @ (want + dt / 2 * k1)
        k3 = Lap @ (want + dt / 2 * k2)
        k4 = Lap @ (want + dt * k3)
        want = want + dt / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    H = ctx.mpo_create(synth.laplacian_mpo(n))
    y = ctx.mps_create(y0)
    st = B.strategy(64, 0.0, sweeps=2)  # no truncation: every rank fits
    for _ in range(4):
        y = EV.rk4_step(ctx, H, y, dt, st)
    got = dense.mps_to_dense(y.read())
    assert np.linalg.norm(got - want) <= 1e-10 * np.linalg.norm(want)


def test_euler_step(ctx):
    n = 9
    vec = np.cos(0.05 * np.arange(2 ** n)) ** 3
    y0 = om.tt_svd(vec, [2] * n, 64)
    Lap = dense.mpo_to_dense(synth.laplacian_mpo(n))
    H = ctx.mpo_create(synth.laplacian_mpo(n))
    y = EV.euler_step(ctx, H, ctx.mps_create(y0), 0.1, B.strategy(64, 0.0, sweeps=2))
    want = vec + 0.1 * (Lap @ vec)
    assert np.linalg.norm(dense.mps_to_dense(y.read()) - want) <= 1e-11 * np.linalg.norm(want)


def _diffusion_setup(ctx, n, nu=0.01):
    dx = 1.0 / 2 ** n
    dt = dx * dx / (20.0 * nu)
    lap = synth.laplacian_mpo(n, dx=dx)
    lap[0] = nu * lap[0]
    return lap, dt


def test_diffusion_benchmark_setting_matches_dense_rk4_and_oracle(ctx):
    # Gaussian (sigma = 0.1) on 2^10 points of [-0.5, 0.5), nu = 0.01,
    # dt = dx^2 / (20 nu), tolerance eps^2 / (n - 1), eps = 1e-6 (Sec. 10.3-10.4)
    from oracle import evolution as oe
    n = 10
    lap, dt = _diffusion_setup(ctx, n)
    tol = 1e-12 / (n - 1)
    st = B.strategy(32, tol, sweeps=4, sweep_tol=1e-14)
    v = synth.gaussian_grid(n)
    y0, _ = ctx.simplify(ctx.mps_create(synth.placement_mps(v, n)), st)
    assert np.linalg.norm(dense.mps_to_dense(y0.read()) - v) <= 1e-6 * np.linalg.norm(v)
    H = ctx.mpo_create(lap)
    y = y0
    for i in range(20):
        y = EV.rk4_step(ctx, H, y, dt, st)
        if i == 1:
            y2 = dense.mps_to_dense(y.read())
    want = oe.dense_rk4(dense.mpo_to_dense(lap), v, dt, 20)
    got = dense.mps_to_dense(y.read())
    err = np.linalg.norm(got - want) / np.linalg.norm(want)
    print("diffusion n=10, 20 steps: rel err vs dense RK4", err, flush=True)
    assert err <= 1e-6
    # two steps against the oracle's MPS-level RK4 from the same compressed start
    yo = y0.read()
    for _ in range(2):
        yo = oe.rk4_step(lap, yo, dt, 32, tol, sweeps=4)
    w2 = dense.mps_to_dense(yo)
    assert np.linalg.norm(y2 - w2) <= 1e-9 * np.linalg.norm(w2)
