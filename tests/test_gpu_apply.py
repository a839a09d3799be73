"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Compared quantities are gauge invariant (norms, overlaps, dense vectors for
small chains, discarded weights); site tensors after an SVD are defined only up
to rotations inside the kept subspace and are never compared entry by entry.
Tolerance: 1e-8 relative in fidelity and norm, the bar the workloads set for
every precision that claims parity; FP64 cases are also held to tighter checks
where the arithmetic allows.
"""

import math

import numpy as np
import pytest

import synth
from oracle import dense, mps as om
from paper_2601_16734_amd import binding as B
from tests.gpu_helpers import cross_fidelity_loss, error_bound_slack, isometry_residual_right, rel_norm_err

pytestmark = pytest.mark.gpu


def rand_mps(rng, dims, bonds):
    return [rng.standard_normal((bonds[k], dims[k], bonds[k + 1])) for k in range(len(dims))]


# ---------------------------------------------------------------- scalar product / norm

@pytest.mark.parametrize("L,chi,seed", [(1, 1, 0), (3, 2, 1), (9, 7, 2), (12, 70, 3), (20, 64, 4)])
def test_scprod_matches_oracle(ctx, L, chi, seed):
    rng = np.random.default_rng(seed)
    a = synth.random_mps(rng, L, 2, chi)
    b = synth.random_mps(rng, L, 2, max(1, chi // 2 + 1))
    ga, gb = ctx.mps_create(a), ctx.mps_create(b)
    got = ctx.scprod(ga, gb)
    ref = om.scprod(a, b)
    scale = math.sqrt(om.scprod(a, a) * om.scprod(b, b))
    assert abs(got - ref) <= 1e-12 * scale
    assert abs(ctx.norm(ga) - math.sqrt(om.scprod(a, a))) <= 1e-12 * math.sqrt(om.scprod(a, a))


def test_mps_roundtrip_mixed_phys(ctx):
    rng = np.random.default_rng(5)
    a = rand_mps(rng, [2, 3, 4, 2], [1, 3, 5, 2, 1])
    g = ctx.mps_create(a)
    back = g.read()
    for x, y in zip(a, back):
        np.testing.assert_array_equal(x, y)
    phys, bonds, center = g.shape()
    assert phys == [2, 3, 4, 2] and bonds == [1, 3, 5, 2, 1] and center == -1
    gf = ctx.mps_create([x.astype(np.float32) for x in a], dtype=np.float32)
    for x, y in zip(a, gf.read()):
        np.testing.assert_array_equal(x.astype(np.float32).astype(np.float64), y)


# ---------------------------------------------------------------- apply + compress, FP64

def run_gpu(ctx, w, precision="fp64", sweeps=None, max_bond=None, tol=None):
    v = ctx.mps_create(w.mps)
    U = ctx.mpo_create(w.mpo)
    st = B.strategy(max_bond or w.max_bond, w.tol if tol is None else tol, sweeps=sweeps or w.sweeps,
                    precision=precision)
    out, err = ctx.mpo_apply(U, v, st)
    return out.read(), err, ctx.last_info(), out


def test_laplacian_small_vs_oracle_and_dense(ctx):
    w = synth.workload_laplacian_small()
    nrm = math.sqrt(om.scprod(w.mps, w.mps))
    w.mps[0] = w.mps[0] / nrm  # normalised input state
    ref = om.apply_simplify(w.mpo, w.mps, w.max_bond, w.tol, sweeps=4)
    got, err, info, h = run_gpu(ctx, w)
    assert [1] + [t.shape[2] for t in got] == ref.ranks
    assert rel_norm_err(info["norm"], ref.norm) <= 1e-12
    assert cross_fidelity_loss(got, ref.mps) <= 1e-12
    uv = dense.mpo_to_dense(w.mpo) @ dense.mps_to_dense(w.mps)
    psi = dense.mps_to_dense(got)
    # projection invariant and the accumulated error bound
    assert abs(psi @ uv - psi @ psi) <= 1e-11 * (uv @ uv)
    assert np.linalg.norm(psi - uv) <= err * (1 + 1e-6) + 1e-12 * np.linalg.norm(uv)
    assert abs(err - ref.error_bound) <= 1e-6 * max(ref.error_bound, 1e-300) + 1e-13 + error_bound_slack(ref)
    for k in range(1, len(got)):
        assert isometry_residual_right(got[k]) <= 1e-12
    assert abs(ctx.norm(h) - ref.norm) <= 1e-12 * ref.norm


def test_laplacian_exact_variant_is_dense_product(ctx):
    w = synth.workload_laplacian_small(max_bond=32, tol=0.0)
    got, err, info, _ = run_gpu(ctx, w)
    uv = dense.mpo_to_dense(w.mpo) @ dense.mps_to_dense(w.mps)
    assert np.linalg.norm(dense.mps_to_dense(got) - uv) <= 1e-11 * np.linalg.norm(uv)


def test_simplify_reproduces_state(ctx):
    rng = np.random.default_rng(11)
    v = synth.random_mps(rng, 9, 2, 6)
    g = ctx.mps_create(v)
    out, err = ctx.simplify(g, B.strategy(32, 0.0, sweeps=1))
    got = out.read()
    assert cross_fidelity_loss(got, v) <= 1e-13
    assert rel_norm_err(ctx.norm(out), math.sqrt(om.scprod(v, v))) <= 1e-12


@pytest.mark.parametrize("L,chi,D,sweeps", [(2, 4, 2, 1), (5, 3, 3, 2), (10, 8, 4, 3), (11, 20, 5, 2)])
def test_random_mpo_small_vs_oracle(ctx, L, chi, D, sweeps):
    w = synth.workload_random_mpo(rep=L, L=L, chi=chi, D=D)
    ref = om.apply_simplify(w.mpo, w.mps, chi, 1e-10, sweeps=sweeps)
    got, err, info, _ = run_gpu(ctx, w, sweeps=sweeps, max_bond=chi, tol=1e-10)
    assert [1] + [t.shape[2] for t in got] == ref.ranks
    assert rel_norm_err(info["norm"], ref.norm) <= 1e-10
    assert cross_fidelity_loss(got, ref.mps) <= 1e-10


@pytest.fixture(scope="module")
def c2_oracle():
    w = synth.workload_random_mpo()
    return w, om.apply_simplify(w.mpo, w.mps, w.max_bond, w.tol, sweeps=w.sweeps)


def test_random_mpo_n20_chi64_fp64(ctx, c2_oracle):
    w, ref = c2_oracle
    got, err, info, _ = run_gpu(ctx, w)
    assert rel_norm_err(info["norm"], ref.norm) <= 1e-8
    assert cross_fidelity_loss(got, ref.mps) <= 1e-8
    assert info["steps"] == 4 * 2 * 19


def test_accumulated_edge_steps_warm_start_from_their_last_visit(ctx, c2_oracle):
    """n=20 chi=64 D=8, 4 sweeps: the first six steps of every pass (bond
    dimensions growing from the chain's end) factorize the shorter side with
    accumulated rotations, each starting from the J that the same step of the
    previous pass in that direction left.  Their rotating Jacobi sweeps in the
    last pass of each direction stay well below the first pass of that
    direction (started from the identity they would stay within ~10% of it),
    and the result keeps FP64 parity with the oracle."""
    w, ref = c2_oracle
    got, err, info, _ = run_gpu(ctx, w)
    assert rel_norm_err(info["norm"], ref.norm) <= 1e-12
    assert cross_fidelity_loss(got, ref.mps) <= 1e-12
    js = ctx.last_jacobi_log()
    n = len(w.mps) - 1  # steps per pass
    passes = 2 * w.sweeps
    assert len(js) == passes * n
    lead = [sum(js[p * n:p * n + 6]) for p in range(passes)]
    print("rotating sweeps of the six leading steps per pass:", lead)
    assert lead[passes - 2] <= 0.8 * lead[0]  # left-to-right passes
    assert lead[passes - 1] <= 0.8 * lead[1]  # right-to-left passes


@pytest.mark.parametrize("precision,bar", [("fp32", 1e-8), ("bf16x3", 1e-8), ("bf16", None)])
def test_random_mpo_n20_chi64_mixed(ctx, c2_oracle, precision, bar):
    w, ref = c2_oracle
    got, err, info, _ = run_gpu(ctx, w, precision=precision)
    ne = rel_norm_err(info["norm"], ref.norm)
    fl = cross_fidelity_loss(got, ref.mps)
    print(f"{precision}: rel norm err {ne:.3e}  fidelity loss {fl:.3e}")
    if bar is None:
        assert ne < 1e-2 and fl < 1e-2   # reported, not held to the FP64 bar
    else:
        assert ne <= bar and fl <= bar


# ---------------------------------------------------------------- validation

def test_invalid_arguments_rejected(ctx):
    w = synth.workload_random_mpo(L=6, chi=4, D=2)
    v = ctx.mps_create(w.mps)
    U = ctx.mpo_create(w.mpo[:5] + [w.mpo[5]])
    U5 = ctx.mpo_create(synth.random_mpo(np.random.default_rng(0), 5, 2, 2))
    with pytest.raises(B.SmpsError) as e:
        ctx.mpo_apply(U5, v, B.strategy(4, 1e-10))
    assert e.value.code == B.EINVAL
    for bad in (B.strategy(0, 1e-10), B.strategy(4, -1.0), B.strategy(4, 1e-10, sweeps=0),
                B.strategy(4, 1e-10, precision=7)):
        with pytest.raises(B.SmpsError) as e:
            ctx.mpo_apply(U, v, bad)
        assert e.value.code == B.EINVAL
    U3 = ctx.mpo_create(synth.random_mpo(np.random.default_rng(1), 6, 3, 2))
    with pytest.raises(B.SmpsError) as e:
        ctx.mpo_apply(U3, v, B.strategy(4, 1e-10))
    assert e.value.code == B.EINVAL
    # a destroyed handle is rejected, not dereferenced
    v.destroy()
    with pytest.raises(B.SmpsError) as e:
        ctx.mpo_apply(U, v, B.strategy(4, 1e-10))
    assert e.value.code == B.EINVAL
    with pytest.raises(B.SmpsError):
        v.shape()


def test_nonfinite_input_reports_numeric_error(ctx):
    w = synth.workload_random_mpo(L=6, chi=4, D=2)
    w.mps[3] = w.mps[3].copy()
    w.mps[3][0, 0, 0] = np.nan
    v = ctx.mps_create(w.mps)
    U = ctx.mpo_create(w.mpo)
    with pytest.raises(B.SmpsError) as e:
        ctx.mpo_apply(U, v, B.strategy(4, 1e-10))
    assert e.value.code == B.ENUMERIC


def test_edge_steps_with_accumulated_rotations_match_oracle_step_by_step(ctx):
    """n=12 chi=32 D=4: the steps near both ends factorize the shorter side
    with accumulated rotations.  Every step's kept rank and discarded weight
    equal the oracle's, the result's sites are exact right isometries, and the
    per-step Jacobi sweep log accounts for every sweep reported."""
    w = synth.workload_random_mpo(rep=5, L=12, chi=32, D=4)
    ref = om.apply_simplify(w.mpo, w.mps, 32, 1e-10, sweeps=2)
    got, err, info, _ = run_gpu(ctx, w, sweeps=2, max_bond=32, tol=1e-10)
    deltas, ranks, _ = ctx.last_log()
    assert list(ranks) == list(ref.step_ranks)
    scale = ref.norm ** 2
    assert np.max(np.abs(np.asarray(deltas) - np.asarray(ref.deltas))) <= 1e-10 * scale
    assert rel_norm_err(info["norm"], ref.norm) <= 1e-12
    assert cross_fidelity_loss(got, ref.mps) <= 1e-12
    assert max(isometry_residual_right(t) for t in got[1:]) <= 1e-13
    sweeps = ctx.last_jacobi_log()
    assert len(sweeps) == info["steps"] and sum(sweeps) == info["jacobi_sweeps"]
    assert all(s >= 0 for s in sweeps)
