"""Benchmark: MPO x MPS apply + two-site variational compression on one MI355X.

Workload (one step): apply a random bond-8 MPO to a random 20-site d=2 MPS of
bond 64 (entries N(0, 1/chi)) and compress back to bond 64 with tolerance
1e-10 and 4 sweeps, i.e. 4 * 2 * 19 = 152 two-site updates ("site-updates").
The step is run in the plain FP64 path and in the mixed-precision paths
(FP32 / split-BF16x3 / BF16 contractions, FP64 factorizations and norms).
`value` is the site-updates/s of the fastest mixed path whose result matches
the FP64 CPU oracle to <= 1e-8 in both the relative norm and the
cross-fidelity loss; the FP64 GPU path is reported beside it.

Prints ONE JSON line (rank 0).  Inputs are resident on the device before the
timed region; timing uses HIP events on the stream the kernels run on.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "site-updates/s, MPO·MPS apply+simplify, mixed vs FP64 GPU at ≤1e-8 rel err"
HBM_PEAK_GBS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precisions", default="fp64,fp32,bf16x3,bf16")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle (no parity check, no baseline)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="CPU baseline: repeat the oracle until this much time has passed")
    ap.add_argument("--a11", action="store_true",
                    help="only measure the learned-rank randomized factorization (train the predictor on the "
                         "n=10 / n=20 / L=100 workloads' spectra, evaluate on the L=64 chi=512 decaying-spectrum "
                         "workload and on a tolerance-bound one) and print its JSON line")
    ap.add_argument("--dmrg", default="", metavar="L,L,...",
                    help="only measure the two-site DMRG ground-state search of the critical transverse-field "
                         "Ising chain (-sum ZZ - sum X) at these chain lengths and print its JSON line")
    ap.add_argument("--diffusion", default="", metavar="N,N,...",
                    help="only measure the RK4 integration of the diffusion equation (Gaussian initial state on "
                         "2^N grid points, 1000 steps) and print its JSON line")
    ap.add_argument("--rk4-steps", type=int, default=1000)
    ap.add_argument("--complex", action="store_true",
                    help="only measure the complex apply + compression (random complex MPO D=4 on a random complex "
                         "MPS n=20 chi=32, max bond 32, tol 1e-10, 4 sweeps) and print its JSON line")
    ap.add_argument("--c3-applies", type=int, default=3,
                    help="timed applies per precision of the L=100 chi=256 sub-record of the default run "
                         "(after one warm-up); 0 skips it")
    ap.add_argument("--c4-steps", type=int, default=3,
                    help="timed batched calls per precision of the 512-chain sub-record of the default run (0: skip)")
    ap.add_argument("--large", action="store_true",
                    help="only measure the L=100 chi=256 XXZ workload (4 sweeps, FP64 and mixed contractions, the "
                         "whole oracle as parity reference; several minutes) and print its JSON line")
    ap.add_argument("--large-sweeps", type=int, default=4,
                    help="sweeps of the --large workload (4 is the measured configuration; fewer for a profile)")
    ap.add_argument("--batched", action="store_true",
                    help="only measure the 512-chain QTT batch (batched by chi, graph-captured, FP64 and mixed; "
                         "against a per-chain loop) and print its JSON line")
    ap.add_argument("--no-loop", action="store_true",
                    help="--batched: skip the per-chain loop comparison (for profiling the batched call)")
    ap.add_argument("--replicas", type=int, default=0, metavar="N",
                    help="only measure N independent copies of the headline workload (n=20 chi=64 D=8, 4 sweeps) "
                         "in one batched, graph-captured call and print its JSON line")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run 4 device copies of MIB MiB (calibrates the HBM byte counters) and exit")
    return ap.parse_args()


def svd_flops(m: int, n: int) -> float:
    """Algorithmic flops of one factorization of an m x n two-site tensor
    that yields the singular values and one set of singular vectors:
    4 l k^2 + 8 k^3 with k = min(m, n), l = max(m, n) (the R-SVD count of
    Golub & Van Loan, Matrix Computations, 4th ed., Fig. 8.6.1)."""
    k, l = min(m, n), max(m, n)
    return 4.0 * l * k * k + 8.0 * k ** 3


def contraction_flops(c, cv, D, d: int, sweeps: int) -> float:
    """Flops of the contractions one apply performs (every bond at its cap c,
    v's bonds cv, MPO bonds D): per update one X tensor (the environment times
    v's site, then times the MPO site), the two-site product theta and the
    environment update; the X tensor of the other side is reused from the
    previous pass."""
    L = len(c) - 1
    f = 0.0
    for _ in range(sweeps):
        for k in range(L - 1):  # left to right: X_L[k], theta, L[k+1]
            f += 2.0 * c[k] * D[k] * cv[k] * d * cv[k + 1] + 2.0 * c[k] * cv[k + 1] * D[k] * d * d * D[k + 1]
            f += 2.0 * c[k] * d * D[k + 1] * cv[k + 1] * d * c[k + 2]
            f += 2.0 * c[k + 1] * c[k] * d * D[k + 1] * cv[k + 1]
        for k in range(L - 2, -1, -1):  # right to left: X_R[k+1], theta, R[k+1]
            f += 2.0 * c[k + 2] * D[k + 2] * cv[k + 2] * d * cv[k + 1]
            f += 2.0 * c[k + 2] * cv[k + 1] * D[k + 2] * d * d * D[k + 1]
            f += 2.0 * c[k] * d * D[k + 1] * cv[k + 1] * d * c[k + 2]
            f += 2.0 * c[k + 1] * d * c[k + 2] * D[k + 1] * cv[k + 1]
    return f


# dense MFMA peaks (TFLOP/s) of the arithmetic each contraction precision runs on,
# and how many MFMA products it issues per algorithmic product
MFMA_PEAK = {"fp64": (78.6, 1), "fp32": (157.3, 1), "bf16x3": (2500.0, 3), "bf16": (2500.0, 1)}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def time_oracle(fn, budget_s: float):
    """Time fn() on all BLAS threads and on one thread, each for about half of
    the budget (at least one call), and return (seconds per call, threads) of
    the faster setting plus both measurements.  Small contractions often run
    faster on one thread than on many."""
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        all_threads = max([tp.get("num_threads", 1) for tp in threadpool_info()] + [1])
    except Exception:
        threadpool_limits, all_threads = None, os.cpu_count()

    def run(limit):
        t0 = time.perf_counter()
        reps = 0
        while True:
            if limit is None or threadpool_limits is None:
                fn()
            else:
                with threadpool_limits(limits=limit):
                    fn()
            reps += 1
            if time.perf_counter() - t0 >= 0.5 * budget_s:
                break
        return (time.perf_counter() - t0) / reps, reps

    many, reps_many = run(None)
    one, reps_one = run(1)
    best = (one, 1, reps_one) if one < many else (many, int(all_threads), reps_many)
    return best, {"s_per_call_all_threads": many, "threads_all": int(all_threads), "s_per_call_1_thread": one}


def source_sha256(sources) -> str:
    """sha256 over the concatenated kernel sources (one path or a list)."""
    import hashlib
    h = hashlib.sha256()
    for src in ([sources] if isinstance(sources, str) else sources):
        h.update(open(src, "rb").read())
    return h.hexdigest()


def measured_traffic(path: str, sources):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current kernel source (None otherwise)."""
    try:
        kv = dict(l.split(": ", 1) for l in open(path).read().splitlines() if ": " in l and not l.startswith(" "))
        if kv.get("kernel_source_sha256", "").strip() != source_sha256(sources):
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def copy_probe(mib: int):
    import torch
    n = mib * (1 << 20) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(4):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": 4 * n, "copy_probe_bytes_written": 4 * n, "copies": 4}))


def learned_rank(args):
    """Train the rank predictor on the spectra of exact sweeps (small exact
    workloads and two seeds of the tolerance-bound family), then time apply +
    compression of the tolerance-bound workload (L=32, chi=512, decaying
    spectra tau ~ U[20, 40] under a product operator, 2 sweeps) with the exact
    factorization, the predictor-sized randomized one and the previous-rank-
    sized one (best of two timed calls after a sizing call)."""
    import numpy as np
    import torch

    import synth
    from paper_2601_16734_amd import binding as B
    from paper_2601_16734_amd import rank_training as RT

    torch.cuda.set_device(0)
    ctx = B.Context(0)
    t0 = time.perf_counter()
    probs = [(w.mpo, w.mps, w.max_bond, w.tol) for w in
             [synth.workload_laplacian_small(r) for r in range(4)] +
             [synth.workload_random_mpo(0, L=12, chi=32, D=4), synth.workload_xxz(0, L=16, chi=32)]]
    F0, Y0 = RT.collect_pairs(ctx, probs, sweeps=4)
    tr = [synth.workload_decaying_tol(r) for r in (1, 2)]
    F1, Y1 = RT.collect_pairs(ctx, [(w.mpo, w.mps, w.max_bond, w.tol) for w in tr], sweeps=2)
    F, Y = np.concatenate([F0, F1]), np.concatenate([Y0, Y1])
    t_collect = time.perf_counter() - t0
    t0 = time.perf_counter()
    loss = RT.train_predictor(ctx, F, Y, epochs=150)
    t_train = time.perf_counter() - t0
    print(f"predictor: {len(Y)} pairs collected in {t_collect:.1f} s, trained in {t_train:.2f} s, "
          f"loss {loss:.4f}", file=sys.stderr, flush=True)
    w = synth.workload_decaying_tol(0)
    U, v = ctx.mpo_create(w.mpo), ctx.mps_create(w.mps)
    res = {}
    for name, fact in [("exact", B.FACT_SVD), ("predictor", B.FACT_RSVD_MLP), ("previous_rank", B.FACT_RSVD_PREV),
                       ("fixed_sketch", B.FACT_RSVD_FIXED)]:
        st = B.strategy(w.max_bond, w.tol, sweeps=2, factorization=fact)
        o, _ = ctx.mpo_apply(U, v, st)
        o.destroy()
        times = []
        for _ in range(2):
            torch.cuda.synchronize()
            t = time.perf_counter()
            o, _ = ctx.mpo_apply(U, v, st)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t)
            info = ctx.last_info()
            o.destroy()
        dt = min(times)
        res[name] = {"seconds": dt, "site_updates_per_s": info["steps"] / dt, "norm": info["norm"],
                     "accepted": info["rsvd_accepted"], "fallbacks": info["rsvd_fallbacks"], "steps": info["steps"]}
        print(f"  {name}: {dt:.2f} s, accepted {info['rsvd_accepted']}, fallbacks {info['rsvd_fallbacks']}",
              file=sys.stderr, flush=True)
    for name in ("predictor", "previous_rank", "fixed_sketch"):
        res[name]["speedup_vs_exact"] = res["exact"]["seconds"] / res[name]["seconds"]
        res[name]["rel_norm_diff_vs_exact"] = abs(res[name]["norm"] - res["exact"]["norm"]) / res["exact"]["norm"]
    res["predictor"]["speedup_vs_previous_rank"] = res["previous_rank"]["seconds"] / res["predictor"]["seconds"]
    out = {"metric": "learned-rank randomized factorization vs exact, apply+compress",
           "config": {"workload": "L=32 d=2 chi=512 decaying spectra tau~U[20,40], product operator, tol 1e-10, "
                                  "2 sweeps (tolerance-bound ranks)"},
           "training": {"pairs": int(len(Y)), "loss": loss, "collect_s": t_collect, "train_s": t_train},
           "modes": res}
    print(json.dumps(out))
    ctx.close()


def dmrg_leg(args):
    """Ground-state search of -sum Z_i Z_{i+1} - sum X_i (open chain) from a
    random bond-4 guess, relative tolerance eps^2 / (n - 1) with eps = 1e-6 on
    the discarded weight, bond cap 256, Krylov dimension 24, sweeps until the
    energy changes by less than 1e-13 (relative) over a sweep.  The time of a
    whole search (inputs resident, one warm-up search first) is reported with
    its two-site updates per second."""
    import numpy as np
    import torch

    import synth
    from paper_2601_16734_amd import binding as B

    torch.cuda.set_device(0)
    ctx = B.Context(0)
    sizes = [int(x) for x in args.dmrg.split(",")]
    res = {}
    for L in sizes:
        H = ctx.mpo_create(synth.tfim_mpo(L, 1.0, 1.0))
        g = ctx.mps_create(synth.random_mps(np.random.default_rng(70), L, 2, 4))
        st = B.strategy(256, 1e-12 / (L - 1), sweeps=10, sweep_tol=1e-13)
        psi, E = ctx.dmrg(H, g, st)  # warm-up
        psi.destroy()
        times = []
        for _ in range(max(1, args.steps)):
            torch.cuda.synchronize()
            t = time.perf_counter()
            psi, E = ctx.dmrg(H, g, st)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t)
            bonds = psi.shape()[1]
            psi.destroy()
        info = ctx.last_info()
        dt = float(np.median(times))
        res[L] = {"seconds": dt, "energy": E, "sweeps": info["sweeps_done"], "site_updates": info["steps"],
                  "site_updates_per_s": info["steps"] / dt, "max_bond": max(bonds)}
        print(f"L={L}: {dt * 1e3:.1f} ms, {info['sweeps_done']} sweeps, {info['steps']} updates, "
              f"chi {max(bonds)}", file=sys.stderr, flush=True)
    out = {"metric": "DMRG two-site updates/s, critical Ising chain ground state", "unit": "site-updates/s",
           "dtype": "f64", "data": "synthetic", "steps": max(1, args.steps),
           "config": {"workload": "dmrg_tfim_critical", "J": 1.0, "h": 1.0, "eps": 1e-6, "bond_cap": 256,
                      "krylov_dim": 24, "sweep_tol": 1e-13},
           "per_L": {str(L): r for L, r in res.items()}}
    if not args.no_cpu:
        # CPU oracle (dense local eigensolver) and the closed-form energies
        from oracle import dmrg as od
        for L, r in res.items():
            ex = od.tfim_ground_energy(L, 1.0, 1.0)
            r["exact_energy"] = ex
            r["rel_energy_error"] = (r["energy"] - ex) / abs(ex)
        L = 16
        Hn, gn = synth.tfim_mpo(L, 1.0, 1.0), synth.random_mps(np.random.default_rng(70), L, 2, 4)
        n_up = 2 * 2 * (L - 1)
        (dt, cores, reps), both = time_oracle(
            lambda: od.dmrg(Hn, gn, max_bond=256, tol=1e-12 / (L - 1), sweeps=2), 8.0)
        out["cpu_baseline"] = {"value": n_up / dt, "unit": "site-updates/s", "cores": int(cores),
                               "kind": "oracle", "cpu_model": cpu_model(),
                               "sample": f"oracle DMRG, L={L}, 2 sweeps ({n_up} updates), {reps} runs on the "
                                         f"faster of all BLAS threads and one thread",
                               "value_all_threads": n_up / both["s_per_call_all_threads"],
                               "value_1_thread": n_up / both["s_per_call_1_thread"]}
    print(json.dumps(out))
    ctx.close()


def diffusion_leg(args):
    """du/dt = nu d^2u/dx^2 on [-0.5, 0.5) with 2^n points, nu = 0.01, open
    second-difference Laplacian, Gaussian initial condition (sigma = 0.1)
    loaded densely and compressed on the device, RK4 steps of
    dt = dx^2 / (20 nu), relative tolerance eps^2 / (n - 1) with eps = 1e-6 on
    the discarded weight, up to 4 sweeps per compression with early exit.
    Each RK4 step is one apply and four compressed linear combinations; the
    timed region covers all the steps with the state resident on the device."""
    import numpy as np
    import torch

    import synth
    from paper_2601_16734_amd import binding as B
    from paper_2601_16734_amd import evolution as EV

    torch.cuda.set_device(0)
    ctx = B.Context(0)
    nu, steps = 0.01, args.rk4_steps
    res, finals = {}, {}
    for n in [int(x) for x in args.diffusion.split(",")]:
        dx = 1.0 / 2 ** n
        dt = dx * dx / (20.0 * nu)
        lap = synth.laplacian_mpo(n, dx=dx)
        lap[0] = nu * lap[0]
        H = ctx.mpo_create(lap)
        st = B.strategy(2 ** (n // 2), 1e-12 / (n - 1), sweeps=4, sweep_tol=1e-14)
        exact = ctx.mps_create(synth.placement_mps(synth.gaussian_grid(n), n))
        y0, _ = ctx.simplify(exact, st)
        y = EV.rk4_step(ctx, H, y0, dt, st)  # warm-up
        y.destroy()
        torch.cuda.synchronize()
        t = time.perf_counter()
        y = y0
        for _ in range(steps):
            y1 = EV.rk4_step(ctx, H, y, dt, st)
            if y is not y0:
                y.destroy()
            y = y1
        torch.cuda.synchronize()
        sec = time.perf_counter() - t
        bonds = y.shape()[1]
        finals[n] = (y.read(), dt)
        y.destroy()
        res[n] = {"seconds": sec, "rk4_steps": steps, "rk4_steps_per_s": steps / sec,
                  "compressions_per_s": 5 * steps / sec, "max_bond": max(bonds), "dt": dt}
        print(f"n={n}: {steps} RK4 steps in {sec:.2f} s ({steps / sec:.1f} steps/s), final bond {max(bonds)}",
              file=sys.stderr, flush=True)
    out = {"metric": "RK4 steps/s, diffusion equation on a quantized grid (apply + combinations + compression)",
           "unit": "RK4 steps/s", "dtype": "f64", "data": "synthetic",
           "config": {"workload": "rk4_diffusion_gaussian", "nu": nu, "rk4_steps": steps, "eps": 1e-6,
                      "dt": "dx^2/(20 nu)"},
           "per_n": {str(n): r for n, r in res.items()}}
    if not args.no_cpu:
        # CPU oracle: dense RK4 of the same discrete system (accuracy) and the
        # MPS-level RK4 step (baseline timing on a bounded sample)
        from oracle import dense
        from oracle import evolution as oe
        for n, r in res.items():
            if n > 12:
                continue
            sites, dt = finals[n]
            lap = synth.laplacian_mpo(n, dx=1.0 / 2 ** n)
            want = oe.dense_rk4(nu * dense.mpo_to_dense(lap), synth.gaussian_grid(n), dt, steps)
            got = dense.mps_to_dense(sites)
            r["rel_error_vs_dense_rk4"] = float(np.linalg.norm(got - want) / np.linalg.norm(want))
        n = min(res)
        dx = 1.0 / 2 ** n
        lap = synth.laplacian_mpo(n, dx=dx)
        lap[0] = nu * lap[0]
        from oracle import mps as om
        y0 = om.simplify(synth.placement_mps(synth.gaussian_grid(n), n), 2 ** (n // 2), 1e-12 / (n - 1), 4).mps
        k = 5
        state = {"y": y0}

        def oracle_steps():
            for _ in range(k):
                state["y"] = oe.rk4_step(lap, state["y"], dx * dx / (20.0 * nu), 2 ** (n // 2), 1e-12 / (n - 1),
                                         sweeps=2)

        (sec, cores, reps), both = time_oracle(oracle_steps, 8.0)
        out["cpu_baseline"] = {"value": k / sec, "unit": "RK4 steps/s", "cores": int(cores), "kind": "oracle",
                               "cpu_model": cpu_model(),
                               "sample": f"oracle RK4 step (2 sweeps per compression), n={n}, {reps} x {k} steps "
                                         f"on the faster of all BLAS threads and one thread",
                               "value_all_threads": k / both["s_per_call_all_threads"],
                               "value_1_thread": k / both["s_per_call_1_thread"]}
    print(json.dumps(out))
    ctx.close()


def complex_leg(args):
    """Complex FP64 apply + compression: entries of both tensors with real and
    imaginary parts drawn like the real workloads'; inputs resident before
    timing; the oracle (complex route F) checks the timed output and is timed
    beside it on the faster of all BLAS threads and one thread."""
    import numpy as np
    import torch

    import synth
    from paper_2601_16734_amd import binding as B

    torch.cuda.set_device(0)
    ctx = B.Context(0)
    n, chi, D, sweeps = 20, 32, 4, 4
    rng = np.random.default_rng(120)
    v = [a + 1j * b for a, b in zip(synth.random_mps(rng, n, 2, chi), synth.random_mps(rng, n, 2, chi))]
    U = [a + 1j * b for a, b in zip(synth.random_mpo(rng, n, 2, D), synth.random_mpo(rng, n, 2, D))]
    zv, zU = ctx.zmps_create(v), ctx.zmpo_create(U)
    st = B.strategy(chi, 1e-10, sweeps=sweeps)
    out, _ = ctx.zmpo_apply(zU, zv, st)  # warm-up
    out.destroy()
    times = []
    for _ in range(max(1, args.steps)):
        torch.cuda.synchronize()
        t = time.perf_counter()
        out, _ = ctx.zmpo_apply(zU, zv, st)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t)
        last = out
    info = ctx.last_info()
    su = sweeps * 2 * (n - 1)
    sec = float(np.median(times))
    res = {"metric": "site-updates/s, complex MPO·MPS apply+simplify (FP64)", "unit": "site-updates/s",
           "value": su / sec, "dtype": "c128", "data": "synthetic", "steps": len(times),
           "ms_per_step": 1e3 * sec,
           "config": {"workload": f"random complex MPO D={D} on random complex MPS n={n} chi={chi}, max bond {chi}, "
                                  f"tol 1e-10, {sweeps} sweeps", "site_updates_per_step": su}}
    if not args.no_cpu:
        from oracle import dense  # noqa: F401
        from oracle import zmps as oz
        ref, nref, _ = oz.apply_simplify(U, v, chi, 1e-10, sweeps=sweeps)
        got = last.read()
        ov = abs(oz.scprod(got, ref))
        res["rel_norm_err"] = abs(info["norm"] - nref) / nref
        res["fidelity_loss"] = float(1 - ov / (info["norm"] * nref))
        (dt, cores, reps), both = time_oracle(lambda: oz.apply_simplify(U, v, chi, 1e-10, sweeps=sweeps),
                                              args.cpu_seconds)
        res["cpu_baseline"] = {"value": su / dt, "unit": "site-updates/s", "cores": int(cores), "kind": "oracle",
                               "cpu_model": cpu_model(),
                               "sample": f"{reps} complex oracle runs of the same workload on the faster of all BLAS "
                                         f"threads and one thread",
                               "value_all_threads": su / both["s_per_call_all_threads"],
                               "value_1_thread": su / both["s_per_call_1_thread"]}
    print(json.dumps(res))
    ctx.close()


def large_leg(args):
    """The L=100 d=2 chi=256 chain under the nearest-neighbour XXZ-type MPO
    (D=5, couplings uniform in [0.5, 1.5]): apply + compression at max bond
    256, tol 1e-10, 4 sweeps, in FP64 and in the mixed contraction precisions
    (FP64 factorizations throughout).  The two-site tensors are 512 x 512 in
    the bulk, too large for one workgroup's LDS, so this measures the blocked
    factorization path.  One apply per precision is timed, with
    no warm-up (the one-time graph captures of the first call are well under
    1% of an apply).  The whole oracle (same sweeps, all BLAS threads) is the
    parity reference for every precision and the CPU baseline."""
    import numpy as np
    import torch

    import synth
    from paper_2601_16734_amd import binding as B

    torch.cuda.set_device(0)
    ctx = B.Context(0)
    w = synth.workload_xxz()
    L, sweeps = len(w.mps), args.large_sweeps
    su = sweeps * 2 * (L - 1)
    v = ctx.mps_create_device([torch.from_numpy(t).to("cuda") for t in w.mps])
    U = ctx.mpo_create(w.mpo)
    torch.cuda.synchronize()
    caps = synth.bond_caps(L, 2, w.max_bond)
    fact_flops = sum(svd_flops(2 * caps[k], 2 * caps[k + 2]) for k in list(range(L - 1)) * (2 * sweeps))
    results, outs = {}, {}
    precs = [p for p in args.precisions.split(",") if p != "bf16"]  # bf16 misses the 1e-8 bar (headline)
    for prec in precs:
        st = B.strategy(w.max_bond, w.tol, sweeps=sweeps, precision=prec)
        torch.cuda.synchronize()
        ctx.set_profiling(True)
        t = time.perf_counter()
        out, _ = ctx.mpo_apply(U, v, st)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t
        fact_ms, fact_n = ctx.kernel_time(0)
        ctx.set_profiling(False)
        info = ctx.last_info()
        outs[prec] = out
        results[prec] = {"ms_per_step": 1e3 * sec, "site_updates_per_s": su / sec, "norm": info["norm"],
                         "factorization_ms_per_step": fact_ms, "factorizations_per_step": fact_n}
        print(f"large leg: {prec} {su / sec:.1f} site-updates/s", file=sys.stderr, flush=True)
    cpu = None
    if not args.no_cpu:
        from oracle import mps as om
        print(f"large leg: oracle, {sweeps} sweeps", file=sys.stderr, flush=True)
        t = time.perf_counter()
        ref = om.apply_simplify(w.mpo, w.mps, w.max_bond, w.tol, sweeps=sweeps)
        dt = time.perf_counter() - t
        try:
            from threadpoolctl import threadpool_info
            threads = max([tp.get("num_threads", 1) for tp in threadpool_info()] + [1])
        except Exception:
            threads = os.cpu_count()
        cpu = {"value": su / dt, "unit": "site-updates/s", "cores": int(threads), "kind": "oracle",
               "cpu_model": cpu_model(),
               "sample": f"one full oracle run of the same workload ({su} site-updates, {dt:.0f} s, FP64 "
                         f"NumPy/SciPy on all BLAS threads: the 512 x 512 SVDs gain from threads)"}
        rr = om.scprod(ref.mps, ref.mps)
        for prec, out in outs.items():
            got = out.read()
            r = results[prec]
            r["rel_norm_err"] = abs(r["norm"] - ref.norm) / ref.norm
            r["fidelity_loss"] = float(1 - abs(om.scprod(got, ref.mps)) / math.sqrt(om.scprod(got, got) * rr))
            r["parity_1e-8"] = bool(r["rel_norm_err"] <= 1e-8 and r["fidelity_loss"] <= 1e-8)
    for out in outs.values():
        out.destroy()
    fp64 = results.get("fp64")
    ok = {p: r for p, r in results.items() if r.get("parity_1e-8", cpu is None)}
    best_p = max(ok, key=lambda p: ok[p]["site_updates_per_s"]) if ok else "fp64"
    best = results[best_p]
    avg_ms = best["factorization_ms_per_step"] / max(1, best["factorizations_per_step"])
    achieved = fact_flops / max(1, best["factorizations_per_step"]) / (avg_ms * 1e-3) / 1e12
    line = {"metric": "site-updates/s, MPO·MPS apply+simplify, mixed vs FP64 GPU at <=1e-8 rel err",
            "value": best["site_updates_per_s"], "unit": "site-updates/s", "n_gpus": 1, "steps": 1,
            "warmup": 0, "ms_per_step": best["ms_per_step"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None,
            "dtype": {"fp64": "f64", "fp32": "f32+f64", "bf16x3": "bf16x3+f64"}[best_p], "data": "synthetic",
            "config": {"workload": "XXZ-type MPO D=5 (couplings U[0.5,1.5]) on random MPS L=100 d=2 chi=256, "
                                   f"max bond 256, tol 1e-10, {sweeps} sweeps", "site_updates_per_step": su,
                       "precision": best_p},
            "fp64_site_updates_per_s": fp64["site_updates_per_s"] if fp64 else None,
            "speedup_vs_fp64": best["site_updates_per_s"] / fp64["site_updates_per_s"] if fp64 else None,
            "per_precision": results,
            "roofline": {"kernel": "one-sided Jacobi SVD of the 512 x 512 two-site tensors (blocked: block pairs "
                                   "in LDS, one launch per round of the tournament over blocks)",
                         "bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": achieved / FP64_VECTOR_PEAK_TFLOPS, "traffic": None,
                         "avg_factorization_ms": avg_ms,
                         "share_of_step": best["factorization_ms_per_step"] / best["ms_per_step"]},
            "cpu_baseline": cpu}
    print(json.dumps(line))
    ctx.close()


def batched_leg(args):
    """The 512-chain QTT batch (n uniform in [8, 30], chi uniform in
    {4, 8, ..., 128}, FP32 N(0, 1/chi) entries, bond-3 Laplacian or bond-2
    shift): every chain compressed at its own chi (tol 1e-10, 4 sweeps) in
    one batched call -- one graph for all 512 chains, per-chain bond caps,
    the blocked factorizations run by persistent teams from a longest-first
    queue.  The capture call is untimed; the timed calls replay the graph.
    Compared with a loop of single-chain calls over all 512 chains (FP64).
    The oracle checks a sample (the first 16 chains) and is timed on the
    first chains in order, within the CPU budget, on one thread."""
    import numpy as np
    import torch

    import synth
    from paper_2601_16734_amd import binding as B

    torch.cuda.set_device(0)
    ctx = B.Context(0)
    ws = synth.workload_batch(count=512)
    sweeps = 4
    vs = [ctx.mps_create(w.mps, dtype=np.float32) for w in ws]
    Us = [ctx.mpo_create(w.mpo) for w in ws]
    caps = [w.max_bond for w in ws]
    steps_of = [sweeps * 2 * (w.meta["n"] - 1) for w in ws]
    su = sum(steps_of)
    precs = [p for p in args.precisions.split(",") if p != "bf16"]
    results, outs = {}, {}
    plan = ctx.plan_apply_batched(Us, vs, B.strategy(max(caps), 1e-10, sweeps=sweeps), max_bonds=caps)
    for prec in precs:
        st = B.strategy(max(caps), 1e-10, sweeps=sweeps, precision=prec)
        t = time.perf_counter()
        first, _ = ctx.mpo_apply_batched(Us, vs, st, max_bonds=caps)  # capture + first replay
        torch.cuda.synchronize()
        capture_sec = time.perf_counter() - t
        for o in first:
            o.destroy()
        times = []
        for _ in range(max(1, args.steps)):
            t = time.perf_counter()
            got, _ = ctx.mpo_apply_batched(Us, vs, st, max_bonds=caps)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t)
            for i in range(len(ws)):
                if outs.setdefault(prec, [None] * len(ws))[i] is not None:
                    outs[prec][i].destroy()
                outs[prec][i] = got[i]
        sec = float(np.median(times))
        results[prec] = {"ms_per_step": 1e3 * sec, "site_updates_per_s": su / sec,
                         "first_call_with_capture_ms": 1e3 * capture_sec}
        print(f"batched leg: {prec} {su / sec:.0f} site-updates/s", file=sys.stderr, flush=True)
    # per-chain loop (single-problem calls) over all 512 chains, FP64
    loop_sec = loop_rate = float("nan")
    for i in range(0 if args.no_loop else 4):  # warm-up
        o, _ = ctx.mpo_apply(Us[i], vs[i], B.strategy(caps[i], 1e-10, sweeps=sweeps))
        o.destroy()
    if not args.no_loop:
        torch.cuda.synchronize()
        t = time.perf_counter()
        for i in range(len(ws)):
            o, _ = ctx.mpo_apply(Us[i], vs[i], B.strategy(caps[i], 1e-10, sweeps=sweeps))
            o.destroy()
        torch.cuda.synchronize()
        loop_sec = time.perf_counter() - t
        loop_rate = su / loop_sec
    cpu = None
    if not args.no_cpu:
        from oracle import mps as om
        refs = {i: om.apply_simplify(ws[i].mpo, [t.astype(np.float64) for t in ws[i].mps], ws[i].max_bond,
                                     1e-10, sweeps=sweeps) for i in range(16)}
        for prec in precs:
            worst_n, worst_f = 0.0, 0.0
            for i, ref in refs.items():
                got = outs[prec][i].read()
                ne = abs(ctx.norm(outs[prec][i]) - ref.norm) / ref.norm
                fl = float(1 - abs(om.scprod(got, ref.mps)) /
                           math.sqrt(om.scprod(got, got) * om.scprod(ref.mps, ref.mps)))
                worst_n, worst_f = max(worst_n, ne), max(worst_f, fl)
            r = results[prec]
            r["sample_rel_norm_err_max"], r["sample_fidelity_loss_max"] = worst_n, worst_f
            r["parity_1e-8"] = bool(worst_n <= 1e-8 and worst_f <= 1e-8)
        try:
            from threadpoolctl import threadpool_limits
        except Exception:
            threadpool_limits = None
        done_su, t0 = 0, time.perf_counter()
        count = 0
        for i, w in enumerate(ws):
            mps64 = [t.astype(np.float64) for t in w.mps]
            if threadpool_limits is not None:
                with threadpool_limits(limits=1):
                    om.apply_simplify(w.mpo, mps64, w.max_bond, 1e-10, sweeps=sweeps)
            else:
                om.apply_simplify(w.mpo, mps64, w.max_bond, 1e-10, sweeps=sweeps)
            done_su += steps_of[i]
            count += 1
            if time.perf_counter() - t0 >= args.cpu_seconds:
                break
        dt = time.perf_counter() - t0
        cpu = {"value": done_su / dt, "unit": "site-updates/s", "cores": 1 if threadpool_limits else os.cpu_count(),
               "kind": "oracle", "cpu_model": cpu_model(),
               "sample": f"the first {count} chains of the batch in order ({done_su} site-updates, {dt:.1f} s), "
                         f"FP64 NumPy/SciPy on one thread"}
    for lst in outs.values():
        for o in lst:
            if o is not None:
                o.destroy()
    fp64 = results.get("fp64")
    ok = {p: r for p, r in results.items() if r.get("parity_1e-8", cpu is None)}
    best_p = max(ok, key=lambda p: ok[p]["site_updates_per_s"]) if ok else "fp64"
    best = results[best_p]
    line = {"metric": "site-updates/s, MPO·MPS apply+simplify, mixed vs FP64 GPU at <=1e-8 rel err",
            "value": best["site_updates_per_s"], "unit": "site-updates/s", "n_gpus": 1, "steps": max(1, args.steps),
            "warmup": 1, "ms_per_step": best["ms_per_step"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None,
            "dtype": {"fp64": "f64", "fp32": "f32+f64", "bf16x3": "bf16x3+f64"}[best_p], "data": "synthetic",
            "config": {"workload": "512 QTT chains, n uniform in [8,30], d=2, chi uniform in {4,...,128}, FP32 "
                                   "entries, bond-3 Laplacian or bond-2 shift MPO, max bond chi, tol 1e-10, 4 sweeps; "
                                   "one batched call (per-chain caps), one graph", "site_updates_per_step": su,
                       "precision": best_p, "graph_kernels": plan["graph_kernels"],
                       "batched_launches": plan["launches"]},
            "fp64_site_updates_per_s": fp64["site_updates_per_s"] if fp64 else None,
            "speedup_vs_fp64": best["site_updates_per_s"] / fp64["site_updates_per_s"] if fp64 else None,
            "per_precision": results,
            "per_chain_loop_all512_fp64": None if args.no_loop else
            {"site_updates_per_s": loop_rate, "seconds": loop_sec,
             "batched_fp64_over_loop": (fp64["site_updates_per_s"] / loop_rate) if fp64 else None},
            "cpu_baseline": cpu}
    print(json.dumps(line))
    ctx.close()


def replicas_leg(args):
    """N independent copies of the headline workload (random MPO D=8 on a
    random MPS n=20 chi=64, max bond 64, tol 1e-10, 4 sweeps) as one batched,
    graph-captured call: one chain keeps one CU busy in its factorizations,
    N chains fill the chip.  The capture call is untimed; the timed calls
    replay the graph.  Every replica's norm is checked against one oracle run;
    the oracle is timed on one thread per chain."""
    import numpy as np
    import torch

    import synth
    from paper_2601_16734_amd import binding as B

    torch.cuda.set_device(0)
    ctx = B.Context(0)
    w = synth.workload_random_mpo()
    n = args.replicas
    su_one = w.sweeps * 2 * (len(w.mps) - 1)
    su = n * su_one
    U = ctx.mpo_create(w.mpo)
    vs = [ctx.mps_create(w.mps) for _ in range(n)]
    ref = None
    if not args.no_cpu:
        from oracle import mps as om
        ref = om.apply_simplify(w.mpo, w.mps, w.max_bond, w.tol, sweeps=w.sweeps)
    results = {}
    for prec in [p for p in args.precisions.split(",") if p != "bf16"]:
        st = B.strategy(w.max_bond, w.tol, sweeps=w.sweeps, precision=prec)
        first, _ = ctx.mpo_apply_batched([U] * n, vs, st)  # capture
        for o in first:
            o.destroy()
        torch.cuda.synchronize()
        times, got = [], None
        for _ in range(max(1, args.steps)):
            if got is not None:
                for o in got:
                    o.destroy()
            t = time.perf_counter()
            got, _ = ctx.mpo_apply_batched([U] * n, vs, st)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t)
        sec = float(np.median(times))
        rec = {"ms_per_step": 1e3 * sec, "site_updates_per_s": su / sec}
        if ref is not None:
            worst = max(abs(ctx.norm(o) - ref.norm) / ref.norm for o in got)
            rec["max_rel_norm_err"] = worst
            rec["parity_1e-8"] = bool(worst <= 1e-8)
        for o in got:
            o.destroy()
        results[prec] = rec
        print(f"replicas leg: {prec} x{n} {su / sec:.0f} site-updates/s", file=sys.stderr, flush=True)
    cpu = None
    if ref is not None:
        (dt, cores, reps), both = time_oracle(
            lambda: om.apply_simplify(w.mpo, w.mps, w.max_bond, w.tol, sweeps=w.sweeps), args.cpu_seconds)
        cpu = {"value": su_one / both["s_per_call_1_thread"], "unit": "site-updates/s", "cores": 1, "kind": "oracle",
               "cpu_model": cpu_model(),
               "sample": f"full apply+compress runs of one chain ({su_one} site-updates each, "
                         f"{both['s_per_call_1_thread']:.2f} s per run on one thread), FP64 NumPy/SciPy; the "
                         f"rate of one core, which independent chains would multiply by the cores given"}
    fp64 = results.get("fp64")
    ok = {p: r for p, r in results.items() if r.get("parity_1e-8", ref is None)}
    best_p = max(ok, key=lambda p: ok[p]["site_updates_per_s"]) if ok else "fp64"
    best = results[best_p]
    line = {"metric": "site-updates/s, MPO·MPS apply+simplify, mixed vs FP64 GPU at <=1e-8 rel err",
            "value": best["site_updates_per_s"], "unit": "site-updates/s", "n_gpus": 1, "steps": max(1, args.steps),
            "warmup": 1, "ms_per_step": best["ms_per_step"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None,
            "dtype": {"fp64": "f64", "fp32": "f32+f64", "bf16x3": "bf16x3+f64"}[best_p], "data": "synthetic",
            "config": {"workload": f"{n} independent copies of: random MPO D=8 on random MPS n=20 d=2 chi=64, "
                                   "max bond 64, tol 1e-10, 4 sweeps; one batched, graph-captured call",
                       "site_updates_per_step": su, "precision": best_p},
            "fp64_site_updates_per_s": fp64["site_updates_per_s"] if fp64 else None,
            "per_precision": results, "cpu_baseline": cpu}
    print(json.dumps(line))
    for v in vs:
        v.destroy()
    ctx.close()


def c3_subrecord(ctx, args, stream):
    """The L=100 d=2 chi=256 chain under the XXZ-type MPO D=5 (couplings
    U[0.5,1.5]), max bond 256, tol 1e-10, 4 sweeps: one warm-up and
    args.c3_applies timed applies per precision (inputs resident in HBM, no
    profiling inside the timed region), each timed result checked against the
    oracle's whole run stored in tests/golden (written by the oracle alone):
    kept ranks of all 792 steps, the final norm (1e-8 bar) and three probe
    overlaps."""
    import numpy as np
    import torch

    import synth
    from paper_2601_16734_amd import binding as B

    with open(os.path.join(ROOT, "tests", "golden", "xxz_L100_chi256_s4.json")) as fh:
        g = json.load(fh)
    w = synth.workload_xxz(0)
    L, sweeps = len(w.mps), g["sweeps"]
    su = sweeps * 2 * (L - 1)
    # the probe states of the stored run (seed stream 90), overlaps taken on the device
    probes = [ctx.mps_create(synth.random_mps(synth.rng_for(90, i), L, 2, 8)) for i in range(3)]
    v = ctx.mps_create_device([torch.from_numpy(t).to("cuda") for t in w.mps])
    U = ctx.mpo_create(w.mpo)
    torch.cuda.synchronize()
    res = {}
    for prec in ("fp64", "fp32", "bf16x3"):
        st = B.strategy(w.max_bond, w.tol, sweeps=sweeps, precision=prec)
        o, _ = ctx.mpo_apply(U, v, st)  # warm-up (graph captures of the blocked split)
        o.destroy()
        torch.cuda.synchronize()
        times, checks = [], []
        for _ in range(max(1, args.c3_applies)):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            out, err = ctx.mpo_apply(U, v, st)
            b.record(stream)
            torch.cuda.synchronize()
            times.append(a.elapsed_time(b))
            _, ranks, _ = ctx.last_log()
            nrm = ctx.last_info()["norm"]
            pr = max(abs(ctx.scprod(p, out) - r) / abs(r) for p, r in zip(probes, g["probe_overlaps"]))
            checks.append((abs(nrm - g["norm"]) / g["norm"], list(ranks) == g["step_ranks"], pr))
            out.destroy()
        ms = float(np.median(times))
        rel = max(c[0] for c in checks)
        res[prec] = {"ms_per_apply_median": ms, "ms_per_apply_all": times, "site_updates_per_s": su / (ms * 1e-3),
                     "rel_norm_err_vs_oracle": rel, "step_ranks_equal_oracle": all(c[1] for c in checks),
                     "probe_overlap_rel_err": max(c[2] for c in checks),
                     "parity_1e-8": bool(rel <= 1e-8 and all(c[1] for c in checks))}
        print(f"c3 sub-record: {prec} {su / (ms * 1e-3):.1f} site-updates/s, norm err {rel:.1e}", file=sys.stderr,
              flush=True)
    for h in probes + [v, U]:
        h.destroy()
    fp64 = res["fp64"]["site_updates_per_s"]
    ok = [p for p in ("fp32", "bf16x3") if res[p]["parity_1e-8"]]
    best = max(ok, key=lambda p: res[p]["site_updates_per_s"]) if ok else None
    return {"workload": "XXZ-type MPO D=5 (couplings U[0.5,1.5]) on random MPS L=100 d=2 chi=256, max bond 256, "
                        f"tol 1e-10, {sweeps} sweeps", "site_updates_per_apply": su, "warmup": 1,
            "applies": max(1, args.c3_applies), "parity_reference": "oracle whole run, tests/golden",
            "per_precision": res, "best_mixed": best,
            "speedup_vs_fp64": (res[best]["site_updates_per_s"] / fp64) if best else None,
            "oracle_cpu_seconds": g.get("oracle_seconds")}


def c4_subrecord(ctx, args, stream):
    """The 512-chain QTT batch (n uniform in [8, 30], chi uniform in {4, ...,
    128}, FP32 N(0, 1/chi) entries promoted to FP64, bond-3 Laplacian or bond-2
    shift), every chain at its own cap, tol 1e-10, 4 sweeps, as one batched
    call (one graph): per precision one capturing call and args.c4_steps timed
    replays (HIP events on the stream, inputs resident), every chain of the
    last result checked against the oracle's whole runs stored in tests/golden
    (written by the oracle alone): final norm (1e-8 bar) and bonds."""
    import numpy as np
    import torch

    import synth
    from paper_2601_16734_amd import binding as B

    with open(os.path.join(ROOT, "tests", "golden", "batch512_s4.json")) as fh:
        g = json.load(fh)
    ws = synth.workload_batch(0)
    sweeps = g["sweeps"]
    su = sum(sweeps * 2 * (w.meta["n"] - 1) for w in ws)
    vs = [ctx.mps_create(w.mps, dtype=np.float32) for w in ws]
    Us = [ctx.mpo_create(w.mpo) for w in ws]
    caps = [w.max_bond for w in ws]
    res = {}
    for prec in ("fp64", "fp32", "bf16x3"):
        st = B.strategy(max(caps), 1e-10, sweeps=sweeps, precision=prec)
        outs, _ = ctx.mpo_apply_batched(Us, vs, st, max_bonds=caps)  # capture + replay
        for o in outs:
            o.destroy()
        torch.cuda.synchronize()
        times = []
        for _ in range(max(1, args.c4_steps)):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            outs, _ = ctx.mpo_apply_batched(Us, vs, st, max_bonds=caps)
            b.record(stream)
            torch.cuda.synchronize()
            times.append(a.elapsed_time(b))
            last = outs
            if len(times) < max(1, args.c4_steps):
                for o in outs:
                    o.destroy()
        errs, bonds_ok = [], 0
        for o, ref in zip(last, g["chains"]):
            errs.append(abs(ctx.norm(o) - ref["norm"]) / ref["norm"])
            bonds_ok += list(o.shape()[1]) == ref["ranks"]
            o.destroy()
        errs = np.array(errs)
        ms = float(np.median(times))
        res[prec] = {"ms_per_call_median": ms, "ms_per_call_all": times, "site_updates_per_s": su / (ms * 1e-3),
                     "rel_norm_err_max": float(errs.max()), "chains_within_1e-8": int(np.sum(errs <= 1e-8)),
                     "chains_bonds_equal": int(bonds_ok),
                     "parity_1e-8": bool(errs.max() <= 1e-8 and bonds_ok == len(ws))}
        print(f"c4 sub-record: {prec} {su / (ms * 1e-3):.0f} site-updates/s, worst norm err {errs.max():.1e}",
              file=sys.stderr, flush=True)
    for h in vs + Us:
        h.destroy()
    fp64 = res["fp64"]["site_updates_per_s"]
    ok = [p for p in ("fp32", "bf16x3") if res[p]["parity_1e-8"]]
    best = max(ok, key=lambda p: res[p]["site_updates_per_s"]) if ok else None
    return {"workload": "512 QTT chains, n uniform in [8,30], d=2, chi uniform in {4,...,128}, FP32 entries, bond-3 "
                        "Laplacian or bond-2 shift MPO, max bond chi, tol 1e-10, 4 sweeps; one batched call, one graph",
            "site_updates_per_call": su, "warmup": 1, "calls": max(1, args.c4_steps),
            "parity_reference": "oracle whole run of every chain, tests/golden", "per_precision": res,
            "best_mixed_at_parity": best,
            "speedup_vs_fp64": (res[best]["site_updates_per_s"] / fp64) if best else None}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU (the method's sweep is sequential along the chain and no multi-GPU "
              "path is built); run it with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.a11:
        learned_rank(args)
        return
    if args.dmrg:
        dmrg_leg(args)
        return
    if args.diffusion:
        diffusion_leg(args)
        return
    if args.complex:
        complex_leg(args)
        return
    if args.large:
        large_leg(args)
        return
    if args.batched:
        batched_leg(args)
        return
    if args.replicas:
        replicas_leg(args)
        return

    import numpy as np
    import torch

    import synth
    from paper_2601_16734_amd import binding as B

    torch.cuda.set_device(0)
    ctx = B.Context(0)
    w = synth.workload_random_mpo()
    L = len(w.mps)
    site_updates = w.sweeps * 2 * (L - 1)

    # inputs resident in HBM before any timing
    dev_tensors = [torch.from_numpy(t).to("cuda") for t in w.mps]
    v = ctx.mps_create_device(dev_tensors)
    U = ctx.mpo_create(w.mpo)
    torch.cuda.synchronize()

    # ---- CPU oracle: parity reference and the reported CPU baseline
    cpu = None
    ref = None
    if not args.no_cpu:
        from oracle import mps as om
        ref = om.apply_simplify(w.mpo, w.mps, w.max_bond, w.tol, sweeps=w.sweeps)
        (dt, cores, reps), both = time_oracle(
            lambda: om.apply_simplify(w.mpo, w.mps, w.max_bond, w.tol, sweeps=w.sweeps), args.cpu_seconds)
        cpu = {"value": site_updates / dt, "unit": "site-updates/s", "cores": int(cores), "kind": "oracle",
               "sample": f"{reps} full apply+compress runs of the same workload ({site_updates} site-updates "
                         f"each, {dt:.2f} s per run, FP64 NumPy/SciPy) on the faster of all BLAS threads and "
                         f"one thread", "cpu_model": cpu_model(),
               "value_all_threads": site_updates / both["s_per_call_all_threads"],
               "threads_all": both["threads_all"], "value_1_thread": site_updates / both["s_per_call_1_thread"]}

    # theta shapes along the sweep (bond dims reach the cap for this workload)
    caps = synth.bond_caps(L, 2, w.max_bond)
    flops_per_apply = 0.0
    for _ in range(w.sweeps):
        for k in list(range(L - 1)) + list(range(L - 2, -1, -1)):
            flops_per_apply += svd_flops(2 * caps[k], 2 * caps[k + 2])

    cflops = contraction_flops(caps, [1] + [t.shape[2] for t in w.mps], [1] + [t.shape[3] for t in w.mpo], 2,
                               w.sweeps)
    results = {}
    stream = torch.cuda.current_stream()
    tuned = {}
    for prec in args.precisions.split(","):
        st = B.strategy(w.max_bond, w.tol, sweeps=w.sweeps, precision=prec)
        # GEMM tile autotuning for this workload's product shapes (setup, untimed)
        tuned[prec] = ctx.autotune_apply(U, v, st, reps=5)
        for _ in range(args.warmup):
            out, _ = ctx.mpo_apply(U, v, st)
            out.destroy()
        torch.cuda.synchronize()
        # timed region: no per-launch profiling events
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        marks = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
        outs = []
        start.record(stream)
        for i in range(args.steps):
            out, _ = ctx.mpo_apply(U, v, st)
            outs.append(out)
            marks[i].record(stream)
        stop.record(stream)
        torch.cuda.synchronize()
        ms = start.elapsed_time(stop) / args.steps
        per = np.array([start.elapsed_time(marks[0])] +
                       [marks[i - 1].elapsed_time(marks[i]) for i in range(1, args.steps)])
        info = ctx.last_info()
        # separate pass (one apply) for the factorization split: HIP events on
        # the context stream around every split launch (category 0) and around
        # the bulk 128 x 128 splits (category 2)
        ctx.set_profiling(True)
        prof_out, _ = ctx.mpo_apply(U, v, st)
        fact_ms, fact_n = ctx.kernel_time(0)
        bulk_ms, bulk_n = ctx.kernel_time(2)
        cat = {c: ctx.kernel_time(c)[0] for c in (1, 3, 4, 5, 6)}
        ctx.set_profiling(False)
        phases = {"factorization": fact_ms, "x_tensors": cat[3], "theta_products": cat[4],
                  "environment_updates": cat[5], "other_contractions": cat[1] - cat[3] - cat[4] - cat[5],
                  "other_launches": cat[6]}
        prof_out.destroy()
        contr_ms = max(1e-9, ms - fact_ms)
        peak, issue = MFMA_PEAK.get(prec, (78.6, 1))
        rec = {"ms_per_step": ms, "site_updates_per_s": site_updates / (ms / 1e3),
               "step_ms_median": float(np.median(per)),
               "step_ms_iqr": float(np.percentile(per, 75) - np.percentile(per, 25)),
               "factorization_ms_per_step": fact_ms,
               "factorization_launches_per_step": fact_n,
               "bulk_split_ms_avg": bulk_ms / max(1, bulk_n), "bulk_splits_per_step": bulk_n,
               "phase_kernel_ms_per_step": phases,
               "norm": info["norm"],
               "contraction_tflops": cflops / (contr_ms * 1e-3) / 1e12,
               "contraction_mfma_frac": issue * cflops / (contr_ms * 1e-3) / 1e12 / peak}
        if ref is not None:
            from oracle import mps as om
            got = outs[-1].read()
            rec["rel_norm_err"] = abs(info["norm"] - ref.norm) / ref.norm
            rec["fidelity_loss"] = float(1 - abs(om.scprod(got, ref.mps)) /
                                         math.sqrt(om.scprod(got, got) * om.scprod(ref.mps, ref.mps)))
            rec["parity_1e-8"] = bool(rec["rel_norm_err"] <= 1e-8 and rec["fidelity_loss"] <= 1e-8)
        for o in outs:
            o.destroy()
        results[prec] = rec

    fp64 = results.get("fp64")
    mixed = {p: r for p, r in results.items() if p != "fp64" and r.get("parity_1e-8", ref is None)}
    best_p = max(mixed, key=lambda p: mixed[p]["site_updates_per_s"]) if mixed else "fp64"
    best = results[best_p]

    # roofline of the dominant kernel: the FP64 one-sided Jacobi split of the
    # bulk 128 x 128 two-site tensor (jacobi_lds_kernel<8, false>), charged the
    # full-SVD count 20 (d chi)^3 per launch, over its average launch time
    # (HIP events on the context stream in the profiled pass)
    f = results[best_p]
    n_bulk = 2 * w.max_bond
    bulk_flops = 20.0 * n_bulk ** 3
    achieved = bulk_flops / (f["bulk_split_ms_avg"] * 1e-3) / 1e12
    roofline = {"kernel": "jacobi_lds_kernel<8, false> (FP64 one-sided Jacobi SVD of the 128 x 128 bulk two-site "
                          "tensor, one workgroup per split)",
                "bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
                "traffic": measured_traffic(os.path.join(ROOT, "profiles", "jacobi_lds_bulk_n20_chi64_traffic.txt"),
                                            [os.path.join(ROOT, "paper_2601_16734_amd", "csrc", x)
                                             for x in ("jacobi.hip", "select.h", "rules.h")]),
                "flops_per_launch": bulk_flops, "avg_launch_ms": f["bulk_split_ms_avg"],
                "launches_per_step": f["bulk_splits_per_step"],
                "share_of_step": f["factorization_ms_per_step"] / f["ms_per_step"],
                # context: a split is one workgroup, so it can use one of the 256 CUs
                "one_cu_peak": FP64_VECTOR_PEAK_TFLOPS / 256, "one_cu_frac": achieved / (FP64_VECTOR_PEAK_TFLOPS / 256)}

    line = {
        "metric": METRIC,
        "value": best["site_updates_per_s"],
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": best["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32+f64", "bf16x3": "bf16x3+f64", "bf16": "bf16+f64"}[best_p],
        "data": "synthetic",
        "config": {"workload": "random MPO D=8 on random MPS n=20 d=2 chi=64, max bond 64, tol 1e-10, 4 sweeps",
                   "site_updates_per_step": site_updates, "precision": best_p,
                   "gemm_shapes_autotuned": tuned.get(best_p)},
        "fp64_site_updates_per_s": fp64["site_updates_per_s"] if fp64 else None,
        "speedup_vs_fp64": (best["site_updates_per_s"] / fp64["site_updates_per_s"]) if fp64 else None,
        "per_precision": results,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    if args.c3_applies > 0:
        line["c3_xxz_L100_chi256"] = c3_subrecord(ctx, args, stream)
    if args.c4_steps > 0:
        line["c4_qtt512_batched"] = c4_subrecord(ctx, args, stream)
    print(json.dumps(line))
    ctx.close()


if __name__ == "__main__":
    main()
