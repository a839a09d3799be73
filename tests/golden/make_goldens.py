"""Write the whole-run reference values of the full-size workloads.

Every number stored here comes from the FP64 oracle (`oracle/`) run on the
seeded inputs of `synth` -- nothing is taken from the GPU library.  The GPU
parity tests compare their whole runs against these files because the oracle
takes minutes per workload, too long to repeat inside a test.

Workloads (inputs drawn by `synth`, same seeds as the tests and the bench):
  * xxz      -- L=100, d=2, chi=256 random MPS, XXZ-type MPO D=5 with couplings
                U[0.5,1.5] per bond; max bond 256, tol 1e-10, 4 sweeps.
  * decaying -- L=64, d=2, chi=512 MPS with bond spectra ~exp(-j/tau),
                tau ~ U[10,100]; random MPO D=8; max bond 512, tol 1e-10,
                4 sweeps.
  * decaying_tol -- the same construction at L=32, chi=512 with tau ~ U[20,40]
                under a product operator (bond 1), so that the tolerance (not
                the cap) binds the kept ranks; 2 sweeps.
  * batch    -- the 512 QTT chains (n ~ U{8..30}, chi ~ U{4,...,128}, float32
                inputs promoted to FP64, Laplacian or shift MPO); max bond =
                own chi, tol 1e-10, 4 sweeps.

For a single chain the file holds, per two-site step of the sweep (Sec. 2.5):
the kept rank, the discarded weight, the kept weight ||psi||^2 and the largest
singular value of the two-site tensor; and for the result: the centre norm
(Sec. 2.4.4), the final bond dimensions, the accumulated error bound (Sec. 2.3)
and the scalar products with three seeded probe MPS of bond 8 (gauge-invariant
fingerprints of the final state).  For the batch: per chain the final norm,
bonds, error bound, total discarded weight and the kept rank of every step.

Usage:  python tests/golden/make_goldens.py [xxz] [decaying] [decaying_tol] [batch]
"""

from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import mps as om  # noqa: E402

PROBE_CONFIG = 90  # seed stream of the probe states


def probes(L: int, count: int = 3, chi: int = 8):
    return [synth.random_mps(synth.rng_for(PROBE_CONFIG, i), L, 2, chi) for i in range(count)]


def single_chain_record(w, sweeps: int) -> dict:
    t = time.perf_counter()
    ref = om.apply_simplify(w.mpo, w.mps, w.max_bond, w.tol, sweeps=sweeps)
    dt = time.perf_counter() - t
    L = len(w.mps)
    return {
        "workload": w.name, "L": L, "max_bond": w.max_bond, "tol": w.tol, "sweeps": sweeps,
        "norm": ref.norm, "ranks": [int(x) for x in ref.ranks], "error_bound": ref.error_bound,
        "discarded": ref.total_discarded,
        "step_ranks": [int(x) for x in ref.step_ranks],
        "step_deltas": [float(x) for x in ref.deltas],
        "step_norms2": [float(x) for x in ref.norms2],
        "step_sigma0": [float(s[3][0]) for s in ref.spectra],
        "probe_overlaps": [float(om.scprod(p, ref.mps)) for p in probes(L)],
        "oracle_seconds": dt,
    }


def write(name: str, rec) -> None:
    path = os.path.join(HERE, name)
    with open(path, "w") as f:
        json.dump(rec, f, indent=0)
        f.write("\n")
    print("wrote", path, flush=True)


def make_xxz() -> None:
    write("xxz_L100_chi256_s4.json", single_chain_record(synth.workload_xxz(0), 4))


def make_decaying() -> None:
    write("decaying_L64_chi512_s4.json", single_chain_record(synth.workload_decaying(0), 4))


def make_decaying_tol() -> None:
    write("decaying_tol_L32_chi512_s2.json", single_chain_record(synth.workload_decaying_tol(0), 2))


def make_batch() -> None:
    chains = []
    t = time.perf_counter()
    for w in synth.workload_batch(0):
        ref = om.apply_simplify([np.asarray(x, np.float64) for x in w.mpo],
                                [np.asarray(x, np.float64) for x in w.mps], w.max_bond, w.tol, sweeps=4)
        chains.append({"name": w.name, "norm": ref.norm, "ranks": [int(x) for x in ref.ranks],
                       "error_bound": ref.error_bound, "discarded": ref.total_discarded,
                       "step_ranks": "".join(f"{int(r)}," for r in ref.step_ranks).rstrip(",")})
    write("batch512_s4.json", {"workload": "512 QTT chains, 4 sweeps", "sweeps": 4, "chains": chains,
                               "oracle_seconds": time.perf_counter() - t})


if __name__ == "__main__":
    which = sys.argv[1:] or ["batch", "xxz", "decaying_tol", "decaying"]
    for name in which:
        {"xxz": make_xxz, "decaying": make_decaying, "decaying_tol": make_decaying_tol,
         "batch": make_batch}[name]()
