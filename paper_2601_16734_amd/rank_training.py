"""Training data and training loop of the rank predictor.

Host orchestration only: the sweeps that produce the spectra, the pairing of
each step with the previous factorization of its bond, the forward/backward
passes and the Adam updates all run in the library (see smps_rank_* in the
C header).  The predictor sizes the sketch of the randomized factorization
(factorization=FACT_RSVD_MLP).
"""

from __future__ import annotations

import numpy as np

from . import binding as B


def collect_pairs(ctx: B.Context, problems, sweeps: int = 4):
    """Run the exact apply + compression on each problem and gather the
    (features, log rank) pairs its steps produce.

    problems: iterable of (mpo tensors, mps tensors, max_bond, tol)."""
    feats, labels = [], []
    for mpo, mps, max_bond, tol in problems:
        U = ctx.mpo_create(mpo)
        v = ctx.mps_create(mps)
        out, _ = ctx.mpo_apply(U, v, B.strategy(max_bond, tol, sweeps=sweeps))
        f, y = ctx.rank_training_pairs()
        feats.append(f)
        labels.append(y)
        out.destroy()
        v.destroy()
        U.destroy()
    if not feats:
        return np.zeros((0, 32), np.float32), np.zeros(0, np.float32)
    return np.concatenate(feats), np.concatenate(labels)


def train_predictor(ctx: B.Context, feats, labels, *, epochs: int = 60, batch: int = 256, lr: float = 1e-3,
                    seed: int = 0) -> float:
    """Initialise the predictor from `seed` and train it with mini-batch Adam;
    returns the mean loss of the last epoch."""
    ctx.rank_mlp_init(seed)
    return ctx.rank_mlp_train(feats, labels, epochs=epochs, batch=batch, lr=lr)
