"""Orchestration of the learned preconditioner correction: argument
marshalling around the library's pair harvesting (hofv_harvest_pairs) and
training loop (hofv_nn_train); every numerical step runs in libhofv.

Training pairs (r, e) with J e = r are produced by the solver itself:

* Krylov-type vectors: from a seeded random right-hand side b,
  v_0 = b/|b|, v_{k+1} = J M v_k / |J M v_k| (M = the plain preconditioner),
  the vectors FGMRES hands to the preconditioner;
* Newton pairs: the residual R(u_k) of a Newton iterate and the solution of
  J e = R(u_k), both scaled by 1/|R(u_k)|.

Each e is solved to ``rtol`` by FGMRES(restart) with the context's plain
preconditioner (the sweeps, or the V-cycle when the context has it enabled).
"""
from __future__ import annotations

from . import api


def harvest(ctx, u, n_starts=4, length=6, newton_steps=2, seed=0, rtol=1e-8, n_sweeps=2, max_iters=3000,
            restart=30, starts=None, pairs=None):
    """A PairSet of n_starts * length Krylov-type pairs and newton_steps
    Newton pairs at state u (device tensor [dim, n_cells])."""
    if pairs is None:
        pairs = api.PairSet(ctx, n_starts * length + newton_steps)
    ctx.harvest_pairs(pairs, u, n_starts=n_starts, length=length, newton_steps=newton_steps, seed=seed,
                      starts=starts, rtol=rtol, restart=restart, max_iters=max_iters, n_sweeps=n_sweeps)
    return pairs


def train(model, pair_sets, epochs=20, lr=1e-3, batch=4, n_sweeps=2, seed=0):
    """hofv_nn_train: minibatches of `batch` pairs from one set each, in a
    seeded order; returns the mean loss per epoch."""
    _, hist = api.nn_train(model, pair_sets, epochs=epochs, lr=lr, batch=batch, n_sweeps=n_sweeps, seed=seed)
    return hist
