"""Orchestration of the learned preconditioner correction (data harvesting and
the training loop); every numerical step runs in libhofv.

Training pairs (r, e) with J e = r are produced by the solver itself:

* Krylov-type vectors: starting from a seeded random right-hand side b, the
  sequence v_0 = b/|b|, v_{k+1} = J M v_k / |J M v_k| (M = the plain
  preconditioner) mimics the vectors FGMRES hands to the preconditioner;
* Newton pairs: the residual R(u_k) of a Newton iterate and the converged
  correction of J du = -R(u_k).

Each e is solved to ``rtol`` by FGMRES(restart) with the context's plain
preconditioner (the sweeps, or the V-cycle when the context has it enabled).
"""
from __future__ import annotations

import numpy as np


def harvest_krylov(ctx, u, n_starts=4, length=6, seed=0, rtol=1e-8, n_sweeps=2, max_iters=3000, restart=30):
    """Returns r, e as device tensors [n_pairs, dim, n_cells]."""
    import torch
    dev = u.device
    D, n = u.shape
    Ru = torch.empty_like(u)
    ctx.residual(u, Ru)
    gen = torch.Generator(device="cpu").manual_seed(int(seed))
    rs, es = [], []
    tmp = torch.empty_like(u)
    for s in range(n_starts):
        v = torch.randn((D, n), generator=gen, dtype=torch.float64).to(dev)
        v /= torch.linalg.norm(v)
        for k in range(length):
            e = torch.zeros_like(u)
            ctx.fgmres_solve(u, Ru, v, e, rtol=rtol, max_iters=max_iters, n_sweeps=n_sweeps, check=False,
                             restart=restart)
            rs.append(v.clone())
            es.append(e)
            ctx.precond_apply(v, tmp, n_sweeps=n_sweeps)
            w = torch.empty_like(u)
            ctx.jvp(u, Ru, tmp, w)
            v = w / torch.linalg.norm(w)
    return torch.stack(rs), torch.stack(es)


def harvest_newton(ctx, u0, n_steps=3, rtol=1e-8, n_sweeps=2, max_iters=3000, restart=30):
    """Pairs (R(u_k), du_k) along a Newton solve from u0 (J du = -R, so e = -du
    for r = R; stored as (r, e) with J e = r)."""
    import torch
    u = u0.clone()
    rs, es = [], []
    R = torch.empty_like(u)
    for _ in range(n_steps):
        ctx.residual(u, R)
        e = torch.zeros_like(u)
        ctx.fgmres_solve(u, R, R, e, rtol=rtol, max_iters=max_iters, n_sweeps=n_sweeps, check=False,
                         restart=restart)
        nr = torch.linalg.norm(R)
        rs.append(R / nr)
        es.append(e / nr)
        u = u - e
    return torch.stack(rs), torch.stack(es)


def train(model, datasets, epochs=20, lr=1e-3, batch=4, n_sweeps=2, seed=0, log=None):
    """datasets: list of (ctx, r, e) with r, e [n_pairs, dim, n_cells].  Each
    optimisation step uses a minibatch of pairs from one mesh.  Returns the
    mean loss per epoch."""
    rng = np.random.default_rng(seed)
    hist = []
    for ep in range(epochs):
        jobs = []
        for di, (ctx, r, e) in enumerate(datasets):
            idx = rng.permutation(r.shape[0])
            for s in range(0, len(idx), batch):
                jobs.append((di, idx[s:s + batch]))
        rng.shuffle(jobs)
        tot, cnt = 0.0, 0
        for di, sel in jobs:
            ctx, r, e = datasets[di]
            import torch
            sel_t = torch.as_tensor(sel, device=r.device)
            loss = ctx.nn_train_step(model, r.index_select(0, sel_t).contiguous(),
                                     e.index_select(0, sel_t).contiguous(), n_sweeps=n_sweeps, lr=lr)
            tot += loss * len(sel)
            cnt += len(sel)
        hist.append(tot / max(cnt, 1))
        if log:
            log(ep, hist[-1])
    return hist
