"""FP64 reference of the learned preconditioner correction (test infrastructure).

The paper has no learned component; this network is specified by the build's
goal (a small message-passing network over face neighbours that corrects the
compact preconditioner's output).  Definition:

* graph: cells, edges = internal faces.  For cell P and neighbour N,
  omega_PN = w_PN / sum_N' w_PN' with w_PN = Gamma_f / |d_PN . n_f| (the
  compact approximate Jacobian's coupling without Kbar), e_PN = d_PN / |d_PN|.
* inputs x_P = [r_P / s_r, z_P / s_z, b_P, 1] (8 numbers, 2D padded with zero
  third components), z = the plain preconditioner's output for residual r,
  s_r = RMS(r), s_z = RMS(z), b_P = 1 if P has a displacement face.
* h0 = relu(x W_e + b_e)                        (8 -> 64)
* 4 layers: A_0 = sum_N omega_PN h_N, A_d = sum_N omega_PN e_PN,d h_N (d = 1..3),
  X = [h, A_0, A_1, A_2, A_3] (320), Y = relu(X W_l + b_l), h <- h + Y
* g = h W_d + b_d (64 -> 3), output z + s_z g.
* loss of a pair (r, e): ||z + s_z g - e||^2 / ||e||^2 (s_z, s_r not differentiated).

``bf16=True`` rounds to bfloat16 (round to nearest even) where the GPU kernels
store or feed bfloat16: the inputs x, every weight matrix, h after each layer,
the aggregates A before the product, and in the backward pass the relu'd
gradient dY before its two products.
"""
from __future__ import annotations

import numpy as np

WIDTH = 64
N_LAYERS = 4
F_IN = 8
K_LAYER = 5 * WIDTH


def bf16_round(a):
    """Round float64/32 values to bfloat16 (nearest even), returned as float64."""
    f = np.asarray(a, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def graph(disc_full):
    """Neighbour lists and weights from an oracle discretisation (all cells).

    Returns nbr (n, 2D) int (-1 none), om (n, 2D), dirs (n, 2D, 3), bflag (n,)."""
    d = disc_full
    n, D = d.n_cells, d.dim
    S = 2 * D
    nbr = -np.ones((n, S), np.int64)
    om = np.zeros((n, S))
    dirs = np.zeros((n, S, 3))
    cnt = np.zeros(n, np.int64)
    dPN = d.cen[d.f_nei] - d.cen[d.f_own]
    w = d.f_area / np.abs(np.sum(dPN * d.f_n, axis=1))
    unit = dPN / np.linalg.norm(dPN, axis=1)[:, None]
    for f in range(d.f_own.size):
        for P, N, sgn in ((d.f_own[f], d.f_nei[f], 1.0), (d.f_nei[f], d.f_own[f], -1.0)):
            k = cnt[P]
            nbr[P, k] = N
            om[P, k] = w[f]
            dirs[P, k, :D] = sgn * unit[f]
            cnt[P] += 1
    om = om / np.maximum(om.sum(axis=1, keepdims=True), 1e-300)
    bflag = np.zeros(n)
    bflag[d.d_own] = 1.0
    return nbr, om, dirs, bflag


def init_params(seed: int):
    """He-style init for hidden layers, zero decoder (starts as the plain preconditioner)."""
    rng = np.random.default_rng(seed)
    p = {"We": rng.standard_normal((F_IN, WIDTH)) * np.sqrt(2.0 / F_IN), "be": np.zeros(WIDTH)}
    for l in range(N_LAYERS):
        p[f"W{l}"] = rng.standard_normal((K_LAYER, WIDTH)) * np.sqrt(2.0 / K_LAYER) * 0.5
        p[f"b{l}"] = np.zeros(WIDTH)
    p["Wd"] = np.zeros((WIDTH, 3))
    p["bd"] = np.zeros(3)
    return p


def aggregate(h, nbr, om, dirs):
    """[A_0, A_1, A_2, A_3] (n, 4, W)."""
    n, S = nbr.shape
    A = np.zeros((n, 4, h.shape[1]))
    for s in range(S):
        N = nbr[:, s]
        ok = N >= 0
        hN = np.where(ok[:, None], h[np.maximum(N, 0)], 0.0)
        w0 = om[:, s] * ok
        A[:, 0] += w0[:, None] * hN
        for dd in range(3):
            A[:, 1 + dd] += (w0 * dirs[:, s, dd])[:, None] * hN
    return A


def aggregate_t(dA, nbr, om, dirs):
    """Adjoint of aggregate: dh[N] += sum_P sum_d omega_PN e_PN,d dA_d[P]."""
    n, S = nbr.shape
    dh = np.zeros((n, dA.shape[2]))
    for s in range(S):
        N = nbr[:, s]
        ok = N >= 0
        coef = np.stack([om[:, s]] + [om[:, s] * dirs[:, s, dd] for dd in range(3)], axis=1) * ok[:, None]
        contrib = np.einsum("nd,ndw->nw", coef, dA)
        np.add.at(dh, N[ok], contrib[ok])
    return dh


def features(r, z, bflag):
    n, D = r.shape
    sr = np.sqrt(np.mean(r * r))
    sz = np.sqrt(np.mean(z * z))
    x = np.zeros((n, F_IN))
    x[:, :D] = r / sr
    x[:, 3:3 + D] = z / sz
    x[:, 6] = bflag
    x[:, 7] = 1.0
    return x, sr, sz


def forward(params, r, z, g_nbr, g_om, g_dirs, bflag, bf16=False, keep=False):
    """Corrected preconditioner output (n, D) and (if keep) the activations."""
    rnd = bf16_round if bf16 else (lambda a: a)
    n, D = r.shape
    x, sr, sz = features(r, z, bflag)
    x = rnd(x)
    pre0 = x @ rnd(params["We"]) + params["be"]
    h = rnd(np.maximum(pre0, 0.0))
    acts = {"x": x, "pre0": pre0, "h": [h], "X": [], "pre": []}
    for l in range(N_LAYERS):
        A = rnd(aggregate(h, g_nbr, g_om, g_dirs))
        X = np.concatenate([h, A.reshape(n, 4 * WIDTH)], axis=1)
        pre = X @ rnd(params[f"W{l}"]) + params[f"b{l}"]
        h = rnd(h + np.maximum(pre, 0.0))
        acts["X"].append(X)
        acts["pre"].append(pre)
        acts["h"].append(h)
    g = h @ rnd(params["Wd"]) + params["bd"]
    out = z + sz * g[:, :D]
    if keep:
        acts.update(sz=sz, sr=sr, g=g)
        return out, acts
    return out


def loss_and_grad(params, r, z, e, g_nbr, g_om, g_dirs, bflag, bf16=False):
    """Loss ||out - e||^2 / ||e||^2 and its gradient w.r.t. every parameter."""
    rnd = bf16_round if bf16 else (lambda a: a)
    n, D = r.shape
    out, a = forward(params, r, z, g_nbr, g_om, g_dirs, bflag, bf16, keep=True)
    ee = np.sum(e * e)
    diff = out - e
    loss = np.sum(diff * diff) / ee
    dout = 2.0 * diff / ee
    dg = np.zeros((n, 3))
    dg[:, :D] = a["sz"] * dout
    grads = {"Wd": a["h"][-1].T @ dg, "bd": dg.sum(axis=0)}
    dh = dg @ rnd(params["Wd"]).T
    for l in range(N_LAYERS - 1, -1, -1):
        dY = dh * (a["pre"][l] > 0)
        grads[f"W{l}"] = a["X"][l].T @ rnd(dY)
        grads[f"b{l}"] = dY.sum(axis=0)
        dX = rnd(dY) @ rnd(params[f"W{l}"]).T
        dA = dX[:, WIDTH:].reshape(n, 4, WIDTH)
        dh = dh + dX[:, :WIDTH] + aggregate_t(dA, g_nbr, g_om, g_dirs)
    dpre0 = dh * (a["pre0"] > 0)
    grads["We"] = a["x"].T @ dpre0
    grads["be"] = dpre0.sum(axis=0)
    return loss, grads, out


def adam_step(params, grads, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) in place; t starts at 1."""
    for k in params:
        m[k] = b1 * m[k] + (1 - b1) * grads[k]
        v[k] = b2 * v[k] + (1 - b2) * grads[k] ** 2
        mh = m[k] / (1 - b1 ** t)
        vh = v[k] / (1 - b2 ** t)
        params[k] = params[k] - lr * mh / (np.sqrt(vh) + eps)
