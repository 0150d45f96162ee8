"""Pins of the FP64 reference of the learned preconditioner correction."""
import numpy as np
import pytest

import workloads as w
from oracle import mpnn
from oracle import precond as opc
from oracle import residual as ores


@pytest.fixture(scope="module")
def setup3d():
    prob = w.cube_mms(5, 1, perturb=0.2, seed=2)
    disc = ores.build(prob)
    nbr, om, dirs, bflag = mpnn.graph(disc)
    A = opc.assemble(disc)
    col = opc.greedy_colours(A)
    r = w.random_state(disc.n_cells, 3, seed=3, scale=1.0)
    z = opc.sgs(A, col, r, 2)
    e = z + 0.1 * w.random_state(disc.n_cells, 3, seed=4, scale=1.0)
    p = mpnn.init_params(0)
    rng = np.random.default_rng(9)
    p["Wd"] = rng.standard_normal(p["Wd"].shape) * 0.1
    p["bd"] = rng.standard_normal(3) * 0.1
    for l in range(mpnn.N_LAYERS):
        p[f"b{l}"] = rng.standard_normal(mpnn.WIDTH) * 0.1
    p["be"] = rng.standard_normal(mpnn.WIDTH) * 0.1
    return disc, (nbr, om, dirs, bflag), r, z, e, p


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    vals = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -9, -3.14159, 1e-3, 65504.0, 2 ** -130, 0.0])
    ref = torch.tensor(vals, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mpnn.bf16_round(vals), ref)
    rng = np.random.default_rng(0)
    x = rng.standard_normal(10000) * 10.0 ** rng.integers(-5, 5, 10000)
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mpnn.bf16_round(x), ref)


def test_graph_weights(setup3d):
    disc, (nbr, om, dirs, bflag), *_ = setup3d
    has = nbr >= 0
    assert np.allclose(om.sum(axis=1), 1.0)
    assert np.allclose(np.linalg.norm(dirs[has], axis=1), 1.0)
    # the neighbour relation is symmetric and directions are opposite
    for P in range(disc.n_cells):
        for s in np.nonzero(has[P])[0]:
            N = nbr[P, s]
            back = np.nonzero(nbr[N] == P)[0]
            assert back.size == 1
            assert np.allclose(dirs[N, back[0]], -dirs[P, s])


def test_aggregate_adjoint(setup3d):
    disc, (nbr, om, dirs, bflag), *_ = setup3d
    rng = np.random.default_rng(1)
    h = rng.standard_normal((disc.n_cells, 7))
    dA = rng.standard_normal((disc.n_cells, 4, 7))
    lhs = np.sum(mpnn.aggregate(h, nbr, om, dirs) * dA)
    rhs = np.sum(h * mpnn.aggregate_t(dA, nbr, om, dirs))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_zero_decoder_returns_plain_preconditioner(setup3d):
    disc, g, r, z, e, _ = setup3d
    p = mpnn.init_params(5)
    assert np.array_equal(mpnn.forward(p, r, z, *g), z)


def test_gradient_check_central_differences(setup3d):
    disc, g, r, z, e, p = setup3d
    loss, grads, _ = mpnn.loss_and_grad(p, r, z, e, *g)
    rng = np.random.default_rng(2)
    for name in ["We", "be", "W0", "b1", "W3", "Wd", "bd"]:
        for _ in range(4):
            idx = tuple(rng.integers(0, s) for s in p[name].shape)
            h = 1e-6 * max(1.0, abs(p[name][idx]))
            pp = {k: v.copy() for k, v in p.items()}
            pm = {k: v.copy() for k, v in p.items()}
            pp[name][idx] += h
            pm[name][idx] -= h
            lp = mpnn.loss_and_grad(pp, r, z, e, *g)[0]
            lm = mpnn.loss_and_grad(pm, r, z, e, *g)[0]
            fd = (lp - lm) / (2 * h)
            assert abs(fd - grads[name][idx]) <= 1e-6 * max(1e-8, np.abs(grads[name]).max()), (name, idx)


def test_homogeneity_and_permutation_equivariance(setup3d):
    disc, (nbr, om, dirs, bflag), r, z, e, p = setup3d
    out = mpnn.forward(p, r, z, nbr, om, dirs, bflag)
    assert np.allclose(mpnn.forward(p, 3.7 * r, 3.7 * z, nbr, om, dirs, bflag), 3.7 * out, rtol=1e-12)
    n = disc.n_cells
    perm = np.random.default_rng(7).permutation(n)
    inv = np.empty(n, np.int64)
    inv[perm] = np.arange(n)
    nbr_p = np.where(nbr[perm] >= 0, inv[np.maximum(nbr[perm], 0)], -1)
    out_p = mpnn.forward(p, r[perm], z[perm], nbr_p, om[perm], dirs[perm], bflag[perm])
    assert np.allclose(out_p, out[perm], rtol=1e-12, atol=1e-14)


def test_adam_reduces_loss(setup3d):
    disc, g, r, z, e, p = setup3d
    p = {k: v.copy() for k, v in p.items()}
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(vv) for k, vv in p.items()}
    l0 = mpnn.loss_and_grad(p, r, z, e, *g)[0]
    for t in range(1, 31):
        _, gr, _ = mpnn.loss_and_grad(p, r, z, e, *g)
        mpnn.adam_step(p, gr, m, v, t, lr=1e-3)
    l1 = mpnn.loss_and_grad(p, r, z, e, *g)[0]
    assert l1 < 0.8 * l0
