"""hofv_jvp_noalloc (the J.v whose reduction scratch is the library's static
device array) against hofv_jvp through the C ABI: two calls in a row, the
second on a smaller mesh, each to the J.v parity bar (1e-6 relative with the
same eps; the arithmetic is the same, so the results agree exactly)."""
import numpy as np
import pytest

import workloads as w

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _case(api, prob, seed):
    ctx = api.context_for(prob)
    n, D = prob.mesh.n_cells, prob.dim
    u = torch.tensor(w.random_state(n, D, seed=seed).T.copy(), device=DEV)
    v = torch.tensor(np.random.default_rng(seed + 1).standard_normal((D, n)), device=DEV)
    Ru = torch.empty_like(u)
    ctx.residual(u, Ru)
    return ctx, u, v, Ru


def test_jvp_noalloc_matches_jvp_on_two_calls():
    from paper_2601_18417_amd import api
    for prob, seed in ((w.cube_mms(12, 3, perturb=0.2, seed=1), 3), (w.square_mms(9, 2, perturb=0.2, seed=2), 5)):
        ctx, u, v, Ru = _case(api, prob, seed)
        for eps in (0.0, 1e-7):  # device eps from the norms, and a given one
            ref = torch.empty_like(u)
            out = torch.full_like(u, float("nan"))
            ctx.jvp(u, Ru, v, ref, eps=eps)
            ctx.jvp_noalloc(u, Ru, v, out, eps=eps)
            torch.cuda.synchronize()
            rel = float(torch.linalg.norm(out - ref) / torch.linalg.norm(ref))
            assert rel <= 1e-6, (prob.name, eps, rel)
            assert torch.equal(out, ref)
        ctx.close()


def test_jvp_noalloc_argument_errors():
    from paper_2601_18417_amd import api
    ctx, u, v, Ru = _case(api, w.square_mms(6, 1), 7)
    with pytest.raises(api.HofvError):
        ctx.jvp_noalloc(u, Ru, v, u)  # output aliases an input
    with pytest.raises(api.HofvError):
        ctx.jvp_noalloc(u, Ru, v, torch.empty_like(u), eps=float("inf"))
