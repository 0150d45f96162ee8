"""CPU checks of the library's host setup (host_only contexts) against the
oracle, and of the C ABI's exported symbols.  No GPU is used."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as w
from oracle import geometry as geo
from oracle import precond as opc
from oracle import residual as ores

api = pytest.importorskip("paper_2601_18417_amd.api")


def _tables(ctx, prob):
    S = prob.stencil_size
    D = prob.dim
    fst = ctx.host_table("face_stencil")
    nf = fst.size // S
    return S, D, nf, fst.reshape(S, nf).T


def _fan(prob):
    prob.face_rule = 1
    return prob


CASES = [lambda: w.square_mms(8, 2, perturb=0.2), lambda: w.square_mms(7, 3),
         lambda: w.cube_mms(6, 3, perturb=0.2), lambda: w.cube_mms(6, 2),
         lambda: w.poly_patch(w.box_mesh((5, 6, 5), perturb=0.2, seed=2), 1, 1,
                              traction_faces=lambda xc, n: xc[:, 1] > 1 - 1e-9),
         lambda: _fan(w.cube_mms(6, 3, perturb=0.2)),
         lambda: w.tri_mms(6, 3, perturb=0.2),
         lambda: w.tet_mms(3, 2, perturb=0.2), lambda: w.tet_mms(4, 3, perturb=0.2, seed=1),
         # face-list meshes with 8-edge / 24-face merged cells (one extrapolation item per face)
         lambda: w.poly_patch(w.split_block_mesh((4, 5), perturb=0.2, seed=2), 3, 3, seed=1,
                              traction_faces=lambda xc, n: xc[:, 1] > 1 - 1e-9),
         lambda: w.poly_patch(w.split_block_mesh((3, 3, 3), perturb=0.15, seed=4, mode="tensor"), 2, 2, seed=3)]


def _items(ctx, n):
    """Extrapolation items of the library's u* tables: (NS, NSI, item of
    (cell, slot)).  Items are cells with NSI slots each (as many as the most
    faces of a cell), or, when a cell has more than 2 dim faces, one item per
    slot with an internal or displacement face (a cell's items consecutive, in
    slot order)."""
    order = ctx.host_table("cell_order")
    cf = ctx.host_table("cell_faces")
    NS = cf.size // n
    cf = cf.reshape(NS, n)
    nf = ctx.host_table("face_own").size
    if order.size == n:
        item = np.argsort(order)
        S = ctx.host_table("cell_stencil").size // n
        NSI = ctx.host_table("cell_extrap").size // (S * n)
        used = (cf != np.iinfo(np.int32).min).any(axis=1)
        assert NSI == np.nonzero(used)[0].max() + 1  # the highest slot in use
        return NS, NSI, lambda P, s: (item[P], s)
    first = {}
    for r in range(order.size - 1, -1, -1):
        first[order[r]] = r
    where = {}
    for P, r0 in first.items():
        used = [s for s in range(NS) if cf[s, P] != np.iinfo(np.int32).min and cf[s, P] < nf]
        for k, s in enumerate(used):
            where[(P, s)] = (r0 + k, 0)
    return NS, 1, lambda P, s: where[(P, s)]


@pytest.mark.parametrize("mk", CASES)
def test_stencils_and_face_coefficients_match_oracle(mk):
    prob = mk()
    disc = ores.build(prob)
    ctx = api.context_for(prob, host_only=True)
    S, D, nf, fst = _tables(ctx, prob)
    own = ctx.host_table("face_own")
    nei = ctx.host_table("face_nei")
    fc = ctx.host_table("face_centre").reshape(nf, D)
    nfi = int(np.count_nonzero(nei >= 0))
    assert nfi == disc.f_own.size and nf - nfi == disc.d_own.size
    key = {(a, b): i for i, (a, b) in enumerate(zip(disc.f_own, disc.f_nei))}
    idx = np.array([key[(own[i], nei[i])] for i in range(nfi)], dtype=np.int64)
    # displacement faces: match by owner and centre
    dk = {(o, tuple(np.round(x, 9))): j for j, (o, x) in enumerate(zip(disc.d_own, disc.d_x))}
    jd = np.array([dk[(own[i], tuple(np.round(fc[i], 9)))] for i in range(nfi, nf)], dtype=np.int64)
    ost = np.concatenate([disc.f_st[idx], disc.d_st[jd]])
    order = np.argsort(ost, axis=1)
    assert np.array_equal(fst, np.take_along_axis(ost, order, 1))  # same sets, id-sorted
    coef = np.transpose(ctx.host_table("face_coef").reshape(S, D, nf), (2, 1, 0))
    oc = np.concatenate([np.einsum("fq,fqis->fis", disc.f_qw, disc.f_C)[idx],
                         np.einsum("fq,fqis->fis", disc.d_qw, disc.d_C)[jd]])
    oc = np.take_along_axis(oc, order[:, None, :], 2)
    assert np.abs(coef - oc).max() <= 1e-11 * np.abs(oc).max()
    order = ctx.host_table("cell_order")  # extrapolation item -> cell
    assert np.array_equal(np.unique(order), np.arange(disc.n_cells))
    assert order.size == disc.n_cells or ctx.host_table("cell_faces").size > 2 * D * disc.n_cells
    cst = ctx.host_table("cell_stencil").reshape(S, order.size).T
    assert np.array_equal(cst, np.sort(disc.c_st[order], axis=1))


@pytest.mark.parametrize("mk", CASES)
def test_extrapolation_rows_match_oracle(mk):
    """u*_{f,P} - u_P from the library's pre-contracted rows equals the
    oracle's derivative tensors contracted with d (eq. alphaJump)."""
    prob = mk()
    disc = ores.build(prob)
    ctx = api.context_for(prob, host_only=True)
    S, D, nf, fst = _tables(ctx, prob)
    n = disc.n_cells
    NS, NSI, where = _items(ctx, n)
    ni = ctx.host_table("cell_order").size
    ext = ctx.host_table("cell_extrap").reshape(S, NSI, ni)  # by extrapolation item
    cst = ctx.host_table("cell_stencil").reshape(S, ni)
    cf = ctx.host_table("cell_faces").reshape(NS, n)
    fc = ctx.host_table("face_centre").reshape(nf, D)
    u = w.random_state(n, D, seed=1, scale=1.0)
    for P in range(0, n, 7 if n > 40 else 1):
        for s in range(NS):
            code = cf[s, P]
            if code == np.iinfo(np.int32).min or code >= nf:
                continue
            f = code if code >= 0 else ~code
            r, si = where(P, s)
            lib = np.einsum("k,kj->j", ext[:, si, r], u[cst[:, r]])
            d = fc[f] - disc.cen[P]
            ref = ores.extrapolate(disc, u, np.array([P]), d[None])[0] - u[P]
            assert np.allclose(lib, ref, rtol=1e-10, atol=1e-10 * np.abs(u).max()), (P, s)


@pytest.mark.parametrize("mesh", [lambda: w.box_mesh((6, 5, 5), perturb=0.2, seed=3),
                                  lambda: w.tet_mesh((4, 4, 4), perturb=0.2, seed=3),
                                  lambda: w.tri_mesh((8, 7), perturb=0.2, seed=3),
                                  lambda: w.split_block_mesh((4, 4), perturb=0.2, seed=3),
                                  lambda: w.split_block_mesh((3, 2, 3), perturb=0.15, seed=3)])
def test_sources_match_oracle_plus_boundary_constants(mesh):
    """Cell sources = body force + traction faces + the u_b-dependent constants
    of displacement faces (ghost gradient term and u_b of the stabilisation),
    which the oracle carries inside its face fluxes: R_oracle(0) equals them."""
    prob = w.poly_patch(mesh(), 2, 2, seed=2, traction_faces=lambda xc, n: xc[:, 0] > 1 - 1e-9)
    disc = ores.build(prob)
    ctx = api.context_for(prob, host_only=True)
    n, D = disc.n_cells, disc.dim
    src = ctx.host_table("cell_src").reshape(D, n).T
    R0 = ores.residual(disc, np.zeros((n, D)))
    assert np.abs(src - R0).max() <= 1e-11 * np.abs(R0).max()


@pytest.mark.parametrize("mk", [lambda: w.cube_mms(5, 1, perturb=0.2), lambda: w.tet_mms(3, 1, perturb=0.2),
                                lambda: w.split_mms((3, 3, 2), 1, perturb=0.15, seed=2)])
def test_preconditioner_tables_match_oracle(mk):
    prob = mk()
    disc = ores.build(prob)
    A = opc.assemble(disc).toarray()
    col = opc.greedy_colours(opc.assemble(disc))
    ctx = api.context_for(prob, host_only=True)
    n = disc.n_cells
    perm = ctx.host_table("pc_perm")
    dinv = ctx.host_table("pc_dinv")
    NS = ctx.host_table("pc_a").size // n  # face slots per cell: 6, or the most faces of a polyhedron
    a = ctx.host_table("pc_a").reshape(NS, n)
    nbr = ctx.host_table("pc_nbr").reshape(NS, n)
    assert np.array_equal(np.sort(perm), np.arange(n))
    assert np.all(np.diff(col[perm]) >= 0)  # colour-major
    assert np.allclose(1.0 / dinv, np.diag(A)[perm], rtol=1e-6)
    off = 0
    for i in range(n):
        P = perm[i]
        for s in range(NS):
            if a[s, i] != 0:
                assert a[s, i] == pytest.approx(A[P, perm[nbr[s, i]]], rel=1e-6)
                off += 1
    assert off == np.count_nonzero(A) - n  # every off-diagonal entry is in a slot


def test_host_only_context_rejects_hot_calls():
    prob = w.square_mms(4, 1)
    ctx = api.context_for(prob, host_only=True)
    lib = ctx.lib
    st = lib.hofv_residual(ctx.h, ctypes.c_void_p(1), ctypes.c_void_p(2), None)
    assert st == -8  # HOFV_ESTATE


def test_setup_rejects_bad_parameters():
    with pytest.raises(api.HofvError):
        api.Context(4, 2, 10, 2, 0, 1.0, 1.0, stencil_quantum=1e-9, host_only=True)
    with pytest.raises(api.HofvError):
        api.Context(2, 2, 10, 2, 1, 1.0, 1.0, stencil_quantum=1e-9, host_only=True)  # NH in 2D
    with pytest.raises(api.HofvError):  # no such face rule
        api.Context(3, 2, 55, 2, 0, 1.0, 1.0, stencil_quantum=1e-9, host_only=True, face_rule=2)
    for nh, fold in ((1, True), (0, False)):  # the fan rule with per-point kernels (2 n_gauss^2 points)
        api.Context(3, 2, 55, 2, nh, 1.0, 1.0, stencil_quantum=1e-9, fold_quadrature=fold, host_only=True,
                    face_rule=1).close()
    ctx = api.Context(2, 3, 10, 2, 0, 1.0, 1.0, stencil_quantum=1e-9, host_only=True)
    mesh = w.box_mesh((2, 2))
    ctx.set_mesh(mesh.verts, mesh.cells)
    ctx.set_bc(np.zeros(8, np.int32), None, None, None)
    with pytest.raises(api.HofvError):  # stencil larger than the mesh
        ctx.setup()


def test_library_exports_every_declared_symbol(repo_root):
    hdr = open(os.path.join(repo_root, "include", "hofv.h")).read()
    names = set(re.findall(r"\b(hofv_[a-z_]+)\s*\(", hdr))
    lib = ctypes.CDLL(os.path.join(repo_root, "paper_2601_18417_amd", "libhofv.so"))
    missing = [nm for nm in names if not hasattr(lib, nm)]
    assert not missing, missing
    assert {"hofv_residual", "hofv_jvp", "hofv_precond_apply", "hofv_fgmres_solve",
            "hofv_newton_solve", "hofv_setup"} <= names


def test_learned_graph_tables_match_oracle():
    from oracle import mpnn
    prob = w.cube_mms(5, 1, perturb=0.2, seed=4)
    disc = ores.build(prob)
    nbr, om, dirs, bflag = mpnn.graph(disc)
    ctx = api.context_for(prob, host_only=True)
    n = disc.n_cells
    gn = ctx.host_table("nn_nbr").reshape(6, n)
    wf = ctx.host_table("nn_wf").reshape(6, n, 4).transpose(0, 2, 1)
    wb = ctx.host_table("nn_wb").reshape(6, n, 4).transpose(0, 2, 1)
    assert np.array_equal(ctx.host_table("nn_bflag"), bflag.astype(np.float32))
    for P in range(n):
        lib = {int(gn[s, P]): (wf[s, :, P], wb[s, :, P]) for s in range(6) if gn[s, P] >= 0}
        ora = {int(nbr[P, k]): k for k in range(6) if nbr[P, k] >= 0}
        assert set(lib) == set(ora)
        for N, k in ora.items():
            ref = np.concatenate([[om[P, k]], om[P, k] * dirs[P, k]])
            assert np.allclose(lib[N][0], ref, rtol=1e-6, atol=1e-7)
            back = [kk for kk in range(6) if nbr[N, kk] == P][0]
            refb = np.concatenate([[om[N, back]], om[N, back] * dirs[N, back]])
            assert np.allclose(lib[N][1], refb, rtol=1e-6, atol=1e-7)


@pytest.mark.parametrize("mk", [CASES[0], CASES[2], CASES[-1], lambda: w.cube_mms(12, 3, perturb=0.2, seed=5)])
def test_item_blocks_cover_stencils(mk):
    """Item blocks of the LDS-staged kernels: consecutive items, at most 256
    per block, a sorted union within the LDS capacity (1024 cells for face
    blocks, 1280 for cell blocks), and every local position maps back to the
    item's stencil entry."""
    prob = mk()
    ctx = api.context_for(prob, host_only=True)
    S = prob.stencil_size
    for kind, stn, cap in (("face", "face_stencil", 1024), ("cell", "cell_stencil", 1280)):
        st = ctx.host_table(stn)
        n = st.size // S
        st = st.reshape(S, n)
        bi = ctx.host_table(f"{kind}_blk_item")
        bc = ctx.host_table(f"{kind}_blk_cell")
        uc = ctx.host_table(f"{kind}_ucell")
        loc = ctx.host_table(f"{kind}_local").reshape(S, n).astype(np.int64)
        assert bi[0] == 0 and bi[-1] == n and np.all(np.diff(bi) > 0) and np.all(np.diff(bi) <= 256)
        assert bc[0] == 0 and bc[-1] == uc.size and np.all(np.diff(bc) <= cap)
        for b in range(bi.size - 1):
            un = uc[bc[b]:bc[b + 1]]
            assert np.all(np.diff(un) > 0)
            items = slice(bi[b], bi[b + 1])
            assert np.array_equal(un[loc[:, items]], st[:, items])
            assert np.array_equal(un, np.unique(st[:, items]))


@pytest.mark.parametrize("mk", [lambda: w.cube_mms(12, 2, perturb=0.0), lambda: w.cube_mms(14, 2, perturb=0.2),
                                lambda: w.cube_mms((10, 10, 10), 1, perturb=0.2, lengths=(1.0, 1.0, 0.1)),
                                lambda: w.cantilever(shape=(60, 6, 6), p=1, n_plus=20)])
def test_multigrid_aggregates_match_oracle(mk):
    prob = mk()
    disc = ores.build(prob)
    lev = opc.hierarchy(opc.assemble(disc))
    ctx = api.context_for(prob, host_only=True, precond_levels=8)
    sizes = ctx.host_table("mg_sizes")
    assert list(sizes) == [l["A"].shape[0] for l in lev]
    for l in range(len(lev) - 1):
        assert np.array_equal(ctx.host_table(f"mg_agg{l}"), lev[l]["agg"]), l


def test_bench_and_entry_points_compile(repo_root):
    import py_compile
    for f in ("bench.py", "__graft_entry__.py"):
        py_compile.compile(os.path.join(repo_root, f), doraise=True)


def test_bench_refuses_more_than_one_gpu(repo_root):
    """bench.py measures one GPU; --gpus 2 ends with status 2 and says so,
    before anything touches a GPU."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(repo_root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=repo_root)
    assert r.returncode == 2 and "one GPU only" in r.stderr and r.stdout == ""


def test_symmetry_faces_get_their_own_flux_codes():
    """Cells on a symmetry plane point one face slot at the symmetry fluxes
    (codes >= the number of internal and displacement faces)."""
    prob = w.poly_patch(w.box_mesh((5, 4, 4), perturb=0.2, seed=4, mode="tensor"), 2, 2, seed=6, symmetric=True)
    disc = ores.build(prob)
    ctx = api.context_for(prob, host_only=True)
    n = disc.n_cells
    cf = ctx.host_table("cell_faces").reshape(6, n)
    nf = len(disc.f_own) + len(disc.d_own)
    sym_codes = cf[(cf >= nf) & (cf != np.iinfo(np.int32).min)]
    assert sorted(sym_codes - nf) == list(range(disc.s_own.size))
    owners = np.nonzero((cf >= nf).any(axis=0))[0]
    assert sorted(owners) == sorted(disc.s_own)


def test_mesh_shapes_and_orientation_are_checked():
    """The binding refuses cell arrays of the wrong width (the library would
    read past them); the library refuses a negatively oriented tetrahedron."""
    mesh = w.tet_mesh((2, 2, 2))
    ctx = api.Context(3, 1, 20, 1, 0, 1.0, 1.0, stencil_quantum=1e-9, host_only=True)
    with pytest.raises(ValueError):
        ctx.set_mesh(mesh.verts, mesh.cells[:, :3])
    with pytest.raises(ValueError):
        ctx.set_mesh(mesh.verts[:, :2], mesh.cells)
    bad = mesh.cells.copy()
    bad[5] = bad[5][[0, 2, 1, 3]]
    with pytest.raises(api.HofvError):
        ctx.set_mesh(mesh.verts, bad)
    ok = api.Context(3, 1, 20, 1, 0, 1.0, 1.0, stencil_quantum=1e-9, host_only=True)
    ok.set_mesh(mesh.verts, mesh.cells)
    assert ok.n_cells == 48
    cen, _, qp = ok.boundary_faces()
    nb = cen.shape[0]
    with pytest.raises(ValueError):  # boundary arrays sized for another mesh
        ok.set_bc(np.zeros(nb - 1, np.int32), None, None, None)
    with pytest.raises(ValueError):
        ok.set_bc(np.zeros(nb, np.int32), np.zeros((nb, 1, 3)), np.zeros((nb - 1, 3)), None)
    ok.set_bc(np.zeros(nb, np.int32), np.zeros(qp.shape), np.zeros((nb, 3)), None)
    with pytest.raises(ValueError):
        ok.set_body_force(np.zeros((48, 1, 3)))
    ok.set_body_force(np.zeros(ok.volume_qpoints().shape))


def test_library_skewness_coefficients_on_sheared_grid():
    """The library's own stabilisation coefficients alpha Kbar Gamma / |d . n|
    (eq. alpha) and approximate-Jacobian couplings Kbar Gamma / |d . n| (Sec. 4.1)
    on the grid sheared by x += s y, against the closed forms (not the oracle):
    slanted faces (1 + s^2), flat faces 1, displacement faces 2 and 2 (1 + s^2)."""
    from test_oracle_residual import SHEAR, sheared_square
    n = 7
    prob = sheared_square(n)
    ctx = api.context_for(prob, host_only=True)
    kb, al, s2 = 2 * prob.mu + prob.lam, prob.alpha, SHEAR ** 2
    ijk = w.cell_ijk(prob.mesh)
    own = ctx.host_table("face_own")  # caller cell ids
    nei = ctx.host_table("face_nei")
    stab = ctx.host_table("face_stab")
    fc = ctx.host_table("face_centre").reshape(-1, 2)
    cen = ctx.host_table("centroids").reshape(-1, 2)
    for f in range(stab.size):
        P = own[f]
        if nei[f] >= 0:
            slanted = ijk[nei[f]][1] == ijk[P][1]
        else:  # a flat boundary face lies straight below or above the centroid's row
            slanted = abs(fc[f, 1] - cen[P, 1]) < 1e-12
        expect = al * kb * (1 + s2 if slanted else 1.0) * (1.0 if nei[f] >= 0 else 2.0)
        assert stab[f] == pytest.approx(expect, rel=1e-12)
    perm = ctx.host_table("pc_perm")
    a = ctx.host_table("pc_a").reshape(4, -1)
    nbr = ctx.host_table("pc_nbr").reshape(4, -1)
    for i in range(perm.size):
        for s in range(4):
            if a[s, i] != 0:
                di, dj = ijk[perm[nbr[s, i]]] - ijk[perm[i]]
                assert abs(di) + abs(dj) == 1
                assert a[s, i] == pytest.approx(kb * (1 + s2) if dj == 0 else kb, rel=1e-6)


def test_stencil_growth_matches_oracle():
    """stencil_grow: the library grows the same stencils as the oracle (a
    tensor-perturbed 12^3 grid at p = 3, whose 85-cell stencils are singular at
    some faces), to the same sizes, with the same folded coefficient per cell;
    the tables take the largest size."""
    prob = w.poly_patch(w.box_mesh((12, 12, 12), perturb=0.2, seed=7, mode="tensor"), 3, 3, seed=2)
    prob.stencil_grow = 10
    disc = ores.build(prob)
    ctx = api.context_for(prob, host_only=True)
    S = prob.stencil_size
    SW = ctx.report["stencil_size"]
    assert SW == disc.f_st.shape[1] > S
    n_or = sum(int(np.sum([np.unique(r).size > S for r in st])) for st in (disc.f_st, disc.d_st))
    n_or += int(np.sum([np.unique(r).size > S for r in disc.c_st if r[0] >= 0]))
    assert ctx.report["n_grown_stencils"] == n_or > 0
    D = 3
    fst = ctx.host_table("face_stencil").reshape(SW, -1).T
    nf = fst.shape[0]
    own = ctx.host_table("face_own")
    nei = ctx.host_table("face_nei")
    coef = np.transpose(ctx.host_table("face_coef").reshape(SW, D, nf), (2, 1, 0))  # (nf, D, SW)
    key = {(a, b): j for j, (a, b) in enumerate(zip(disc.f_own, disc.f_nei))}
    oc = np.einsum("fq,fqis->fis", disc.f_qw, disc.f_C)
    grown_faces = 0
    for i in range(nf):
        if nei[i] < 0:
            continue
        j = key[(own[i], nei[i])]
        big = np.unique(disc.f_st[j]).size > S
        grown_faces += big
        if not big and i % 9:
            continue
        ids = np.unique(fst[i])
        assert np.array_equal(ids, np.unique(disc.f_st[j]))
        lib = np.zeros((D, ids.size))
        ora = np.zeros((D, ids.size))
        np.add.at(lib.T, np.searchsorted(ids, fst[i]), coef[i].T)
        np.add.at(ora.T, np.searchsorted(ids, disc.f_st[j]), oc[j].T)
        assert np.abs(lib - ora).max() <= 1e-11 * np.abs(ora).max()
    assert grown_faces > 0


def _poly_ctx(m):
    mu, lam = w.lame_from_young(1.0, 0.3)
    return api.Context(m.dim, 1, 10 if m.dim == 2 else 45, 1, 0, mu, lam, stencil_quantum=1e-9, host_only=True)


@pytest.mark.parametrize("dim", [2, 3])
def test_face_list_meshes_that_do_not_close_are_refused(dim):
    """hofv_set_mesh_polyhedra refuses a face list whose cells do not close: a
    loop given the wrong way round, a missing face, a repeated face; and a face
    whose two cells are the same."""
    m = w.split_block_mesh((3, 3) if dim == 2 else (2, 2, 2), perturb=0.1, seed=1)

    def attempt(fp, fv, fc):
        ctx = _poly_ctx(m)
        try:
            ctx.set_mesh_poly(m.verts, fp, fv, fc, m.n_cells)
        except api.HofvError as e:
            return str(e)
        return None

    assert attempt(m.face_ptr, m.face_verts, m.face_cells) is None  # the mesh itself is accepted
    inner = int(np.nonzero(m.face_cells[:, 1] >= 0)[0][0])
    fv = m.face_verts.copy()
    a, b = m.face_ptr[inner], m.face_ptr[inner + 1]
    fv[a:b] = fv[a:b][::-1].copy()
    assert "close" in attempt(m.face_ptr, fv, m.face_cells)
    # a missing face (one of a merged cell's) and a repeated one
    deg = np.bincount(m.face_cells[m.face_cells >= 0], minlength=m.n_cells)
    big = int(np.argmax(deg))
    f = int(np.nonzero((m.face_cells[:, 0] == big) | (m.face_cells[:, 1] == big))[0][0])
    keep = np.ones(m.face_cells.shape[0], bool)
    keep[f] = False
    loops = [m.face_verts[m.face_ptr[i]:m.face_ptr[i + 1]] for i in range(keep.size)]
    sub = [loops[i] for i in np.nonzero(keep)[0]]
    fp = np.concatenate([[0], np.cumsum([len(x) for x in sub])])
    assert "close" in attempt(fp, np.concatenate(sub), m.face_cells[keep])
    rep = loops + [loops[f]]
    fp = np.concatenate([[0], np.cumsum([len(x) for x in rep])])
    assert "close" in attempt(fp, np.concatenate(rep), np.vstack([m.face_cells, m.face_cells[f:f + 1]]))
    fc = m.face_cells.copy()
    fc[inner, 1] = fc[inner, 0]
    assert "bad face cells" in attempt(m.face_ptr, m.face_verts, fc)


def test_limits_of_255_are_enforced():
    """A cell of 294 faces (a merged 7 x 7 x 7 block), a stencil of more than
    255 cells and stencil growth above 255 are refused with HOFV_EINVAL; the
    largest accepted cells (216 faces, 252 edges) set up."""
    m = w.merged_block_mesh(w.box_mesh((9, 9, 9)), (1, 1, 1), (8, 8, 8))
    fc = m.face_cells
    assert np.bincount(fc[fc >= 0]).max() == 294
    with pytest.raises(api.HofvError, match="more than 255 faces"):
        api.context_for(w.poly_patch(m, 1, 1, seed=1), host_only=True)
    for mk in (lambda: w.merged_block_mesh(w.box_mesh((8, 8, 8), perturb=0.15, seed=5, mode="tensor"),
                                           (1, 1, 1), (7, 7, 7)),
               lambda: w.merged_block_mesh(w.box_mesh((65, 65), perturb=0.2, seed=5), (1, 1), (64, 64))):
        api.context_for(w.poly_patch(mk(), 1, 2, seed=3), host_only=True).close()
    prob = w.cube_mms(8, 2, perturb=0.2)
    prob.n_plus = 250  # |S| = 10 + 250
    with pytest.raises(api.HofvError, match="above 255"):
        api.context_for(prob, host_only=True)
    prob = w.cube_mms(8, 2, perturb=0.2)
    prob.stencil_grow = 256
    with pytest.raises(api.HofvError):
        api.context_for(prob, host_only=True)


@pytest.mark.parametrize("kind", ["quads", "tris", "hexes", "tets"])
def test_geometry_is_translation_stable(kind):
    """Centroids of cells far from the origin (|x| / h ~ 10^3 to 10^4, where a
    2D shoelace formula in absolute coordinates would lose about (|x| / h)^2
    of its precision) agree with the oracle's to 1e-10 of the cell size."""
    if kind in ("quads", "tris"):
        mk = w.box_mesh if kind == "quads" else w.tri_mesh
        mesh = mk((64, 48), lengths=(1.0, 0.75), origin=(100.0, -50.0), perturb=0.2, seed=3)
        h = 1.0 / 64
    else:
        mk = w.box_mesh if kind == "hexes" else w.tet_mesh
        mesh = mk((24, 20, 16), lengths=(1.0, 0.8, 0.64), origin=(100.0, -50.0, 30.0), perturb=0.2, seed=3)
        h = 1.0 / 24
    ctx = api.context_for(w.poly_patch(mesh, 1, 1, seed=1), host_only=True)
    vol, cen = geo.cell_volume_centroid(mesh.verts[mesh.cells])
    assert np.abs(ctx.cell_centroids() - cen).max() <= 1e-10 * h
