"""The high-order finite-volume residual R(u) (paper Secs. 3.2-3.5, Apps. A-B).

Test infrastructure (see package docstring).

    R_P(u) = sum_{f in int}  Gamma_f n_f . [sum_q alpha_q sigma_{f,q}]          (eq. divStressDiscret)
           + sum_{b in disp} Gamma_b n_b . [sum_q alpha_q sigma_{b,q}]
           + sum_{b in trac} Gamma_b sum_q alpha_q T_{b,q}
           + sum_{f in int u disp} t_{alpha,f} Gamma_f                             (eq. alpha)
           + sum_q beta_q f_b(x_{Omega,q}) Omega_P                                  (eq. bodyTerm)

with internal-face terms added to the owner and subtracted from the neighbour.
R(u) = 0 is static equilibrium (Sec. 4.1).

* (grad u)_{f,q} = sum_N c_{x_N} (x) u_N (+ c_b (x) u_{b,q} on displacement faces),
  eq. faceQuadGrad, stored as G[i][j] = d u_j / d x_i.
* Linear elasticity: sigma = mu G + mu G^T + lambda tr(G) I (eq. linearElastic).
* Neo-Hookean (total Lagrangian): F = I + G^T, J = det F, b = F F^T,
  bbar = J^{-2/3} b, sigma = (mu/J) dev(bbar) + (kappa/2)(J^2-1)/J I (eq. neoHook),
  P = J sigma F^{-T} (eq. nanson), face term n_o . P^T (eq. momentum_TL);
  kappa = lambda + 2 mu / 3.  J^{-2/3} is evaluated as exp(-2/3 ln J) so the
  complex-step derivative goes through; J, b and dev(bbar) are formed from
  H = grad u^T without cancelling O(1) terms (see piola_neo_hookean).
* alpha-stabilisation: t = alpha Kbar / |d_PN . n_f| (u*_{f,N} - u*_{f,P}), Kbar = 2 mu + lambda;
  on displacement faces t = alpha Kbar / |d_Pb . n_b| (u_b(x_b) - u*_{b,P}).  The
  extrapolations u* use u_P itself plus d . grad u + 1/2 d^2 : grad grad u
  + 1/6 d^3 ::: grad grad grad u from the cell stencil (eq. alphaJump, App. B).
* Traction faces: Gamma_b sum_q alpha_q T_{b,q} (the weights alpha_q are taken to
  apply, as in the other surface terms; the printed equation omits them).
* Symmetry faces (Sec. 3.5): the stencil is the ceil(|S|/2) cells nearest to the
  face centre plus their mirror images through the face plane; the gradient is
  sum_N c_N (x) u_N + sum_N c'_N (x) (R_b u_N), R_b = I - 2 n n, with c and c'
  from one reconstruction over both sets of positions; the face term is
  Gamma n . sum_q alpha_q sigma_q as on displacement faces, with no
  stabilisation term.
* Loads (u_b, T, f_b) are multiplied by ``load`` for load increments.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from workloads.fields import DISP, SYMM, TRAC

from . import geometry as geo
from .lsq import SingularStencil, pivot_ok, reconstruction, row_index
from .stencil import nearest


@dataclass
class Discretisation:
    dim: int
    p: int
    n_cells: int
    material: int
    mu: float
    lam: float
    alpha: float
    cen: np.ndarray
    vol: np.ndarray
    # internal faces (possibly only those touching active cells)
    f_own: np.ndarray
    f_nei: np.ndarray
    f_n: np.ndarray
    f_area: np.ndarray
    f_x: np.ndarray
    f_qw: np.ndarray
    f_st: np.ndarray      # (nf, S)
    f_C: np.ndarray       # (nf, Nq, D, S)
    # displacement faces
    d_own: np.ndarray
    d_n: np.ndarray
    d_area: np.ndarray
    d_x: np.ndarray
    d_qw: np.ndarray
    d_st: np.ndarray
    d_C: np.ndarray       # (nd, Nq, D, S)
    d_Cg: np.ndarray      # (nd, Nq, D) ghost coefficients
    d_ubq: np.ndarray     # (nd, Nq, D) prescribed u at q-points (load 1)
    d_ubc: np.ndarray     # (nd, D) prescribed u at face centre (load 1)
    # cell stencils and derivative coefficients (for cells that need u*)
    c_st: np.ndarray      # (n_c, S), -1 rows where not built
    c_D1: np.ndarray      # (n_c, D, S)
    c_D2: np.ndarray | None  # (n_c, D, D, S)
    c_D3: np.ndarray | None  # (n_c, D, D, D, S)
    # constant sources at load 1
    b_body: np.ndarray    # (n_c, D)
    b_trac: np.ndarray    # (n_c, D)
    active: np.ndarray    # (n_c,) bool: cells whose R is complete
    max_cond: float = 0.0
    # symmetry faces: half stencil (n_s, ceil(S/2)), coefficients of the cells
    # and of their mirror images (n_s, Nq, D, ceil(S/2)); None when there are none
    s_own: np.ndarray | None = None
    s_n: np.ndarray | None = None
    s_area: np.ndarray | None = None
    s_x: np.ndarray | None = None
    s_qw: np.ndarray | None = None
    s_st: np.ndarray | None = None
    s_C: np.ndarray | None = None
    s_Cg: np.ndarray | None = None

    @property
    def kbar(self):
        return 2.0 * self.mu + self.lam


def _face_coefficients(xq, st, cen, p, k, ghost_weight=None):
    """Gradient rows at every face q-point: (nf, Nq, D, S) and ghost (nf, Nq, D)."""
    nf, nq, D = xq.shape
    S = st.shape[1]
    pts = xq.reshape(nf * nq, D)
    Xs = np.repeat(cen[st], nq, axis=0)  # (nf*nq, S, D)
    A, cond = reconstruction(pts, Xs, p, k, ghost_weight)
    rows = row_index(D, p)
    grad_rows = [rows[tuple(1 if d == i else 0 for d in range(D))] for i in range(D)]
    C = A[:, grad_rows, :S].reshape(nf, nq, D, S)
    Cg = A[:, grad_rows, S].reshape(nf, nq, D) if ghost_weight is not None else None
    return C, Cg, cond.max(initial=0.0)


def _symmetry_coefficients(xq, st, cen, xf, nrm, p, k):
    """Gradient rows at symmetry-face q-points over the half stencil (cells) and
    its mirror images through the face plane: two (nf, Nq, D, S_half) arrays."""
    nf, nq, D = xq.shape
    Sh = st.shape[1]
    Xp = cen[st]
    dist = np.einsum("fsd,fd->fs", Xp - xf[:, None, :], nrm)
    Xg = Xp - 2.0 * dist[..., None] * nrm[:, None, :]
    Xs = np.repeat(np.concatenate([Xp, Xg], axis=1), nq, axis=0)
    A, cond = reconstruction(xq.reshape(nf * nq, D), Xs, p, k)
    rows = row_index(D, p)
    grad_rows = [rows[tuple(1 if d == i else 0 for d in range(D))] for i in range(D)]
    C = A[:, grad_rows, :].reshape(nf, nq, D, 2 * Sh)
    return C[..., :Sh], C[..., Sh:], cond.max(initial=0.0)


def _cell_coefficients(cells, st, cen, p, k):
    """Derivative tensors at cell centroids: D1 (m,D,S), D2 (m,D,D,S), D3 (m,D,D,D,S)."""
    D = cen.shape[1]
    A, cond = reconstruction(cen[cells], cen[st], p, k)
    rows = row_index(D, p)

    def row(*axes):
        e = [0] * D
        for a in axes:
            e[a] += 1
        return rows[tuple(e)]

    m, S = st.shape
    D1 = np.stack([A[:, row(i), :] for i in range(D)], axis=1)
    D2 = D3 = None
    if p >= 2:
        D2 = np.empty((m, D, D, S))
        for i in range(D):
            for j in range(D):
                D2[:, i, j] = A[:, row(i, j), :]
    if p >= 3:
        D3 = np.empty((m, D, D, D, S))
        for i in range(D):
            for j in range(D):
                for l in range(D):
                    D3[:, i, j, l] = A[:, row(i, j, l), :]
    return D1, D2, D3, cond.max(initial=0.0)


def build(problem, active=None) -> Discretisation:
    """Set up geometry, stencils, coefficients and sources for ``problem``.

    ``active`` (optional bool mask or index array) restricts the work to what the
    residual of those cells needs; R is then only complete on active cells.
    """
    mesh = problem.mesh
    D, p, S = mesh.dim, problem.p, problem.stencil_size
    n_c = mesh.n_cells
    poly = hasattr(mesh, "face_cells")  # a face-list (polygonal / polyhedral) mesh
    if poly:
        own, nei, loops = geo.poly_faces(mesh)
        faces = geo.Faces(owner=own, neigh=nei, verts=None, owner_slot=None, neigh_slot=None)
        fg = geo.polygon_face_geometry(mesh.verts, loops, problem.n_gauss)
        vol, cen, vq_pts, vq_w, vq_cell = geo.poly_cells(mesh, own, nei, loops, p + 2)
    else:
        X = mesh.verts[mesh.cells]
        vol, cen = geo.cell_volume_centroid(X)
        faces = geo.enumerate_faces(mesh.cells, D)
        fg = geo.face_geometry(mesh.verts, faces.verts, problem.n_gauss, fan=problem.face_rule == 1)
    act = np.ones(n_c, bool)
    if active is not None:
        act = np.zeros(n_c, bool)
        act[np.asarray(active)] = True
    touch = act[faces.owner] | np.where(faces.neigh >= 0, act[np.maximum(faces.neigh, 0)], False)
    internal = (faces.neigh >= 0) & touch
    bnd = (faces.neigh < 0) & touch
    loads = problem.loads
    btype = loads.bc_type(fg.centre[bnd], fg.normal[bnd]) if bnd.any() else np.zeros(0, np.int32)
    bidx = np.nonzero(bnd)[0]
    disp = bidx[btype == DISP]
    trac = bidx[btype == TRAC]
    sym = bidx[btype == SYMM]
    q = problem.stencil_quantum
    k = problem.k_weight

    fi = np.nonzero(internal)[0]
    nq = fg.qpts.shape[1]
    grow = int(getattr(problem, "stencil_grow", 0))

    def stencils(ref, ok):
        """The S nearest cells of each reference point; with stencil_grow = g > 0
        a stencil whose least-squares systems fail the pivot test becomes the
        S + g, S + 2g, ... nearest (up to 255 cells and the cell count): a larger n+
        where the conditioning needs it (Sec. 5's ill-conditioning study).
        Returns the per-point cell lists and their sizes."""
        st = nearest(ref, cen, S, q) if ref.shape[0] else np.zeros((0, S), np.int64)
        rows = list(st)
        size = np.full(ref.shape[0], S)
        if grow <= 0 or ref.shape[0] == 0:
            return rows, size
        bad = ~ok(np.arange(ref.shape[0]), st)
        step = 0
        while bad.any():
            step += 1
            Sg = S + step * grow
            if Sg > 255 or Sg > n_c:
                raise SingularStencil("a stencil still fails the pivot test after growing it")
            idx = np.nonzero(bad)[0]
            stg = nearest(ref[idx], cen, Sg, q)
            for j, i in enumerate(idx):
                rows[i] = stg[j]
                size[i] = Sg
            bad[:] = False
            bad[idx[~ok(idx, stg)]] = True
        return rows, size

    def faces_ok(fids, ghost):
        def ok(idx, st):  # every weighted point of each face
            okq = pivot_ok(fg.qpts[fids[idx]].reshape(-1, D), np.repeat(cen[st], nq, axis=0), p, k, ghost)
            return np.all(okq.reshape(idx.size, nq) | (fg.qw[fids[idx]] == 0.0), axis=1)
        return ok

    f_rows, f_size = stencils(fg.centre[fi], faces_ok(fi, None))
    d_rows, d_size = stencils(fg.centre[disp], faces_ok(disp, problem.ghost_weight))
    # cells whose u* is needed: both sides of internal faces, owners of disp faces
    need = np.zeros(n_c, bool)
    need[faces.owner[fi]] = True
    need[faces.neigh[fi]] = True
    need[faces.owner[disp]] = True
    cells = np.nonzero(need)[0]
    c_rows, c_size = stencils(cen[cells], lambda idx, st: pivot_ok(cen[cells[idx]], cen[st], p, k))
    # one table width: the largest stencil; shorter ones are padded with their
    # last cell and zero coefficients (a zero coefficient adds nothing)
    SW = int(max([S] + [int(z.max()) for z in (f_size, d_size, c_size) if z.size]))

    def padded(rows, size):
        out = np.zeros((len(rows), SW), np.int64)
        for i, r in enumerate(rows):
            out[i, :size[i]] = r
            out[i, size[i]:] = r[-1]
        return out

    def face_tables(fids, rows, size, ghost):
        C = np.zeros((len(rows), nq, D, SW))
        Cg = np.zeros((len(rows), nq, D))
        cmax = 0.0
        for s_ in np.unique(size):
            g = np.nonzero(size == s_)[0]
            Cs, Cgs, c = _face_coefficients(fg.qpts[fids[g]], np.array([rows[i] for i in g]), cen, p, k, ghost)
            C[g, :, :, :s_] = Cs
            if Cgs is not None:
                Cg[g] = Cgs
            cmax = max(cmax, c)
        return padded(rows, size), C, Cg, cmax

    f_st, f_C, _, c1 = face_tables(fi, f_rows, f_size, None)
    d_st, d_C, d_Cg, c2 = face_tables(disp, d_rows, d_size, problem.ghost_weight)
    sym_kw, c4 = {}, 0.0
    if sym.size:
        s_st = nearest(fg.centre[sym], cen, (S + 1) // 2, q)
        s_C, s_Cg, c4 = _symmetry_coefficients(fg.qpts[sym], s_st, cen, fg.centre[sym], fg.normal[sym], p, k)
        sym_kw = dict(s_own=faces.owner[sym], s_n=fg.normal[sym], s_area=fg.area[sym], s_x=fg.centre[sym],
                      s_qw=fg.qw[sym], s_st=s_st, s_C=s_C, s_Cg=s_Cg)

    c_st = np.full((n_c, SW), -1, np.int64)
    c_st[cells] = padded(c_rows, c_size)
    c_D1 = np.zeros((n_c, D, SW))
    c_D2 = np.zeros((n_c, D, D, SW)) if p >= 2 else None
    c_D3 = np.zeros((n_c, D, D, D, SW)) if p >= 3 else None
    c3 = 0.0
    for s_ in np.unique(c_size):
        g = np.nonzero(c_size == s_)[0]
        D1, D2, D3, c = _cell_coefficients(cells[g], np.array([c_rows[i] for i in g]), cen, p, k)
        c_D1[cells[g], ..., :s_] = D1
        if D2 is not None:
            c_D2[cells[g], ..., :s_] = D2
        if D3 is not None:
            c_D3[cells[g], ..., :s_] = D3
        c3 = max(c3, c)

    # body force: (p+2)^D Gauss points of the cell map (of each sub-simplex of a
    # polyhedral cell)
    b_body = np.zeros((n_c, D))
    ac = np.nonzero(act)[0]
    if poly:
        sel = act[vq_cell]
        if sel.any():
            fb = loads.body(vq_pts[sel])
            np.add.at(b_body, vq_cell[sel], vq_w[sel, None] * fb)
    elif ac.size:
        pts, W = geo.cell_quadrature(X[ac], p + 2)
        fb = loads.body(pts.reshape(-1, D)).reshape(pts.shape)
        b_body[ac] = np.einsum("cq,cqd->cd", W, fb)
    # traction faces
    b_trac = np.zeros((n_c, D))
    if trac.size:
        nq = fg.qpts.shape[1]
        T = loads.traction(fg.qpts[trac].reshape(-1, D), np.repeat(fg.normal[trac], nq, axis=0))
        T = T.reshape(trac.size, nq, D)
        contrib = fg.area[trac, None] * np.einsum("fq,fqd->fd", fg.qw[trac], T)
        np.add.at(b_trac, faces.owner[trac], contrib)
    # prescribed displacements
    nq = fg.qpts.shape[1]
    d_ubq = loads.u_b(fg.qpts[disp].reshape(-1, D)).reshape(disp.size, nq, D)
    d_ubc = loads.u_b(fg.centre[disp])

    return Discretisation(
        dim=D, p=p, n_cells=n_c, material=problem.material, mu=problem.mu, lam=problem.lam,
        alpha=problem.alpha, cen=cen, vol=vol,
        f_own=faces.owner[fi], f_nei=faces.neigh[fi], f_n=fg.normal[fi], f_area=fg.area[fi],
        f_x=fg.centre[fi], f_qw=fg.qw[fi], f_st=f_st, f_C=f_C,
        d_own=faces.owner[disp], d_n=fg.normal[disp], d_area=fg.area[disp], d_x=fg.centre[disp],
        d_qw=fg.qw[disp], d_st=d_st, d_C=d_C, d_Cg=d_Cg, d_ubq=d_ubq, d_ubc=d_ubc,
        c_st=c_st, c_D1=c_D1, c_D2=c_D2, c_D3=c_D3, b_body=b_body, b_trac=b_trac, active=act,
        max_cond=float(max(c1, c2, c3, c4)), **sym_kw)


# ----------------------------------------------------------------------------- stresses

def cell_gradient(disc: Discretisation, u: np.ndarray) -> np.ndarray:
    """Post-processing (Sec. 5's stress errors): grad u at every cell centroid
    from the cell stencil's least-squares gradient rows, G[i][j] = d u_j / d x_i
    (cells without a stencil get 0)."""
    st = np.maximum(disc.c_st, 0)
    return np.einsum("cis,csj->cij", disc.c_D1, np.asarray(u, float)[st])


def stress_linear(G, mu, lam):
    """eq. linearElastic with G[..., i, j] = d u_j / d x_i."""
    D = G.shape[-1]
    tr = np.trace(G, axis1=-2, axis2=-1)
    return mu * G + mu * np.swapaxes(G, -1, -2) + lam * tr[..., None, None] * np.eye(D)


def piola_neo_hookean(G, mu, lam):
    """First Piola-Kirchhoff stress P = J sigma F^{-T} of eq. neoHook (3D).

    With H = G^T (so F = I + H) the same quantities are formed from H alone:
    J - 1 = tr H + ((tr H)^2 - tr(H H)) / 2 + det H (the expansion of
    det(I + H)), b - I = H + H^T + H H^T, dev(bbar) = J^{-2/3} dev(b - I) (dev I
    = 0), J^2 - 1 = (J - 1)(J + 1) and ln J = log1p(J - 1).  Forming J, b and
    dev(bbar) from F instead subtracts numbers of size 1 whose difference is
    the strain, which at the strains of a finite-difference product (~1e-8)
    leaves only about half of the digits.
    """
    D = G.shape[-1]
    if D != 3:
        raise ValueError("the neo-Hookean law is implemented in 3D only")
    kappa = lam + 2.0 * mu / 3.0
    I = np.eye(3)
    H = np.swapaxes(G, -1, -2)
    Ht = G
    trH = np.trace(H, axis1=-2, axis2=-1)
    Jm1 = trH + 0.5 * (trH * trH - np.trace(H @ H, axis1=-2, axis2=-1)) + np.linalg.det(H)
    J = 1.0 + Jm1
    B = H + Ht + H @ Ht
    devB = B - (np.trace(B, axis1=-2, axis2=-1) / 3.0)[..., None, None] * I
    jm23 = np.exp(-2.0 / 3.0 * np.log1p(Jm1))
    sigma = (mu / J * jm23)[..., None, None] * devB + (0.5 * kappa * Jm1 * (J + 1.0) / J)[..., None, None] * I
    Finv_T = np.swapaxes(np.linalg.inv(I + H), -1, -2)
    return J[..., None, None] * sigma @ Finv_T


def face_term(disc, G, normal, area, qw):
    """Gamma n . [sum_q alpha_q S_q] where S = sigma (LE) or P^T (NH)."""
    if disc.material == 0:
        Sq = stress_linear(G, disc.mu, disc.lam)
    else:
        Sq = np.swapaxes(piola_neo_hookean(G, disc.mu, disc.lam), -1, -2)
    Sbar = np.einsum("fq,fqij->fij", qw, Sq)
    return area[:, None] * np.einsum("fi,fij->fj", normal, Sbar)


# ----------------------------------------------------------------------------- u*

def extrapolate(disc, u, cells, d):
    """u*_{f,X} = u_X + d.grad u_X + 1/2 d^2 : grad grad u_X + 1/6 d^3 ::: grad^3 u_X."""
    st = disc.c_st[cells]
    ug = u[st]  # (m, S, D)
    grad = np.einsum("mis,msj->mij", disc.c_D1[cells], ug)
    val = u[cells] + np.einsum("mi,mij->mj", d, grad)
    if disc.p >= 2:
        H = np.einsum("miks,msj->mikj", disc.c_D2[cells], ug)
        val = val + 0.5 * np.einsum("mi,mk,mikj->mj", d, d, H)
    if disc.p >= 3:
        T = np.einsum("mikls,msj->miklj", disc.c_D3[cells], ug)
        val = val + (1.0 / 6.0) * np.einsum("mi,mk,ml,miklj->mj", d, d, d, T)
    return val


# ----------------------------------------------------------------------------- residual

def face_fluxes(disc, u, load=1.0):
    """Internal-face fluxes (owner side) and displacement-face fluxes."""
    kbar = disc.kbar
    # internal faces
    G = np.einsum("fqis,fsj->fqij", disc.f_C, u[disc.f_st])
    Ff = face_term(disc, G, disc.f_n, disc.f_area, disc.f_qw)
    dPN = disc.cen[disc.f_nei] - disc.cen[disc.f_own]
    a = disc.alpha * kbar / np.abs(np.sum(dPN * disc.f_n, axis=1))
    uP = extrapolate(disc, u, disc.f_own, disc.f_x - disc.cen[disc.f_own])
    uN = extrapolate(disc, u, disc.f_nei, disc.f_x - disc.cen[disc.f_nei])
    Ff = Ff + (a[:, None] * (uN - uP)) * disc.f_area[:, None]
    # displacement faces
    Fd = np.zeros((disc.d_own.size, disc.dim), dtype=Ff.dtype)
    if disc.d_own.size:
        ubq = load * disc.d_ubq
        G = (np.einsum("fqis,fsj->fqij", disc.d_C, u[disc.d_st])
             + np.einsum("fqi,fqj->fqij", disc.d_Cg, ubq))
        Fd = face_term(disc, G, disc.d_n, disc.d_area, disc.d_qw)
        dPb = disc.d_x - disc.cen[disc.d_own]
        ab = disc.alpha * kbar / np.abs(np.sum(dPb * disc.d_n, axis=1))
        uP = extrapolate(disc, u, disc.d_own, dPb)
        Fd = Fd + (ab[:, None] * (load * disc.d_ubc - uP)) * disc.d_area[:, None]
    return Ff, Fd


def symmetry_fluxes(disc, u):
    """Face terms of the symmetry faces (owner side), (n_s, D)."""
    if disc.s_own is None:
        return np.zeros((0, disc.dim))
    ug = u[disc.s_st]
    n = disc.s_n
    Ru = ug - 2.0 * np.einsum("fsd,fd->fs", ug, n)[..., None] * n[:, None, :]
    G = np.einsum("fqis,fsj->fqij", disc.s_C, ug) + np.einsum("fqis,fsj->fqij", disc.s_Cg, Ru)
    return face_term(disc, G, n, disc.s_area, disc.s_qw)


def residual(disc, u, load=1.0, inertia=None):
    """R(u), (n_c, D).  u is (n_c, D) float64 or complex128.

    inertia = (m, s) adds the BDF2 inertia of a time step (App. D, one point
    per cell at the centroid): R_P += s_P - m_P u_P (oracle.dynamics builds m
    and s from rho, dt and the history)."""
    u = np.asarray(u)
    Ff, Fd = face_fluxes(disc, u, load)
    R = np.zeros((disc.n_cells, disc.dim), dtype=np.result_type(u.dtype, np.float64))
    np.add.at(R, disc.f_own, Ff)
    np.add.at(R, disc.f_nei, -Ff)
    np.add.at(R, disc.d_own, Fd)
    if disc.s_own is not None:
        np.add.at(R, disc.s_own, symmetry_fluxes(disc, u))
    R += load * (disc.b_body + disc.b_trac)
    if inertia is not None:
        m, s = inertia
        R += s - m[:, None] * u
    return R
