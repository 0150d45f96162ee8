"""Mesh geometry for straight-edged quads and triangles (2D), trilinear
hexahedra and tetrahedra (3D).

Test infrastructure (see package docstring).  Follows Sec. 3.1 of the paper
("Solution Domain Discretisation"): cell centroid x_P and volume Omega_P, face
centre x_f, unit normal n_f (outward from the owner P), area Gamma_f, and
quadrature points x_{f,q} with weights alpha_q summing to one.

Readings where the paper is silent for these element shapes:

* Cells are handled through their (bi/tri)linear isoparametric map; Omega_P and
  x_P are integrated exactly with 2 Gauss-Legendre points per direction.
* A 3D face is the bilinear surface through its four vertices.  Its single
  normal and area come from the exact vector area S_f = 1/2 (x2-x0) x (x3-x1):
  Gamma_f = |S_f|, n_f = S_f / Gamma_f.  Quadrature points are the n_g x n_g
  Gauss-Legendre points of the bilinear map, alpha_q proportional to
  w_i w_j |x_s x x_t| and normalised to sum 1.
* 2D faces are edges with n_g Gauss-Legendre points, alpha_q = w_q / 2.
* The face centre is x_f = sum_q alpha_q x_{f,q}.
* The body-force volume quadrature uses (p+2)^D Gauss-Legendre points of the
  cell map with weights w detJ (so that sum_q beta_q Omega_P = sum_q w_q detJ_q).
* Tetrahedra (the paper's tetrahedral meshes; its symmetric Dunavant and
  Shunn-Ham rules are not reproduced): a tetrahedron is flat-faced, Omega_P is
  its determinant / 6 and x_P the mean of its vertices.  A triangle face with
  vertices x0, x1, x2 is integrated through the collapsed map
  x0 + a (x1 - x0 + b (x2 - x1)), whose area element is 2 Gamma a: n_g
  Gauss-Jacobi points of weight a times n_g Gauss-Legendre points in b.  The
  cell map x0 + a (x1 - x0 + b (x2 - x1 + c (x3 - x2))) has detJ = 6 Omega a^2 b:
  Gauss-Jacobi points of weights a^2 and b, Gauss-Legendre in c, p + 2 each.
  With n points per direction these conical products are exact for total
  degree 2n - 1.
* Fan rule for quadrilateral faces (Sec. 3.1 subdivides polygonal faces by
  fan triangulation): the fan starts at the face's lowest-numbered vertex y0,
  keeping the cyclic order, giving triangles (y0, y1, y2) and (y0, y2, y3);
  each gets the triangle rule above, its weights scaled by its area over the
  sum of both areas (the paper's consistent face area).  The face's area and
  normal still come from its vector area.
* Triangles (2D): Omega_P = det / 2, x_P the vertex mean, and the cell rule
  through x0 + a (x1 - x0 + b (x2 - x1)) (detJ = 2 Omega a): Gauss-Jacobi in a,
  Gauss-Legendre in b.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from scipy.special import roots_jacobi

# local faces, vertex order giving the outward normal of the cell
QUAD_FACES = np.array([[3, 0], [1, 2], [0, 1], [2, 3]])
HEX_FACES = np.array([[0, 4, 7, 3], [1, 2, 6, 5], [0, 1, 5, 4], [3, 7, 6, 2],
                      [0, 3, 2, 1], [4, 5, 6, 7]])
QUAD_REF = np.array([[0, 0], [1, 0], [1, 1], [0, 1]], float)
# the face opposite each vertex, ordered for the outward normal of a tetrahedron
# with (x1 - x0) x (x2 - x0) . (x3 - x0) > 0
TET_FACES = np.array([[1, 2, 3], [0, 3, 2], [0, 1, 3], [0, 2, 1]])
# edges of a counter-clockwise triangle, opposite vertices 2, 0, 1
TRI_FACES = np.array([[0, 1], [1, 2], [2, 0]])
HEX_REF = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0],
                    [0, 0, 1], [1, 0, 1], [1, 1, 1], [0, 1, 1]], float)


def gauss_01(n: int):
    """n-point Gauss-Legendre rule mapped to [0, 1] (weights sum to 1)."""
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def jacobi_01(n: int, beta: int):
    """n-point Gauss rule for the weight u^beta on [0, 1] (weights sum to
    1 / (beta + 1)), from scipy's Gauss-Jacobi rule on [-1, 1], u = (1 + x) / 2."""
    x, w = roots_jacobi(n, 0.0, float(beta))
    return 0.5 * (x + 1.0), w / 2.0 ** (beta + 1)


def is_tet(X: np.ndarray) -> bool:
    return X.shape[-1] == 3 and X.shape[-2] == 4


def is_tri(X: np.ndarray) -> bool:
    return X.shape[-1] == 2 and X.shape[-2] == 3


def tri_quadrature(X: np.ndarray, n: int):
    """Conical-product rule on triangles X (n_c, 3, 2): points (n_c, n^2, 2),
    weights (n_c, n^2) integrating over the physical cell."""
    a, wa = jacobi_01(n, 1)
    b, wb = gauss_01(n)
    A, B = (g.ravel() for g in np.meshgrid(a, b, indexing="ij"))
    W = np.outer(wa, wb).ravel()
    x0, x1, x2 = X[:, 0], X[:, 1], X[:, 2]
    pts = x0[:, None] + A[None, :, None] * ((x1 - x0)[:, None] + B[None, :, None] * (x2 - x1)[:, None])
    e1, e2 = x1 - x0, x2 - x0
    det = e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0]
    return pts, W[None, :] * det[:, None]


def tet_quadrature(X: np.ndarray, n: int):
    """Conical-product rule on tetrahedra X (n_c, 4, 3): points (n_c, n^3, 3),
    weights (n_c, n^3) integrating over the physical cell."""
    a, wa = jacobi_01(n, 2)
    b, wb = jacobi_01(n, 1)
    c, wc = gauss_01(n)
    A, B, Cc = (g.ravel() for g in np.meshgrid(a, b, c, indexing="ij"))
    W = np.einsum("i,j,k->ijk", wa, wb, wc).ravel()
    x0, x1, x2, x3 = X[:, 0], X[:, 1], X[:, 2], X[:, 3]
    pts = x0[:, None] + A[None, :, None] * ((x1 - x0)[:, None] + B[None, :, None]
                                            * ((x2 - x1)[:, None] + Cc[None, :, None] * (x3 - x2)[:, None]))
    det = np.einsum("cd,cd->c", np.cross(x1 - x0, x2 - x0), x3 - x0)
    return pts, W[None, :] * det[:, None]


def shape_functions(ref: np.ndarray, xi: np.ndarray):
    """(Bi/tri)linear shape functions N_a(xi) and dN_a/dxi_j at points xi (m, D)."""
    m, D = xi.shape
    na = ref.shape[0]
    N = np.ones((m, na))
    dN = np.ones((m, na, D))
    for a in range(na):
        for d in range(D):
            f = xi[:, d] if ref[a, d] else 1.0 - xi[:, d]
            df = 1.0 if ref[a, d] else -1.0
            N[:, a] *= f
            for j in range(D):
                dN[:, a, j] *= df if j == d else f
    return N, dN


def cell_quadrature(X: np.ndarray, n: int):
    """Tensor Gauss-Legendre quadrature of the cell map.

    X: (n_c, 2^D, D) vertex coordinates.  Returns points (n_c, n^D, D) and
    weights w * detJ (n_c, n^D), which integrate over the physical cell.
    """
    if is_tet(X):
        return tet_quadrature(X, n)
    if is_tri(X):
        return tri_quadrature(X, n)
    D = X.shape[2]
    ref = QUAD_REF if D == 2 else HEX_REF
    t, w = gauss_01(n)
    grids = np.meshgrid(*([t] * D), indexing="ij")
    wgrid = np.meshgrid(*([w] * D), indexing="ij")
    xi = np.stack([g.ravel() for g in grids], axis=1)
    wq = np.prod(np.stack([g.ravel() for g in wgrid], axis=1), axis=1)
    N, dN = shape_functions(ref, xi)
    pts = np.einsum("qa,cad->cqd", N, X)
    J = np.einsum("qaj,cai->cqij", dN, X)  # dx_i / dxi_j
    detJ = np.linalg.det(J)
    return pts, wq[None, :] * detJ


def cell_volume_centroid(X: np.ndarray):
    if is_tet(X):
        det = np.einsum("cd,cd->c", np.cross(X[:, 1] - X[:, 0], X[:, 2] - X[:, 0]), X[:, 3] - X[:, 0])
        return det / 6.0, X.mean(axis=1)
    if is_tri(X):
        e1, e2 = X[:, 1] - X[:, 0], X[:, 2] - X[:, 0]
        return 0.5 * (e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0]), X.mean(axis=1)
    pts, W = cell_quadrature(X, 2)
    vol = W.sum(axis=1)
    cen = np.einsum("cq,cqd->cd", W, pts) / vol[:, None]
    return vol, cen


@dataclass
class Faces:
    """All faces of a mesh.  Internal faces have neigh >= 0, boundary faces -1."""
    owner: np.ndarray   # (n_f,)
    neigh: np.ndarray   # (n_f,)
    verts: np.ndarray   # (n_f, 2|4) vertex ids in the owner's outward order
    owner_slot: np.ndarray  # local face index in the owner cell
    neigh_slot: np.ndarray  # local face index in the neighbour cell (-1 boundary)


def enumerate_faces(cells: np.ndarray, dim: int) -> Faces:
    """Match local faces of all cells by their (sorted) vertex sets.

    The owner is the lower cell id (its copy appears first), the neighbour the
    other one; a face seen once is a boundary face.
    """
    if cells.shape[1] == dim + 1:
        lf = TRI_FACES if dim == 2 else TET_FACES
    else:
        lf = QUAD_FACES if dim == 2 else HEX_FACES
    nlf = lf.shape[0]
    n_c = cells.shape[0]
    fv = cells[:, lf]                      # (n_c, nlf, nv)
    flat = fv.reshape(n_c * nlf, -1)
    keys = np.sort(flat, axis=1)
    uniq, inv, counts = np.unique(keys, axis=0, return_inverse=True, return_counts=True)
    inv = inv.ravel()
    if np.any(counts > 2):
        raise ValueError("non-manifold mesh: a face is shared by more than two cells")
    n_f = uniq.shape[0]
    rows = np.arange(n_c * nlf)
    first = np.full(n_f, -1, np.int64)
    second = np.full(n_f, -1, np.int64)
    for r in rows:  # rows are in increasing cell order
        f = inv[r]
        if first[f] < 0:
            first[f] = r
        else:
            second[f] = r
    owner = first // nlf
    neigh = np.where(second >= 0, second // nlf, -1)
    return Faces(owner=owner, neigh=neigh, verts=flat[first],
                 owner_slot=first % nlf, neigh_slot=np.where(second >= 0, second % nlf, -1))


@dataclass
class FaceGeom:
    centre: np.ndarray  # (n_f, D)
    normal: np.ndarray  # (n_f, D) unit, outward from owner
    area: np.ndarray    # (n_f,)
    qpts: np.ndarray    # (n_f, Nq, D)
    qw: np.ndarray      # (n_f, Nq), sums to 1


def _triangle_points(x0, x1, x2, n):
    """Conical-product points (n_f, n^2, 3) and weights summing to 1."""
    a, wa = jacobi_01(n, 1)
    t, w = gauss_01(n)
    A, B = (g.ravel() for g in np.meshgrid(a, t, indexing="ij"))
    pts = x0[:, None] + A[None, :, None] * ((x1 - x0)[:, None] + B[None, :, None] * (x2 - x1)[:, None])
    return pts, 2.0 * np.outer(wa, w).ravel()


def face_geometry(verts: np.ndarray, fverts: np.ndarray, n_gauss: int, fan: bool = False) -> FaceGeom:
    """Geometry and quadrature of faces given their ordered vertex ids."""
    P = verts[fverts]  # (n_f, nv, D)
    t, w = gauss_01(n_gauss)
    if P.shape[1] == 2:
        a, b = P[:, 0], P[:, 1]
        e = b - a
        area = np.sqrt(np.sum(e * e, axis=1))
        normal = np.stack([e[:, 1], -e[:, 0]], axis=1) / area[:, None]
        qpts = a[:, None, :] + t[None, :, None] * e[:, None, :]
        qw = np.broadcast_to(w, (P.shape[0], w.size)).copy()
    elif P.shape[1] == 3:
        x0, x1, x2 = P[:, 0], P[:, 1], P[:, 2]
        S = 0.5 * np.cross(x1 - x0, x2 - x0)
        area = np.sqrt(np.sum(S * S, axis=1))
        normal = S / area[:, None]
        qpts, wt = _triangle_points(x0, x1, x2, n_gauss)
        qw = np.broadcast_to(wt, (P.shape[0], wt.size)).copy()
    elif fan:
        x0, x1, x2, x3 = P[:, 0], P[:, 1], P[:, 2], P[:, 3]
        S = 0.5 * np.cross(x2 - x0, x3 - x1)
        area = np.sqrt(np.sum(S * S, axis=1))
        normal = S / area[:, None]
        m = np.argmin(fverts, axis=1)
        Y = np.stack([P[np.arange(P.shape[0]), (m + k) % 4] for k in range(4)], axis=1)
        parts, wts = [], []
        tri_area = [0.5 * np.linalg.norm(np.cross(Y[:, b] - Y[:, 0], Y[:, c] - Y[:, 0]), axis=1)
                    for b, c in ((1, 2), (2, 3))]
        for (b, c), At in zip(((1, 2), (2, 3)), tri_area):
            pts, wt = _triangle_points(Y[:, 0], Y[:, b], Y[:, c], n_gauss)
            parts.append(pts)
            wts.append(wt[None, :] * (At / (tri_area[0] + tri_area[1]))[:, None])
        qpts = np.concatenate(parts, axis=1)
        qw = np.concatenate(wts, axis=1)
        # Sec. 3.1: the face area is the sum of the sub-triangle areas (the
        # normal stays the vector area's direction, one per face)
        area = tri_area[0] + tri_area[1]
    else:
        x0, x1, x2, x3 = P[:, 0], P[:, 1], P[:, 2], P[:, 3]
        S = 0.5 * np.cross(x2 - x0, x3 - x1)
        area = np.sqrt(np.sum(S * S, axis=1))
        normal = S / area[:, None]
        s, tt = np.meshgrid(t, t, indexing="ij")
        ws, wt = np.meshgrid(w, w, indexing="ij")
        s = s.ravel(); tt = tt.ravel(); wq = (ws * wt).ravel()
        qpts = ((1 - s)[None, :, None] * (1 - tt)[None, :, None] * x0[:, None]
                + s[None, :, None] * (1 - tt)[None, :, None] * x1[:, None]
                + s[None, :, None] * tt[None, :, None] * x2[:, None]
                + (1 - s)[None, :, None] * tt[None, :, None] * x3[:, None])
        xs = (1 - tt)[None, :, None] * (x1 - x0)[:, None] + tt[None, :, None] * (x2 - x3)[:, None]
        xt = (1 - s)[None, :, None] * (x3 - x0)[:, None] + s[None, :, None] * (x2 - x1)[:, None]
        jac = np.sqrt(np.sum(np.cross(xs, xt) ** 2, axis=2))
        qw = wq[None, :] * jac
        qw = qw / qw.sum(axis=1, keepdims=True)
    centre = np.einsum("fq,fqd->fd", qw, qpts)
    return FaceGeom(centre, normal, area, qpts, qw)


# ---- face-list (polygonal / polyhedral) meshes (Sec. 3.1) --------------------
#
# Readings: a polygonal face of m vertices is cut into m - 2 triangles by a fan
# from its lowest-numbered vertex (cyclic order kept), each with the triangle
# rule above and weights scaled by its area over the sum of the areas; Gamma_f
# is that sum and n_f the direction of the face's vector area
# 1/2 sum_k x_k x x_{k+1}.  Faces with fewer points than the mesh's largest
# count are padded with zero-weight points at their centre.  A cell is cut
# into tetrahedra (triangles in 2D) joining the mean of its vertices to the
# fan triangles (edges) of its faces, oriented outward; Omega_P and x_P are
# their summed volumes and volume-weighted centroids, and the body force is
# integrated by the conical-product rule with p + 2 points per direction on
# each of them.


def poly_faces(mesh):
    """Owner (lower cell id) and neighbour of every face of a face-list mesh,
    and its vertex loop oriented outward from the owner."""
    fc = np.asarray(mesh.face_cells)
    c0, c1 = fc[:, 0], fc[:, 1]
    flip = (c1 >= 0) & (c1 < c0)
    owner = np.where(flip, c1, c0)
    neigh = np.where(flip, c0, c1)
    ptr = np.asarray(mesh.face_ptr)
    loops = []
    for f in range(fc.shape[0]):
        L = np.asarray(mesh.face_verts[ptr[f]:ptr[f + 1]], np.int64)
        loops.append(L[::-1].copy() if flip[f] else L)
    return owner, neigh, loops


def _fan(L):
    """Fan triangles (vertex ids) of the loop L from its lowest vertex."""
    m = len(L)
    s = int(np.argmin(L))
    Y = [L[(s + k) % m] for k in range(m)]
    return [(Y[0], Y[k], Y[k + 1]) for k in range(1, m - 1)]


def polygon_face_geometry(verts, loops, n_gauss):
    """FaceGeom of the faces given by vertex loops (2D: edges)."""
    D = verts.shape[1]
    if D == 2:
        return face_geometry(verts, np.asarray(loops, np.int64), n_gauss)
    nf = len(loops)
    nq = max(len(L) - 2 for L in loops) * n_gauss * n_gauss
    centre = np.zeros((nf, 3))
    normal = np.zeros((nf, 3))
    area = np.zeros(nf)
    qpts = np.zeros((nf, nq, 3))
    qw = np.zeros((nf, nq))
    for f, L in enumerate(loops):
        P = verts[L]
        S = 0.5 * np.sum(np.cross(P, np.roll(P, -1, axis=0)), axis=0)
        normal[f] = S / np.linalg.norm(S)
        tris = _fan(L)
        At = np.array([0.5 * np.linalg.norm(np.cross(verts[b] - verts[a], verts[c] - verts[a])) for a, b, c in tris])
        pts, wts = [], []
        for (a, b, c), A in zip(tris, At):
            x, wt = _triangle_points(verts[a][None], verts[b][None], verts[c][None], n_gauss)
            pts.append(x[0])
            wts.append(wt * A / At.sum())
        x = np.concatenate(pts)
        wq = np.concatenate(wts)
        area[f] = At.sum()
        centre[f] = wq @ x
        qpts[f, :x.shape[0]] = x
        qpts[f, x.shape[0]:] = centre[f]
        qw[f, :x.shape[0]] = wq
    return FaceGeom(centre, normal, area, qpts, qw)


def poly_cells(mesh, owner, neigh, loops, n_vol):
    """Volumes, centroids and body-force quadrature (points, weights, cell of
    each point) of the cells of a face-list mesh; n_vol points per direction
    on each sub-simplex."""
    D = mesh.dim
    n_c = mesh.n_cells
    vsum = np.zeros((n_c, D))
    vcnt = np.zeros(n_c)
    cell_verts = [set() for _ in range(n_c)]
    for f, L in enumerate(loops):
        for c in (owner[f], neigh[f]):
            if c >= 0:
                cell_verts[c].update(int(v) for v in L)
    for c in range(n_c):
        ids = np.array(sorted(cell_verts[c]))
        vsum[c] = mesh.verts[ids].sum(axis=0)
        vcnt[c] = ids.size
    apex = vsum / vcnt[:, None]
    simp, cell_of = [], []
    for f, L in enumerate(loops):
        for c, Lc in ((owner[f], L), (neigh[f], L[::-1])):
            if c < 0:
                continue
            if D == 2:
                simp.append(np.stack([apex[c], mesh.verts[Lc[0]], mesh.verts[Lc[1]]]))
                cell_of.append(c)
            else:
                for a, b, cc in _fan(np.asarray(Lc)):
                    simp.append(np.stack([apex[c], mesh.verts[a], mesh.verts[b], mesh.verts[cc]]))
                    cell_of.append(c)
    X = np.array(simp)
    cell_of = np.array(cell_of, np.int64)
    if D == 2:
        e1, e2 = X[:, 1] - X[:, 0], X[:, 2] - X[:, 0]
        vs = 0.5 * (e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0])
        pts, W = tri_quadrature(X, n_vol)
    else:
        vs = np.einsum("cd,cd->c", np.cross(X[:, 1] - X[:, 0], X[:, 2] - X[:, 0]), X[:, 3] - X[:, 0]) / 6.0
        pts, W = tet_quadrature(X, n_vol)
    vol = np.zeros(n_c)
    np.add.at(vol, cell_of, vs)
    mom = np.zeros((n_c, D))
    np.add.at(mom, cell_of, vs[:, None] * X.mean(axis=1))
    cen = mom / vol[:, None]
    nq = pts.shape[1]
    return vol, cen, pts.reshape(-1, D), W.reshape(-1), np.repeat(cell_of, nq)
