"""Seeded structured mesh generators (inputs only, no discretisation arithmetic).

Both the CPU oracle and the GPU library consume the arrays made here.  A mesh
is a vertex array ``verts`` (n_verts, dim) float64 and a connectivity array
``cells`` (n_cells, 4 | 8) int64 in VTK order:

* 2D quad:  0 (x0,y0), 1 (x1,y0), 2 (x1,y1), 3 (x0,y1)  -- counter-clockwise.
* 3D hex:   0..3 as the quad on the bottom z-plane, 4..7 the same on the top.
* 3D tet:   (n_cells, 4), positively oriented ((x1-x0) x (x2-x0) . (x3-x0) > 0).
* 2D tri:   (n_cells, 3), counter-clockwise.

Cells and vertices are numbered lexicographically with i (x) fastest.

Perturbation (the "randomly perturbed by up to +-20 % of spacing" meshes): every
interior vertex, every axis, gets an independent uniform offset in
[-a*h_axis, +a*h_axis] drawn from ``numpy.random.default_rng(seed)`` in vertex
order (i fastest), axis-minor.  Boundary vertices are not moved, so the domain
stays an exact box.  ``mode="tensor"`` instead perturbs the 1D grid lines of
each axis (faces stay planar).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Mesh:
    dim: int
    verts: np.ndarray  # (n_verts, dim) float64
    cells: np.ndarray  # (n_cells, 2**dim) int64, VTK order
    shape: tuple       # cells per axis
    lengths: tuple     # box edge lengths
    origin: tuple

    @property
    def n_cells(self) -> int:
        return int(self.cells.shape[0])

    @property
    def n_verts(self) -> int:
        return int(self.verts.shape[0])

    def spacing(self) -> np.ndarray:
        return np.asarray(self.lengths, float) / np.asarray(self.shape, float)


def _grid_lines(n: int, length: float, origin: float) -> np.ndarray:
    return origin + length * np.arange(n + 1, dtype=np.float64) / n


def box_mesh(shape, lengths=None, origin=None, perturb: float = 0.0,
             seed: int = 0, mode: str = "random") -> Mesh:
    """Structured quad (len(shape)==2) or hex (len(shape)==3) mesh of a box.

    ``perturb`` is the maximum vertex offset as a fraction of the local cell
    spacing along each axis; ``mode`` is "random" (per interior vertex) or
    "tensor" (per interior grid line, keeps faces planar).
    """
    shape = tuple(int(s) for s in shape)
    dim = len(shape)
    if dim not in (2, 3):
        raise ValueError("shape must have 2 or 3 entries")
    lengths = tuple(float(v) for v in (lengths or (1.0,) * dim))
    origin = tuple(float(v) for v in (origin or (0.0,) * dim))
    h = np.asarray(lengths) / np.asarray(shape)

    lines = [_grid_lines(shape[a], lengths[a], origin[a]) for a in range(dim)]
    if perturb and mode == "tensor":
        rng = np.random.default_rng(seed)
        for a in range(dim):
            off = rng.uniform(-perturb * h[a], perturb * h[a], size=shape[a] + 1)
            off[0] = off[-1] = 0.0
            lines[a] = lines[a] + off

    nv = [s + 1 for s in shape]
    if dim == 2:
        X, Y = np.meshgrid(lines[0], lines[1], indexing="xy")  # (ny+1, nx+1)
        verts = np.stack([X.ravel(), Y.ravel()], axis=1)
    else:
        Z, Y, X = np.meshgrid(lines[2], lines[1], lines[0], indexing="ij")
        verts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    verts = np.ascontiguousarray(verts, dtype=np.float64)

    if perturb and mode == "random":
        rng = np.random.default_rng(seed)
        off = rng.uniform(-1.0, 1.0, size=verts.shape) * (perturb * h)[None, :]
        idx = np.indices(nv[::-1]).reshape(dim, -1)[::-1].T  # (n_verts, dim): i, j[, k]
        interior = np.all((idx > 0) & (idx < np.asarray(shape)[None, :]), axis=1)
        verts[interior] += off[interior]
    elif perturb and mode != "tensor":
        raise ValueError("mode must be 'random' or 'tensor'")

    def vid(i, j, k=0):
        return (k * nv[1] + j) * nv[0] + i

    if dim == 2:
        j, i = np.meshgrid(np.arange(shape[1]), np.arange(shape[0]), indexing="ij")
        i = i.ravel(); j = j.ravel()
        cells = np.stack([vid(i, j), vid(i + 1, j), vid(i + 1, j + 1), vid(i, j + 1)], axis=1)
    else:
        k, j, i = np.meshgrid(np.arange(shape[2]), np.arange(shape[1]), np.arange(shape[0]), indexing="ij")
        i = i.ravel(); j = j.ravel(); k = k.ravel()
        cells = np.stack([vid(i, j, k), vid(i + 1, j, k), vid(i + 1, j + 1, k), vid(i, j + 1, k),
                          vid(i, j, k + 1), vid(i + 1, j, k + 1), vid(i + 1, j + 1, k + 1), vid(i, j + 1, k + 1)], axis=1)
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    return Mesh(dim, verts, cells, shape, lengths, origin)


# Kuhn split of a hex (VTK numbering) into six tetrahedra along its 0-6
# diagonal: one per ordering of the axes, the path 0 -> ... -> 6 stepping one
# axis at a time.  Every hex of a structured grid splits the same way, so the
# triangles of neighbouring hexes match.
_KUHN = np.array([[0, 1, 2, 6], [0, 1, 5, 6], [0, 3, 2, 6], [0, 3, 7, 6], [0, 4, 5, 6], [0, 4, 7, 6]])


def tet_mesh(shape, lengths=None, origin=None, perturb: float = 0.0, seed: int = 0,
             mode: str = "random") -> Mesh:
    """Tetrahedral mesh of a box: the structured hex mesh of ``box_mesh`` (same
    vertices and perturbation) with every hex split into six tetrahedra, each
    ordered for positive volume.  ``shape`` stays the hex grid's."""
    hx = box_mesh(shape, lengths, origin, perturb, seed, mode)
    if hx.dim != 3:
        raise ValueError("tetrahedral meshes are 3D")
    cells = hx.cells[:, _KUHN].reshape(-1, 4)
    X = hx.verts[cells]
    det = np.einsum("cd,cd->c", np.cross(X[:, 1] - X[:, 0], X[:, 2] - X[:, 0]), X[:, 3] - X[:, 0])
    neg = det < 0
    cells[neg] = cells[neg][:, [0, 2, 1, 3]]
    return Mesh(3, hx.verts, np.ascontiguousarray(cells, np.int64), hx.shape, hx.lengths, hx.origin)


def tri_mesh(shape, lengths=None, origin=None, perturb: float = 0.0, seed: int = 0,
             mode: str = "random") -> Mesh:
    """Triangular mesh of a rectangle: the structured quad mesh of ``box_mesh``
    (same vertices and perturbation) with every quad split along its 0-2
    diagonal, each triangle ordered counter-clockwise."""
    q = box_mesh(shape, lengths, origin, perturb, seed, mode)
    if q.dim != 2:
        raise ValueError("triangular meshes are 2D")
    cells = q.cells[:, [[0, 1, 2], [0, 2, 3]]].reshape(-1, 3)
    X = q.verts[cells]
    e1, e2 = X[:, 1] - X[:, 0], X[:, 2] - X[:, 0]
    neg = e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0] < 0
    cells[neg] = cells[neg][:, [0, 2, 1]]
    return Mesh(2, q.verts, np.ascontiguousarray(cells, np.int64), q.shape, q.lengths, q.origin)


def cell_ijk(mesh: Mesh) -> np.ndarray:
    """Structured (i, j[, k]) index of every cell, (n_cells, dim)."""
    return np.indices(mesh.shape[::-1]).reshape(mesh.dim, -1)[::-1].T.copy()


# ---- face-list (polygonal / polyhedral) meshes --------------------------------

@dataclass
class PolyMesh:
    """A mesh given by its faces: face f has the vertex loop
    face_verts[face_ptr[f]:face_ptr[f + 1]] (2 vertices in 2D) whose right-hand
    normal points out of cell face_cells[f, 0] and into face_cells[f, 1]
    (-1 on the boundary).  Cells are the regions the faces enclose."""
    dim: int
    verts: np.ndarray       # (n_verts, dim)
    face_ptr: np.ndarray    # (n_faces + 1,) int64
    face_verts: np.ndarray  # int64
    face_cells: np.ndarray  # (n_faces, 2) int64
    n_cells_: int
    shape: tuple            # cells per axis of the fine grid it was made from
    lengths: tuple
    origin: tuple
    fine_cell_of: np.ndarray  # (n_fine_cells,) the polyhedral cell holding each fine cell

    @property
    def n_cells(self) -> int:
        return int(self.n_cells_)

    @property
    def n_verts(self) -> int:
        return int(self.verts.shape[0])

    @property
    def n_faces(self) -> int:
        return int(self.face_cells.shape[0])

    def spacing(self) -> np.ndarray:
        return np.asarray(self.lengths, float) / np.asarray(self.shape, float)


# outward vertex loops of the faces of a VTK quad / hexahedron
_QUAD_EDGES = np.array([[3, 0], [1, 2], [0, 1], [2, 3]])
_HEX_LOOPS = np.array([[0, 4, 7, 3], [1, 2, 6, 5], [0, 1, 5, 4], [3, 7, 6, 2], [0, 3, 2, 1], [4, 5, 6, 7]])


def split_block_mesh(coarse_shape, lengths=None, origin=None, perturb: float = 0.0, seed: int = 0,
                     mode: str = "random") -> PolyMesh:
    """A polygonal (2D) or polyhedral (3D) mesh with hanging vertices: the
    structured mesh of ``box_mesh`` with twice as many cells per axis (same
    perturbation rules) in which the 2^dim fine cells of every coarse block
    (I, J[, K]) with I + J (+ K) even are merged into one cell.  A merged cell
    keeps the fine faces on its block's boundary, so it has 8 edges (2D) or 24
    quadrilateral faces (3D), each shared with one fine neighbour; the other
    cells are the fine quads or hexahedra.  Cells are numbered in the order
    their first fine cell appears (lexicographic, i fastest)."""
    cs = tuple(int(s) for s in coarse_shape)
    dim = len(cs)
    fine = box_mesh(tuple(2 * s for s in cs), lengths, origin, perturb, seed, mode)
    ijk = cell_ijk(fine)
    blk = ijk // 2
    merged = blk.sum(axis=1) % 2 == 0
    bid = np.ravel_multi_index(tuple(blk[:, a] for a in range(dim)[::-1]), cs[::-1])
    cell_of = np.full(fine.n_cells, -1, np.int64)
    block_cell = {}
    nxt = 0
    for f in range(fine.n_cells):
        if merged[f]:
            b = int(bid[f])
            if b not in block_cell:
                block_cell[b] = nxt
                nxt += 1
            cell_of[f] = block_cell[b]
        else:
            cell_of[f] = nxt
            nxt += 1
    loops = _QUAD_EDGES if dim == 2 else _HEX_LOOPS
    nl = loops.shape[0]
    fv = fine.cells[:, loops]                       # (n_fine, nl, nvf)
    flat = fv.reshape(fine.n_cells * nl, -1)
    keys = np.sort(flat, axis=1)
    _, inv, counts = np.unique(keys, axis=0, return_inverse=True, return_counts=True)
    inv = inv.ravel()
    first = np.full(counts.size, -1, np.int64)
    second = np.full(counts.size, -1, np.int64)
    for r in range(flat.shape[0]):
        u = inv[r]
        if first[u] < 0:
            first[u] = r
        else:
            second[u] = r
    c0 = cell_of[first // nl]
    c1 = np.where(second >= 0, cell_of[np.maximum(second, 0) // nl], -1)
    keep = c0 != c1  # faces inside a merged block disappear
    first, c0, c1 = first[keep], c0[keep], c1[keep]
    order = np.lexsort((c1, c0))
    first, c0, c1 = first[order], c0[order], c1[order]
    nvf = flat.shape[1]
    face_verts = flat[first].reshape(-1)
    face_ptr = np.arange(first.size + 1, dtype=np.int64) * nvf
    return PolyMesh(dim, fine.verts, face_ptr, np.ascontiguousarray(face_verts, np.int64),
                    np.ascontiguousarray(np.stack([c0, c1], axis=1), np.int64), nxt, fine.shape,
                    fine.lengths, fine.origin, cell_of)


_TRI_EDGES = np.array([[0, 1], [1, 2], [2, 0]])
_TET_FACES = np.array([[0, 2, 1], [0, 1, 3], [1, 2, 3], [0, 3, 2]])


def face_list_mesh(mesh: Mesh) -> PolyMesh:
    """The same cells (triangles, quads, tetrahedra or hexahedra, cell i stays
    cell i) given as a face list.  Each face's loop is turned, where needed,
    so that its right-hand normal points away from its first cell's vertex
    mean; faces are listed by (first cell, second cell)."""
    dim, nv = mesh.dim, mesh.cells.shape[1]
    loops = {(2, 3): _TRI_EDGES, (2, 4): _QUAD_EDGES, (3, 4): _TET_FACES, (3, 8): _HEX_LOOPS}[(dim, nv)]
    nl = loops.shape[0]
    flat = mesh.cells[:, loops].reshape(mesh.n_cells * nl, -1).copy()
    owner = np.repeat(np.arange(mesh.n_cells), nl)
    X = mesh.verts[flat]
    if dim == 2:
        d = X[:, 1] - X[:, 0]
        normal = np.stack([d[:, 1], -d[:, 0]], axis=1)
    else:
        normal = np.cross(X[:, 1] - X[:, 0], X[:, 2] - X[:, 0])
    away = X.mean(axis=1) - mesh.verts[mesh.cells].mean(axis=1)[owner]
    turn = np.einsum("fd,fd->f", normal, away) < 0
    flat[turn] = flat[turn][:, ::-1]
    keys = np.sort(flat, axis=1)
    _, inv, counts = np.unique(keys, axis=0, return_inverse=True, return_counts=True)
    inv = inv.ravel()
    first = np.full(counts.size, -1, np.int64)
    second = np.full(counts.size, -1, np.int64)
    for r in range(flat.shape[0]):
        if first[inv[r]] < 0:
            first[inv[r]] = r
        else:
            second[inv[r]] = r
    c0 = owner[first]
    c1 = np.where(second >= 0, owner[np.maximum(second, 0)], -1)
    order = np.lexsort((c1, c0))
    first, c0, c1 = first[order], c0[order], c1[order]
    nvf = flat.shape[1]
    return PolyMesh(dim, mesh.verts, np.arange(first.size + 1, dtype=np.int64) * nvf,
                    np.ascontiguousarray(flat[first].reshape(-1), np.int64),
                    np.ascontiguousarray(np.stack([c0, c1], axis=1), np.int64), mesh.n_cells, mesh.shape,
                    mesh.lengths, mesh.origin, np.arange(mesh.n_cells))


def merged_block_mesh(mesh: Mesh, lo, hi) -> PolyMesh:
    """The face list of a structured mesh with the cells whose (i, j[, k]) lie
    in [lo, hi) merged into one cell (the faces inside the block dropped): a
    3 x 3 x 3 block gives a cell of 54 faces, a 5 x 5 block one of 20 edges.
    The merged cell takes the number of the block's first cell."""
    pm = face_list_mesh(mesh)
    ijk = cell_ijk(mesh)
    inside = np.all((ijk >= np.asarray(lo)) & (ijk < np.asarray(hi)), axis=1)
    first = int(np.nonzero(inside)[0][0])
    new = np.full(mesh.n_cells, -1, np.int64)
    nxt = 0
    for P in range(mesh.n_cells):
        if inside[P] and P != first:
            continue
        new[P] = nxt
        nxt += 1
    new[inside] = new[first]
    fc = np.where(pm.face_cells >= 0, new[np.maximum(pm.face_cells, 0)], -1)
    keep = fc[:, 0] != fc[:, 1]
    loops = np.split(pm.face_verts, pm.face_ptr[1:-1])
    kept = [loops[f] for f in np.nonzero(keep)[0]]
    ptr = np.concatenate([[0], np.cumsum([v.size for v in kept])]).astype(np.int64)
    return PolyMesh(mesh.dim, mesh.verts, ptr, np.concatenate(kept).astype(np.int64),
                    np.ascontiguousarray(fc[keep]), nxt, mesh.shape, mesh.lengths, mesh.origin, new)
