"""Named synthetic workloads shaped like the paper's benchmarks (inputs only).

Each builder returns a :class:`Problem`: a seeded mesh, the discretisation
parameters (order p, stencil surplus n+, Gauss points per face direction, alpha,
weight shape k, ghost weight), the material, and the loads as point functions.

* ``square_mms``   - 2D plane-strain manufactured solution on the unit square
                     (32 x 32 quads, p = 2, 2 Gauss points per edge).
* ``cube_mms``     - 3D linear elastic manufactured trigonometric solution on a
                     perturbed hex mesh of the unit cube (64^3, p = 3, 2x2 points).
* ``cantilever``   - 3D neo-Hookean cantilever 200 x 20 x 20 on [0,10]x[0,1]^2,
                     clamped at x = 0, dead tip traction, 10 load increments.
* ``poly_patch``   - any mesh with a random polynomial field of degree <= p and
                     its exact loads (patch tests).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .fields import (Loads, cantilever_loads, lame_from_young, mms_2d_unit, mms_3d_trig, symmetric_poly_field,
                     mms_loads, random_poly_field)
from .meshes import Mesh, box_mesh, split_block_mesh, tet_mesh, tri_mesh

LINEAR_ELASTIC, NEO_HOOKEAN = 0, 1

PAPER_N_PLUS = {2: {1: 10, 2: 10, 3: 10}, 3: {1: 45, 2: 55, 3: 65}}


@dataclass
class Problem:
    name: str
    mesh: Mesh
    p: int
    n_plus: int
    n_gauss: int
    material: int
    mu: float
    lam: float
    loads: Loads
    alpha: float = 0.1
    k_weight: float = 6.0
    ghost_weight: float = 1.0
    stencil_quantum: float = 0.0
    n_increments: int = 1
    face_rule: int = 0  # quad faces: 0 tensor Gauss-Legendre, 1 fan triangulation
    stencil_grow: int = 0  # > 0: grow stencils that fail the pivot test by this many cells at a time
    meta: dict = field(default_factory=dict)

    @property
    def dim(self):
        return self.mesh.dim

    @property
    def stencil_size(self):
        d, p = self.dim, self.p
        nt = (p + 1) * (p + 2) // 2 if d == 2 else (p + 1) * (p + 2) * (p + 3) // 6
        return nt + self.n_plus


def default_gauss(p: int) -> int:
    return 1 if p == 1 else 2


def quantum_for(mesh: Mesh) -> float:
    """Squared-distance quantum used to break stencil ties (1e-6 h_min^2)."""
    return 1e-6 * float(np.min(mesh.spacing())) ** 2


def square_mms(n: int = 32, p: int = 2, perturb: float = 0.0, seed: int = 0,
               E: float = 1.0, nu: float = 0.3, n_plus=None, n_gauss=None) -> Problem:
    mesh = box_mesh((n, n), perturb=perturb, seed=seed)
    mu, lam = lame_from_young(E, nu)
    return Problem(f"square_mms_{n}_p{p}", mesh, p, PAPER_N_PLUS[2][p] if n_plus is None else n_plus,
                   n_gauss or default_gauss(p), LINEAR_ELASTIC, mu, lam,
                   mms_loads(mms_2d_unit(), mu, lam), stencil_quantum=quantum_for(mesh))


def cube_mms(n: int = 64, p: int = 3, perturb: float = 0.2, seed: int = 0,
             E: float = 1.0, nu: float = 0.3, n_plus=None, n_gauss=None, lengths=None,
             mode: str = "random") -> Problem:
    shape = (n, n, n) if np.isscalar(n) else tuple(n)
    mesh = box_mesh(shape, lengths=lengths, perturb=perturb, seed=seed, mode=mode)
    mu, lam = lame_from_young(E, nu)
    return Problem(f"cube_mms_{'x'.join(map(str, shape))}_p{p}", mesh, p,
                   PAPER_N_PLUS[3][p] if n_plus is None else n_plus,
                   n_gauss or default_gauss(p), LINEAR_ELASTIC, mu, lam,
                   mms_loads(mms_3d_trig(), mu, lam), stencil_quantum=quantum_for(mesh))


def tri_mms(n: int = 16, p: int = 2, perturb: float = 0.2, seed: int = 0,
            E: float = 1.0, nu: float = 0.3, n_plus=None, n_gauss=None) -> Problem:
    """The 2D manufactured problem of square_mms on n x n quads of the unit
    square (perturbed as there), each split into two triangles."""
    mesh = tri_mesh((n, n), perturb=perturb, seed=seed)
    mu, lam = lame_from_young(E, nu)
    return Problem(f"tri_mms_{n}_p{p}", mesh, p, PAPER_N_PLUS[2][p] if n_plus is None else n_plus,
                   n_gauss or default_gauss(p), LINEAR_ELASTIC, mu, lam,
                   mms_loads(mms_2d_unit(), mu, lam), stencil_quantum=quantum_for(mesh))


def tet_mms(n: int = 16, p: int = 2, perturb: float = 0.2, seed: int = 0,
            E: float = 1.0, nu: float = 0.3, n_plus=None, n_gauss=None, mode: str = "random") -> Problem:
    """The 3D manufactured problem on a tetrahedral mesh: n^3 hexes of the unit
    cube (perturbed as in cube_mms), each split into six tetrahedra."""
    shape = (n, n, n) if np.isscalar(n) else tuple(n)
    mesh = tet_mesh(shape, perturb=perturb, seed=seed, mode=mode)
    mu, lam = lame_from_young(E, nu)
    return Problem(f"tet_mms_{'x'.join(map(str, shape))}_p{p}", mesh, p,
                   PAPER_N_PLUS[3][p] if n_plus is None else n_plus,
                   n_gauss or default_gauss(p), LINEAR_ELASTIC, mu, lam,
                   mms_loads(mms_3d_trig(), mu, lam), stencil_quantum=quantum_for(mesh))


def split_mms(coarse, p: int = 2, perturb: float = 0.2, seed: int = 0, E: float = 1.0, nu: float = 0.3,
              n_plus=None, n_gauss=None, mode: str = "random") -> Problem:
    """The manufactured problem of square_mms (2D) or cube_mms (3D) on the
    polygonal / polyhedral mesh of split_block_mesh(coarse): every other 2^dim
    block of the doubled grid merged into one 8-edge or 24-face cell."""
    shape = tuple(coarse)
    mesh = split_block_mesh(shape, perturb=perturb, seed=seed, mode=mode)
    D = len(shape)
    mu, lam = lame_from_young(E, nu)
    field = mms_2d_unit() if D == 2 else mms_3d_trig()
    return Problem(f"split_mms_{'x'.join(map(str, shape))}_p{p}", mesh, p,
                   PAPER_N_PLUS[D][p] if n_plus is None else n_plus,
                   n_gauss or default_gauss(p), LINEAR_ELASTIC, mu, lam,
                   mms_loads(field, mu, lam), stencil_quantum=quantum_for(mesh))


def cantilever(shape=(200, 20, 20), p: int = 2, mu: float = 1.0, lam: float = 10.0,
               tip_traction: float = 2.18e-3, n_increments: int = 10, perturb: float = 0.0,
               seed: int = 0, n_plus=None) -> Problem:
    L = 10.0
    mesh = box_mesh(shape, lengths=(L, 1.0, 1.0), perturb=perturb, seed=seed)
    loads = cantilever_loads(L, (0.0, -tip_traction, 0.0))
    return Problem(f"cantilever_{'x'.join(map(str, shape))}_p{p}", mesh, p,
                   PAPER_N_PLUS[3][p] if n_plus is None else n_plus, default_gauss(p),
                   NEO_HOOKEAN, mu, lam, loads, stencil_quantum=quantum_for(mesh),
                   n_increments=n_increments)


def vibrating_column(shape=(50, 5, 5), p: int = 1, E: float = 15.293e6, nu: float = 0.3,
                     rho: float = 1000.0, dt: float = 1e-3) -> Problem:
    """The paper's vibrating 3D column (Sec. 5, case 7): 6 m x 0.2 m x 0.2 m,
    neo-Hookean, clamped at one end, a sudden traction of 50 kPa in each of the
    two transverse directions on the other end, BDF2 with dt = 1 ms.  Laid along
    x here (the paper stands it along z); 1250 cells by default as in the paper.
    rho and dt ride in ``meta``."""
    mu, lam = lame_from_young(E, nu)
    mesh = box_mesh(shape, lengths=(6.0, 0.2, 0.2))
    loads = cantilever_loads(6.0, (0.0, 5e4, 5e4))
    return Problem(f"column_{'x'.join(map(str, shape))}_p{p}", mesh, p, PAPER_N_PLUS[3][p], default_gauss(p),
                   NEO_HOOKEAN, mu, lam, loads, stencil_quantum=quantum_for(mesh), meta={"rho": rho, "dt": dt})


def poly_patch(mesh: Mesh, p: int, degree: int, seed: int = 0, E: float = 1.0, nu: float = 0.3,
               n_plus=None, n_gauss=None, scale: float = 1.0, traction_faces=None,
               symmetric: bool = False) -> Problem:
    """Polynomial manufactured problem; symmetric=True takes a field symmetric
    about x = 0 and makes the mesh's x = 0 faces symmetry planes."""
    mu, lam = lame_from_young(E, nu)
    if symmetric:
        fld = symmetric_poly_field(mesh.dim, degree, seed, scale)
        tol = 1e-9 * float(np.max(mesh.lengths))
        sym = lambda xc, n: np.abs(xc[:, 0] - mesh.origin[0]) < tol
        assert abs(mesh.origin[0]) < tol, "the symmetry plane is x = 0"
    else:
        fld = random_poly_field(mesh.dim, degree, seed, scale)
        sym = None
    return Problem(f"poly{degree}_p{p}", mesh, p,
                   PAPER_N_PLUS[mesh.dim][p] if n_plus is None else n_plus,
                   n_gauss or default_gauss(p), LINEAR_ELASTIC, mu, lam,
                   mms_loads(fld, mu, lam, traction_faces, sym), stencil_quantum=quantum_for(mesh))


def random_state(n_cells: int, dim: int, seed: int, scale: float = 1e-3) -> np.ndarray:
    """Seeded N(0,1)*scale displacement state (n_cells, dim)."""
    return np.random.default_rng(seed).standard_normal((n_cells, dim)) * scale
