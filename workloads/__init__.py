"""Seeded synthetic inputs (meshes, manufactured fields, loads, named problems).

This package holds no finite-volume arithmetic: it is the one module that both
the CPU oracle and the GPU library's tests and benchmark read their inputs from.
"""
from .meshes import (Mesh, PolyMesh, box_mesh, cell_ijk, face_list_mesh, merged_block_mesh,  # noqa: F401
                     split_block_mesh, tet_mesh, tri_mesh)
from .fields import (DISP, TRAC, Loads, PolyField, TrigField, body_force_le,  # noqa: F401
                     lame_from_young, mms_2d_unit, mms_3d_trig, mms_loads, random_poly_field,
                     traction_le)
from .configs import (LINEAR_ELASTIC, NEO_HOOKEAN, Problem, cantilever, cube_mms, vibrating_column,  # noqa: F401
                      poly_patch, random_state, split_mms, square_mms, tet_mms, tri_mms)
