"""ctypes declarations of the libhofv C ABI (include/hofv.h).

Loading fails loudly: there is no fallback implementation of any step.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# HOFV_LIB may name another build of the same library (e.g. a variant under test)
LIB_PATH = os.environ.get("HOFV_LIB") or os.path.join(HERE, "libhofv.so")

HOFV_OK = 0
STATUS = {0: "HOFV_OK", -1: "HOFV_EINVAL", -2: "HOFV_ENOMEM", -3: "HOFV_EHIP", -4: "HOFV_ESINGULAR",
          -5: "HOFV_ENOCONV", -6: "HOFV_ENAN", -7: "HOFV_EINVERTED", -8: "HOFV_ESTATE"}

LINEAR_ELASTIC, NEO_HOOKEAN = 0, 1
BC_DISPLACEMENT, BC_TRACTION = 0, 1


class Params(C.Structure):
    _fields_ = [("dim", C.c_int32), ("order_p", C.c_int32), ("n_plus", C.c_int32), ("n_gauss", C.c_int32),
                ("material", C.c_int32), ("fold_quadrature", C.c_int32), ("mu", C.c_double),
                ("lambda_", C.c_double), ("alpha", C.c_double), ("k_weight", C.c_double),
                ("ghost_weight", C.c_double), ("stencil_quantum", C.c_double), ("host_only", C.c_int32),
                ("precond_levels", C.c_int32), ("face_rule", C.c_int32), ("stencil_grow", C.c_int32)]


class SetupReport(C.Structure):
    _fields_ = [("stencil_size", C.c_int32), ("n_colours", C.c_int32), ("n_internal_faces", C.c_int64),
                ("n_disp_faces", C.c_int64), ("n_trac_faces", C.c_int64), ("max_cond", C.c_double),
                ("device_bytes", C.c_double), ("residual_bytes", C.c_double), ("setup_seconds", C.c_double),
                ("n_grown_stencils", C.c_int64)]


class KrylovOpts(C.Structure):
    _fields_ = [("restart", C.c_int32), ("max_iters", C.c_int32), ("rtol", C.c_double),
                ("n_sweeps", C.c_int32), ("learned", C.c_int32), ("side", C.c_int32), ("gs_passes", C.c_int32),
                ("graphs", C.c_int32)]


class KrylovStats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("rel_residual", C.c_double),
                ("seconds", C.c_double), ("fallbacks", C.c_int32), ("stalled", C.c_int32)]


class NewtonOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("eta", C.c_double), ("max_newton", C.c_int32),
                ("n_increments", C.c_int32), ("max_line_search", C.c_int32), ("krylov", KrylovOpts),
                ("forcing", C.c_int32), ("predictor", C.c_int32)]


class HarvestOpts(C.Structure):
    _fields_ = [("n_starts", C.c_int32), ("length", C.c_int32), ("newton_steps", C.c_int32),
                ("seed", C.c_uint64), ("rtol", C.c_double), ("restart", C.c_int32), ("max_iters", C.c_int32),
                ("n_sweeps", C.c_int32)]


class TrainOpts(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_double), ("n_sweeps", C.c_int32),
                ("seed", C.c_uint64), ("epoch_loss", C.POINTER(C.c_double))]


class TrainStats(C.Structure):
    _fields_ = [("steps", C.c_int32), ("loss_first", C.c_double), ("loss_last", C.c_double),
                ("seconds", C.c_double)]


class NewtonStats(C.Structure):
    _fields_ = [("newton_iters", C.c_int32), ("krylov_iters", C.c_int32), ("converged", C.c_int32),
                ("rel_residual", C.c_double), ("seconds", C.c_double), ("fallbacks", C.c_int32)]


P = C.c_void_p
D = C.POINTER(C.c_double)
I64 = C.c_int64
ST = C.c_int

# name -> (restype, argtypes); every function returns hofv_status except hofv_last_error
SIGNATURES = {
    "hofv_create": (ST, [C.POINTER(Params), C.POINTER(P)]),
    "hofv_destroy": (ST, [P]),
    "hofv_last_error": (C.c_char_p, [P]),
    "hofv_set_mesh": (ST, [P, I64, D, I64, C.POINTER(C.c_int64)]),
    "hofv_set_mesh_simplices": (ST, [P, I64, D, I64, C.POINTER(C.c_int64)]),
    "hofv_set_mesh_polyhedra": (ST, [P, I64, D, I64, I64, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                     C.POINTER(C.c_int64)]),
    "hofv_volume_qpoints_csr": (ST, [P, C.POINTER(I64), C.POINTER(C.POINTER(C.c_int64)), C.POINTER(D)]),
    "hofv_boundary_faces": (ST, [P, C.POINTER(I64), C.POINTER(C.c_int32), C.POINTER(D), C.POINTER(D), C.POINTER(D)]),
    "hofv_volume_qpoints": (ST, [P, C.POINTER(C.c_int32), C.POINTER(D)]),
    "hofv_cell_centroids": (ST, [P, C.POINTER(D)]),
    "hofv_set_bc": (ST, [P, C.POINTER(C.c_int32), D, D, D]),
    "hofv_set_body_force": (ST, [P, D]),
    "hofv_setup": (ST, [P, C.POINTER(SetupReport)]),
    "hofv_set_load_scale": (ST, [P, C.c_double]),
    "hofv_set_multigrid": (ST, [P, C.c_int32]),
    "hofv_set_nej": (ST, [P, C.c_int32]),
    "hofv_nej_apply": (ST, [P, P, P, P]),
    "hofv_residual": (ST, [P, P, P, P]),
    "hofv_jvp": (ST, [P, P, P, P, P, C.c_double, P]),
    "hofv_jvp_noalloc": (ST, [P, P, P, P, P, C.c_double, P]),
    "hofv_precond_apply": (ST, [P, P, P, C.c_int32, C.c_int32, P]),
    "hofv_fgmres_solve": (ST, [P, P, P, P, P, C.POINTER(KrylovOpts), C.POINTER(KrylovStats), P]),
    "hofv_newton_solve": (ST, [P, P, C.POINTER(NewtonOpts), C.POINTER(NewtonStats), P]),
    "hofv_set_dynamics": (ST, [P, C.c_double, C.c_double]),
    "hofv_dyn_reset": (ST, [P, P, P, P, P, P]),
    "hofv_dyn_step": (ST, [P, P, C.POINTER(NewtonOpts), C.POINTER(NewtonStats), P]),
    "hofv_set_timing": (ST, [P, C.c_int32]),
    "hofv_set_timing_only": (ST, [P, C.c_char_p]),
    "hofv_kernel_time": (ST, [P, C.c_char_p, D, C.POINTER(C.c_int64)]),
    "hofv_kernel_bytes": (ST, [P, C.c_char_p, D]),
    "hofv_nn_param_count": (C.c_int64, []),
    "hofv_nn_create": (ST, [C.c_uint64, C.POINTER(P)]),
    "hofv_nn_destroy": (ST, [P]),
    "hofv_nn_set_params": (ST, [P, C.POINTER(C.c_float), C.c_int64]),
    "hofv_nn_get_params": (ST, [P, C.POINTER(C.c_float), C.c_int64]),
    "hofv_nn_attach": (ST, [P, P]),
    "hofv_nn_train_step": (ST, [P, P, P, P, C.c_int32, C.c_int32, C.c_double, C.POINTER(C.c_double), P]),
    "hofv_nn_gradient": (ST, [P, P, P, P, P, C.POINTER(C.c_float), C.POINTER(C.c_double), P]),
    "hofv_nn_forward": (ST, [P, P, P, P, P, P]),
    "hofv_nn_save": (ST, [P, C.c_char_p]),
    "hofv_nn_load": (ST, [P, C.c_char_p]),
    "hofv_pairset_create": (ST, [P, C.c_int32, C.POINTER(P)]),
    "hofv_pairset_destroy": (ST, [P]),
    "hofv_pairset_data": (ST, [P, C.POINTER(C.c_int32), C.POINTER(P), C.POINTER(P)]),
    "hofv_pairset_copy": (ST, [P, C.c_int32, C.c_int32, P, P, P]),
    "hofv_harvest_pairs": (ST, [P, P, P, C.POINTER(HarvestOpts), P, P]),
    "hofv_nn_train": (ST, [P, C.c_int32, C.POINTER(P), C.POINTER(TrainOpts), C.POINTER(TrainStats), P]),
    "hofv_host_table": (ST, [P, C.c_char_p, C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(P)]),
}

_lib = None


def load():
    """Load libhofv.so (built in-tree by build()); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(python -m paper_2601_18417_amd.build); there is no fallback path")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
