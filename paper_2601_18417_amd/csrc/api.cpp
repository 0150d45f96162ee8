// C ABI entry points of libhofv (declared in include/hofv.h).
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "common.h"

namespace hofv {

static std::string g_create_error;

hofv_status fail(hofv_ctx* c, hofv_status s, const std::string& msg) {
  if (c) c->err = msg;
  else g_create_error = msg;
  return s;
}

hofv_status fgmres_impl(hofv_ctx* c, const double* u, const double* Ru, const double* rhs, double* x,
                        const hofv_krylov_opts* o, hofv_krylov_stats* stats, hipStream_t st);
hofv_status newton_impl(hofv_ctx* c, double* u, const hofv_newton_opts* o, hofv_newton_stats* stats,
                        hipStream_t st);

hofv_status harvest_impl(hofv_ctx* c, const double* u, const double* starts, const hofv_harvest_opts* o,
                         double* r_out, double* e_out, hipStream_t st);

hofv_status jvp_impl(hofv_ctx* c, const double* u, const double* Ru, const double* v, double* Jv, double eps,
                     hipStream_t st) {
  hofv_status s;
  if ((s = launch_jvp_pack(c, u, v, eps, st))) return s;
  return launch_residual(c, c->dev.w, Jv, Ru, c->dev.eps, st);
}

hofv_status precond_dispatch(hofv_ctx* c, const double* r, double* z, int sweeps, int learned, hipStream_t st) {
  if (c->nej.k > 0) {
    if (learned) return fail(c, HOFV_EINVAL, "the learned correction is trained on the approximate Jacobian");
    return nej_solve(c, r, z, sweeps, st);
  }
  if (!learned || !c->nn) return launch_precond(c, r, z, sweeps, st);
  hofv_status s;
  if (!c->nnw.zaj) {
    if ((s = dev_alloc(c, &c->nnw.zaj, (size_t)c->D * c->nc))) return s;
  }
  if ((s = launch_precond(c, r, c->nnw.zaj, sweeps, st))) return s;
  return nn_apply(c, c->nn, r, c->nnw.zaj, z, st);
}

static hofv_status need(hofv_ctx* c, int state, const char* what) {
  if (!c) return fail(nullptr, HOFV_EINVAL, "null context");
  if (c->state == 5 && state == 4) return fail(c, HOFV_ESTATE, std::string(what) + " on a host_only context");
  if (c->state < state) return fail(c, HOFV_ESTATE, std::string(what) + " called out of order");
  return HOFV_OK;
}

static hofv_status set_device(hofv_ctx* c) {
  HOFV_HIP(c, hipSetDevice(c->device));
  return HOFV_OK;
}

}  // namespace hofv

using namespace hofv;

extern "C" {

hofv_status hofv_create(const hofv_params* prm, hofv_ctx** out) {
  if (!out) return fail(nullptr, HOFV_EINVAL, "out is NULL");
  *out = nullptr;
  if (!prm) return fail(nullptr, HOFV_EINVAL, "params is NULL");
  if (prm->dim != 2 && prm->dim != 3) return fail(nullptr, HOFV_EINVAL, "dim must be 2 or 3");
  if (prm->order_p < 1 || prm->order_p > 3) return fail(nullptr, HOFV_EINVAL, "order_p must be 1, 2 or 3");
  if (prm->n_plus < 0) return fail(nullptr, HOFV_EINVAL, "n_plus must be >= 0");
  if (prm->n_gauss < 1 || prm->n_gauss > 3) return fail(nullptr, HOFV_EINVAL, "n_gauss must be 1..3");
  if (prm->material != HOFV_LINEAR_ELASTIC && prm->material != HOFV_NEO_HOOKEAN)
    return fail(nullptr, HOFV_EINVAL, "unknown material");
  if (prm->material == HOFV_NEO_HOOKEAN && prm->dim != 3)
    return fail(nullptr, HOFV_EINVAL, "the neo-Hookean law needs dim = 3");
  if (!(prm->stencil_quantum > 0)) return fail(nullptr, HOFV_EINVAL, "stencil_quantum must be > 0");
  if (prm->precond_levels < 0 || prm->precond_levels > 16)
    return fail(nullptr, HOFV_EINVAL, "precond_levels must be 0..16");
  if (prm->face_rule != 0 && prm->face_rule != 1) return fail(nullptr, HOFV_EINVAL, "face_rule must be 0 or 1");
  if (prm->stencil_grow < 0 || prm->stencil_grow > 255)
    return fail(nullptr, HOFV_EINVAL, "stencil_grow must be 0..255");
  if (!(prm->mu > 0) || !(prm->k_weight > 0) || prm->alpha < 0 || prm->ghost_weight <= 0)
    return fail(nullptr, HOFV_EINVAL, "mu, k_weight, ghost_weight must be > 0 and alpha >= 0");
  hofv_ctx* c = new (std::nothrow) hofv_ctx();
  if (!c) return fail(nullptr, HOFV_ENOMEM, "out of host memory");
  c->prm = *prm;
  c->D = prm->dim;
  int dev = -1;
  if (!prm->host_only && hipGetDevice(&dev) != hipSuccess) {
    delete c;
    return fail(nullptr, HOFV_EHIP, "no HIP device");
  }
  c->device = dev;
  *out = c;
  return HOFV_OK;
}

hofv_status hofv_destroy(hofv_ctx* c) {
  if (!c) return HOFV_OK;
  if (c->device >= 0) {
    hipSetDevice(c->device);
    hipDeviceSynchronize();
  }
  for (hipGraphExec_t g : c->kry.step_graph)
    if (g) hipGraphExecDestroy(g);
  if (c->kry.cap_stream) hipStreamDestroy(c->kry.cap_stream);
  for (void* p : c->allocations) hipFree(p);
  for (hipEvent_t e : c->ev_pool) hipEventDestroy(e);
  delete c;
  return HOFV_OK;
}

const char* hofv_last_error(const hofv_ctx* c) { return c ? c->err.c_str() : g_create_error.c_str(); }

hofv_status hofv_set_mesh(hofv_ctx* c, int64_t n_verts, const double* verts, int64_t n_cells,
                          const int64_t* cell_verts) {
  if (!c) return fail(nullptr, HOFV_EINVAL, "null context");
  if (c->state != 0) return fail(c, HOFV_ESTATE, "set_mesh may be called once");
  if (n_verts <= 0 || n_cells <= 0 || !verts || !cell_verts) return fail(c, HOFV_EINVAL, "empty mesh");
  if (n_cells >= INT32_MAX / 8) return fail(c, HOFV_EINVAL, "too many cells for 32-bit indices");
  const int D = c->D, ncv = D == 2 ? 4 : 8;
  c->nv = n_verts;
  c->nc = n_cells;
  c->verts.assign(verts, verts + n_verts * D);
  c->cells.assign(cell_verts, cell_verts + n_cells * ncv);
  for (int64_t v : c->cells)
    if (v < 0 || v >= n_verts) return fail(c, HOFV_EINVAL, "cell vertex index out of range");
  hofv_status s;
  if ((s = build_topology(c))) return s;
  if ((s = build_geometry(c))) return s;
  c->state = 1;
  return HOFV_OK;
}

hofv_status hofv_set_mesh_simplices(hofv_ctx* c, int64_t n_verts, const double* verts, int64_t n_cells,
                                    const int64_t* cell_verts) {
  if (!c) return fail(nullptr, HOFV_EINVAL, "null context");
  if (c->state != 0) return fail(c, HOFV_ESTATE, "set_mesh may be called once");
  if (n_verts <= 0 || n_cells <= 0 || !verts || !cell_verts) return fail(c, HOFV_EINVAL, "empty mesh");
  if (n_cells >= INT32_MAX / 8) return fail(c, HOFV_EINVAL, "too many cells for 32-bit indices");
  const int D = c->D;
  c->nv = n_verts;
  c->nc = n_cells;
  c->verts.assign(verts, verts + n_verts * D);
  c->cells.assign(cell_verts, cell_verts + n_cells * (D + 1));
  for (int64_t v : c->cells)
    if (v < 0 || v >= n_verts) return fail(c, HOFV_EINVAL, "cell vertex index out of range");
  hofv_status s;
  if ((s = build_topology(c))) return s;
  if ((s = build_geometry(c))) return s;
  c->state = 1;
  return HOFV_OK;
}

hofv_status hofv_set_mesh_polyhedra(hofv_ctx* c, int64_t n_verts, const double* verts, int64_t n_cells,
                                   int64_t n_faces, const int64_t* face_ptr, const int64_t* face_verts,
                                   const int64_t* face_cells) {
  if (!c) return fail(nullptr, HOFV_EINVAL, "null context");
  if (c->state != 0) return fail(c, HOFV_ESTATE, "set_mesh may be called once");
  if (n_verts <= 0 || n_cells <= 0 || n_faces <= 0 || !verts || !face_ptr || !face_verts || !face_cells)
    return fail(c, HOFV_EINVAL, "empty mesh");
  if (n_cells >= INT32_MAX / 8 || n_faces >= INT32_MAX / 2) return fail(c, HOFV_EINVAL, "too many cells for 32-bit indices");
  c->nv = n_verts;
  c->nc = n_cells;
  c->verts.assign(verts, verts + n_verts * c->D);
  c->cells.clear();
  hofv_status s;
  if ((s = build_topology_poly(c, n_faces, face_ptr, face_verts, face_cells))) return s;
  if ((s = build_geometry(c))) return s;
  c->state = 1;
  return HOFV_OK;
}

hofv_status hofv_boundary_faces(hofv_ctx* c, int64_t* n_bfaces, int32_t* n_q, const double** centres,
                                const double** normals, const double** qpoints) {
  hofv_status s = need(c, 1, "boundary_faces");
  if (s) return s;
  if (n_bfaces) *n_bfaces = (int64_t)c->bface.size();
  if (n_q) *n_q = c->nq;
  if (centres) *centres = c->b_centre.data();
  if (normals) *normals = c->b_normal.data();
  if (qpoints) *qpoints = c->b_qp.data();
  return HOFV_OK;
}

hofv_status hofv_cell_centroids(hofv_ctx* c, const double** centroids) {
  hofv_status s = need(c, 1, "cell_centroids");
  if (s) return s;
  if (!centroids) return fail(c, HOFV_EINVAL, "null argument");
  *centroids = c->cen.data();
  return HOFV_OK;
}

hofv_status hofv_volume_qpoints(hofv_ctx* c, int32_t* n_qv, const double** points) {
  hofv_status s = need(c, 1, "volume_qpoints");
  if (s) return s;
  for (int64_t P = 0; P < c->nc; ++P)
    if (c->vq_ptr[P + 1] - c->vq_ptr[P] != c->nqv)
      return fail(c, HOFV_EINVAL, "cells have different numbers of volume points: use hofv_volume_qpoints_csr");
  if (n_qv) *n_qv = c->nqv;
  if (points) *points = c->vq_pts.data();
  return HOFV_OK;
}

hofv_status hofv_volume_qpoints_csr(hofv_ctx* c, int64_t* n_points, const int64_t** cell_ptr,
                                    const double** points) {
  hofv_status s = need(c, 1, "volume_qpoints_csr");
  if (s) return s;
  if (n_points) *n_points = c->vq_ptr[c->nc];
  if (cell_ptr) *cell_ptr = c->vq_ptr.data();
  if (points) *points = c->vq_pts.data();
  return HOFV_OK;
}

hofv_status hofv_set_bc(hofv_ctx* c, const int32_t* type, const double* u_b_q, const double* u_b_centre,
                        const double* traction_q) {
  hofv_status s = need(c, 1, "set_bc");
  if (s) return s;
  if (c->state >= 4) return fail(c, HOFV_ESTATE, "set_bc after setup");
  const size_t nb = c->bface.size();
  const int D = c->D, nq = c->nq;
  c->btype.assign(nb, HOFV_BC_DISPLACEMENT);
  if (type) {
    for (size_t b = 0; b < nb; ++b) {
      if (type[b] != HOFV_BC_DISPLACEMENT && type[b] != HOFV_BC_TRACTION && type[b] != HOFV_BC_SYMMETRY)
        return fail(c, HOFV_EINVAL, "unknown boundary condition type");
      c->btype[b] = type[b];
    }
  }
  c->ubq.assign(nb * nq * D, 0.0);
  c->ubc.assign(nb * D, 0.0);
  c->tq.assign(nb * nq * D, 0.0);
  if (u_b_q) std::memcpy(c->ubq.data(), u_b_q, c->ubq.size() * sizeof(double));
  if (u_b_centre) std::memcpy(c->ubc.data(), u_b_centre, c->ubc.size() * sizeof(double));
  if (traction_q) std::memcpy(c->tq.data(), traction_q, c->tq.size() * sizeof(double));
  c->state = std::max(c->state, 2);
  return HOFV_OK;
}

hofv_status hofv_set_body_force(hofv_ctx* c, const double* values) {
  hofv_status s = need(c, 1, "set_body_force");
  if (s) return s;
  if (c->state >= 4) return fail(c, HOFV_ESTATE, "set_body_force after setup");
  if (values) c->fb.assign(values, values + (size_t)c->vq_ptr[c->nc] * c->D);
  else c->fb.clear();
  c->state = std::max(c->state, 3);
  return HOFV_OK;
}

hofv_status hofv_setup(hofv_ctx* c, hofv_setup_report* rep) {
  hofv_status s = need(c, 1, "setup");
  if (s) return s;
  if (c->state >= 4) return fail(c, HOFV_ESTATE, "setup may be called once");
  if (c->btype.empty() && !c->bface.empty()) {
    if ((s = hofv_set_bc(c, nullptr, nullptr, nullptr, nullptr))) return s;
  }
  if (!c->prm.host_only && (s = set_device(c))) return s;
  if ((s = build_tables(c))) return s;
  if (!c->prm.host_only && (s = noalloc_init(c))) return s;
  c->state = c->prm.host_only ? 5 : 4;
  if (rep) *rep = c->report;
  return HOFV_OK;
}

hofv_status hofv_set_load_scale(hofv_ctx* c, double sc) {
  hofv_status s = need(c, 1, "set_load_scale");
  if (s) return s;
  if (!std::isfinite(sc)) return fail(c, HOFV_EINVAL, "load scale must be finite");
  c->load = sc;
  return HOFV_OK;
}

hofv_status hofv_set_multigrid(hofv_ctx* c, int32_t enable) {
  hofv_status s = need(c, 4, "set_multigrid");
  if (s) return s;
  if (enable && c->dev.mg.size() < 2) return fail(c, HOFV_EINVAL, "no multigrid hierarchy was built at setup");
  if (enable && c->dev.dyn_m) return fail(c, HOFV_EINVAL, "the multigrid hierarchy is built for the static operator");
  c->use_mg = enable != 0;
  return HOFV_OK;
}

hofv_status hofv_set_nej(hofv_ctx* c, int32_t inner_iters) {
  hofv_status s = need(c, 4, "set_nej");
  if (s) return s;
  if ((s = set_device(c))) return s;
  return nej_set(c, inner_iters);
}

hofv_status hofv_nej_apply(hofv_ctx* c, const double* d_v, double* d_out, void* stream) {
  hofv_status s = need(c, 4, "nej_apply");
  if (s) return s;
  if (!d_v || !d_out || (const void*)d_v == (void*)d_out) return fail(c, HOFV_EINVAL, "bad v/out pointers");
  if (c->prm.material != HOFV_LINEAR_ELASTIC)
    return fail(c, HOFV_EINVAL, "the near-exact Jacobian is defined for the linear elastic law");
  if ((s = set_device(c))) return s;
  if ((s = nej_zero(c))) return s;
  return launch_nej(c, d_v, d_out, (hipStream_t)stream);
}

hofv_status hofv_set_dynamics(hofv_ctx* c, double rho, double dt) {
  hofv_status s = need(c, 4, "set_dynamics");
  if (s) return s;
  if ((s = set_device(c))) return s;
  return dyn_set(c, rho, dt);
}

hofv_status hofv_dyn_reset(hofv_ctx* c, const double* d_u_t, const double* d_u_tm1, const double* d_v_t,
                           const double* d_v_tm1, void* stream) {
  hofv_status s = need(c, 4, "dyn_reset");
  if (s) return s;
  if (!d_u_t || !d_u_tm1 || !d_v_t || !d_v_tm1) return fail(c, HOFV_EINVAL, "null pointer");
  if ((s = set_device(c))) return s;
  return dyn_reset(c, d_u_t, d_u_tm1, d_v_t, d_v_tm1, (hipStream_t)stream);
}

hofv_status hofv_dyn_step(hofv_ctx* c, double* d_u, const hofv_newton_opts* opts, hofv_newton_stats* stats,
                          void* stream) {
  hofv_status s = need(c, 4, "dyn_step");
  if (s) return s;
  if (!d_u || !opts) return fail(c, HOFV_EINVAL, "null pointer");
  if (opts->forcing != 0 && opts->forcing != 1) return fail(c, HOFV_EINVAL, "forcing must be 0 or 1");
  if ((s = set_device(c))) return s;
  hofv_newton_stats tmp{};
  return dyn_step(c, d_u, opts, stats ? stats : &tmp, (hipStream_t)stream);
}

hofv_status hofv_residual(hofv_ctx* c, const double* d_u, double* d_R, void* stream) {
  hofv_status s = need(c, 4, "residual");
  if (s) return s;
  if (!d_u || !d_R || (const void*)d_u == (void*)d_R) return fail(c, HOFV_EINVAL, "bad u/R pointers");
  if ((s = set_device(c))) return s;
  return launch_residual(c, d_u, d_R, nullptr, nullptr, (hipStream_t)stream);
}

hofv_status hofv_jvp(hofv_ctx* c, const double* d_u, const double* d_Ru, const double* d_v, double* d_Jv,
                     double eps, void* stream) {
  hofv_status s = need(c, 4, "jvp");
  if (s) return s;
  if (!d_u || !d_Ru || !d_v || !d_Jv) return fail(c, HOFV_EINVAL, "null pointer");
  if ((const void*)d_Jv == (const void*)d_u || (const void*)d_Jv == (const void*)d_Ru ||
      (const void*)d_Jv == (const void*)d_v)
    return fail(c, HOFV_EINVAL, "Jv must not alias the inputs");
  if (!std::isfinite(eps)) return fail(c, HOFV_EINVAL, "eps must be finite");
  if ((s = set_device(c))) return s;
  return jvp_impl(c, d_u, d_Ru, d_v, d_Jv, eps, (hipStream_t)stream);
}

hofv_status hofv_jvp_noalloc(hofv_ctx* c, const double* d_u, const double* d_Ru, const double* d_v, double* d_Jv,
                             double eps, void* stream) {
  hofv_status s = need(c, 4, "jvp_noalloc");
  if (s) return s;
  if (!d_u || !d_Ru || !d_v || !d_Jv) return fail(c, HOFV_EINVAL, "null pointer");
  if ((const void*)d_Jv == (const void*)d_u || (const void*)d_Jv == (const void*)d_Ru ||
      (const void*)d_Jv == (const void*)d_v)
    return fail(c, HOFV_EINVAL, "Jv must not alias the inputs");
  if (!std::isfinite(eps)) return fail(c, HOFV_EINVAL, "eps must be finite");
  if ((s = set_device(c))) return s;
  return jvp_noalloc_impl(c, d_u, d_Ru, d_v, d_Jv, eps, (hipStream_t)stream);
}

hofv_status hofv_precond_apply(hofv_ctx* c, const double* d_r, double* d_z, int32_t n_sweeps, int32_t learned,
                               void* stream) {
  hofv_status s = need(c, 4, "precond_apply");
  if (s) return s;
  if (!d_r || !d_z || (const void*)d_r == (void*)d_z) return fail(c, HOFV_EINVAL, "bad r/z pointers");
  if (n_sweeps < 1) return fail(c, HOFV_EINVAL, "n_sweeps must be >= 1");
  if ((s = set_device(c))) return s;
  return precond_dispatch(c, d_r, d_z, n_sweeps, learned, (hipStream_t)stream);
}

hofv_status hofv_fgmres_solve(hofv_ctx* c, const double* d_u, const double* d_Ru, const double* d_rhs,
                              double* d_x, const hofv_krylov_opts* opts, hofv_krylov_stats* stats, void* stream) {
  hofv_status s = need(c, 4, "fgmres_solve");
  if (s) return s;
  if (!d_u || !d_Ru || !d_rhs || !d_x || !opts) return fail(c, HOFV_EINVAL, "null pointer");
  if ((s = set_device(c))) return s;
  hofv_krylov_stats tmp{};
  s = fgmres_impl(c, d_u, d_Ru, d_rhs, d_x, opts, stats ? stats : &tmp, (hipStream_t)stream);
  if (s == HOFV_OK && !(stats ? stats : &tmp)->converged)
    return fail(c, HOFV_ENOCONV, "FGMRES did not reach the tolerance");
  return s;
}

hofv_status hofv_newton_solve(hofv_ctx* c, double* d_u, const hofv_newton_opts* opts, hofv_newton_stats* stats,
                              void* stream) {
  hofv_status s = need(c, 4, "newton_solve");
  if (s) return s;
  if (!d_u || !opts) return fail(c, HOFV_EINVAL, "null pointer");
  if (opts->forcing != 0 && opts->forcing != 1) return fail(c, HOFV_EINVAL, "forcing must be 0 or 1");
  if (opts->predictor != 0 && opts->predictor != 1) return fail(c, HOFV_EINVAL, "predictor must be 0 or 1");
  if ((s = set_device(c))) return s;
  hofv_newton_stats tmp{};
  return newton_impl(c, d_u, opts, stats ? stats : &tmp, (hipStream_t)stream);
}

hofv_status hofv_host_table(hofv_ctx* c, const char* name, int64_t* count, int32_t* elem_bytes,
                            const void** data) {
  if (!c || !name) return fail(c, HOFV_EINVAL, "null argument");
  if (c->state != 5) return fail(c, HOFV_ESTATE, "host tables exist after setup of a host_only context");
  auto it = c->host_tables.find(name);
  if (it == c->host_tables.end()) return fail(c, HOFV_EINVAL, std::string("unknown table ") + name);
  if (count) *count = it->second.elem ? (int64_t)(it->second.bytes.size() / it->second.elem) : 0;
  if (elem_bytes) *elem_bytes = it->second.elem;
  if (data) *data = it->second.bytes.data();
  return HOFV_OK;
}

int64_t hofv_nn_param_count(void) { return kNnParams; }

hofv_status hofv_nn_create(uint64_t seed, hofv_nn** out) {
  if (!out) return fail(nullptr, HOFV_EINVAL, "out is NULL");
  *out = nullptr;
  hofv_nn* m = new (std::nothrow) hofv_nn();
  if (!m) return fail(nullptr, HOFV_ENOMEM, "out of host memory");
  if (hipGetDevice(&m->device) != hipSuccess) {
    delete m;
    return fail(nullptr, HOFV_EHIP, "no HIP device");
  }
  if (nn_alloc_model(m) != HOFV_OK) {
    nn_free_model(m);
    delete m;
    return fail(nullptr, HOFV_ENOMEM, "device allocation of the model failed");
  }
  // He initialisation (splitmix64 + Box-Muller), zero biases and decoder
  std::vector<float> p(kNnParams, 0.f);
  uint64_t st = seed ^ 0x9E3779B97F4A7C15ull;
  auto next = [&]() {
    st += 0x9E3779B97F4A7C15ull;
    uint64_t z = st;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return (double)((z ^ (z >> 31)) >> 11) * (1.0 / 9007199254740992.0);
  };
  auto normal = [&]() {
    double u1 = next(), u2 = next();
    if (u1 < 1e-300) u1 = 1e-300;
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
  };
  for (int64_t i = 0; i < kNnIn * kNnWidth; ++i) p[kNnOffWe + i] = (float)(normal() * std::sqrt(2.0 / kNnIn));
  for (int l = 0; l < kNnLayers; ++l)
    for (int64_t i = 0; i < kNnLayerK * kNnWidth; ++i)
      p[kNnOffW(l) + i] = (float)(normal() * std::sqrt(2.0 / kNnLayerK) * 0.5);
  hofv_status s = hofv_nn_set_params(m, p.data(), kNnParams);
  if (s) {
    nn_free_model(m);
    delete m;
    return s;
  }
  *out = m;
  return HOFV_OK;
}

hofv_status hofv_nn_destroy(hofv_nn* m) {
  if (!m) return HOFV_OK;
  hipSetDevice(m->device);
  hipDeviceSynchronize();
  nn_free_model(m);
  delete m;
  return HOFV_OK;
}

hofv_status hofv_nn_set_params(hofv_nn* m, const float* host, int64_t n) {
  if (!m || !host || n != kNnParams) return fail(nullptr, HOFV_EINVAL, "bad model or parameter count");
  if (hipSetDevice(m->device) != hipSuccess) return fail(nullptr, HOFV_EHIP, "hipSetDevice");
  if (hipMemcpy(m->p, host, kNnParams * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(m->m, 0, kNnParams * 4) != hipSuccess || hipMemset(m->v, 0, kNnParams * 4) != hipSuccess ||
      hipMemset(m->g, 0, kNnParams * 4) != hipSuccess)
    return fail(nullptr, HOFV_EHIP, "parameter upload failed");
  m->step = 0;
  if (nn_refresh(m, nullptr) != HOFV_OK || hipDeviceSynchronize() != hipSuccess)
    return fail(nullptr, HOFV_EHIP, "parameter refresh failed");
  return HOFV_OK;
}

hofv_status hofv_nn_get_params(hofv_nn* m, float* host, int64_t n) {
  if (!m || !host || n != kNnParams) return fail(nullptr, HOFV_EINVAL, "bad model or parameter count");
  if (hipSetDevice(m->device) != hipSuccess || hipDeviceSynchronize() != hipSuccess ||
      hipMemcpy(host, m->p, kNnParams * 4, hipMemcpyDeviceToHost) != hipSuccess)
    return fail(nullptr, HOFV_EHIP, "parameter download failed");
  return HOFV_OK;
}

hofv_status hofv_nn_attach(hofv_ctx* c, hofv_nn* m) {
  hofv_status s = need(c, 4, "nn_attach");
  if (s) return s;
  if (m && m->device != c->device) return fail(c, HOFV_EINVAL, "model and context are on different devices");
  c->nn = m;
  return HOFV_OK;
}

}  // extern "C"

namespace hofv {
// One optimisation step over the pairs r[i], e[i] (device pointers) of ctx's
// mesh: z_AJ = plain preconditioner(r), gradients of ||z - e||^2 / ||e||^2
// averaged over the pairs, then Adam.  *loss: the mean loss before the step.
static hofv_status train_step(hofv_ctx* c, hofv_nn* m, const double* const* r, const double* const* e, int n,
                              int sweeps, double lr, double* loss, hipStream_t st) {
  hofv_status s;
  if (!c->nnw.zaj) {
    if ((s = dev_alloc(c, &c->nnw.zaj, (size_t)c->D * c->nc))) return s;
  }
  if (nn_zero_grad(m, st) || nn_zero_scalar(m->loss, st)) return fail(c, HOFV_EHIP, "zeroing failed");
  for (int i = 0; i < n; ++i) {
    if ((s = launch_precond(c, r[i], c->nnw.zaj, sweeps, st))) return s;
    if ((s = nn_grad(c, m, r[i], c->nnw.zaj, e[i], 1.0f / n, m->loss, st))) return s;
  }
  double l = 0;
  HOFV_HIP(c, hipMemcpyAsync(&l, m->loss, sizeof(double), hipMemcpyDeviceToHost, st));
  if (nn_adam(m, lr, st)) return fail(c, HOFV_EHIP, "Adam step failed");
  HOFV_HIP(c, hipStreamSynchronize(st));
  if (loss) *loss = l / n;
  if (!std::isfinite(l)) return fail(c, HOFV_ENAN, "non-finite training loss");
  return HOFV_OK;
}

// splitmix64 (Steele, Lea and Flood 2014): the order of the training pairs
struct SplitMix {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  // uniform in [0, k) by rejection of the biased top range
  uint64_t below(uint64_t k) {
    const uint64_t lim = UINT64_MAX - UINT64_MAX % k;
    uint64_t x;
    do x = next(); while (x >= lim);
    return x % k;
  }
  template <class T>
  void shuffle(std::vector<T>& v) {  // Fisher-Yates
    for (size_t i = v.size(); i > 1; --i) std::swap(v[i - 1], v[below(i)]);
  }
};
}  // namespace hofv

extern "C" {

hofv_status hofv_nn_train_step(hofv_ctx* c, hofv_nn* m, const double* d_r, const double* d_e, int32_t n_pairs,
                               int32_t n_sweeps, double lr, double* loss, void* stream) {
  hofv_status s = need(c, 4, "nn_train_step");
  if (s) return s;
  if (!m || !d_r || !d_e || n_pairs < 1 || n_sweeps < 1 || !(lr >= 0)) return fail(c, HOFV_EINVAL, "bad argument");
  if (m->device != c->device) return fail(c, HOFV_EINVAL, "model and context are on different devices");
  if ((s = set_device(c))) return s;
  const size_t len = (size_t)c->D * c->nc;
  std::vector<const double*> r(n_pairs), e(n_pairs);
  for (int i = 0; i < n_pairs; ++i) {
    r[i] = d_r + i * len;
    e[i] = d_e + i * len;
  }
  return train_step(c, m, r.data(), e.data(), n_pairs, n_sweeps, lr, loss, (hipStream_t)stream);
}

hofv_status hofv_pairset_create(hofv_ctx* c, int32_t capacity, hofv_pairset** out) {
  if (!out) return fail(c, HOFV_EINVAL, "out is NULL");
  *out = nullptr;
  hofv_status s = need(c, 4, "pairset_create");
  if (s) return s;
  if (capacity < 1) return fail(c, HOFV_EINVAL, "capacity must be >= 1");
  if ((s = set_device(c))) return s;
  hofv_pairset* p = new (std::nothrow) hofv_pairset();
  if (!p) return fail(c, HOFV_ENOMEM, "out of host memory");
  p->ctx = c;
  p->cap = capacity;
  const size_t bytes = (size_t)capacity * c->D * c->nc * sizeof(double);
  if (hipMalloc((void**)&p->r, bytes) != hipSuccess || hipMalloc((void**)&p->e, bytes) != hipSuccess) {
    if (p->r) hipFree(p->r);
    delete p;
    return fail(c, HOFV_ENOMEM, "device allocation of the pair set failed");
  }
  *out = p;
  return HOFV_OK;
}

hofv_status hofv_pairset_destroy(hofv_pairset* p) {
  if (!p) return HOFV_OK;
  hipSetDevice(p->ctx->device);
  hipDeviceSynchronize();
  hipFree(p->r);
  hipFree(p->e);
  delete p;
  return HOFV_OK;
}

hofv_status hofv_pairset_data(const hofv_pairset* p, int32_t* n_pairs, const double** d_r, const double** d_e) {
  if (!p) return fail(nullptr, HOFV_EINVAL, "null pair set");
  if (n_pairs) *n_pairs = p->n;
  if (d_r) *d_r = p->r;
  if (d_e) *d_e = p->e;
  return HOFV_OK;
}

hofv_status hofv_pairset_copy(const hofv_pairset* p, int32_t first, int32_t count, double* d_r, double* d_e,
                              void* stream) {
  if (!p) return fail(nullptr, HOFV_EINVAL, "null pair set");
  hofv_ctx* c = p->ctx;
  if (first < 0 || count < 0 || first + count > p->n) return fail(c, HOFV_EINVAL, "pairs outside the set");
  hofv_status s = set_device(c);
  if (s) return s;
  const size_t len = (size_t)c->D * c->nc, bytes = (size_t)count * len * sizeof(double);
  hipStream_t st = (hipStream_t)stream;
  if (d_r && bytes) HOFV_HIP(c, hipMemcpyAsync(d_r, p->r + (size_t)first * len, bytes, hipMemcpyDeviceToDevice, st));
  if (d_e && bytes) HOFV_HIP(c, hipMemcpyAsync(d_e, p->e + (size_t)first * len, bytes, hipMemcpyDeviceToDevice, st));
  return HOFV_OK;
}

hofv_status hofv_harvest_pairs(hofv_ctx* c, const double* d_u, const double* d_starts, const hofv_harvest_opts* o,
                               hofv_pairset* set, void* stream) {
  hofv_status s = need(c, 4, "harvest_pairs");
  if (s) return s;
  if (!d_u || !o || !set) return fail(c, HOFV_EINVAL, "null pointer");
  if (set->ctx != c) return fail(c, HOFV_EINVAL, "the pair set belongs to another context");
  if (o->n_starts < 0 || o->length < 0 || o->newton_steps < 0) return fail(c, HOFV_EINVAL, "negative pair counts");
  if (c->nej.k > 0) return fail(c, HOFV_EINVAL, "pairs are harvested with the approximate Jacobian, not the NEJ");
  const int64_t add = (int64_t)o->n_starts * o->length + o->newton_steps;
  if (set->n + add > set->cap) return fail(c, HOFV_EINVAL, "the pairs do not fit the pair set");
  if ((s = set_device(c))) return s;
  const size_t len = (size_t)c->D * c->nc;
  s = harvest_impl(c, d_u, d_starts, o, set->r + (size_t)set->n * len, set->e + (size_t)set->n * len,
                   (hipStream_t)stream);
  if (s == HOFV_OK) set->n += (int32_t)add;
  return s;
}

hofv_status hofv_nn_train(hofv_nn* m, int32_t n_sets, hofv_pairset* const* sets, const hofv_train_opts* o,
                          hofv_train_stats* stats, void* stream) {
  if (!m || !sets || !o || n_sets < 1) return fail(nullptr, HOFV_EINVAL, "bad argument");
  if (o->epochs < 1 || o->batch < 1 || o->n_sweeps < 1 || !(o->lr >= 0))
    return fail(nullptr, HOFV_EINVAL, "epochs, batch and n_sweeps must be >= 1 and lr >= 0");
  for (int i = 0; i < n_sets; ++i) {
    if (!sets[i] || sets[i]->n < 1) return fail(nullptr, HOFV_EINVAL, "empty or null pair set");
    hofv_status s = need(sets[i]->ctx, 4, "nn_train");
    if (s) return s;
    if (sets[i]->ctx->device != m->device) return fail(sets[i]->ctx, HOFV_EINVAL, "model and pair set devices differ");
  }
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t st = (hipStream_t)stream;
  SplitMix rng{o->seed};
  hofv_train_stats out{};
  for (int ep = 0; ep < o->epochs; ++ep) {
    // minibatches: each set's pairs in a random order, cut into batches
    struct Job {
      int set;
      std::vector<int> idx;
    };
    std::vector<Job> jobs;
    for (int i = 0; i < n_sets; ++i) {
      std::vector<int> perm(sets[i]->n);
      for (int k = 0; k < sets[i]->n; ++k) perm[k] = k;
      rng.shuffle(perm);
      for (size_t b = 0; b < perm.size(); b += (size_t)o->batch)
        jobs.push_back({i, std::vector<int>(perm.begin() + b, perm.begin() + std::min(perm.size(), b + o->batch))});
    }
    rng.shuffle(jobs);
    double tot = 0.0;
    int64_t cnt = 0;
    for (const Job& j : jobs) {
      hofv_pairset* p = sets[j.set];
      hofv_ctx* c = p->ctx;
      if (hipSetDevice(c->device) != hipSuccess) return fail(c, HOFV_EHIP, "hipSetDevice");
      const size_t len = (size_t)c->D * c->nc;
      std::vector<const double*> r, e;
      for (int k : j.idx) {
        r.push_back(p->r + (size_t)k * len);
        e.push_back(p->e + (size_t)k * len);
      }
      double l = 0.0;
      hofv_status s = train_step(c, m, r.data(), e.data(), (int)r.size(), o->n_sweeps, o->lr, &l, st);
      if (s) return s;
      tot += l * (double)r.size();
      cnt += (int64_t)r.size();
      ++out.steps;
    }
    const double mean = tot / (double)std::max<int64_t>(cnt, 1);
    if (ep == 0) out.loss_first = mean;
    out.loss_last = mean;
    if (o->epoch_loss) o->epoch_loss[ep] = mean;
  }
  out.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (stats) *stats = out;
  return HOFV_OK;
}

hofv_status hofv_nn_save(hofv_nn* m, const char* path) {
  if (!m || !path) return fail(nullptr, HOFV_EINVAL, "null argument");
  std::vector<float> p(kNnParams);
  hofv_status s = hofv_nn_get_params(m, p.data(), kNnParams);
  if (s) return s;
  FILE* f = std::fopen(path, "wb");
  if (!f) return fail(nullptr, HOFV_EINVAL, std::string("cannot write ") + path);
  const int64_t cnt = kNnParams;
  const bool ok = std::fwrite("HOFVNN01", 1, 8, f) == 8 && std::fwrite(&cnt, sizeof cnt, 1, f) == 1 &&
                  std::fwrite(p.data(), sizeof(float), p.size(), f) == p.size();
  if (std::fclose(f) != 0 || !ok) return fail(nullptr, HOFV_EINVAL, std::string("cannot write ") + path);
  return HOFV_OK;
}

hofv_status hofv_nn_load(hofv_nn* m, const char* path) {
  if (!m || !path) return fail(nullptr, HOFV_EINVAL, "null argument");
  FILE* f = std::fopen(path, "rb");
  if (!f) return fail(nullptr, HOFV_EINVAL, std::string("cannot read ") + path);
  char tag[8];
  int64_t cnt = 0;
  std::vector<float> p(kNnParams);
  bool ok = std::fread(tag, 1, 8, f) == 8 && std::memcmp(tag, "HOFVNN01", 8) == 0 &&
            std::fread(&cnt, sizeof cnt, 1, f) == 1 && cnt == kNnParams &&
            std::fread(p.data(), sizeof(float), p.size(), f) == p.size();
  std::fclose(f);
  if (!ok) return fail(nullptr, HOFV_EINVAL, std::string(path) + " is not a model of this network");
  return hofv_nn_set_params(m, p.data(), kNnParams);
}

hofv_status hofv_nn_gradient(hofv_ctx* c, hofv_nn* m, const double* d_r, const double* d_zaj, const double* d_e,
                             float* host_grad, double* loss, void* stream) {
  hofv_status s = need(c, 4, "nn_gradient");
  if (s) return s;
  if (!m || !d_r || !d_zaj || !d_e || !host_grad) return fail(c, HOFV_EINVAL, "bad argument");
  if ((s = set_device(c))) return s;
  hipStream_t st = (hipStream_t)stream;
  if (nn_zero_grad(m, st) || nn_zero_scalar(m->loss, st)) return fail(c, HOFV_EHIP, "zeroing failed");
  if ((s = nn_grad(c, m, d_r, d_zaj, d_e, 1.0f, m->loss, st))) return s;
  double l = 0;
  HOFV_HIP(c, hipMemcpyAsync(&l, m->loss, sizeof(double), hipMemcpyDeviceToHost, st));
  HOFV_HIP(c, hipMemcpyAsync(host_grad, m->g, kNnParams * 4, hipMemcpyDeviceToHost, st));
  HOFV_HIP(c, hipStreamSynchronize(st));
  if (loss) *loss = l;
  return HOFV_OK;
}

hofv_status hofv_nn_forward(hofv_ctx* c, hofv_nn* m, const double* d_r, const double* d_zaj, double* d_z,
                            void* stream) {
  hofv_status s = need(c, 4, "nn_forward");
  if (s) return s;
  if (!m || !d_r || !d_zaj || !d_z) return fail(c, HOFV_EINVAL, "bad argument");
  if ((s = set_device(c))) return s;
  return nn_apply(c, m, d_r, d_zaj, d_z, (hipStream_t)stream);
}

hofv_status hofv_set_timing(hofv_ctx* c, int32_t enable) {
  if (!c) return fail(nullptr, HOFV_EINVAL, "null context");
  if (c->device >= 0) hipDeviceSynchronize();
  c->timers.clear();
  c->ev_used = 0;
  c->timing = enable != 0;
  c->timing_only.clear();
  return HOFV_OK;
}

hofv_status hofv_set_timing_only(hofv_ctx* c, const char* name) {
  hofv_status s = hofv_set_timing(c, 1);
  if (s) return s;
  if (name) c->timing_only = name;
  return HOFV_OK;
}

hofv_status hofv_kernel_time(hofv_ctx* c, const char* name, double* total_ms, int64_t* count) {
  if (!c || !name) return fail(c, HOFV_EINVAL, "null argument");
  double tot = 0;
  int64_t n = 0;
  for (auto& t : c->timers) {
    if (t.name != name) continue;
    HOFV_HIP(c, hipEventSynchronize(t.stop));
    float ms = 0;
    HOFV_HIP(c, hipEventElapsedTime(&ms, t.start, t.stop));
    tot += ms;
    ++n;
  }
  if (total_ms) *total_ms = tot;
  if (count) *count = n;
  return HOFV_OK;
}

hofv_status hofv_kernel_bytes(hofv_ctx* c, const char* name, double* bytes) {
  if (!c || !name || !bytes) return fail(c, HOFV_EINVAL, "null argument");
  auto it = c->kernel_bytes.find(name);
  if (it == c->kernel_bytes.end()) return fail(c, HOFV_EINVAL, std::string("no byte model for ") + name);
  *bytes = it->second;
  return HOFV_OK;
}

}  // extern "C"
