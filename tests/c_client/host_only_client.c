/* A plain C11 client of the C ABI: a host-only context (no GPU), a 6 x 5 quad
 * mesh of the unit square, displacement boundaries, setup, the centroids, and
 * a hot call refused on a host-only context.  tests/test_c_client.py builds it
 * with gcc against include/hofv.h and libhofv.so and checks its output. */
#include <stdio.h>
#include <string.h>
#include "hofv.h"

#define CHECK(call)                                                            \
  do {                                                                         \
    hofv_status s_ = (call);                                                   \
    if (s_ != HOFV_OK) {                                                       \
      printf("FAIL %s: %d %s\n", #call, (int)s_, hofv_last_error(ctx));       \
      return 1;                                                                \
    }                                                                          \
  } while (0)

int main(void) {
  enum { NX = 6, NY = 5, NV = (NX + 1) * (NY + 1), NC = NX * NY };
  hofv_params p;
  memset(&p, 0, sizeof p);
  p.dim = 2;
  p.order_p = 2;
  p.n_plus = 10;
  p.n_gauss = 2;
  p.material = HOFV_LINEAR_ELASTIC;
  p.fold_quadrature = 1;
  p.mu = 0.3846153846153846;
  p.lambda = 0.5769230769230769;
  p.alpha = 0.1;
  p.k_weight = 6.0;
  p.ghost_weight = 1.0;
  p.stencil_quantum = 1e-9;
  p.host_only = 1;
  p.precond_levels = 1;
  hofv_ctx* ctx = NULL;
  if (hofv_create(&p, &ctx) != HOFV_OK) {
    printf("FAIL create: %s\n", hofv_last_error(NULL));
    return 1;
  }
  double verts[NV * 2];
  int64_t cells[NC * 4];
  for (int j = 0; j <= NY; ++j)
    for (int i = 0; i <= NX; ++i) {
      verts[2 * (j * (NX + 1) + i)] = (double)i / NX;
      verts[2 * (j * (NX + 1) + i) + 1] = (double)j / NY;
    }
  for (int j = 0; j < NY; ++j)
    for (int i = 0; i < NX; ++i) {
      int64_t* c = &cells[4 * (j * NX + i)];
      c[0] = j * (NX + 1) + i;
      c[1] = c[0] + 1;
      c[2] = c[1] + NX + 1;
      c[3] = c[0] + NX + 1;
    }
  CHECK(hofv_set_mesh(ctx, NV, verts, NC, cells));
  int64_t nb = 0;
  int32_t nq = 0;
  const double *bc, *bn, *bq;
  CHECK(hofv_boundary_faces(ctx, &nb, &nq, &bc, &bn, &bq));
  int32_t type[64];
  if (nb > 64) return 2;
  for (int64_t b = 0; b < nb; ++b) type[b] = HOFV_BC_DISPLACEMENT;
  CHECK(hofv_set_bc(ctx, type, NULL, NULL, NULL));
  CHECK(hofv_set_body_force(ctx, NULL));
  hofv_setup_report rep;
  CHECK(hofv_setup(ctx, &rep));
  const double* cen = NULL;
  CHECK(hofv_cell_centroids(ctx, &cen));
  const hofv_status hot = hofv_residual(ctx, NULL, NULL, NULL);
  printf("boundary %lld nq %d stencil %d internal %lld centroid %.6f %.6f hot %d\n", (long long)nb, (int)nq,
         (int)rep.stencil_size, (long long)rep.n_internal_faces, cen[0], cen[1], (int)hot);
  return hofv_destroy(ctx) == HOFV_OK ? 0 : 3;
}
