/* A plain C11 client of the C ABI on the GPU, without Python or torch: the
 * problem of host_only_client.c on a device context, u = (x^2, x y) at the
 * cell centroids copied to device memory it allocates itself, one residual
 * on the default stream, and R printed component-major.  tests/test_c_client.py
 * builds it with gcc against include/hofv.h, libhofv.so and the HIP runtime,
 * runs it and compares R with the oracle's. */
#include <hip/hip_runtime_api.h>
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
#define HIP(call)                                                              \
  do {                                                                         \
    if ((call) != hipSuccess) {                                                \
      printf("FAIL %s\n", #call);                                              \
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
  double u[2 * NC], R[2 * NC];
  for (int c = 0; c < NC; ++c) {
    u[c] = cen[2 * c] * cen[2 * c];
    u[NC + c] = cen[2 * c] * cen[2 * c + 1];
  }
  double *du = NULL, *dR = NULL;
  HIP(hipMalloc((void**)&du, sizeof u));
  HIP(hipMalloc((void**)&dR, sizeof R));
  HIP(hipMemcpy(du, u, sizeof u, hipMemcpyHostToDevice));
  CHECK(hofv_residual(ctx, du, dR, NULL));
  HIP(hipDeviceSynchronize());
  HIP(hipMemcpy(R, dR, sizeof R, hipMemcpyDeviceToHost));
  for (int k = 0; k < 2 * NC; ++k) printf("%.17g\n", R[k]);
  HIP(hipFree(du));
  HIP(hipFree(dR));
  return hofv_destroy(ctx) == HOFV_OK ? 0 : 3;
}
