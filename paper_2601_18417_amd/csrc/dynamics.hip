// BDF2 dynamics (App. D) with one integration point per cell, the centroid.
//
// With velocity v = du/dt and acceleration both taken by BDF2,
//   v^{t+1} = (3 u^{t+1} - 4 u^t + u^{t-1}) / (2 dt),
//   a^{t+1} = (3 v^{t+1} - 4 v^t + v^{t-1}) / (2 dt),
// the inertia term rho a Omega_P of cell P is, in u_P = u^{t+1}_P,
//   rho Omega_P a = m_P u_P - s_P,   m_P = 9 rho Omega_P / (4 dt^2),
//   s_P = -rho Omega_P (3 (-4 u^t + u^{t-1}) / (2 dt) - 4 v^t + v^{t-1}) / (2 dt),
// and the dynamic residual is R_P(u) + s_P - m_P u_P (the cell-sum kernel adds
// it).  The compact approximate Jacobian gains the same -m_P on its diagonal.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "common.h"

namespace hofv {

hofv_status newton_impl(hofv_ctx* c, double* u, const hofv_newton_opts* o, hofv_newton_stats* stats,
                        hipStream_t st);

namespace {

constexpr int kB = 256;

inline unsigned nblk(int64_t n) { return (unsigned)((n + kB - 1) / kB); }

// s = -rho vol (3 (-4 u_t + u_tm1) / (2 dt) - 4 v_t + v_tm1) / (2 dt), n = D nc entries
__global__ __launch_bounds__(kB) void k_dyn_source(int64_t nc, int D, const double* __restrict__ rv, double dt,
                                                   const double* __restrict__ ut, const double* __restrict__ utm1,
                                                   const double* __restrict__ vt, const double* __restrict__ vtm1,
                                                   double* __restrict__ s) {
  const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (i >= (int64_t)D * nc) return;
  const double h = 0.5 / dt;
  s[i] = -rv[i % nc] * ((3.0 * (-4.0 * ut[i] + utm1[i]) * h - 4.0 * vt[i] + vtm1[i]) * h);
}

// history after a step to u: v_new = (3 u - 4 u_t + u_tm1) / (2 dt), then shift
__global__ __launch_bounds__(kB) void k_dyn_advance(int64_t n, double dt, const double* __restrict__ u,
                                                    double* __restrict__ ut, double* __restrict__ utm1,
                                                    double* __restrict__ vt, double* __restrict__ vtm1) {
  const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (i >= n) return;
  const double un = u[i], a = ut[i], b = utm1[i], va = vt[i];
  const double vn = (3.0 * un - 4.0 * a + b) * (0.5 / dt);
  utm1[i] = a;
  ut[i] = un;
  vtm1[i] = va;
  vt[i] = vn;
}

}  // namespace

hofv_status dyn_set(hofv_ctx* c, double rho, double dt) {
  DeviceTables& t = c->dev;
  const int64_t nc = c->nc, n = (int64_t)c->D * nc;
  const bool on = rho > 0.0;
  if (on && !(dt > 0.0 && std::isfinite(dt) && std::isfinite(rho)))
    return fail(c, HOFV_EINVAL, "dynamics need rho > 0 and dt > 0");
  std::vector<double> m(nc, 0.0), rv(nc, 0.0);
  if (on)
    for (int64_t P = 0; P < nc; ++P) {
      rv[P] = rho * c->vol[P];
      m[P] = 9.0 * rv[P] / (4.0 * dt * dt);
    }
  // the sweeps' diagonal: A_PP - m_P by sweep position
  std::vector<float> pd(nc), pdinv(nc);
  for (int64_t i = 0; i < nc; ++i) {
    const double d = c->pc_diag[i] - m[c->pc_perm[i]];
    pd[i] = (float)d;
    pdinv[i] = (float)(1.0 / d);
  }
  HOFV_HIP(c, hipMemcpy(t.p_diag, pd.data(), nc * sizeof(float), hipMemcpyHostToDevice));
  HOFV_HIP(c, hipMemcpy(t.p_dinv, pdinv.data(), nc * sizeof(float), hipMemcpyHostToDevice));
  if (!on) {
    t.dyn_m = nullptr;  // the buffers stay allocated for a later call
    c->dyn_rho = c->dyn_dt = 0.0;
    c->dyn_ready = false;
    return HOFV_OK;
  }
  hofv_status s;
  if (!t.dyn_rv) {
    double* mm = nullptr;
    if ((s = dev_alloc(c, &t.dyn_rv, nc)) || (s = dev_alloc(c, &mm, nc)) || (s = dev_alloc(c, &t.dyn_s, n)) ||
        (s = dev_alloc(c, &t.dyn_ut, n)) || (s = dev_alloc(c, &t.dyn_utm1, n)) || (s = dev_alloc(c, &t.dyn_vt, n)) ||
        (s = dev_alloc(c, &t.dyn_vtm1, n)))
      return s;
    t.dyn_m_buf = mm;
  }
  HOFV_HIP(c, hipMemcpy(t.dyn_rv, rv.data(), nc * sizeof(double), hipMemcpyHostToDevice));
  HOFV_HIP(c, hipMemcpy(t.dyn_m_buf, m.data(), nc * sizeof(double), hipMemcpyHostToDevice));
  HOFV_HIP(c, hipMemset(t.dyn_s, 0, n * sizeof(double)));
  t.dyn_m = t.dyn_m_buf;
  c->use_mg = false;  // the hierarchy is built for the static operator
  c->dyn_rho = rho;
  c->dyn_dt = dt;
  c->dyn_ready = false;
  return HOFV_OK;
}

hofv_status dyn_reset(hofv_ctx* c, const double* u_t, const double* u_tm1, const double* v_t, const double* v_tm1,
                      hipStream_t st) {
  DeviceTables& t = c->dev;
  if (!t.dyn_m) return fail(c, HOFV_ESTATE, "dyn_reset without hofv_set_dynamics");
  const int64_t n = (int64_t)c->D * c->nc;
  const size_t bytes = n * sizeof(double);
  HOFV_HIP(c, hipMemcpyAsync(t.dyn_ut, u_t, bytes, hipMemcpyDeviceToDevice, st));
  HOFV_HIP(c, hipMemcpyAsync(t.dyn_utm1, u_tm1, bytes, hipMemcpyDeviceToDevice, st));
  HOFV_HIP(c, hipMemcpyAsync(t.dyn_vt, v_t, bytes, hipMemcpyDeviceToDevice, st));
  HOFV_HIP(c, hipMemcpyAsync(t.dyn_vtm1, v_tm1, bytes, hipMemcpyDeviceToDevice, st));
  k_dyn_source<<<nblk(n), kB, 0, st>>>(c->nc, c->D, t.dyn_rv, c->dyn_dt, t.dyn_ut, t.dyn_utm1, t.dyn_vt, t.dyn_vtm1,
                                       t.dyn_s);
  HOFV_HIP(c, hipGetLastError());
  HOFV_HIP(c, hipStreamSynchronize(st));
  c->dyn_ready = true;
  return HOFV_OK;
}

hofv_status dyn_step(hofv_ctx* c, double* u, const hofv_newton_opts* o, hofv_newton_stats* stats, hipStream_t st) {
  DeviceTables& t = c->dev;
  if (!t.dyn_m || !c->dyn_ready) return fail(c, HOFV_ESTATE, "dyn_step needs hofv_set_dynamics and hofv_dyn_reset");
  const int64_t n = (int64_t)c->D * c->nc;
  hofv_newton_opts one = *o;
  one.n_increments = 0;  // the step is solved at the current load factor
  one.predictor = 0;
  const hofv_status s = newton_impl(c, u, &one, stats, st);
  if (s != HOFV_OK) return s;  // the history stays at the last accepted step
  k_dyn_advance<<<nblk(n), kB, 0, st>>>(n, c->dyn_dt, u, t.dyn_ut, t.dyn_utm1, t.dyn_vt, t.dyn_vtm1);
  k_dyn_source<<<nblk(n), kB, 0, st>>>(c->nc, c->D, t.dyn_rv, c->dyn_dt, t.dyn_ut, t.dyn_utm1, t.dyn_vt, t.dyn_vtm1,
                                       t.dyn_s);
  HOFV_HIP(c, hipGetLastError());
  HOFV_HIP(c, hipStreamSynchronize(st));
  return HOFV_OK;
}

}  // namespace hofv
