// Krylov and Newton drivers on one HIP stream.
//
// FGMRES(m) with right preconditioning (Saad's flexible variant) and
// classical Gram-Schmidt applied twice: per iteration z_j = M(v_j),
// w = J z_j (finite-difference product), h = V^T w and w -= V h twice,
// v_{j+1} = w / ||w||.  Hessenberg columns stay on the device; the host reads
// them every kCheck iterations and applies the Givens rotations, so the GPU
// does not wait for the host between iterations.
// Dot products are deterministic: fixed block partials reduced in fixed order.
//
// Newton (Sec. 4.1 with the Armijo backtracking reading of the line search):
// per load increment, J du = -R by FGMRES, u += lam du with lam = 1, 1/2, ...
// accepted at ||R(u + lam du)|| <= (1 - 1e-4 lam) ||R(u)||; or full steps
// (lam = 1 unless the trial state is inadmissible).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"
#include "givens.h"
#include "reduce.h"

namespace hofv {

namespace {

constexpr int kB = 256;
constexpr int kDotChunk = kGsChunk;  // vectors per multi-dot launch (accumulators in registers)
constexpr int kMaxRestart = 2048;  // longest FGMRES cycle (slender bodies need long Krylov bases)
constexpr int kCheck = 8;         // FGMRES iterations queued between host reads
constexpr double kLearnedCycle = 0.75;  // slowest accepted residual reduction of a learned cycle
constexpr double kStallCycle = 0.99;    // a plain cycle keeping more of the residual ends the solve
// device scalars of the Krylov driver (K.h): Hessenberg column, ||z||^2 of a
// learned output, the cycle's beta, the second Gram-Schmidt pass, a norm
constexpr int kHcol = 0, kZz = kMaxRestart + 2, kBeta = kMaxRestart + 3, kH2 = kMaxRestart + 4,
              kNorm = 2 * kMaxRestart + 6, kHsize = 2 * kMaxRestart + 8;

inline unsigned nblk(int64_t n) { return (unsigned)((n + kB - 1) / kB); }

// ---- grid-wide sums ----------------------------------------------------------
// A grid-wide sum is done in two fixed-order stages: each of nb <= kRedParts
// blocks reduces its elements (wavefront butterflies, then its wavefronts in
// order; reduce.h) to one partial per value, part[i * kRedParts + block]; the
// consumer of the sum (the next kernel) adds the partials of every block in
// the same fixed order, so all its blocks agree on the total bit for bit.

// Threads per block of the streaming Krylov kernels.  The grid has at most
// kRedParts blocks (one partial each), so 256-thread blocks would leave two
// waves per SIMD; 1024-thread blocks keep enough loads in flight where the
// registers allow (the 32-vector fused pass needs about 210 VGPRs and keeps 256).
constexpr int kDotT = 1024;
template <int NV>
constexpr int gs_threads() { return NV <= 16 ? 1024 : kB; }

// partials of sum_l V_i[l] w[l], i < nv <= NV
template <int NV>
__global__ __launch_bounds__(kDotT) void k_dot(int64_t n, int nv, const double* __restrict__ V, int64_t ld,
                                               const double* __restrict__ w, double* __restrict__ part) {
  __shared__ double sred[(kDotT / 64) * NV], sout[NV];
  double acc[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = 0.0;
  for (int64_t l = (int64_t)blockIdx.x * kDotT + threadIdx.x; l < n; l += (int64_t)gridDim.x * kDotT) {
    const double x = w[l];
#pragma unroll
    for (int i = 0; i < NV; ++i)
      if (i < nv) acc[i] += V[(int64_t)i * ld + l] * x;
  }
  block_reduce<NV, kDotT>(acc, sred, sout);
  if ((int)threadIdx.x < nv) part[(int64_t)threadIdx.x * kRedParts + blockIdx.x] = sout[threadIdx.x];
}

// out[i] = sum over the nb (<= kRedParts) partials of value i, for every
// thread of an NT-thread block (thread t adds partials t, t + NT, ... in
// that order, then the block reduces in its fixed order)
template <int NV, int NT>
__device__ __attribute__((always_inline)) inline void reduce_parts(int nb, int nv, const double* __restrict__ part, double* sred, double* out) {
  static_assert(NT * 2 >= kRedParts, "at most two partials per thread");
  double a[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double s = 0.0;
    if (i < nv) {
      const int t = threadIdx.x;
      if (t < nb) s = part[(int64_t)i * kRedParts + t];
      if (t + NT < nb) s += part[(int64_t)i * kRedParts + t + NT];
    }
    a[i] = s;
  }
  block_reduce<NV, NT>(a, sred, out);
}

// out[i] (+)= the total of value i, i < nv (one block)
template <int NV>
__global__ __launch_bounds__(kB) void k_dot_final(int nb, int nv, const double* __restrict__ part,
                                                  double* __restrict__ out, int accumulate) {
  __shared__ double sred[(kB / 64) * NV], sout[NV];
  reduce_parts<NV, kB>(nb, nv, part, sred, sout);
  if ((int)threadIdx.x < nv) out[threadIdx.x] = accumulate ? out[threadIdx.x] + sout[threadIdx.x] : sout[threadIdx.x];
}

// One fused classical Gram-Schmidt pass: h = the totals of part_in (the
// previous pass's V^T w), w -= V h, and the partials of the new V^T w
// (NORM = 0) or of w.w (NORM = 1) into part_out.  Block 0 stores h at hout.
// Each V_i[l] is read once for both products.
template <int NV, int NORM, int NT = gs_threads<NV>()>
__global__ __launch_bounds__(NT) void k_gs_pass(int64_t n, int nv, const double* __restrict__ V, int64_t ld, int nb_in,
                                                const double* __restrict__ part_in, double* __restrict__ hout,
                                                double* __restrict__ w, double* __restrict__ part_out) {
  constexpr int NO = NORM ? 1 : NV;
  __shared__ double sred[(NT / 64) * NV], h[NV], sout[NO];
  reduce_parts<NV, NT>(nb_in, nv, part_in, sred, h);
  if (blockIdx.x == 0 && (int)threadIdx.x < nv) hout[threadIdx.x] = h[threadIdx.x];
  double acc[NO];
#pragma unroll
  for (int i = 0; i < NO; ++i) acc[i] = 0.0;
  for (int64_t l = (int64_t)blockIdx.x * NT + threadIdx.x; l < n; l += (int64_t)gridDim.x * NT) {
    double vv[NV];
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      vv[i] = i < nv ? V[(int64_t)i * ld + l] : 0.0;
      s += h[i] * vv[i];
    }
    const double x = w[l] - s;
    w[l] = x;
    if constexpr (NORM) {
      acc[0] += x * x;
    } else {
#pragma unroll
      for (int i = 0; i < NV; ++i) acc[i] += vv[i] * x;
    }
  }
  block_reduce<NO, NT>(acc, sred, sout);
  if ((int)threadIdx.x < (NORM ? 1 : nv)) part_out[(int64_t)threadIdx.x * kRedParts + blockIdx.x] = sout[threadIdx.x];
}

// Normalisation closing an Arnoldi step: ||w||^2 = the total of part_norm,
// w /= ||w|| (0 if ||w|| = 0); block 0 writes Hessenberg column j: h_i =
// first + second pass (i <= j), h_{j+1} = ||w||, and zz (a learned output's
// squared norm).
__global__ __launch_bounds__(kDotT) void k_gs_scale(int64_t n, int j, int nb, const double* __restrict__ part_norm,
                                                    double* __restrict__ w, double* __restrict__ hd, int ldh,
                                                    double* __restrict__ H, double* __restrict__ zz, int twice) {
  __shared__ double sred[kDotT / 64], sn[1];
  reduce_parts<1, kDotT>(nb, 1, part_norm, sred, sn);
  const double nrm = sqrt(sn[0]);
  for (int64_t l = (int64_t)blockIdx.x * kDotT + threadIdx.x; l < n; l += (int64_t)gridDim.x * kDotT)
    w[l] = nrm > 0.0 ? w[l] / nrm : 0.0;
  if (blockIdx.x != 0) return;
  for (int i = threadIdx.x; i <= j; i += kDotT) H[(int64_t)j * ldh + i] = twice ? hd[kHcol + i] + hd[kH2 + i] : hd[kHcol + i];
  if (threadIdx.x == 0) {
    hd[kHcol + j + 1] = sn[0];
    H[(int64_t)j * ldh + j + 1] = nrm;
    zz[j] = hd[kZz];
  }
}

// w[l] += sign * sum_i h[i] V_i[l]
__global__ __launch_bounds__(kB) void k_multiaxpy(int64_t n, int nv, const double* __restrict__ V, int64_t ld,
                                                  const double* __restrict__ h, double sign, double* __restrict__ w) {
  const int64_t l = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (l >= n) return;
  double s = 0.0;
  for (int i = 0; i < nv; ++i) s += h[i] * V[(int64_t)i * ld + l];
  w[l] += sign * s;
}

// y = x * (1 / d[0]) if d[0] > 0 (d is a squared norm when sq != 0)
__global__ __launch_bounds__(kB) void k_scale_by(int64_t n, const double* __restrict__ x, const double* __restrict__ d,
                                                 int sq, double* __restrict__ y) {
  const int64_t l = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (l >= n) return;
  const double nrm = sq ? sqrt(d[0]) : d[0];
  y[l] = nrm > 0.0 ? x[l] / nrm : 0.0;
}

__global__ __launch_bounds__(kB) void k_lincomb(int64_t n, double a, const double* __restrict__ x, double b,
                                                const double* __restrict__ y, double* __restrict__ z) {
  const int64_t l = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (l < n) z[l] = a * x[l] + b * y[l];
}

__global__ __launch_bounds__(kB) void k_fill(int64_t n, double v, double* __restrict__ z) {
  const int64_t l = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (l < n) z[l] = v;
}

__global__ __launch_bounds__(kB) void k_fill_i(int n, int v, int32_t* __restrict__ z) {
  const int l = blockIdx.x * kB + threadIdx.x;
  if (l < n) z[l] = v;
}

}  // namespace

// template argument for nv values: the smallest power of two >= nv (<= kGsChunk)
#define HOFV_NV_DISPATCH(nv, CALL) \
  do {                             \
    if ((nv) <= 1) { constexpr int NVT = 1; CALL; }        \
    else if ((nv) <= 2) { constexpr int NVT = 2; CALL; }   \
    else if ((nv) <= 4) { constexpr int NVT = 4; CALL; }   \
    else if ((nv) <= 8) { constexpr int NVT = 8; CALL; }   \
    else if ((nv) <= 16) { constexpr int NVT = 16; CALL; } \
    else { constexpr int NVT = 32; CALL; }                 \
  } while (0)

static int red_blocks(int64_t n) { return (int)std::min<int64_t>(kRedParts, nblk(n)); }

// dots of x against nv rows of V (stride ld), kDotChunk rows per pass; result
// on device in out[0..nv)
static hofv_status dots(hofv_ctx* c, int64_t n, int nv, const double* V, int64_t ld, const double* x, double* out,
                        int accumulate, hipStream_t st) {
  const int nb = red_blocks(n);
  double* part = c->dev.part;
  for (int c0 = 0; c0 < nv; c0 += kDotChunk) {
    const int nvc = std::min(kDotChunk, nv - c0);
    HOFV_NV_DISPATCH(nvc, (k_dot<NVT><<<nb, kDotT, 0, st>>>(n, nvc, V + (int64_t)c0 * ld, ld, x, part),
                           k_dot_final<NVT><<<1, kB, 0, st>>>(nb, nvc, part, out + c0, accumulate)));
  }
  HOFV_HIP(c, hipGetLastError());
  return HOFV_OK;
}

// Arnoldi step j: w (= J z_j) is orthogonalised against V_0..V_j by classical
// Gram-Schmidt applied twice (or once, passes = 1) and normalised; Hessenberg column j goes to
// H[j ldh ..] (h_i = first + second pass), the Gram-Schmidt scalars to hd.
// Up to kGsChunk basis vectors the passes are fused (dot; axpy + dot;
// axpy + norm; scale: four launches, the basis read three times); longer
// bases take chunked dots and separate axpys.
static hofv_status cgs2(hofv_ctx* c, int64_t n, int j, const double* V, double* w, double* hd, double* H, int ldh,
                        double* zz, hipStream_t st, int passes = 2) {
  const int nv = j + 1, nb = red_blocks(n);
  double* pA = c->dev.part;
  double* pB = pA + (size_t)kGsChunk * kRedParts;
  double* pC = pB + (size_t)kGsChunk * kRedParts;
  if (nv <= kGsChunk && passes == 2) {
    HOFV_NV_DISPATCH(nv, (k_dot<NVT><<<nb, kDotT, 0, st>>>(n, nv, V, n, w, pA),
                          k_gs_pass<NVT, 0><<<nb, gs_threads<NVT>(), 0, st>>>(n, nv, V, n, nb, pA, hd + kHcol, w, pB),
                          k_gs_pass<NVT, 1><<<nb, gs_threads<NVT>(), 0, st>>>(n, nv, V, n, nb, pB, hd + kH2, w, pC)));
  } else if (nv <= kGsChunk) {  // one pass: dot; axpy + norm
    HOFV_NV_DISPATCH(nv, (k_dot<NVT><<<nb, kDotT, 0, st>>>(n, nv, V, n, w, pA),
                          k_gs_pass<NVT, 1><<<nb, gs_threads<NVT>(), 0, st>>>(n, nv, V, n, nb, pA, hd + kHcol, w, pC)));
  } else {
    hofv_status s;
    if ((s = dots(c, n, nv, V, n, w, hd + kHcol, 0, st))) return s;
    k_multiaxpy<<<nblk(n), kB, 0, st>>>(n, nv, V, n, hd + kHcol, -1.0, w);
    if (passes == 2) {
      if ((s = dots(c, n, nv, V, n, w, hd + kH2, 0, st))) return s;
      k_multiaxpy<<<nblk(n), kB, 0, st>>>(n, nv, V, n, hd + kH2, -1.0, w);
    }
    k_dot<1><<<nb, kDotT, 0, st>>>(n, 1, w, n, w, pC);
  }
  k_gs_scale<<<nb, kDotT, 0, st>>>(n, j, nb, pC, w, hd, ldh, H, zz, passes == 2);
  HOFV_HIP(c, hipGetLastError());
  return HOFV_OK;
}

static hofv_status host_norm(hofv_ctx* c, int64_t n, const double* x, double* out, hipStream_t st) {
  hofv_status s = dots(c, n, 1, x, n, x, c->kry.h + kNorm, 0, st);
  if (s) return s;
  double v;
  HOFV_HIP(c, hipMemcpyAsync(&v, c->kry.h + kNorm, sizeof(double), hipMemcpyDeviceToHost, st));
  HOFV_HIP(c, hipStreamSynchronize(st));
  *out = std::sqrt(v);
  return HOFV_OK;
}

static hofv_status ensure_krylov(hofv_ctx* c, int m) {
  Krylov& k = c->kry;
  if (k.V && k.m >= m) return HOFV_OK;
  const int64_t n = (int64_t)c->D * c->nc;
  if (k.V) {  // grow: release the old set
    for (void* p : {(void*)k.V, (void*)k.Z, (void*)k.Hd, (void*)k.zz}) {
      hipFree(p);
      c->allocations.erase(std::remove(c->allocations.begin(), c->allocations.end(), p), c->allocations.end());
    }
    c->device_bytes -= ((size_t)(2 * k.m + 1) * n + (size_t)(k.m + 2) * k.m) * sizeof(double);
    k.V = k.Z = k.Hd = k.zz = nullptr;
    k.m = 0;
  }
  hofv_status s;
  if ((s = dev_alloc(c, &k.V, (size_t)(m + 1) * n))) return s;
  if ((s = dev_alloc(c, &k.Z, (size_t)m * n))) return s;
  if ((s = dev_alloc(c, &k.Hd, (size_t)(m + 1) * m))) return s;
  if ((s = dev_alloc(c, &k.zz, (size_t)m))) return s;
  if (!k.h) {
    if ((s = dev_alloc(c, &k.h, kHsize))) return s;
    if ((s = dev_alloc(c, &k.tmp, (size_t)n))) return s;
    if ((s = dev_alloc(c, &k.tmp2, (size_t)n))) return s;
  }
  k.m = m;
  return HOFV_OK;
}

hofv_status jvp_impl(hofv_ctx* c, const double* u, const double* Ru, const double* v, double* Jv, double eps,
                     hipStream_t st);
hofv_status precond_dispatch(hofv_ctx* c, const double* r, double* z, int sweeps, int learned, hipStream_t st);

// Captured Arnoldi steps stay valid while the host values their launches hold
// (key) do not change; otherwise they are dropped and captured afresh.
static hofv_status graphs_prepare(hofv_ctx* c, const std::vector<uintptr_t>& key, int m) {
  Krylov& K = c->kry;
  if (!K.cap_stream) HOFV_HIP(c, hipStreamCreateWithFlags(&K.cap_stream, hipStreamNonBlocking));
  if (K.graph_key == key && (int)K.step_graph.size() == m) return HOFV_OK;
  for (hipGraphExec_t g : K.step_graph)
    if (g) HOFV_HIP(c, hipGraphExecDestroy(g));
  K.step_graph.assign(m, nullptr);
  K.step_seen.assign(m, 0);
  K.graph_key = key;
  return HOFV_OK;
}

// Step j launched one by one the first time, captured on the context's
// stream and replayed on st from the second time on.
template <class Step>
static hofv_status graph_step(hofv_ctx* c, int j, Step&& step, hipStream_t st) {
  Krylov& K = c->kry;
  if (!K.step_seen[j]) {
    K.step_seen[j] = 1;
    return step(st);
  }
  if (!K.step_graph[j]) {
    HOFV_HIP(c, hipStreamBeginCapture(K.cap_stream, hipStreamCaptureModeThreadLocal));
    const hofv_status s = step(K.cap_stream);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(K.cap_stream, &g);
    if (s) {
      if (g) hipGraphDestroy(g);
      return s;
    }
    HOFV_HIP(c, e);
    const hipError_t ei = hipGraphInstantiate(&K.step_graph[j], g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    HOFV_HIP(c, ei);
  }
  HOFV_HIP(c, hipGraphLaunch(K.step_graph[j], st));
  return HOFV_OK;
}

hofv_status fgmres_impl(hofv_ctx* c, const double* u, const double* Ru, const double* rhs, double* x,
                        const hofv_krylov_opts* o, hofv_krylov_stats* stats, hipStream_t st) {
  auto t0 = std::chrono::steady_clock::now();
  if (o->restart > kMaxRestart) return fail(c, HOFV_EINVAL, "FGMRES restart above 2048");
  const int m = o->restart > 0 ? o->restart : 30;
  const int maxit = o->max_iters > 0 ? o->max_iters : 1000;
  const double rtol = o->rtol > 0 ? o->rtol : 1e-6;
  const int sweeps = o->n_sweeps > 0 ? o->n_sweeps : 2;
  hofv_status s = ensure_krylov(c, m);
  if (s) return s;
  Krylov& K = c->kry;
  const int64_t n = (int64_t)c->D * c->nc;
  double* hd = K.h;
  double bnorm, xnorm;
  // left preconditioning (eq. jfnk as printed): GMRES on M J x = M rhs, stopping
  // on the preconditioned residual; M must then be one fixed operator
  const bool left = o->side == 1;
  if (left && o->learned) return fail(c, HOFV_EINVAL, "the learned correction needs right preconditioning");
  if (c->nej.k > 0 && (left || o->learned))
    return fail(c, HOFV_EINVAL, "the near-exact Jacobian preconditioner needs right preconditioning, unlearned");
  if (o->side != 0 && o->side != 1) return fail(c, HOFV_EINVAL, "side must be 0 (right) or 1 (left)");
  if (o->gs_passes < 0 || o->gs_passes > 2) return fail(c, HOFV_EINVAL, "gs_passes must be 0, 1 or 2");
  const int passes = o->gs_passes == 1 ? 1 : 2;
  if (o->graphs < 0 || o->graphs > 1) return fail(c, HOFV_EINVAL, "graphs must be 0 or 1");
  const bool graphs = o->graphs == 1 && !left && !o->learned && c->nej.k == 0 && !c->timing;
  if (graphs) {
    uint64_t load_bits;
    std::memcpy(&load_bits, &c->load, sizeof load_bits);
    const std::vector<uintptr_t> key = {(uintptr_t)u, (uintptr_t)Ru, (uintptr_t)K.V, (uintptr_t)K.Z,
                                        (uintptr_t)K.h, (uintptr_t)K.Hd, (uintptr_t)K.zz, (uintptr_t)m,
                                        (uintptr_t)sweeps, (uintptr_t)passes, (uintptr_t)c->use_mg,
                                        (uintptr_t)load_bits, (uintptr_t)c->dev.dyn_m, (uintptr_t)c->dev.dyn_s};
    if ((s = graphs_prepare(c, key, m))) return s;
  }
  if ((s = host_norm(c, n, x, &xnorm, st))) return s;
  if (left) {
    if ((s = precond_dispatch(c, rhs, K.tmp2, sweeps, 0, st))) return s;
    if ((s = host_norm(c, n, K.tmp2, &bnorm, st))) return s;
  } else if ((s = host_norm(c, n, rhs, &bnorm, st))) {
    return s;
  }
  stats->iters = 0;
  stats->converged = 0;
  stats->fallbacks = 0;
  stats->stalled = 0;
  int learned = o->learned;
  if (!std::isfinite(bnorm) || !std::isfinite(xnorm)) return fail(c, HOFV_ENAN, "NaN/Inf in FGMRES input");
  if (bnorm == 0.0) {
    k_fill<<<nblk(n), kB, 0, st>>>(n, 0.0, x);
    stats->converged = 1;
    stats->rel_residual = 0.0;
    HOFV_HIP(c, hipStreamSynchronize(st));
    return HOFV_OK;
  }
  GivensLsq lsq;
  std::vector<double> y(m);
  int it = 0;
  double beta = 0, beta_cycle = -1.0;
  for (;;) {
    // V_0 = rhs - J x (left: M (rhs - J x))
    double* r0 = left ? K.tmp2 : K.V;
    if (xnorm > 0) {
      if ((s = jvp_impl(c, u, Ru, x, K.tmp, 0.0, st))) return s;
      k_lincomb<<<nblk(n), kB, 0, st>>>(n, 1.0, rhs, -1.0, K.tmp, r0);
    } else {
      k_lincomb<<<nblk(n), kB, 0, st>>>(n, 1.0, rhs, 0.0, rhs, r0);
    }
    if (left && (s = precond_dispatch(c, r0, K.V, sweeps, 0, st))) return s;
    if ((s = host_norm(c, n, K.V, &beta, st))) return s;
    if (!std::isfinite(beta)) return fail(c, HOFV_ENAN, "NaN/Inf in the FGMRES residual");
    if (beta <= rtol * bnorm || it >= maxit) break;
    // a learned correction whose last full cycle reduced the residual by less
    // than kLearnedCycle hands the rest of the solve to the plain preconditioner
    if (learned && beta_cycle > 0.0 && beta > kLearnedCycle * beta_cycle) {
      learned = 0;
      ++stats->fallbacks;
    } else if (beta_cycle > 0.0 && beta > kStallCycle * beta_cycle) {
      // the true residual no longer follows the least-squares one (the
      // finite-difference product is linear only to its precision)
      stats->stalled = 1;
      break;
    }
    beta_cycle = beta;
    k_fill<<<1, kB, 0, st>>>(1, beta, hd + kBeta);
    k_scale_by<<<nblk(n), kB, 0, st>>>(n, K.V, hd + kBeta, 0, K.V);
    lsq.reset(m, beta);
    int kdone = 0;
    // Iterations are queued kCheck at a time; their Hessenberg columns stay on
    // the device until the host reads them all at once and applies the Givens
    // rotations.  Columns past the converged one are discarded; a non-finite
    // column (a learned output gone bad) rolls back to that iteration, which
    // is redone with the plain preconditioner.
    int j = 0, jp = 0;  // next iteration to queue / to process on the host
    bool done = false;
    std::vector<double> hblk((size_t)(m + 1) * kCheck), zzb(kCheck);
    while (!done) {
      auto step = [&](hipStream_t q) -> hofv_status {
        double* vj = K.V + (size_t)j * n;
        double* zj = K.Z + (size_t)j * n;
        double* w = K.V + (size_t)(j + 1) * n;
        hofv_status r;
        if (left) {  // w = M J v_j (z_j holds J v_j)
          if ((r = jvp_impl(c, u, Ru, vj, zj, 0.0, q))) return r;
          if ((r = precond_dispatch(c, zj, w, sweeps, 0, q))) return r;
        } else {  // w = J z_j, z_j = M v_j
          if ((r = precond_dispatch(c, vj, zj, sweeps, learned, q))) return r;
          // ||z_j||^2 of a learned output (a NaN z_j would only show up later:
          // its finite-difference product is defined to be zero)
          if (learned && (r = dots(c, n, 1, zj, n, zj, hd + kZz, 0, q))) return r;
          if ((r = jvp_impl(c, u, Ru, zj, w, 0.0, q))) return r;
        }
        return cgs2(c, n, j, K.V, w, hd, K.Hd, m + 1, K.zz, q, passes);
      };
      if ((s = graphs ? graph_step(c, j, step, st) : step(st))) return s;
      ++j;
      if (j - jp < kCheck && j < m && it + (j - jp) < maxit) continue;
      const int nq = j - jp;
      HOFV_HIP(c, hipMemcpyAsync(hblk.data(), K.Hd + (size_t)jp * (m + 1), (size_t)nq * (m + 1) * sizeof(double),
                                 hipMemcpyDeviceToHost, st));
      HOFV_HIP(c, hipMemcpyAsync(zzb.data(), K.zz + jp, nq * sizeof(double), hipMemcpyDeviceToHost, st));
      HOFV_HIP(c, hipStreamSynchronize(st));
      int redo = -1;
      for (int q = 0; q < nq && !done; ++q) {
        const int jj = jp + q;
        const double* col = &hblk[(size_t)q * (m + 1)];
        bool finite = !learned || std::isfinite(zzb[q]);
        for (int i = 0; i <= jj + 1; ++i) finite = finite && std::isfinite(col[i]);
        if (!finite) {
          if (!learned) return fail(c, HOFV_ENAN, "NaN/Inf in Arnoldi");
          learned = 0;  // the plain preconditioner takes over for the rest of the solve
          ++stats->fallbacks;
          redo = jj;
          break;
        }
        if (!lsq.add(col)) {
          // the rotated column is zero: z_j adds no direction.  A learned
          // output redoes the iteration with the plain preconditioner; a plain
          // one ends the cycle with the columns accepted so far
          if (learned) {
            learned = 0;
            ++stats->fallbacks;
            redo = jj;
            break;
          }
          ++it;
          done = true;
          break;
        }
        ++it;
        kdone = lsq.k;
        if (lsq.residual() <= rtol * bnorm || it >= maxit || kdone == m) done = true;
      }
      if (redo >= 0) {
        j = jp = redo;
        continue;
      }
      jp = j;
    }
    lsq.solve(y.data());
    HOFV_HIP(c, hipMemcpyAsync(hd, y.data(), kdone * sizeof(double), hipMemcpyHostToDevice, st));
    k_multiaxpy<<<nblk(n), kB, 0, st>>>(n, kdone, left ? K.V : K.Z, n, hd, 1.0, x);
    HOFV_HIP(c, hipGetLastError());
    xnorm = 1.0;
  }
  stats->iters = it;
  stats->rel_residual = beta / bnorm;
  stats->converged = beta <= rtol * bnorm;
  stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return HOFV_OK;
}

// ---------------------------------------------------------------- near-exact Jacobian

constexpr int kMaxNej = 64;  // longest inner GMRES of the near-exact Jacobian

hofv_status nej_zero(hofv_ctx* c) {
  if (c->nej.zero) return HOFV_OK;
  const size_t nz = std::max<size_t>(c->faces.size(), (size_t)c->D * c->nc);
  hofv_status s = dev_alloc(c, &c->nej.zero, nz);
  if (s) return s;
  HOFV_HIP(c, hipMemset(c->nej.zero, 0, nz * sizeof(double)));
  return HOFV_OK;
}

hofv_status nej_set(hofv_ctx* c, int k) {
  if (k < 0 || k > kMaxNej) return fail(c, HOFV_EINVAL, "near-exact Jacobian inner iterations must be 0..64");
  if (k > 0 && c->prm.material != HOFV_LINEAR_ELASTIC)
    return fail(c, HOFV_EINVAL, "the near-exact Jacobian is defined for the linear elastic law");
  Nej& N = c->nej;
  const int64_t n = (int64_t)c->D * c->nc;
  hofv_status s;
  if (k > N.cap) {
    if (N.V) {  // grow: release the old basis
      for (void* p : {(void*)N.V, (void*)N.Hd, (void*)N.zz, (void*)N.y}) {
        hipFree(p);
        c->allocations.erase(std::remove(c->allocations.begin(), c->allocations.end(), p), c->allocations.end());
      }
      c->device_bytes -= ((size_t)(N.cap + 1) * n + (size_t)(N.cap + 1) * N.cap + 2 * (size_t)N.cap) * sizeof(double);
      N.V = N.Hd = N.zz = N.y = nullptr;
      N.cap = 0;
    }
    if ((s = dev_alloc(c, &N.V, (size_t)(k + 1) * n)) || (s = dev_alloc(c, &N.Hd, (size_t)(k + 1) * k)) ||
        (s = dev_alloc(c, &N.zz, (size_t)k)) || (s = dev_alloc(c, &N.y, (size_t)k)))
      return s;
    N.cap = k;
  }
  if (k > 0 && (s = nej_zero(c))) return s;
  if (k > 0 && !N.t) {
    if ((s = dev_alloc(c, &N.t, (size_t)n)) || (s = dev_alloc(c, &N.h, kHsize))) return s;
  }
  N.k = k;
  return HOFV_OK;
}

// z ~ A^{-1} r for the near-exact Jacobian A: k iterations of GMRES from zero,
// right-preconditioned by the approximate Jacobian M (sweeps or V-cycle), so
// z = M (V_k y) with y minimising ||beta e_1 - H y||.  The Arnoldi vectors use
// the same CGS2 as the outer solver; the host reads the Hessenberg matrix once.
hofv_status nej_solve(hofv_ctx* c, const double* r, double* z, int sweeps, hipStream_t st) {
  Nej& N = c->nej;
  const int k = N.k;
  const int64_t n = (int64_t)c->D * c->nc;
  double* hd = N.h;
  hofv_status s;
  if ((s = dots(c, n, 1, r, n, r, hd + kBeta, 0, st))) return s;
  k_scale_by<<<nblk(n), kB, 0, st>>>(n, r, hd + kBeta, 1, N.V);
  for (int j = 0; j < k; ++j) {
    double* vj = N.V + (size_t)j * n;
    double* w = N.V + (size_t)(j + 1) * n;
    if ((s = launch_precond(c, vj, N.t, sweeps, st))) return s;
    if ((s = launch_nej(c, N.t, w, st))) return s;
    if ((s = cgs2(c, n, j, N.V, w, hd, N.Hd, k + 1, N.zz, st))) return s;
  }
  HOFV_HIP(c, hipGetLastError());
  N.hbuf.resize((size_t)(k + 1) * k + 1);
  HOFV_HIP(c, hipMemcpyAsync(N.hbuf.data(), N.Hd, (size_t)(k + 1) * k * sizeof(double), hipMemcpyDeviceToHost, st));
  HOFV_HIP(c, hipMemcpyAsync(N.hbuf.data() + (size_t)(k + 1) * k, hd + kBeta, sizeof(double), hipMemcpyDeviceToHost,
                             st));
  HOFV_HIP(c, hipStreamSynchronize(st));
  const double beta = std::sqrt(N.hbuf[(size_t)(k + 1) * k]);
  // column j holds rows 0..j+1; the rows below were never written
  bool finite = std::isfinite(beta);
  for (int j = 0; j < k; ++j)
    for (int i = 0; i <= j + 1; ++i) finite = finite && std::isfinite(N.hbuf[(size_t)j * (k + 1) + i]);
  if (!finite) return fail(c, HOFV_ENAN, "NaN/Inf in the near-exact Jacobian solve");
  if (beta == 0.0) {
    k_fill<<<nblk(n), kB, 0, st>>>(n, 0.0, z);
    HOFV_HIP(c, hipGetLastError());
    return HOFV_OK;
  }
  // least squares by Givens rotations; a zero subdiagonal ends the Krylov
  // space there (the solve is exact within it), a zero rotated column is dropped
  GivensLsq lsq;
  lsq.reset(k, beta);
  for (int j = 0; j < k; ++j) {
    const double* col = &N.hbuf[(size_t)j * (k + 1)];
    if (!lsq.add(col) || col[j + 1] == 0.0) break;
  }
  const int kk = lsq.k;
  N.ybuf.assign(k, 0.0);
  lsq.solve(N.ybuf.data());
  HOFV_HIP(c, hipMemcpyAsync(N.y, N.ybuf.data(), (size_t)k * sizeof(double), hipMemcpyHostToDevice, st));
  k_fill<<<nblk(n), kB, 0, st>>>(n, 0.0, N.t);
  k_multiaxpy<<<nblk(n), kB, 0, st>>>(n, kk, N.V, n, N.y, 1.0, N.t);
  HOFV_HIP(c, hipGetLastError());
  s = launch_precond(c, N.t, z, sweeps, st);
  if (s) return s;
  // the host vector y is reused by the next call only after this one has run
  HOFV_HIP(c, hipStreamSynchronize(st));
  return HOFV_OK;
}

hofv_status newton_impl(hofv_ctx* c, double* u, const hofv_newton_opts* o, hofv_newton_stats* stats,
                        hipStream_t st) {
  auto t0 = std::chrono::steady_clock::now();
  const int64_t n = (int64_t)c->D * c->nc;
  if (o->krylov.restart > kMaxRestart) return fail(c, HOFV_EINVAL, "FGMRES restart above 2048");
  hofv_status s = ensure_krylov(c, o->krylov.restart > 0 ? o->krylov.restart : 30);
  if (s) return s;
  // workspace: R, du, rhs, ut, Rt and (secant predictor) the previous
  // increment's converged state; released on every way out
  struct Workspace {
    hofv_ctx* c;
    hipStream_t st;
    std::vector<double*> bufs;
    size_t bytes = 0;
    ~Workspace() {
      (void)hipStreamSynchronize(st);  // an early error return may leave work queued
      for (double* p : bufs) {
        hipFree(p);
        c->allocations.erase(std::remove(c->allocations.begin(), c->allocations.end(), (void*)p),
                             c->allocations.end());
      }
      c->device_bytes -= bytes;
    }
    hofv_status get(double** p, int64_t count) {
      hofv_status s = dev_alloc(c, p, (size_t)count);
      if (s == HOFV_OK) {
        bufs.push_back(*p);
        bytes += (size_t)count * sizeof(double);
      }
      return s;
    }
  } ws{c, st, {}};
  double *R, *du, *rhs, *ut, *Rt, *up = nullptr;
  if ((s = ws.get(&R, n)) || (s = ws.get(&du, n)) || (s = ws.get(&rhs, n)) || (s = ws.get(&ut, n)) ||
      (s = ws.get(&Rt, n)))
    return s;
  // n_increments <= 0: one solve at the load factor set by hofv_set_load_scale
  const int ninc = std::max(1, o->n_increments);
  const bool predict = o->predictor == 1 && ninc > 1;
  if (predict && (s = ws.get(&up, n))) return s;
  const double load0 = c->load;
  const double tol = o->tol > 0 ? o->tol : 1e-8;
  hofv_krylov_opts ko = o->krylov;
  const double eta0 = o->eta > 0 ? o->eta : 1e-4;
  stats->newton_iters = 0;
  stats->krylov_iters = 0;
  stats->converged = 1;
  stats->fallbacks = 0;
  hofv_status result = HOFV_OK;
  for (int inc = 1; inc <= ninc && result == HOFV_OK; ++inc) {
    c->load = o->n_increments > 0 ? (double)inc / ninc : load0;
    if ((s = launch_residual(c, u, R, nullptr, nullptr, st))) { result = s; break; }
    double r0, rn;
    if ((s = host_norm(c, n, R, &r0, st))) { result = s; break; }
    rn = r0;
    if (predict && inc > 1) {
      // start from u_i + (u_i - u_{i-1}) unless that state is inadmissible;
      // r0 stays the residual of u_i at the new load
      k_lincomb<<<nblk(n), kB, 0, st>>>(n, 2.0, u, -1.0, up, ut);
      HOFV_HIP(c, hipMemcpyAsync(up, u, n * sizeof(double), hipMemcpyDeviceToDevice, st));
      k_fill_i<<<1, kB, 0, st>>>(1, 0, c->dev.flag);
      if ((s = launch_residual(c, ut, Rt, nullptr, nullptr, st))) { result = s; break; }
      int32_t flag = 0;
      HOFV_HIP(c, hipMemcpyAsync(&flag, c->dev.flag, sizeof(int32_t), hipMemcpyDeviceToHost, st));
      double rt;
      if ((s = host_norm(c, n, Rt, &rt, st))) { result = s; break; }
      if (!flag && std::isfinite(rt)) {
        HOFV_HIP(c, hipMemcpyAsync(u, ut, n * sizeof(double), hipMemcpyDeviceToDevice, st));
        HOFV_HIP(c, hipMemcpyAsync(R, Rt, n * sizeof(double), hipMemcpyDeviceToDevice, st));
        rn = rt;
      }
    } else if (predict) {
      HOFV_HIP(c, hipMemcpyAsync(up, u, n * sizeof(double), hipMemcpyDeviceToDevice, st));
    }
    int itn = 0;
    double rprev = r0;
    ko.rtol = eta0;
    while (rn > tol * r0 && itn < (o->max_newton > 0 ? o->max_newton : 50)) {
      if (o->forcing == 1 && itn > 0) {
        // Eisenstat-Walker choice 2 (gamma = 0.9, alpha = 2) with their
        // safeguard, at most eta0, and no tighter than the increment's
        // tolerance asks of this step
        const double prev = ko.rtol;
        double e = 0.9 * (rn / rprev) * (rn / rprev);
        if (0.9 * prev * prev > 0.1) e = std::max(e, 0.9 * prev * prev);
        e = std::min(e, eta0);
        ko.rtol = std::max(e, 0.5 * tol * r0 / rn);
      }
      rprev = rn;
      k_lincomb<<<nblk(n), kB, 0, st>>>(n, -1.0, R, 0.0, R, rhs);
      k_fill<<<nblk(n), kB, 0, st>>>(n, 0.0, du);
      hofv_krylov_stats ks{};
      if ((s = fgmres_impl(c, u, R, rhs, du, &ko, &ks, st))) { result = s; break; }
      stats->krylov_iters += ks.iters;
      stats->fallbacks += ks.fallbacks;
      if (ko.learned && !ks.converged) {
        // the learned correction missed the tolerance: redo the step with the plain one
        hofv_krylov_opts kp = ko;
        kp.learned = 0;
        k_fill<<<nblk(n), kB, 0, st>>>(n, 0.0, du);
        if ((s = fgmres_impl(c, u, R, rhs, du, &kp, &ks, st))) { result = s; break; }
        stats->krylov_iters += ks.iters;
        ++stats->fallbacks;
      }
      double lam = 1.0, rt = 0.0;
      bool accepted = false;
      // max_line_search < 0: full steps, halved only while the trial state is
      // not admissible (an inverted cell or a non-finite residual)
      const bool full = o->max_line_search < 0;
      const int maxls = o->max_line_search > 0 ? o->max_line_search : 10;
      for (int ls = 0; ls <= maxls; ++ls) {
        k_lincomb<<<nblk(n), kB, 0, st>>>(n, 1.0, u, lam, du, ut);
        k_fill_i<<<1, kB, 0, st>>>(1, 0, c->dev.flag);
        if ((s = launch_residual(c, ut, Rt, nullptr, nullptr, st))) { result = s; break; }
        int32_t flag = 0;
        HOFV_HIP(c, hipMemcpyAsync(&flag, c->dev.flag, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        if ((s = host_norm(c, n, Rt, &rt, st))) { result = s; break; }
        if (!flag && std::isfinite(rt) && (full || rt <= (1.0 - 1e-4 * lam) * rn)) { accepted = true; break; }
        if (!full && ls == maxls && !flag && std::isfinite(rt)) { accepted = true; break; }  // last trial
        lam *= 0.5;
      }
      if (result) break;
      if (!accepted) { result = fail(c, HOFV_EINVERTED, "line search found no admissible step"); break; }
      HOFV_HIP(c, hipMemcpyAsync(u, ut, n * sizeof(double), hipMemcpyDeviceToDevice, st));
      HOFV_HIP(c, hipMemcpyAsync(R, Rt, n * sizeof(double), hipMemcpyDeviceToDevice, st));
      rn = rt;
      ++itn;
      ++stats->newton_iters;
    }
    stats->rel_residual = r0 > 0 ? rn / r0 : 0.0;
    if (!(rn <= tol * r0)) stats->converged = 0;
  }
  HOFV_HIP(c, hipStreamSynchronize(st));
  stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (result == HOFV_OK && !stats->converged)
    return fail(c, HOFV_ENOCONV, "Newton did not reach the tolerance");
  return result;
}

}  // namespace hofv

namespace hofv {

// ---------------------------------------------------------------- training pairs
// Pairs (r, e) with J e = r for the learned correction, written consecutively
// at r_out / e_out (declared with hofv_harvest_pairs in hofv.h).
hofv_status harvest_impl(hofv_ctx* c, const double* u, const double* starts, const hofv_harvest_opts* o,
                         double* r_out, double* e_out, hipStream_t st) {
  const int64_t n = (int64_t)c->D * c->nc;
  hofv_krylov_opts ko{};
  ko.restart = o->restart > 0 ? o->restart : 30;
  ko.max_iters = o->max_iters > 0 ? o->max_iters : 3000;
  ko.rtol = o->rtol > 0 ? o->rtol : 1e-8;
  ko.n_sweeps = o->n_sweeps > 0 ? o->n_sweeps : 2;
  ko.learned = 0;
  ko.side = 0;
  ko.gs_passes = 0;
  hofv_status s = ensure_krylov(c, ko.restart);
  if (s) return s;
  // workspace: R(u), the current v, M v and the Newton state, released on return
  struct Ws {
    hofv_ctx* c;
    hipStream_t st;
    std::vector<double*> b;
    size_t bytes = 0;
    ~Ws() {
      (void)hipStreamSynchronize(st);
      for (double* p : b) {
        hipFree(p);
        c->allocations.erase(std::remove(c->allocations.begin(), c->allocations.end(), (void*)p),
                             c->allocations.end());
      }
      c->device_bytes -= bytes;
    }
  } ws{c, st, {}};
  double *Ru, *v, *t, *uk;
  for (double** p : {&Ru, &v, &t, &uk}) {
    if ((s = dev_alloc(c, p, (size_t)n))) return s;
    ws.b.push_back(*p);
    ws.bytes += (size_t)n * sizeof(double);
  }
  double* nrm = c->kry.h + kNorm;
  int64_t k = 0;  // pairs written
  hofv_krylov_stats ks{};
  if (o->n_starts > 0 && o->length > 0) {
    if ((s = launch_residual(c, u, Ru, nullptr, nullptr, st))) return s;
    for (int sidx = 0; sidx < o->n_starts; ++sidx) {
      if (starts) {
        HOFV_HIP(c, hipMemcpyAsync(v, starts + (size_t)sidx * n, n * sizeof(double), hipMemcpyDeviceToDevice, st));
      } else if ((s = fill_normal(n, o->seed + ((uint64_t)sidx << 40), v, st))) {
        return fail(c, s, "normal generator launch failed");
      }
      if ((s = dots(c, n, 1, v, n, v, nrm, 0, st))) return s;
      k_scale_by<<<nblk(n), kB, 0, st>>>(n, v, nrm, 1, v);
      for (int l = 0; l < o->length; ++l, ++k) {
        double* rk = r_out + (size_t)k * n;
        double* ek = e_out + (size_t)k * n;
        HOFV_HIP(c, hipMemcpyAsync(rk, v, n * sizeof(double), hipMemcpyDeviceToDevice, st));
        k_fill<<<nblk(n), kB, 0, st>>>(n, 0.0, ek);
        if ((s = fgmres_impl(c, u, Ru, rk, ek, &ko, &ks, st))) return s;
        if ((s = precond_dispatch(c, v, t, ko.n_sweeps, 0, st))) return s;
        if ((s = jvp_impl(c, u, Ru, t, v, 0.0, st))) return s;
        if ((s = dots(c, n, 1, v, n, v, nrm, 0, st))) return s;
        k_scale_by<<<nblk(n), kB, 0, st>>>(n, v, nrm, 1, v);
      }
    }
  }
  if (o->newton_steps > 0) {
    HOFV_HIP(c, hipMemcpyAsync(uk, u, n * sizeof(double), hipMemcpyDeviceToDevice, st));
    for (int it = 0; it < o->newton_steps; ++it, ++k) {
      double* rk = r_out + (size_t)k * n;
      double* ek = e_out + (size_t)k * n;
      if ((s = launch_residual(c, uk, Ru, nullptr, nullptr, st))) return s;
      k_fill<<<nblk(n), kB, 0, st>>>(n, 0.0, ek);
      if ((s = fgmres_impl(c, uk, Ru, Ru, ek, &ko, &ks, st))) return s;
      // u_{k+1} = u_k - e_k, then (R, e) / ||R||
      k_lincomb<<<nblk(n), kB, 0, st>>>(n, 1.0, uk, -1.0, ek, uk);
      if ((s = dots(c, n, 1, Ru, n, Ru, nrm, 0, st))) return s;
      k_scale_by<<<nblk(n), kB, 0, st>>>(n, Ru, nrm, 1, rk);
      k_scale_by<<<nblk(n), kB, 0, st>>>(n, ek, nrm, 1, ek);
    }
  }
  HOFV_HIP(c, hipGetLastError());
  HOFV_HIP(c, hipStreamSynchronize(st));
  return HOFV_OK;
}

}  // namespace hofv
