// Learned correction of the compact preconditioner: a message-passing network
// over face neighbours, trained and run on the GPU.
//
//   x_P = [r_P / s_r, z_P / s_z, b_P, 1]              (z = plain preconditioner output)
//   h0  = relu(x We + be)                              (8 -> 64, FP32 FMA)
//   4 x: X = [h, A0, A1, A2, A3], A0 = sum_N om h_N, Ad = sum_N om e_d h_N
//        h <- h + relu(X W_l + b_l)                    (320 -> 64, BF16 MFMA, FP32 accumulate)
//   g   = h Wd + bd                                     (64 -> 3, FP32 FMA)
//   z'  = z + s_z g                                     (FP64 out)
// Training: loss ||z' - e||^2 / ||e||^2 per pair, hand-written backward
// (dX = dY W^T and dW = X^T dY on BF16 MFMA, the aggregation's transpose as a
// gather), Adam on FP32 master weights with BF16 copies for the products.
//
// MFMA v_mfma_f32_16x16x32_bf16 (gfx950): lane i holds A[i%16][8(i/16)..+7],
// B[8(i/16)..+7][i%16] and accumulates C[4(i/16)+j][i%16], j < 4.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"
#include "mpnn.h"

namespace hofv {

namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned short us8 __attribute__((ext_vector_type(8)));

constexpr int kW = kNnWidth;     // 64
constexpr int kK = 5 * kNnWidth; // 320
constexpr int kB = 256;

inline unsigned nblk(int64_t n, int per = kB) { return (unsigned)((n + per - 1) / per); }

// float -> bfloat16, round to nearest even (gfx950 converts natively)
__device__ inline unsigned short f2bf(float f) { return __builtin_bit_cast(unsigned short, (__bf16)f); }
__device__ inline float bf2f(unsigned short b) { return __uint_as_float((uint32_t)b << 16); }

__device__ inline bf8 as_bf8(us8 v) { return __builtin_bit_cast(bf8, v); }

// ---- features ---------------------------------------------------------------

// s[0] = sum r^2, s[1] = sum z^2 partials -> rms in s[2], s[3]; s[4] = sum e^2
template <int D>
__global__ __launch_bounds__(kB) void k_nn_features(int64_t nc, const double* __restrict__ r,
                                                    const double* __restrict__ z, const float* __restrict__ bflag,
                                                    const double* __restrict__ sc, unsigned short* __restrict__ x) {
  const int64_t P = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (P >= nc) return;
  const double ir = sc[2] > 0 ? 1.0 / sc[2] : 0.0, iz = sc[3] > 0 ? 1.0 / sc[3] : 0.0;
  unsigned short v[8];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    v[c] = f2bf(c < D ? (float)(r[(int64_t)c * nc + P] * ir) : 0.0f);
    v[3 + c] = f2bf(c < D ? (float)(z[(int64_t)c * nc + P] * iz) : 0.0f);
  }
  v[6] = f2bf(bflag[P]);
  v[7] = f2bf(1.0f);
#pragma unroll
  for (int j = 0; j < 8; ++j) x[P * 8 + j] = v[j];
}

// ---- encoder ------------------------------------------------------------------

__global__ __launch_bounds__(kB) void k_nn_encoder(int64_t nc, const unsigned short* __restrict__ x,
                                                   const unsigned short* __restrict__ We /*[8][64] bf16*/,
                                                   const float* __restrict__ be, unsigned short* __restrict__ h) {
  __shared__ float sWe[8 * kW + kW];
  for (int i = threadIdx.x; i < 8 * kW; i += kB) sWe[i] = bf2f(We[i]);
  for (int i = threadIdx.x; i < kW; i += kB) sWe[8 * kW + i] = be[i];
  __syncthreads();
  const int64_t P = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (P >= nc) return;
  const us8 xv = *reinterpret_cast<const us8*>(x + P * 8);
  float xf[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) xf[j] = bf2f(xv[j]);
#pragma unroll
  for (int c8 = 0; c8 < kW / 8; ++c8) {
    us8 o;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int c = 8 * c8 + q;
      float s = sWe[8 * kW + c];
#pragma unroll
      for (int j = 0; j < 8; ++j) s += xf[j] * sWe[j * kW + c];
      o[q] = f2bf(fmaxf(s, 0.0f));
    }
    *reinterpret_cast<us8*>(h + P * kW + 8 * c8) = o;
  }
}

// ---- message-passing layer, forward -----------------------------------------
// A block stages the layer's transposed BF16 weights Wt[64][320] in LDS once
// (rows padded to 328 entries against bank conflicts); its 8 wavefronts then
// run kNnTiles tiles of 16 cells each.  The product is computed transposed,
// Y^T = W^T X^T: the A operand is a 16-channel slice of Wt (from LDS) and the
// B operand the 16 cells' X (lane i: cell i%16, k-octet i/16), built from h
// and from aggregates gathered in registers and rounded to BF16.  The
// accumulator of lane i then holds channels 16 t + 4 (i/16) + j of cell i%16,
// so the epilogue moves 4 consecutive channels (8 bytes) per load/store.
constexpr int kNnTiles = 2;
constexpr int kWtPad = kK + 8;
constexpr int kLayerThreads = 512;
constexpr int kLayerWaves = kLayerThreads / 64;
constexpr int kLayerCells = kLayerWaves * 16 * kNnTiles;  // cells per block

typedef unsigned short us4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kLayerThreads) void k_nn_layer(
    int64_t nc, const unsigned short* __restrict__ h, const int32_t* __restrict__ nbr /*[2D][nc]*/,
    const float4* __restrict__ wf /*[2D][nc]*/, int NS, const unsigned short* __restrict__ Wt /*[64][320]*/,
    const float* __restrict__ b, unsigned short* __restrict__ hout, unsigned short* __restrict__ Yout,
    unsigned short* __restrict__ Xout) {
  __shared__ __align__(16) unsigned short sW[kW * kWtPad];
  for (int i = threadIdx.x; i < kW * kK / 8; i += kLayerThreads) {
    const int n = i / (kK / 8), k8 = i % (kK / 8);
    *reinterpret_cast<us8*>(sW + n * kWtPad + 8 * k8) = *reinterpret_cast<const us8*>(Wt + (int64_t)n * kK + 8 * k8);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row = lane & 15, oct = lane >> 4;
  float4 bc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) bc[t] = *reinterpret_cast<const float4*>(b + 16 * t + 4 * oct);
  for (int tile = 0; tile < kNnTiles; ++tile) {
    const int64_t base = (int64_t)blockIdx.x * kLayerCells + (tile * kLayerWaves + wave) * 16;
    if (base >= nc) break;
    const int64_t P = base + row;
    const bool live = P < nc;
    f4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = (f4){0.f, 0.f, 0.f, 0.f};
    auto mfma_step = [&](int step, const us8& xk) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const us8 wk = *reinterpret_cast<const us8*>(sW + (16 * t + row) * kWtPad + 32 * step + 8 * oct);
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf8(wk), as_bf8(xk), acc[t], 0, 0, 0);
      }
    };
    // self part: k in [0, 64)
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
      us8 a = (us8){0, 0, 0, 0, 0, 0, 0, 0};
      if (live) a = *reinterpret_cast<const us8*>(h + P * kW + 32 * kb + 8 * oct);
      if (Xout && live) *reinterpret_cast<us8*>(Xout + P * kK + 32 * kb + 8 * oct) = a;
      mfma_step(kb, a);
    }
    // aggregates: k in [64 (1 + d), 64 (2 + d))
    float ag[2][4][8];
#pragma unroll
    for (int kb = 0; kb < 2; ++kb)
#pragma unroll
      for (int d = 0; d < 4; ++d)
#pragma unroll
        for (int j = 0; j < 8; ++j) ag[kb][d][j] = 0.0f;
    if (live) {
      for (int s = 0; s < NS; ++s) {
        const int32_t N = nbr[(int64_t)s * nc + P];
        if (N < 0) continue;
        const float4 w4 = wf[(int64_t)s * nc + P];
        const float wv[4] = {w4.x, w4.y, w4.z, w4.w};
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) {
          const us8 hv = *reinterpret_cast<const us8*>(h + (int64_t)N * kW + 32 * kb + 8 * oct);
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const float v = bf2f(hv[j]);
#pragma unroll
            for (int d = 0; d < 4; ++d) ag[kb][d][j] += wv[d] * v;
          }
        }
      }
    }
#pragma unroll
    for (int kb = 0; kb < 2; ++kb)
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        us8 a;
#pragma unroll
        for (int j = 0; j < 8; ++j) a[j] = f2bf(ag[kb][d][j]);
        if (Xout && live) *reinterpret_cast<us8*>(Xout + P * kK + 64 * (1 + d) + 32 * kb + 8 * oct) = a;
        mfma_step(2 + 2 * d + kb, a);
      }
    // epilogue: lane holds channels 16 t + 4 oct + j of cell P
    if (live) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int c0 = 16 * t + 4 * oct;
        const us4 hv = *reinterpret_cast<const us4*>(h + P * kW + c0);
        const float bb[4] = {bc[t].x, bc[t].y, bc[t].z, bc[t].w};
        us4 ho, yo;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float y = fmaxf(acc[t][j] + bb[j], 0.0f);
          ho[j] = f2bf(bf2f(hv[j]) + y);
          yo[j] = f2bf(y);
        }
        *reinterpret_cast<us4*>(hout + P * kW + c0) = ho;
        if (Yout) *reinterpret_cast<us4*>(Yout + P * kW + c0) = yo;
      }
    }
  }
}

// ---- decoder (+ loss terms) ---------------------------------------------------
// out = z + s_z (h Wd + bd); with e != null also dg = s_z 2 (out - e) / ||e||^2
// (written to dg[nc][3]) and per-block partial losses.
template <int D>
__global__ __launch_bounds__(kB) void k_nn_decoder(int64_t nc, const unsigned short* __restrict__ h,
                                                   const unsigned short* __restrict__ Wd /*[64][3] bf16*/,
                                                   const float* __restrict__ bd, const double* __restrict__ z,
                                                   const double* __restrict__ sc, double* __restrict__ out,
                                                   const double* __restrict__ e, float* __restrict__ dg,
                                                   double* __restrict__ part) {
  __shared__ double red[kB];
  const int64_t P = (int64_t)blockIdx.x * kB + threadIdx.x;
  double l = 0.0;
  if (P < nc) {
    float g[3] = {bd[0], bd[1], bd[2]};
#pragma unroll
    for (int c8 = 0; c8 < kW / 8; ++c8) {
      const us8 hv8 = *reinterpret_cast<const us8*>(h + P * kW + 8 * c8);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const float hv = bf2f(hv8[q]);
        const int c = 8 * c8 + q;
#pragma unroll
        for (int j = 0; j < 3; ++j) g[j] += hv * bf2f(Wd[c * 3 + j]);
      }
    }
    const double sz = sc[3];
    const double ie = e ? 1.0 / sc[4] : 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      if (j < D) {
        const double o = z[(int64_t)j * nc + P] + sz * (double)g[j];
        if (out) out[(int64_t)j * nc + P] = o;
        if (e) {
          const double diff = o - e[(int64_t)j * nc + P];
          l += diff * diff * ie;
          dg[P * 3 + j] = (float)(sz * 2.0 * diff * ie);
        }
      } else if (e) {
        dg[P * 3 + j] = 0.0f;
      }
    }
  }
  if (!e) return;
  red[threadIdx.x] = l;
  __syncthreads();
  for (int s = kB / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// ---- backward -----------------------------------------------------------------

// dh[P][c] = sum_j dg[P][j] Wd[c][j]; grad partials of Wd (64x3) and bd (3)
// per block: part[block][0..195)
__global__ __launch_bounds__(kB) void k_nn_decoder_bwd(int64_t nc, const unsigned short* __restrict__ h,
                                                       const unsigned short* __restrict__ Wd,
                                                       const float* __restrict__ dg, float* __restrict__ dh,
                                                       float* __restrict__ part) {
  __shared__ float red[kB];
  const int64_t t = (int64_t)blockIdx.x * kB + threadIdx.x;  // t = P * 64 + c
  const int64_t P = t / kW;
  const int c = (int)(t % kW);
  float g[3] = {0.f, 0.f, 0.f}, hv = 0.f;
  if (P < nc) {
#pragma unroll
    for (int j = 0; j < 3; ++j) g[j] = dg[P * 3 + j];
    hv = bf2f(h[P * kW + c]);
    dh[t] = g[0] * bf2f(Wd[c * 3]) + g[1] * bf2f(Wd[c * 3 + 1]) + g[2] * bf2f(Wd[c * 3 + 2]);
  }
  // the block holds 4 cells x 64 channels: dWd[c][j] sums over its 4 cells
  for (int j = 0; j < 3; ++j) {
    red[threadIdx.x] = hv * g[j];
    __syncthreads();
    if (threadIdx.x < kW) {
      float s = 0.f;
      for (int q = 0; q < kB / kW; ++q) s += red[q * kW + threadIdx.x];
      part[(int64_t)blockIdx.x * 195 + threadIdx.x * 3 + j] = s;
    }
    __syncthreads();
  }
  if (threadIdx.x < 3) {
    float s = 0.f;
    for (int q = 0; q < kB / kW; ++q) {
      const int64_t PP = (int64_t)blockIdx.x * (kB / kW) + q;
      if (PP < nc) s += dg[PP * 3 + threadIdx.x];
    }
    part[(int64_t)blockIdx.x * 195 + 192 + threadIdx.x] = s;
  }
}

// dY = dh * (Y > 0) as BF16, and per-block partial bias grads (64 per block of 4 cells)
__global__ __launch_bounds__(kB) void k_nn_relu_bwd(int64_t nc, const float* __restrict__ dh,
                                                    const unsigned short* __restrict__ Y,
                                                    unsigned short* __restrict__ dY, float* __restrict__ part) {
  __shared__ float red[kB];
  const int64_t t = (int64_t)blockIdx.x * kB + threadIdx.x;
  float v = 0.f;
  if (t < nc * kW) {
    v = bf2f(Y[t]) > 0.f ? dh[t] : 0.f;
    dY[t] = f2bf(v);
  }
  red[threadIdx.x] = v;
  __syncthreads();
  if (threadIdx.x < kW) {
    float s = 0.f;
    for (int q = 0; q < kB / kW; ++q) s += red[q * kW + threadIdx.x];
    part[(int64_t)blockIdx.x * kW + threadIdx.x] = s;
  }
}

// dX = dY W^T : [nc x 64] x [64 x 320]; W row-major bf16 [320][64].
// Writes dh_in = dh + dX[:, 0:64] and dA = dX[:, 64:320] (fp32).
__global__ __launch_bounds__(kB) void k_nn_dx(int64_t nc, const unsigned short* __restrict__ dY,
                                              const unsigned short* __restrict__ W, const float* __restrict__ dh,
                                              float* __restrict__ dh_in, float* __restrict__ dA) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t base = ((int64_t)blockIdx.x * 4 + wave) * 16;
  const int row = lane & 15, oct = lane >> 4;
  const int64_t P = base + row;
  us8 a[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    a[s] = (us8){0, 0, 0, 0, 0, 0, 0, 0};
    if (P < nc) a[s] = *reinterpret_cast<const us8*>(dY + P * kW + 32 * s + 8 * oct);
  }
  for (int t = 0; t < kK / 16; ++t) {
    f4 acc = (f4){0.f, 0.f, 0.f, 0.f};
    const int n = 16 * t + row;  // output column (k of the forward)
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const us8 bw = *reinterpret_cast<const us8*>(W + (int64_t)n * kW + 32 * s + 8 * oct);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf8(a[s]), as_bf8(bw), acc, 0, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t Q = base + 4 * oct + j;
      if (Q >= nc) continue;
      if (n < kW) dh_in[Q * kW + n] = dh[Q * kW + n] + acc[j];
      else dA[Q * (kK - kW) + (n - kW)] = acc[j];
    }
  }
}

// dh_in[P] += sum_s sum_d wb[s][d][P] dA_d[N_s]   (adjoint of the aggregation)
__global__ __launch_bounds__(kB) void k_nn_agg_t(int64_t nc, const int32_t* __restrict__ nbr,
                                                 const float* __restrict__ wb, int NS, const float* __restrict__ dA,
                                                 float* __restrict__ dh_in) {
  const int64_t t = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (t >= nc * kW) return;
  const int64_t P = t / kW;
  const int c = (int)(t % kW);
  float s = 0.f;
  for (int k = 0; k < NS; ++k) {
    const int32_t N = nbr[(int64_t)k * nc + P];
    if (N < 0) continue;
#pragma unroll
    for (int d = 0; d < 4; ++d) s += wb[((int64_t)k * nc + P) * 4 + d] * dA[(int64_t)N * (kK - kW) + d * kW + c];
  }
  dh_in[t] += s;
}

// dW = X^T dY over a chunk of cells per block (split-K): part[block][320][64].
// Wave w of the block owns output rows [80 w, 80 w + 80) = 5 M-tiles x 4 N-tiles.
constexpr int kDwCells = 256;
__global__ __launch_bounds__(kB) void k_nn_dw(int64_t nc, const unsigned short* __restrict__ X,
                                              const unsigned short* __restrict__ dY, float* __restrict__ part) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row = lane & 15, oct = lane >> 4;
  const int64_t c0 = (int64_t)blockIdx.x * kDwCells;
  f4 acc[5][4];
#pragma unroll
  for (int m = 0; m < 5; ++m)
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[m][t] = (f4){0.f, 0.f, 0.f, 0.f};
  for (int ks = 0; ks < kDwCells / 32; ++ks) {
    const int64_t cb = c0 + 32 * ks + 8 * oct;  // this lane's 8 cells (K index)
    us8 bv[4];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int j = 0; j < 8; ++j) bv[t][j] = (cb + j < nc) ? dY[(cb + j) * kW + 16 * t + row] : (unsigned short)0;
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      const int mr = 80 * wave + 16 * m + row;  // k of the forward
      us8 av;
#pragma unroll
      for (int j = 0; j < 8; ++j) av[j] = (cb + j < nc) ? X[(cb + j) * kK + mr] : (unsigned short)0;
#pragma unroll
      for (int t = 0; t < 4; ++t)
        acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf8(av), as_bf8(bv[t]), acc[m][t], 0, 0, 0);
    }
  }
  float* o = part + (int64_t)blockIdx.x * kK * kW;
#pragma unroll
  for (int m = 0; m < 5; ++m)
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int j = 0; j < 4; ++j) o[(int64_t)(80 * wave + 16 * m + 4 * oct + j) * kW + 16 * t + row] = acc[m][t][j];
}

// encoder backward: dpre = dh0 * (h0 > 0); part[block][8*64 + 64] over 4 cells
__global__ __launch_bounds__(kB) void k_nn_encoder_bwd(int64_t nc, const unsigned short* __restrict__ x,
                                                       const unsigned short* __restrict__ h0,
                                                       const float* __restrict__ dh, float* __restrict__ part) {
  __shared__ float red[kB];
  const int64_t t = (int64_t)blockIdx.x * kB + threadIdx.x;
  const int64_t P = t / kW;
  float dp = 0.f;
  if (P < nc) dp = bf2f(h0[t]) > 0.f ? dh[t] : 0.f;
  for (int j = 0; j < 9; ++j) {
    const float xv = (P < nc) ? (j < 8 ? bf2f(x[P * 8 + j]) : 1.0f) : 0.f;
    red[threadIdx.x] = xv * dp;
    __syncthreads();
    if (threadIdx.x < kW) {
      float s = 0.f;
      for (int q = 0; q < kB / kW; ++q) s += red[q * kW + threadIdx.x];
      part[(int64_t)blockIdx.x * 576 + j * kW + threadIdx.x] = s;  // j = 8 is the bias
    }
    __syncthreads();
  }
}

// s = sum over the rows b of group g (b0 <= b < b1, in order) of part[b * stride + i],
// stored as part2[g * count + i], or added as grad[i] += scale * s when grad is
// given; a block takes 64 outputs and one group, its four row lanes
// interleaved and combined in a fixed order (deterministic)
constexpr int kNnRedGroups = 128;
__global__ __launch_bounds__(kB) void k_nn_reduce_rows(int64_t count, int64_t nb, int64_t stride, int64_t per_group,
                                                       const float* __restrict__ part, float* __restrict__ part2,
                                                       float scale, float* __restrict__ grad) {
  __shared__ float red[4][64];
  const int o = threadIdx.x & 63, r4 = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 64 + o;
  const int64_t g = blockIdx.y;
  const int64_t b0 = g * per_group, b1 = b0 + per_group < nb ? b0 + per_group : nb;
  float s = 0.f;
  if (i < count)
    for (int64_t b = b0 + r4; b < b1; b += 4) s += part[b * stride + i];
  red[r4][o] = s;
  __syncthreads();
  if (r4 == 0 && i < count) {
    const float t = (red[0][o] + red[1][o]) + (red[2][o] + red[3][o]);
    if (grad) grad[i] += scale * t;
    else part2[g * count + i] = t;
  }
}

__global__ __launch_bounds__(kB) void k_nn_sum_d(int nb, const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double red[kB];
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += kB) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = kB / 2; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] += red[0];
}

// sums of squares of up to 3 vectors -> sc[0..2] partials -> sc: [2] rms r, [3] rms z, [4] |e|^2
__global__ __launch_bounds__(kB) void k_nn_norms(int64_t n, const double* __restrict__ r, const double* __restrict__ z,
                                                 const double* __restrict__ e, double* __restrict__ part) {
  __shared__ double red[3][kB];
  double a = 0, b = 0, c = 0;
  for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kB) {
    a += r[i] * r[i];
    b += z[i] * z[i];
    if (e) c += e[i] * e[i];
  }
  red[0][threadIdx.x] = a;
  red[1][threadIdx.x] = b;
  red[2][threadIdx.x] = c;
  __syncthreads();
  for (int k = kB / 2; k > 0; k >>= 1) {
    if (threadIdx.x < k)
      for (int q = 0; q < 3; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int q = 0; q < 3; ++q) part[q * 512 + blockIdx.x] = red[q][0];
}

__global__ __launch_bounds__(kB) void k_nn_norms_final(int nb, int64_t n, const double* __restrict__ part,
                                                       double* __restrict__ sc) {
  __shared__ double red[3][kB];
  double v[3] = {0, 0, 0};
  for (int i = threadIdx.x; i < nb; i += kB)
    for (int q = 0; q < 3; ++q) v[q] += part[q * 512 + i];
  for (int q = 0; q < 3; ++q) red[q][threadIdx.x] = v[q];
  __syncthreads();
  for (int k = kB / 2; k > 0; k >>= 1) {
    if (threadIdx.x < k)
      for (int q = 0; q < 3; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    sc[2] = sqrt(red[0][0] / (double)n);
    sc[3] = sqrt(red[1][0] / (double)n);
    sc[4] = red[2][0];
  }
}

// Adam (Kingma & Ba) on the FP32 master copy, then refresh of the BF16 copies
__global__ __launch_bounds__(kB) void k_nn_adam(int64_t np, float* __restrict__ p, float* __restrict__ m,
                                                float* __restrict__ v, const float* __restrict__ g, float lr, float b1,
                                                float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (i >= np) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// BF16 copies: We [8][64], per layer Wt [64][320] (transposed) and W [320][64], Wd [64][3]
__global__ __launch_bounds__(kB) void k_nn_refresh(const float* __restrict__ p, unsigned short* __restrict__ We,
                                                   unsigned short* __restrict__ Wt, unsigned short* __restrict__ Wr,
                                                   unsigned short* __restrict__ Wd) {
  const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (i < 8 * kW) We[i] = f2bf(p[kNnOffWe + i]);
  if (i < 3 * kW) Wd[i] = f2bf(p[kNnOffWd + i]);
  if (i < (int64_t)kNnLayers * kK * kW) {
    const int l = (int)(i / (kK * kW));
    const int64_t r = i % (kK * kW);
    const int k = (int)(r / kW), c = (int)(r % kW);
    const float w = p[kNnOffW(l) + r];
    Wr[(int64_t)l * kK * kW + r] = f2bf(w);
    Wt[(int64_t)l * kK * kW + (int64_t)c * kK + k] = f2bf(w);
  }
}

// out[i] standard normal: Box-Muller on outputs 2 (i / 2) + 1 and + 2 of splitmix64
// seeded with `seed` (the k-th output mixes seed + k * 0x9E3779B97F4A7C15)
__device__ inline double splitmix_unit(uint64_t seed, uint64_t k) {
  uint64_t z = seed + k * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (double)((z >> 11) + 1) * (1.0 / 9007199254740992.0);  // (0, 1]
}

__global__ __launch_bounds__(kB) void k_normal(int64_t n, uint64_t seed, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (i >= n) return;
  const uint64_t pr = (uint64_t)(i / 2);
  const double u1 = splitmix_unit(seed, 2 * pr + 1), u2 = splitmix_unit(seed, 2 * pr + 2);
  const double rad = sqrt(-2.0 * log(u1)), th = 6.283185307179586 * u2;
  out[i] = (i & 1) ? rad * sin(th) : rad * cos(th);
}

__global__ __launch_bounds__(kB) void k_nn_zero_f(int64_t n, float* __restrict__ a) {
  const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (i < n) a[i] = 0.f;
}

__global__ __launch_bounds__(kB) void k_nn_zero_d(int64_t n, double* __restrict__ a) {
  const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (i < n) a[i] = 0.0;
}

}  // namespace

// ---------------------------------------------------------------------------
hofv_status nn_alloc_model(hofv_nn* m) {
  auto al = [&](void** p, size_t bytes) -> bool { return hipMalloc(p, bytes) == hipSuccess; };
  const size_t np = kNnParams;
  if (!al((void**)&m->loss, sizeof(double))) return HOFV_ENOMEM;
  if (!al((void**)&m->p, np * 4) || !al((void**)&m->m, np * 4) || !al((void**)&m->v, np * 4) ||
      !al((void**)&m->g, np * 4) || !al((void**)&m->We, 8 * kW * 2) || !al((void**)&m->Wd, 3 * kW * 2) ||
      !al((void**)&m->Wt, (size_t)kNnLayers * kK * kW * 2) || !al((void**)&m->Wr, (size_t)kNnLayers * kK * kW * 2))
    return HOFV_ENOMEM;
  return HOFV_OK;
}

void nn_free_model(hofv_nn* m) {
  for (void* p : {(void*)m->p, (void*)m->m, (void*)m->v, (void*)m->g, (void*)m->We, (void*)m->Wd, (void*)m->Wt,
                  (void*)m->Wr, (void*)m->loss})
    if (p) hipFree(p);
}

hofv_status nn_refresh(hofv_nn* m, hipStream_t st) {
  k_nn_refresh<<<nblk((int64_t)kNnLayers * kK * kW), kB, 0, st>>>(m->p, m->We, m->Wt, m->Wr, m->Wd);
  return hipGetLastError() == hipSuccess ? HOFV_OK : HOFV_EHIP;
}

static hofv_status ensure_ws(hofv_ctx* c, bool train) {
  NnWork& w = c->nnw;
  const int64_t nc = c->nc;
  hofv_status s;
  if (!w.h) {
    if ((s = dev_alloc(c, &w.x, (size_t)nc * 8))) return s;
    if ((s = dev_alloc(c, &w.h, (size_t)(kNnLayers + 1) * nc * kW))) return s;
    if (!w.zaj && (s = dev_alloc(c, &w.zaj, (size_t)c->D * nc))) return s;
    if ((s = dev_alloc(c, &w.sc, 16))) return s;
    if ((s = dev_alloc(c, &w.dpart, 3 * 512 + 8))) return s;
  }
  if (train && !w.X) {
    if ((s = dev_alloc(c, &w.X, (size_t)kNnLayers * nc * kK))) return s;
    if ((s = dev_alloc(c, &w.Y, (size_t)kNnLayers * nc * kW))) return s;
    if ((s = dev_alloc(c, &w.dY, (size_t)nc * kW))) return s;
    if ((s = dev_alloc(c, &w.dh, (size_t)nc * kW))) return s;
    if ((s = dev_alloc(c, &w.dh2, (size_t)nc * kW))) return s;
    if ((s = dev_alloc(c, &w.dA, (size_t)nc * (kK - kW)))) return s;
    if ((s = dev_alloc(c, &w.dg, (size_t)nc * 3))) return s;
    const int64_t nbw = (nc + kDwCells - 1) / kDwCells;
    const int64_t nb4 = (nc * kW + kB - 1) / kB;
    const size_t part = std::max<size_t>((size_t)nbw * kK * kW, (size_t)nb4 * 576);
    if ((s = dev_alloc(c, &w.part, part))) return s;
    if ((s = dev_alloc(c, &w.part2, (size_t)kNnRedGroups * kK * kW))) return s;
    if ((s = dev_alloc(c, &w.lpart, (size_t)nblk(nc) + 8))) return s;
  }
  return HOFV_OK;
}

// forward of the correction: z_out = zaj + s_z g.  r, zaj: caller layout [D][nc].
template <int D>
static hofv_status nn_forward(hofv_ctx* c, hofv_nn* m, const double* r, const double* zaj, const double* e,
                              double* out, bool train, hipStream_t st) {
  NnWork& w = c->nnw;
  const DeviceTables& t = c->dev;
  const int64_t nc = c->nc, n = (int64_t)D * nc;
  const int nb = (int)std::min<int64_t>(512, nblk(n));
  k_nn_norms<<<nb, kB, 0, st>>>(n, r, zaj, e, w.dpart);
  k_nn_norms_final<<<1, kB, 0, st>>>(nb, n, w.dpart, w.sc);
  k_nn_features<D><<<nblk(nc), kB, 0, st>>>(nc, r, zaj, t.g_bflag, w.sc, w.x);
  k_nn_encoder<<<nblk(nc), kB, 0, st>>>(nc, w.x, m->We, m->p + kNnOffbe, w.h);
  const unsigned lb = (unsigned)((nc + kLayerCells - 1) / kLayerCells);
  for (int l = 0; l < kNnLayers; ++l) {
    const unsigned short* hin = w.h + (size_t)l * nc * kW;
    unsigned short* hout = w.h + (size_t)(l + 1) * nc * kW;
    TIMED_NN(c, "k_nn_layer", st,
             (k_nn_layer<<<lb, kLayerThreads, 0, st>>>(nc, hin, t.g_nbr, reinterpret_cast<const float4*>(t.g_wf), t.ns,
                                                       m->Wt + (size_t)l * kK * kW,
                                            m->p + kNnOffb(l), hout, train ? w.Y + (size_t)l * nc * kW : nullptr,
                                            train ? w.X + (size_t)l * nc * kK : nullptr)));
  }
  k_nn_decoder<D><<<nblk(nc), kB, 0, st>>>(nc, w.h + (size_t)kNnLayers * nc * kW, m->Wd, m->p + kNnOffbd, zaj,
                                           w.sc, out, e, w.dg, w.lpart);
  if (hipGetLastError() != hipSuccess) return fail(c, HOFV_EHIP, "MPNN forward launch failed");
  return HOFV_OK;
}

hofv_status nn_apply(hofv_ctx* c, hofv_nn* m, const double* r, const double* zaj, double* z, hipStream_t st) {
  hofv_status s = ensure_ws(c, false);
  if (s) return s;
  return c->D == 2 ? nn_forward<2>(c, m, r, zaj, nullptr, z, false, st)
                   : nn_forward<3>(c, m, r, zaj, nullptr, z, false, st);
}

// gradient of the loss of one pair (r, e), accumulated (scaled) into m->g;
// the pair's loss is added to *loss_dev.
// grad[i] += scale * sum_b part[b * stride + i], i < count (count <= kK kW), in
// two fixed-order stages: row groups in parallel, then the group sums
static void reduce_grad(int64_t count, int64_t nb, int64_t stride, const float* part, float* part2, float scale,
                        float* grad, hipStream_t st) {
  const int64_t per = (nb + kNnRedGroups - 1) / kNnRedGroups;
  const int64_t groups = (nb + per - 1) / per;
  const unsigned bx = (unsigned)((count + 63) / 64);
  k_nn_reduce_rows<<<dim3(bx, (unsigned)groups), kB, 0, st>>>(count, nb, stride, per, part, part2, 0.f, nullptr);
  k_nn_reduce_rows<<<dim3(bx, 1), kB, 0, st>>>(count, groups, count, groups, part2, nullptr, scale, grad);
}

template <int D>
static hofv_status nn_grad_pair(hofv_ctx* c, hofv_nn* m, const double* r, const double* zaj, const double* e,
                                float scale, double* loss_dev, hipStream_t st) {
  NnWork& w = c->nnw;
  const DeviceTables& t = c->dev;
  const int64_t nc = c->nc;
  hofv_status s = nn_forward<D>(c, m, r, zaj, e, nullptr, true, st);
  if (s) return s;
  const unsigned nbc = nblk(nc);
  k_nn_sum_d<<<1, kB, 0, st>>>((int)nbc, w.lpart, loss_dev);
  // decoder
  const int64_t nb4 = (nc * kW + kB - 1) / kB;
  k_nn_decoder_bwd<<<(unsigned)nb4, kB, 0, st>>>(nc, w.h + (size_t)kNnLayers * nc * kW, m->Wd, w.dg, w.dh, w.part);
  reduce_grad(195, nb4, 195, w.part, w.part2, scale, m->g + kNnOffWd, st);
  float* dh = w.dh;
  float* dh2 = w.dh2;
  const unsigned lb = (unsigned)((nc + 63) / 64);
  const int64_t nbw = (nc + kDwCells - 1) / kDwCells;
  for (int l = kNnLayers - 1; l >= 0; --l) {
    k_nn_relu_bwd<<<(unsigned)nb4, kB, 0, st>>>(nc, dh, w.Y + (size_t)l * nc * kW, w.dY, w.part);
    reduce_grad(kW, nb4, kW, w.part, w.part2, scale, m->g + kNnOffb(l), st);
    TIMED_NN(c, "k_nn_dw", st,
             (k_nn_dw<<<(unsigned)nbw, kB, 0, st>>>(nc, w.X + (size_t)l * nc * kK, w.dY, w.part)));
    reduce_grad((int64_t)kK * kW, nbw, (int64_t)kK * kW, w.part, w.part2, scale, m->g + kNnOffW(l), st);
    TIMED_NN(c, "k_nn_dx", st,
             (k_nn_dx<<<lb, kB, 0, st>>>(nc, w.dY, m->Wr + (size_t)l * kK * kW, dh, dh2, w.dA)));
    k_nn_agg_t<<<(unsigned)nb4, kB, 0, st>>>(nc, t.g_nbr, t.g_wb, t.ns, w.dA, dh2);
    std::swap(dh, dh2);
  }
  k_nn_encoder_bwd<<<(unsigned)nb4, kB, 0, st>>>(nc, w.x, w.h, dh, w.part);
  // part rows: j < 8 -> dWe[j][c], j = 8 -> dbe[c]; kNnOffWe..kNnOffbe are adjacent
  reduce_grad(576, nb4, 576, w.part, w.part2, scale, m->g + kNnOffWe, st);
  if (hipGetLastError() != hipSuccess) return fail(c, HOFV_EHIP, "MPNN backward launch failed");
  return HOFV_OK;
}

hofv_status nn_grad(hofv_ctx* c, hofv_nn* m, const double* r, const double* zaj, const double* e, float scale,
                    double* loss_dev, hipStream_t st) {
  hofv_status s = ensure_ws(c, true);
  if (s) return s;
  return c->D == 2 ? nn_grad_pair<2>(c, m, r, zaj, e, scale, loss_dev, st)
                   : nn_grad_pair<3>(c, m, r, zaj, e, scale, loss_dev, st);
}

hofv_status fill_normal(int64_t n, uint64_t seed, double* out, hipStream_t st) {
  k_normal<<<nblk(n), kB, 0, st>>>(n, seed, out);
  return hipGetLastError() == hipSuccess ? HOFV_OK : HOFV_EHIP;
}

hofv_status nn_zero_grad(hofv_nn* m, hipStream_t st) {
  k_nn_zero_f<<<nblk(kNnParams), kB, 0, st>>>(kNnParams, m->g);
  return hipGetLastError() == hipSuccess ? HOFV_OK : HOFV_EHIP;
}

hofv_status nn_zero_scalar(double* p, hipStream_t st) {
  k_nn_zero_d<<<1, kB, 0, st>>>(1, p);
  return hipGetLastError() == hipSuccess ? HOFV_OK : HOFV_EHIP;
}

hofv_status nn_adam(hofv_nn* m, double lr, hipStream_t st) {
  m->step += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - std::pow(b1, (float)m->step), c2 = 1.f - std::pow(b2, (float)m->step);
  k_nn_adam<<<nblk(kNnParams), kB, 0, st>>>(kNnParams, m->p, m->m, m->v, m->g, (float)lr, b1, b2, 1e-8f, c1, c2);
  if (hipGetLastError() != hipSuccess) return HOFV_EHIP;
  return nn_refresh(m, st);
}

}  // namespace hofv
