// Deterministic wavefront reductions for gfx950 (wave64).
//
// A thread holds NV partial sums (NV a power of two <= 64).  The wavefront
// first halves the set at every butterfly step (lane l and lane l ^ o swap the
// halves each keeps, so after log2(NV) steps every lane holds one value), then
// sums the remaining lane groups; the workgroup adds its wavefronts' results
// in wavefront order.  Every step has a fixed order, so a sum does not depend
// on timing: repeated runs give identical bits.
#pragma once

#include <hip/hip_runtime.h>

namespace hofv {

constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v / 2); }

// After the call lane l holds the wavefront sum of value index l >> (6 - log2 NV)
// (the lanes of one group of 64 / NV hold the same value).
template <int NV>
__device__ __attribute__((always_inline)) inline double wave_reduce_scatter(double (&a)[NV]) {
  static_assert(NV >= 1 && NV <= 64 && (NV & (NV - 1)) == 0, "NV must be a power of two <= 64");
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int s = 0; s < ilog2c(NV); ++s) {
    const int o = 32 >> s, half = (NV >> s) / 2;
    const bool upper = (lane & o) != 0;
#pragma unroll
    for (int k = 0; k < half; ++k) {
      // select between the two register values (an index chosen at run time
      // would move the array to scratch memory)
      const double lo = a[k], hi = a[k + half];
      const double send = upper ? lo : hi;
      const double keep = upper ? hi : lo;
      a[k] = keep + __shfl_xor(send, o, 64);
    }
  }
  double v = a[0];
#pragma unroll
  for (int o = (64 / NV) / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Workgroup sum of NV values per thread (blockDim.x = NT, a multiple of 64);
// out[i] (shared, NV entries) holds the sum of index i for every thread
// after the call.  sred: shared scratch of (NT / 64) * NV doubles.
template <int NV, int NT>
__device__ __attribute__((always_inline)) inline void block_reduce(double (&a)[NV], double* sred, double* out) {
  constexpr int W = NT / 64, G = 64 / NV;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const double v = wave_reduce_scatter<NV>(a);
  if (lane % G == 0) sred[wave * NV + lane / G] = v;
  __syncthreads();
  if (threadIdx.x < NV) {
    double s = sred[threadIdx.x];
#pragma unroll
    for (int w = 1; w < W; ++w) s += sred[w * NV + threadIdx.x];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

}  // namespace hofv
