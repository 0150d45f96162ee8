// Learned preconditioner correction: model layout and workspace.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "hofv.h"

namespace hofv {

constexpr int kNnWidth = 64;
constexpr int kNnLayers = 4;
constexpr int kNnIn = 8;
constexpr int64_t kNnLayerK = 5 * kNnWidth;  // [h, A0, A1, A2, A3]

// flat FP32 parameter layout: We[8][64], be[64], {W_l[320][64], b_l[64]} x 4, Wd[64][3], bd[3]
constexpr int64_t kNnOffWe = 0;
constexpr int64_t kNnOffbe = kNnOffWe + kNnIn * kNnWidth;
constexpr int64_t kNnLayerSize = kNnLayerK * kNnWidth + kNnWidth;
constexpr int64_t kNnOffW(int l) { return kNnOffbe + kNnWidth + l * kNnLayerSize; }
constexpr int64_t kNnOffb(int l) { return kNnOffW(l) + kNnLayerK * kNnWidth; }
constexpr int64_t kNnOffWd = kNnOffW(kNnLayers);
constexpr int64_t kNnOffbd = kNnOffWd + 3 * kNnWidth;
constexpr int64_t kNnParams = kNnOffbd + 3;

// per-context activations and gradient workspace (allocated on first use)
struct NnWork {
  unsigned short* x = nullptr;   // [nc][8] bf16 inputs
  unsigned short* h = nullptr;   // [layers + 1][nc][64] bf16
  unsigned short* X = nullptr;   // [layers][nc][320] bf16 (training)
  unsigned short* Y = nullptr;   // [layers][nc][64] bf16 relu outputs (training)
  unsigned short* dY = nullptr;  // [nc][64] bf16
  float* dh = nullptr;           // [nc][64]
  float* dh2 = nullptr;          // [nc][64]
  float* dA = nullptr;           // [nc][256]
  float* dg = nullptr;           // [nc][3]
  float* part = nullptr;         // block partials of parameter gradients
  float* part2 = nullptr;        // row-group sums of those partials [kNnRedGroups][count]
  double* lpart = nullptr;       // block partials of the loss
  double* zaj = nullptr;         // [D][nc] plain preconditioner output
  double* sc = nullptr;          // scalars: [2] rms r, [3] rms z, [4] |e|^2, [5] loss
  double* dpart = nullptr;       // norm partials
};

}  // namespace hofv

// training pairs (r, e), J e = r, on one context's mesh
struct hofv_pairset {
  hofv_ctx* ctx = nullptr;
  int32_t cap = 0, n = 0;
  double* r = nullptr;  // [cap][dim][n_cells]
  double* e = nullptr;
};

struct hofv_nn {
  int device = 0;
  int64_t step = 0;
  double* loss = nullptr;         // device accumulator of a training step's loss
  float* p = nullptr;             // FP32 master parameters
  float* m = nullptr;             // Adam first moments
  float* v = nullptr;             // Adam second moments
  float* g = nullptr;             // gradient accumulator
  unsigned short* We = nullptr;   // bf16 [8][64]
  unsigned short* Wd = nullptr;   // bf16 [64][3]
  unsigned short* Wt = nullptr;   // bf16 per layer [64][320] (forward B operand)
  unsigned short* Wr = nullptr;   // bf16 per layer [320][64] (backward B operand)
};

namespace hofv {
hofv_status nn_alloc_model(hofv_nn* m);
void nn_free_model(hofv_nn* m);
hofv_status nn_refresh(hofv_nn* m, hipStream_t st);
hofv_status nn_apply(hofv_ctx* c, hofv_nn* m, const double* r, const double* zaj, double* z, hipStream_t st);
hofv_status nn_grad(hofv_ctx* c, hofv_nn* m, const double* r, const double* zaj, const double* e, float scale,
                    double* loss_dev, hipStream_t st);
hofv_status nn_zero_grad(hofv_nn* m, hipStream_t st);
hofv_status nn_zero_scalar(double* p, hipStream_t st);
hofv_status nn_adam(hofv_nn* m, double lr, hipStream_t st);
// standard normal values of splitmix64 seeded with `seed` (Box-Muller on output pairs)
hofv_status fill_normal(int64_t n, uint64_t seed, double* out, hipStream_t st);
}  // namespace hofv

#define TIMED_NN(ctx, name, st, launch)        \
  do {                                         \
    hipEvent_t ev_;                            \
    ::hofv::timer_begin(ctx, name, st, &ev_);  \
    launch;                                    \
    ::hofv::timer_end(ctx, name, st, ev_);     \
  } while (0)
