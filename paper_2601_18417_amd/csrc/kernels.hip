// HIP kernels of the residual R(u), the finite-difference J.v and the FP32
// preconditioner sweeps for gfx950 (wave64).
//
// Residual = k_extrap (cells) -> k_face_* (faces) -> k_cell_sum (cells):
//   k_extrap   u*_{f,P} - u_P = sum_k E[k][slot][P] u(S_P[k]) for every face slot
//              of P (eq. alphaJump, pre-contracted at setup);
//   k_face_le  linear elasticity with quadrature-summed gradient coefficients:
//              G = sum_k c[k] (x) u(S_f[k]), F = Gamma n . sigma(G)
//              + alpha Kbar Gamma / |d.n| (u*_N - u*_P)     (eqs. faceQuadGrad, alpha);
//   k_face_q   per-quadrature-point gradients, linear elastic or neo-Hookean
//              (first Piola stress P = sigma cof(F), traction P n_o);
//   k_cell_sum R_P = sum of +-F over the cell's faces + load * src_P, or, for
//              J.v, (that - R(u)_P) / eps.
// One thread owns one face or one cell, one workgroup one item block (items
// consecutive along a Morton curve).  Per-item tables are stored
// k-major/item-minor so the 64 lanes of a wavefront read 64 consecutive words
// of each coefficient stream; the stencil values of u come from an LDS copy
// of the block's stencil union, staged once per workgroup, so the only
// scattered global loads are the staging gathers (L2 hits: a cell is in the
// unions of a few neighbouring blocks).
#include <hip/hip_runtime.h>

#include <cfloat>
#include <map>
#include <mutex>

#include "common.h"
#include "reduce.h"

namespace hofv {

namespace {

constexpr int kBlock = 256;
// chunk sizes (stencil entries) of the pipelined contractions
#ifndef HOFV_FACE_CHUNK
#define HOFV_FACE_CHUNK 2
#endif
#ifndef HOFV_EXTRAP_CHUNK
#define HOFV_EXTRAP_CHUNK 1
#endif
constexpr int kFaceChunk = HOFV_FACE_CHUNK, kExtrapChunk = HOFV_EXTRAP_CHUNK, kFaceQChunk = 1;

inline unsigned blocks_for(int64_t n, int per = kBlock) { return (unsigned)((n + per - 1) / per); }

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2.  Remap so that XCD x takes runs of G consecutive logical blocks in turn
// (blocks 8 G k + x G .. 8 G k + x G + G - 1): neighbouring item blocks, whose
// stencil unions overlap, share an L2 in runs of G, while every XCD works
// through the whole mesh, boundary-face blocks included, at the same pace
// (one contiguous range per XCD was slower: the face and extrapolation
// kernels gain 2 and 9 % with G = 8 and 2).  The last nb mod 8 G blocks keep
// their index; bijective for any grid.
template <int G>
__device__ inline int64_t xcd_block() {
  const int64_t nb = gridDim.x, b = blockIdx.x, M = nb / (8 * G) * (8 * G);
  if (b >= M) return b;
  const int64_t x = b % 8, k = b / 8;
  return (k / G) * (8 * G) + x * G + k % G;
}

// displacement of cell n from the padded gather copy (4 doubles per cell in
// 3D, 2 in 2D): one 16-byte and one 8-byte load from one 32-byte segment
template <int D>
__device__ inline void load_u(const double* __restrict__ ug, int64_t n, double* un) {
  const double2 a = *reinterpret_cast<const double2*>(ug + (D == 3 ? 4 : 2) * n);
  un[0] = a.x;
  un[1] = a.y;
  if constexpr (D == 3) un[2] = ug[4 * n + 2];
}

// Raw buffer resource over [base, base + bytes): loads through it at byte
// offsets >= bytes return zero instead of touching memory.
__device__ inline __amdgpu_buffer_rsrc_t buffer_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

#ifndef HOFV_NT
#define HOFV_NT 2
#endif
constexpr int kNt = HOFV_NT;  // cache policy bits of the coefficient-stream buffer loads (2: nontemporal)

// Copies the stencil union of item block b into LDS, one plane per
// component: lds[j][r] = u_j(ucell[blk_cell[b] + r]).
template <int D, int CAP>
__device__ inline void stage_union(int64_t b, const int32_t* __restrict__ blk_cell,
                                   const int32_t* __restrict__ ucell, const double* __restrict__ ug,
                                   double (*lds)[CAP]) {
  const int32_t c0 = blk_cell[b];
  const int32_t n = min(blk_cell[b + 1] - c0, CAP);
  for (int r = threadIdx.x; r < n; r += kBlockItems) {
    double un[D];
    load_u<D>(ug, ucell[c0 + r], un);
#pragma unroll
    for (int j = 0; j < D; ++j) lds[j][r] = un[j];
  }
  __syncthreads();
}

// Stencil contraction acc[i][j] = sum_k C[k][i] u(entry k)[j] over the S
// entries of one item, u read from the block's LDS copy through the 16-bit
// local positions loc[k][item]; loc and C are the block's segments, k-major
// with item stride ld = the block's item count (row i of entry k at
// C[(k I + i) ld + item]).
// Software-pipelined in chunks of U entries: while chunk j is accumulated,
// the coefficients of chunk j+1 and the positions of chunk j+2 are in flight.
// Two coefficient register sets alternate roles so that no loaded value is
// copied (a copy would wait for the load); the sched_barriers keep each
// set's loads ahead of the other set's use.  Buffer loads (not plain loads)
// keep the compiler from sinking the loop-carried loads back to their uses.
// Chunk indices past the last full pair are clamped onto the last chunk
// (cache hits) instead of branching.
template <int D, int I, int U, int CAP>
__device__ inline void contract_lds(int S, int64_t ld, int64_t item, const uint16_t* __restrict__ loc,
                                    const double* __restrict__ C, const double (*lds)[CAP],
                                    double (&acc)[I][D]) {
  const int nch = S / (2 * U) * 2;
  const uint32_t vi = (uint32_t)item * 2u, vc = (uint32_t)item * 8u, ldu = (uint32_t)ld;
  auto load_idx = [&](int ch, uint32_t(&dst)[U]) {
    ch = ch < nch ? ch : nch - 1;
    const __amdgpu_buffer_rsrc_t r = buffer_rsrc(loc + (int64_t)ch * U * ld, (uint32_t)U * ldu * 2u);
#pragma unroll
    for (int e = 0; e < U; ++e)
      dst[e] = __builtin_amdgcn_raw_buffer_load_b16(r, vi, (int)((uint32_t)e * ldu * 2u), kNt);
  };
  auto load_c = [&](int ch, double(&dst)[U][I]) {
    ch = ch < nch ? ch : nch - 1;
    const __amdgpu_buffer_rsrc_t r = buffer_rsrc(C + (int64_t)ch * U * I * ld, (uint32_t)(U * I) * ldu * 8u);
#pragma unroll
    for (int e = 0; e < U; ++e)
#pragma unroll
      for (int i = 0; i < I; ++i)
        dst[e][i] = __builtin_bit_cast(
            double, __builtin_amdgcn_raw_buffer_load_b64(r, vc, (int)((uint32_t)(e * I + i) * ldu * 8u), kNt));
  };
  auto fma = [&](const uint32_t(&l)[U], const double(&c)[U][I]) {
#pragma unroll
    for (int e = 0; e < U; ++e) {
      double uu[D];
#pragma unroll
      for (int j = 0; j < D; ++j) uu[j] = lds[j][l[e]];
#pragma unroll
      for (int i = 0; i < I; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) acc[i][j] += c[e][i] * uu[j];
    }
  };
  if (nch > 0) {
    uint32_t ia[U], ib[U];
    double ca[U][I], cb[U][I];
    load_idx(0, ia);
    load_c(0, ca);
    load_idx(1, ib);
    int j = 0;
    do {
      __builtin_amdgcn_sched_barrier(0);
      load_c(j + 1, cb);
      __builtin_amdgcn_sched_barrier(0);
      fma(ia, ca);
      load_idx(j + 2, ia);
      __builtin_amdgcn_sched_barrier(0);
      load_c(j + 2, ca);
      __builtin_amdgcn_sched_barrier(0);
      fma(ib, cb);
      load_idx(j + 3, ib);
      j += 2;
    } while (j < nch);
  }
  for (int k = nch * U; k < S; ++k) {
    const uint32_t l[1] = {loc[(int64_t)k * ld + item]};
    double c[1][I];
#pragma unroll
    for (int i = 0; i < I; ++i) c[0][i] = __builtin_nontemporal_load(&C[((int64_t)k * I + i) * ld + item]);
    double uu[D];
#pragma unroll
    for (int j = 0; j < D; ++j) uu[j] = lds[j][l[0]];
#pragma unroll
    for (int i = 0; i < I; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) acc[i][j] += c[0][i] * uu[j];
  }
}

// u*_{f,P} - u_P = sum_k E[k][slot][r] u(S_P[k]) for every face slot of
// extrapolation item r (NS slots: a cell's faces, or one face of it); its
// cell P = cell[r]; ustar is indexed by item (nc: the number of items)
template <int D, int NS>
__global__ __launch_bounds__(kBlockItems) void k_extrap(int64_t nc, int S, const int32_t* __restrict__ blk_item,
                                                    const int32_t* __restrict__ blk_cell,
                                                    const int32_t* __restrict__ ucell,
                                                    const uint16_t* __restrict__ loc, const double* __restrict__ E,
                                                    const int32_t* __restrict__ cell, const double* __restrict__ ug,
                                                    double* __restrict__ ustar) {
  __shared__ double lds[D][kLdsCellCells];
  const int64_t b = xcd_block<2>();
  stage_union<D, kLdsCellCells>(b, blk_cell, ucell, ug, lds);
  const int64_t i0 = blk_item[b], nb = blk_item[b + 1] - i0, ti = threadIdx.x;
  if (ti >= nb) return;
  const int64_t r = i0 + ti;
  double acc[NS][D];
#pragma unroll
  for (int s = 0; s < NS; ++s)
#pragma unroll
    for (int c = 0; c < D; ++c) acc[s][c] = 0.0;
  contract_lds<D, NS, kExtrapChunk, kLdsCellCells>(S, nb, ti, loc + i0 * S, E + i0 * S * NS, lds, acc);
  double uP[D];
  load_u<D>(ug, cell[r], uP);
#pragma unroll
  for (int c = 0; c < D; ++c)
#pragma unroll
    for (int s = 0; s < NS; ++s) ustar[((int64_t)s * D + c) * nc + r] = uP[c] + acc[s][c];
}

// stabilisation part alpha Kbar Gamma/|d.n| (u*_N - u*_P); on displacement
// faces only -u*_P (the u_b part is a constant source)
template <int D>
__device__ inline void add_stab(int64_t f, int64_t nfi, int64_t nc, const int32_t* own, const int32_t* nei,
                                const int32_t* slots, const double* stab, const double* ustar, double* t) {
  const int32_t P = own[f];
  const int32_t sl = slots[f];
  const double a = stab[f];
#pragma unroll
  for (int j = 0; j < D; ++j) {
    double jump = -ustar[((int64_t)(sl & 0xff) * D + j) * nc + P];
    if (f < nfi) jump += ustar[((int64_t)(sl >> 8) * D + j) * nc + nei[f]];
    t[j] += a * jump;
  }
}

template <int D>
__global__ __launch_bounds__(kBlockItems) void k_face_le(int64_t nf, int64_t nfi, int64_t nc, int S,
                                                     const int32_t* __restrict__ blk_item,
                                                     const int32_t* __restrict__ blk_cell,
                                                     const int32_t* __restrict__ ucell,
                                                     const uint16_t* __restrict__ loc, const double* __restrict__ C,
                                                     const int32_t* __restrict__ own, const int32_t* __restrict__ nei,
                                                     const int32_t* __restrict__ slots,
                                                     const double* __restrict__ Sv, const double* __restrict__ stab,
                                                     double mu, double lam, const double* __restrict__ ug,
                                                     const double* __restrict__ ustar, double* __restrict__ F) {
  __shared__ double lds[D][kLdsFaceCells];
  const int64_t b = xcd_block<8>();
  stage_union<D, kLdsFaceCells>(b, blk_cell, ucell, ug, lds);
  const int64_t i0 = blk_item[b], nb = blk_item[b + 1] - i0, ti = threadIdx.x;
  if (ti >= nb) return;
  const int64_t f = i0 + ti;
  double G[D][D];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) G[i][j] = 0.0;
  contract_lds<D, D, kFaceChunk, kLdsFaceCells>(S, nb, ti, loc + i0 * S, C + i0 * S * D, lds, G);
  double tr = 0.0;
#pragma unroll
  for (int i = 0; i < D; ++i) tr += G[i][i];
  double sv[D], t[D];
#pragma unroll
  for (int i = 0; i < D; ++i) sv[i] = Sv[(int64_t)i * nf + f];
#pragma unroll
  for (int j = 0; j < D; ++j) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) s += sv[i] * (mu * (G[i][j] + G[j][i]) + (i == j ? lam * tr : 0.0));
    t[j] = s;
  }
  add_stab<D>(f, nfi, nc, own, nei, slots, stab, ustar, t);
#pragma unroll
  for (int j = 0; j < D; ++j) F[(int64_t)j * nf + f] = t[j];
}

// neo-Hookean face traction at one quadrature point: t_j += sum_i sv_i P_ji with
// P the first Piola-Kirchhoff stress of the gradient G (G[i][j] = d u_j / d x_i)
// and sv the point's weighted area vector; flag[0] = 1 at an inverted point
__device__ inline void nh_traction(const double (*G)[3], const double* sv, double mu, double lam, double* t,
                                   int32_t* __restrict__ flag) {
  // F = I + H with H = G^T, J = det F, bbar = J^{-2/3} F F^T,
  // sigma = mu/J dev(bbar) + kappa/2 (J^2 - 1)/J I, P = J sigma F^{-T} = sigma cof(F).
  // Evaluated from H so that no O(1) terms cancel at small strain (a
  // finite-difference product perturbs H by ~1e-8):
  // J - 1 = tr H + ((tr H)^2 - tr(H H))/2 + det H, dev(bbar) = J^{-2/3} dev(B)
  // with B = b - I = H + H^T + H H^T, J^2 - 1 = (J - 1)(J + 1).
  double H[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) H[a][c] = G[c][a];
  double cof[3][3];  // cofactors of F = I + H
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int a1 = (a + 1) % 3, a2 = (a + 2) % 3, c1 = (c + 1) % 3, c2 = (c + 2) % 3;
      const double f11 = (a1 == c1 ? 1.0 : 0.0) + H[a1][c1], f22 = (a2 == c2 ? 1.0 : 0.0) + H[a2][c2];
      const double f12 = (a1 == c2 ? 1.0 : 0.0) + H[a1][c2], f21 = (a2 == c1 ? 1.0 : 0.0) + H[a2][c1];
      cof[a][c] = f11 * f22 - f12 * f21;
    }
  const double trH = H[0][0] + H[1][1] + H[2][2];
  double trHH = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) trHH += H[a][c] * H[c][a];
  const double detH = H[0][0] * (H[1][1] * H[2][2] - H[1][2] * H[2][1]) -
                      H[0][1] * (H[1][0] * H[2][2] - H[1][2] * H[2][0]) +
                      H[0][2] * (H[1][0] * H[2][1] - H[1][1] * H[2][0]);
  double Jm1 = trH + 0.5 * (trH * trH - trHH) + detH;
  double J = 1.0 + Jm1;
  if (!(J > 0.0)) {
    flag[0] = 1;
    J = 1.0;
    Jm1 = 0.0;
  }
  const double kappa = lam + 2.0 * mu / 3.0;
  const double cb = cbrt(J);
  const double invJ = 1.0 / J;
  const double sdev = mu * invJ / (cb * cb);
  double B[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) B[a][c] = H[a][c] + H[c][a] + (H[a][0] * H[c][0] + H[a][1] * H[c][1] + H[a][2] * H[c][2]);
  const double trB = (B[0][0] + B[1][1] + B[2][2]) / 3.0;
  const double pr = 0.5 * kappa * Jm1 * (J + 1.0) * invJ;
  double sig[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) sig[a][c] = sdev * (B[a][c] - (a == c ? trB : 0.0)) + (a == c ? pr : 0.0);
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double Pji = sig[j][0] * cof[0][i] + sig[j][1] * cof[1][i] + sig[j][2] * cof[2][i];
      s += sv[i] * Pji;
    }
    t[j] += s;
  }
}

// per-quadrature-point face kernel; MAT 0 linear elastic, 1 neo-Hookean (D = 3)
template <int D, int NQ, int MAT>
__global__ __launch_bounds__(kBlockItems) void k_face_q(int64_t nf, int64_t nfi, int64_t nc, int S,
                                                    const int32_t* __restrict__ blk_item,
                                                    const int32_t* __restrict__ blk_cell,
                                                    const int32_t* __restrict__ ucell,
                                                    const uint16_t* __restrict__ loc, const double* __restrict__ C,
                                                    const int32_t* __restrict__ own, const int32_t* __restrict__ nei,
                                                    const int32_t* __restrict__ slots,
                                                    const double* __restrict__ Sv, const double* __restrict__ stab,
                                                    const double* __restrict__ ghost, double load, double mu,
                                                    double lam, const double* __restrict__ ug,
                                                    const double* __restrict__ ustar, double* __restrict__ F,
                                                    int32_t* __restrict__ flag) {
  __shared__ double lds[D][kLdsFaceCells];
  const int64_t b = xcd_block<8>();
  stage_union<D, kLdsFaceCells>(b, blk_cell, ucell, ug, lds);
  const int64_t i0 = blk_item[b], nb = blk_item[b + 1] - i0, ti = threadIdx.x;
  if (ti >= nb) return;
  const int64_t f = i0 + ti;
  double G[NQ * D][D];  // row q D + i: d u / d x_i at point q
#pragma unroll
  for (int r = 0; r < NQ * D; ++r)
#pragma unroll
    for (int j = 0; j < D; ++j) G[r][j] = 0.0;
  contract_lds<D, NQ * D, kFaceQChunk, kLdsFaceCells>(S, nb, ti, loc + i0 * S, C + i0 * S * NQ * D, lds, G);
  if (MAT == 1 && f >= nfi) {
    const int64_t nfd = nf - nfi, fd = f - nfi;
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
      for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) G[q * D + i][j] += load * ghost[(((int64_t)q * D + i) * D + j) * nfd + fd];
  }
  double t[D];
#pragma unroll
  for (int j = 0; j < D; ++j) t[j] = 0.0;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    double sv[D];
#pragma unroll
    for (int i = 0; i < D; ++i) sv[i] = Sv[((int64_t)q * D + i) * nf + f];
    if constexpr (MAT == 0) {
      double tr = 0.0;
#pragma unroll
      for (int i = 0; i < D; ++i) tr += G[q * D + i][i];
#pragma unroll
      for (int j = 0; j < D; ++j) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i) s += sv[i] * (mu * (G[q * D + i][j] + G[q * D + j][i]) + (i == j ? lam * tr : 0.0));
        t[j] += s;
      }
    } else {
      nh_traction(&G[q * D], sv, mu, lam, t, flag);
    }
  }
  add_stab<D>(f, nfi, nc, own, nei, slots, stab, ustar, t);
#pragma unroll
  for (int j = 0; j < D; ++j) F[(int64_t)j * nf + f] = t[j];
}

// symmetry faces (linear elastic): F_s[j] = sum_N sum_k T[N][j][k] u_N,k over the
// face's half stencil, u from the gather copy; one thread per face
template <int D>
__global__ __launch_bounds__(kBlock) void k_face_sym(int64_t nfs, int Sh, const int32_t* __restrict__ st,
                                                     const double* __restrict__ T, const double* __restrict__ ug,
                                                     double* __restrict__ Fs) {
  constexpr int W = D == 3 ? 4 : 2;
  const int64_t f = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (f >= nfs) return;
  double t[D];
#pragma unroll
  for (int j = 0; j < D; ++j) t[j] = 0.0;
  for (int N = 0; N < Sh; ++N) {
    const int64_t cell = st[(int64_t)N * nfs + f];
    double u[D];
#pragma unroll
    for (int k = 0; k < D; ++k) u[k] = ug[W * cell + k];
#pragma unroll
    for (int j = 0; j < D; ++j)
#pragma unroll
      for (int k = 0; k < D; ++k) t[j] += T[(((int64_t)N * D + j) * D + k) * nfs + f] * u[k];
  }
#pragma unroll
  for (int j = 0; j < D; ++j) Fs[(int64_t)j * nfs + f] = t[j];
}

// symmetry faces, neo-Hookean: the gradient at each point from the cells and
// their images (which carry R u, R = I - 2 n n), then the point traction
template <int NQ>
__global__ __launch_bounds__(kBlock) void k_face_sym_nh(int64_t nfs, int Sh, const int32_t* __restrict__ st,
                                                        const double* __restrict__ C, const double* __restrict__ sv,
                                                        const double* __restrict__ nrm, double mu, double lam,
                                                        const double* __restrict__ ug, double* __restrict__ Fs,
                                                        int32_t* __restrict__ flag) {
  const int64_t f = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (f >= nfs) return;
  const double n[3] = {nrm[f], nrm[nfs + f], nrm[2 * nfs + f]};
  double G[NQ * 3][3];
#pragma unroll
  for (int r = 0; r < NQ * 3; ++r)
#pragma unroll
    for (int j = 0; j < 3; ++j) G[r][j] = 0.0;
  for (int N = 0; N < Sh; ++N) {
    const int64_t cell = st[(int64_t)N * nfs + f];
    const double u[3] = {ug[4 * cell], ug[4 * cell + 1], ug[4 * cell + 2]};
    const double un = u[0] * n[0] + u[1] * n[1] + u[2] * n[2];
    const double ru[3] = {u[0] - 2.0 * un * n[0], u[1] - 2.0 * un * n[1], u[2] - 2.0 * un * n[2]};
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const double c0 = C[((((int64_t)N * NQ + q) * 2 + 0) * 3 + a) * nfs + f];
        const double c1 = C[((((int64_t)N * NQ + q) * 2 + 1) * 3 + a) * nfs + f];
#pragma unroll
        for (int j = 0; j < 3; ++j) G[q * 3 + a][j] += c0 * u[j] + c1 * ru[j];
      }
  }
  double t[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const double s[3] = {sv[((int64_t)q * 3) * nfs + f], sv[((int64_t)q * 3 + 1) * nfs + f],
                         sv[((int64_t)q * 3 + 2) * nfs + f]};
    nh_traction(&G[q * 3], s, mu, lam, t, flag);
  }
#pragma unroll
  for (int j = 0; j < 3; ++j) Fs[(int64_t)j * nfs + f] = t[j];
}

// NST > 0: NST face slots per cell, thread k takes cell k.  NST = 0 (face-list
// meshes with ns > 2 D slots, of which a cell uses its first ones): order[]
// lists the n_big cells with more than 2 D faces first; the
// first n_big g threads take those, g lanes a cell (lane l: slots l, l + g,
// ..., added up by shuffles within the group), the others one cell each over
// its first 2 D slots.
template <int D, int NST>
__global__ __launch_bounds__(kBlock) void k_cell_sum(int64_t nc, int64_t nf, int ns, const int32_t* __restrict__ cf,
                                                      const double* __restrict__ F, const double* __restrict__ src,
                                                      double load, const double* __restrict__ Ru,
                                                      const double* __restrict__ eps, const double* __restrict__ ug,
                                                      const double* __restrict__ dm, const double* __restrict__ ds,
                                                      const double* __restrict__ Fs, int64_t nfs,
                                                      double* __restrict__ R, const int32_t* __restrict__ order,
                                                      int64_t n_big, int g) {
  constexpr int W = D == 3 ? 4 : 2;
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double acc[D];
#pragma unroll
  for (int c = 0; c < D; ++c) acc[c] = 0.0;
  auto take = [&](int32_t f) {
    if (f == kNoFace) return;
#pragma unroll
    for (int c = 0; c < D; ++c) {
      if (f >= nf) acc[c] += Fs[(int64_t)c * nfs + (f - nf)];  // symmetry face
      else if (f >= 0) acc[c] += F[(int64_t)c * nf + f];
      else acc[c] -= F[(int64_t)c * nf + ~f];
    }
  };
  int64_t P;
  // R(u)'s entries of the cell are loaded as soon as P is known, alongside the fluxes
  double ru[D], e = 0.0;
  auto own = [&]() {
#pragma unroll
    for (int c = 0; c < D; ++c) ru[c] = Ru ? Ru[(int64_t)c * nc + P] : 0.0;
    if (Ru) e = eps[0];
  };
  const int64_t nbt = NST > 0 ? 0 : n_big * g;  // threads of the many-faced cells
  if (NST == 0 && k < nbt) {
    P = order[k / g];
    const int l = (int)(k % g);
    // a lane's slot ids are loaded together before the fluxes they point to
    for (int s0 = l; s0 < ns; s0 += 8 * g) {
      int32_t f[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) f[j] = s0 + j * g < ns ? cf[(int64_t)(s0 + j * g) * nc + P] : kNoFace;
#pragma unroll
      for (int j = 0; j < 8; ++j) take(f[j]);
    }
    // groups are aligned within the wavefront (g divides 64 and every lane of
    // a group is below nbt), so the butterfly stays inside the group
    for (int o = g / 2; o > 0; o >>= 1)
#pragma unroll
      for (int c = 0; c < D; ++c) acc[c] += __shfl_xor(acc[c], o, 64);
    if (l != 0) return;
    own();
#pragma unroll
    for (int c = 0; c < D; ++c) acc[c] += load * src[(int64_t)c * nc + P];
  } else {
    const int64_t i = NST > 0 ? k : k - nbt + n_big;
    if (i >= nc) return;
    P = NST > 0 ? i : (int64_t)order[i];
    own();
#pragma unroll
    for (int c = 0; c < D; ++c) acc[c] = load * src[(int64_t)c * nc + P];
    constexpr int S0 = NST > 0 ? NST : 2 * D;
    int32_t f0[S0];
#pragma unroll
    for (int s = 0; s < S0; ++s) f0[s] = cf[(int64_t)s * nc + P];
    if (nfs == 0 && nf > 0) {
      // no symmetry faces: the row is selected rather than branched on, so
      // that the loads of all slots are in flight together (an empty slot
      // reads row 0 and adds nothing)
      double v[S0][D];
#pragma unroll
      for (int s = 0; s < S0; ++s) {
        const int32_t f = f0[s];
        const int64_t i = f == kNoFace ? 0 : f < 0 ? (int64_t)~f : (int64_t)f;
#pragma unroll
        for (int c = 0; c < D; ++c) v[s][c] = F[(int64_t)c * nf + i];
      }
#pragma unroll
      for (int s = 0; s < S0; ++s)
#pragma unroll
        for (int c = 0; c < D; ++c)
          acc[c] = f0[s] == kNoFace ? acc[c] : f0[s] < 0 ? acc[c] - v[s][c] : acc[c] + v[s][c];
    } else {
#pragma unroll
      for (int s = 0; s < S0; ++s) take(f0[s]);
    }
  }
#pragma unroll
  for (int c = 0; c < D; ++c) {
    double a = acc[c];
    // BDF2 inertia at the centroid: s_P - m_P u_P (u from the gather copy)
    if (dm) a += ds[(int64_t)c * nc + P] - dm[P] * ug[(int64_t)W * P + c];
    if (Ru) a = e > 0.0 ? (a - ru[c]) / e : 0.0;
    R[(int64_t)c * nc + P] = a;
  }
}

// ---- eps = sqrt((1 + ||u||) eps_mach) / ||v|| on the device -----------------

// partials of ||u||^2 and ||v||^2: part[block], part[kRedParts + block]
__global__ __launch_bounds__(kBlock) void k_sumsq2(int64_t n, const double* __restrict__ a,
                                                   const double* __restrict__ b, double* __restrict__ part) {
  __shared__ double sred[(kBlock / 64) * 2], sout[2];
  double acc[2] = {0.0, 0.0};
  // a thread's strided entries are loaded 8 at a time and added in index
  // order (an entry past n loads as 0 and adds nothing to the sums of squares)
  constexpr int U = 8;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i0 = (int64_t)blockIdx.x * kBlock + threadIdx.x; i0 < n; i0 += U * stride) {
    double x[U], y[U];
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const int64_t i = i0 + j * stride;
      x[j] = i < n ? a[i] : 0.0;
      y[j] = i < n ? b[i] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < U; ++j) {
      acc[0] += x[j] * x[j];
      acc[1] += y[j] * y[j];
    }
  }
  block_reduce<2, kBlock>(acc, sred, sout);
  if (threadIdx.x < 2) part[threadIdx.x * kRedParts + blockIdx.x] = sout[threadIdx.x];
}

// Padded gather copy of u (+ eps v when v != null): ug[P][0..D) = u[.][P] + eps v[.][P].
// eps is eps_host when nb == 0, else sqrt((1 + ||u||) eps_mach) / ||v|| (0 when
// v = 0) from the nb block partials of k_sumsq2, added up by every block in
// the same fixed order; block 0 stores it at eps_out for the cell sum.
template <int D>
__global__ __launch_bounds__(kBlock) void k_pack(int64_t nc, const double* __restrict__ u,
                                                 const double* __restrict__ v, double eps_host, int nb,
                                                 const double* __restrict__ part, double* __restrict__ eps_out,
                                                 double* __restrict__ ug) {
  constexpr int W = D == 3 ? 4 : 2;
  const int64_t P = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const bool live = P < nc;
  // the cell's u and v are loaded before the partials are added up
  double uu[D], vv[D];
#pragma unroll
  for (int c = 0; c < D; ++c) {
    uu[c] = live ? u[(int64_t)c * nc + P] : 0.0;
    vv[c] = v && live ? v[(int64_t)c * nc + P] : 0.0;
  }
  double e = eps_host;
  if (v && nb > 0) {
    __shared__ double sred[(kBlock / 64) * 2], sn[2];
    double a[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int t = threadIdx.x;
      double s = t < nb ? part[q * kRedParts + t] : 0.0;
      if (t + kBlock < nb) s += part[q * kRedParts + t + kBlock];
      a[q] = s;
    }
    block_reduce<2, kBlock>(a, sred, sn);
    const double nu = sqrt(sn[0]), nv = sqrt(sn[1]);
    e = nv > 0.0 ? sqrt((1.0 + nu) * DBL_EPSILON) / nv : 0.0;
  }
  if (v && blockIdx.x == 0 && threadIdx.x == 0) eps_out[0] = e;
  if (!live) return;
  double x[W];
#pragma unroll
  for (int c = 0; c < W; ++c) x[c] = 0.0;
#pragma unroll
  for (int c = 0; c < D; ++c) x[c] = v ? uu[c] + e * vv[c] : uu[c];
  double2* o = reinterpret_cast<double2*>(ug + (int64_t)W * P);
  o[0] = make_double2(x[0], x[1]);
  if constexpr (W == 4) o[1] = make_double2(x[2], x[3]);
}

// ---- FP32 multicolour Gauss-Seidel ----------------------------------------

template <int D>
__global__ __launch_bounds__(kBlock) void k_pc_in(int64_t nc, const int32_t* __restrict__ perm,
                                                  const double* __restrict__ r, float* __restrict__ r32,
                                                  float* __restrict__ z32) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= nc) return;
  const int32_t P = perm[i];
#pragma unroll
  for (int c = 0; c < D; ++c) {
    r32[(int64_t)c * nc + i] = (float)r[(int64_t)c * nc + P];
    z32[(int64_t)c * nc + i] = 0.0f;
  }
}

// acc -= sum over a row's slots of a_s z[nbr_s]: NST slots known at compile
// time, or (NST = 0) 2 D slots and then slots 2 D .. nsb - 1 when nsb > 0,
// 8 a step; each step loads its slot entries together before the gathers.
// Unused slots hold the row itself with a zero coefficient.
template <int D, int NST>
__device__ inline void slot_products(float (&acc)[D], int64_t i, int64_t n, int nsb, const int32_t* __restrict__ nbr,
                                     const float* __restrict__ a, const float* __restrict__ z) {
  constexpr int S0 = NST > 0 ? NST : 2 * D;
  int32_t N0[S0];
  float a0[S0];
#pragma unroll
  for (int s = 0; s < S0; ++s) {
    N0[s] = nbr[(int64_t)s * n + i];
    a0[s] = a[(int64_t)s * n + i];
  }
#pragma unroll
  for (int s = 0; s < S0; ++s)
#pragma unroll
    for (int c = 0; c < D; ++c) acc[c] -= a0[s] * z[(int64_t)c * n + N0[s]];
  if (NST > 0) return;
  for (int s0 = S0; s0 < nsb; s0 += 8) {
    int32_t N[8];
    float aa[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const bool in = s0 + j < nsb;
      N[j] = in ? nbr[(int64_t)(s0 + j) * n + i] : (int32_t)i;
      aa[j] = in ? a[(int64_t)(s0 + j) * n + i] : 0.0f;
    }
#pragma unroll
    for (int j = 0; j < 8; ++j)
#pragma unroll
      for (int c = 0; c < D; ++c) acc[c] -= aa[j] * z[(int64_t)c * n + N[j]];
  }
}

// NST > 0: one lane a position, NST slots.  NST = 0 (ns > 2 D slots): the
// positions begin .. big_end - 1 (cells with more than 2 D faces) take g lanes
// each (lane l: slots l, l + g, ..., added up by shuffles within the group),
// the others one lane over their first 2 D slots
template <int D, int NST>
__global__ __launch_bounds__(kBlock) void k_pc_sweep(int64_t nc, int64_t begin, int64_t end, int ns,
                                                     const int32_t* __restrict__ nbr, const float* __restrict__ a,
                                                     const float* __restrict__ dinv, const float* __restrict__ r32,
                                                     float* __restrict__ z32, int64_t big_end, int g) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t nbt = NST > 0 ? 0 : (big_end - begin) * g;
  float acc[D];
  int64_t i;
  if (NST == 0 && k < nbt) {
    i = begin + k / g;
    const int l = (int)(k % g);
#pragma unroll
    for (int c = 0; c < D; ++c) acc[c] = 0.0f;
    for (int s0 = l; s0 < ns; s0 += 8 * g) {
      int32_t N[8];
      float aa[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const bool in = s0 + j * g < ns;
        N[j] = in ? nbr[(int64_t)(s0 + j * g) * nc + i] : (int32_t)i;
        aa[j] = in ? a[(int64_t)(s0 + j * g) * nc + i] : 0.0f;
      }
#pragma unroll
      for (int j = 0; j < 8; ++j)
#pragma unroll
        for (int c = 0; c < D; ++c) acc[c] -= aa[j] * z32[(int64_t)c * nc + N[j]];
    }
    // groups are aligned within the wavefront (g divides 64, all lanes of a
    // group are below nbt)
    for (int o = g / 2; o > 0; o >>= 1)
#pragma unroll
      for (int c = 0; c < D; ++c) acc[c] += __shfl_xor(acc[c], o, 64);
    if (l != 0) return;
#pragma unroll
    for (int c = 0; c < D; ++c) acc[c] += r32[(int64_t)c * nc + i];
  } else {
    i = begin + (NST > 0 ? k : k - nbt + (big_end - begin));
    if (i >= end) return;
#pragma unroll
    for (int c = 0; c < D; ++c) acc[c] = r32[(int64_t)c * nc + i];
    slot_products<D, NST>(acc, i, nc, 0, nbr, a, z32);
  }
  const float di = dinv[i];
#pragma unroll
  for (int c = 0; c < D; ++c) z32[(int64_t)c * nc + i] = acc[c] * di;
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_pc_out(int64_t nc, const int32_t* __restrict__ perm,
                                                   const float* __restrict__ z32, double* __restrict__ z) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= nc) return;
  const int32_t P = perm[i];
#pragma unroll
  for (int c = 0; c < D; ++c) z[(int64_t)c * nc + P] = (double)z32[(int64_t)c * nc + i];
}

// ---- multigrid V-cycle on the approximate Jacobian (FP32, D right-hand sides)

// t = r - A z on level 0 (slot rows in colour-major order); NST = 0 (ns > 2 D
// slots): rows flagged in big walk all ns slots, the others the first 2 D
template <int D, int NST>
__global__ __launch_bounds__(kBlock) void k_mg_res0(int64_t n, int ns, const int32_t* __restrict__ nbr,
                                                    const float* __restrict__ a, const float* __restrict__ diag,
                                                    const float* __restrict__ r, const float* __restrict__ z,
                                                    float* __restrict__ t, const uint8_t* __restrict__ big) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const float di = diag[i];
  float acc[D];
#pragma unroll
  for (int c = 0; c < D; ++c) acc[c] = r[(int64_t)c * n + i] - di * z[(int64_t)c * n + i];
  slot_products<D, NST>(acc, i, n, NST > 0 || !big[i] ? 0 : ns, nbr, a, z);
#pragma unroll
  for (int c = 0; c < D; ++c) t[(int64_t)c * n + i] = acc[c];
}

// CSR row products with G lanes per row (G a power of two <= 64): lane l of a
// row's group takes entries l, l + G, ...; the partial sums are combined by
// butterfly shuffles within the wavefront
template <int G>
__device__ inline float group_sum(float v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// t = r - A z on a coarse level (off-diagonal CSR + diagonal)
template <int D, int G>
__global__ __launch_bounds__(kBlock) void k_mg_res(int64_t n, const int32_t* __restrict__ ptr,
                                                   const int32_t* __restrict__ col, const float* __restrict__ val,
                                                   const float* __restrict__ diag, const float* __restrict__ r,
                                                   const float* __restrict__ z, float* __restrict__ t) {
  const int64_t g = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / G;
  const int lane = threadIdx.x % G;
  const bool live = g < n;
  const int64_t i = live ? g : n - 1;
  float acc[D];
#pragma unroll
  for (int c = 0; c < D; ++c) acc[c] = 0.0f;
  if (live)
    for (int32_t u = ptr[i] + lane; u < ptr[i + 1]; u += G) {
      const int32_t j = col[u];
      const float v = val[u];
#pragma unroll
      for (int c = 0; c < D; ++c) acc[c] += v * z[(int64_t)c * n + j];
    }
#pragma unroll
  for (int c = 0; c < D; ++c) acc[c] = group_sum<G>(acc[c]);
  if (!live || lane != 0) return;
  const float di = diag[i];
#pragma unroll
  for (int c = 0; c < D; ++c) t[(int64_t)c * n + i] = r[(int64_t)c * n + i] - di * z[(int64_t)c * n + i] - acc[c];
}

// y = M x (add = 0) or y += M x (add = 1), M in CSR with ny rows over nx columns
template <int D, int G>
__global__ __launch_bounds__(kBlock) void k_mg_spmv(int64_t ny, const int32_t* __restrict__ ptr,
                                                    const int32_t* __restrict__ col, const float* __restrict__ val,
                                                    const float* __restrict__ x, int64_t nx, float* __restrict__ y,
                                                    int add) {
  const int64_t g = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / G;
  const int lane = threadIdx.x % G;
  const bool live = g < ny;
  const int64_t i = live ? g : ny - 1;
  float acc[D];
#pragma unroll
  for (int c = 0; c < D; ++c) acc[c] = 0.0f;
  if (live)
    for (int32_t u = ptr[i] + lane; u < ptr[i + 1]; u += G) {
      const int32_t j = col[u];
      const float v = val[u];
#pragma unroll
      for (int c = 0; c < D; ++c) acc[c] += v * x[(int64_t)c * nx + j];
    }
#pragma unroll
  for (int c = 0; c < D; ++c) acc[c] = group_sum<G>(acc[c]);
  if (!live || lane != 0) return;
#pragma unroll
  for (int c = 0; c < D; ++c) y[(int64_t)c * ny + i] = (add ? y[(int64_t)c * ny + i] : 0.0f) + acc[c];
}

// first damped Jacobi step from z = 0: z = w_i r_i
template <int D>
__global__ __launch_bounds__(kBlock) void k_mg_jinit(int64_t n, const float* __restrict__ wdinv,
                                                     const float* __restrict__ r, float* __restrict__ z) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const float w = wdinv[i];
#pragma unroll
  for (int c = 0; c < D; ++c) z[(int64_t)c * n + i] = w * r[(int64_t)c * n + i];
}

// one damped Jacobi step into the other iterate: zo = z + w_i (r - A z)_i,
// the residual formed as in k_mg_res
template <int D, int G>
__global__ __launch_bounds__(kBlock) void k_mg_jstep(int64_t n, const int32_t* __restrict__ ptr,
                                                     const int32_t* __restrict__ col, const float* __restrict__ val,
                                                     const float* __restrict__ diag, const float* __restrict__ wdinv,
                                                     const float* __restrict__ r, const float* __restrict__ z,
                                                     float* __restrict__ zo) {
  const int64_t g = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / G;
  const int lane = threadIdx.x % G;
  const bool live = g < n;
  const int64_t i = live ? g : n - 1;
  float acc[D];
#pragma unroll
  for (int c = 0; c < D; ++c) acc[c] = 0.0f;
  if (live)
    for (int32_t u = ptr[i] + lane; u < ptr[i + 1]; u += G) {
      const int32_t j = col[u];
      const float v = val[u];
#pragma unroll
      for (int c = 0; c < D; ++c) acc[c] += v * z[(int64_t)c * n + j];
    }
#pragma unroll
  for (int c = 0; c < D; ++c) acc[c] = group_sum<G>(acc[c]);
  if (!live || lane != 0) return;
  const float di = diag[i], w = wdinv[i];
#pragma unroll
  for (int c = 0; c < D; ++c) {
    const float zi = z[(int64_t)c * n + i];
    const float t = r[(int64_t)c * n + i] - di * zi - acc[c];
    zo[(int64_t)c * n + i] = zi + w * t;
  }
}

// z = C r with the coarsest level's dense inverse C (column-major)
template <int D>
__global__ __launch_bounds__(kBlock) void k_mg_dense(int64_t n, const float* __restrict__ cinv,
                                                     const float* __restrict__ r, float* __restrict__ z) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  float acc[D];
#pragma unroll
  for (int c = 0; c < D; ++c) acc[c] = 0.0f;
  for (int64_t k = 0; k < n; ++k) {
    const float v = cinv[k * n + i];
#pragma unroll
    for (int c = 0; c < D; ++c) acc[c] += v * r[(int64_t)c * n + k];
  }
#pragma unroll
  for (int c = 0; c < D; ++c) z[(int64_t)c * n + i] = acc[c];
}

}  // namespace

// ---------------------------------------------------------------------------
// events come from a pool kept by the context (created once, reused after
// every hofv_set_timing), so a timed launch costs two event records only
static hipEvent_t pooled_event(hofv_ctx* c) {
  if (c->ev_used == c->ev_pool.size()) {
    hipEvent_t e;
    hipEventCreate(&e);
    c->ev_pool.push_back(e);
  }
  return c->ev_pool[c->ev_used++];
}

void timer_begin(hofv_ctx* c, const char* name, hipStream_t st, hipEvent_t* ev) {
  *ev = nullptr;
  if (!c->timing || (!c->timing_only.empty() && c->timing_only != name)) return;
  *ev = pooled_event(c);
  hipEventRecord(*ev, st);
}

void timer_end(hofv_ctx* c, const char* name, hipStream_t st, hipEvent_t ev) {
  if (!c->timing || !ev) return;
  hipEvent_t e2 = pooled_event(c);
  hipEventRecord(e2, st);
  c->timers.push_back({name, ev, e2});
}

#define TIMED(name, launch)              \
  do {                                   \
    hipEvent_t ev_;                      \
    timer_begin(c, name, st, &ev_);      \
    launch;                              \
    timer_end(c, name, st, ev_);         \
  } while (0)

// R(ug) where ug is the padded gather copy (k_pack)
template <int D>
static hofv_status residual_impl(hofv_ctx* c, const double* u, double* R, const double* Ru, const double* eps,
                                 hipStream_t st) {
  DeviceTables& t = c->dev;
  const int64_t nc = c->nc, nf = t.nf;
  const bool nh = c->prm.material == HOFV_NEO_HOOKEAN;
  const bool fold = !nh && c->prm.fold_quadrature;
  const int64_t ni = t.n_items;  // u* is indexed by extrapolation item
  // one item per face (nsi = 1), or per cell with as many slots as the most
  // faces of a cell: dim + 1 (simplices) to 2 dim (quads, hexahedra)
#define EXTRAP(NSI)                                                                                         \
  TIMED("k_extrap", (k_extrap<D, NSI><<<t.ncb, kBlockItems, 0, st>>>(ni, t.S, t.c_blk_item, t.c_blk_cell, \
                                                                     t.c_ucell, t.c_local, t.c_extrap, t.c_cell, u, \
                                                                     t.ustar)))
  if (t.nsi == 1) EXTRAP(1);
  else if (t.nsi == D + 1) EXTRAP(D + 1);
  else if (t.nsi == 2 * D - 1) EXTRAP(2 * D - 1);  // in 3D: cells of at most five faces
  else if (t.nsi == 2 * D) EXTRAP(2 * D);
  else return fail(c, HOFV_EINVAL, "unsupported number of face slots per extrapolation item");
#undef EXTRAP
  if (nf > 0) {
    if (fold) {
      TIMED("k_face_le", (k_face_le<D><<<t.nfb, kBlockItems, 0, st>>>(
                             nf, t.nfi, ni, t.S, t.f_blk_item, t.f_blk_cell, t.f_ucell, t.f_local, t.f_coef, t.f_own,
                             t.f_nei, t.f_slots, t.f_area_vec, t.f_stab, c->prm.mu, c->prm.lambda, u, t.ustar,
                             t.flux)));
    } else {
#define FACEQ(NQ, MAT, NAME)                                                                                  \
  TIMED(NAME, (k_face_q<D, NQ, MAT><<<t.nfb, kBlockItems, 0, st>>>(                                                \
                  nf, t.nfi, ni, t.S, t.f_blk_item, t.f_blk_cell, t.f_ucell, t.f_local, t.f_coef, t.f_own,     \
                  t.f_nei, t.f_slots, t.f_area_vec, t.f_stab, t.f_ghost, c->load, c->prm.mu, c->prm.lambda, u, \
                  t.ustar, t.flux, t.flag)))
      const int nq = t.nq;
      if (nh) {
        if constexpr (D == 3) {
          if (nq == 1) FACEQ(1, 1, "k_face_nh");
          else if (nq == 2) FACEQ(2, 1, "k_face_nh");
          else if (nq == 4) FACEQ(4, 1, "k_face_nh");
          else if (nq == 8) FACEQ(8, 1, "k_face_nh");
          else if (nq == 9) FACEQ(9, 1, "k_face_nh");
          else return fail(c, HOFV_EINVAL, "unsupported number of face quadrature points");
        } else {
          return fail(c, HOFV_EINVAL, "the neo-Hookean law needs dim = 3");
        }
      } else {
        if (nq == 1) FACEQ(1, 0, "k_face_q");
        else if (nq == 2) FACEQ(2, 0, "k_face_q");
        else if (nq == 3) FACEQ(3, 0, "k_face_q");
        else if (nq == 4) FACEQ(4, 0, "k_face_q");
        else if (nq == 8) FACEQ(8, 0, "k_face_q");
        else if (nq == 9) FACEQ(9, 0, "k_face_q");
        else return fail(c, HOFV_EINVAL, "unsupported number of face quadrature points");
      }
#undef FACEQ
    }
  }
  if (t.sym_nf > 0) {
    if (!nh) {
      k_face_sym<D><<<blocks_for(t.sym_nf), kBlock, 0, st>>>(t.sym_nf, t.sym_S, t.sym_st, t.sym_T, u, t.sym_flux);
    } else if constexpr (D == 3) {
      const unsigned g = blocks_for(t.sym_nf);
#define SYMNH(Q)                                                                                                    \
  k_face_sym_nh<Q><<<g, kBlock, 0, st>>>(t.sym_nf, t.sym_S, t.sym_st, t.sym_C, t.sym_sv, t.sym_n, c->prm.mu,        \
                                         c->prm.lambda, u, t.sym_flux, t.flag)
      if (t.nq == 1) SYMNH(1);
      else if (t.nq == 2) SYMNH(2);
      else if (t.nq == 4) SYMNH(4);
      else if (t.nq == 8) SYMNH(8);
      else if (t.nq == 9) SYMNH(9);
      else return fail(c, HOFV_EINVAL, "unsupported number of face quadrature points");
#undef SYMNH
    }
  }
  // simplices (every face in a cell's first dim + 1 slots) walk those slots only
  if (t.ns == 2 * D && t.nsi == D + 1)
    TIMED("k_cell_sum", (k_cell_sum<D, D + 1><<<blocks_for(nc), kBlock, 0, st>>>(
                            nc, nf, t.ns, t.c_faces, t.flux, t.c_src, c->load, Ru, eps, u, t.dyn_m, t.dyn_s,
                            t.sym_flux, t.sym_nf, R, nullptr, 0, 1)));
  else if (t.ns == 2 * D)
    TIMED("k_cell_sum", (k_cell_sum<D, 2 * D><<<blocks_for(nc), kBlock, 0, st>>>(
                            nc, nf, t.ns, t.c_faces, t.flux, t.c_src, c->load, Ru, eps, u, t.dyn_m, t.dyn_s,
                            t.sym_flux, t.sym_nf, R, nullptr, 0, 1)));
  else  // face-list meshes with cells of more than 2 dim faces
    TIMED("k_cell_sum", (k_cell_sum<D, 0><<<blocks_for(nc + t.n_big * (t.grp - 1)), kBlock, 0, st>>>(
                            nc, nf, t.ns, t.c_faces, t.flux, t.c_src, c->load, Ru, eps, u, t.dyn_m, t.dyn_s,
                            t.sym_flux, t.sym_nf, R, t.c_order, t.n_big, t.grp)));
  HOFV_HIP(c, hipGetLastError());
  return HOFV_OK;
}

hofv_status launch_residual(hofv_ctx* c, const double* u, double* R, const double* Ru, const double* eps,
                            hipStream_t st) {
  // Ru == nullptr: R = R(u).  Otherwise u is the packed copy already made by
  // launch_jvp_pack (u + eps v) and R receives (R(u + eps v) - Ru) / eps.
  if (!Ru) {
    if (c->D == 2) k_pack<2><<<blocks_for(c->nc), kBlock, 0, st>>>(c->nc, u, nullptr, 0.0, 0, nullptr, nullptr, c->dev.w);
    else k_pack<3><<<blocks_for(c->nc), kBlock, 0, st>>>(c->nc, u, nullptr, 0.0, 0, nullptr, nullptr, c->dev.w);
  }
  const double* ug = c->dev.w;
  return c->D == 2 ? residual_impl<2>(c, ug, R, Ru, eps, st) : residual_impl<3>(c, ug, R, Ru, eps, st);
}

// The near-exact Jacobian of App. C: the derivative of the discrete linear
// elastic equations without the alpha-stabilisation.  The residual is affine
// in u, so with the stabilisation coefficients, the loads and the inertia
// source set to zero it is that linear operator itself (for dynamics, minus
// the mass term m_P, which belongs to the step's Jacobian).
hofv_status launch_nej(hofv_ctx* c, const double* v, double* out, hipStream_t st) {
  DeviceTables& t = c->dev;
  const double load = c->load;
  double* stab = t.f_stab;
  double* ds = t.dyn_s;
  c->load = 0.0;
  t.f_stab = c->nej.zero;
  if (t.dyn_m) t.dyn_s = c->nej.zero;
  // the launches take the values at enqueue time; restore them at once
  const hofv_status s = launch_residual(c, v, out, nullptr, nullptr, st);
  c->load = load;
  t.f_stab = stab;
  t.dyn_s = ds;
  return s;
}

// u + eps v into the gather copy, eps = eps_host if > 0, else from device norms
// (k_sumsq2's partials, added up inside k_pack); eps lands in dev.eps
hofv_status launch_jvp_pack(hofv_ctx* c, const double* u, const double* v, double eps_host, hipStream_t st) {
  DeviceTables& t = c->dev;
  const int64_t nc = c->nc, n = (int64_t)c->D * nc;
  int nb = 0;
  if (!(eps_host > 0)) {
    nb = (int)std::min<int64_t>(kRedParts, blocks_for(n));
    TIMED("k_sumsq2", (k_sumsq2<<<nb, kBlock, 0, st>>>(n, u, v, t.scratch)));
  }
  const double e = eps_host > 0 ? eps_host : 0.0;
  if (c->D == 2)
    TIMED("k_pack", (k_pack<2><<<blocks_for(nc), kBlock, 0, st>>>(nc, u, v, e, nb, t.scratch, t.eps, t.w)));
  else
    TIMED("k_pack", (k_pack<3><<<blocks_for(nc), kBlock, 0, st>>>(nc, u, v, e, nb, t.scratch, t.eps, t.w)));
  HOFV_HIP(c, hipGetLastError());
  return HOFV_OK;
}

// ---- J.v without library allocations ---------------------------------------
// hofv_jvp_noalloc keeps the partial sums of its device eps and eps itself in
// this file-scope array instead of the context's buffers.  Each GPU holds one
// copy until the process ends, and every call on that GPU shares it.  In host
// code `scratch` names a host-side stand-in: kernels get the device address
// that noalloc_init looked up, never the name itself.
constexpr int64_t kNoAllocDoubles = 2048;  // 16 KiB
static __device__ __align__(256) double scratch[kNoAllocDoubles];

namespace {
std::mutex g_noalloc_mu;
std::map<int, double*> g_noalloc_ptr;  // device -> address of `scratch` on it
}  // namespace

// Looks up the device address of `scratch` on the context's device (current
// here), once per device.  Called by hofv_setup.
hofv_status noalloc_init(hofv_ctx* c) {
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (g_noalloc_ptr.count(c->device)) return HOFV_OK;
  double* p = nullptr;
  const hipError_t e = hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return fail(c, HOFV_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_noalloc_ptr[c->device] = p;
  return HOFV_OK;
}

// The J.v of jvp_impl with the eps partials (2 x nb) and eps in `scratch`;
// no allocation and no timing events.
hofv_status jvp_noalloc_impl(hofv_ctx* c, const double* u, const double* Ru, const double* v, double* Jv,
                             double eps_host, hipStream_t st) {
  double* buf = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    auto it = g_noalloc_ptr.find(c->device);
    if (it != g_noalloc_ptr.end()) buf = it->second;
  }
  if (!buf) return fail(c, HOFV_ESTATE, "the static scratch of this device was not looked up (hofv_setup)");
  const int64_t nc = c->nc, n = (int64_t)c->D * nc;
  const int nb = eps_host > 0 ? 0 : (int)std::min<int64_t>(kRedParts, blocks_for(n));
  // partials [2][kRedParts] then eps
  const int64_t need = 2 * (int64_t)kRedParts + 1;
  if (need > kNoAllocDoubles)
    return fail(c, HOFV_EINVAL, "the J.v reduction needs more than the 2048-double static scratch");
  double* part = buf;
  double* eps_dev = buf + 2 * kRedParts;
  DeviceTables& t = c->dev;
  if (nb > 0) k_sumsq2<<<nb, kBlock, 0, st>>>(n, u, v, part);
  const double e = eps_host > 0 ? eps_host : 0.0;
  if (c->D == 2) k_pack<2><<<blocks_for(nc), kBlock, 0, st>>>(nc, u, v, e, nb, part, eps_dev, t.w);
  else k_pack<3><<<blocks_for(nc), kBlock, 0, st>>>(nc, u, v, e, nb, part, eps_dev, t.w);
  HOFV_HIP(c, hipGetLastError());
  const bool timing = c->timing;  // timing events could be created on first use
  c->timing = false;
  const hofv_status s = launch_residual(c, t.w, Jv, Ru, eps_dev, st);
  c->timing = timing;
  return s;
}

// s symmetric multicolour Gauss-Seidel sweeps on level 0, continuing from p_z:
// colours 0..C-1 then C-1..0; an immediately repeated colour is skipped
// (cells of one colour are uncoupled, so it is a no-op)
template <int D>
static void sgs_sweeps(hofv_ctx* c, int sweeps, hipStream_t st) {
  DeviceTables& t = c->dev;
  const int64_t nc = c->nc;
  int last = -1;
  for (int s = 0; s < sweeps; ++s) {
    for (int pass = 0; pass < 2; ++pass)
      for (int k = 0; k < t.n_colours; ++k) {
        const int col = pass == 0 ? k : t.n_colours - 1 - k;
        if (col == last) continue;
        last = col;
        const int64_t b = t.colour_start[col], e = t.colour_start[col + 1];
        if (e > b && t.ns == 2 * D && t.nsi == D + 1)  // simplices: dim + 1 slots
          TIMED("k_pc_sweep", (k_pc_sweep<D, D + 1><<<blocks_for(e - b), kBlock, 0, st>>>(
                                  nc, b, e, t.ns, t.p_nbr, t.p_a, t.p_dinv, t.p_r, t.p_z, b, 1)));
        else if (e > b && t.ns == 2 * D)
          TIMED("k_pc_sweep", (k_pc_sweep<D, 2 * D><<<blocks_for(e - b), kBlock, 0, st>>>(
                                  nc, b, e, t.ns, t.p_nbr, t.p_a, t.p_dinv, t.p_r, t.p_z, b, 1)));
        else if (e > b)  // the colour's cells with more than 2 dim faces come first
          TIMED("k_pc_sweep",
                (k_pc_sweep<D, 0><<<blocks_for(e - b + (t.colour_big_end[col] - b) * (t.grp - 1)), kBlock, 0, st>>>(
                    nc, b, e, t.ns, t.p_nbr, t.p_a, t.p_dinv, t.p_r, t.p_z, t.colour_big_end[col], t.grp)));
      }
  }
}

template <int D>
static void mg_res(int64_t n, const int32_t* ptr, const int32_t* col, const float* val, const float* diag,
                   const float* r, const float* z, float* t, int g, hipStream_t st) {
  const unsigned nb = blocks_for(n * g);
#define RES(G) k_mg_res<D, G><<<nb, kBlock, 0, st>>>(n, ptr, col, val, diag, r, z, t)
  switch (g) {
    case 1: RES(1); break;
    case 2: RES(2); break;
    case 4: RES(4); break;
    case 8: RES(8); break;
    case 16: RES(16); break;
    case 32: RES(32); break;
    default: RES(64); break;
  }
#undef RES
}

template <int D>
static void mg_spmv(int64_t ny, const int32_t* ptr, const int32_t* col, const float* val, const float* x, int64_t nx,
                    float* y, int add, int g, hipStream_t st) {
  const unsigned nb = blocks_for(ny * g);
#define SPMV(G) k_mg_spmv<D, G><<<nb, kBlock, 0, st>>>(ny, ptr, col, val, x, nx, y, add)
  switch (g) {
    case 1: SPMV(1); break;
    case 2: SPMV(2); break;
    case 4: SPMV(4); break;
    case 8: SPMV(8); break;
    case 16: SPMV(16); break;
    case 32: SPMV(32); break;
    default: SPMV(64); break;
  }
#undef SPMV
}

// steps damped Jacobi steps zo = z + w (r - A z) on a coarse level, each into
// the other of its two iterates; returns the one holding the result
template <int D>
static float* mg_jacobi_steps(DeviceTables::MgLevel& m, float* z, int steps, hipStream_t st) {
  const unsigned nb = blocks_for(m.n * m.g_a);
  for (int s = 0; s < steps; ++s) {
    float* zo = z == m.z ? m.z2 : m.z;
#define JSTEP(G) k_mg_jstep<D, G><<<nb, kBlock, 0, st>>>(m.n, m.ptr, m.col, m.val, m.diag, m.wdinv, m.r, z, zo)
    switch (m.g_a) {
      case 1: JSTEP(1); break;
      case 2: JSTEP(2); break;
      case 4: JSTEP(4); break;
      case 8: JSTEP(8); break;
      case 16: JSTEP(16); break;
      case 32: JSTEP(32); break;
      default: JSTEP(64); break;
    }
#undef JSTEP
    z = zo;
  }
  return z;
}

// V-cycle on level l for r_l (level 0: p_r), result in z_l (level 0: p_z, zero on
// entry).  Level 0 is smoothed by Gauss-Seidel sweeps, coarser levels by damped
// Jacobi steps: the first from z = 0 (z = w r), the others each forming the
// residual and the update in one launch, alternating between z and z2 so that
// the 2 sweeps - 1 of them end in z.
template <int D>
static void mg_vcycle(hofv_ctx* c, int l, int sweeps, hipStream_t st) {
  DeviceTables& t = c->dev;
  DeviceTables::MgLevel& m = t.mg[l];
  const int nl = (int)t.mg.size();
  float* r = l == 0 ? t.p_r : m.r;
  float* z = l == 0 ? t.p_z : m.z;
  if (l == nl - 1) {
    k_mg_dense<D><<<blocks_for(m.n), kBlock, 0, st>>>(m.n, m.cinv, r, z);
    return;
  }
  if (l == 0) {
    sgs_sweeps<D>(c, sweeps, st);
  } else {
    k_mg_jinit<D><<<blocks_for(m.n), kBlock, 0, st>>>(m.n, m.wdinv, r, m.z2);
    z = mg_jacobi_steps<D>(m, m.z2, sweeps - 1, st);
  }
  if (l == 0 && t.ns == 2 * D && t.nsi == D + 1)  // simplices: dim + 1 slots
    k_mg_res0<D, D + 1><<<blocks_for(m.n), kBlock, 0, st>>>(m.n, t.ns, t.p_nbr, t.p_a, t.p_diag, r, z, m.t, nullptr);
  else if (l == 0 && t.ns == 2 * D)
    k_mg_res0<D, 2 * D><<<blocks_for(m.n), kBlock, 0, st>>>(m.n, t.ns, t.p_nbr, t.p_a, t.p_diag, r, z, m.t, nullptr);
  else if (l == 0)
    k_mg_res0<D, 0><<<blocks_for(m.n), kBlock, 0, st>>>(m.n, t.ns, t.p_nbr, t.p_a, t.p_diag, r, z, m.t, t.p_big);
  else
    mg_res<D>(m.n, m.ptr, m.col, m.val, m.diag, r, z, m.t, m.g_a, st);
  DeviceTables::MgLevel& q = t.mg[l + 1];
  mg_spmv<D>(q.n, m.r_ptr, m.r_col, m.r_val, m.t, m.n, q.r, 0, m.g_r, st);
  mg_vcycle<D>(c, l + 1, sweeps, st);
  mg_spmv<D>(m.n, m.p_ptr, m.p_col, m.p_val, q.z, q.n, z, 1, m.g_p, st);
  if (l == 0) sgs_sweeps<D>(c, sweeps, st);
  else mg_jacobi_steps<D>(m, z, sweeps, st);  // ends in m.z
}

template <int D>
static hofv_status precond_impl(hofv_ctx* c, const double* r, double* z, int sweeps, hipStream_t st) {
  DeviceTables& t = c->dev;
  const int64_t nc = c->nc;
  if (sweeps < 1) return fail(c, HOFV_EINVAL, "the preconditioner needs at least one sweep");
  k_pc_in<D><<<blocks_for(nc), kBlock, 0, st>>>(nc, t.p_perm, r, t.p_r, t.p_z);
  if (c->use_mg && t.mg.size() > 1) mg_vcycle<D>(c, 0, sweeps, st);
  else sgs_sweeps<D>(c, sweeps, st);
  k_pc_out<D><<<blocks_for(nc), kBlock, 0, st>>>(nc, t.p_perm, t.p_z, z);
  HOFV_HIP(c, hipGetLastError());
  return HOFV_OK;
}

hofv_status launch_precond(hofv_ctx* c, const double* r, double* z, int sweeps, hipStream_t st) {
  return c->D == 2 ? precond_impl<2>(c, r, z, sweeps, st) : precond_impl<3>(c, r, z, sweeps, st);
}

}  // namespace hofv
