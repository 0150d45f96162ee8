// Internal declarations shared by the host setup and the HIP kernels of libhofv.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "hofv.h"
#include "mpnn.h"

namespace hofv {

// Stencil kernels run one workgroup of kBlockItems threads per item block and
// stage the block's stencil union in LDS: at most kLdsFaceCells cells for the
// face kernels, kLdsCellCells for the cell extrapolation (cell stencils of
// neighbouring cells overlap less than those of neighbouring faces).
#ifndef HOFV_BLOCK_ITEMS
#define HOFV_BLOCK_ITEMS 256
#endif
constexpr int kBlockItems = HOFV_BLOCK_ITEMS;
#ifndef HOFV_LDS_FACE
#define HOFV_LDS_FACE 1024
#endif
#ifndef HOFV_LDS_CELL
#define HOFV_LDS_CELL 1280
#endif
constexpr int kLdsFaceCells = HOFV_LDS_FACE;
constexpr int kLdsCellCells = HOFV_LDS_CELL;

// grid-wide sums: at most kRedParts block partials per value; fused
// Gram-Schmidt passes handle up to kGsChunk basis vectors
constexpr int kRedParts = 512;
constexpr int kGsChunk = 32;

// cell-face slot code for the face -> cell sum: f >= 0 owner side, ~f (< 0)
// neighbour side, kNoFace for traction/unused slots
constexpr int32_t kNoFace = INT32_MIN;

struct TimerRec {
  std::string name;
  hipEvent_t start, stop;
};

// Device-resident tables built by hofv_setup.  Layouts are "k-major, item
// minor": entry (k, item) of a per-face table lives at k * n_items + item so a
// wavefront that owns 64 consecutive items reads 64 consecutive words.
struct DeviceTables {
  int32_t S = 0;         // stencil size
  int32_t nq = 0;        // quadrature points per face
  int64_t nf = 0;        // internal + displacement faces handled by the face kernel
  int64_t nfi = 0;       // internal faces (first nfi entries)
  // item blocks of the stencil kernels (faces f_*, cells c_*): block b owns
  // items [blk_item[b], blk_item[b+1]) and the stencil union
  // ucell[blk_cell[b] .. blk_cell[b+1]); local[k][i] is the position of
  // stencil entry k of item i in its block's union
  int32_t nfb = 0, ncb = 0;
  int32_t* f_blk_item = nullptr;  // [nfb + 1]
  int32_t* f_blk_cell = nullptr;  // [nfb + 1]
  int32_t* f_ucell = nullptr;     // [f_blk_cell[nfb]]
  uint16_t* f_local = nullptr;    // [S][nf]
  int32_t* c_blk_item = nullptr;
  int32_t* c_blk_cell = nullptr;
  int32_t* c_ucell = nullptr;
  uint16_t* c_local = nullptr;    // [S][nc]
  int32_t* c_cell = nullptr;      // [n_items] cell of each extrapolation item (Morton order)
  int32_t ns = 0;                 // face slots per cell
  int32_t nsi = 0;                // face slots per extrapolation item: the most faces of a cell, or 1 (one item per cell face)
  int64_t n_items = 0;            // extrapolation items
  // faces
  double* f_coef = nullptr;      // folded: [S][D][nf]; per-point: [S][nq][D][nf]
  int32_t* f_own = nullptr;      // [nf] owner's extrapolation item
  int32_t* f_nei = nullptr;      // [nf] neighbour's extrapolation item (-1 on displacement faces)
  int32_t* f_slots = nullptr;    // [nf] owner slot | neighbour slot << 8
  double* f_area_vec = nullptr;  // folded: [D][nf] = Gamma n; per-point: [nq][D][nf] = alpha_q Gamma n
  double* f_stab = nullptr;      // [nf] alpha Kbar Gamma / |d . n|
  double* f_ghost = nullptr;     // per-point NH: [nq][D][D][nfd] ghost gradient at load 1
  // cells (extrapolation tables are indexed by extrapolation item)
  double* c_extrap = nullptr;    // [S][2D][nc] extrapolation rows (u* - u_P)
  int32_t* c_faces = nullptr;    // [2D][nc] slot codes
  double* c_src = nullptr;       // [D][nc] constant sources at load 1
  // transient
  double* ustar = nullptr;       // [nsi][D][n_items]
  double* flux = nullptr;        // [D][nf]
  double* w = nullptr;           // [nc][4 | 2] padded gather copy of u (or u + eps v)
  double* scratch = nullptr;     // reduction partials
  double* part = nullptr;        // [3][kGsChunk][kRedParts] partials of the Krylov sums
  double* eps = nullptr;         // device scalar(s)
  int32_t* flag = nullptr;       // device error flags (NH inverted element)
  // preconditioner (colour-major numbering)
  int32_t n_colours = 0;
  std::vector<int64_t> colour_start;  // n_colours + 1
  int32_t* p_perm = nullptr;     // [nc] position -> cell
  int32_t* p_nbr = nullptr;      // [2D][nc] neighbour positions (self where none)
  float* p_a = nullptr;          // [2D][nc] off-diagonal A_PN
  float* p_dinv = nullptr;       // [nc] 1 / A_PP
  // cells with more than 2 dim face slots (face-list meshes): the kernels that
  // walk a cell's slots give each of these a group of grp lanes (grp 2 dim
  // >= ns), which take its slots in turn and add up by shuffles, and one lane
  // to each other cell, for 2 dim slots; these cells come first
  int64_t n_big = 0;
  int grp = 1;
  int32_t* c_order = nullptr;    // [nc] cells with more than 2 dim faces, then the others (ascending)
  uint8_t* p_big = nullptr;      // [nc] by colour-major position: more than 2 dim faces
  std::vector<int64_t> colour_big_end;  // per colour: end of its positions with more than 2 dim faces
  float* p_r = nullptr;          // [D][nc]
  float* p_z = nullptr;          // [D][nc]
  float* p_diag = nullptr;       // [nc] A_PP (multigrid residual)
  // symmetry faces: half stencils and per-entry traction matrices (linear
  // elastic) or per-point coefficients (neo-Hookean); their fluxes live in
  // sym_flux, cell codes >= nf point there
  int64_t sym_nf = 0;
  int32_t sym_S = 0;
  int32_t* sym_st = nullptr;     // [S_half][nfs] stencil cells
  double* sym_T = nullptr;       // [S_half][D][D][nfs] traction per unit u_N,k (linear elastic)
  double* sym_C = nullptr;       // [S_half][nq][2][D][nfs] point coefficients of cell and image (NH)
  double* sym_sv = nullptr;      // [nq][D][nfs] weighted area vectors (NH)
  double* sym_n = nullptr;       // [D][nfs] unit normals (NH)
  double* sym_flux = nullptr;    // [D][nfs]
  // BDF2 inertia (App. D, one point per cell): R_P += s_P - m_P u_P
  double* dyn_rv = nullptr;      // [nc] rho * volume
  double* dyn_m = nullptr;       // [nc] 9 rho vol / (4 dt^2); null: static
  double* dyn_m_buf = nullptr;   // the buffer dyn_m points to when dynamics are on
  double* dyn_s = nullptr;       // [D][nc] the step's constant part
  double *dyn_ut = nullptr, *dyn_utm1 = nullptr, *dyn_vt = nullptr, *dyn_vtm1 = nullptr;  // [D][nc] history
  // multigrid levels 1.. of the approximate Jacobian (empty: sweeps only);
  // transfer operators of level l map level l (level 0 in colour-major
  // order) to level l + 1
  struct MgLevel {
    int64_t n = 0;
    int32_t *ptr = nullptr, *col = nullptr;  // off-diagonal CSR (levels >= 1)
    float *val = nullptr, *diag = nullptr, *wdinv = nullptr;  // wdinv = (omega / rho) / a_ii
    int32_t *p_ptr = nullptr, *p_col = nullptr, *r_ptr = nullptr, *r_col = nullptr;
    float *p_val = nullptr, *r_val = nullptr;  // P (rows: this level) and P^T
    float *r = nullptr, *z = nullptr, *t = nullptr;  // [D][n]
    float* z2 = nullptr;  // [D][n] the other iterate of the Jacobi steps (levels 1 .. L-2)
    float* cinv = nullptr;  // coarsest level: dense inverse, column-major
    int g_a = 1, g_p = 1, g_r = 1;  // lanes per CSR row of A, P, P^T
  };
  std::vector<MgLevel> mg;  // mg[0] holds level 0's transfer operators and residual
  // face-neighbour graph of the learned correction
  int32_t* g_nbr = nullptr;      // [2D][nc] neighbour or -1
  float* g_wf = nullptr;         // [2D][nc][4] omega_PN, omega_PN e_PN,d (d = 1..3)
  float* g_wb = nullptr;         // [2D][nc][4] weights of h_P in the aggregates of neighbour s
  float* g_bflag = nullptr;      // [nc] 1 if the cell has a displacement face
};

struct Krylov {
  int m = 0;
  double* V = nullptr;   // [(m+1)][n]
  double* Z = nullptr;   // [m][n]
  double* h = nullptr;   // device Hessenberg column scratch [2 (m+2)]
  double* tmp = nullptr; // [n]
  double* tmp2 = nullptr;
  double* hbuf = nullptr;  // pinned host copy
  double* Hd = nullptr;    // device Hessenberg columns of a cycle, column-major [m][m + 1]
  double* zz = nullptr;    // squared norms of learned preconditioner outputs [m]
  // Arnoldi steps replayed as HIP graphs (hofv_krylov_opts.graphs): step j is
  // captured, on cap_stream, the second time it runs
  std::vector<hipGraphExec_t> step_graph;  // [m], null until captured
  std::vector<uint8_t> step_seen;          // step j has run launched one by one
  std::vector<uintptr_t> graph_key;        // the host values the captured launches hold
  hipStream_t cap_stream = nullptr;
};

// near-exact Jacobian preconditioner (App. C): k right-preconditioned GMRES
// iterations on the stabilisation-free linear operator per application
struct Nej {
  int k = 0;               // inner iterations (0: off)
  int cap = 0;             // allocated basis size
  double* zero = nullptr;  // [max(nf, D nc)] zeros in place of the stabilisation and inertia sources
  double* V = nullptr;     // [(cap+1)][n]
  double* t = nullptr;     // [n]
  double* h = nullptr;     // device scalars in the Krylov driver's layout
  double* Hd = nullptr;    // [cap][cap + 1]
  double* zz = nullptr;    // [cap]
  double* y = nullptr;     // [cap]
  std::vector<double> hbuf, ybuf;
};

}  // namespace hofv

struct hofv_ctx {
  hofv_params prm{};
  int device = 0;
  int state = 0;  // 0 created, 1 mesh, 2 bc set, 3 body set, 4 ready
  std::string err;
  double load = 1.0;

  // mesh (host)
  int D = 0;
  int64_t nv = 0, nc = 0;
  std::vector<double> verts;
  std::vector<int64_t> cells;
  std::vector<double> cen, vol;  // [nc][D], [nc]

  // all faces: owner/neighbour/slots and ordered vertex ids
  struct Face {
    int64_t own, nei;
    int32_t sown, snei;
    int64_t v[4];
  };
  std::vector<Face> faces;           // internal faces first, then boundary faces
  // face-list (polygonal / polyhedral) meshes: each face's vertex loop,
  // outward from its owner, in the order of `faces`
  bool poly = false;
  std::vector<int64_t> fv_ptr, fv;
  int NS = 0;                        // face slots per cell (most faces of one cell)
  std::vector<int64_t> vq_ptr;       // [nc + 1] volume quadrature points of each cell
  int64_t n_internal = 0;
  std::vector<int64_t> bface;        // indices into faces of boundary faces (caller order)
  int32_t nq = 0, nqv = 0;
  // geometry of every face: centre, unit normal, area, q-points, weights
  std::vector<double> f_centre, f_normal, f_area, f_qp, f_qw;
  // boundary views handed to the caller
  std::vector<double> b_centre, b_normal, b_qp;
  std::vector<double> vq_pts, vq_w;  // [n_points][D], [n_points], cell P's from vq_ptr[P]

  // boundary data from the caller
  std::vector<int32_t> btype;
  std::vector<double> ubq, ubc, tq, fb;

  hofv_setup_report report{};
  // approximate Jacobian diagonal by sweep position (static) and the position's
  // cell, for re-deriving the sweeps' diagonal when an inertia term is added
  std::vector<double> pc_diag;
  std::vector<int64_t> pc_perm;
  double dyn_rho = 0.0, dyn_dt = 0.0;
  bool dyn_ready = false;  // history set by hofv_dyn_reset
  hofv::DeviceTables dev;
  hofv::Krylov kry;
  hofv::Nej nej;
  hofv::NnWork nnw;
  hofv_nn* nn = nullptr;  // attached learned correction (not owned)
  std::vector<void*> allocations;
  size_t device_bytes = 0;

  // host copies of the setup tables (host_only contexts)
  struct HostTable {
    std::vector<char> bytes;
    int32_t elem = 0;
  };
  std::map<std::string, HostTable> host_tables;

  // timing
  bool timing = false;
  std::string timing_only;  // non-empty: only launches of this kernel are timed
  bool use_mg = false;  // apply the approximate Jacobian by the V-cycle
  std::vector<hofv::TimerRec> timers;
  std::vector<hipEvent_t> ev_pool;  // events of the timers, reused
  size_t ev_used = 0;
  std::map<std::string, double> kernel_bytes;
};

namespace hofv {

// error helpers
hofv_status fail(hofv_ctx* c, hofv_status s, const std::string& msg);
#define HOFV_HIP(ctx, call)                                                               \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return ::hofv::fail(ctx, HOFV_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <class T>
hofv_status dev_alloc(hofv_ctx* c, T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, count * sizeof(T));
  if (e != hipSuccess) return fail(c, HOFV_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  c->allocations.push_back(q);
  c->device_bytes += count * sizeof(T);
  *p = static_cast<T*>(q);
  return HOFV_OK;
}

template <class T>
hofv_status upload(hofv_ctx* c, T** p, const std::vector<T>& host) {
  hofv_status s = dev_alloc(c, p, host.size());
  if (s) return s;
  if (!host.empty()) HOFV_HIP(c, hipMemcpy(*p, host.data(), host.size() * sizeof(T), hipMemcpyHostToDevice));
  return HOFV_OK;
}

// host setup stages (setup_*.cpp)
hofv_status build_topology(hofv_ctx* c);
hofv_status build_topology_poly(hofv_ctx* c, int64_t n_faces, const int64_t* face_ptr, const int64_t* face_verts,
                                const int64_t* face_cells);
hofv_status build_geometry(hofv_ctx* c);
hofv_status build_tables(hofv_ctx* c);

// item blocks for LDS-staged stencil gathers (setup_blocks.cpp)
// Per-stencil-entry tables are stored block by block: block b (items
// [i0, i0 + nb)) owns the contiguous segment [i0 S R, (i0 + nb) S R) of a
// table with R rows per entry, holding row r of entry k of its items at
// (k R + r) nb + (i - i0), so one workgroup streams one contiguous segment.
struct StencilBlocks {
  std::vector<int32_t> item, cell, cells;
  std::vector<int32_t> block_of;  // [n]
  std::vector<uint16_t> local;    // positions in the block's union, R = 1
  int32_t max_cells = 0;
  size_t at(int64_t i, int k, int r, int R, int S) const {
    const int64_t b = block_of[i], i0 = item[b], nb = item[b + 1] - i0;
    return (size_t)i0 * S * R + ((size_t)k * R + r) * nb + (size_t)(i - i0);
  }
  // the same table in the plain k-major layout [(k R + r) n + i]
  template <class T>
  std::vector<T> unblocked(const std::vector<T>& v, int R, int S) const {
    const int64_t n = (int64_t)block_of.size();
    std::vector<T> out(v.size());
    for (int64_t i = 0; i < n; ++i)
      for (int k = 0; k < S; ++k)
        for (int r = 0; r < R; ++r) out[((size_t)k * R + r) * n + i] = v[at(i, k, r, R, S)];
    return out;
  }
};
// indices of pts[n][D] sorted by Morton code over the bounding box
std::vector<int64_t> morton_order(const double* pts, int D, int64_t n);
// st: item-major stencils [n][S] of items already in block order
StencilBlocks make_blocks(const int32_t* st, int64_t n, int S, int64_t nc, int max_items, int max_cells);

// stencils: cells nearest to each point, ties by (rint(d2/quantum), id)
void nearest_cells(const std::vector<double>& cen, int D, int64_t nc, const double* pts,
                   int64_t npts, int S, double quantum, int32_t* out);

// Least-squares fit at xt over the stencil X[S][D] (plus a co-located ghost
// node when ghost_w > 0).  For each target writes the stencil coefficients
// out[r][0..m), m = S (+1 ghost), of one linear functional of the fit:
//  kind kTargetGradient: targets[r] is an axis i, functional = d u / d x_i;
//  kind kTargetExtrap:   targets[r*D..] is a vector d, functional =
//                        u~(x + d) - u~(x) of the fitted Taylor polynomial.
// Returns false when rank deficient (min|R_ii| <= 1e-14 max|R_ii|).
enum { kTargetGradient = 0, kTargetExtrap = 1 };
bool ls_functionals(int D, int p, double kshape, const double* xt, const double* X, int S,
                    double ghost_w, int kind, int n_targets, const double* targets, double* out,
                    double* cond, double* h_out);
int n_basis(int D, int p);
void basis_exponents(int D, int p, int (*e)[3]);

// smoothed-aggregation hierarchy of the approximate Jacobian (setup_amg.cpp):
// a0 is level 0 in CSR (sorted columns, diagonal included) in cell order,
// perm the colour-major order of level 0's vectors; uploads c->dev.mg
hofv_status build_multigrid(hofv_ctx* c, const std::vector<int64_t>& ptr, const std::vector<int32_t>& col,
                            const std::vector<double>& val, const std::vector<int32_t>& pos, int max_levels);

// kernel launchers (kernels.hip)
hofv_status launch_residual(hofv_ctx* c, const double* u, double* R, const double* Ru,
                            const double* eps_dev, hipStream_t st);
hofv_status launch_jvp_pack(hofv_ctx* c, const double* u, const double* v, double eps_host, hipStream_t st);
// J.v whose eps reduction lives in a static device array (no allocation)
hofv_status noalloc_init(hofv_ctx* c);
hofv_status jvp_noalloc_impl(hofv_ctx* c, const double* u, const double* Ru, const double* v, double* Jv,
                             double eps_host, hipStream_t st);
hofv_status launch_precond(hofv_ctx* c, const double* r, double* z, int sweeps, hipStream_t st);
hofv_status launch_nej(hofv_ctx* c, const double* v, double* out, hipStream_t st);
// krylov.hip: the near-exact Jacobian preconditioner
hofv_status nej_zero(hofv_ctx* c);
hofv_status nej_set(hofv_ctx* c, int k);
hofv_status nej_solve(hofv_ctx* c, const double* r, double* z, int sweeps, hipStream_t st);
// dynamics.hip
hofv_status dyn_set(hofv_ctx* c, double rho, double dt);
hofv_status dyn_reset(hofv_ctx* c, const double* u_t, const double* u_tm1, const double* v_t, const double* v_tm1,
                      hipStream_t st);
hofv_status dyn_step(hofv_ctx* c, double* u, const hofv_newton_opts* o, hofv_newton_stats* stats, hipStream_t st);

// timing helpers
void timer_begin(hofv_ctx* c, const char* name, hipStream_t st, hipEvent_t* ev);
void timer_end(hofv_ctx* c, const char* name, hipStream_t st, hipEvent_t ev);

}  // namespace hofv
