/*
 * hofv.h - C ABI of the MI355X (gfx950) library for the Jacobian-free
 * Newton-Krylov solution of high-order cell-centred finite-volume solid
 * mechanics (Batistic, Castrillo, Cardiff, arXiv 2601.18417).
 *
 * Problem statement (paper Sec. 4.1): find the cell-centroid displacements u
 * with R(u) = 0, where R is the high-order finite-volume residual of Secs. 3.2-3.5
 * (least-squares face-point gradients, linear-elastic or neo-Hookean
 * tractions, alpha-stabilisation, face-to-cell sum, body force and boundary
 * loads), by Newton's method with the finite-difference Jacobian-vector
 * product J v ~ (R(u + eps v) - R(u)) / eps inside a Krylov solver that is
 * preconditioned by the compact-stencil approximate Jacobian.
 *
 * Conventions for every function:
 *  - The return value is a hofv_status; 0 is success.  Nothing throws or
 *    aborts across this interface; hofv_last_error() describes the last
 *    failure on a context.
 *  - Host arrays passed in are copied before the call returns; the caller
 *    keeps ownership.  Host pointers handed out by the library stay valid
 *    until hofv_destroy().
 *  - "Device" pointers are HIP device allocations (e.g. from PyTorch tensors)
 *    on the device that was current at hofv_create().  Field vectors are FP64,
 *    component-major: v[c * n_cells + P], c < dim, in the caller's cell
 *    numbering.  They must stay alive until the work queued on `stream`
 *    completes.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Hot
 *    calls only queue work on it, except where a call says it synchronises.
 *  - Call order: create -> set_mesh -> (boundary_faces, volume_qpoints) ->
 *    set_bc -> set_body_force -> setup -> hot calls.  Out of order: HOFV_ESTATE.
 *  - A context is used by one host thread at a time.
 */
#ifndef HOFV_H
#define HOFV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hofv_ctx hofv_ctx;

typedef enum {
  HOFV_OK = 0,
  HOFV_EINVAL = -1,     /* bad argument */
  HOFV_ENOMEM = -2,     /* host or device allocation failed */
  HOFV_EHIP = -3,       /* a HIP runtime call failed */
  HOFV_ESINGULAR = -4,  /* a least-squares stencil is rank deficient */
  HOFV_ENOCONV = -5,    /* an iterative solve did not reach its tolerance */
  HOFV_ENAN = -6,       /* NaN/Inf met in a solve */
  HOFV_EINVERTED = -7,  /* neo-Hookean: det F <= 0 at a quadrature point */
  HOFV_ESTATE = -8      /* call made out of order */
} hofv_status;

enum { HOFV_LINEAR_ELASTIC = 0, HOFV_NEO_HOOKEAN = 1 };
/* Symmetry planes (Sec. 3.5): the face's stencil is the ceil(|S|/2) nearest cells and
 * their mirror images, the images carrying R_b u (R_b = I - 2 n n); both laws; no
 * stabilisation term on such faces; u_b and traction values given for them are
 * ignored. */
enum { HOFV_BC_DISPLACEMENT = 0, HOFV_BC_TRACTION = 1, HOFV_BC_SYMMETRY = 2 };

/* Discretisation parameters (paper Secs. 3.4-3.5). */
typedef struct {
  int32_t dim;            /* 2 (plane strain: quads, triangles) or 3 (hexahedra, tetrahedra) */
  int32_t order_p;        /* reconstruction order p = 1, 2, 3 (2nd/3rd/4th order) */
  int32_t n_plus;         /* surplus stencil nodes n+, |S| = N_t + n+ (Sec. 3.5.2) */
  int32_t n_gauss;        /* Gauss-Legendre points per face direction */
  int32_t material;       /* HOFV_LINEAR_ELASTIC or HOFV_NEO_HOOKEAN (3D only) */
  int32_t fold_quadrature;/* 1: linear elasticity sums the face-point coefficients
                             over the quadrature points at setup (same R, fewer
                             bytes); 0: per-point gradients.  Ignored for NH. */
  double mu, lambda;      /* Lame parameters; Kbar = 2 mu + lambda (Sec. 3.4) */
  double alpha;           /* stabilisation scale, eq. alpha (paper default 0.1) */
  double k_weight;        /* shape k of eq. weightFunc (paper: 6) */
  double ghost_weight;    /* weight of displacement ghost nodes (paper: 1) */
  double stencil_quantum; /* squared distances closer than this tie; ties are
                             broken by lower caller cell id (> 0 required) */
  int32_t host_only;      /* 1: no device is used; hofv_setup builds the tables on
                             the host and keeps them for hofv_host_table (for
                             inspection on machines without a GPU); hot calls
                             then fail with HOFV_ESTATE */
  int32_t precond_levels; /* application of the compact approximate Jacobian:
                             1 (or 0): n_sweeps symmetric multicolour Gauss-Seidel
                             sweeps; >= 2: a smoothed-aggregation multigrid
                             V-cycle of at most that many levels whose finest
                             smoother is those sweeps (n_sweeps damped Jacobi
                             steps on coarser levels, exact coarsest solve) */
  int32_t face_rule;      /* quadrature of hexahedral (quadrilateral) faces,
                             Sec. 3.1: 0: n_gauss x n_gauss Gauss-Legendre points
                             of the bilinear face; 1: fan triangulation from the
                             face's lowest-numbered vertex into two triangles with the
                             simplex rule on each (2 n_gauss^2 points), each
                             triangle's weights scaled by its area over the sum of
                             the two areas, and the face area Gamma_f that sum (on
                             a warped face larger than the vector area's length).
                             The normal is the vector area's direction either way;
                             rule 0 takes Gamma_f as that vector's length.  Either
                             rule serves both laws and both quadrature forms;
                             triangle faces and 2D edges ignore it. */
  int32_t stencil_grow;   /* 0: a stencil that fails the pivot test of its QR
                             (min |R_ii| <= 1e-14 max |R_ii|) is an error
                             (HOFV_ESINGULAR).  g > 0: such a face or cell
                             stencil is replaced by the |S| + g, |S| + 2g, ...
                             nearest cells (same tie rule) until it passes, up
                             to 255 cells and the mesh's cell count (the remedy of
                             Sec. 5's ill-conditioning study, a larger n+,
                             applied where the test fails); the tables then
                             take the largest size and shorter stencils are
                             padded with zero coefficients.  Symmetry-face
                             stencils are not grown. */
} hofv_params;

/* Creates a context on the current HIP device.  *out is NULL on failure. */
hofv_status hofv_create(const hofv_params* params, hofv_ctx** out);

/* Frees every host and device buffer of ctx.  NULL is accepted. */
hofv_status hofv_destroy(hofv_ctx* ctx);

/* Last error message of ctx (or of the last failed hofv_create when ctx is
 * NULL); valid until the next call on ctx. */
const char* hofv_last_error(const hofv_ctx* ctx);

/* Mesh (Sec. 3.1): verts [n_verts][dim] FP64; cell_verts [n_cells][4 | 8]
 * int64 in VTK quad/hexahedron order.  Faces are matched by vertex sets. */
hofv_status hofv_set_mesh(hofv_ctx* ctx, int64_t n_verts, const double* verts,
                          int64_t n_cells, const int64_t* cell_verts);

/* Simplex mesh (Sec. 3.1; the paper's triangular and tetrahedral cases of
 * Sec. 5): cell_verts [n_cells][dim + 1] int64, triangles counter-clockwise,
 * tetrahedra with (x1 - x0) x (x2 - x0) . (x3 - x0) > 0 (HOFV_EINVAL from the
 * geometry stage otherwise).  Faces (edges in 2D, flat triangles in 3D) are
 * matched by vertex sets; a triangle face has n_gauss^2 quadrature points, an
 * edge n_gauss, a cell (order_p + 2)^dim, from conical-product
 * Gauss-Jacobi/Gauss-Legendre rules exact for total degree 2 n - 1 with n
 * points per direction.  Everything after the mesh (stencils, tables,
 * kernels, solvers) is the same as for quads and hexahedra.  Called instead
 * of hofv_set_mesh, once. */
hofv_status hofv_set_mesh_simplices(hofv_ctx* ctx, int64_t n_verts, const double* verts, int64_t n_cells,
                                    const int64_t* cell_verts);

/* Polygonal (2D) or polyhedral (3D) mesh given by its faces (Sec. 3.1: the
 * paper's arbitrary convex polyhedra): face f has the vertex loop
 * face_verts[face_ptr[f] .. face_ptr[f + 1]) (2 vertices in 2D, at least 3 in
 * 3D, face_ptr[0] = 0) whose right-hand normal points out of cell
 * face_cells[2 f] and into face_cells[2 f + 1] (-1: boundary face).  A 3D face
 * is cut into triangles by a fan from its lowest-numbered vertex; its area is
 * the sum of the triangle areas, its normal the direction of its vector area
 * 1/2 sum x_k x x_{k+1}, and its quadrature points are n_gauss^2 per triangle
 * (faces with fewer triangles than the mesh's largest are padded with
 * zero-weight points at their centre, so n_q = (most vertices - 2) n_gauss^2;
 * face_rule is ignored).  A cell is cut into triangles (2D) or tetrahedra
 * (3D) joining the mean of its distinct vertices to its faces' edges or fan
 * triangles: its volume and centroid are theirs summed, and its body-force
 * points are (order_p + 2)^dim per simplex (see hofv_volume_qpoints_csr).
 * Cells with more than 2 dim faces give each face its own extrapolation item.
 * HOFV_EINVAL for malformed input (bad indices, a face cell equal on both
 * sides, a cell with fewer than dim + 1 faces or more than 255, a cell whose
 * faces do not close, i.e. whose outward vector areas do not sum to zero to
 * 1e-9 of their sizes: a missing or repeated face or a loop given the wrong
 * way round; non-positive volume).  Called instead of hofv_set_mesh, once. */
hofv_status hofv_set_mesh_polyhedra(hofv_ctx* ctx, int64_t n_verts, const double* verts, int64_t n_cells,
                                    int64_t n_faces, const int64_t* face_ptr, const int64_t* face_verts,
                                    const int64_t* face_cells);

/* Boundary faces in the library's order, so that the caller can evaluate its
 * boundary conditions there: face centres x_b [n][dim], unit outward normals
 * [n][dim], quadrature points x_{b,q} [n][n_q][dim] with n_q = n_gauss^(dim-1).
 * Pointers are owned by ctx. */
hofv_status hofv_boundary_faces(hofv_ctx* ctx, int64_t* n_bfaces, int32_t* n_q,
                                const double** centres, const double** normals,
                                const double** qpoints);

/* Cell centroids x_P [n_cells][dim] (caller numbering), the points where the
 * unknowns live (Sec. 3, point-valued finite volume).  Owned by ctx. */
hofv_status hofv_cell_centroids(hofv_ctx* ctx, const double** centroids);

/* Volume quadrature points of the body-force integral (eq. bodyTerm),
 * [n_cells][n_qv][dim], n_qv = (p+2)^dim Gauss-Legendre points of the cell map.
 * HOFV_EINVAL when cells have different point counts (polyhedral meshes). */
hofv_status hofv_volume_qpoints(hofv_ctx* ctx, int32_t* n_qv, const double** points);

/* The same points for any mesh: cell P's are points[cell_ptr[P] ..
 * cell_ptr[P + 1]) ([n_points][dim]); cell_ptr has n_cells + 1 entries.
 * Pointers are owned by ctx. */
hofv_status hofv_volume_qpoints_csr(hofv_ctx* ctx, int64_t* n_points, const int64_t** cell_ptr,
                                    const double** points);

/* Boundary conditions (Sec. 3.5.3), per boundary face in hofv_boundary_faces
 * order: type[n] (HOFV_BC_*); u_b at the quadrature points [n][n_q][dim] and at
 * the face centre [n][dim] (read on displacement faces); nominal traction at
 * the quadrature points [n][n_q][dim] (read on traction faces).  NULL arrays
 * mean zero. */
hofv_status hofv_set_bc(hofv_ctx* ctx, const int32_t* type, const double* u_b_q,
                        const double* u_b_centre, const double* traction_q);

/* Body force f_b at the volume quadrature points, in their order ([n_points][dim]
 * of hofv_volume_qpoints_csr, i.e. [n_cells][n_qv][dim] when the counts are
 * equal); NULL = 0. */
hofv_status hofv_set_body_force(hofv_ctx* ctx, const double* values);

typedef struct {
  int32_t stencil_size;    /* |S| */
  int32_t n_colours;       /* colours of the preconditioner sweeps */
  int64_t n_internal_faces, n_disp_faces, n_trac_faces;
  double max_cond;         /* largest max|R_ii| / min|R_ii| of the LS QRs */
  double device_bytes;     /* device memory held by the context */
  double residual_bytes;   /* algorithmic HBM bytes of one residual */
  double setup_seconds;
  int64_t n_grown_stencils;  /* face and cell stencils enlarged by stencil_grow */
} hofv_setup_report;

/* Builds stencils (Sec. 3.5.2), least-squares coefficients (Sec. 3.5.1,
 * Householder QR), sources, the compact preconditioner and its colouring on
 * the host, then copies everything to the device.  Synchronises.  Fails with
 * HOFV_ESINGULAR when a stencil is rank deficient (min|R_ii| <= 1e-14 max). */
hofv_status hofv_setup(hofv_ctx* ctx, hofv_setup_report* report);

/* Load factor s for load increments: u_b, tractions and f_b are scaled by s. */
hofv_status hofv_set_load_scale(hofv_ctx* ctx, double s);

/* Selects how hofv_precond_apply (and the solvers) apply the approximate
 * Jacobian: enable != 0 uses the multigrid V-cycle built at setup
 * (precond_levels >= 2; HOFV_EINVAL if none was built), 0 the sweeps alone.
 * The default follows precond_levels. */
hofv_status hofv_set_multigrid(hofv_ctx* ctx, int32_t enable);

/* Near-exact Jacobian (App. C, linear elastic law only): the derivative of the
 * discrete momentum equations without the alpha-stabilisation term of
 * Sec. 3.4, with the full face stencils.  The residual is affine in u, so
 * d_out = A d_v is evaluated matrix-free as the residual of d_v with the
 * stabilisation, every load (u_b, tractions, f_b) and the inertia source set
 * to zero; with dynamics on, A includes the -m_P u_P mass term of the step.
 * Device arrays [dim][n_cells], no aliasing; ordered on `stream`, does not
 * synchronise.  HOFV_EINVAL for the neo-Hookean law or bad pointers. */
hofv_status hofv_nej_apply(hofv_ctx* ctx, const double* d_v, double* d_out, void* stream);

/* Uses the near-exact Jacobian as the preconditioner of hofv_precond_apply and
 * the solvers: z ~ A^{-1} r by inner_iters (1..64) iterations of GMRES from
 * zero on A, right-preconditioned by the approximate Jacobian (the sweeps or
 * the V-cycle, as selected), so each application costs inner_iters residual
 * evaluations and inner_iters + 1 approximate-Jacobian applications.  The
 * result depends on r nonlinearly, so the outer solve must be the flexible
 * right-preconditioned FGMRES (side 0) without the learned correction
 * (HOFV_EINVAL otherwise).  inner_iters = 0 switches it off.  Allocates the
 * inner basis ((inner_iters + 1) [dim][n_cells] vectors) on first use or
 * growth; HOFV_EINVAL for the neo-Hookean law or inner_iters outside 0..64. */
hofv_status hofv_set_nej(hofv_ctx* ctx, int32_t inner_iters);

/* R = R(u) (eq. divStressDiscret with eqs. faceQuadGrad, alpha, alphaJump,
 * bodyTerm).  d_u, d_R: device [dim][n_cells]; they must not alias. */
hofv_status hofv_residual(hofv_ctx* ctx, const double* d_u, double* d_R, void* stream);

/* Jv = (R(u + eps v) - R(u)) / eps (Sec. 4.1).  d_Ru must hold R(u).
 * eps <= 0 selects eps = sqrt((1 + ||u||_2) eps_mach) / ||v||_2 computed on the
 * device (Jv = 0 when v = 0).  d_Jv must not alias the inputs. */
hofv_status hofv_jvp(hofv_ctx* ctx, const double* d_u, const double* d_Ru, const double* d_v,
                     double* d_Jv, double eps, void* stream);

/* hofv_jvp for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same product and arguments, with the block partial sums of the device eps
 * (eps <= 0) and eps itself kept in a library-wide static device array of
 * 2048 doubles (16 KiB) per GPU instead of the context's buffers; one call
 * needs 2 min(512, ceil(dim n_cells / 256)) + 1 of them, at most 1025, so every
 * mesh fits (HOFV_EINVAL otherwise).  The call makes no hipMalloc/hipFree and
 * records no timing events.  All calls on one GPU share the array and
 * overwrite it (nothing in it has to start at zero): calls that overlap on one
 * GPU, from concurrent streams or threads, race.  Needs hofv_setup, which
 * looks up the array's address on the context's device (HOFV_ESTATE before). */
hofv_status hofv_jvp_noalloc(hofv_ctx* ctx, const double* d_u, const double* d_Ru, const double* d_v,
                             double* d_Jv, double eps, void* stream);

/* z ~ P^{-1} r with P the compact approximate Jacobian (Sec. 4.1): n_sweeps
 * symmetric multicolour Gauss-Seidel sweeps in FP32 from z = 0, or the
 * V-cycle (hofv_set_multigrid).  learned != 0 adds the network correction
 * (hofv_nn_*) when one is loaded.  With hofv_set_nej on, z ~ A^{-1} r for the
 * near-exact Jacobian A instead (learned != 0 is then HOFV_EINVAL).  d_r, d_z
 * must not alias. */
hofv_status hofv_precond_apply(hofv_ctx* ctx, const double* d_r, double* d_z, int32_t n_sweeps,
                               int32_t learned, void* stream);

typedef struct {
  int32_t restart;       /* m of FGMRES(m), default 30 (<= 0), at most 2048
                            (HOFV_EINVAL above); the basis takes (2m + 1) n doubles */
  int32_t max_iters;     /* total Krylov iterations */
  double rtol;           /* stop at ||rhs - J x|| <= rtol ||rhs|| */
  int32_t n_sweeps;      /* preconditioner sweeps per application */
  int32_t learned;       /* use the learned correction */
  int32_t side;          /* 0: right-preconditioned flexible GMRES (default);
                            1: left-preconditioned GMRES on M J x = M rhs as eq. jfnk
                            prints it: the stopping test and rel_residual are then
                            those of the preconditioned residual M (rhs - J x)
                            against M rhs; not with learned (HOFV_EINVAL) */
  int32_t gs_passes;     /* classical Gram-Schmidt passes per Arnoldi step: 0 or 2:
                            twice (default); 1: once, the orthogonalisation PETSc's
                            GMRES uses unless told otherwise (Sec. 4.1 names PETSc
                            and no other); others HOFV_EINVAL */
  int32_t graphs;        /* 0: every launch of an Arnoldi step made by the host
                            (default); 1: each step j of a right-preconditioned,
                            unlearned solve is captured as a HIP graph the
                            second time it runs and replayed from then on, on a
                            stream of the context's own for the capture and the
                            caller's for the replays; the captured steps are
                            kept across solves while the state and Ru pointers,
                            sweeps, passes, restart, multigrid and dynamics
                            settings and load scale stay the same, and rebuilt
                            otherwise.  Results are bit for bit those of 0.  For
                            small meshes, where launching rather than the GPU
                            sets the pace (a few per cent there; nothing on
                            large ones).  Ignored with learned, side 1, the
                            near-exact Jacobian or kernel timing on; others
                            HOFV_EINVAL */
} hofv_krylov_opts;

typedef struct {
  int32_t iters;
  int32_t converged;
  double rel_residual;   /* final ||rhs - J x|| / ||rhs|| (recomputed) */
  double seconds;
  int32_t fallbacks;     /* iterations redone with the plain preconditioner
                            because the learned one produced NaN/Inf */
  int32_t stalled;       /* 1: ended because a full cycle reduced the recomputed
                            residual by less than 1 % */
} hofv_krylov_stats;

/* Solves J(u) x = rhs by right-preconditioned flexible GMRES(m) with J v from
 * hofv_jvp and z = M(v) from hofv_precond_apply; x holds the initial guess on
 * entry.  Iterations are queued eight at a time and the host reads their
 * Hessenberg columns at once (Givens rotations on the host); columns past the
 * converged iteration are discarded, so up to seven extra iterations of work
 * may be spent at the end of a solve.
 * With opts->learned, an iteration whose Hessenberg column is not finite is
 * redone with the plain preconditioner, which is then kept for the rest of
 * the solve; so is a restart cycle that reduced the residual by less than a
 * factor 0.75 (both counted in stats->fallbacks).  A plain cycle that reduced
 * the residual, recomputed at the restart, by less than 1 % ends the solve
 * (stats->stalled, converged 0, x kept): past the residual that the precision
 * of the finite-difference product allows, the least-squares estimate goes on
 * falling while the true residual stays. */
hofv_status hofv_fgmres_solve(hofv_ctx* ctx, const double* d_u, const double* d_Ru,
                              const double* d_rhs, double* d_x, const hofv_krylov_opts* opts,
                              hofv_krylov_stats* stats, void* stream);

typedef struct {
  double tol;            /* ||R|| <= tol ||R_0|| per load increment */
  double eta;            /* Krylov rtol per Newton step */
  int32_t max_newton;    /* per increment */
  int32_t n_increments;  /* load factors i / n, i = 1..n; <= 0: one solve at the
                            factor set by hofv_set_load_scale */
  int32_t max_line_search; /* backtracking halvings (0: 10); < 0: full steps
                              (see hofv_newton_solve) */
  hofv_krylov_opts krylov; /* krylov.rtol is ignored: eta and forcing set it */
  int32_t forcing;       /* 0: Krylov rtol = eta on every step; 1: Eisenstat-Walker
                            choice 2, eta_k = 0.9 (||R_k|| / ||R_k-1||)^2, raised to
                            0.9 eta_k-1^2 when that exceeds 0.1, at most eta (which
                            is also the first step's), and at least
                            0.5 tol ||R_0|| / ||R_k|| */
  int32_t predictor;     /* 0: each increment starts from the last converged state;
                            1: from u_i + (u_i - u_{i-1}) (secant in the load
                            factor), unless that state has an inverted cell or a
                            non-finite residual; ||R_0|| is still that of u_i at
                            the new load */
} hofv_newton_opts;

typedef struct {
  int32_t newton_iters;
  int32_t krylov_iters;
  int32_t converged;
  double rel_residual;   /* of the last increment */
  double seconds;
  int32_t fallbacks;     /* FGMRES iterations redone with the plain preconditioner,
                            plus linear solves repeated with it after the learned
                            one missed the Krylov tolerance */
} hofv_newton_stats;

/* Newton with backtracking line search on ||R||_2 (accept the first
 * ||R(u + lam du)|| <= (1 - 1e-4 lam) ||R(u)||, lam = 1, 1/2, ..., else the
 * last trial), J du = -R by hofv_fgmres_solve, for each load increment.  With
 * opts->max_line_search < 0 every step is a full one (lam = 1) unless its
 * trial state has an inverted cell (J <= 0 at a face point) or a non-finite
 * residual, in which case lam is halved up to 10 times; a load concentrated on
 * a few cells (a tip traction) makes ||R|| a poor merit function, since the
 * first full step of a bending problem spreads a larger geometric residual
 * over the whole body before the next steps remove it.  With krylov.learned, a linear
 * solve that misses its tolerance is repeated with the plain preconditioner.
 * d_u: initial guess in, solution out.  Synchronises. */
hofv_status hofv_newton_solve(hofv_ctx* ctx, double* d_u, const hofv_newton_opts* opts,
                              hofv_newton_stats* stats, void* stream);

/* ---- dynamics: BDF2 inertia (App. D, eq. inertiaTerm) -------------------------
 * One integration point per cell (the centroid, u_P itself).  Velocity and
 * acceleration are both BDF2 differences, so the inertia rho a Omega_P is
 * m_P u_P - s_P with m_P = 9 rho Omega_P / (4 dt^2) and s_P built from u and v
 * at the two previous time levels; R_P gains s_P - m_P u_P and the compact
 * approximate Jacobian gains -m_P on its diagonal (its sweeps include it).
 *
 * hofv_set_dynamics: rho > 0 and dt > 0 switch the term on (rho <= 0 switches it
 * off and restores the static preconditioner).  The multigrid hierarchy is
 * built for the static operator: it is switched off here, and
 * hofv_set_multigrid(1) returns HOFV_EINVAL while dynamics are on.  Allocates
 * 6 D n_c + 2 n_c doubles on the first call.  Synchronises.
 * hofv_dyn_reset: the history u^t, u^{t-1}, v^t, v^{t-1} (device [D][n_c], copied;
 * a start from rest passes u0, u0, 0, 0).  HOFV_ESTATE without dynamics.
 * hofv_dyn_step: one time step, a Newton solve (opts as hofv_newton_solve, with
 * n_increments and predictor ignored) at the load factor set by
 * hofv_set_load_scale, from the guess in d_u; on success the history advances
 * to the result (v by BDF2).  On any error the history stays where it was.
 * All three synchronise. */
hofv_status hofv_set_dynamics(hofv_ctx* ctx, double rho, double dt);
hofv_status hofv_dyn_reset(hofv_ctx* ctx, const double* d_u_t, const double* d_u_tm1, const double* d_v_t,
                           const double* d_v_tm1, void* stream);
hofv_status hofv_dyn_step(hofv_ctx* ctx, double* d_u, const hofv_newton_opts* opts, hofv_newton_stats* stats,
                          void* stream);

/* ---- learned correction of the preconditioner -------------------------------
 * A message-passing network over face neighbours (not part of the paper):
 * z = z_AJ + s_z g(x), x_P = [r_P/s_r, z_AJ,P/s_z, displacement-face flag, 1],
 * s = RMS values, encoder 8->64, 4 layers h += relu([h, A0..A3] W_l + b_l)
 * with A0 = sum_N omega_PN h_N, Ad = sum_N omega_PN e_PN,d h_N (omega from the
 * compact Jacobian's face couplings, e the unit centroid-to-centroid vector),
 * decoder 64->3.  BF16 weights/activations with FP32 accumulation on MFMA;
 * FP32 master weights and Adam state.  A model lives on the device that was
 * current at hofv_nn_create and may be attached to any context there. */
typedef struct hofv_nn hofv_nn;

/* Number of FP32 parameters; flat layout We[8][64], be[64], then per layer
 * W[320][64], b[64], then Wd[64][3], bd[3]. */
int64_t hofv_nn_param_count(void);

/* New model: He-initialised hidden layers, zero decoder (so that the
 * corrected preconditioner starts equal to the plain one), zero Adam state. */
hofv_status hofv_nn_create(uint64_t seed, hofv_nn** out);
hofv_status hofv_nn_destroy(hofv_nn* nn);

/* Copy the FP32 parameters from/to host memory (n = hofv_nn_param_count()).
 * set_params also resets the Adam state.  Synchronises. */
hofv_status hofv_nn_set_params(hofv_nn* nn, const float* host, int64_t n);
hofv_status hofv_nn_get_params(hofv_nn* nn, float* host, int64_t n);

/* Attach (nn != NULL) or detach the model used by hofv_precond_apply with
 * learned != 0 and by the solvers' learned option.  The caller keeps
 * ownership and must keep it alive while attached. */
hofv_status hofv_nn_attach(hofv_ctx* ctx, hofv_nn* nn);

/* One optimisation step on n_pairs (residual, correction) pairs of ctx's mesh:
 * d_r, d_e hold n_pairs device vectors [n_pairs][dim][n_cells] FP64.  For each
 * pair z_AJ = plain preconditioner(r) with n_sweeps sweeps, loss
 * ||z - e||^2 / ||e||^2; gradients are averaged over the pairs and Adam
 * (beta 0.9, 0.999, eps 1e-8, step lr) updates the model.  *loss receives the
 * mean loss before the step.  Synchronises. */
hofv_status hofv_nn_train_step(hofv_ctx* ctx, hofv_nn* nn, const double* d_r, const double* d_e,
                               int32_t n_pairs, int32_t n_sweeps, double lr, double* loss, void* stream);

/* Loss and gradient of one pair with an explicit z_AJ (device [dim][n_cells]);
 * host_grad receives hofv_nn_param_count() floats.  Does not update the model.
 * Synchronises. */
hofv_status hofv_nn_gradient(hofv_ctx* ctx, hofv_nn* nn, const double* d_r, const double* d_zaj,
                             const double* d_e, float* host_grad, double* loss, void* stream);

/* Corrected preconditioner output for an explicit z_AJ: d_z = z_AJ + s_z g. */
hofv_status hofv_nn_forward(hofv_ctx* ctx, hofv_nn* nn, const double* d_r, const double* d_zaj, double* d_z,
                            void* stream);

/* Writes the FP32 parameters to a file: the 8 bytes "HOFVNN01", the int64
 * parameter count, then that many float32 values (host byte order).
 * Synchronises.  HOFV_EINVAL if the file cannot be written. */
hofv_status hofv_nn_save(hofv_nn* nn, const char* path);

/* Reads a file written by hofv_nn_save into the model (its count must equal
 * hofv_nn_param_count(); HOFV_EINVAL otherwise) and resets the Adam state. */
hofv_status hofv_nn_load(hofv_nn* nn, const char* path);

/* ---- training pairs and the training loop --------------------------------
 * The network is trained on pairs (r, e) with J(u) e = r that the solver
 * produces itself (the learned correction is not part of the paper).  A pair
 * set holds up to `capacity` pairs on one context's mesh: device vectors
 * [capacity][dim][n_cells] FP64 for r and for e, owned by the set, which must
 * be destroyed before its context. */
typedef struct hofv_pairset hofv_pairset;
hofv_status hofv_pairset_create(hofv_ctx* ctx, int32_t capacity, hofv_pairset** out);
hofv_status hofv_pairset_destroy(hofv_pairset* set);
/* Pairs held and device pointers to r and e ([n_pairs][dim][n_cells], valid
 * until the set is destroyed). */
hofv_status hofv_pairset_data(const hofv_pairset* set, int32_t* n_pairs, const double** d_r, const double** d_e);
/* Copies pairs first .. first + count - 1 into caller device buffers
 * [count][dim][n_cells] (either may be NULL); ordered on `stream`.
 * HOFV_EINVAL outside 0 .. n_pairs. */
hofv_status hofv_pairset_copy(const hofv_pairset* set, int32_t first, int32_t count, double* d_r, double* d_e,
                              void* stream);

typedef struct {
  int32_t n_starts;      /* Krylov-type sequences */
  int32_t length;        /* pairs per sequence */
  int32_t newton_steps;  /* Newton pairs */
  uint64_t seed;         /* start vectors drawn when d_starts is NULL */
  double rtol;           /* each e solved by FGMRES to ||r - J e|| <= rtol ||r|| */
  int32_t restart, max_iters, n_sweeps;  /* of those FGMRES solves (plain preconditioner) */
} hofv_harvest_opts;

/* Appends training pairs at the state d_u (device [dim][n_cells]) to `set`,
 * each e solved with the context's plain preconditioner (the sweeps, or the
 * V-cycle when selected):
 *  - Krylov-type: for each start s, v_0 = b_s / ||b_s|| and
 *    v_{k+1} = J M v_k / ||J M v_k||, k < length (the vectors FGMRES feeds the
 *    preconditioner), pairs (v_k, e_k) with J e_k = v_k; b_s is
 *    d_starts + s dim n_cells when d_starts is given, else standard normal
 *    values by Box-Muller from consecutive outputs k = 1, 2, ... of the
 *    splitmix64 generator (Steele, Lea and Flood) seeded with seed + s 2^40,
 *    two values per pair of outputs;
 *  - Newton: from u_0 = d_u, e_k with J(u_k) e_k = R(u_k) and the pair
 *    (R(u_k), e_k) / ||R(u_k)||, u_{k+1} = u_k - e_k, k < newton_steps.
 * FGMRES solves that miss rtol are kept (their e is the best iterate).
 * HOFV_EINVAL if the pairs do not fit the set's capacity (nothing is added).
 * Synchronises. */
hofv_status hofv_harvest_pairs(hofv_ctx* ctx, const double* d_u, const double* d_starts,
                               const hofv_harvest_opts* opts, hofv_pairset* set, void* stream);

typedef struct {
  int32_t epochs;
  int32_t batch;         /* pairs per optimisation step, all from one set */
  double lr;             /* Adam step */
  int32_t n_sweeps;      /* plain preconditioner sweeps inside the loss */
  uint64_t seed;         /* order of the pairs and of the minibatches */
  double* epoch_loss;    /* optional host array [epochs]: mean loss per epoch */
} hofv_train_opts;

typedef struct {
  int32_t steps;         /* optimisation steps taken */
  double loss_first, loss_last;  /* mean loss of the first and last epoch */
  double seconds;
} hofv_train_stats;

/* Trains nn over n_sets pair sets (each on its own context; the contexts may
 * differ in mesh and dimension): every epoch cuts each set, in a seeded
 * random order, into minibatches of `batch` pairs and takes one
 * hofv_nn_train_step on each minibatch, the minibatches of all sets in a
 * seeded random order (splitmix64, Fisher-Yates).  Synchronises. */
hofv_status hofv_nn_train(hofv_nn* nn, int32_t n_sets, hofv_pairset* const* sets, const hofv_train_opts* opts,
                          hofv_train_stats* stats, void* stream);

/* Per-kernel timing with HIP events recorded on the launch stream around
 * every kernel while enabled.  hofv_kernel_time synchronises and returns the
 * summed milliseconds and launch count of the kernel called `name` since the
 * last reset (enable = 1 resets). */
hofv_status hofv_set_timing(hofv_ctx* ctx, int32_t enable);
/* As hofv_set_timing(ctx, 1), but events are recorded only around launches
 * of the kernel called `name` (NULL: every kernel), so that timing one kernel
 * does not put event records between all the others. */
hofv_status hofv_set_timing_only(hofv_ctx* ctx, const char* name);
hofv_status hofv_kernel_time(hofv_ctx* ctx, const char* name, double* total_ms, int64_t* count);

/* Host copy of a setup table of a host_only context (after hofv_setup):
 * name is one of "face_stencil" [S][nf] i32, "cell_stencil" [S][nc] i32,
 * "face_coef" f64 ([S][dim][nf] folded, [S][nq][dim][nf] per point),
 * "cell_extrap" [S][2 dim][nc] f64, "face_own", "face_nei" [nf] i32,
 * "face_area_vec" f64, "face_stab" [nf] f64, "cell_faces" [2 dim][nc] i32,
 * "cell_src" [dim][nc] f64, "pc_perm" [nc] i32, "pc_dinv" [nc] f32,
 * "pc_a" [2 dim][nc] f32, "pc_nbr" [2 dim][nc] i32, "centroids" [nc][dim] f64,
 * "face_centre" [nf][dim] f64.
 * *data stays valid until hofv_destroy; *count is the number of elements and
 * *elem_bytes their size. */
hofv_status hofv_host_table(hofv_ctx* ctx, const char* name, int64_t* count, int32_t* elem_bytes,
                            const void** data);

/* Algorithmic HBM bytes of one launch of kernel `name` (the byte model). */
hofv_status hofv_kernel_bytes(hofv_ctx* ctx, const char* name, double* bytes);

#ifdef __cplusplus
}
#endif

#endif /* HOFV_H */
