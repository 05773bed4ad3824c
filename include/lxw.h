/*
 * lxw.h -- C interface of the MI355X (gfx950) library for the positivity-preserving
 * Lax-Wendroff discontinuous Galerkin (LxW-DG) time step for the compressible Euler equations
 * (S. A. Moe, J. A. Rossmanith, D. C. Seal, "Positivity-preserving discontinuous Galerkin
 * methods with Lax-Wendroff time discretizations", arXiv:1601.08145).
 *
 * The calls follow the paper's statement of the problem: a mesh of elements (Sec. 1.2), the gas
 * constant gamma (Eq. (eos)), the polynomial degree M_D (Eq. (broken_space)), the initial modal
 * coefficients Q^(l) (Sec. 1.2), the CFL number (Sec. 4.1), boundary conditions (Sec. 2.4), and
 * advancing to a final time T (Eq. (exact-taylor)).
 *
 * Conventions shared by every call:
 *  - All functions return lxw_status: LXW_OK (0) or a negative error code.  No C++ exception
 *    crosses this interface.  lxw_last_error() returns a thread-local message for the most recent
 *    failure on the calling thread, naming the offending element where there is one.
 *  - Host arrays passed in are copied; the caller keeps ownership.  Device pointers (flag
 *    LXW_DEVICE_PTR) stay owned by the caller and are only used during the call, on the solver's
 *    stream.
 *  - Element order in every array is the caller's order (the library reorders elements
 *    internally for locality and maps back).
 *  - Modal coefficients are float64, row-major Q[n_elem][n_var][n_modes], with n_var = 3 in 1D
 *    (rho, M, E) and 4 in 2D (rho, Mx, My, E), in the documented orthonormal basis (see
 *    lxw_refelem_info): phi_1 == 1, so Q[i][v][0] is the cell average of variable v.
 *  - Reference elements: 1D [-1,1]; quadrilateral [-1,1]^2 with vertices (-1,-1), (1,-1), (1,1),
 *    (-1,1); triangle (0,0), (1,0), (0,1).  Local edge k joins vertices k and k+1 (mod count);
 *    in 1D local edge 0 is the left end and 1 the right end.  Tetrahedron (0,0,0), (1,0,0),
 *    (0,1,0), (0,0,1) (3D, the construction of Sec. 3.3 carried face by face, as the paper
 *    remarks): local face k is opposite vertex k.  n_var = 5 in 3D (rho, Mx, My, Mz, E).
 *  - Basis: Gram-Schmidt orthonormalisation, under (1/|T0|) int_{T0} f g, of the monomials
 *    1D {1, x, x^2}; quadrilateral {1, x, y, x^2, xy, y^2, x^2 y, x y^2, x^2 y^2} (tensor Legendre,
 *    9 modes); triangle {1, x, y, x^2, xy, y^2} (6 modes); tetrahedron {1, x, y, z, x^2, xy, xz,
 *    y^2, yz, z^2} (10 modes).  At degree 3 (line and triangle, the
 *    construction of Sec. 2.2 one order further): 1D {1, x, x^2, x^3} (4 modes), triangle
 *    {1, x, y, x^2, xy, y^2, x^3, x^2 y, x y^2, y^3} (10 modes); n_modes in Q is then the
 *    degree's count, not the mesh's (lxw_mesh_get_info reports degree 2).
 */
#ifndef LXW_H
#define LXW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lxw_status;

enum {
  LXW_OK = 0,
  LXW_ERR_ARG = -1,         /* invalid argument (null pointer, size, enum value) */
  LXW_ERR_UNSUPPORTED = -2, /* valid but not implemented (e.g. degree 4, or degree 3 on quadrilaterals) */
  LXW_ERR_MESH = -3,        /* non-positive area, clockwise triangle, bad connectivity */
  LXW_ERR_STATE = -4,       /* input state violates rho_bar >= eps0, p_bar > 0 (Sec. 1.5 Step 1,
                               Sec. 3.1 Step 0) or is not finite */
  LXW_ERR_POSITIVITY = -5,  /* a cell average lost positivity during a step */
  LXW_ERR_NONFINITE = -6,   /* a non-finite value appeared during a step */
  LXW_ERR_CFL = -7,         /* the first-order Lax-Friedrichs update is not positive (Gamma < 0,
                               Sec. 3.2): the time step is too large for the CFL condition */
  LXW_ERR_DEVICE = -8,      /* a HIP runtime call failed */
  LXW_ERR_OOM = -9          /* device or host allocation failed */
};

/* Boundary conditions (Sec. 2.4).  Periodic pairs opposite sides.  Transparent: ghost state
 * equals the interior trace.  Reflective: normal momentum negated, tangential kept, and the same
 * for q_t and q_tt (and q_ttt at degree 3).  Inflow: a fixed Dirichlet state (lxw_params.inflow)
 * with q_t = q_tt = 0 (and q_ttt = 0). */
enum { LXW_BC_PERIODIC = 0, LXW_BC_TRANSPARENT = 1, LXW_BC_REFLECTIVE = 2, LXW_BC_INFLOW = 3 };

/* Mesh kinds. */
enum { LXW_LINE = 0, LXW_QUAD = 1, LXW_TRI = 2, LXW_TET = 3 };

/* Arithmetic of the step. */
enum {
  LXW_FP64 = 0,      /* everything in float64 */
  LXW_FP32_MIXED = 1 /* higher modes, point values, F_T, traces and edge point fluxes in float32;
                        cell averages, the flux limiter (Gamma, corner states, damping-factor
                        solve), the point pressure and theta of the moment limiter, the wave
                        speed, dt and t in float64 */
};

/* Shock-capturing limiter modes. */
enum { LXW_SHOCK_OFF = 0, LXW_SHOCK_PLAIN = 1 };

/* Where the global wave speed s is measured (lxw_params.wave_speed). */
enum { LXW_SPEED_POINTS = 0, LXW_SPEED_AVERAGES = 1 };

/* State transfer flags (LXW_STATE_UNCHECKED may be or-ed with either pointer kind). */
enum { LXW_HOST_PTR = 0, LXW_DEVICE_PTR = 1, LXW_STATE_UNCHECKED = 2 };

typedef struct lxw_mesh lxw_mesh;
typedef struct lxw_solver lxw_solver;
typedef struct lxw_batch lxw_batch;
typedef struct lxw_indicator lxw_indicator;

typedef struct lxw_params {
  double gamma;      /* ratio of specific heats, Eq. (eos); > 1 */
  int32_t degree;    /* polynomial degree M_D: 2, or 3 on line and triangle meshes for single-mesh
                        solvers without the learned indicator (LXW_ERR_UNSUPPORTED else).  Degree 3
                        adds q_ttt to the time-averaged flux (Sec. 2.2: F_T to dt^3); it is stable
                        at smaller Courant numbers than degree 2 (0.05 where 0.1 is not) */
  double cfl;        /* CFL number nu: dt = nu / (s * max_i |dT_i| / (2 |T_i|)), s the global
                        maximum wave speed; the paper uses 0.08 (Sec. 4.1); must be in (0, 1] */
  double eps0;       /* density cutoff eps0 of Sec. 3.1 Step 0 (1e-12 in the paper); > 0 */
  double alpha0;     /* shock-limiter relaxation constant: delta = alpha0 h^1.5 (500, Sec. 4.1) */
  int32_t precision; /* LXW_FP64 or LXW_FP32_MIXED */
  int32_t shock;     /* LXW_SHOCK_OFF or LXW_SHOCK_PLAIN */
  double inflow[4];  /* inflow state for LXW_BC_INFLOW edges: (rho, Mx, My, E); 1D uses
                        (rho, Mx, -, E) */
  int32_t theta_exact; /* 0: the moment limiter's pressure factor by the concavity bound of
                        Sec. 3.1 (the paper's method); 1: by the exact root of the quadratic
                        rho p = (gamma-1)(a theta^2 + b theta + c) of Sec. 3.1 (the optimal factor the
                        paper mentions), moved inside by a relative 1e-10 and checked in float64,
                        never below the concavity value */
  int32_t wave_speed;  /* the global wave speed s (Sec. 4.1: an estimate of the largest speed):
                        LXW_SPEED_POINTS (default) the largest |u| + c over the cell averages and
                        every limited point; LXW_SPEED_AVERAGES over the cell averages only (the
                        speeds the Lax-Friedrichs fluxes of the positivity argument need; near
                        vacuum the limited points' speeds can exceed them a hundredfold) */
} lxw_params;

/* Fills p with the paper's defaults: gamma 1.4, degree 2, CFL 0.08, eps0 1e-12, alpha0 500,
 * FP64, plain shock limiter, inflow (1, 0, 0, 2.5), concavity bound (theta_exact 0), wave speed
 * over the limited points (LXW_SPEED_POINTS). */
lxw_status lxw_params_default(lxw_params* p);

/* Message of the last failure on this thread (never null; empty when none). */
const char* lxw_last_error(void);

/* ---- Meshes (Sec. 1.2; edges, normals n_e with |n_e| = edge length, i_e, j_e and eps_ik as
 * defined in Sec. 3.3, Eq. (epsik)) --------------------------------------------------------- */

/* Uniform 1D mesh of n cells on [x0, x1]; bc_left/bc_right are LXW_BC_* (both periodic or
 * neither).  Errors: LXW_ERR_ARG for n < 2, x1 <= x0, or an unpaired periodic side. */
lxw_status lxw_mesh_create_1d(int32_t n, double x0, double x1, int32_t bc_left, int32_t bc_right,
                              lxw_mesh** out);

/* Cartesian mesh of nx x ny rectangles on [x0,x1] x [y0,y1]; caller element index i + nx*j.
 * bc = {x-low, x-high, y-low, y-high}; periodic must be set on both sides of a direction. */
lxw_status lxw_mesh_create_cart(int32_t nx, int32_t ny, double x0, double x1, double y0, double y1,
                                const int32_t bc[4], lxw_mesh** out);

/* Cartesian mesh with cells removed (the solid of the paper's Cartesian shock-diffraction problem
 * over a step, Sec. 4): as lxw_mesh_create_cart, where keep[nx*ny] (host, read during the call;
 * cell (i, j) at i + nx*j) is 0 for a removed cell.  The kept cells are numbered in that
 * row-major order (the caller's element index), and their edges facing a removed cell get the
 * boundary type wall_bc (LXW_BC_REFLECTIVE, LXW_BC_TRANSPARENT or LXW_BC_INFLOW); a periodic
 * partner that is removed counts as such a face.  keep == NULL keeps every cell.  Errors: as
 * lxw_mesh_create_cart; LXW_ERR_ARG for a wall_bc that is not one of those three or a mask that
 * keeps no cell. */
lxw_status lxw_mesh_create_cart_masked(int32_t nx, int32_t ny, double x0, double x1, double y0, double y1,
                                       const int32_t bc[4], const uint8_t* keep, int32_t wall_bc,
                                       lxw_mesh** out);

/* Unstructured triangle mesh: xy[n_nodes][2] node coordinates, tri[n_tri][3] counter-clockwise
 * vertex indices.  bnd_tag (nullable, [n_tri][3]) gives the LXW_BC_* code of local edge k of
 * each triangle when that edge is on the boundary (ignored inside; transparent when null).
 * Edges tagged LXW_BC_PERIODIC are paired with the boundary edge whose midpoint differs by
 * period[0] in x or period[1] in y (period nullable otherwise).  Errors: LXW_ERR_MESH for a
 * clockwise or degenerate triangle, an edge shared by more than two triangles, or an unpaired
 * periodic edge; LXW_ERR_ARG for null arrays or out-of-range indices. */
lxw_status lxw_mesh_create_tri(int32_t n_nodes, const double* xy, int32_t n_tri, const int32_t* tri,
                               const int32_t* bnd_tag, const double* period, lxw_mesh** out);

/* Tetrahedral mesh (3D P2; Sec. 3.3's closing remark): n_nodes nodes xyz[n][3], n_tet positively
 * oriented tetrahedra tet[n_tet][4] (det [v1-v0, v2-v0, v3-v0] > 0), optional boundary codes
 * bnd_tag[n_tet][4] for the boundary faces (face k opposite vertex k; periodic, transparent or
 * reflective; null: transparent), period[3] (lengths; 0 for an axis that is not periodic) when a
 * code is periodic: periodic faces are paired by their centroids modulo the period.  Quadrature:
 * 27-point collapsed Gauss rule inside (degree 5), the 7-point triangle rule on each face.  Errors:
 * LXW_ERR_UNSUPPORTED for inflow sides; LXW_ERR_MESH for a degenerate or negatively oriented
 * tetrahedron, a face shared by more than two tetrahedra or an unpaired periodic face;
 * LXW_ERR_ARG for null arrays or out-of-range indices.  Tetrahedral meshes take single-mesh
 * solvers of degree 2 without the learned indicator. */
lxw_status lxw_mesh_create_tet(int32_t n_nodes, const double* xyz, int32_t n_tet, const int32_t* tet,
                               const int32_t* bnd_tag, const double* period, lxw_mesh** out);

lxw_status lxw_mesh_destroy(lxw_mesh* m);

typedef struct lxw_mesh_info {
  int32_t kind;      /* LXW_LINE, LXW_QUAD, LXW_TRI, LXW_TET */
  int32_t dim;       /* 1, 2 or 3 */
  int32_t n_elem;
  int32_t n_edge;
  int32_t n_var;     /* 3, 4 or 5 */
  int32_t n_modes;   /* 3, 9, 6 or 10 */
  int32_t n_faces;   /* edges (faces) per element K: 2, 4, 3 or 4 */
  double min_area, max_area;
} lxw_mesh_info;

lxw_status lxw_mesh_get_info(const lxw_mesh* m, lxw_mesh_info* out);

/* Reference-element tables so that callers can L2-project initial data (Sec. 1.2).  For mesh
 * kind `kind`: n_pts interior quadrature points xi[n_pts][dim] with weights w[n_pts] normalised
 * to sum to 1, and basis values phi[n_pts][n_modes].  Pass null arrays to query n_pts only.
 * Projection: Q_l = sum_m w_m f(x(xi_m)) phi_l(xi_m), exact for f of degree <= 3 (triangle
 * 7-point degree-5 rule; 3-point and 3x3 Gauss-Legendre in 1D and on quadrilaterals). */
lxw_status lxw_refelem_info(int32_t kind, int32_t* n_pts, double* xi, double* w, double* phi);

/* The same at polynomial degree `degree` (2, or 3 for LXW_LINE and LXW_TRI; LXW_ERR_UNSUPPORTED
 * else).  Degree 3: the 4-point Gauss-Legendre rule in 1D and a 16-point collapsed Gauss rule on
 * the triangle (both exact to degree 7), phi[n_pts][4] or [n_pts][10]; the projection is exact for
 * f of degree <= 4. */
lxw_status lxw_refelem_info_deg(int32_t kind, int32_t degree, int32_t* n_pts, double* xi, double* w, double* phi);

/* ---- Solver ------------------------------------------------------------------------------ */

/* Creates a solver on device 0 for mesh m (which must outlive it).  stream: a hipStream_t (null
 * for the default stream); every kernel of the solver runs on it.  Allocates all device memory
 * the step needs.  Device arrays use 32-bit indices: n_var * n_modes * n_elem and
 * 2 * q * n_var * n_edges (q = degree + 1 edge points in 2D, 1 in 1D) must not exceed 2^31 - 1 (about 89
 * million P2 triangles or 59 million Q2 quadrilaterals per solver).  Errors: LXW_ERR_ARG / LXW_ERR_UNSUPPORTED for bad parameters or a
 * mesh above that size, LXW_ERR_OOM, LXW_ERR_DEVICE. */
lxw_status lxw_solver_create(const lxw_mesh* m, const lxw_params* p, void* stream, lxw_solver** out);
lxw_status lxw_solver_destroy(lxw_solver* s);

/* Sets the state: Q as described above (host or device memory per flags) and the time t0.
 * Checks rho_bar >= eps0, p_bar > 0 and finiteness of every coefficient (LXW_ERR_STATE, naming
 * the first bad element in the caller's order).  With LXW_STATE_UNCHECKED in flags these host-side
 * checks are skipped (a state the caller already trusts, e.g. one read back from a solver of the
 * same mesh); the device-side checks of the next step still report a cell average that is not
 * positive (LXW_ERR_POSITIVITY) or not finite (LXW_ERR_NONFINITE), naming the element.
 * Synchronous. */
lxw_status lxw_set_state(lxw_solver* s, const double* Q, double t0, int32_t flags);

/* Copies the state after the last completed step (shock-capturing limiter applied) into Q and
 * the time into *t (t nullable).  Synchronous; also reports a pending device error. */
lxw_status lxw_get_state(lxw_solver* s, double* Q, double* t, int32_t flags);

/* One step of Sec. 3.3 (moment limiter, F_T, edge fluxes, flux limiter, update) followed by the
 * shock-capturing limiter, with dt = min(dt_CFL, T - t).  Synchronous; *dt_taken nullable.
 * Errors: LXW_ERR_ARG if t >= T; LXW_ERR_POSITIVITY / LXW_ERR_NONFINITE / LXW_ERR_CFL from the
 * device checks (the state is then left as the failing step produced it). */
lxw_status lxw_step(lxw_solver* s, double T, double* dt_taken);

typedef struct lxw_stats {
  int64_t steps;     /* steps taken by the call */
  double t;          /* time reached */
  double last_dt;
  double last_s;     /* global wave speed of the last step */
} lxw_stats;

/* Steps until t == T (the last dt is clipped) or max_steps steps.  Synchronous.  The end time is
 * kept on the device, where every step is clipped to it and a step at t == T changes nothing;
 * the steps are enqueued in chunks (replays of the captured step graph, as lxw_run_steps) with
 * one synchronisation per chunk, and the result equals that of single lxw_step calls to T. */
lxw_status lxw_advance(lxw_solver* s, double T, int64_t max_steps, lxw_stats* out);

/* Enqueues n_steps steps with no final time (dt from the CFL condition each step) on the
 * solver's stream and returns without waiting; errors are reported by lxw_sync.  Unless per-kernel
 * timing or stage read-out is on, the steps are replays of one step captured in a HIP graph (on a
 * stream the library creates; the replays go to the solver's stream).  Results are identical
 * either way. */
lxw_status lxw_run_steps(lxw_solver* s, int64_t n_steps);

/* lxw_set_graph(s, 0) makes lxw_run_steps launch every kernel itself instead of replaying the
 * captured graph; 1 (the default) restores graph replay. */
lxw_status lxw_set_graph(lxw_solver* s, int32_t enable);

/* Waits for the solver's stream and reports any device error. */
lxw_status lxw_sync(lxw_solver* s);

/* ---- Diagnostics ----------------------------------------------------------------------------
 * lxw_set_debug(s, 1) makes later steps keep copies of their intermediate results, which
 * lxw_debug_stage then returns in float64 and in the caller's element order:
 *   LXW_STAGE_QLIM     Q after the shock and moment limiters, at the start of the step [N][V][ML]
 *   LXW_STAGE_THETA    moment-limiter theta [N]
 *   LXW_STAGE_VOL      volume term V_l = (1/|T|) int grad phi_l . F_T [N][V][ML] (mode 1 is 0)
 *   LXW_STAGE_FLXW     f^LxW of each local edge, oriented out of the element [N][K][V]
 *   LXW_STAGE_FLXF     f^LxF likewise [N][K][V]
 *   LXW_STAGE_C        damping factor candidate Lambda_ik * min mu of each local edge [N][K]
 *   LXW_STAGE_LAME     Lambda_e of each local edge [N][K]
 *   LXW_STAGE_QUPD     Q after the update, before the shock-capturing limiter [N][V][ML]
 *   LXW_STAGE_THETA_SC shock-limiter theta applied after the update [N]
 *   LXW_STAGE_SDT      {s, dt} [2]
 * Per-kernel timing: lxw_set_timing(s, 1) records HIP events around every kernel of later steps;
 * lxw_kernel_times returns, per kernel id (LXW_K_*), the summed milliseconds and launch counts.
 * A step ends inside the LXW_K_UPDATE kernel; LXW_K_FINAL counts only the kernel that closes a
 * state read-out which applied the pending shock-capturing limiter. */
enum {
  LXW_STAGE_QLIM = 0, LXW_STAGE_THETA = 1, LXW_STAGE_VOL = 2, LXW_STAGE_FLXW = 3, LXW_STAGE_FLXF = 4,
  LXW_STAGE_C = 6, LXW_STAGE_LAME = 7, LXW_STAGE_QUPD = 8, LXW_STAGE_THETA_SC = 9, LXW_STAGE_SDT = 10
};
enum { LXW_K_PRE = 0, LXW_K_DT = 1, LXW_K_ELEM = 2, LXW_K_EDGE = 3, LXW_K_FLIM = 4, LXW_K_UPDATE = 5,
       LXW_K_FINAL = 6, LXW_K_IND = 7, LXW_K_COUNT = 8 };

lxw_status lxw_set_debug(lxw_solver* s, int32_t keep_stages);
lxw_status lxw_debug_stage(lxw_solver* s, int32_t stage, double* out);
lxw_status lxw_set_timing(lxw_solver* s, int32_t enable);
lxw_status lxw_kernel_times(lxw_solver* s, double* ms /*[LXW_K_COUNT]*/, int64_t* launches /*[LXW_K_COUNT]*/);

/* ---- Launch shapes and the autotuner --------------------------------------------------------
 * Every element kernel runs one lane per element and the edge kernel one lane per edge, so the
 * workgroup size block[k] of kernel k (indexed by LXW_K_*) is also its number of elements (edges)
 * per workgroup.  LXW_K_PRE, LXW_K_ELEM, LXW_K_EDGE, LXW_K_FLIM and LXW_K_UPDATE accept 64, 128 or
 * 256 (defaults 256, 128, 256, 256, 256); the entries of LXW_K_DT, LXW_K_FINAL and LXW_K_IND are
 * ignored.
 * persistent (batches of triangle meshes only): 0 (default) runs a step as one launch per phase,
 * replayed from a HIP graph; 128 or 256 runs lxw_batch_advance_steps as one cooperative launch of a
 * persistent kernel (up to 1024 steps per launch) whose workgroups of that many lanes stay resident
 * and run every phase of every step over tiles of elements and edges, with grid-wide barriers where
 * the per-phase launches have kernel boundaries.  It applies while per-kernel timing, stage
 * read-out and the learned indicator are off (the per-phase launches run otherwise).
 * Launch shapes change no result bit. */
typedef struct lxw_tune {
  int32_t block[LXW_K_COUNT];
  int32_t persistent;
} lxw_tune;

lxw_status lxw_get_tune(const lxw_solver* s, lxw_tune* out);
/* LXW_ERR_ARG for a size other than 64, 128, 256 in a tunable entry or a persistent value other
 * than 0, 128, 256; LXW_ERR_UNSUPPORTED for a non-zero persistent on a solver that does not run a
 * batch of triangle meshes. */
lxw_status lxw_set_tune(lxw_solver* s, const lxw_tune* t);
/* Times each allowed size of each tunable kernel on the solver's own mesh and current state (one
 * warm-up step, then trial_steps timed steps per candidate, kernels tuned one after another),
 * keeps the fastest per kernel; for a batch of triangle meshes it then times trial_steps whole
 * steps of the per-phase launches (graph replay) against the persistent kernel at 128 and 256 lanes
 * per workgroup and keeps the fastest.  It restores the state, time and counters it found, so tuning does not change the
 * trajectory.  Synchronous; the chosen shapes also go to *out (nullable).  A device error during
 * the trials is returned after the state has been restored. */
lxw_status lxw_autotune(lxw_solver* s, int32_t trial_steps, lxw_tune* out);

/* ---- Batched form -------------------------------------------------------------------------
 * n independent meshes of one kind advanced together: each kernel of a step is one launch over
 * every element (edge) of every mesh, and a step is replayed from a HIP graph.  Each mesh keeps its
 * own wave speed s, time step dt (the CFL condition of Sec. 4.1 per mesh) and time t; the scheme
 * per mesh is exactly that of a single-mesh solver, bit for bit (same kernels, same arithmetic).
 * Parameters are shared.  meshes[i] must outlive the batch.  Errors: LXW_ERR_ARG for n < 1, a null
 * mesh, meshes of different kinds or more than 2^28 elements or edges in total; as
 * lxw_solver_create otherwise. */
lxw_status lxw_batch_create(int32_t n, const lxw_mesh* const* meshes, const lxw_params* p, void* stream,
                            lxw_batch** out);
lxw_status lxw_batch_destroy(lxw_batch* b);
/* State of mesh i, layout and checks as lxw_set_state / lxw_get_state; time t0 for that mesh.
 * Synchronous. */
lxw_status lxw_batch_set_state(lxw_batch* b, int32_t i, const double* Q, double t0, int32_t flags);
lxw_status lxw_batch_get_state(lxw_batch* b, int32_t i, double* Q, double* t, int32_t flags);
/* Enqueues n_steps steps of every mesh (no final time) and returns without waiting. */
lxw_status lxw_batch_advance_steps(lxw_batch* b, int64_t n_steps);
/* Waits, then reports mesh i: steps since its state was set, t, last dt and last s. */
lxw_status lxw_batch_stats(lxw_batch* b, int32_t i, lxw_stats* out);
/* The solver that runs the batch, for lxw_sync, lxw_set_tune / lxw_get_tune / lxw_autotune,
 * lxw_set_graph, lxw_set_timing, lxw_kernel_times, and (triangle meshes) lxw_solver_set_indicator
 * and lxw_indicator_decisions, whose flags then follow the meshes' caller orders one after
 * another (the per-mesh calls above handle state;
 * lxw_step, lxw_advance, lxw_set_state, lxw_get_state and lxw_set_debug return
 * LXW_ERR_UNSUPPORTED on it).  Owned by the batch. */
lxw_solver* lxw_batch_solver(lxw_batch* b);

/* ---- Learned troubled-cell indicator (P2 triangles) ---------------------------------------
 * The paper detects troubled cells with the shock-capturing limiter it cites (Sec. 1.5 Step 5,
 * Sec. 4.1).  The learned form keeps that limiter and the positivity limiters of Secs. 3.1-3.3 and
 * replaces only the detection: a multilayer perceptron 48 -> 64 (ReLU) -> 64 (ReLU) -> 1 (sigmoid)
 * gives each cell a probability p that the shock-capturing limiter acts on it; cells with
 * p < tau_lo skip that limiter, cells with p >= tau_hi are flagged and the rest use the plain
 * detection (both run the limiter, which then acts only where its bounds are violated).
 * Features (48 per triangle): cells c = (i, n_0, n_1, n_2), n_k the neighbour across local edge k
 * (i itself on the boundary); for rho and then E the 24 values Q[c][var][l] (c-major, l = 0..5)
 * with the centre cell's average subtracted from the four mode-1 entries, divided by
 * (max |value| + delta_i + 1e-6 |centre average| + 1e-30), delta_i = alpha0 h_i^1.5 the
 * shock-capturing limiter's relaxation (h_i = sqrt(2 |T_i|)).  Parameters: one float32 vector of LXW_IND_NPARAM values W1[48][64],
 * b1[64], W2[64][64], b2[64], w3[64], b3 (row-major, input index first).  Inference runs the
 * two hidden layers on the bf16 matrix cores (inputs, weights and hidden activations rounded to
 * bfloat16, float32 accumulation); training runs in float32.  Random numbers (initial weights,
 * sample order) come from the caller. */
enum { LXW_IND_NFEAT = 48, LXW_IND_NPARAM = 7361 };

typedef struct lxw_adam {
  double lr, beta1, beta2, eps; /* Adam (Kingma & Ba); e.g. 1e-3, 0.9, 0.999, 1e-8 */
  double w_pos, w_neg;          /* class weights of the cross-entropy (y = 1, y = 0) */
} lxw_adam;

/* Creates an indicator with parameters params (host, LXW_IND_NPARAM floats) whose kernels run on
 * stream (a hipStream_t, null for the default stream). */
lxw_status lxw_indicator_create(const float* params, void* stream, lxw_indicator** out);
lxw_status lxw_indicator_destroy(lxw_indicator* ind);
/* Master float32 parameters to / from host memory; setting them resets the Adam state. */
lxw_status lxw_indicator_get_params(const lxw_indicator* ind, float* out);
lxw_status lxw_indicator_set_params(lxw_indicator* ind, const float* params);
/* Binary file: 8-byte tag "LXWIND01", int32 LXW_IND_NPARAM, the float32 parameters. */
lxw_status lxw_indicator_save(const lxw_indicator* ind, const char* path);
lxw_status lxw_indicator_load(lxw_indicator* ind, const char* path);

/* Probabilities p[n] of features X[n][48] (device memory, float32) by the inference kernel. */
lxw_status lxw_indicator_predict(lxw_indicator* ind, const float* X, int32_t n, float* p);

/* Gradient of the class-weighted cross-entropy
 *   L = -(1/n) sum_i [w_pos y_i log p_i + w_neg (1 - y_i) log(1 - p_i)]
 * over X[n][48], y[n] (device, float32) by the training kernels: grad[LXW_IND_NPARAM] (host) and
 * *loss (nullable).  Synchronous. */
lxw_status lxw_indicator_grad(lxw_indicator* ind, const float* X, const float* y, int32_t n, double w_pos,
                              double w_neg, float* grad, double* loss);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight training
 * loops, harnesses that forbid hipMalloc): the gradient of lxw_indicator_grad, with X[n][48], y[n],
 * grad[LXW_IND_NPARAM] and loss (nullable, one float) all device memory owned by the caller,
 * enqueued on the indicator's stream without waiting (the results are there once that stream has
 * reached this point).  Allocates nothing: its per-workgroup partial gradients live in a fixed
 * device workspace of the library (3.6 MiB per device, held until the process ends), which limits
 * n to 1 .. LXW_IND_NOALLOC_MAX (LXW_ERR_ARG otherwise).  Calls that overlap on one device share
 * that workspace and race; calls ordered on one stream do not.  Results equal lxw_indicator_grad's
 * bit for bit. */
enum { LXW_IND_NOALLOC_MAX = 8192 };
lxw_status lxw_indicator_grad_noalloc(lxw_indicator* ind, const float* X, const float* y, int32_t n, double w_pos,
                                      double w_neg, float* grad, float* loss);

/* n_updates Adam updates with float32 master weights; update u uses the minibatch of samples
 * order[u*batch .. (u+1)*batch) of X[n_samples][48], y[n_samples] (all device memory; order
 * entries outside [0, n_samples) are clamped).  *last_loss (nullable): the last minibatch's loss.
 * Synchronous; the inference weights follow the new parameters. */
lxw_status lxw_indicator_train(lxw_indicator* ind, const float* X, const float* y, int32_t n_samples,
                               const int32_t* order, int32_t n_updates, int32_t batch, const lxw_adam* hp,
                               double* last_loss);

/* Training data from a solver whose shock-capturing limiter is pending (after lxw_step, with no
 * state read in between): features X[n_elem][48] (float32) of the state that limiter is about to
 * see and the factor theta_sc[n_elem] it will apply (1: the cell is left alone), both in the
 * caller's element order, host or device memory per flags.  Changes nothing.  Single triangle
 * meshes only (LXW_ERR_UNSUPPORTED else); LXW_ERR_ARG if no limiter is pending. */
lxw_status lxw_indicator_collect(lxw_solver* s, float* X, double* theta_sc, int32_t flags);

/* Uses ind (which must outlive the solver's use of it) for later steps of s; null restores the
 * plain limiter everywhere.  Needs 0 <= tau_lo <= tau_hi <= 1.  Resets the decision counts. */
lxw_status lxw_solver_set_indicator(lxw_solver* s, const lxw_indicator* ind, double tau_lo, double tau_hi);
/* Decisions since lxw_solver_set_indicator: counts[3] = (skipped, plain detection, flagged), and
 * (flags nullable) the last decision per element in the caller's order (0, 1, 2).  Synchronous. */
lxw_status lxw_indicator_decisions(lxw_solver* s, int64_t* counts, uint8_t* flags);

#ifdef __cplusplus
}
#endif

#endif /* LXW_H */
