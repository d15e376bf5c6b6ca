/*
 * teno.h -- C ABI of libteno: the per-cell, per-Runge-Kutta-stage residual of
 * the unstructured-mesh finite-volume TENO scheme (Ji, Liang & Fu, "A class of
 * new high-order finite-volume TENO schemes for hyperbolic conservation laws
 * with unstructured meshes") for the 2D Euler equations on triangle meshes
 * (periodic, or with transmissive, reflective and prescribed boundaries), in
 * FP64, on AMD Instinct MI355X (gfx950).
 *
 * Conventions for every call
 *  - Return value: TENO_OK (0) or a negative teno_status; teno_last_error()
 *    returns a message for the calling thread.  No C++ exception crosses the
 *    ABI.  Argument and shape errors are reported synchronously.
 *  - State arrays (U, R, lambda, U_bar) are caller-owned DEVICE pointers to
 *    double[n_cell][4] = (rho, rho*u, rho*v, E), contiguous, in the library's
 *    INTERNAL cell order (see teno_mesh_permutation).  Flags are caller-owned
 *    device uint16_t[n_cell].  dt is a caller-owned device double.
 *  - Work is enqueued on the caller's HIP stream (hipStream_t passed as void*;
 *    NULL = legacy default stream) and returns without synchronising, except
 *    where a call says otherwise.  Per-step calls never allocate.
 *  - Mesh and set-up calls are host-only (no GPU needed).
 */
#ifndef TENO_H
#define TENO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum teno_status {
  TENO_OK = 0,
  TENO_EARG = -1,      /* bad argument, size or state of the object            */
  TENO_EMESH = -2,     /* degenerate triangle, open or non-manifold edge       */
  TENO_ESTENCIL = -3,  /* mesh too small for the requested stencils            */
  TENO_ERANK = -4,     /* rank-deficient least-squares matrix                  */
  TENO_EHIP = -5,      /* HIP runtime error (message names the call)           */
  TENO_ENOMEM = -6     /* host or device allocation failed                     */
} teno_status;

/* Boundary conditions of boundary faces (meshes with an open axis).  The
 * paper's shock-tube, explosion and double-Mach-reflection tests (Sec.
 * 5.4-5.6, 5.8) need walls, inflow and outflow; it does not state how they
 * are imposed.  Each kind fixes the outer state of the face's Riemann
 * problem at every Gauss point: */
typedef enum teno_bc {
  TENO_BC_TRANSMISSIVE = 1, /* outflow: the inner face state (zero gradient)  */
  TENO_BC_REFLECTIVE = 2,   /* slip wall: the inner state, normal momentum    */
                            /* reversed                                       */
  TENO_BC_PRESCRIBED = 3    /* inflow or far field: a given conservative state */
} teno_bc;

typedef struct teno_mesh teno_mesh;
typedef struct teno_solver teno_solver;
typedef struct teno_batch teno_batch;

/* Scheme parameters.  Defaults (teno_default_params) are the paper's fixed
 * built-in values: C_T = 1e-6 in both selection steps and eps = 1e-12 with
 * exponent 6 in the scale separation (Sec. 3.2-3.3), gamma = 1.4.  For the
 * CWENO variant the paper uses power = 4, eps = 1e-14 and dk_prime = 1e4
 * (Sec. 2.4). */
typedef struct teno_params {
  int32_t order;     /* 3..6: large-stencil degree order-1, Sec. 2.2 eq. 03   */
  int32_t n_quad;    /* Gauss points per face, 0 = ceil(order/2)              */
  int32_t variant;   /* 0 = TENO (Sec. 3), 1 = LINEAR (large stencil only),   */
                     /* 2 = CWENO (Sec. 2.4; no selection, flags 0, no        */
                     /* frozen or adjoint calls, no batches)                  */
  int32_t power;     /* exponent of the weights (paper: 6 TENO, 4 CWENO)      */
  double ct;         /* cutoff C_T in [0, 1/3] (paper: 1e-6)                  */
  double eps;        /* epsilon of the weights (paper: 1e-12 TENO, 1e-14 CWENO) */
  double gamma;      /* ratio of specific heats                               */
  double tie_rel;    /* near-tie band: |chi/C_T - 1| <= tie_rel is counted    */
  int32_t fallback;  /* 1: a cell with a non-physical face state uses its    */
                     /* cell average on every face and flags 0 (not in the   */
                     /* paper; default 0)                                     */
  int32_t reorder;   /* 1 = Morton order of cells (default), 0 = user order   */
  int32_t n_threads; /* host threads for set-up, 0 = hardware concurrency     */
  int32_t characteristic; /* 1: select in characteristic variables, edge by */
                     /* edge (Sec. 2.3; eigenvectors of the flux Jacobian in */
                     /* the edge normal at the cell mean): flags become one  */
                     /* word per local edge, no frozen or adjoint calls, no  */
                     /* batches; 0: conservative variables (default)         */
  double dk_prime;   /* CWENO: d_K = 1 - 1/dk_prime > 0 (paper: 1e4)          */
} teno_params;

typedef struct teno_info {
  int32_t n_cell, n_face, order, n_quad;
  int32_t n_coef_large, rows_large;  /* unknowns / rows of the large stencil */
  int32_t n_coef_small, rows_small;  /* 5 / 11 for the third-order stencils  */
  int64_t matrix_doubles_per_cell;   /* streamed pseudo-inverse entries      */
  int64_t device_bytes;              /* library-owned device memory          */
  double min_rcond;                  /* min over stencils of min|R_jj|/max|R_jj| */
  int64_t face_state_doubles;        /* one stage's face states in the library  */
                                     /* layout (teno_rk_step, teno_vjp_rk_step) */
  int64_t n_bface;                   /* boundary faces (0 on a periodic mesh)  */
} teno_info;

/* Device-side diagnostics, accumulated until reset. */
typedef struct teno_diag {
  int64_t nonphysical;    /* cells with rho<=0, p<=0 or NaN at the average or */
                          /* a face point, per reconstruction                 */
  int64_t first_bad_cell; /* lowest USER id among them, -1 if none            */
  int64_t near_ties;      /* chi within tie_rel of C_T                        */
  int64_t fallbacks;      /* cells reconstructed at first order               */
} teno_diag;

const char* teno_last_error(void);
void teno_default_params(teno_params* p);

/* ---- mesh and set-up (host only) --------------------------------------- */

/* Geometry and faces, Sec. 2.1.  xy: host double[n_vert][2]; tri: host
 * int32[n_cell][3] (orientation fixed to counter-clockwise internally by
 * swapping the last two vertices); period: host double[2], the period of
 * each axis or 0 for an open axis; NULL opens both.  On a mesh periodic in
 * both axes every edge must be shared by exactly two cells, else
 * TENO_EMESH; with an open axis an edge with one cell is a boundary face
 * (transmissive until teno_mesh_set_boundary says otherwise).  Copies its
 * inputs; *out is owned by the caller. */
int teno_mesh_create(int32_t n_vert, const double* xy, int32_t n_cell, const int32_t* tri,
                     const double* period, teno_mesh** out);

/* Stencils (Sec. 3.1: one central stencil of 2N_k cells incl. the target and
 * three directional third-order stencils of 12 cells), reference-space
 * least-squares matrices and their Householder pseudo-inverses
 * (Sec. 2.2 eqs. 02-10), cell reordering and device packing.
 * Errors: TENO_ESTENCIL (also when a tile of 16 consecutive cells of the
 * internal order has more than 384 distinct stencil members, which the
 * default reordering keeps far below), TENO_ERANK, TENO_EARG (bad
 * parameters, or a mesh with n_cell * 4 ceil(rows / 4) >= 2^31 stencil rows,
 * about 28 million cells at order 6). */
int teno_mesh_setup(teno_mesh* m, const teno_params* p);

int teno_mesh_info(const teno_mesh* m, teno_info* out);

/* perm[internal] = user cell id (host int32[n_cell]). */
int teno_mesh_permutation(const teno_mesh* m, int32_t* perm);

/* Boundary faces, numbered b = 0 .. n_bface-1 (0 on a doubly periodic
 * mesh).  verts: host int32[n_bface][2], the user vertex ids of face b in
 * the counter-clockwise order of its cell; cell: host int32[n_bface] (nullable),
 * the user id of that cell. */
int teno_mesh_boundary_count(const teno_mesh* m, int32_t* n_bface);
int teno_mesh_boundary_faces(const teno_mesh* m, int32_t* verts, int32_t* cell);

/* Boundary condition of every boundary face: kind host int32[n_bface]
 * (teno_bc), state host double[n_bface][4] conservative (read for
 * TENO_BC_PRESCRIBED faces; NULL when there are none).  Takes effect for
 * solvers created afterwards. */
int teno_mesh_set_boundary(teno_mesh* m, const int32_t* kind, const double* state);

/* Members of stencil k (0..2 directional across local edge k, 3 = central)
 * of USER cell `cell`, as user ids nearest first, target excluded. Returns the
 * row count. */
int teno_mesh_stencil(const teno_mesh* m, int32_t cell, int32_t k, int32_t* members);

/* Least-squares operator of that stencil: coef = M (U_s - U_0) with
 * M = pinv(A) diag(|V'_s|), host double[n_coef][rows] row-major.
 * Returns the row count. */
int teno_mesh_lsq_operator(const teno_mesh* m, int32_t cell, int32_t k, double* M);

void teno_mesh_destroy(teno_mesh* m);

/* ---- solver: device data and per-stage work ---------------------------- */

/* Uploads mesh, stencil and matrix data to `device` and allocates all
 * workspaces; the only allocating call.  Requires teno_mesh_setup. */
int teno_solver_create(const teno_mesh* m, int32_t device, teno_solver** out);
void teno_solver_destroy(teno_solver* s);

/* Semi-discrete residual R(U) = dU/dt, Sec. 2.1 semi-discrete equation:
 * reconstruction with TENO selection (Sec. 2.2-3.3), rotated HLL flux at the
 * face Gauss points (Sec. 4), face-flux gather per cell.  flags (nullable):
 * output, bit 4v+3 = large stencil kept for variable v, bits 4v..4v+2 = small
 * stencil kept in the second selection step.  With characteristic != 0 the
 * flags are uint16_t[3][n_cell], word e for local edge e, v counting the
 * characteristic variables (speeds u.n - c, u.n entropy, u.n shear,
 * u.n + c). */
int teno_residual(teno_solver* s, const double* U, double* R, uint16_t* flags, void* stream);

/* Same residual with the selection frozen to `flags` (input). */
int teno_residual_frozen(teno_solver* s, const double* U, double* R, const uint16_t* flags,
                         void* stream);

/* Reconstruction only: face-point states of every cell, device
 * double[3*n_quad][n_cell][4] (point e*n_quad+kappa of local edge e, Gauss
 * point kappa along the edge from its first vertex), and flags (nullable). */
int teno_reconstruct(teno_solver* s, const double* U, double* face_states, uint16_t* flags,
                     void* stream);

/* dt = cfl * min_i |V_i| / sum_j |A_ij| (|u_i . n_ij| + c_i) from the cell
 * averages (constant-CFL step of Sec. 5), written to device *dt_dev. */
int teno_max_dt(teno_solver* s, const double* U, double cfl, double* dt_dev, void* stream);

/* One stage of SSP-RK3 (Sec. 2.1 time discretisation), k = 0, 1, 2:
 *   k=0: Uk1 = Un + dt R(Un)                      (Uk must equal Un)
 *   k=1: Uk1 = 3/4 Un + 1/4 Uk + 1/4 dt R(Uk)
 *   k=2: Uk1 = 1/3 Un + 2/3 Uk + 2/3 dt R(Uk)
 * Uk1 may alias Un (each cell reads only its own Un).  flags nullable (out),
 * or input when frozen != 0. */
int teno_rk_stage(teno_solver* s, int32_t k, const double* Un, const double* Uk, double* Uk1,
                  const double* dt_dev, uint16_t* flags, int32_t frozen, void* stream);

/* One full SSP-RK3 step in place on U using library-owned stage buffers.
 * flags3: nullable device uint16_t[3][n_cell] (out, or in when frozen != 0).
 * (uint16_t[3][3][n_cell] with characteristic != 0, output only.)
 * stages: nullable device double[3][n_cell][4], receives the stage inputs
 * U^n, U^(1), U^(2) (what the adjoint needs).
 * face_states3: nullable device double[3][face_state_doubles] (teno_info);
 * when given, each stage's face Gauss-point states are computed into it (in
 * the library's layout, opaque to the caller) and kept for
 * teno_vjp_rk_step. */
int teno_rk_step(teno_solver* s, double* U, const double* dt_dev, uint16_t* flags3,
                 int32_t frozen, double* stages, double* face_states3, void* stream);

/* teno_max_dt for callers that cannot allocate (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same dt,
 * bit for bit, but the per-block minima live in a static device array of
 * the library (65,536 doubles, one copy per GPU for the life of the
 * process) instead of the solver's workspace.  The call allocates nothing
 * and makes no allocating library call.  Meshes of more than 16,777,216
 * cells are refused (TENO_EARG).  Every call on one GPU shares that array:
 * calls that overlap on one GPU (other streams, other threads) race and
 * must be ordered by the caller.  The array's address on each GPU is taken
 * on the first call there. */
int teno_max_dt_static(teno_solver* s, const double* U, double cfl, double* dt_dev, void* stream);

/* One SSP-RK3 step in place on U (as teno_rk_step, unfrozen) that also
 * leaves the next step's constant-CFL dt (as teno_max_dt of the new U, bit
 * for bit) in dt_dev: the last stage's update kernel forms it from the
 * states it writes, so a loop of steps needs teno_max_dt only before its
 * first step.  dt_dev is the step's dt on entry and the next one on return;
 * flags3 nullable (out). */
int teno_rk_step_dt(teno_solver* s, double* U, double* dt_dev, double cfl, uint16_t* flags3,
                    void* stream);

/* Adjoint of the residual with the selection frozen to `flags`:
 * U_bar = (dR/dU)^T lam.  The reconstruction is linear in U for fixed
 * selection, so this is exact wherever the HLL flux is differentiable.  On
 * a mesh with boundary faces the outer states are differentiated through
 * their conditions (transmissive and reflective follow the inner state,
 * prescribed states are constants: the ones set when the call runs).
 * TENO_EARG for CWENO or characteristic variables (as for
 * teno_vjp_rk_step). */
int teno_vjp_residual(teno_solver* s, const double* U, const uint16_t* flags, const double* lam,
                      double* U_bar, void* stream);

/* Adjoint of one SSP-RK3 step (frozen dt and selection): given the stage
 * inputs (teno_rk_step's `stages`), their flags3 and lam_out = adjoint of
 * U^{n+1}, writes lam_in = adjoint of U^n.  lam_in may alias lam_out.
 * face_states3: nullable; the face states teno_rk_step kept for these
 * stages, which saves reconstructing them (same result either way). */
int teno_vjp_rk_step(teno_solver* s, const double* stages, const uint16_t* flags3,
                     const double* face_states3, const double* dt_dev, const double* lam_out,
                     double* lam_in, void* stream);

/* Replaces the prescribed boundary states (time-dependent inflow, e.g. the
 * moving shock of the double Mach reflection): state_dev device
 * double[n_bface][4], copied on `stream`; entries of faces of other kinds are
 * ignored. */
int teno_solver_set_boundary_states(teno_solver* s, const double* state_dev, void* stream);

/* Reads (and optionally resets) the device diagnostics; synchronises the
 * stream. */
int teno_diagnostics(teno_solver* s, teno_diag* out, int32_t reset, void* stream);

/* Kernel timing with HIP events around the launches of the selected kinds
 * (off by default).  kinds: bit k selects kind k (0 reconstruct, 1 flux +
 * update, 2 dt, 3 adjoint); 0 turns timing off, 15 times everything.
 * teno_profile_read returns, per kind, the summed milliseconds and launch
 * counts; synchronises. */
int teno_profile_enable(teno_solver* s, int32_t kinds);
int teno_profile_read(teno_solver* s, double* ms, int64_t* launches, int32_t reset);

/* ---- batch of independent meshes --------------------------------------- */

/* Schedule of a batch (teno_batch_set_tuning). */
typedef struct teno_batch_tuning {
  int32_t order_mode;    /* 0: one reconstruction launch per stage for every
                            order (dispatch per work item); 1: one launch per
                            order present, each with that order's registers */
  int32_t waves_per_cu;  /* persistent wavefronts per compute unit, 1..32;   */
                         /* 0: one wavefront per work item (no persistence)  */
  int32_t item_order;    /* 0: mesh order; 1: largest order first            */
  int32_t use_graph;     /* 1: capture one step as a HIP graph and replay it  */
} teno_batch_tuning;

/* Groups solvers created on the same device (meshes of any size and order,
 * each set up with its own parameters) so that one SSP-RK3 step of all of
 * them runs as persistent launches over a shared work list: per stage one
 * reconstruction launch (or one per order, see tuning) over (mesh, tile)
 * items and one flux/update launch over (mesh, 64-cell) items.  The solvers
 * must outlive the batch; their workspaces are reused.  Meshes with boundary
 * faces take their conditions and prescribed states from their solvers.
 * TENO_EARG for CWENO or characteristic variables. */
int teno_batch_create(teno_solver* const* solvers, int32_t n, teno_batch** out);

int teno_batch_set_tuning(teno_batch* b, const teno_batch_tuning* t);
int teno_batch_get_tuning(const teno_batch* b, teno_batch_tuning* t);

/* dt_dev[m] = CFL step of mesh m from U[m] (device double[n]); two launches.
 * Leaves a captured step graph in place. */
int teno_batch_max_dt(teno_batch* b, double* const* U, double cfl, double* dt_dev, void* stream);

/* One SSP-RK3 step of every mesh, in place on U[m] (device state of mesh m,
 * internal order), with step dt_dev[m].  The kernels take every pointer from
 * per-mesh device descriptors, which teno_batch_max_dt and teno_batch_rk_step
 * rewrite (a host-to-device copy and a wait on the stream) only when U,
 * dt_dev or the flag buffers differ from the last call.  With use_graph the
 * first call after teno_batch_create or teno_batch_set_tuning captures the
 * step as a HIP graph and every call replays it; a loop over the same
 * buffers makes no host wait per step. */
int teno_batch_rk_step(teno_batch* b, double* const* U, const double* dt_dev, void* stream);

/* Stage flags of the batched steps (Sec. 3.3 selection, encoded as for
 * teno_rk_step): flags3[m] is a device uint16_t[3][n_cell of mesh m] that
 * every later step overwrites with its three stages' flags; flags3 = NULL
 * stops writing them.  Host array of n pointers, copied. */
int teno_batch_set_flags(teno_batch* b, uint16_t* const* flags3);

/* Counters of the batch since teno_batch_create. */
typedef struct teno_batch_stats {
  int64_t captures;           /* step graphs captured and instantiated        */
  int64_t replays;            /* graph launches                               */
  int64_t descriptor_writes;  /* descriptor uploads (each waits on the stream) */
} teno_batch_stats;
int teno_batch_get_stats(const teno_batch* b, teno_batch_stats* out);

void teno_batch_destroy(teno_batch* b);

#ifdef __cplusplus
}
#endif
#endif /* TENO_H */
