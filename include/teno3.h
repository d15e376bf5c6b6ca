/*
 * teno3.h -- C ABI of the tetrahedral path of libteno: the per-cell,
 * per-Runge-Kutta-stage TENO residual of the 3D Euler equations on
 * tetrahedral meshes (Ji, Liang & Fu, "A class of new high-order
 * finite-volume TENO schemes for hyperbolic conservation laws with
 * unstructured meshes": Sec. 2-4 written in (xi, eta, zeta); Sec. 5.9 runs
 * the scheme on a tetrahedral mesh), in FP64, on AMD Instinct MI355X.
 *
 * Conventions as in teno.h (status codes, teno_last_error, caller streams,
 * no allocation in per-step calls), with five conservative variables:
 * state arrays are caller-owned DEVICE pointers to double[n_cell][5] =
 * (rho, rho u, rho v, rho w, E) in the library's INTERNAL cell order
 * (teno3_mesh_permutation).  Flags are device uint32_t[n_cell]: for
 * variable v, bit 5v+4 = large stencil kept (Sec. 3.3 step i), bits
 * 5v..5v+3 = small directional stencil k (through local face k) kept in
 * step ii.
 *
 * Readings where the paper is silent: local face e of a tetrahedron is the
 * face opposite vertex e; stencils as in 2D with cones through the three
 * vertices of a face (K = 4 small stencils of 19 rows, degree 2); face
 * quadrature by symmetric triangle rules (6 points of degree 4 at orders
 * 3-4, 7 of degree 5 at orders 5-6); each boundary face is transmissive or
 * reflective.  TENO and LINEAR only (no CWENO, characteristic variables,
 * adjoint or batches on tetrahedra).
 */
#ifndef TENO3_H
#define TENO3_H

#include <stdint.h>

#include "teno.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct teno3_mesh teno3_mesh;
typedef struct teno3_solver teno3_solver;

/* Geometry and faces (Sec. 2.1).  xyz: host double[n_vert][3]; tet: host
 * int32[n_cell][4] (orientation fixed internally by swapping the last two
 * vertices); period: host double[3], the period of each axis or 0 for an
 * open axis (NULL opens all).  With an open axis a triangle with one cell is
 * a boundary face, transmissive until teno3_mesh_set_boundary. */
int teno3_mesh_create(int32_t n_vert, const double* xyz, int32_t n_cell, const int32_t* tet,
                      const double* period, teno3_mesh** out);

/* Boundary faces b = 0 .. n_bface-1 in the order of their sorted vertex
 * triples: verts host int32[n_bface][3] (user vertex ids in the cell's local
 * face order), cell host int32[n_bface] (nullable). */
int teno3_mesh_boundary_count(const teno3_mesh* m, int32_t* n_bface);
int teno3_mesh_boundary_faces(const teno3_mesh* m, int32_t* verts, int32_t* cell);

/* kind: host int32[n_bface], TENO_BC_TRANSMISSIVE or TENO_BC_REFLECTIVE;
 * takes effect for solvers created afterwards. */
int teno3_mesh_set_boundary(teno3_mesh* m, const int32_t* kind);

/* Stencils, least-squares pseudo-inverses (Sec. 2.2 eqs. 02-10 with n_d = 3),
 * cell reordering and packing.  Uses order, variant (0 TENO, 1 LINEAR), ct
 * (in [0, 1/4]), eps, power, gamma, tie_rel, fallback, reorder, n_threads of
 * teno_params.  Errors: TENO_ESTENCIL, TENO_ERANK, TENO_EARG. */
int teno3_mesh_setup(teno3_mesh* m, const teno_params* p);

/* n_cell, n_face, order, n_quad (= face points), n_coef_large, rows_large,
 * n_coef_small (9), rows_small (19), matrix_doubles_per_cell, min_rcond,
 * face_state_doubles, n_bface. */
int teno3_mesh_info(const teno3_mesh* m, teno_info* out);

/* perm[internal] = user cell id (host int32[n_cell]). */
int teno3_mesh_permutation(const teno3_mesh* m, int32_t* perm);

/* Members of stencil k (0..3 directional through local face k, 4 = central)
 * of USER cell `cell`, user ids nearest first; returns the row count. */
int teno3_mesh_stencil(const teno3_mesh* m, int32_t cell, int32_t k, int32_t* members);

/* Its operator coef = M (U_s - U_0), M = pinv(A) diag(|V'_s|): host
 * double[n_coef][rows] row-major; returns the row count. */
int teno3_mesh_lsq_operator(const teno3_mesh* m, int32_t cell, int32_t k, double* M);

void teno3_mesh_destroy(teno3_mesh* m);

/* Uploads mesh, stencil and operator data to `device` and allocates all
 * workspaces (the only allocating call). */
int teno3_solver_create(const teno3_mesh* m, int32_t device, teno3_solver** out);
void teno3_solver_destroy(teno3_solver* s);

/* Face-point states of every cell: device double[4 n_pt][n_cell][5] (point
 * e n_pt + k of local face e, rule point k in the cell's face order), and
 * flags (nullable, out). */
int teno3_reconstruct(teno3_solver* s, const double* U, double* face_states, uint32_t* flags,
                      void* stream);

/* R(U) = dU/dt (Sec. 2.1): reconstruction with TENO selection, HLL fluxes
 * at the face points, face-flux gather; flags nullable (out). */
int teno3_residual(teno3_solver* s, const double* U, double* R, uint32_t* flags, void* stream);

/* dt = cfl * min_i |V_i| / sum_f |A_if| (|u_i . n_if| + c_i) into device *dt_dev. */
int teno3_max_dt(teno3_solver* s, const double* U, double cfl, double* dt_dev, void* stream);

/* SSP-RK3 stage k (as teno_rk_stage) and a full step in place on U with
 * library stage buffers; flags (nullable, out) uint32_t[n_cell] per stage,
 * flags3 uint32_t[3][n_cell]. */
int teno3_rk_stage(teno3_solver* s, int32_t k, const double* Un, const double* Uk, double* Uk1,
                   const double* dt_dev, uint32_t* flags, void* stream);
int teno3_rk_step(teno3_solver* s, double* U, const double* dt_dev, uint32_t* flags3,
                  void* stream);

/* Device diagnostics (non-physical states, near ties, fallbacks);
 * synchronises the stream. */
int teno3_diagnostics(teno3_solver* s, teno_diag* out, int32_t reset, void* stream);

/* Kernel timing with HIP events (kinds: bit 0 reconstruct, 1 flux + update,
 * 2 dt); read returns summed milliseconds and launch counts per kind. */
int teno3_profile_enable(teno3_solver* s, int32_t kinds);
int teno3_profile_read(teno3_solver* s, double* ms, int64_t* launches, int32_t reset);

#ifdef __cplusplus
}
#endif
#endif /* TENO3_H */
