/*
 * lbm3d.h -- C ABI of the D3Q19 step on gfx950: the method's time step
 * carried to three dimensions.
 *
 * The paper works in two dimensions and names three-dimensional flows as
 * the next step (Sec. 5).  The step here is the two-dimensional one of
 * Secs. 2.1-2.3 on 19 velocities:
 *   stream + collide          Sec. 2.1, Eqs. 1-4, BGK
 *   Zou & He faces            Sec. 2.2, Eqs. 5-11 carried to 3D: velocity
 *                             inlet u = (u_in, 0, 0) at x = 0, pressure
 *                             outlet rho = rho_out with zero transverse
 *                             velocity at x = nx-1; each unknown is the
 *                             opposite population plus the equilibrium
 *                             difference, and the unknowns with a transverse
 *                             component are corrected so that the node
 *                             carries exactly the prescribed transverse
 *                             momentum (the construction of Hecht & Harting
 *                             2010, which reduces to Eqs. 8-10 in 2D)
 *   bounce-back on solids     Sec. 2.3, Eq. 12, half-way
 *   momentum-exchange force   Sec. 2.3, Eqs. 14-15, FP64 sums per step
 *
 * Conventions
 *   - Numbering q: 0 rest; 1-6 = +x, -x, +y, -y, +z, -z; 7-18 the edges
 *     (1,1,0) (-1,-1,0) (1,-1,0) (-1,1,0) (1,0,1) (-1,0,-1) (1,0,-1)
 *     (-1,0,1) (0,1,1) (0,-1,-1) (0,1,-1) (0,-1,1), opposite pairs
 *     (2k+1, 2k+2); weights 1/3, 1/18, 1/36.
 *   - Host arrays are [q][z][y][x] (x fastest); scalar fields [z][y][x];
 *     velocity fields [3][z][y][x].
 *   - Mask: 0 fluid, 1 body (links to it are force-summed); solid nodes are
 *     never updated.  With LBM_X_INOUT the planes x = 0 and x = nx-1 must
 *     be fluid.
 *   - Lattice units dx = dt = 1, c_s^2 = 1/3, tau = 3 nu + 1/2.
 *   - Status codes, lbm_last_error(), the caller-owned 256-byte aligned
 *     workspace and the asynchronous stream semantics are those of lbm.h.
 *   - Arithmetic: LBM_FP64 (offsets f - w in double) or LBM_FP32_OFFSET
 *     (offsets in float); the force sums are FP64 in a fixed order.
 */
#ifndef LBM3D_H
#define LBM3D_H

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm3d_ctx lbm3d_ctx;

typedef struct {
  int32_t nx, ny, nz;          /* lattice size, each >= 4 (nx*ny*nz < 2^31)     */
  int32_t precision;           /* LBM_FP64 or LBM_FP32_OFFSET                    */
  int32_t lateral_y;           /* LBM_LATERAL_WALLS or LBM_LATERAL_PERIODIC      */
  int32_t lateral_z;           /* the same for z                                 */
  int32_t xbc;                 /* LBM_X_INOUT or LBM_X_PERIODIC                  */
  int32_t reserved;            /* 0                                              */
  double tau;                  /* BGK relaxation time, > 1/2                     */
  double u_in;                 /* inlet velocity, |u_in| < 0.5                   */
  double rho_out;              /* outlet density, > 0                            */
  int64_t history_cap;         /* steps of force history kept on the device      */
  void* stream;                /* hipStream_t, borrowed                          */
} lbm3d_params;

typedef struct {
  double fx, fy, fz;           /* force on the body at the last step             */
  double dmass;                /* sum of rho - 1 over the fluid nodes            */
  int64_t step;                /* steps taken                                    */
  int32_t nonfinite;           /* 1 if a non-finite value appeared               */
  int32_t reserved;
} lbm3d_force_out;

size_t lbm3d_workspace_bytes(const lbm3d_params* p);

lbm_status lbm3d_create(const lbm3d_params* p, void* dev_workspace, size_t bytes,
                        lbm3d_ctx** out);
/* Wait for the context's stream, then release the context (not the
 * workspace).  NULL is a no-op. */
lbm_status lbm3d_destroy(lbm3d_ctx* c);

/* Geometry (host nz*ny*nx bytes, copied) and the initial state
 * f = f^eq(1, (u_in, 0, 0)) on fluid nodes, f^eq(1, 0) on solid ones; resets
 * the step count and the history (synchronises). */
lbm_status lbm3d_set_geometry(lbm3d_ctx* c, const uint8_t* host_mask);

/* State f = f^eq(rho, u) on fluid nodes from host FP64 fields rho [z][y][x]
 * and u [3][z][y][x] (synchronises). */
lbm_status lbm3d_init_fields(lbm3d_ctx* c, const double* rho, const double* u);

/* Advance nsteps steps (asynchronous). */
lbm_status lbm3d_step(lbm3d_ctx* c, int64_t nsteps);

/* Synchronise and read the last step's force, mass defect and flags. */
lbm_status lbm3d_forces(lbm3d_ctx* c, lbm3d_force_out* out);

/* Synchronise and copy up to cap steps of force history (oldest first) into
 * fx, fy, fz; *n receives the number copied. */
lbm_status lbm3d_force_history(lbm3d_ctx* c, double* fx, double* fy, double* fz, int64_t cap,
                               int64_t* n);

/* Synchronise and copy the post-collision state (absolute f, 19*nz*ny*nx
 * doubles) to host; solid nodes hold their initial equilibrium. */
lbm_status lbm3d_read_populations(lbm3d_ctx* c, double* host);

/* Replace the post-collision state by host (absolute f, 19*nz*ny*nx
 * doubles), rounded to the storage precision (synchronises). */
lbm_status lbm3d_write_populations(lbm3d_ctx* c, const double* host);

lbm_status lbm3d_sync(lbm3d_ctx* c);

#ifdef __cplusplus
}
#endif

#endif /* LBM3D_H */
