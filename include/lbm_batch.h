/*
 * lbm_batch.h -- many uneven D2Q9 lattices advanced together, one launch per
 * step or one persistent launch (C ABI).  Used to generate the training data
 * of the outflow network.
 *
 * Every lattice takes exactly the single-lattice step of lbm.h (Sec. 2.1
 * Eqs. 1-4, Zou & He columns of Sec. 2.2, half-way bounce-back of Sec. 2.3,
 * momentum exchange of Eqs. 14-15) with FP32 offset storage and a Zou & He
 * pressure outlet: a lattice of a batch evolves bit for bit like the same
 * lattice stepped alone with LBM_FP32_OFFSET.  All lattices of a batch share
 * the collision operator and the lateral condition; size, geometry, tau,
 * inlet velocity and noise seed are per lattice.
 *
 * In the persistent mode one call of lbm_batch_step runs a cooperative
 * (co-resident) grid whose waves stride over the rows of all lattices (64
 * columns at a time) and separates time steps with a grid-wide barrier.
 * The barrier's wait is bounded: if it does not complete within the spin
 * limit the kernel stops and the next synchronising call returns LBM_EHIP.
 * In the per-step mode every step is a launch of its own (see
 * LBM_BATCH_PER_STEP below).
 *
 * Logging (Sec. 3.1: interior populations as network inputs, the next
 * column as ground truth).  A lattice with log_role 1 ("source") writes, at
 * every logging step, for each row y: the pre-collision population offsets
 * f - w of columns log_x-1, log_x-2, log_x-3 into x[s][9 j + q]
 * (j = log_x-1-column), and the corrections f(log_x) - f(log_x-1) of
 * populations 3, 6, 7 into t[s][0..2].  A lattice with log_role 2
 * ("ablation") writes its columns log_x-1 .. log_x-3 into x_ablation[s].
 * Sample s = slot * log_rows + log_row0 + y.  Logging steps are the steps
 * taken when log_start + k log_every steps have been taken before them,
 * k = 0 .. log_slots-1.
 *
 * Conventions as in lbm.h: caller-owned workspace and stream, host arrays
 * copied, status codes and lbm_last_error().
 */
#ifndef LBM_BATCH_H
#define LBM_BATCH_H

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_batch lbm_batch;

typedef struct {
  int32_t nx, ny;          /* >= 8 each                                         */
  double tau;              /* > 0.5                                            */
  double u_in, rho_out;    /* Zou & He inlet velocity and outlet density        */
  const uint8_t* mask;     /* host ny*nx: 0 fluid, 1 body, 2 inert solid;
                              columns 0 and nx-1 fluid                          */
  uint64_t seed;           /* SplitMix64 seed of the initial velocity noise     */
  int32_t log_role;        /* 0 none, 1 source, 2 ablation                      */
  int32_t log_x;           /* logged column (4 <= log_x <= nx-1 for role 1,
                              3 <= log_x <= nx-1 for role 2)                    */
  int32_t log_row0;        /* first sample row of this lattice in a slot        */
  int32_t reserved;
} lbm_batch_lattice;

typedef struct {
  int32_t collision, lateral;   /* LBM_BGK / LBM_MRT, LBM_LATERAL_*             */
  double s_e, s_eps, s_q;       /* MRT rates; s_q <= 0: the Lambda = 3/16 value
                                   of each lattice's tau                        */
  double noise_amp;             /* initial velocity noise amplitude             */
  int64_t history_cap;          /* force history kept per lattice               */
  int64_t log_start, log_every, log_slots;
  int32_t log_rows;             /* sample rows per logging slot                  */
  int32_t spin_limit;           /* barrier wait bound in polls; 0: default      */
  int32_t launch;               /* LBM_BATCH_PER_STEP (0) or LBM_BATCH_PERSISTENT */
  int32_t groups_per_cu;        /* persistent grid: workgroups per CU (0: 4);
                                   EINVAL if more than the kernel's resources
                                   let one CU hold at once                      */
  void* stream;                 /* hipStream_t, borrowed                        */
} lbm_batch_params;

/* Launch modes.  PER_STEP (the default): one launch per step (the kernel
 * boundary separates the steps; every wave takes one row item and each
 * launch first sums the previous step's partials), then one launch that
 * sums the last step's.  PERSISTENT: one cooperative launch per
 * lbm_batch_step call, steps separated by the grid barrier.  Both run the
 * same node code: the results are identical bit for bit. */
enum { LBM_BATCH_PER_STEP = 0, LBM_BATCH_PERSISTENT = 1 };

size_t lbm_batch_workspace_bytes(const lbm_batch_params* p, const lbm_batch_lattice* lat,
                                 int32_t n);

/* Create the batch, upload every geometry and initialise every lattice as
 * lbm_set_geometry does (f^eq(1, (u_in, 0) + noise)). */
lbm_status lbm_batch_create(const lbm_batch_params* p, const lbm_batch_lattice* lat, int32_t n,
                            void* dev_workspace, size_t bytes, lbm_batch** out);
/* Wait for the batch's stream (a persistent launch included), then release
 * the batch (not the workspace).  NULL is a no-op. */
lbm_status lbm_batch_destroy(lbm_batch* b);

/* Advance every live lattice by nsteps (one cooperative launch, or one
 * launch per step, as params.launch selects). */
lbm_status lbm_batch_step(lbm_batch* b, int64_t nsteps);

/* Per-lattice read-outs (synchronising), as lbm_forces, lbm_force_history
 * and lbm_read_populations. */
lbm_status lbm_batch_forces(lbm_batch* b, int32_t lattice, lbm_force_out* out);
lbm_status lbm_batch_force_history(lbm_batch* b, int32_t lattice, double* fx, double* fy,
                                   int64_t cap, int64_t* n);
lbm_status lbm_batch_read_populations(lbm_batch* b, int32_t lattice, double* host);

/* 1 for every lattice retired after a non-finite force or mass (its later
 * steps and samples are void), else 0; host array of n int32. */
lbm_status lbm_batch_retired(lbm_batch* b, int32_t* flags);

/* Device pointers of the data set (synchronising): x and x_ablation
 * [n][27], t [n][3] FP32, n = slots logged so far * log_rows.  The
 * pointers stay valid until lbm_batch_destroy. */
lbm_status lbm_batch_dataset(lbm_batch* b, const float** x, const float** x_ablation,
                             const float** t, int64_t* n);

#ifdef __cplusplus
}
#endif

#endif /* LBM_BATCH_H */
