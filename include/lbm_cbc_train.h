/*
 * lbm_cbc_train.h -- closed-loop training of the tuning network of the
 * characteristic outflow on the GPU (C ABI).
 *
 * Sec. 4.2 of Bedrunka et al.: the network that sets sigma and kappa_2 of
 * the characteristic outflow (Eqs. 27-28) per outlet node is trained through
 * the solver.  A segment starts from a state of the reflection-free reference
 * run, advances n_t steps on the truncated lattice with the network in the
 * loop, and is scored at step n_t by
 *     loss_s = mean_Omega (rho - rho_ref)^2 + mean_Omega |U - U_ref|^2
 * over the n_t columns next to the outlet, Omega = {nx - n_t <= x <= nx-1}
 * (the section's n_t layers; its strict bound at the outlet would leave
 * n_t - 1), every row; a step of the optimiser minimises the mean of loss_s
 * over all segments held, with the exact gradient of the rollout (reverse
 * mode, adjoint kernels written out for every part of the step) and Adam
 * (Kingma & Ba 2015).
 *
 * The step inside a segment is the library's: BGK collision (Eq. 2), pull
 * streaming (Eq. 1) with periodic rows, and the characteristic outlet with
 * the network (Eqs. 18-29 as in lbm_set_outflow_cbc, previous time
 * derivatives zero at the start of the segment).  The segment lattice has no
 * solid nodes.  A segment's loss depends only on the last 2 n_t + 3 columns
 * of its start state (a disturbance travels one column per step, so nothing
 * further upstream reaches Omega within n_t steps, nor the three columns the
 * outlet reads): the trainer advances that strip alone, W = 2 n_max + 3
 * columns wide, and fills the populations that would enter its left edge
 * from upstream with copies of the edge column (they never reach Omega).
 * The caller hands over the strip, which must not contain the inlet.
 *
 * Arithmetic in the precision chosen (populations stored as offsets f - w
 * in FP64 or FP32), network weights held as FP32 masters (the form the
 * step reads), gradients summed over each block of 64 outlet rows in the
 * precision chosen and over the blocks in FP64, all in a fixed order: runs
 * are reproducible.  Memory: the whole trajectory of every segment is kept,
 * about (n_max + 3) * 9 * ny * W * n_seg values of the precision.
 *
 * Conventions as in lbm.h: asynchronous on the given stream unless a
 * comment says it synchronises, caller-owned workspace, status codes and
 * lbm_last_error().  The backward outlet kernels run on a second stream
 * that the trainer creates on its first gradient or step (on the device
 * current then) and joins back into the given stream before the call's
 * work ends there; lbm_cbc_train_destroy waits for it and releases it.
 */
#ifndef LBM_CBC_TRAIN_H
#define LBM_CBC_TRAIN_H

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Parameters of the 9-20-20-2 tuning network in the order of the gradient
 * and weight arrays: w1 [20][9], b1 [20], w2 [20][20], b2 [20], w3 [2][20],
 * b3 [2], row-major [out][in]. */
#define LBM_CBC_NPARAMS 662

/* The same trainer drives the outflow reconstruction of Eq. 16 (Sec. 3.1)
 * instead when its network is set with lbm_cbc_train_set_nn: at every
 * outlet row the unknowns are g_i = f_i(L-1) + s_i, i = 3, 6, 7, where
 * f(L-1) are the streamed populations of column L-1 and s = o sd_out +
 * mu_out, o the 9-20-20-3 network (tanh hidden layers, linear output) of
 * the standardised pre-collision offsets f - w of column L-1, z = (f - w -
 * mu_in) / sd_in; the outlet node then collides like every other (no
 * fallback inside a segment: the fallback is a selection, not a function
 * the training differentiates).  Parameters in the order of the gradient
 * and weight arrays: w1 [20][9], b1 [20], w2 [20][20], b2 [20], w3 [3][20],
 * b3 [3], row-major [out][in]. */
#define LBM_NN9_NPARAMS 683

typedef struct {
  const float* w1;      /* [20][9]  */
  const float* b1;      /* [20]     */
  const float* w2;      /* [20][20] */
  const float* b2;      /* [20]     */
  const float* w3;      /* [3][20]  */
  const float* b3;      /* [3]      */
  float mu_in[9], sd_in[9];     /* input standardisation, sd > 0  */
  float mu_out[3], sd_out[3];   /* output map, sd_out > 0         */
} lbm_nn9_net;

typedef struct lbm_cbc_trainer lbm_cbc_trainer;

typedef struct {
  int32_t ny;           /* rows of the lattice (periodic), >= 3               */
  int32_t n_max;        /* longest segment, 1 .. 64; strip W = 2 n_max + 3    */
  int32_t n_seg;        /* segments held, 1 .. 65535                          */
  int32_t precision;    /* LBM_FP64 or LBM_FP32_OFFSET                        */
  double tau;           /* BGK relaxation time, > 1/2                         */
  double mach;          /* M of Eq. 28, 0 <= M < 1                            */
  double length;        /* L of Eq. 28 (the truncated lattice length), > 0    */
  double rho_inf;       /* far-field density, > 0                             */
  double lr, beta1, beta2, eps;   /* Adam: lr > 0, 0 <= beta < 1, eps > 0     */
  void* stream;         /* hipStream_t, borrowed                              */
} lbm_cbc_train_params;

size_t lbm_cbc_train_workspace_bytes(const lbm_cbc_train_params* p);

lbm_status lbm_cbc_train_create(const lbm_cbc_train_params* p, void* dev_workspace,
                                size_t bytes, lbm_cbc_trainer** out);
lbm_status lbm_cbc_train_destroy(lbm_cbc_trainer* t);

/* Segment data, host FP64 arrays, copied (synchronises):
 *   a0   [n_seg][9][ny][W]  post-collision populations (absolute values) of
 *                           the last W = 2 n_max + 3 columns at the start;
 *   ref  [n_seg][3][ny][n_max]  reference rho, u, v at step n_t(s): entry
 *                           n_max - n_t(s) + j holds column nx - n_t(s) + j
 *                           (j < n_t(s)); the other entries are ignored;
 *   n_t  [n_seg]            steps of each segment, 1 .. n_max. */
lbm_status lbm_cbc_train_set_segments(lbm_cbc_trainer* t, const double* a0, const double* ref,
                                      const int32_t* n_t);

/* Per-segment relaxation time and Mach number (host arrays of n_seg doubles,
 * copied; NULL keeps the trainer's tau or mach for every segment), so that
 * one training set can span several flows; tau > 1/2, 0 <= mach < 1.
 * lbm_cbc_train_set_segments resets both to the trainer's values.
 * Synchronises. */
lbm_status lbm_cbc_train_set_segment_params(lbm_cbc_trainer* t, const double* tau,
                                            const double* mach);

/* The network: weights become the FP32 masters, standardisation and output
 * maps are kept fixed (as in lbm_cbc_net); resets Adam.  The segments then
 * run the characteristic outlet. */
lbm_status lbm_cbc_train_set_net(lbm_cbc_trainer* t, const lbm_cbc_net* net);

/* The Eq. 16 network (host arrays, copied; synchronises): weights become
 * the FP32 masters, the standardisation and output map stay fixed; resets
 * Adam.  The segments then run the Eq. 16 outlet (mach, length and rho_inf
 * of the parameters are not used).  Gradients and weights then have
 * LBM_NN9_NPARAMS entries.  EINVAL for a NULL or non-finite argument or an
 * sd that is not positive. */
lbm_status lbm_cbc_train_set_nn(lbm_cbc_trainer* t, const lbm_nn9_net* net);

/* Loss and gradient of the current weights over every segment, without an
 * update (synchronises).  grad: host array of LBM_CBC_NPARAMS doubles
 * (LBM_NN9_NPARAMS with the Eq. 16 network), or NULL. */
lbm_status lbm_cbc_train_gradient(lbm_cbc_trainer* t, double* loss, double* grad);

/* nsteps optimiser steps, each on the full set of segments (asynchronous). */
lbm_status lbm_cbc_train_step(lbm_cbc_trainer* t, int64_t nsteps);

/* Synchronise; the loss of the weights before the last step's update. */
lbm_status lbm_cbc_train_loss(lbm_cbc_trainer* t, double* loss);

/* Synchronise and copy the FP32 master weights (LBM_CBC_NPARAMS floats;
 * LBM_NN9_NPARAMS with the Eq. 16 network). */
lbm_status lbm_cbc_train_get_weights(lbm_cbc_trainer* t, float* theta);

/* Synchronise and copy segment seg's state at its step n_t of the last
 * forward pass (absolute post-collision populations, [9][ny][W] doubles). */
lbm_status lbm_cbc_train_final_state(lbm_cbc_trainer* t, int32_t seg, double* host);

#ifdef __cplusplus
}
#endif

#endif /* LBM_CBC_TRAIN_H */
