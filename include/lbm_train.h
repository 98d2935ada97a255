/*
 * lbm_train.h -- training of the outflow MLP on the GPU (C ABI).
 *
 * Sec. 3.1 of Bedrunka et al.: the network that reconstructs the unknown
 * outlet populations, f_i^B(L) = f_i(L-1) + s_i (Eq. 16), is fitted by the
 * mean squared error between reconstructed and reference populations
 * (Eq. 17).  Here the samples are
 *   x [n][27]  population offsets f - w at x = L-1, L-2, L-3 of one row
 *              (feature k = 9 j + q for column L-1-j), FP32, device memory;
 *   t [n][3]   the corrections f_ref(L) - f(L-1) of populations 3, 6, 7,
 *              FP32, device memory;
 * inputs and targets are standardised per column with the data's mean and
 * standard deviation, and the loss is the mean over the batch and the three
 * outputs of (o - (t - mu_out)/sd_out)^2, o the network output.  Since
 * s = o sd_out + mu_out, this is Eq. 17 up to the per-output factor sd_out^2.
 *
 * Arithmetic: BF16 operands with FP32 accumulation (MFMA 16x16x32) for every
 * matrix product of the forward and backward passes, tanh and elementwise
 * work in FP32, FP32 master weights and Adam moments (Kingma & Ba 2015),
 * per-batch gradient sums in FP64 in a fixed order (runs are reproducible).
 * Batches are drawn on the device: sample j of step s is row
 * ((r >> 32) * n) >> 32 of the data, r the SplitMix64 output
 * k = s * batch + j + 1 of the stream seeded with `seed`.
 *
 * Conventions as in lbm.h: asynchronous on the given stream, caller-owned
 * workspace, status codes and lbm_last_error().
 */
#ifndef LBM_TRAIN_H
#define LBM_TRAIN_H

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_trainer lbm_trainer;

typedef struct {
  int32_t batch;        /* samples per step: a multiple of 64, 64 .. 65536      */
  double lr, beta1, beta2, eps;   /* Adam                                       */
  uint64_t seed;        /* SplitMix64 seed of the batch sampling               */
  void* stream;         /* hipStream_t, borrowed                               */
} lbm_train_params;

/* Host-side weights, FP32 row-major [out][in] (as in lbm_mlp). */
typedef struct {
  float *w1, *b1, *w2, *b2, *w3, *b3;          /* 64x27, 64, 64x64, 64, 3x64, 3 */
  float *mu_in, *sd_in, *mu_out, *sd_out;      /* 27, 27, 3, 3                  */
} lbm_mlp_host;

size_t lbm_train_workspace_bytes(const lbm_train_params* p);

lbm_status lbm_train_create(const lbm_train_params* p, void* dev_workspace, size_t bytes,
                            lbm_trainer** out);
/* Wait for the trainer's stream, then release it (not the workspace).  NULL
 * is a no-op. */
lbm_status lbm_train_destroy(lbm_trainer* t);

/* Attach the data (device pointers, kept by reference: they must stay valid
 * while the trainer uses them) and compute the standardisation of every
 * input and target column on the device (mean and standard deviation over
 * all n samples, FP64, fixed order).  n >= 2. */
lbm_status lbm_train_set_data(lbm_trainer* t, const float* dev_x, const float* dev_t,
                              int64_t n);

/* Set the FP32 master weights (host arrays; w->mu_* / sd_* are ignored: the
 * standardisation comes from the data) and reset the Adam moments. */
lbm_status lbm_train_set_weights(lbm_trainer* t, const lbm_mlp* w);

/* Advance nsteps optimiser steps (asynchronous). */
lbm_status lbm_train_step(lbm_trainer* t, int64_t nsteps);

/* Synchronise and read the mean loss of the last step. */
lbm_status lbm_train_loss(lbm_trainer* t, double* loss);

/* Synchronise and copy the FP32 master weights and the standardisation
 * into caller arrays (sizes as in lbm_mlp_host). */
lbm_status lbm_train_get_weights(lbm_trainer* t, const lbm_mlp_host* out);

/* Loss and gradients of the current weights on the batch of given rows
 * (dev_rows: n_rows int32 indices in device memory, n_rows a multiple of
 * 64), without an update.  grad receives the 6147 gradients on the host in
 * the order w1, b1, w2, b2, w3, b3 (row-major). */
lbm_status lbm_train_gradient(lbm_trainer* t, const int32_t* dev_rows, int32_t n_rows,
                              float* grad, double* loss);

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc -- the loss and
 * gradient of lbm_train_gradient without a trainer or a workspace: the
 * network *w (27-64-64-3, FP32 host arrays; its mu_in, sd_in, mu_out,
 * sd_out are the standardisation, z = (x - mu) * (1/sd) in FP32) on the
 * samples dev_x [.][27], dev_t [.][3] (device FP32) at the n_rows rows
 * dev_rows (device int32, each a valid sample index), n_rows a multiple of
 * 64 and at most 4096.  Same kernels and summation order as
 * lbm_train_gradient: with the trainer's weights and standardisation (as
 * lbm_train_get_weights returns them) the results are identical.  grad
 * receives the 6147 gradients on the host (order of lbm_train_gradient),
 * loss the mean loss; the call synchronises the stream (hipStream_t).
 * It allocates nothing: its state, per-tile partial sums and summed
 * gradient live in a 2 MiB static device array that each GPU holds for the
 * life of the process (its address is looked up on the first call on that
 * device) and that every call on that GPU reuses, so calls that overlap on
 * one GPU (other threads, other streams) race and must be serialised by
 * the caller.  EINVAL for a bad network or n_rows beyond 4096; EHIP if the
 * symbol lookup or a launch fails. */
lbm_status lbm_mlp_gradient_noalloc(const lbm_mlp* w, const float* dev_x, const float* dev_t,
                                    const int32_t* dev_rows, int32_t n_rows, float* grad,
                                    double* loss, void* stream);

/* The rows the sampler draws for optimiser step `step` (host array of
 * `batch` int32). */
lbm_status lbm_train_sample_rows(lbm_trainer* t, int64_t step, int32_t* rows);

#ifdef __cplusplus
}
#endif

#endif /* LBM_TRAIN_H */
