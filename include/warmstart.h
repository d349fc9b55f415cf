/*
 * warmstart.h -- learned initial guess for the per-step GMRES solve of the theta-L
 * Hele-Shaw evolution (thetal.h).  An addition to the method of the paper: the GMRES
 * answer does not depend on it (every solve still runs to the same FP64 residual
 * tolerance); it only changes the number of iterations.
 *
 * Features per marker k of the state at step n (Sec. 5 variables):
 *     eta_k, L / L_ref, theta_a,k (= kappa_k L / 2pi), phi1_k / s1, (phi1_k - phi2_k) / s2
 * with phi1, phi2 the densities of the two previous solves, s1 = RMS(phi1) and
 * s2 = RMS(phi1 - phi2).
 * Network: circular 1-D convolutions with 5 taps (tap t reads marker k + t - 2 mod M),
 * widths 5 -> 64 -> 64 -> 64 -> 1, SiLU after the first three layers.
 * Initial guess: x0 = 2 phi1 - phi2 + s2 sigma net(features), i.e. the network corrects
 * the linear extrapolation of the density; sigma is a fixed target scale.  Before two
 * previous solves exist x0 = phi1; a non-finite prediction (or s2 = 0) also gives phi1.
 * Training target: (phi_n - 2 phi1 + phi2) / (s2 sigma), mean squared error, Adam.
 *
 * Arithmetic: activations and weights in bfloat16, accumulation in FP32 (the two 64 -> 64
 * layers on MFMA matrix cores); FP32 master weights, gradients and Adam moments; the
 * guess is assembled in FP64.
 *
 * Parameter vector (FP32, this order; weights indexed [out channel][tap][in channel]):
 *   W1 64x5x5, b1 64, W2 64x5x64, b2 64, W3 64x5x64, b3 64, W4 1x5x64, b4 1  (43073 values)
 *
 * Conventions as in kfbi.h (device pointers *_dev, host structs, KFBI_* status codes).
 */
#ifndef WARMSTART_H
#define WARMSTART_H

#include "thetal.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct kfbi_ws kfbi_ws;

typedef struct {
  int M;                      /* markers (as the thetaL object it serves)             */
  int max_batch;              /* largest training / forward batch, >= 1               */
  int capacity;               /* samples the training set can hold, >= 1              */
  double L_ref;               /* length scale of the L feature (> 0)                  */
  float lr, beta1, beta2, eps;  /* Adam                                               */
  unsigned long long seed;    /* weight initialisation and shuffling                  */
  double target_scale;        /* sigma; 0 = the RMS of the stored targets at the first
                                 kfbi_ws_train call (then kept)                        */
  void* stream;               /* hipStream_t (NULL = default stream)                  */
} kfbi_ws_cfg;

int kfbi_ws_create(const kfbi_ws_cfg* cfg, kfbi_ws** out);
int kfbi_ws_destroy(kfbi_ws* ws);

/* Number of parameters (43073). */
int kfbi_ws_n_params(const kfbi_ws* ws, int* n);
/* FP32 master weights to / from a HOST array of n_params floats.  Setting the weights
 * resets the Adam moments.  Synchronises. */
int kfbi_ws_get_weights(const kfbi_ws* ws, float* params_host);
int kfbi_ws_set_weights(kfbi_ws* ws, const float* params_host);

/* Initial guess x0_dev [M] (FP64) for the next thetaL_step of th; also keeps the features
 * of this state as a pending training sample.  Asynchronous. */
int kfbi_ws_predict(kfbi_ws* ws, thetaL* th, double* x0_dev);
/* After thetaL_step: completes the pending sample with the target from the new density
 * and appends it to the training set (no-op if the state had fewer than two previous
 * solves, or the set is full).  *stored (nullable) = 1 if a sample was stored. */
int kfbi_ws_record(kfbi_ws* ws, thetaL* th, int* stored);
int kfbi_ws_n_samples(const kfbi_ws* ws, int* n);
/* Forget the stored samples. */
int kfbi_ws_clear(kfbi_ws* ws);

/* Adam training on samples [0, n_train) of the set: `epochs` passes over a seeded
 * shuffle in batches of `batch` (the last partial batch is dropped).  loss_host (epochs
 * floats, nullable) receives the mean training loss of each epoch.  Synchronises. */
int kfbi_ws_train(kfbi_ws* ws, int n_train, int epochs, int batch, float* loss_host);
/* Mean loss over samples [first, first + count) of the set.  Synchronises.
 * KFBI_E_STATE before the target scale is known. */
int kfbi_ws_eval(kfbi_ws* ws, int first, int count, float* loss_host);

/* The target scale sigma in use (0 before it is set). */
int kfbi_ws_target_scale(const kfbi_ws* ws, double* sigma);

/* Raw network access for checks.  feat_dev: [B][M][5] FP32 features (rounded to
 * bfloat16 on entry), out_dev: [B][M] FP32 network outputs.  target_dev: [B][M] FP32;
 * grad_dev: n_params FP32 gradient of the mean squared error; loss_host: the loss.
 * B <= max_batch.  forward is asynchronous, backward synchronises. */
int kfbi_ws_forward(kfbi_ws* ws, int B, const float* feat_dev, float* out_dev);
int kfbi_ws_backward(kfbi_ws* ws, int B, const float* feat_dev, const float* target_dev,
                     float* grad_dev, float* loss_host);

#ifdef __cplusplus
}
#endif
#endif /* WARMSTART_H */
