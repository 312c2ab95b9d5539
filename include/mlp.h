/*
 * mlp.h - C ABI of the warm-start network on MI355X (gfx950): forward pass,
 * mean-squared-error backward pass and Adam, as hand-written BF16 MFMA
 * kernels with FP32 accumulation.
 *
 * Purpose: the paper computes cycle-averaged density and mean-energy
 * profiles of e, O- and O2+ across the gap for a given voltage and pressure
 * (section 3, the quasi-stationary profiles after many rf cycles).  The
 * network maps (U / U_max, normalised log p, x / L) to those six profiles
 * (log densities and mean energies, standardised by the caller) so that a
 * discharge can be loaded close to its periodic steady state
 * (pic_load_profiles in pic.h).  The paper itself has no such network.
 *
 * Network: 3 inputs -> 4 hidden layers of 256 units with GELU
 * (z Phi(z), exact error function) -> 6 outputs.  Parameters, in this order
 * in every flat FP32 vector (199942 values): W0 [256][3], b0 [256],
 * W1 [256][256], b1, W2, b2, W3, b3, W4 [6][256], b4 [6]; W[o][i] multiplies
 * input i of output o.
 *
 * Precision: the weights used in products are bfloat16 copies of FP32 master
 * weights; the input and every hidden activation are stored as bfloat16; the
 * output-layer and hidden-unit gradients entering products are rounded to
 * bfloat16; every product is summed in FP32 on the matrix cores; biases,
 * pre-activations, losses and gradients of the parameters are FP32.
 *
 * Memory: the library allocates no device memory.  mlp_query reports the
 * size of one caller-owned device workspace (parameters, gradients, Adam
 * moments, activations for up to max_batch samples).  Device pointers passed
 * to calls (inputs, targets, outputs) are caller-owned.  All work is
 * enqueued on the stream given to mlp_create; calls that return host data
 * synchronise it.  Errors: 0 on success, negative codes of pic.h
 * (PIC_EINVAL, PIC_EHIP, PIC_ENODEVICE); mlp_last_error() gives a message.
 */
#ifndef MLP_H
#define MLP_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MLP_NIN 3
#define MLP_NHID 256
#define MLP_NLAYER 5        /* 4 hidden + output */
#define MLP_NOUT 6
#define MLP_NPARAM 199942

typedef struct mlp_handle mlp_handle;

/* Device bytes for a network that processes batches of up to max_batch
   samples (1 .. 1048576).  Pure host call. */
int mlp_query(int32_t max_batch, uint64_t *workspace_bytes);

/* `workspace`: caller-owned device memory of at least mlp_query bytes;
   `stream`: hipStream_t (NULL = default).  Parameters start at zero; Adam
   moments and step count at zero. */
int mlp_create(int32_t max_batch, void *workspace, uint64_t workspace_bytes, void *stream, mlp_handle **out);
int mlp_destroy(mlp_handle *h);

/* Copies MLP_NPARAM FP32 master parameters from / to the host (the bfloat16
   copies are refreshed from the master values).  Both synchronise. */
int mlp_set_params(mlp_handle *h, const float *host_params);
int mlp_get_params(mlp_handle *h, float *host_params);

/* Inference: y [batch][6] (FP32, device) from x [batch][3] (FP32, device).
   Asynchronous. */
int mlp_forward(mlp_handle *h, int32_t batch, const float *x, float *y);

/* Inference for callers that cannot allocate device memory or enqueue copies
   (code under HIP graph capture, tight serving loops, harnesses that forbid
   allocation): the same outputs as mlp_forward, bit for bit, with the hidden
   activations in a static array of the library (MLP_STATIC_SCRATCH_BYTES per
   device, held until the process ends) instead of the handle's workspace, and
   the outputs written straight into y.  Allocates nothing and makes no copy.
   1 <= batch <= MLP_STATIC_MAX_BATCH, else PIC_EINVAL.  x [batch][3] and
   y [batch][6] are FP32 device arrays.  Asynchronous on the handle's stream.
   Every call on one device shares that device's array: calls that overlap in
   time on one device (other streams, other threads, other handles) race.
   Nothing in the array needs clearing: each call writes what it reads. */
#define MLP_STATIC_MAX_BATCH 4096
#define MLP_STATIC_SCRATCH_BYTES 8413184   /* the input (256-aligned), then 8 B per hidden unit per sample:
                                              a 4 B pre-activation and two 2 B activation buffers */
int mlp_forward_static(mlp_handle *h, int32_t batch, const float *x, float *y);

/* Training pass: forward with the activations kept, loss
   L = mean over the batch and the 6 outputs of (y - t)^2 for targets
   t [batch][6] (FP32, device), then the gradient of L with respect to every
   parameter into the handle's gradient buffer.  If loss_host is non-NULL the
   call synchronises and stores L there. */
int mlp_backward(mlp_handle *h, int32_t batch, const float *x, const float *t, float *loss_host);

/* Copies the MLP_NPARAM FP32 gradients of the last mlp_backward to the host. */
int mlp_get_grads(mlp_handle *h, float *host_grads);

/* One bias-corrected Adam step on the master parameters with the gradients of
   the last mlp_backward: m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
   p -= lr (m / (1 - b1^k)) / (sqrt(v / (1 - b2^k)) + eps), k = 1, 2, ... the
   handle's step count; the bfloat16 copies are refreshed.  Asynchronous. */
int mlp_adam(mlp_handle *h, float lr, float beta1, float beta2, float eps);

const char *mlp_last_error(const mlp_handle *h);

#ifdef __cplusplus
}
#endif
#endif
