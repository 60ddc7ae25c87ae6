/*
 * emu.h - C ABI of the summary-statistics emulator in libcpm.
 *
 * The paper does not define this part.  It is a learned stand-in for whole
 * runs of the batched model: a multilayer perceptron maps a parameter point
 * of a 2D run to the eight cell-level summary statistics that
 * cpm_batch_summary() computes from such a run (means and variances of cell
 * volume, surface, speed and persistence time; speed and directional
 * persistence are the motility read-outs of the paper's Results, Fig. 5B).
 * The plain model stays the fallback and the reference for the emulator's error.
 *
 * Network: 6 -> 256 -> 256 -> 256 -> 8, exact (erf) GELU after each hidden
 * layer, linear output.  A point's six inputs are, in order, ln lambda_V,
 * ln J(cell,cell), ln J(cell,medium), ln T, ln lambda_act and L / 512; its
 * eight outputs are, in order, mean and variance of volume, of surface, of
 * speed and of persistence time.  Inputs and targets are z-scored with a
 * stored normalisation (emu_fit_norm / emu_set_norm); a target column with a
 * positive offset `off` is learnt as log(t + off) (for quantities that span
 * decades and may be 0).  emu_forward returns outputs in the targets' own
 * units.
 *
 * Arithmetic: matrix products on the matrix cores with bf16 operands
 * (weights, activations, gradients of pre-activations, rounded to nearest
 * even) and fp32 accumulation; biases, pre-activations, GELU, the loss and
 * Adam in fp32 on fp32 master parameters, whose bf16 copies are refreshed
 * after every update.
 *
 * Parameters: one packed fp32 vector of emu_param_count() = 135,432 values,
 * W1 (256 x 6), b1 (256), W2 (256 x 256), b2 (256), W3 (256 x 256), b3 (256),
 * W4 (8 x 256), b4 (8); W is (out x in), row-major, and a layer computes
 * z = x W^T + b.
 *
 * Normalisation vector (36 fp32): input means (6), input standard
 * deviations (6), target means (8) and standard deviations (8) after the
 * transform, target offsets (8; 0 = no transform).
 *
 * Training loss: mean over the n x 8 normalised outputs of the squared
 * error.  Adam with beta1 = 0.9, beta2 = 0.999, eps = 1e-8 and bias
 * correction; the step count restarts at emu_set_params().
 *
 * Memory: every pointer argument named d_* is device memory on the current
 * device, owned by the caller; x is n x 6 and targets / outputs n x 8 fp32,
 * row-major.  The workspace (size from emu_workspace_bytes for the largest
 * batch, 256-byte aligned) is borrowed until emu_destroy.
 *
 * Streams: every call enqueues on `stream` (a hipStream_t, NULL = default
 * stream) and returns without waiting, except where stated.  Calls on one
 * handle must not overlap on different streams.
 *
 * Errors: CPM_* codes from cpm.h; cpm_last_error() holds the message.
 */
#ifndef EMU_H
#define EMU_H

#include <stddef.h>
#include <stdint.h>

#include "cpm.h"

#ifdef __cplusplus
extern "C" {
#endif

#define EMU_IN 6
#define EMU_OUT 8
#define EMU_NORM 36

typedef struct emu_handle emu_handle;

/* Number of packed parameters (135,432).  Pure host. */
int emu_param_count(int64_t *count);

/* Workspace bytes for batches of up to max_batch points (1 <= max_batch
 * <= 2^20).  Pure host.  CPM_EINVAL on a bad size. */
int emu_workspace_bytes(int32_t max_batch, size_t *bytes);

/* Create a handle on the workspace: all parameters zero, normalisation the
 * identity (means 0, standard deviations 1).  CPM_EINVAL (null pointer, bad
 * size, misaligned workspace), CPM_ENOMEM (workspace too small),
 * CPM_EDEVICE. */
int emu_init(int32_t max_batch, void *d_workspace, size_t workspace_bytes, void *stream, emu_handle **out);

/* Copy a packed parameter vector in (and reset the Adam state and step
 * count) or out. */
int emu_set_params(emu_handle *h, const float *d_params, void *stream);
int emu_get_params(emu_handle *h, float *d_params, void *stream);

/* Set the normalisation from a device vector of EMU_NORM values (standard
 * deviations must be positive; not checked on the device), or fit it to a
 * data set: column means and population standard deviations of x (n x 6) and
 * targets (n x 8), in fp64 sums; a column with no spread gets 1.  Target
 * columns j with bit j of log_mask set get off_j = G_j / 100, G_j the
 * geometric mean of the column's positive values (off_j = 1 if it has none),
 * and are fitted as log(t + off_j); targets must then exceed -off_j. */
int emu_set_norm(emu_handle *h, const float *d_norm, void *stream);
int emu_get_norm(emu_handle *h, float *d_norm, void *stream);
int emu_fit_norm(emu_handle *h, const float *d_x, const float *d_targets, int32_t n, int32_t log_mask,
                 void *stream);

/* Outputs d_y (n x 8, de-normalised) for inputs d_x (n x 6),
 * 1 <= n <= max_batch. */
int emu_forward(emu_handle *h, const float *d_x, int32_t n, float *d_y, void *stream);

/* Gradient of the loss at the current parameters into the handle's gradient
 * buffer, and copies of it (d_grad, packed like the parameters) and of the
 * loss (d_loss, one float) where those are not NULL. */
int emu_grads(emu_handle *h, const float *d_x, const float *d_targets, int32_t n, float *d_grad, float *d_loss,
              void *stream);

/* One Adam step of size lr (> 0) with the gradient d_grad (packed, device),
 * or with the handle's gradient buffer when d_grad is NULL. */
int emu_adam(emu_handle *h, const float *d_grad, float lr, void *stream);

/* emu_grads then emu_adam on one mini-batch. */
int emu_train_step(emu_handle *h, const float *d_x, const float *d_targets, int32_t n, float lr, float *d_loss,
                   void *stream);

/* Adam steps taken since emu_set_params / emu_init.  Pure host. */
int emu_step_count(emu_handle *h, int64_t *steps);

int emu_destroy(emu_handle *h);

#ifdef __cplusplus
}
#endif

#endif /* EMU_H */
