/*
 * dmnet.h -- C-ABI of the warm-start network in libdm (gfx950).
 *
 * The paper notes that initial guesses of the probe and object may be
 * "pre-existing results" instead of random ones (Section III, last
 * paragraph).  This network supplies such a guess for the object: from each
 * view's diffraction frame it predicts the object patch under that view's
 * window; the patches are stitched into an initial object with the Eq. 5
 * weights (dm_warm_start in dm.h).  Plain DM from the cold start remains the
 * fallback and the reference the warm start is measured against.
 *
 * Network (U-Net style encoder-decoder, NCHW float32 activations):
 *   input   [n][1][S][S]: log1p of 2x2-binned intensities / 10, zero
 *           frequency at the centre (see dmnet_preprocess)
 *   encoder level l = 0..L-1, C_l = C0 * 2^l channels: two 3x3 convolutions
 *           (zero padding) each followed by ReLU; 2x2 average pooling between
 *           levels
 *   decoder level l = L-2..0: nearest 2x upsampling, concat [upsampled, skip
 *           of level l], two 3x3 convolutions with ReLU
 *   head    1x1 convolution C0 -> 2 (real, imaginary part of the patch)
 *   loss    mean squared error over all outputs; Adam optimiser
 * Weights are stored as bfloat16 (round to nearest even from float32 master
 * copies); biases stay float32 and bias gradients sum the unrounded output
 * gradients.  Every 3x3 convolution (forward, data gradient, weight gradient)
 * runs on the matrix cores as an implicit GEMM with bfloat16 operands -- its
 * input activations and output gradients rounded to nearest even -- and
 * float32 accumulation; the 1x1 head runs on the vector units with float32
 * activations.  DMNET_FLAG_FP32_WEIGHTS uses the float32 masters and float32
 * activations throughout, on the vector units (for gradient checks).
 *
 * Parameter vector (float32, dmnet_n_params entries): for each convolution in
 * the order enc0a, enc0b, enc1a, ..., enc(L-1)b, dec(L-2)a, dec(L-2)b, ...,
 * dec0a, dec0b, head: weights [Cout][Cin][k][k] then biases [Cout].
 *
 * Memory: every device buffer is the caller's; the network's parameters,
 * optimiser state and activations for up to `batch` samples live in the
 * caller's workspace (dmnet_workspace_bytes).  All calls enqueue on the
 * stream given to dmnet_create; calls that return a loss synchronise.
 * Status codes are those of dm.h.
 */
#ifndef DMNET_H_
#define DMNET_H_

#include <stddef.h>
#include <stdint.h>

#include "dm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dmnet dmnet; /* opaque */

#define DMNET_FLAG_FP32_WEIGHTS 1u

typedef struct {
  int32_t batch;     /* largest number of samples per call, >= 1          */
  int32_t size;      /* S: input/output edge, divisible by 2^(levels-1)  */
  int32_t base_ch;   /* C0 >= 1                                          */
  int32_t levels;    /* L in [2, 6]                                      */
  float lr, beta1, beta2, eps;  /* Adam                                  */
  uint32_t flags;    /* DMNET_FLAG_*                                     */
  int32_t reserved;  /* must be 0                                        */
} dmnet_desc;

/* Number of float32 parameters; 0 if the descriptor is invalid. */
size_t dmnet_n_params(const dmnet_desc* desc);
/* Workspace bytes for dmnet_create; 0 if the descriptor is invalid. */
size_t dmnet_workspace_bytes(const dmnet_desc* desc);

/* Create the network; parameters are zero until dmnet_set_params. */
dm_status dmnet_create(dmnet** out, const dmnet_desc* desc, void* workspace_dev,
                       size_t workspace_bytes, void* hip_stream);

/* Copy parameters in (float32 [n_params], device) and reset Adam's state
 * and step count; or copy the float32 master parameters out. */
dm_status dmnet_set_params(dmnet* net, const float* params_dev);
dm_status dmnet_get_params(dmnet* net, float* params_dev);

/* y [n][2][S][S] = network(x [n][1][S][S]), 1 <= n <= batch. */
dm_status dmnet_forward(dmnet* net, const float* x_dev, float* y_dev, int32_t n);

/* Loss of (x, target [n][2][S][S]) and its gradient with respect to the
 * parameters (float32 [n_params], device; may be NULL); no update.
 * Synchronises. */
dm_status dmnet_loss_grad(dmnet* net, const float* x_dev, const float* target_dev, int32_t n,
                          float* grads_dev, float* loss_host);

/* One Adam step on (x, target); *loss_host gets the loss before the step
 * (NULL: do not synchronise). */
dm_status dmnet_train_step(dmnet* net, const float* x_dev, const float* target_dev,
                           int32_t n, float* loss_host);

/* x [n][1][F/2][F/2] = log1p(2x2 sums of I [n][F][F]) / 10 (negative
 * intensities count as 0), the binned frame shifted by S/2 in both
 * directions so that the block holding the zero frequency (frame pixel
 * [0][0], the DFT convention of dm.h) lands at [S/2][S/2].  F/2 must equal
 * the network size S. */
dm_status dmnet_preprocess(dmnet* net, const float* I_dev, int32_t n, int32_t frame,
                           float* x_dev);

/* patches [n][2S][2S] complex64 = bilinear 2x upsampling of y [n][2][S][S]
 * (channel 0 real, 1 imaginary; sample points at pixel centres, edges
 * clamped). */
dm_status dmnet_patches(dmnet* net, const float* y_dev, int32_t n, void* patches_dev);

void dmnet_free(dmnet* net);
const char* dmnet_last_error(const dmnet* net);

#ifdef __cplusplus
}
#endif

#endif /* DMNET_H_ */
