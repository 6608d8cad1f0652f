/*
 * qumond_unet.h -- the learned initial guess for the QUMOND solve.
 *
 * A 3D U-Net maps the Newtonian potential Phi_N and the Eq. 2 source S of a
 * box (Angus et al., arXiv:1201.3185, Sec. 2, steps 2 and 3) to a prediction
 * of the QUMOND potential Phi (step 4), which seeds the second multigrid
 * solve (qumond_solve_mond with a guess; plain FMG remains the fallback and
 * the residual the judge).  Four levels n -> (n+1)/2 -> ... (n = 2^J + 1,
 * J >= 4; 129 -> 65 -> 33 -> 17), channels 16/32/64/64, 3x3x3 convolutions
 * with ReLU, stride-2 convolutions down, trilinear up-sampling concatenated
 * with the skip tensor and a convolution up, and a 1x1x1 output head.
 * Activations and weights are BF16, accumulation FP32 (MFMA), master weights
 * and Adam state FP32.
 *
 * Scaling (chosen by the caller from quantities known before the solve):
 * the network sees and predicts departures from the potentials of a
 * softened point mass of the box's total mass M, B_N = -GM / r_s and
 * B_Q = the QUMOND monopole of qumond.h at r_s, r_s = sqrt(r^2 + soft^2) (r
 * from the box centre), which carry the mass-dependent part of Phi that the
 * scaled fields alone would hide: input channel 0 = (Phi_N - B_N) / c_phin,
 * channel 1 = h^2 S / c_out, output Phi = B_Q + c_out * prediction.  GM = 0
 * turns the baselines off.  All arrays are device pointers except where
 * marked host; calls are asynchronous on the net's stream unless they return
 * a host value.
 */
#ifndef QUMOND_UNET_H
#define QUMOND_UNET_H

#include <stdint.h>
#include "qumond.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qumond_unet qumond_unet;

/* He-normal initial weights from a 64-bit seed (deterministic). */
qumond_status qumond_unet_create(int32_t n, uint64_t seed, void *hip_stream, qumond_unet **out);
qumond_status qumond_unet_destroy(qumond_unet *net);
int64_t qumond_unet_param_count(const qumond_unet *net);
/* FP32 master weights in layer order (host buffer of param_count floats).
 * set_params also clears the Adam state.  Synchronise. */
qumond_status qumond_unet_get_params(qumond_unet *net, float *host);
qumond_status qumond_unet_set_params(qumond_unet *net, const float *host);

/* Gradients of the last qumond_unet_train_step, same layout as the params. */
qumond_status qumond_unet_get_grads(qumond_unet *net, float *host);

/* One training sample from the method's fields: x (n^3 x 2 BF16, the two
 * input channels) and target (n^3 FP32, (Phi - B_Q) / c_out).  GM (>= 0),
 * a0 (>= 0) and soft (kpc, > 0) define the baselines; the box side is
 * h (n - 1). */
qumond_status qumond_unet_prepare_sample(qumond_unet *net, const double *phin, const double *S, const double *phi,
                                         double h, double c_phin, double c_out, double GM, double a0, double soft,
                                         void *x, float *target);

/* One Adam step (learning rate lr) on the mean squared error over interior
 * nodes between the prediction for x and target; loss (host, optional;
 * synchronises) gets the loss before the step. */
qumond_status qumond_unet_train_step(qumond_unet *net, const void *x, const float *target, float lr, double *loss);

/* Prediction for (Phi_N, S): guess = B_Q + c_out * network output (n^3 FP64). */
qumond_status qumond_unet_infer(qumond_unet *net, const double *phin, const double *S, double h, double c_phin,
                                double c_out, double GM, double a0, double soft, double *guess);

/* Single-layer entry points (BF16 channel-last tensors with slot width equal
 * to the channel count; weights [cout][kpad], kpad = 27 cin rounded up to 32;
 * cin a multiple of 8, cout of 16).  fwd: y = act(conv(x) + bias) with stride
 * 1 or 2 (n_out = n_in or (n_in+1)/2, zero padding); dgrad: dx from dy;
 * wgrad: dw (FP32 [cout][kpad]) = sum over output voxels of dy x. */
qumond_status qumond_k_conv3d_fwd(int32_t n_in, int32_t cin, const void *x, int32_t cout, const void *w,
                                  const float *bias, int32_t stride, int32_t relu, void *y, void *stream);
qumond_status qumond_k_conv3d_dgrad(int32_t n_in, int32_t cin, int32_t cout, const void *w, int32_t stride,
                                    const void *dy, void *dx, void *stream);
qumond_status qumond_k_conv3d_wgrad(int32_t n_in, int32_t cin, const void *x, int32_t cout, const void *dy,
                                    int32_t stride, float *dw, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* QUMOND_UNET_H */
