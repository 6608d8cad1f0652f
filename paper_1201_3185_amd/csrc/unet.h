// Internal declarations of the U-Net kernels (unet_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace qm {

// A channel slice of a channel-last BF16 grid: element (v, c) at p[v * cs + c].
struct Tensor {
    __bf16 *p;
    int n;    // points per side
    int cs;   // slot width (channels per voxel slot)
};

constexpr int kMaxSplit = 256;
constexpr int kLossBlocks = 256;

void launch_conv3d_fwd(Tensor x, int cin, const __bf16 *wt, int kpad, int cout, const float *bias, Tensor y,
                       int stride, int relu, hipStream_t s);
void launch_dgrad_weights(const __bf16 *wt, int cin, int cout, int kpad, __bf16 *wd, int kpad_d, hipStream_t s);
void launch_dilate(Tensor src, Tensor dst, int c, hipStream_t s);
int wgrad_splits(int cout, int kpad, int nout);
void launch_wgrad(Tensor x, int cin, Tensor dy, int cout, int kpad, int stride, float *partial, float *dw,
                  hipStream_t s);
void launch_bgrad(Tensor dy, int c, float *partial, float *db, hipStream_t s);
void launch_relu_bwd(Tensor g, Tensor y, int c, hipStream_t s);
void launch_add(Tensor dst, Tensor src, int c, hipStream_t s);
void launch_upsample(Tensor src, Tensor dst, int c, hipStream_t s);
void launch_upsample_adj(Tensor gf, Tensor gc, int c, hipStream_t s);
void launch_head_fwd(Tensor x, int c, const float *w, const float *b, float *yh, hipStream_t s);
void launch_head_bwd(const float *dyh, Tensor x, int c, const float *w, Tensor dx, float *partial, float *dwb,
                     hipStream_t s);
void launch_mse(const float *yh, const float *tg, int n, float *dy, double *partial, double *loss, hipStream_t s);
void launch_adam(float *w, float *m, float *v, const float *g, int count, float lr, int step, __bf16 *wb, hipStream_t s);
void launch_to_bf16(const float *src, __bf16 *dst, int count, hipStream_t s);
// channel 0 = (phin - base) inv_cn, channel 1 = S h2_cs
void launch_prep_input(int n, const double *phin, const double *base, const double *S, double inv_cn, double h2_cs,
                       Tensor x, hipStream_t s);
void launch_expand_input(const __bf16 *xc, Tensor x, hipStream_t s);
// out = a in + base;  target = a (in - base)
void launch_scale_out(const float *in, int count, double a, const double *base, double *out, hipStream_t s);
void launch_scale_in(const double *in, const double *base, int count, double a, float *out, hipStream_t s);

inline int kpad_of(int cin) { return (27 * cin + 31) / 32 * 32; }

}  // namespace qm
