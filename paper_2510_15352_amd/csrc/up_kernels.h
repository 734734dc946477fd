// Host-side launchers of the learned-upsampler kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gs {

constexpr float kUpDepthScale = 10.0f;  // network depth channel = depth / 10 m
constexpr float kUpDepthInv = 0.1f;
constexpr float kUpDepthWeight = 0.1f;  // loss weight of the depth channel

// UP_EPI_RELU_BF16_IN4: the first layer at inference, reading its input
// from x0f (FP32, four channels) instead of the padded BF16 copy.
enum { UP_EPI_RELU_BF16 = 0, UP_EPI_F32 = 1, UP_EPI_MASK_BF16 = 2, UP_EPI_HEAD = 3,
       UP_EPI_RELU_BF16_IN4 = 4 };

int up_conv_blocks(int n, int h, int w);
int up_head_blocks(int n, int h, int w);
// x0b may be null (inference: the first layer reads x0f).
void launch_up_input(const float *rgb, const float *depth, int64_t npix, float *x0f,
                     uint16_t *x0b, hipStream_t st);
// epi UP_EPI_HEAD (32 -> 64, inference): the head is fused into the
// epilogue, writing full-resolution rgb / depth from x0f (out unused).
void launch_up_conv(int cin, int cout, int epi, const uint16_t *in, const uint16_t *wt,
                    const float *bias, int n, int h, int w, const uint16_t *mask, void *out,
                    hipStream_t st, const float *x0f = nullptr, float *rgb = nullptr,
                    float *depth = nullptr);
void launch_up_wgrad(int cin, int cout, const uint16_t *x, const uint16_t *dy, int n, int h,
                     int w, float *part, float *partb, hipStream_t st);
void launch_sum_partials(float *part, int nblk, int len, float *grad, hipStream_t st);
void launch_up_head(bool train, const float *x0f, const float *y, int h, int w, int n,
                    float *rgb, float *depth, const float *t_rgb, const float *t_depth,
                    float *loss_part, uint16_t *dy, hipStream_t st);
void launch_pack_weights(const float *w, int cout, int cin, int cinp, uint16_t *wf, uint16_t *wd,
                         hipStream_t st);
void launch_adam(float *p, float *m, float *v, const float *g, int n, float lr, int step,
                 hipStream_t st);
void launch_up_score(const float *x0f, int n, int h, int w, float *score, hipStream_t st);
void launch_up_flag(const float *score, int n, float thr, uint32_t *mask, uint32_t *count,
                    hipStream_t st);
void launch_frame_psnr(const float *a, const float *b, int n, int64_t npix, float *out,
                       hipStream_t st);
void launch_quarter_intr(const float *in, int n, float *out, hipStream_t st);

}  // namespace gs
