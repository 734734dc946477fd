// Learned 4x upsampler: BF16 MFMA 3x3 convolutions (FP32 accumulation) for
// inference and training, pixel-shuffle head with bilinear skip, MSE loss,
// Adam.
//
// Network: x0 (low-res RGB + depth / 10) -> conv 4->32, ReLU -> conv 32->32,
// ReLU -> conv 32->32, ReLU -> conv 32->64 -> 4x pixel shuffle (channel
// c*16 + i*4 + j of low-res pixel (y, x) goes to full-res pixel (4y+i, 4x+j),
// channel c) + bilinear 4x upsampling of x0 (half-pixel centres, clamped).
//
// Activations are NHWC BF16 with 32 or 64 channels (the 4-channel input is
// zero-padded to 32). A convolution is an implicit GEMM on
// v_mfma_f32_16x16x32_bf16: M = 16 consecutive pixels of one row, N = 16
// output channels, K = 32 input channels of one of the nine taps.
//   forward      out[p][n] = act(b[n] + sum_t sum_k in[p + off(t)][k] Wt[t][n][k])
//   data grad    the same kernel with Wt'[t][ci][co] = w[co][8 - t][ci] and a
//                ReLU-mask epilogue (zero padding is its own adjoint)
//   weight grad  dW[co][t][ci] = sum_p dY[p][co] X[p + off(t)][ci]: M = 16 co,
//                N = 16 (t, ci), K = 32 pixels; one partial per block, summed
//                in a fixed order by a second kernel (deterministic).
#include <algorithm>
#include <cmath>

#include "gs_device.h"
#include "up_kernels.h"

namespace gs {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kTY = 8;    // output tile rows
constexpr int kTX = 32;   // output tile columns
constexpr int kHY = kTY + 2, kHX = kTX + 2;  // input tile with halo

__device__ __forceinline__ uint16_t bf16_bits(float f)
{
    // round to nearest even
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);  // inf / nan
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_to_f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// ------------------------------------------------------------ input prep --
// x0f[n][y][x][4] = (r, g, b, depth / 10) (FP32, for the skip) and, when
// x0b is given (training), x0b[n][y][x][32] = the same in BF16, channels
// 4..31 zero.
__global__ void k_up_input(const float *__restrict__ rgb, const float *__restrict__ depth,
                           int64_t npix, float *__restrict__ x0f, uint16_t *__restrict__ x0b)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npix) return;
    const float v[4] = {rgb[p * 3 + 0], rgb[p * 3 + 1], rgb[p * 3 + 2], depth[p] * kUpDepthInv};
    if (x0b) {
        uint4 *dst = reinterpret_cast<uint4 *>(x0b + p * 32);
        uint32_t w0 = (uint32_t)bf16_bits(v[0]) | ((uint32_t)bf16_bits(v[1]) << 16);
        uint32_t w1 = (uint32_t)bf16_bits(v[2]) | ((uint32_t)bf16_bits(v[3]) << 16);
        dst[0] = make_uint4(w0, w1, 0u, 0u);
        dst[1] = make_uint4(0u, 0u, 0u, 0u);
        dst[2] = make_uint4(0u, 0u, 0u, 0u);
        dst[3] = make_uint4(0u, 0u, 0u, 0u);
    }
    reinterpret_cast<float4 *>(x0f)[p] = make_float4(v[0], v[1], v[2], v[3]);
}

// Source rows / columns and weight of bilinear 4x upsampling (half-pixel
// centres, clamped at the border) for full-resolution index t.
__device__ __forceinline__ void bilinear_src(int t, int n_in, int &i0, int &i1, float &f)
{
    float s = ((float)t + 0.5f) * 0.25f - 0.5f;
    s = fmaxf(s, 0.0f);
    i0 = min((int)s, n_in - 1);
    i1 = min(i0 + 1, n_in - 1);
    f = s - (float)i0;
}

// ------------------------------------------------------------ conv (MFMA) --
enum { EPI_RELU_BF16 = 0, EPI_F32 = 1, EPI_MASK_BF16 = 2, EPI_HEAD = 3 };

// Outputs of the fused head: full-resolution RGB and depth of the images.
struct HeadOut {
    const float *x0f;  // low-res input (r, g, b, depth / 10) for the bilinear skip
    float *rgb, *depth;
};

// One block = an 8 x 32 output tile of one image, 4 waves; wave w owns rows
// 2w and 2w+1 (4 M-tiles of 16 pixels) and all COUT/16 N-tiles.
// IN4 (first layer at inference): the input tile is built from the FP32
// four-channel x0f (head.x0f) in LDS, BF16 with channels 4..31 zero, exactly
// the values the padded BF16 copy would hold.
// EPI_HEAD (inference, 32 -> 64): the epilogue is the network head, 4x
// pixel shuffle plus the bilinear skip, writing full-resolution RGB and
// depth directly: lane (lr, lk) holds channels c * 16 + lr (c = 0..3) of its
// low-res pixels, i.e. the four outputs of sub-pixel (lr / 4, lr % 4).
template <int CIN, int COUT, int EPI, bool IN4 = false>
__global__ __launch_bounds__(256) void k_conv3x3(const uint16_t *__restrict__ in,
                                                 const uint16_t *__restrict__ wt,
                                                 const float *__restrict__ bias, int H, int W,
                                                 int tiles_x, int tiles_y,
                                                 const uint16_t *__restrict__ mask, void *out,
                                                 HeadOut head)
{
    constexpr int NT = COUT / 16;
    __shared__ __attribute__((aligned(16))) uint16_t s_in[kHY * kHX * CIN];
    __shared__ __attribute__((aligned(16))) uint16_t s_w[9 * COUT * CIN];
    // the head's bilinear skip reads the FP32 input of the tile and its halo
    __shared__ float4 s_x0[EPI == EPI_HEAD ? kHY * kHX : 1];
    const int tid = threadIdx.x;
    const int img = blockIdx.x / (tiles_x * tiles_y);
    const int t2 = blockIdx.x % (tiles_x * tiles_y);
    const int ty0 = (t2 / tiles_x) * kTY, tx0 = (t2 % tiles_x) * kTX;
    const int64_t img_base = (int64_t)img * H * W;
    // stage the input tile (zero outside the image) and the weights in
    // 16-byte pieces: every piece of the thread is loaded before the first
    // LDS write, so a block waits for one memory latency, not one per piece
    constexpr int PPX = CIN / 8;  // 16-byte pieces per pixel
    constexpr int NIN = kHY * kHX * PPX, NIN_T = (NIN + 255) / 256;
    constexpr int NWT = 9 * COUT * CIN / 8, NWT_T = (NWT + 255) / 256;
    constexpr int NPX_T = (kHY * kHX + 255) / 256;
    uint4 vin[IN4 ? 1 : NIN_T], vw[NWT_T];
    float4 vpx[(IN4 || EPI == EPI_HEAD) ? NPX_T : 1];
    if constexpr (IN4) {
        static_assert(CIN == 32, "the first layer's input is padded to 32 channels");
#pragma unroll
        for (int k = 0; k < NPX_T; ++k) {
            const int pix = tid + k * 256;
            const int y = ty0 - 1 + pix / kHX, x = tx0 - 1 + pix % kHX;
            vpx[k] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (pix < kHY * kHX && y >= 0 && y < H && x >= 0 && x < W)
                vpx[k] = reinterpret_cast<const float4 *>(head.x0f)[img_base + (int64_t)y * W + x];
        }
    } else {
        if constexpr (EPI == EPI_HEAD) {
#pragma unroll
            for (int k = 0; k < NPX_T; ++k) {
                const int pix = tid + k * 256;
                const int y = ty0 - 1 + pix / kHX, x = tx0 - 1 + pix % kHX;
                vpx[k] = make_float4(0.f, 0.f, 0.f, 0.f);
                if (pix < kHY * kHX && y >= 0 && y < H && x >= 0 && x < W)
                    vpx[k] = reinterpret_cast<const float4 *>(head.x0f)[img_base + (int64_t)y * W + x];
            }
        }
#pragma unroll
        for (int k = 0; k < NIN_T; ++k) {
            const int e = tid + k * 256;
            const int pix = e / PPX, part = e % PPX;
            const int y = ty0 - 1 + pix / kHX, x = tx0 - 1 + pix % kHX;
            vin[k] = make_uint4(0u, 0u, 0u, 0u);
            if (e < NIN && y >= 0 && y < H && x >= 0 && x < W)
                vin[k] = reinterpret_cast<const uint4 *>(in + (img_base + (int64_t)y * W + x) * CIN)[part];
        }
    }
#pragma unroll
    for (int k = 0; k < NWT_T; ++k) {
        const int e = tid + k * 256;
        vw[k] = make_uint4(0u, 0u, 0u, 0u);
        if (e < NWT) vw[k] = reinterpret_cast<const uint4 *>(wt)[e];
    }
    if constexpr (IN4) {
#pragma unroll
        for (int k = 0; k < NPX_T; ++k) {
            const int pix = tid + k * 256;
            if (pix < kHY * kHX) {
                const float4 v = vpx[k];
                uint4 *d = reinterpret_cast<uint4 *>(s_in) + pix * PPX;
                d[0] = make_uint4((uint32_t)bf16_bits(v.x) | ((uint32_t)bf16_bits(v.y) << 16),
                                  (uint32_t)bf16_bits(v.z) | ((uint32_t)bf16_bits(v.w) << 16), 0u, 0u);
#pragma unroll
                for (int q = 1; q < PPX; ++q) d[q] = make_uint4(0u, 0u, 0u, 0u);
            }
        }
    } else {
#pragma unroll
        for (int k = 0; k < NIN_T; ++k)
            if (tid + k * 256 < NIN) reinterpret_cast<uint4 *>(s_in)[tid + k * 256] = vin[k];
        if constexpr (EPI == EPI_HEAD) {
#pragma unroll
            for (int k = 0; k < NPX_T; ++k)
                if (tid + k * 256 < kHY * kHX) s_x0[tid + k * 256] = vpx[k];
        }
    }
#pragma unroll
    for (int k = 0; k < NWT_T; ++k)
        if (tid + k * 256 < NWT) reinterpret_cast<uint4 *>(s_w)[tid + k * 256] = vw[k];
    __syncthreads();

    const int wave = tid >> 6, lane = tid & 63;
    const int lr = lane & 15, lk = lane >> 4;
    // this lane's output-channel biases, loaded while the MFMAs run
    float bch[NT];
#pragma unroll
    for (int n = 0; n < NT; ++n)
        bch[n] = (EPI == EPI_F32 || EPI == EPI_RELU_BF16) ? bias[n * 16 + lr] : 0.0f;
    floatx4 acc[4][NT];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = 0; n < NT; ++n) acc[m][n] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const int ky = t / 3, kx = t % 3;
#pragma unroll
        for (int c0 = 0; c0 < CIN; c0 += 32) {
            bf16x8 a[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int row = wave * 2 + (m >> 1), col = (m & 1) * 16 + lr;
                const int pix = (row + ky) * kHX + col + kx;
                a[m] = *reinterpret_cast<const bf16x8 *>(s_in + pix * CIN + c0 + lk * 8);
            }
#pragma unroll
            for (int n = 0; n < NT; ++n) {
                const bf16x8 b =
                    *reinterpret_cast<const bf16x8 *>(s_w + (t * COUT + n * 16 + lr) * CIN + c0 + lk * 8);
#pragma unroll
                for (int m = 0; m < 4; ++m)
                    acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m], b, acc[m][n], 0, 0, 0);
            }
        }
    }
    if constexpr (EPI == EPI_HEAD) {
        static_assert(COUT == 64, "the head takes 64 channels");
        const int si = lr >> 2, sj = lr & 3;
        const int H4 = 4 * H, W4 = 4 * W;
        float bs[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) bs[c] = bias[c * 16 + lr];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int y = ty0 + wave * 2 + (m >> 1);
            if (y >= H) continue;
            const int Y = 4 * y + si;
            int y0, y1;
            float fy;
            bilinear_src(Y, H, y0, y1, fy);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int x = tx0 + (m & 1) * 16 + lk * 4 + i;
                if (x >= W) continue;
                const int X = 4 * x + sj;
                int xa, xb;
                float fx;
                bilinear_src(X, W, xa, xb, fx);
                // the sources lie within one pixel of (y, x): inside the staged halo
                const int r0 = (y0 - ty0 + 1) * kHX, r1 = (y1 - ty0 + 1) * kHX;
                const int ca = xa - tx0 + 1, cb = xb - tx0 + 1;
                const float4 v00 = s_x0[r0 + ca], v01 = s_x0[r0 + cb];
                const float4 v10 = s_x0[r1 + ca], v11 = s_x0[r1 + cb];
                const float s00[4] = {v00.x, v00.y, v00.z, v00.w};
                const float s01[4] = {v01.x, v01.y, v01.z, v01.w};
                const float s10[4] = {v10.x, v10.y, v10.z, v10.w};
                const float s11[4] = {v11.x, v11.y, v11.z, v11.w};
                float pred[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const float yv = acc[m][c][i] + bs[c];
                    const float top = s00[c] * (1.0f - fx) + s01[c] * fx;
                    const float bot = s10[c] * (1.0f - fx) + s11[c] * fx;
                    pred[c] = top * (1.0f - fy) + bot * fy + yv;
                }
                const int64_t q = (int64_t)img * H4 * W4 + (int64_t)Y * W4 + X;
                head.rgb[q * 3 + 0] = pred[0];
                head.rgb[q * 3 + 1] = pred[1];
                head.rgb[q * 3 + 2] = pred[2];
                head.depth[q] = pred[3] * kUpDepthScale;
            }
        }
    } else {
        // epilogue: lane holds channel n*16 + lr of pixels 4*lk + i of each M-tile
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int y = ty0 + wave * 2 + (m >> 1);
            if (y >= H) continue;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int x = tx0 + (m & 1) * 16 + lk * 4 + i;
                if (x >= W) continue;
                const int64_t p = img_base + (int64_t)y * W + x;
#pragma unroll
                for (int n = 0; n < NT; ++n) {
                    const int ch = n * 16 + lr;
                    float v = acc[m][n][i];
                    if (EPI == EPI_F32) {
                        reinterpret_cast<float *>(out)[p * COUT + ch] = v + bch[n];
                    } else if (EPI == EPI_RELU_BF16) {
                        v = fmaxf(v + bch[n], 0.0f);
                        reinterpret_cast<uint16_t *>(out)[p * COUT + ch] = bf16_bits(v);
                    } else {
                        v = bf16_to_f(mask[p * COUT + ch]) > 0.0f ? v : 0.0f;  // ReLU'(z) = [a > 0]
                        reinterpret_cast<uint16_t *>(out)[p * COUT + ch] = bf16_bits(v);
                    }
                }
            }
        }
    }
}

// ------------------------------------------------------------ weight grad --
// Partial dW of one 8 x 32 tile: part[blk][co][t * CIN + ci] (FP32) and the
// bias partial partb[blk][co]. Operands are gathered from LDS copies of the
// tile (dY, NHWC) and of the input tile with halo.
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void k_conv3x3_wgrad(const uint16_t *__restrict__ x,
                                                       const uint16_t *__restrict__ dy, int H,
                                                       int W, int tiles_x, int tiles_y,
                                                       float *__restrict__ part,
                                                       float *__restrict__ partb)
{
    constexpr int KN = 9 * CIN;     // GEMM N (tap, ci)
    constexpr int NTN = KN / 16;    // N-tiles
    constexpr int MT = COUT / 16;   // M-tiles
    constexpr int NPW = (NTN + 3) / 4;  // N-tiles per wave
    __shared__ __attribute__((aligned(16))) uint16_t s_x[kHY * kHX * CIN];
    __shared__ __attribute__((aligned(16))) uint16_t s_dy[kTY * kTX * COUT];
    const int tid = threadIdx.x;
    const int img = blockIdx.x / (tiles_x * tiles_y);
    const int t2 = blockIdx.x % (tiles_x * tiles_y);
    const int ty0 = (t2 / tiles_x) * kTY, tx0 = (t2 % tiles_x) * kTX;
    const int64_t img_base = (int64_t)img * H * W;
    for (int e = tid; e < kHY * kHX * (CIN / 8); e += 256) {
        const int pix = e / (CIN / 8), part8 = e % (CIN / 8);
        const int y = ty0 - 1 + pix / kHX, xx = tx0 - 1 + pix % kHX;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (y >= 0 && y < H && xx >= 0 && xx < W)
            v = reinterpret_cast<const uint4 *>(x + (img_base + (int64_t)y * W + xx) * CIN)[part8];
        reinterpret_cast<uint4 *>(s_x)[e] = v;
    }
    for (int e = tid; e < kTY * kTX * (COUT / 8); e += 256) {
        const int pix = e / (COUT / 8), part8 = e % (COUT / 8);
        const int y = ty0 + pix / kTX, xx = tx0 + pix % kTX;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);  // outside the image: no gradient
        if (y < H && xx < W)
            v = reinterpret_cast<const uint4 *>(dy + (img_base + (int64_t)y * W + xx) * COUT)[part8];
        reinterpret_cast<uint4 *>(s_dy)[e] = v;
    }
    __syncthreads();
    const int wave = tid >> 6, lane = tid & 63;
    const int lr = lane & 15, lk = lane >> 4;
    floatx4 acc[MT][NPW];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int j = 0; j < NPW; ++j) acc[m][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < kTY * kTX; k0 += 32) {
        // this lane's 8 pixels of the K-chunk
        bf16x8 a[MT];
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int p = k0 + lk * 8 + i;
                a[m][i] = __builtin_bit_cast(__bf16, s_dy[p * COUT + m * 16 + lr]);
            }
#pragma unroll
        for (int j = 0; j < NPW; ++j) {
            const int nt = wave + 4 * j;
            if (nt >= NTN) break;
            const int kn = nt * 16 + lr;
            const int t = kn / CIN, ci = kn % CIN;
            const int ky = t / 3, kx = t % 3;
            bf16x8 b;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int p = k0 + lk * 8 + i;
                const int py = p / kTX, px = p % kTX;
                b[i] = __builtin_bit_cast(__bf16, s_x[((py + ky) * kHX + px + kx) * CIN + ci]);
            }
#pragma unroll
            for (int m = 0; m < MT; ++m)
                acc[m][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m], b, acc[m][j], 0, 0, 0);
        }
    }
    float *dst = part + (int64_t)blockIdx.x * COUT * KN;
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int j = 0; j < NPW; ++j) {
            const int nt = wave + 4 * j;
            if (nt >= NTN) break;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int co = m * 16 + lk * 4 + i;
                dst[co * KN + nt * 16 + lr] = acc[m][j][i];
            }
        }
    // bias partial: sum of dY over the tile
    if (tid < COUT) {
        float s = 0.0f;
        for (int p = 0; p < kTY * kTX; ++p) s += bf16_to_f(s_dy[p * COUT + tid]);
        partb[(int64_t)blockIdx.x * COUT + tid] = s;
    }
}

// grad[j] = sum over blocks of part[blk][j] in two fixed-order stages: the
// blocks are cut into runs of L; stage one sums run s (in block order) into
// its own first row, part[s L][j] (only the thread summing that run reads
// it), stage two sums those rows in run order.
__global__ void k_sum_runs(float *__restrict__ part, int nblk, int len, int L)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= len) return;
    const int b0 = (int)blockIdx.y * L, b1 = min(b0 + L, nblk);
    float s = 0.0f;
    for (int b = b0; b < b1; ++b) s += part[(int64_t)b * len + j];
    part[(int64_t)b0 * len + j] = s;
}

__global__ void k_sum_run_heads(const float *__restrict__ part, int nruns, int len, int L,
                                float *__restrict__ grad)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= len) return;
    float s = 0.0f;
    for (int r = 0; r < nruns; ++r) s += part[(int64_t)r * L * len + j];
    grad[j] = s;
}

// ------------------------------------------------------------------ head --
// Full-res pixel (Y, X) of image n: pred_c = bilinear(x0)[c] + y[4-tuple].
// Inference writes rgb / depth; training also reads the target, accumulates
// the weighted squared error per block and writes dL/dy (BF16, low-res
// layout, 64 channels).

template <bool TRAIN>
__global__ __launch_bounds__(256) void k_up_head(const float *__restrict__ x0f,
                                                 const float *__restrict__ y, int h, int w,
                                                 int n_img, float *__restrict__ rgb_out,
                                                 float *__restrict__ depth_out,
                                                 const float *__restrict__ t_rgb,
                                                 const float *__restrict__ t_depth,
                                                 float inv_npix, float *__restrict__ loss_part,
                                                 uint16_t *__restrict__ dy)
{
    const int H = h * 4, W = w * 4;
    const int64_t total = (int64_t)n_img * H * W;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float err = 0.0f;
    if (q < total) {
        const int n = (int)(q / ((int64_t)H * W));
        const int rem = (int)(q % ((int64_t)H * W));
        const int Y = rem / W, X = rem % W;
        int y0, y1, xa, xb;
        float fy, fx;
        bilinear_src(Y, h, y0, y1, fy);
        bilinear_src(X, w, xa, xb, fx);
        const float4 *xi = reinterpret_cast<const float4 *>(x0f) + (int64_t)n * h * w;
        const float4 v00 = xi[y0 * w + xa], v01 = xi[y0 * w + xb];
        const float4 v10 = xi[y1 * w + xa], v11 = xi[y1 * w + xb];
        const int ly = Y >> 2, lx = X >> 2, si = Y & 3, sj = X & 3;
        const int64_t lp = ((int64_t)n * h + ly) * w + lx;
        const float *yp = y + lp * 64 + si * 4 + sj;
        float pred[4];
        const float s00[4] = {v00.x, v00.y, v00.z, v00.w}, s01[4] = {v01.x, v01.y, v01.z, v01.w};
        const float s10[4] = {v10.x, v10.y, v10.z, v10.w}, s11[4] = {v11.x, v11.y, v11.z, v11.w};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const float top = s00[c] * (1.0f - fx) + s01[c] * fx;
            const float bot = s10[c] * (1.0f - fx) + s11[c] * fx;
            pred[c] = top * (1.0f - fy) + bot * fy + yp[c * 16];
        }
        if (!TRAIN) {
            rgb_out[q * 3 + 0] = pred[0];
            rgb_out[q * 3 + 1] = pred[1];
            rgb_out[q * 3 + 2] = pred[2];
            depth_out[q] = pred[3] * kUpDepthScale;
        } else {
            const float tg[4] = {t_rgb[q * 3 + 0], t_rgb[q * 3 + 1], t_rgb[q * 3 + 2],
                                 t_depth[q] * kUpDepthInv};
            const float wc[4] = {1.0f, 1.0f, 1.0f, kUpDepthWeight};
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const float d = pred[c] - tg[c];
                err += wc[c] * d * d;
                dy[lp * 64 + c * 16 + si * 4 + sj] = bf16_bits(2.0f * wc[c] * d * inv_npix);
            }
        }
    }
    if (TRAIN) {
        // block sum of the squared error (fixed order)
        __shared__ float s[256];
        s[threadIdx.x] = err;
        __syncthreads();
        for (int d = 128; d > 0; d >>= 1) {
            if ((int)threadIdx.x < d) s[threadIdx.x] += s[threadIdx.x + d];
            __syncthreads();
        }
        if (threadIdx.x == 0) loss_part[blockIdx.x] = s[0];
    }
}

// --------------------------------------------------------------- weights --
// Scale intrinsics by 1/4 for the low-resolution render.
__global__ void k_quarter_intr(const float *__restrict__ in, int n, float *__restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n * 4) out[i] = in[i] * 0.25f;
}

void launch_quarter_intr(const float *in, int n, float *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_quarter_intr, dim3((n * 4 + 255) / 256), dim3(256), 0, st, in, n, out);
}

// BF16 GEMM-ready copies of the FP32 master weights w[co][t][ci] (t = 3 ky + kx):
// forward  wf[t][co][ci'] (ci' padded to CINP with zeros);
// data grad wd[t][ci][co] = w[co][8 - t][ci].
__global__ void k_pack_weights(const float *__restrict__ w, int cout, int cin, int cinp,
                               uint16_t *__restrict__ wf, uint16_t *__restrict__ wd)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 9 * cout * cinp) return;
    const int t = e / (cout * cinp), co = (e / cinp) % cout, ci = e % cinp;
    const float v = ci < cin ? w[(co * 9 + t) * cin + ci] : 0.0f;
    wf[e] = bf16_bits(v);
    if (wd && ci < cin) wd[((8 - t) * cin + ci) * cout + co] = bf16_bits(v);
}

// Adam with bias correction; p, m, v, g FP32. omb1 = 1 - b1 and omb2 = 1 - b2
// come rounded from their exact values (1 - fl32(0.999) is 1.3e-5 off).
__global__ void k_adam(float *__restrict__ p, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, int n, float lr, float b1, float b2,
                       float omb1, float omb2, float eps, float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + omb1 * gi;
    const float vi = b2 * v[i] + omb2 * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// Per-frame confidence score of a low-res input: mean squared forward
// difference (x and y) of the four input channels.
__global__ __launch_bounds__(256) void k_up_score(const float *__restrict__ x0f, int h, int w,
                                                  float *__restrict__ score)
{
    const int n = blockIdx.x;
    const float4 *xi = reinterpret_cast<const float4 *>(x0f) + (int64_t)n * h * w;
    float s = 0.0f;
    for (int p = threadIdx.x; p < h * w; p += 256) {
        const int y = p / w, x = p % w;
        const float4 a = xi[p];
        if (x + 1 < w) {
            const float4 b = xi[p + 1];
            s += (a.x - b.x) * (a.x - b.x) + (a.y - b.y) * (a.y - b.y) + (a.z - b.z) * (a.z - b.z) +
                 (a.w - b.w) * (a.w - b.w);
        }
        if (y + 1 < h) {
            const float4 b = xi[p + w];
            s += (a.x - b.x) * (a.x - b.x) + (a.y - b.y) * (a.y - b.y) + (a.z - b.z) * (a.z - b.z) +
                 (a.w - b.w) * (a.w - b.w);
        }
    }
    __shared__ float r[256];
    r[threadIdx.x] = s;
    __syncthreads();
    for (int d = 128; d > 0; d >>= 1) {
        if ((int)threadIdx.x < d) r[threadIdx.x] += r[threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0) score[n] = r[0] / (float)(h * w);
}

// Per-frame PSNR (dB) of clamped RGB against a reference render.
__global__ __launch_bounds__(256) void k_frame_psnr(const float *__restrict__ a,
                                                    const float *__restrict__ b, int64_t npix,
                                                    float *__restrict__ out)
{
    const int n = blockIdx.x;
    const float *pa = a + (int64_t)n * npix * 3, *pb = b + (int64_t)n * npix * 3;
    float s = 0.0f;
    for (int64_t i = threadIdx.x; i < npix * 3; i += 256) {
        const float d = fminf(fmaxf(pa[i], 0.0f), 1.0f) - fminf(fmaxf(pb[i], 0.0f), 1.0f);
        s += d * d;
    }
    __shared__ float r[256];
    r[threadIdx.x] = s;
    __syncthreads();
    for (int d = 128; d > 0; d >>= 1) {
        if ((int)threadIdx.x < d) r[threadIdx.x] += r[threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const float mse = fmaxf(r[0] / (float)(npix * 3), 1e-12f);
        out[n] = -10.0f * log10f(mse);
    }
}

// ---------------------------------------------------------------- launch --
static void tiles_of(int h, int w, int &tx, int &ty)
{
    tx = (w + kTX - 1) / kTX;
    ty = (h + kTY - 1) / kTY;
}

int up_conv_blocks(int n, int h, int w)
{
    int tx, ty;
    tiles_of(h, w, tx, ty);
    return n * tx * ty;
}

void launch_up_input(const float *rgb, const float *depth, int64_t npix, float *x0f,
                     uint16_t *x0b, hipStream_t st)
{
    hipLaunchKernelGGL(k_up_input, dim3((unsigned)((npix + 255) / 256)), dim3(256), 0, st, rgb,
                       depth, npix, x0f, x0b);
}

void launch_up_conv(int cin, int cout, int epi, const uint16_t *in, const uint16_t *wt,
                    const float *bias, int n, int h, int w, const uint16_t *mask, void *out,
                    hipStream_t st, const float *x0f, float *rgb, float *depth)
{
    int tx, ty;
    tiles_of(h, w, tx, ty);
    dim3 grid(n * tx * ty), block(256);
    const HeadOut head{x0f, rgb, depth};
    if (epi == UP_EPI_RELU_BF16_IN4 && cin == 32 && cout == 32) {
        hipLaunchKernelGGL((k_conv3x3<32, 32, EPI_RELU_BF16, true>), grid, block, 0, st, in, wt,
                           bias, h, w, tx, ty, mask, out, head);
        return;
    }
#define GS_CONV(CI, CO, E)                                                                     \
    if (cin == CI && cout == CO && epi == E) {                                                 \
        hipLaunchKernelGGL((k_conv3x3<CI, CO, E>), grid, block, 0, st, in, wt, bias, h, w, tx, \
                           ty, mask, out, head);                                               \
        return;                                                                                \
    }
    GS_CONV(32, 32, EPI_RELU_BF16)
    GS_CONV(32, 64, EPI_F32)
    GS_CONV(32, 64, EPI_HEAD)
    GS_CONV(64, 32, EPI_MASK_BF16)
    GS_CONV(32, 32, EPI_MASK_BF16)
#undef GS_CONV
}

void launch_up_wgrad(int cin, int cout, const uint16_t *x, const uint16_t *dy, int n, int h,
                     int w, float *part, float *partb, hipStream_t st)
{
    int tx, ty;
    tiles_of(h, w, tx, ty);
    dim3 grid(n * tx * ty), block(256);
    if (cin == 32 && cout == 32)
        hipLaunchKernelGGL((k_conv3x3_wgrad<32, 32>), grid, block, 0, st, x, dy, h, w, tx, ty,
                           part, partb);
    else if (cin == 32 && cout == 64)
        hipLaunchKernelGGL((k_conv3x3_wgrad<32, 64>), grid, block, 0, st, x, dy, h, w, tx, ty,
                           part, partb);
}

void launch_sum_partials(float *part, int nblk, int len, float *grad, hipStream_t st)
{
    // runs of at least 32 blocks, at most 256 runs
    const int nr0 = std::max(1, std::min(256, nblk / 32));
    const int L = (nblk + nr0 - 1) / nr0;
    const int nruns = (nblk + L - 1) / L;
    const unsigned gx = (unsigned)((len + 255) / 256);
    hipLaunchKernelGGL(k_sum_runs, dim3(gx, (unsigned)nruns), dim3(256), 0, st, part, nblk, len, L);
    hipLaunchKernelGGL(k_sum_run_heads, dim3(gx), dim3(256), 0, st, part, nruns, len, L, grad);
}

int up_head_blocks(int n, int h, int w) { return (int)(((int64_t)n * h * w * 16 + 255) / 256); }

void launch_up_head(bool train, const float *x0f, const float *y, int h, int w, int n,
                    float *rgb, float *depth, const float *t_rgb, const float *t_depth,
                    float *loss_part, uint16_t *dy, hipStream_t st)
{
    const int blocks = up_head_blocks(n, h, w);
    const float inv = 1.0f / (float)((int64_t)n * h * w * 16);
    if (train)
        hipLaunchKernelGGL(k_up_head<true>, dim3(blocks), dim3(256), 0, st, x0f, y, h, w, n, rgb,
                           depth, t_rgb, t_depth, inv, loss_part, dy);
    else
        hipLaunchKernelGGL(k_up_head<false>, dim3(blocks), dim3(256), 0, st, x0f, y, h, w, n, rgb,
                           depth, t_rgb, t_depth, inv, loss_part, dy);
}

void launch_pack_weights(const float *w, int cout, int cin, int cinp, uint16_t *wf, uint16_t *wd,
                         hipStream_t st)
{
    const int n = 9 * cout * cinp;
    hipLaunchKernelGGL(k_pack_weights, dim3((n + 255) / 256), dim3(256), 0, st, w, cout, cin, cinp,
                       wf, wd);
}

void launch_adam(float *p, float *m, float *v, const float *g, int n, float lr, int step,
                 hipStream_t st)
{
    // Kingma & Ba defaults; the bias corrections 1 / (1 - b^step) in FP64
    const double b1 = 0.9, b2 = 0.999;
    const float c1 = (float)(1.0 / (1.0 - std::pow(b1, (double)step)));
    const float c2 = (float)(1.0 / (1.0 - std::pow(b2, (double)step)));
    hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, st, p, m, v, g, n, lr,
                       (float)b1, (float)b2, (float)(1.0 - b1), (float)(1.0 - b2), 1e-8f, c1, c2);
}

void launch_up_score(const float *x0f, int n, int h, int w, float *score, hipStream_t st)
{
    hipLaunchKernelGGL(k_up_score, dim3(n), dim3(256), 0, st, x0f, h, w, score);
}

// Fallback flags of the upsampled form: mask[i] = 1 when camera i's score is
// not at most the threshold (NaN scores are flagged), and *count (zeroed by
// the caller) gains the number of flagged cameras.
__global__ __launch_bounds__(256) void k_up_flag(const float *__restrict__ score, int n, float thr,
                                                 uint32_t *__restrict__ mask,
                                                 uint32_t *__restrict__ count)
{
    const int i = blockIdx.x * 256 + (int)threadIdx.x;
    const bool f = i < n && !(score[i] <= thr);
    if (i < n) mask[i] = f ? 1u : 0u;
    const uint64_t b = __ballot(f);
    if (__lane_id() == 0 && b) atomicAdd(count, (uint32_t)__popcll(b));
}

void launch_up_flag(const float *score, int n, float thr, uint32_t *mask, uint32_t *count,
                    hipStream_t st)
{
    hipLaunchKernelGGL(k_up_flag, dim3((n + 255) / 256), dim3(256), 0, st, score, n, thr, mask,
                       count);
}

void launch_frame_psnr(const float *a, const float *b, int n, int64_t npix, float *out,
                       hipStream_t st)
{
    hipLaunchKernelGGL(k_frame_psnr, dim3(n), dim3(256), 0, st, a, b, npix, out);
}

}  // namespace gs
