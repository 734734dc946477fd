// Tile binning (instance emission, tile ranges) and the LDS-staged
// front-to-back rasteriser, as a one-block-per-tile grid or a persistent
// work queue.
#include <algorithm>

#include "gs_device.h"
#include "kernels.h"

namespace gs {

// counts[0] = visible pairs, counts[1] = instances, counts[2] = instances
// kept (min(instances, cap)); flags accumulate over the chunks of a render.
__global__ void k_finalize_counts(uint32_t *counts, uint32_t cap, RenderFlags *flags)
{
    const uint32_t inst = counts[1];
    counts[2] = inst < cap ? inst : cap;
    if (inst > cap) flags->overflow = 1;
    if (inst > flags->max_inst) flags->max_inst = inst;
    flags->visible += counts[0];
    flags->instances += inst;
}

__global__ void k_zero_u32(uint32_t *p, uint64_t n)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// -------------------------------------------------------------- ranges --
__global__ __launch_bounds__(256) void k_ranges(const uint32_t *__restrict__ ikeys,
                                                const uint32_t *__restrict__ n_dev,
                                                uint2 *__restrict__ ranges)
{
    const uint32_t n = *n_dev;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint32_t k = ikeys[i];
        if (i == 0 || ikeys[i - 1] != k) ranges[k].x = i;
        if (i + 1 == n || ikeys[i + 1] != k) ranges[k].y = i + 1;
    }
}

// -------------------------------------------------------------- raster --
// One block per (camera, tile); each wave owns an 8x8 pixel sub-tile, one
// pixel per lane. Per LDS batch of B records (staged in the tile-local form
// of the compositing step), every wave first keeps only the records that can
// reach its 8x8 rectangle (may_touch_local, 64 records per ballot, compacted
// with mbcnt into a per-wave list of LDS byte offsets), then walks that list
// front to back. A skipped record has alpha < 1/255 at every pixel of the
// wave, so the per-pixel result is the same as walking the full tile list.
// The block stops when a barrier count says every pixel is done.
template <int TW, int TH, int B, bool COUNT = false>
__device__ __forceinline__ void raster_tile(int cl, int tile, const RasterArgs &a, float4 *sA,
                                            float4 *sB, float4 *sC, float *sT, uint32_t *sL,
                                            RenderFlags *cnt = nullptr)
{
    static_assert(TW % 8 == 0 && TH % 8 == 0, "tiles are made of 8x8 wave sub-tiles");
    constexpr int NT = TW * TH;
    constexpr int SX = TW / 8;
    const int wave = (int)threadIdx.x >> 6;
    const uint32_t lane = __lane_id();
    const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
    const int ox = tx * TW, oy = ty * TH;
    // the wave's pixel rectangle in tile-local pixels, clipped to the image
    const int lx0 = (wave % SX) * 8, ly0 = (wave / SX) * 8;
    const int lx1 = min(lx0 + 7, a.W - 1 - ox), ly1 = min(ly0 + 7, a.H - 1 - oy);
    const int lxi = lx0 + (int)(lane & 7u), lyi = ly0 + (int)(lane >> 3);
    const int pxi = ox + lxi, pyi = oy + lyi;
    const bool inside = pxi < a.W && pyi < a.H;
    const float lx = (float)lxi, ly = (float)lyi;
    const float fox = (float)ox + 0.5f, foy = (float)oy + 0.5f;
    const uint2 rg = a.ranges[(uint32_t)cl * (uint32_t)a.tiles_per_cam + (uint32_t)tile];
    uint32_t *list = sL + wave * B;
    const uint64_t lt = lanemask_lt();
    const char *lds = reinterpret_cast<const char *>(sA);
    Pixel s;
    s.T = inside ? 1.0f : -1.0f;
    s.r = 0.0f; s.g = 0.0f; s.b = 0.0f; s.zw = 0.0f;
    uint32_t n_eval = 0, n_contrib = 0;
    for (uint32_t base = rg.x; base < rg.y; base += B) {
        const int cnt_b = (int)min((uint32_t)B, rg.y - base);
        __syncthreads();
        for (int j = (int)threadIdx.x; j < cnt_b; j += NT) {
            const uint32_t slot = a.ivals[base + j];
            const float4 A = a.recA[slot], Bv = a.recB[slot], C = a.recC[slot];
            const float Xo = fox - A.x, Yo = foy - A.y;
            sA[j] = make_float4(A.z, A.w, fmaf(A.z, Xo, A.w * Yo), Bv.x);
            sB[j] = make_float4(Bv.x * Yo, -__builtin_amdgcn_logf(Bv.y), Bv.z, Bv.w);
            sC[j] = make_float4(C.x, C.y, Xo, Yo);
            sT[j] = C.z;
        }
        __syncthreads();
        int n = 0;
        if (__ballot(s.T > 0.0f) != 0ull) {
            for (int c0 = 0; c0 < cnt_b; c0 += 64) {
                const int j = c0 + (int)lane;
                bool hit = false;
                if (j < cnt_b) {
                    const float4 A = sA[j], C = sC[j];
                    hit = may_touch_local(A.x, A.y, A.w, C.z, C.w, sT[j], lx0, lx1, ly0, ly1);
                }
                const uint64_t m = __ballot(hit);
                if (hit) list[n + __popcll(m & lt)] = (uint32_t)j * 16u;
                n += __popcll(m);
            }
        }
        __syncthreads();  // per-wave lists written before they are read
        if (__ballot(s.T > 0.0f) != 0ull) {
            // four list entries per step (one 16-byte LDS read), a wave-level
            // completion test after each step, then the remainder one by one
            int k = 0;
            bool live = true;
            for (; k + 4 <= n; k += 4) {
                const uint4 jj = *reinterpret_cast<const uint4 *>(list + k);
                const uint32_t off[4] = {jj.x, jj.y, jj.z, jj.w};
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const float4 A = *reinterpret_cast<const float4 *>(lds + off[u]);
                    const float4 Bv = *reinterpret_cast<const float4 *>(lds + B * 16 + off[u]);
                    const float2 C = *reinterpret_cast<const float2 *>(lds + 2 * B * 16 + off[u]);
                    if (COUNT) {
                        n_eval += s.T > 0.0f;
                        n_contrib += composite(s, lx, ly, A, Bv, C);
                    } else {
                        composite(s, lx, ly, A, Bv, C);
                    }
                }
                if (__ballot(s.T > 0.0f) == 0ull) {
                    live = false;
                    break;
                }
            }
            for (; live && k < n; ++k) {
                const uint32_t o = list[k];
                const float4 A = *reinterpret_cast<const float4 *>(lds + o);
                const float4 Bv = *reinterpret_cast<const float4 *>(lds + B * 16 + o);
                const float2 C = *reinterpret_cast<const float2 *>(lds + 2 * B * 16 + o);
                if (COUNT) {
                    n_eval += s.T > 0.0f;
                    n_contrib += composite(s, lx, ly, A, Bv, C);
                } else {
                    composite(s, lx, ly, A, Bv, C);
                }
            }
        }
        if (__syncthreads_count(s.T > 0.0f) == 0) break;
    }
    if (COUNT) {
        // one atomic per wave
        uint64_t e = n_eval, c = n_contrib;
        for (int d = 32; d > 0; d >>= 1) {
            e += __shfl_down(e, d, 64);
            c += __shfl_down(c, d, 64);
        }
        if (lane == 0) {
            atomicAdd(&cnt->pairs_eval, (unsigned long long)e);
            atomicAdd(&cnt->pairs_contrib, (unsigned long long)c);
        }
    }
    if (inside) {
        const int64_t cg = a.cam_global[cl];
        const int64_t pix = (cg * a.H + pyi) * (int64_t)a.W + pxi;
        const float T = fabsf(s.T);
        const float accw = 1.0f - T;
        const float r = fmaf(T, a.bg_r, s.r), g = fmaf(T, a.bg_g, s.g), b = fmaf(T, a.bg_b, s.b);
        if (a.blend == 0) {
            a.rgb[pix * 3 + 0] = r;
            a.rgb[pix * 3 + 1] = g;
            a.rgb[pix * 3 + 2] = b;
            a.depth[pix] = accw > 0.0f ? s.zw / accw : 0.0f;
            if (a.alpha) a.alpha[pix] = accw;
        } else if (a.blend == 1) {
            a.rgb[pix * 3 + 0] = a.blend_w * r;
            a.rgb[pix * 3 + 1] = a.blend_w * g;
            a.rgb[pix * 3 + 2] = a.blend_w * b;
            a.depth[pix] = s.zw;
            a.alpha[pix] = accw;
        } else {
            a.rgb[pix * 3 + 0] = fmaf(a.blend_w, r, a.rgb[pix * 3 + 0]);
            a.rgb[pix * 3 + 1] = fmaf(a.blend_w, g, a.rgb[pix * 3 + 1]);
            a.rgb[pix * 3 + 2] = fmaf(a.blend_w, b, a.rgb[pix * 3 + 2]);
            a.depth[pix] += s.zw;
            a.alpha[pix] += accw;
        }
    }
}

// sA, sB, sC are consecutive (the walk addresses them from sA's base).
#define GS_RASTER_SHARED                                        \
    __shared__ float4 sRec[3 * B];                              \
    __shared__ float sT[B];                                     \
    __shared__ __attribute__((aligned(16))) uint32_t sL[(TW * TH / 64) * B]; \
    float4 *sA = sRec, *sB = sRec + B, *sC = sRec + 2 * B;

template <int TW, int TH, int B>
__global__ __launch_bounds__(TW *TH) void k_raster(RasterArgs a)
{
    GS_RASTER_SHARED
    raster_tile<TW, TH, B>((int)blockIdx.y, (int)blockIdx.x, a, sA, sB, sC, sT, sL);
}

// Instrumented grid form: same per-pixel arithmetic, plus counts of
// evaluated and accumulated (pixel, Gaussian) pairs.
template <int TW, int TH, int B>
__global__ __launch_bounds__(TW *TH) void k_raster_count(RasterArgs a, RenderFlags *cnt)
{
    GS_RASTER_SHARED
    raster_tile<TW, TH, B, true>((int)blockIdx.y, (int)blockIdx.x, a, sA, sB, sC, sT, sL, cnt);
}

// Persistent form: a grid sized to the resident capacity pulls
// (camera, tile) items from a device counter until they run out.
template <int TW, int TH, int B>
__global__ __launch_bounds__(TW *TH) void k_raster_persistent(RasterArgs a, uint32_t *queue,
                                                              uint32_t n_items)
{
    GS_RASTER_SHARED
    __shared__ uint32_t s_item;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(queue, 1u);
        __syncthreads();
        const uint32_t item = s_item;
        __syncthreads();
        if (item >= n_items) break;
        raster_tile<TW, TH, B>((int)(item / (uint32_t)a.tiles_per_cam),
                               (int)(item % (uint32_t)a.tiles_per_cam), a, sA, sB, sC, sT, sL);
    }
}

// ----------------------------------------------------------- motion blur --
__global__ void k_blur_poses(const float *__restrict__ poses, const float *__restrict__ vel,
                             int n_cams, const float *__restrict__ offs, int K,
                             float *__restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n_cams * K) return;
    const int k = (int)(t / n_cams), i = (int)(t - (int64_t)k * n_cams);
    const float *p = poses + (int64_t)i * 12;
    float *o = out + t * 12;
    const float dt = offs[k];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        o[r * 4 + 0] = p[r * 4 + 0];
        o[r * 4 + 1] = p[r * 4 + 1];
        o[r * 4 + 2] = p[r * 4 + 2];
        // separately rounded product and difference (no contraction)
        o[r * 4 + 3] = __fsub_rn(p[r * 4 + 3], __fmul_rn(vel[(int64_t)i * 3 + r], dt));
    }
}

__global__ void k_blur_finalize(float *__restrict__ depth, const float *__restrict__ asum,
                                float *__restrict__ alpha_out, int64_t n_px, float inv_k)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_px;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float s = asum[i];
        depth[i] = s > 0.0f ? depth[i] / s : 0.0f;
        if (alpha_out) alpha_out[i] = s * inv_k;
    }
}

void launch_blur_poses(const float *poses, const float *vel, int n_cams, const float *offs, int K,
                       float *out, hipStream_t st)
{
    const int64_t n = (int64_t)n_cams * K;
    hipLaunchKernelGGL(k_blur_poses, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, poses,
                       vel, n_cams, offs, K, out);
}

void launch_blur_finalize(float *depth, float *alpha_sum, float *alpha_out, int64_t n_px,
                          float inv_k, hipStream_t st)
{
    const int64_t blocks = std::min<int64_t>((n_px + 255) / 256, 65536);
    hipLaunchKernelGGL(k_blur_finalize, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256),
                       0, st, depth, alpha_sum, alpha_out, n_px, inv_k);
}

// --------------------------------------------------------------- launch --
void launch_finalize_counts(uint32_t *counts, uint32_t cap, RenderFlags *flags, hipStream_t st)
{
    hipLaunchKernelGGL(k_finalize_counts, dim3(1), dim3(1), 0, st, counts, cap, flags);
}

void launch_zero_u32(uint32_t *p, uint64_t n, hipStream_t st)
{
    if (n == 0) return;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)blocks), dim3(256), 0, st, p, n);
}

void launch_ranges(const uint32_t *ikeys, const uint32_t *n_dev, uint2 *ranges, uint32_t n_max,
                   hipStream_t st)
{
    uint32_t blocks = (n_max + 255) / 256;
    blocks = blocks < 1 ? 1 : (blocks > 16384 ? 16384 : blocks);
    hipLaunchKernelGGL(k_ranges, dim3(blocks), dim3(256), 0, st, ikeys, n_dev, ranges);
}

#define GS_RASTER_CASES(X) \
    X(16, 16, 64) X(16, 16, 128) X(16, 16, 256) \
    X(32, 8, 64) X(32, 8, 128) X(32, 8, 256) \
    X(8, 8, 64) X(16, 8, 64) X(16, 8, 128) \
    X(32, 16, 128) X(32, 16, 256)

bool raster_supported(int tw, int th, int b)
{
#define X(TW_, TH_, B_) if (tw == TW_ && th == TH_ && b == B_) return true;
    GS_RASTER_CASES(X)
#undef X
    return false;
}

int raster_occupancy(int tw, int th, int b)
{
    int blocks = 0;
#define X(TW_, TH_, B_)                                                                       \
    if (tw == TW_ && th == TH_ && b == B_) {                                                  \
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(                                     \
                &blocks, (const void *)k_raster_persistent<TW_, TH_, B_>, TW_ * TH_, 0) !=    \
            hipSuccess)                                                                       \
            blocks = 1;                                                                       \
    }
    GS_RASTER_CASES(X)
#undef X
    return blocks < 1 ? 1 : blocks;
}

void launch_raster(int tw, int th, int b, bool persistent, const RasterArgs &a, int n_cams,
                   uint32_t *queue, int persistent_blocks, RenderFlags *count, hipStream_t st)
{
    const int tiles = a.tiles_per_cam;
    const uint32_t n_items = (uint32_t)tiles * (uint32_t)n_cams;
#define X(TW_, TH_, B_)                                                                          \
    if (tw == TW_ && th == TH_ && b == B_) {                                                     \
        if (count) {                                                                             \
            hipLaunchKernelGGL((k_raster_count<TW_, TH_, B_>), dim3(tiles, n_cams),             \
                               dim3(TW_ * TH_), 0, st, a, count);                                \
        } else if (persistent) {                                                                 \
            launch_zero_u32(queue, 1, st);                                                       \
            int blocks = persistent_blocks;                                                      \
            if ((uint32_t)blocks > n_items) blocks = (int)n_items;                               \
            if (blocks < 1) blocks = 1;                                                          \
            hipLaunchKernelGGL((k_raster_persistent<TW_, TH_, B_>), dim3(blocks),               \
                               dim3(TW_ * TH_), 0, st, a, queue, n_items);                       \
        } else {                                                                                 \
            hipLaunchKernelGGL((k_raster<TW_, TH_, B_>), dim3(tiles, n_cams), dim3(TW_ * TH_), 0, \
                               st, a);                                                           \
        }                                                                                        \
        return;                                                                                  \
    }
    GS_RASTER_CASES(X)
#undef X
}

}  // namespace gs
