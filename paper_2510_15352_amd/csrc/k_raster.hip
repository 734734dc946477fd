// The front-to-back rasteriser (every wave walks its own culled copy of the
// tile's list), as a one-block-per-tile grid or a persistent work queue;
// motion-blur pose and finishing kernels.
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

// -------------------------------------------------------------- raster --
// One block per (camera, tile); each wave owns an 8x8 pixel block, one pixel
// per lane, and walks the tile's list on its own (no block barrier). Per
// batch of B records, 64 at a time with one record per lane, the wave keeps
// only the records that can reach the bounding rectangle of its live pixels
// (may_touch; pixels outside the image and finished pixels are not live),
// appends them in list order to a wave-private LDS list together with the
// record's block-relative offsets E0, F0, then walks that list front to
// back. A skipped record has alpha < 1/255 at every live pixel of the wave
// and leaves the finished ones unchanged, so the per-pixel result is the
// same as walking the full tile list. A wave stops once all of its pixels
// are done.
template <int TW, int TH, int B, bool COUNT = false>
__device__ __forceinline__ void raster_tile(int cl, int tile, const RasterArgs &a, float4 *sR0,
                                            float4 *sR1, float2 *sEF,
                                            RenderFlags *cnt = nullptr)
{
    static_assert(TW % 8 == 0 && TH % 8 == 0, "tiles are made of 8x8 wave blocks");
    static_assert(B % 64 == 0, "batches are whole sets of 64 records");
    constexpr int SX = TW / 8;
    // tiles of at most two wave blocks (small splats, long lists) also test
    // each record's pixel box against the live lanes
    constexpr bool kBoxCull = TW * TH <= 128;
    // a masked-out camera keeps its frame (block-uniform test, before any work)
    if (a.cam_mask && a.cam_mask[a.cam_global[cl]] == 0u) return;
    // wave-uniform: kept in scalar registers with everything derived from it
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const uint32_t lane = __lane_id();
    const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
    const int wx0 = tx * TW + (wave % SX) * 8, wy0 = ty * TH + (wave / SX) * 8;
    const int pxi = wx0 + (int)(lane & 7u), pyi = wy0 + (int)(lane >> 3);
    const bool inside = pxi < a.W && pyi < a.H;
    const float lx = (float)(lane & 7u), ly = (float)(lane >> 3);
    const float cx0 = (float)wx0 + 0.5f, cy0 = (float)wy0 + 0.5f;
    const uint2 rg = a.ranges[(uint32_t)cl * (uint32_t)a.tiles_per_cam + (uint32_t)tile];
    float4 *L0 = sR0 + wave * B;
    float4 *L1 = sR1 + wave * B;
    float2 *LE = sEF + wave * B;
    const uint64_t lt = lanemask_lt();
    Pixel s;
    s.U = inside ? kAlphaMax : -1.0f;
    s.r = 0.0f; s.g = 0.0f; s.b = 0.0f; s.zw = 0.0f;
    uint32_t n_eval = 0, n_contrib = 0, n_issue = 0;
    // Record of the lane in the current set of 64, in registers. The next
    // set's slot is loaded before the culling and its record after it, so
    // both are in flight while the wave culls and walks.
    bool pf = rg.x + lane < rg.y;
    uint32_t pslot = pf ? a.ivals[rg.x + lane] : 0u;
    float4 pA = make_float4(0.f, 0.f, 0.f, 0.f), pB = pA, pC = pA;
    if (pf) {
        pA = a.rec[(size_t)pslot * 3];
        pB = a.rec[(size_t)pslot * 3 + 1];
        pC = a.rec[(size_t)pslot * 3 + 2];
    }
    uint64_t lm = __ballot(s.U > 0.0f);
    for (uint32_t base = rg.x; lm != 0ull && base < rg.y; base += B) {
        // The batch is culled against the bounding rectangle of the wave's
        // live pixels (lane = 8 row + column): rows from the first and last
        // live lane, columns from the OR of the eight rows. A finished pixel
        // is left unchanged by every record, so a record that reaches none
        // of the live ones is dropped like one outside the block.
        const int r0 = __builtin_ctzll(lm) >> 3, r1 = (63 - __builtin_clzll(lm)) >> 3;
        uint32_t cm = (uint32_t)lm | (uint32_t)(lm >> 32);
        cm |= cm >> 16;
        cm |= cm >> 8;
        const int c0 = __builtin_ctz(cm & 0xffu), c1 = 31 - __builtin_clz(cm & 0xffu);
        const float ox = (float)c0, oy = (float)r0;
        const float lw = (float)(c1 - c0), lh = (float)(r1 - r0);
        int n = 0;
#pragma unroll
        for (int sb = 0; sb < B / 64; ++sb) {
            const uint32_t j0 = base + (uint32_t)(sb * 64);
            if (j0 >= rg.y) break;
            const bool have = pf;
            const float4 A = pA, Bv = pB, C = pC;
            const uint32_t nj = j0 + 64u;
            pf = nj + lane < rg.y;
            if (pf) pslot = a.ivals[nj + lane];
            // R0 = (ex, ey, fy, log2 0.99 - log2 o), R1 = (r, g, b, z); centre (u, v),
            // reach tau
            bool hit = false;
            float4 R0 = A, R1 = A;
            float E0 = 0.0f, F0 = 0.0f;
            if (have) {
                R0 = make_float4(A.z, A.w, Bv.x, kLog2AlphaMax - __builtin_amdgcn_logf(Bv.y));
                R1 = make_float4(Bv.z, Bv.w, C.x, C.y);
                const float Xw = cx0 - A.x, Yw = cy0 - A.y;
                hit = may_touch(R0.x, R0.y, R0.z, Xw + ox, Yw + oy, lw, lh, C.z);
                if (kBoxCull && hit) {
                    // The box of the ellipse q <= tau (half-widths
                    // sqrt(tau) sqrt(ey^2 + fy^2) / (ex fy) and sqrt(tau) / fy,
                    // widened for rounding) as a lane mask, against the
                    // live lanes themselves rather than their rectangle.
                    const float rt = fmaf(__builtin_sqrtf(C.z), 1.0001f, 1e-3f);
                    const float ify = __builtin_amdgcn_rcpf(R0.z);
                    const float hy = rt * ify;
                    const float hx = rt * ify * __builtin_sqrtf(fmaf(R0.y, R0.y, R0.z * R0.z)) *
                                     __builtin_amdgcn_rcpf(R0.x);
                    const int c0 = (int)ceilf(fmaxf(-Xw - hx, 0.0f));
                    const int c1 = (int)floorf(fminf(hx - Xw, 7.0f));
                    const int r0 = (int)ceilf(fmaxf(-Yw - hy, 0.0f));
                    const int r1 = (int)floorf(fminf(hy - Yw, 7.0f));
                    if (c0 > c1 || r0 > r1) {
                        hit = false;
                    } else {
                        const uint32_t cb = (2u << c1) - (1u << c0);
                        const uint64_t rb = (~0ull >> (8 * (7 - r1))) & (~0ull << (8 * r0));
                        hit = ((uint64_t)cb * 0x0101010101010101ull & rb & lm) != 0ull;
                    }
                }
                E0 = fmaf(R0.x, Xw, R0.y * Yw);
                F0 = R0.z * Yw;
            }
            const uint64_t m = __ballot(hit);
            if (hit) {
                const int p = n + (int)__popcll(m & lt);
                L0[p] = R0;
                L1[p] = R1;
                LE[p] = make_float2(E0, F0);
            }
            n += (int)__popcll(m);
            if (pf) {
                pA = a.rec[(size_t)pslot * 3];
                pB = a.rec[(size_t)pslot * 3 + 1];
                pC = a.rec[(size_t)pslot * 3 + 2];
            }
        }
        __builtin_amdgcn_wave_barrier();  // list entries written before they are read
        // four list entries per step, a wave-level completion test after
        // each step, then the remainder one by one
        int k = 0;
        for (; k + 4 <= n; k += 4) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const float4 R0 = L0[k + u], R1 = L1[k + u];
                const float2 ef = LE[k + u];
                if (COUNT) {
                    n_eval += s.U > 0.0f;
                    ++n_issue;
                    n_contrib += composite(s, lx, ly, R0, R1, ef.x, ef.y);
                } else {
                    composite(s, lx, ly, R0, R1, ef.x, ef.y);
                }
            }
            if (__ballot(s.U > 0.0f) == 0ull) break;
        }
        if (__ballot(s.U > 0.0f) != 0ull) {
            for (; k < n; ++k) {
                const float4 R0 = L0[k], R1 = L1[k];
                const float2 ef = LE[k];
                if (COUNT) {
                    n_eval += s.U > 0.0f;
                    ++n_issue;
                    n_contrib += composite(s, lx, ly, R0, R1, ef.x, ef.y);
                } else {
                    composite(s, lx, ly, R0, R1, ef.x, ef.y);
                }
            }
        }
        lm = __ballot(s.U > 0.0f);
        __builtin_amdgcn_wave_barrier();  // list read before the next batch rewrites it
    }
    if (COUNT) {
        // one atomic per wave
        uint64_t e = n_eval, c = n_contrib, is = n_issue;
        for (int d = 32; d > 0; d >>= 1) {
            e += __shfl_down(e, d, 64);
            c += __shfl_down(c, d, 64);
            is += __shfl_down(is, d, 64);
        }
        if (lane == 0) {
            atomicAdd(&cnt->pairs_eval, (unsigned long long)e);
            atomicAdd(&cnt->pairs_contrib, (unsigned long long)c);
            atomicAdd(&cnt->pairs_issued, (unsigned long long)is);
        }
    }
    if (inside) {
        const int64_t cg = a.cam_global[cl];
        const int64_t pix = (cg * a.H + pyi) * (int64_t)a.W + pxi;
        const float T = fabsf(s.U) / kAlphaMax;
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

// one list of B entries per wave: R0, R1 and (E0, F0)
#define GS_RASTER_SHARED                       \
    __shared__ float4 sR0[(TW * TH / 64) * B]; \
    __shared__ float4 sR1[(TW * TH / 64) * B]; \
    __shared__ float2 sEF[(TW * TH / 64) * B];

// Grid forms: one block per (camera, tile) item, item = block index.
__device__ __forceinline__ uint32_t xcd_item() { return blockIdx.x; }

template <int TW, int TH, int B>
__global__ __launch_bounds__(TW *TH) __attribute__((amdgpu_waves_per_eu(8, 8)))
void k_raster(RasterArgs a, uint32_t n_items)
{
    GS_RASTER_SHARED
    const uint32_t item = xcd_item();
    if (item >= n_items) return;
    raster_tile<TW, TH, B>((int)(item / (uint32_t)a.tiles_per_cam),
                           (int)(item % (uint32_t)a.tiles_per_cam), a, sR0, sR1, sEF);
}

// Instrumented grid form: same per-pixel arithmetic, plus counts of
// evaluated and accumulated (pixel, Gaussian) pairs.
template <int TW, int TH, int B>
__global__ __launch_bounds__(TW *TH) void k_raster_count(RasterArgs a, uint32_t n_items,
                                                         RenderFlags *cnt)
{
    GS_RASTER_SHARED
    const uint32_t item = xcd_item();
    if (item >= n_items) return;
    raster_tile<TW, TH, B, true>((int)(item / (uint32_t)a.tiles_per_cam),
                                 (int)(item % (uint32_t)a.tiles_per_cam), a, sR0, sR1, sEF, cnt);
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
                               (int)(item % (uint32_t)a.tiles_per_cam), a, sR0, sR1, sEF);
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
        // separately rounded product and difference: no fused multiply-add
#pragma clang fp contract(off)
        o[r * 4 + 0] = p[r * 4 + 0];
        o[r * 4 + 1] = p[r * 4 + 1];
        o[r * 4 + 2] = p[r * 4 + 2];
        const float step = vel[(int64_t)i * 3 + r] * dt;
        o[r * 4 + 3] = p[r * 4 + 3] - step;
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

#define GS_RASTER_CASES(X) \
    X(16, 16, 64) X(16, 16, 128) X(16, 16, 256) \
    X(32, 8, 64) X(32, 8, 128) X(32, 8, 256) \
    X(8, 8, 64) X(16, 8, 64) X(16, 8, 128) \
    X(32, 16, 64) X(32, 16, 128)

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
    const uint32_t grid = n_items;
#define X(TW_, TH_, B_)                                                                          \
    if (tw == TW_ && th == TH_ && b == B_) {                                                     \
        if (count) {                                                                             \
            hipLaunchKernelGGL((k_raster_count<TW_, TH_, B_>), dim3(grid), dim3(TW_ * TH_), 0,  \
                               st, a, n_items, count);                                           \
        } else if (persistent) {                                                                 \
            launch_zero_u32(queue, 1, st);                                                       \
            int blocks = persistent_blocks;                                                      \
            if ((uint32_t)blocks > n_items) blocks = (int)n_items;                               \
            if (blocks < 1) blocks = 1;                                                          \
            hipLaunchKernelGGL((k_raster_persistent<TW_, TH_, B_>), dim3(blocks),               \
                               dim3(TW_ * TH_), 0, st, a, queue, n_items);                       \
        } else {                                                                                 \
            hipLaunchKernelGGL((k_raster<TW_, TH_, B_>), dim3(grid), dim3(TW_ * TH_), 0, st, a,  \
                               n_items);                                                         \
        }                                                                                        \
        return;                                                                                  \
    }
    GS_RASTER_CASES(X)
#undef X
}

}  // namespace gs
