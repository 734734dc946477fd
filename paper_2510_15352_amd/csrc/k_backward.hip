// Backward pass of the splat renderer: the gradient of a linear function of
// the rendered RGB, expected depth and accumulated alpha,
//   L = sum_pixels  gR . RGB + gD depth + gA alpha,
// with respect to every Gaussian's mean, scales, rotation quaternion,
// opacity and SH coefficients. The paper's scenes are 3D Gaussian splats
// optimised by rendering them differentiably against images (Sec. 2.3 and
// Sec. 3.1); this is the reverse-mode derivative of the forward pass, with
// every discrete decision (near plane, skip, stop, clamps) taken as the
// forward pass takes it.
//
// Per chunk of cameras, after the forward binning stages:
//   k_bwd_counts / k_bwd_base  emission position of each record's first
//                              tile instance (the emission's own scan)
//   k_bwd_raster               per (pixel, Gaussian) pair the derivative
//                              with respect to the record's screen-space
//                              quantities, summed over each wave's 64 pixels
//                              and stored at (emission position, wave)
//   k_bwd_record               per record, the sum over its instances and
//                              waves in a fixed order
//   k_bwd_gauss                per Gaussian, the EWA projection and SH colour
//                              differentiated and summed over the chunk's
//                              cameras in camera order
// Every sum has a fixed order, so the gradients are deterministic.
#include "gs_device.h"
#include "kernels.h"

namespace gs {

constexpr float kLn2 = 0.69314718055994530942f;
// log2(e) / 2: the record's conic factor is the conic's scaled by its root
constexpr float kKappa2 = 0.72134752044448170368f;

// Sum over the wave's 64 lanes with DPP moves (no LDS round trips): pairs,
// quads, half rows and rows of 16 in every lane, then row 0 into row 1 and
// row 2 into row 3, then rows 0-1 into rows 2-3; the total ends in lane 63.
// The order of the additions is fixed, so the sum is deterministic.
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ float dpp_add(float v)
{
    return v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK,
                                                           0xF, true));
}

// Sum over one row of 16 lanes, in every lane of the row.
__device__ __forceinline__ float row_sum(float v)
{
    v = dpp_add<0xB1>(v);   // quad_perm [1, 0, 3, 2]
    v = dpp_add<0x4E>(v);   // quad_perm [2, 3, 0, 1]
    v = dpp_add<0x124>(v);  // row_ror 4
    v = dpp_add<0x128>(v);  // row_ror 8
    return v;
}

// (first, second) of a swap of the odd half-waves (rows of 32 lanes, W = 32)
// or odd rows of 16 lanes (W = 16) of a with the even ones of b, added:
// lanes of even rows get a's sum over the row pair, odd rows b's.
template <int W>
__device__ __forceinline__ float swap_add(float a, float b)
{
    const auto r = W == 32 ? __builtin_amdgcn_permlane32_swap(__float_as_uint(a),
                                                              __float_as_uint(b), false, false)
                           : __builtin_amdgcn_permlane16_swap(__float_as_uint(a),
                                                              __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// The ten per-lane values summed over the wave and spread over its rows of
// 16 lanes (every addition in a fixed order): values k and k + 5 are paired
// across the two half-waves, then (0, 1), (2, 3) and (4, 4) across rows, and
// each row is summed. Afterwards every lane of row r (r = lane / 16) holds
// in q[0] the total of value (r & 1) + 5 (r >> 1), in q[1] that of value
// 2 + (r & 1) + 5 (r >> 1), and in q[2] that of value 4 + 5 (r >> 1).
__device__ __forceinline__ void wave_sum10(const float *v, float *q)
{
    float p[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) p[k] = swap_add<32>(v[k], v[k + 5]);
    q[0] = row_sum(swap_add<16>(p[0], p[1]));
    q[1] = row_sum(swap_add<16>(p[2], p[3]));
    q[2] = row_sum(swap_add<16>(p[4], p[4]));
}

// ------------------------------------------------- emission positions --
// cnt[i] = tiles of the i-th depth-sorted record's box (i < n_vis)
__global__ void k_bwd_counts(const uint2 *__restrict__ srect, const uint32_t *__restrict__ n_vis,
                             uint32_t *__restrict__ cnt)
{
    const uint32_t n = *n_vis;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const TileBox b = tile_box(srect[i], 4, 4);
        cnt[i] = (uint32_t)(b.bw * b.bh);
    }
}

// inst_base[slot of record i] = base[i]
__global__ void k_bwd_base(const uint32_t *__restrict__ dvals, const uint32_t *__restrict__ base,
                           const uint32_t *__restrict__ n_vis, uint32_t *__restrict__ inst_base)
{
    const uint32_t n = *n_vis;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        inst_base[dvals[i]] = base[i];
}

// partial[0 .. kept * 4 * 10) = 0 (kept = counts[2])
__global__ void k_bwd_zero(float *__restrict__ partial, const uint32_t *__restrict__ counts)
{
    const uint64_t n = (uint64_t)counts[2] * (kBwdWaves * kBwdVals);
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        partial[i] = 0.0f;
}

// ------------------------------------------------------------- raster --
// One block per (camera, 16x16 tile), one 8x8 pixel block per wave, one
// pixel per lane. Each wave walks its tile's list twice with the forward
// pass's own arithmetic and culling (so every decision is the forward's):
// the first walk gives the pixel's final sums, the second the derivative
// of each contributing pair. For contributor i with weight w_i = a_i T_i and
// per-pixel scalar colour g_i = gR . c_i + gZ z_i + gW (gZ = gD / W,
// gW = gA - gD Z / W^2 with Z = sum w z, W = sum w),
//   dL/da_i = T_i g_i - S_i / (1 - a_i),
// where S_i = sum_{j > i} w_j g_j + T_final gR . bg is the total minus the
// prefix so far. Through a = o 2^-q (unless clamped at 0.99) with
// q = e^2 + f^2, e = ex dx + ey dy, f = fy dy (dx = pixel centre - u), the
// decisions taken in the forward's scaled form (a / 0.99, 0.99 T), the
// pair contributes to (u, v, conic xx, conic xy, conic yy, opacity, r, g, b,
// z). The ten sums over the wave go to partial[(instance * 4 + wave) * 10].
__global__ __launch_bounds__(256) void k_bwd_raster(BwdArgs a, uint32_t n_items)
{
    constexpr int B = kBwdBatch;
    __shared__ float4 sR0[kBwdWaves * B];
    __shared__ float4 sR1[kBwdWaves * B];
    __shared__ float4 sX[kBwdWaves * B];
    __shared__ uint2 sI[kBwdWaves * B];
    const uint32_t item = blockIdx.x;
    if (item >= n_items) return;
    const int cl = (int)(item / (uint32_t)a.tiles_per_cam);
    const int tile = (int)(item % (uint32_t)a.tiles_per_cam);
    const int wave = (int)threadIdx.x >> 6;
    const uint32_t lane = __lane_id();
    const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
    const int wx0 = tx * 16 + (wave & 1) * 8, wy0 = ty * 16 + (wave >> 1) * 8;
    const int pxi = wx0 + (int)(lane & 7u), pyi = wy0 + (int)(lane >> 3);
    const bool inside = pxi < a.W && pyi < a.H;
    const float lx = (float)(lane & 7u), ly = (float)(lane >> 3);
    const float ww = (float)(min(wx0 + 7, a.W - 1) - wx0), wh = (float)(min(wy0 + 7, a.H - 1) - wy0);
    const float cx0 = (float)wx0 + 0.5f, cy0 = (float)wy0 + 0.5f;
    const uint2 rg = a.ranges[(uint32_t)cl * (uint32_t)a.tiles_per_cam + (uint32_t)tile];
    float4 *L0 = sR0 + wave * B;
    float4 *L1 = sR1 + wave * B;
    float4 *LX = sX + wave * B;
    uint2 *LI = sI + wave * B;
    const uint64_t lt = lanemask_lt();
    float gr = 0.0f, gg = 0.0f, gb = 0.0f, gd = 0.0f, ga = 0.0f;
    if (inside) {
        const int64_t pix = ((int64_t)a.cam_global[cl] * a.H + pyi) * (int64_t)a.W + pxi;
        if (a.g_rgb) {
            gr = a.g_rgb[pix * 3 + 0];
            gg = a.g_rgb[pix * 3 + 1];
            gb = a.g_rgb[pix * 3 + 2];
        }
        if (a.g_depth) gd = a.g_depth[pix];
        if (a.g_alpha) ga = a.g_alpha[pix];
    }
    float tot = 0.0f, gz = 0.0f, gw = 0.0f;
    for (int pass = 0; pass < 2; ++pass) {
        float U = inside ? kAlphaMax : -1.0f;  // 0.99 x the transmittance
        float r = 0.0f, g = 0.0f, b = 0.0f, zw = 0.0f, ws = 0.0f, pre = 0.0f;
        bool live = __ballot(U > 0.0f) != 0ull;
        for (uint32_t base = rg.x; live && base < rg.y; base += B) {
            int n = 0;
#pragma unroll
            for (int sb = 0; sb < B / 64; ++sb) {
                const uint32_t j = base + (uint32_t)(sb * 64) + lane;
                bool hit = false;
                float4 R0 = make_float4(0.f, 0.f, 0.f, 0.f), R1 = R0, X = R0;
                uint2 I = make_uint2(0u, 0u);
                if (j < rg.y) {
                    const uint32_t slot = a.ivals[j];
                    const float4 A = a.rec[(size_t)slot * 3];
                    const float4 Bv = a.rec[(size_t)slot * 3 + 1];
                    const float4 C = a.rec[(size_t)slot * 3 + 2];
                    R0 = make_float4(A.z, A.w, Bv.x, kLog2AlphaMax - __builtin_amdgcn_logf(Bv.y));
                    R1 = make_float4(Bv.z, Bv.w, C.x, C.y);
                    const float Xw = cx0 - A.x, Yw = cy0 - A.y;
                    hit = may_touch(R0.x, R0.y, R0.z, Xw, Yw, ww, wh, C.z);
                    X = make_float4(fmaf(R0.x, Xw, R0.y * Yw), R0.z * Yw, Xw, Yw);
                    if (pass == 1 && hit) {
                        const TileBox bx = tile_box(a.rect[slot], 4, 4);
                        I = make_uint2(a.inst_base[slot] + (uint32_t)((ty - bx.ty0) * bx.bw + (tx - bx.tx0)),
                                       __float_as_uint(Bv.y));
                    }
                }
                const uint64_t m = __ballot(hit);
                if (hit) {
                    const int p = n + (int)__popcll(m & lt);
                    L0[p] = R0;
                    L1[p] = R1;
                    LX[p] = X;
                    LI[p] = I;
                }
                n += (int)__popcll(m);
            }
            __builtin_amdgcn_wave_barrier();  // list entries written before they are read
            for (int k = 0; k < n; ++k) {
                const float4 R0 = L0[k], R1 = L1[k], X = LX[k];
                // the forward step (same operations as the renderer's)
                const float e = fmaf(R0.x, lx, fmaf(R0.y, ly, X.x));
                const float f = fmaf(R0.z, ly, X.y);
                const float q = fmaf(e, e, fmaf(f, f, R0.w));
                const float raw = __builtin_amdgcn_exp2f(-q);  // alpha / 0.99, unclamped
                const float sa = fminf(raw, 1.0f);
                const bool hit = sa >= kScaledAlphaMin;
                const float wt = sa * U;
                const float Un = fmaf(-kAlphaMax, wt, U);
                const bool acc = hit & (Un >= kScaledTMin);
                const float w = acc ? wt : 0.0f;
                if (pass == 0) {
                    r = fmaf(w, R1.x, r);
                    g = fmaf(w, R1.y, g);
                    b = fmaf(w, R1.z, b);
                    zw = fmaf(w, R1.w, zw);
                    ws += w;
                } else if (__ballot(acc) != 0ull) {
                    float v[kBwdVals];
#pragma unroll
                    for (int t = 0; t < kBwdVals; ++t) v[t] = 0.0f;
                    if (acc) {
                        const float gi = fmaf(gr, R1.x, fmaf(gg, R1.y, fmaf(gb, R1.z, fmaf(gz, R1.w, gw))));
                        const float s = tot - pre - w * gi;
                        // approximate reciprocals (1 ulp): gradients, not decisions
                        const float alpha = kAlphaMax * sa, T = U * (1.0f / kAlphaMax);
                        const float da = T * gi - s * __builtin_amdgcn_rcpf(1.0f - alpha);
                        pre = fmaf(w, gi, pre);
                        const bool clamped = raw > 1.0f;
                        const float dq = clamped ? 0.0f : -kLn2 * alpha * da;
                        const float o = __uint_as_float(LI[k].y);
                        const float dx = lx + X.z, dy = ly + X.w;
                        v[0] = dq * (-2.0f * e * R0.x);
                        v[1] = dq * (-2.0f * fmaf(e, R0.y, f * R0.z));
                        v[2] = dq * kKappa2 * dx * dx;
                        v[3] = dq * 2.0f * kKappa2 * dx * dy;
                        v[4] = dq * kKappa2 * dy * dy;
                        v[5] = clamped ? 0.0f : da * (alpha * __builtin_amdgcn_rcpf(o));
                        v[6] = gr * w;
                        v[7] = gg * w;
                        v[8] = gb * w;
                        v[9] = gz * w;
                    }
                    static_assert(kBwdVals == 10, "the wave sum spreads ten values");
                    float q[3];
                    wave_sum10(v, q);
                    if ((lane & 15u) == 0u) {
                        const int r = (int)(lane >> 4);
                        const int t0 = (r & 1) + 5 * (r >> 1);
                        float *dst = a.partial + ((size_t)LI[k].x * kBwdWaves + wave) * kBwdVals;
                        dst[t0] = q[0];
                        dst[t0 + 2] = q[1];
                        if ((r & 1) == 0) dst[4 + 5 * (r >> 1)] = q[2];
                    }
                }
                U = acc ? Un : (hit ? -fabsf(U) : U);
                if (__ballot(U > 0.0f) == 0ull) break;
            }
            live = __ballot(U > 0.0f) != 0ull;
            __builtin_amdgcn_wave_barrier();  // list read before the next batch rewrites it
        }
        if (pass == 0) {
            const float tf = fabsf(U) / kAlphaMax;
            gz = ws > 0.0f ? gd / ws : 0.0f;
            gw = ws > 0.0f ? ga - gd * zw / (ws * ws) : ga;
            tot = gr * r + gg * g + gb * b + gz * zw + gw * ws +
                  tf * (gr * a.bg_r + gg * a.bg_g + gb * a.bg_b);
        }
    }
}

// ------------------------------------------------------------ records --
// rgrad[slot * 10 + t] = sum over the record's instances j (in order) and
// the four waves of partial[((base + j) * 4 + wave) * 10 + t]
__global__ void k_bwd_record(const uint32_t *__restrict__ dvals, const uint32_t *__restrict__ base,
                             const uint32_t *__restrict__ cnt, const uint32_t *__restrict__ counts,
                             const float *__restrict__ partial, float *__restrict__ rgrad)
{
    const uint32_t n = counts[0], kept = counts[2];
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint32_t b0 = base[i], c = cnt[i];
        float v[kBwdVals];
#pragma unroll
        for (int t = 0; t < kBwdVals; ++t) v[t] = 0.0f;
        for (uint32_t j = 0; j < c && b0 + j < kept; ++j)
            for (int wv = 0; wv < kBwdWaves; ++wv) {
                const float *p = partial + ((size_t)(b0 + j) * kBwdWaves + wv) * kBwdVals;
#pragma unroll
                for (int t = 0; t < kBwdVals; ++t) v[t] += p[t];
            }
        float *o = rgrad + (size_t)dvals[i] * kBwdVals;
#pragma unroll
        for (int t = 0; t < kBwdVals; ++t) o[t] = v[t];
    }
}

// ---------------------------------------------------------- Gaussians --
// Values and gradients (with respect to the unit direction's x, y, z) of
// the real SH basis functions of degree <= DEG, the polynomial forms of the
// renderer's colour evaluation differentiated term by term.
template <int DEG>
__device__ __forceinline__ void sh_basis_grad(float x, float y, float z, float *Y, float *Gx,
                                              float *Gy, float *Gz)
{
    Y[0] = 0.28209479177387814f;
    Gx[0] = Gy[0] = Gz[0] = 0.0f;
    if (DEG >= 1) {
        const float c1 = 0.48860251190291992f;
        Y[1] = -c1 * y; Gx[1] = 0.0f; Gy[1] = -c1; Gz[1] = 0.0f;
        Y[2] = c1 * z;  Gx[2] = 0.0f; Gy[2] = 0.0f; Gz[2] = c1;
        Y[3] = -c1 * x; Gx[3] = -c1; Gy[3] = 0.0f; Gz[3] = 0.0f;
    }
    if (DEG >= 2) {
        const float c2a = 1.09254843059207907f, c2b = 0.31539156525252001f,
                    c2c = 0.54627421529603954f;
        const float xx = x * x, yy = y * y, zz = z * z;
        Y[4] = c2a * x * y;  Gx[4] = c2a * y; Gy[4] = c2a * x; Gz[4] = 0.0f;
        Y[5] = -c2a * y * z; Gx[5] = 0.0f; Gy[5] = -c2a * z; Gz[5] = -c2a * y;
        Y[6] = c2b * (2.0f * zz - xx - yy);
        Gx[6] = -2.0f * c2b * x; Gy[6] = -2.0f * c2b * y; Gz[6] = 4.0f * c2b * z;
        Y[7] = -c2a * x * z; Gx[7] = -c2a * z; Gy[7] = 0.0f; Gz[7] = -c2a * x;
        Y[8] = c2c * (xx - yy); Gx[8] = 2.0f * c2c * x; Gy[8] = -2.0f * c2c * y; Gz[8] = 0.0f;
        if (DEG >= 3) {
            const float c3a = 0.59004358992664352f, c3b = 2.89061144264055406f,
                        c3c = 0.45704579946446574f, c3d = 0.37317633259011540f,
                        c3e = 1.44530572132027703f;
            Y[9] = -c3a * y * (3.0f * xx - yy);
            Gx[9] = -6.0f * c3a * x * y; Gy[9] = -3.0f * c3a * (xx - yy); Gz[9] = 0.0f;
            Y[10] = c3b * x * y * z;
            Gx[10] = c3b * y * z; Gy[10] = c3b * x * z; Gz[10] = c3b * x * y;
            Y[11] = -c3c * y * (4.0f * zz - xx - yy);
            Gx[11] = 2.0f * c3c * x * y; Gy[11] = -c3c * (4.0f * zz - xx - 3.0f * yy);
            Gz[11] = -8.0f * c3c * y * z;
            Y[12] = c3d * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
            Gx[12] = -6.0f * c3d * x * z; Gy[12] = -6.0f * c3d * y * z;
            Gz[12] = c3d * (6.0f * zz - 3.0f * xx - 3.0f * yy);
            Y[13] = -c3c * x * (4.0f * zz - xx - yy);
            Gx[13] = -c3c * (4.0f * zz - 3.0f * xx - yy); Gy[13] = 2.0f * c3c * x * y;
            Gz[13] = -8.0f * c3c * x * z;
            Y[14] = c3e * z * (xx - yy);
            Gx[14] = 2.0f * c3e * x * z; Gy[14] = -2.0f * c3e * y * z; Gz[14] = c3e * (xx - yy);
            Y[15] = -c3a * x * (xx - 3.0f * yy);
            Gx[15] = -3.0f * c3a * (xx - yy); Gy[15] = 6.0f * c3a * x * y; Gz[15] = 0.0f;
        }
    }
}

// One thread per stored Gaussian g: for every camera of the chunk that sees
// it (visibility bit of its slot), the record gradient is carried back
// through the projection (u, v, the conic of Sigma' = T M M^T T^T + 0.3 I
// with T = J W and M = R(q) S, the depth z) to the camera-space mean and M,
// and through the colour max(0, sum k Y(d) + 0.5) to the SH coefficients
// and the direction d = (mean - C) / |mean - C|. The gradient of M is
// summed over the cameras and turned into scale and quaternion gradients at
// the end. Results are added to the caller's arrays at the caller's index.
template <int DEG>
__global__ __launch_bounds__(256) void k_bwd_gauss(BwdGaussArgs a)
{
    constexpr int NC = (DEG + 1) * (DEG + 1);
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= a.n) return;
    const float4 po = a.pos_op[g];
    const float4 m01 = a.m01[g], m23 = a.m23[g];
    const float2 m8r = a.m8r[g];
    const float M[9] = {m01.x, m01.y, m01.z, m01.w, m23.x, m23.y, m23.z, m23.w, m8r.x};
    float k[NC * 3];
#pragma unroll
    for (int j = 0; j < NC * 3; ++j) k[j] = a.sh[(int64_t)j * a.n + g];
    float dmean[3] = {0.f, 0.f, 0.f}, dM[9], dop = 0.0f, dk[NC * 3];
#pragma unroll
    for (int j = 0; j < 9; ++j) dM[j] = 0.0f;
#pragma unroll
    for (int j = 0; j < NC * 3; ++j) dk[j] = 0.0f;
    bool any = false;
    for (int c = 0; c < a.n_cams; ++c) {
        const uint32_t slot = a.cam_slot[c] + (uint32_t)g;
        if (!((a.vis[slot >> 6] >> (slot & 63u)) & 1ull)) continue;
        any = true;
        const CamParams &cam = a.cams[c];
        const float *rgv = a.rgrad + (size_t)slot * kBwdVals;
        const float du = rgv[0], dv = rgv[1], dA = rgv[2], dB = rgv[3], dC = rgv[4];
        const float dR = rgv[6], dG = rgv[7], dBl = rgv[8], dzc = rgv[9];
        dop += rgv[5];
        const float *R = cam.R;
        const float x = fmaf(R[0], po.x, fmaf(R[1], po.y, fmaf(R[2], po.z, cam.t[0])));
        const float y = fmaf(R[3], po.x, fmaf(R[4], po.y, fmaf(R[5], po.z, cam.t[1])));
        const float z = fmaf(R[6], po.x, fmaf(R[7], po.y, fmaf(R[8], po.z, cam.t[2])));
        const float iz = 1.0f / z;
        const float xz = x * iz, yz = y * iz;
        const bool freex = !(xz < cam.lxn) && !(xz > cam.lxp);
        const bool freey = !(yz < cam.lyn) && !(yz > cam.lyp);
        const float txc = fminf(fmaxf(xz, cam.lxn), cam.lxp);
        const float tyc = fminf(fmaxf(yz, cam.lyn), cam.lyp);
        const float j00 = cam.fx * iz, j02 = -cam.fx * txc * iz;
        const float j11 = cam.fy * iz, j12 = -cam.fy * tyc * iz;
        float t0[3], t1[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            t0[i] = fmaf(j02, R[6 + i], j00 * R[i]);
            t1[i] = fmaf(j12, R[6 + i], j11 * R[3 + i]);
        }
        float p[3], q[3];
#pragma unroll
        for (int kk = 0; kk < 3; ++kk) {
            p[kk] = fmaf(t0[0], M[kk], fmaf(t0[1], M[3 + kk], t0[2] * M[6 + kk]));
            q[kk] = fmaf(t1[0], M[kk], fmaf(t1[1], M[3 + kk], t1[2] * M[6 + kk]));
        }
        const float pp = fmaf(p[0], p[0], fmaf(p[1], p[1], p[2] * p[2]));
        const float qq = fmaf(q[0], q[0], fmaf(q[1], q[1], q[2] * q[2]));
        const float pq = fmaf(p[0], q[0], fmaf(p[1], q[1], p[2] * q[2]));
        const float cx_ = p[1] * q[2] - p[2] * q[1], cy_ = p[2] * q[0] - p[0] * q[2],
                    cz_ = p[0] * q[1] - p[1] * q[0];
        const float cross2 = fmaf(cx_, cx_, fmaf(cy_, cy_, cz_ * cz_));
        const float sa = pp + kLowPass, sc = qq + kLowPass, sb = pq;
        const float det = fmaf(kLowPass, pp + qq, cross2) + kLowPass * kLowPass;
        // conic (c, -b, a) / det differentiated with respect to a, b, c
        const float id2 = 1.0f / (det * det);
        const float dsa = (-sc * sc * dA + sb * sc * dB - sb * sb * dC) * id2;
        const float dsb = (2.0f * sb * sc * dA - fmaf(sa, sc, sb * sb) * dB + 2.0f * sa * sb * dC) * id2;
        const float dsc = (-sb * sb * dA + sa * sb * dB - sa * sa * dC) * id2;
        float dp[3], dq[3];
#pragma unroll
        for (int kk = 0; kk < 3; ++kk) {
            dp[kk] = fmaf(2.0f * dsa, p[kk], dsb * q[kk]);
            dq[kk] = fmaf(2.0f * dsc, q[kk], dsb * p[kk]);
        }
        float dt0[3], dt1[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            dt0[j] = fmaf(dp[0], M[j * 3], fmaf(dp[1], M[j * 3 + 1], dp[2] * M[j * 3 + 2]));
            dt1[j] = fmaf(dq[0], M[j * 3], fmaf(dq[1], M[j * 3 + 1], dq[2] * M[j * 3 + 2]));
#pragma unroll
            for (int kk = 0; kk < 3; ++kk) dM[j * 3 + kk] += fmaf(t0[j], dp[kk], t1[j] * dq[kk]);
        }
        const float dj00 = fmaf(dt0[0], R[0], fmaf(dt0[1], R[1], dt0[2] * R[2]));
        const float dj02 = fmaf(dt0[0], R[6], fmaf(dt0[1], R[7], dt0[2] * R[8]));
        const float dj11 = fmaf(dt1[0], R[3], fmaf(dt1[1], R[4], dt1[2] * R[5]));
        const float dj12 = fmaf(dt1[0], R[6], fmaf(dt1[1], R[7], dt1[2] * R[8]));
        float diz = cam.fx * dj00 - cam.fx * txc * dj02 + cam.fy * dj11 - cam.fy * tyc * dj12;
        const float dtx = -cam.fx * iz * dj02, dty = -cam.fy * iz * dj12;
        float dX = 0.0f, dY = 0.0f, dZ = dzc;
        if (freex) { dX += dtx * iz; diz += dtx * x; }
        if (freey) { dY += dty * iz; diz += dty * y; }
        // u = fx x / z + cx, v = fy y / z + cy
        dX += du * cam.fx * iz;
        diz += du * cam.fx * x;
        dY += dv * cam.fy * iz;
        diz += dv * cam.fy * y;
        dZ -= diz * iz * iz;
        // camera-space position = R_wc mean + t_wc
#pragma unroll
        for (int kk = 0; kk < 3; ++kk) dmean[kk] += fmaf(R[kk], dX, fmaf(R[3 + kk], dY, R[6 + kk] * dZ));
        // colour
        const float vx = po.x - cam.C[0], vy = po.y - cam.C[1], vz = po.z - cam.C[2];
        const float inv = rsqrtf(fmaf(vx, vx, fmaf(vy, vy, vz * vz)));
        const float ux = vx * inv, uy = vy * inv, uz = vz * inv;
        float Y[NC], Gx[NC], Gy[NC], Gz[NC];
        sh_basis_grad<DEG>(ux, uy, uz, Y, Gx, Gy, Gz);
        float pre[3] = {0.5f, 0.5f, 0.5f};
#pragma unroll
        for (int m = 0; m < NC; ++m)
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) pre[ch] = fmaf(Y[m], k[m * 3 + ch], pre[ch]);
        const float dc[3] = {pre[0] < 0.0f ? 0.0f : dR, pre[1] < 0.0f ? 0.0f : dG,
                             pre[2] < 0.0f ? 0.0f : dBl};
        float ddx = 0.0f, ddy = 0.0f, ddz = 0.0f;
#pragma unroll
        for (int m = 0; m < NC; ++m) {
            const float s = fmaf(dc[0], k[m * 3], fmaf(dc[1], k[m * 3 + 1], dc[2] * k[m * 3 + 2]));
            ddx = fmaf(s, Gx[m], ddx);
            ddy = fmaf(s, Gy[m], ddy);
            ddz = fmaf(s, Gz[m], ddz);
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) dk[m * 3 + ch] = fmaf(Y[m], dc[ch], dk[m * 3 + ch]);
        }
        // d = v / |v|: dv = (dd - d (d . dd)) / |v|
        const float dd = fmaf(ux, ddx, fmaf(uy, ddy, uz * ddz));
        dmean[0] += (ddx - ux * dd) * inv;
        dmean[1] += (ddy - uy * dd) * inv;
        dmean[2] += (ddz - uz * dd) * inv;
    }
    if (!any) return;
    // M = R(qhat) diag(s): ds_k = sum_j dM_jk R_jk, dR_jk = dM_jk s_k, then
    // R(qhat) and qhat = q / |q| differentiated
    const float4 qn = a.quat[g];   // unit (w, x, y, z)
    const float4 sn = a.scale[g];  // (sx, sy, sz, 1 / |q|)
    const float qw = qn.x, qx = qn.y, qy = qn.z, qz = qn.w;
    const float Rq[9] = {1.0f - 2.0f * (qy * qy + qz * qz), 2.0f * (qx * qy - qw * qz),
                         2.0f * (qx * qz + qw * qy),        2.0f * (qx * qy + qw * qz),
                         1.0f - 2.0f * (qx * qx + qz * qz), 2.0f * (qy * qz - qw * qx),
                         2.0f * (qx * qz - qw * qy),        2.0f * (qy * qz + qw * qx),
                         1.0f - 2.0f * (qx * qx + qy * qy)};
    const float s3[3] = {sn.x, sn.y, sn.z};
    float ds[3], dRq[9];
#pragma unroll
    for (int kk = 0; kk < 3; ++kk)
        ds[kk] = fmaf(dM[kk], Rq[kk], fmaf(dM[3 + kk], Rq[3 + kk], dM[6 + kk] * Rq[6 + kk]));
#pragma unroll
    for (int j = 0; j < 9; ++j) dRq[j] = dM[j] * s3[j % 3];
    const float dw = 2.0f * (-qz * dRq[1] + qy * dRq[2] + qz * dRq[3] - qx * dRq[5] - qy * dRq[6] +
                             qx * dRq[7]);
    const float dx = 2.0f * (qy * dRq[1] + qz * dRq[2] + qy * dRq[3] - 2.0f * qx * dRq[4] -
                             qw * dRq[5] + qz * dRq[6] + qw * dRq[7] - 2.0f * qx * dRq[8]);
    const float dy = 2.0f * (-2.0f * qy * dRq[0] + qx * dRq[1] + qw * dRq[2] + qx * dRq[3] +
                             qz * dRq[5] - qw * dRq[6] + qz * dRq[7] - 2.0f * qy * dRq[8]);
    const float dz = 2.0f * (-2.0f * qz * dRq[0] - qw * dRq[1] + qx * dRq[2] + qw * dRq[3] -
                             2.0f * qz * dRq[4] + qy * dRq[5] + qx * dRq[6] + qy * dRq[7]);
    const float qd = fmaf(qw, dw, fmaf(qx, dx, fmaf(qy, dy, qz * dz)));
    const int64_t pg = a.perm[g];
#pragma unroll
    for (int kk = 0; kk < 3; ++kk) {
        a.d_means[pg * 3 + kk] += dmean[kk];
        a.d_scales[pg * 3 + kk] += ds[kk];
    }
    a.d_quats[pg * 4 + 0] += (dw - qw * qd) * sn.w;
    a.d_quats[pg * 4 + 1] += (dx - qx * qd) * sn.w;
    a.d_quats[pg * 4 + 2] += (dy - qy * qd) * sn.w;
    a.d_quats[pg * 4 + 3] += (dz - qz * qd) * sn.w;
    a.d_opacity[pg] += dop;
#pragma unroll
    for (int j = 0; j < NC * 3; ++j) a.d_sh[pg * NC * 3 + j] += dk[j];
}

// ---------------------------------------------------------------- launch --
static unsigned grid_for(uint64_t n, uint64_t cap = 16384)
{
    uint64_t b = (n + 255) / 256;
    return (unsigned)(b < 1 ? 1 : (b > cap ? cap : b));
}

void launch_bwd_emission(const uint2 *srect, const uint32_t *dvals, const uint32_t *counts,
                         uint32_t n_max, uint32_t *cnt, uint32_t *base, uint32_t *inst_base,
                         float *partial, uint32_t cap, const ScanTemp &tmp, hipStream_t st)
{
    hipLaunchKernelGGL(k_bwd_counts, dim3(grid_for(n_max)), dim3(256), 0, st, srect, counts, cnt);
    scan_u32(cnt, counts, n_max, base, nullptr, tmp, st);
    hipLaunchKernelGGL(k_bwd_base, dim3(grid_for(n_max)), dim3(256), 0, st, dvals, base, counts,
                       inst_base);
    hipLaunchKernelGGL(k_bwd_zero, dim3(grid_for((uint64_t)cap * kBwdWaves * kBwdVals)), dim3(256),
                       0, st, partial, counts);
}

void launch_bwd_raster(const BwdArgs &a, int n_cams, hipStream_t st)
{
    const uint32_t n_items = (uint32_t)a.tiles_per_cam * (uint32_t)n_cams;
    hipLaunchKernelGGL(k_bwd_raster, dim3(n_items), dim3(256), 0, st, a, n_items);
}

void launch_bwd_record(const uint32_t *dvals, const uint32_t *base, const uint32_t *cnt,
                       const uint32_t *counts, uint32_t n_max, const float *partial, float *rgrad,
                       hipStream_t st)
{
    hipLaunchKernelGGL(k_bwd_record, dim3(grid_for(n_max)), dim3(256), 0, st, dvals, base, cnt,
                       counts, partial, rgrad);
}

void launch_bwd_gauss(int deg, const BwdGaussArgs &a, hipStream_t st)
{
    const unsigned grid = (unsigned)((a.n + 255) / 256);
    if (grid == 0) return;
    switch (deg) {
    case 0: hipLaunchKernelGGL(k_bwd_gauss<0>, dim3(grid), dim3(256), 0, st, a); break;
    case 1: hipLaunchKernelGGL(k_bwd_gauss<1>, dim3(grid), dim3(256), 0, st, a); break;
    case 2: hipLaunchKernelGGL(k_bwd_gauss<2>, dim3(grid), dim3(256), 0, st, a); break;
    default: hipLaunchKernelGGL(k_bwd_gauss<3>, dim3(grid), dim3(256), 0, st, a); break;
    }
}

}  // namespace gs
