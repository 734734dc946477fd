// Scene preparation, camera setup, per-(camera, Gaussian) EWA projection with
// SH colour, and order-preserving compaction of the visible pairs.
#include "gs_device.h"
#include "kernels.h"

namespace gs {

// ------------------------------------------------------------ scene prep --
// M = R(q/|q|) diag(scale); rad = sqrt(2 ln(255 o)) * largest scale; SH
// re-laid out planar [(k*3 + c)][n] so that a wave reading one coefficient
// of 64 Gaussians is one coalesced 256 B load.
// bad[0] is set when a value is non-finite, a scale is not positive, an
// opacity leaves [0, 1] or a quaternion is zero.
__global__ void k_scene_prep(const float *__restrict__ means, const float *__restrict__ scales,
                             const float *__restrict__ quats, const float *__restrict__ opacity,
                             const float *__restrict__ sh, int64_t n, int ncoef,
                             float4 *__restrict__ pos_op, float4 *__restrict__ m01,
                             float4 *__restrict__ m23, float2 *__restrict__ m8r,
                             float *__restrict__ sh_planar, float4 *__restrict__ quat,
                             float4 *__restrict__ scale, int *__restrict__ bad)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    const float mx = means[g * 3 + 0], my = means[g * 3 + 1], mz = means[g * 3 + 2];
    const float sx = scales[g * 3 + 0], sy = scales[g * 3 + 1], sz = scales[g * 3 + 2];
    float qw = quats[g * 4 + 0], qx = quats[g * 4 + 1], qy = quats[g * 4 + 2], qz = quats[g * 4 + 3];
    const float o = opacity[g];
    const float qn2 = qw * qw + qx * qx + qy * qy + qz * qz;
    bool ok = isfinite(mx) && isfinite(my) && isfinite(mz) && sx > 0.0f && sy > 0.0f &&
              sz > 0.0f && isfinite(sx) && isfinite(sy) && isfinite(sz) && o >= 0.0f &&
              o <= 1.0f && qn2 > 0.0f && isfinite(qn2);
    const float qi = rsqrtf(qn2);
    qw *= qi; qx *= qi; qy *= qi; qz *= qi;
    if (quat) quat[g] = make_float4(qw, qx, qy, qz);
    if (scale) scale[g] = make_float4(sx, sy, sz, qi);
    const float R00 = 1.0f - 2.0f * (qy * qy + qz * qz), R01 = 2.0f * (qx * qy - qw * qz),
                R02 = 2.0f * (qx * qz + qw * qy);
    const float R10 = 2.0f * (qx * qy + qw * qz), R11 = 1.0f - 2.0f * (qx * qx + qz * qz),
                R12 = 2.0f * (qy * qz - qw * qx);
    const float R20 = 2.0f * (qx * qz - qw * qy), R21 = 2.0f * (qy * qz + qw * qx),
                R22 = 1.0f - 2.0f * (qx * qx + qy * qy);
    pos_op[g] = make_float4(mx, my, mz, o);
    m01[g] = make_float4(R00 * sx, R01 * sy, R02 * sz, R10 * sx);
    m23[g] = make_float4(R11 * sy, R12 * sz, R20 * sx, R21 * sy);
    const float smax = fmaxf(sx, fmaxf(sy, sz));
    const float r2 = 2.0f * logf(o * 255.0f);
    m8r[g] = make_float2(R22 * sz, o >= kAlphaMin ? sqrtf(fmaxf(r2, 0.0f)) * smax : 0.0f);
    for (int k = 0; k < ncoef * 3; ++k) {
        const float c = sh[g * ncoef * 3 + k];
        ok = ok && isfinite(c);
        sh_planar[(int64_t)k * n + g] = c;
    }
    if (!ok) atomicOr(bad, 1);
}

// ---------------------------------------------------------- camera setup --
// R_wc = R_cw^T, t_wc = -R_wc C from the camera-to-world pose [R_cw | C];
// tangent clamp range 1.3x the image half-extent on each side.
__global__ void k_camera_setup(const float *__restrict__ poses, const float *__restrict__ intr,
                               const int32_t *__restrict__ cam_global, int n_cams, int W, int H,
                               const uint32_t *__restrict__ mask, CamParams *__restrict__ out)
{
    const int cl = blockIdx.x * blockDim.x + threadIdx.x;
    if (cl >= n_cams) return;
    const int64_t cg = cam_global ? cam_global[cl] : cl;
    const float *P = poses + cg * 12;
    CamParams c;
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) c.R[r * 3 + k] = P[k * 4 + r];
    const float C0 = P[3], C1 = P[7], C2 = P[11];
    c.C[0] = C0; c.C[1] = C1; c.C[2] = C2;
    for (int r = 0; r < 3; ++r)
        c.t[r] = -fmaf(c.R[r * 3 + 0], C0, fmaf(c.R[r * 3 + 1], C1, c.R[r * 3 + 2] * C2));
    c.fx = intr[cg * 4 + 0]; c.fy = intr[cg * 4 + 1];
    c.cx = intr[cg * 4 + 2]; c.cy = intr[cg * 4 + 3];
    c.lxn = -kTanClamp * c.cx / c.fx;
    c.lxp = kTanClamp * ((float)W - c.cx) / c.fx;
    c.lyn = -kTanClamp * c.cy / c.fy;
    c.lyp = kTanClamp * ((float)H - c.cy) / c.fy;
    c.kx = sqrtf(1.0f + fmaxf(c.lxn * c.lxn, c.lxp * c.lxp));
    c.ky = sqrtf(1.0f + fmaxf(c.lyn * c.lyn, c.lyp * c.lyp));
    c.active = (mask == nullptr || mask[cg] != 0u) ? 1.0f : 0.0f;
    for (int k = 0; k < 6; ++k) c.pad[k] = 0.0f;
    out[cl] = c;
}

// ------------------------------------------------------------- projection --
// One block = one ProjItem: 256 Gaussians of one scene, each thread keeps
// its Gaussian's parameters (incl. up to 48 SH coefficients) in registers
// and loops over the item's cameras, so a scene's parameters are read from
// HBM once per camera group instead of once per camera. Every visible pair
// writes its raster record into the camera's slot range; visibility is
// recorded as one 64-bit ballot word per wave (the compaction input).
template <int DEG>
__global__ __launch_bounds__(256) void k_project(
    const ProjItem *__restrict__ items, const SceneDev *__restrict__ scenes,
    const CamParams *__restrict__ cams, const uint32_t *__restrict__ cam_slot,
    float near, int W, int H, float4 *__restrict__ rec, uint2 *__restrict__ rect,
    uint32_t *__restrict__ zbits,
    uint64_t *__restrict__ vis)
{
    constexpr int NC = (DEG + 1) * (DEG + 1);
    __shared__ CamParams s_cam[kProjCams];
    __shared__ uint32_t s_slot[kProjCams];
    const ProjItem it = items[blockIdx.x];
    {
        // the item's camera constants, staged once per block
        float *dst = reinterpret_cast<float *>(s_cam);
        const float *src = reinterpret_cast<const float *>(cams + it.cam0);
        for (int j = (int)threadIdx.x; j < it.ncam * 32; j += 256) dst[j] = src[j];
        if ((int)threadIdx.x < it.ncam) s_slot[threadIdx.x] = cam_slot[it.cam0 + threadIdx.x];
    }
    const SceneDev sc = scenes[it.scene];
    const int g = it.g0 + (int)threadIdx.x;
    const bool in_range = g < sc.n;
    const int wave_g0 = it.g0 + (int)(threadIdx.x & ~63u);
    const bool wave_live = wave_g0 < sc.n;  // this wave owns a visibility word
    float4 po = make_float4(0.f, 0.f, 0.f, 0.f), a = po, b = po;
    float2 m8r = make_float2(0.f, 0.f);
    float k[NC * 3];
    // a block whose cameras are all masked out loads no Gaussian
    bool any_active = false;
    for (int ci = 0; ci < it.ncam; ++ci) any_active |= cams[it.cam0 + ci].active > 0.0f;
    if (in_range && any_active) {
        po = sc.pos_op[g];
        a = sc.m01[g];
        b = sc.m23[g];
        m8r = sc.m8r[g];
#pragma unroll
        for (int j = 0; j < NC * 3; ++j) k[j] = sc.sh[(int64_t)j * sc.n + g];
    } else {
#pragma unroll
        for (int j = 0; j < NC * 3; ++j) k[j] = 0.0f;
    }
    __syncthreads();
    for (int ci = 0; ci < it.ncam; ++ci) {
        const CamParams &cam = s_cam[ci];
        Projected P;
        bool visible = in_range && cam.active > 0.0f &&
                       project_gaussian(cam, po, a, b, m8r, near, W, H, P);
        const uint32_t slot = s_slot[ci] + (uint32_t)g;
        if (visible) {
            float dx = po.x - cam.C[0], dy = po.y - cam.C[1], dz = po.z - cam.C[2];
            const float inv = rsqrtf(fmaf(dx, dx, fmaf(dy, dy, dz * dz)));
            float r, gg, bb;
            sh_colour<DEG>(k, dx * inv, dy * inv, dz * inv, r, gg, bb);
            P.B.z = r;
            P.B.w = gg;
            P.C.x = bb;
            float4 *r3 = rec + (size_t)slot * 3;  // one 48-byte record
            r3[0] = P.A;
            r3[1] = P.B;
            r3[2] = P.C;
            rect[slot] = make_uint2((uint32_t)P.x0 | ((uint32_t)P.x1 << 16),
                                    (uint32_t)P.y0 | ((uint32_t)P.y1 << 16));
            zbits[slot] = __float_as_uint(P.C.y);
        }
        const uint64_t word = __ballot(visible);
        if (wave_live && __lane_id() == 0) vis[slot >> 6] = word;
    }
}

// ------------------------------------------------------ debug projection --
template <int DEG>
__global__ void k_debug_project(SceneDev sc, const int32_t *__restrict__ perm,
                                const CamParams *__restrict__ cam_p, float near, int W, int H,
                                float *__restrict__ out)
{
    constexpr int NC = (DEG + 1) * (DEG + 1);
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= sc.n) return;
    const CamParams cam = *cam_p;
    float k[NC * 3];
#pragma unroll
    for (int j = 0; j < NC * 3; ++j) k[j] = sc.sh[(int64_t)j * sc.n + g];
    const float4 po = sc.pos_op[g];
    Projected P;
    const bool visible = project_gaussian(cam, po, sc.m01[g], sc.m23[g], sc.m8r[g], near, W, H, P);
    float *o = out + (int64_t)perm[g] * 16;  // in the caller's index order
    for (int j = 0; j < 16; ++j) o[j] = 0.0f;
    if (!visible) {
        o[11] = 1.0f;  // x0 > x1 marks "not visible"
        return;
    }
    float dx = po.x - cam.C[0], dy = po.y - cam.C[1], dz = po.z - cam.C[2];
    const float inv = rsqrtf(fmaf(dx, dx, fmaf(dy, dy, dz * dz)));
    float r, gg, bb;
    sh_colour<DEG>(k, dx * inv, dy * inv, dz * inv, r, gg, bb);
    // conic back from the factor: A = ex^2, B = ex ey, C = ey^2 + fy^2 (unscaled)
    const float s = 1.0f / kHalfLog2e_sqrt;
    const float ex = P.A.z * s, ey = P.A.w * s, fy = P.B.x * s;
    o[0] = P.A.x; o[1] = P.A.y; o[2] = P.C.y; o[3] = P.B.y;
    o[4] = ex * ex; o[5] = ex * ey; o[6] = fmaf(ey, ey, fy * fy);
    o[7] = r; o[8] = gg; o[9] = bb;
    o[10] = (float)P.x0; o[11] = (float)P.x1; o[12] = (float)P.y0; o[13] = (float)P.y1;
    o[14] = 1.0f;
}

// ---------------------------------------------------------------- launch --
void launch_scene_prep(const float *means, const float *scales, const float *quats,
                       const float *opacity, const float *sh, int64_t n, int ncoef, float4 *pos_op,
                       float4 *m01, float4 *m23, float2 *m8r, float *sh_planar, float4 *quat,
                       float4 *scale, int *bad, hipStream_t st)
{
    const int bs = 256;
    const int64_t grid = (n + bs - 1) / bs;
    hipLaunchKernelGGL(k_scene_prep, dim3((unsigned)grid), dim3(bs), 0, st, means, scales, quats,
                       opacity, sh, n, ncoef, pos_op, m01, m23, m8r, sh_planar, quat, scale, bad);
}

void launch_camera_setup(const float *poses, const float *intr, const int32_t *cam_global,
                         int n_cams, int W, int H, CamParams *out, hipStream_t st,
                         const uint32_t *mask)
{
    const int bs = 64;
    hipLaunchKernelGGL(k_camera_setup, dim3((n_cams + bs - 1) / bs), dim3(bs), 0, st, poses,
                       intr, cam_global, n_cams, W, H, mask, out);
}

void launch_project(int deg, const ProjItem *items, int n_items, const SceneDev *scenes,
                    const CamParams *cams, const uint32_t *cam_slot, float near, int W, int H,
                    float4 *rec, uint2 *rect, uint32_t *zbits,
                    uint64_t *vis, hipStream_t st)
{
    if (n_items <= 0) return;
    dim3 grid(n_items), block(256);
    switch (deg) {
    case 0: hipLaunchKernelGGL(k_project<0>, grid, block, 0, st, items, scenes, cams, cam_slot, near, W, H, rec, rect, zbits, vis); break;
    case 1: hipLaunchKernelGGL(k_project<1>, grid, block, 0, st, items, scenes, cams, cam_slot, near, W, H, rec, rect, zbits, vis); break;
    case 2: hipLaunchKernelGGL(k_project<2>, grid, block, 0, st, items, scenes, cams, cam_slot, near, W, H, rec, rect, zbits, vis); break;
    default: hipLaunchKernelGGL(k_project<3>, grid, block, 0, st, items, scenes, cams, cam_slot, near, W, H, rec, rect, zbits, vis); break;
    }
}

void launch_debug_project(const SceneDev &sc, const int32_t *perm, const CamParams *cam,
                          float near, int W, int H, float *out, hipStream_t st)
{
    const int bs = 256;
    dim3 grid((unsigned)((sc.n + bs - 1) / bs));
    switch (sc.deg) {
    case 0: hipLaunchKernelGGL(k_debug_project<0>, grid, dim3(bs), 0, st, sc, perm, cam, near, W, H, out); break;
    case 1: hipLaunchKernelGGL(k_debug_project<1>, grid, dim3(bs), 0, st, sc, perm, cam, near, W, H, out); break;
    case 2: hipLaunchKernelGGL(k_debug_project<2>, grid, dim3(bs), 0, st, sc, perm, cam, near, W, H, out); break;
    default: hipLaunchKernelGGL(k_debug_project<3>, grid, dim3(bs), 0, st, sc, perm, cam, near, W, H, out); break;
    }
}

}  // namespace gs
