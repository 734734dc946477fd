// Device-side building blocks of the renderer (gfx950, wave64).
//
// Everything here is FP32. The per-Gaussian projection and the per-pixel
// compositing step are single inline functions used by every kernel form
// (plain, batched, persistent, any tile shape), so all forms produce
// bitwise-identical images.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gs {

// Fixed rules of the splat renderer (cited 3DGS, Sec. 2.3 of the paper):
// alpha clamp, skip threshold, stop threshold, low-pass, tangent clamp.
constexpr float kAlphaMax = 0.99f;
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kTMin = 1e-4f;
// The walk's scaled form of the same rules (see composite): thresholds on
// alpha / kAlphaMax and on kAlphaMax x the transmittance, and log2(kAlphaMax).
constexpr float kScaledAlphaMin = kAlphaMin / kAlphaMax;
constexpr float kScaledTMin = kTMin * kAlphaMax;
constexpr float kLog2AlphaMax = -0.0144995696951150891f;
constexpr float kLowPass = 0.3f;
constexpr float kTanClamp = 1.3f;
// sqrt(log2(e) / 2): folds the -1/2 of the Gaussian exponent and the change
// to base 2 into the per-Gaussian factor of the quadratic form.
constexpr float kHalfLog2e_sqrt = 0.84932180028801904272f;

constexpr int kWave = 64;

// Per-camera constants (step "camera setup"), one per chunk-local camera.
struct CamParams {
    float R[9];    // world -> camera rotation (row-major), R_wc = R_cw^T
    float t[3];    // world -> camera translation, t_wc = -R_wc C
    float C[3];    // camera centre in the world frame
    float fx, fy, cx, cy;
    float lxn, lxp, lyn, lyp;  // clamped tangent range of x/z and y/z
    float kx, ky;              // sqrt(1 + max clamped tangent^2): bounds |row of J| z / f
    float active;              // 1: render this camera; 0: it sees nothing (masked out)
    float pad[6];
};
static_assert(sizeof(CamParams) == 32 * 4, "CamParams is 128 B");

// Device view of one uploaded scene (structure of arrays).
struct SceneDev {
    const float4 *pos_op;  // [n] (mx, my, mz, opacity)
    const float4 *m01;     // [n] M = R(q) S row-major: (m00, m01, m02, m10)
    const float4 *m23;     // [n] (m11, m12, m20, m21)
    const float2 *m8r;     // [n] (m22, rad): rad = sqrt(2 ln(255 o)) * largest scale, the
                           // radius of the alpha >= 1/255 region (0 when o < 1/255)
    const float *sh;       // [(deg+1)^2 * 3][n] planar
    int64_t n;
    int32_t deg;
    int32_t pad;
};

// One projection work item: Gaussians [g0, g0 + 256) of `scene` seen by the
// chunk-local cameras [cam0, cam0 + ncam), ncam <= kProjCams. A block loads
// its Gaussians once for all of the item's cameras, so the scene is read
// once per kProjCams cameras.
constexpr int kProjCams = 64;

struct ProjItem {
    int32_t scene;
    int32_t g0;
    int32_t cam0;
    int32_t ncam;
};

// Raster-ready record of a visible (camera, Gaussian) pair, 48 contiguous
// bytes (the raster gathers it per tile instance):
//   A = (u, v, e_x, e_y)   with  e = e_x dx + e_y dy
//   B = (f_y, opacity, r, g)     f = f_y dy
//   C = (b, z, tau, 0)
// so that alpha = min(0.99, o * 2^-q), q = e^2 + f^2, at offset (dx, dy).
// (e, f) is the upper-triangular factor U of the conic, U^T U = Sigma'^-1,
// scaled by sqrt(log2(e)/2): a sum of squares, free of the cancellation of
// the expanded quadratic form for thin, magnified Gaussians.
// tau bounds q from above wherever alpha can reach 1/255 (log2(255 o) plus
// a rounding margin): a pixel rectangle whose smallest q exceeds tau cannot
// receive anything from the Gaussian. The binning record `rect` is the
// inclusive pixel box (x0 | x1 << 16, y0 | y1 << 16).

__device__ __forceinline__ uint64_t lanemask_lt()
{
    const uint32_t lane = __lane_id();
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Real SH (Condon-Shortley phase) colour, degree DEG, direction (x, y, z)
// unit; k[(l^2 + l + m) * 3 + c]. Polynomial forms of Y_lm derived from
// Y_lm = sqrt2 K_l^|m| P_l^|m|(cos th) {cos, sin}(|m| phi),
// K_l^m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!).
template <int DEG>
__device__ __forceinline__ void sh_colour(const float *k, float x, float y, float z, float &r,
                                          float &g, float &b)
{
    // l = 0: 1/(2 sqrt(pi))
    float y00 = 0.28209479177387814f;
    float acc[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[c] = y00 * k[c];
    if (DEG >= 1) {
        // l = 1: sqrt(3/(4 pi)) * (-y, z, -x)
        const float c1 = 0.48860251190291992f;
        float b1[3] = {-c1 * y, c1 * z, -c1 * x};
#pragma unroll
        for (int m = 0; m < 3; ++m)
#pragma unroll
            for (int c = 0; c < 3; ++c) acc[c] = fmaf(b1[m], k[(1 + m) * 3 + c], acc[c]);
    }
    if (DEG >= 2) {
        const float xx = x * x, yy = y * y, zz = z * z;
        // l = 2: (1/2)sqrt(15/pi) xy, -(1/2)sqrt(15/pi) yz,
        //        (1/4)sqrt(5/pi)(2zz - xx - yy), -(1/2)sqrt(15/pi) xz,
        //        (1/4)sqrt(15/pi)(xx - yy)
        const float c2a = 1.09254843059207907f;
        const float c2b = 0.31539156525252001f;
        const float c2c = 0.54627421529603954f;
        float b2[5] = {c2a * x * y, -c2a * y * z, c2b * (2.0f * zz - xx - yy), -c2a * x * z,
                       c2c * (xx - yy)};
#pragma unroll
        for (int m = 0; m < 5; ++m)
#pragma unroll
            for (int c = 0; c < 3; ++c) acc[c] = fmaf(b2[m], k[(4 + m) * 3 + c], acc[c]);
        if (DEG >= 3) {
            // l = 3: -(1/4)sqrt(35/(2pi)) y(3xx - yy), (1/2)sqrt(105/pi) xyz,
            //        -(1/4)sqrt(21/(2pi)) y(4zz - xx - yy),
            //        (1/4)sqrt(7/pi) z(2zz - 3xx - 3yy),
            //        -(1/4)sqrt(21/(2pi)) x(4zz - xx - yy),
            //        (1/4)sqrt(105/pi) z(xx - yy), -(1/4)sqrt(35/(2pi)) x(xx - 3yy)
            const float c3a = 0.59004358992664352f;
            const float c3b = 2.89061144264055406f;
            const float c3c = 0.45704579946446574f;
            const float c3d = 0.37317633259011540f;
            const float c3e = 1.44530572132027703f;
            float b3[7] = {-c3a * y * (3.0f * xx - yy),
                           c3b * x * y * z,
                           -c3c * y * (4.0f * zz - xx - yy),
                           c3d * z * (2.0f * zz - 3.0f * xx - 3.0f * yy),
                           -c3c * x * (4.0f * zz - xx - yy),
                           c3e * z * (xx - yy),
                           -c3a * x * (xx - 3.0f * yy)};
#pragma unroll
            for (int m = 0; m < 7; ++m)
#pragma unroll
                for (int c = 0; c < 3; ++c) acc[c] = fmaf(b3[m], k[(9 + m) * 3 + c], acc[c]);
        }
    }
    r = fmaxf(acc[0] + 0.5f, 0.0f);
    g = fmaxf(acc[1] + 0.5f, 0.0f);
    b = fmaxf(acc[2] + 0.5f, 0.0f);
}

struct Projected {
    float4 A, B, C;
    int x0, x1, y0, y1;  // inclusive pixel-centre box
};

// Smallest q(dx, dy) = (a dx + b dy)^2 + (c dy)^2 (a, c > 0) over the
// rectangle [X0, X1] x [Y0, Y1]: 0 if it holds the origin, otherwise the
// smallest of the four edge minima (1D quadratics, minimiser clamped to the
// edge). Evaluating q at a point of the edge can only over-estimate the
// edge minimum by the (second-order) error of the minimiser.
__device__ __forceinline__ float rect_min_q(float a, float b, float c, float X0, float X1, float Y0,
                                            float Y1)
{
    if (X0 <= 0.0f && X1 >= 0.0f && Y0 <= 0.0f && Y1 >= 0.0f) return 0.0f;
    const float ia = __builtin_amdgcn_rcpf(a);
    const float kv = a * b * __builtin_amdgcn_rcpf(fmaf(b, b, c * c));
    float best;
    {
        const float dx0 = fminf(fmaxf(-b * Y0 * ia, X0), X1);
        const float e0 = fmaf(a, dx0, b * Y0), f0 = c * Y0;
        const float dx1 = fminf(fmaxf(-b * Y1 * ia, X0), X1);
        const float e1 = fmaf(a, dx1, b * Y1), f1 = c * Y1;
        best = fminf(fmaf(e0, e0, f0 * f0), fmaf(e1, e1, f1 * f1));
    }
    {
        const float dy0 = fminf(fmaxf(-kv * X0, Y0), Y1);
        const float e0 = fmaf(a, X0, b * dy0), f0 = c * dy0;
        const float dy1 = fminf(fmaxf(-kv * X1, Y0), Y1);
        const float e1 = fmaf(a, X1, b * dy1), f1 = c * dy1;
        best = fminf(best, fminf(fmaf(e0, e0, f0 * f0), fmaf(e1, e1, f1 * f1)));
    }
    return best;
}

// Tiles of the footprint box: key = first + ty * tiles_x + tx.
struct TileBox {
    int tx0, ty0, bw, bh;
};

// Tile sizes are powers of two: lw = log2(tile width), lh = log2(tile height).
__device__ __forceinline__ TileBox tile_box(uint2 r, int lw, int lh)
{
    TileBox b;
    b.tx0 = (int)((r.x & 0xffffu) >> lw);
    b.ty0 = (int)((r.y & 0xffffu) >> lh);
    b.bw = (int)((r.x >> 16) >> lw) - b.tx0 + 1;
    b.bh = (int)((r.y >> 16) >> lh) - b.ty0 + 1;
    return b;
}

// Can the Gaussian (conic factor ex, ey, fy; threshold tau) reach alpha >=
// 1/255 at some pixel centre of a rectangle? The centres are at offsets
// [X0, X0 + w] x [Y0, Y0 + h] (pixel steps) from the Gaussian's mean.
__device__ __forceinline__ bool may_touch(float ex, float ey, float fy, float X0, float Y0,
                                         float w, float h, float tau)
{
    return rect_min_q(ex, ey, fy, X0, X0 + w, Y0, Y0 + h) <= tau;
}

// EWA projection of one Gaussian into one camera (steps: cull at the near
// plane; T = J W; Sigma' = T M M^T T^T + 0.3 I with M = R(q) S; conic
// factor; exact footprint box of alpha >= 1/255). Returns false when the
// Gaussian is behind the near plane, too transparent or off-image.
// Colour is filled by the caller (it needs the SH coefficients).
__device__ __forceinline__ bool project_gaussian(const CamParams &cam, float4 pos_op, float4 m01,
                                                 float4 m23, float2 m8r, float near, int W, int H,
                                                 Projected &P)
{
    const float mx = pos_op.x, my = pos_op.y, mz = pos_op.z, o = pos_op.w;
    const float x = fmaf(cam.R[0], mx, fmaf(cam.R[1], my, fmaf(cam.R[2], mz, cam.t[0])));
    const float y = fmaf(cam.R[3], mx, fmaf(cam.R[4], my, fmaf(cam.R[5], mz, cam.t[1])));
    const float z = fmaf(cam.R[6], mx, fmaf(cam.R[7], my, fmaf(cam.R[8], mz, cam.t[2])));
    if (!(z > near) || !(o >= kAlphaMin)) return false;
    {
        // Conservative screen test before the full projection. The exact box
        // half-width is sqrt(2 ln(255 o) Sigma'_xx) with Sigma'_xx <=
        // |J row|^2 (largest scale)^2 + 0.3 and sqrt(2 ln 255 * 0.3) < 1.83;
        // 1% and one pixel of slack cover the approximate reciprocal.
        const float rz = __builtin_amdgcn_rcpf(z);
        const float ub = fmaf(cam.fx * x, rz, cam.cx), vb = fmaf(cam.fy * y, rz, cam.cy);
        const float ex = fmaf(1.01f * m8r.y * rz, cam.fx * cam.kx, 2.84f);
        const float ey = fmaf(1.01f * m8r.y * rz, cam.fy * cam.ky, 2.84f);
        if (ub + ex < 0.0f || ub - ex > (float)W || vb + ey < 0.0f || vb - ey > (float)H)
            return false;
    }
    const float iz = 1.0f / z;
    const float xz = x * iz, yz = y * iz;
    const float u = fmaf(cam.fx, xz, cam.cx);
    const float v = fmaf(cam.fy, yz, cam.cy);
    const float txc = fminf(fmaxf(xz, cam.lxn), cam.lxp);
    const float tyc = fminf(fmaxf(yz, cam.lyn), cam.lyp);
    const float j00 = cam.fx * iz, j02 = -cam.fx * txc * iz;
    const float j11 = cam.fy * iz, j12 = -cam.fy * tyc * iz;
    // rows of T = J W
    const float t00 = fmaf(j02, cam.R[6], j00 * cam.R[0]);
    const float t01 = fmaf(j02, cam.R[7], j00 * cam.R[1]);
    const float t02 = fmaf(j02, cam.R[8], j00 * cam.R[2]);
    const float t10 = fmaf(j12, cam.R[6], j11 * cam.R[3]);
    const float t11 = fmaf(j12, cam.R[7], j11 * cam.R[4]);
    const float t12 = fmaf(j12, cam.R[8], j11 * cam.R[5]);
    // M = R(q) S, row-major m[3][3]
    const float M00 = m01.x, M01 = m01.y, M02 = m01.z, M10 = m01.w;
    const float M11 = m23.x, M12 = m23.y, M20 = m23.z, M21 = m23.w, M22 = m8r.x;
    // p = T_0 M, q = T_1 M  (so Sigma'_0 = [[p.p, p.q], [p.q, q.q]])
    const float p0 = fmaf(t00, M00, fmaf(t01, M10, t02 * M20));
    const float p1 = fmaf(t00, M01, fmaf(t01, M11, t02 * M21));
    const float p2 = fmaf(t00, M02, fmaf(t01, M12, t02 * M22));
    const float q0 = fmaf(t10, M00, fmaf(t11, M10, t12 * M20));
    const float q1 = fmaf(t10, M01, fmaf(t11, M11, t12 * M21));
    const float q2 = fmaf(t10, M02, fmaf(t11, M12, t12 * M22));
    const float pp = fmaf(p0, p0, fmaf(p1, p1, p2 * p2));
    const float qq = fmaf(q0, q0, fmaf(q1, q1, q2 * q2));
    const float pq = fmaf(p0, q0, fmaf(p1, q1, p2 * q2));
    // det(Sigma') = |p x q|^2 + 0.3 (|p|^2 + |q|^2) + 0.09 (Lagrange identity)
    const float cx_ = p1 * q2 - p2 * q1, cy_ = p2 * q0 - p0 * q2, cz_ = p0 * q1 - p1 * q0;
    const float cross2 = fmaf(cx_, cx_, fmaf(cy_, cy_, cz_ * cz_));
    const float a = pp + kLowPass, c = qq + kLowPass, b = pq;
    const float det = fmaf(kLowPass, pp + qq, cross2) + kLowPass * kLowPass;
    if (!(det > 0.0f)) return false;
    // upper factor of Sigma'^-1 = [[c, -b], [-b, a]] / det:
    //   e = sqrt(c/det) dx - b/sqrt(c det) dy,  f = dy / sqrt(c)
    const float rc = rsqrtf(c);
    const float rdet = rsqrtf(det);
    const float ex = c * rc * rdet;  // sqrt(c) / sqrt(det)
    const float ey = -b * rc * rdet;
    const float fy = rc;
    // footprint: alpha >= 1/255 <=> e^2 + f^2 <= r2 = 2 ln(o / alpha_min);
    // box half-extents r sqrt(Sigma'_xx), r sqrt(Sigma'_yy), widened a little
    // so that FP32 rounding never drops a contributing pixel.
    const float r2 = fmaxf(2.0f * logf(o * 255.0f), 0.0f);
    const float ext_x = fmaf(sqrtf(r2 * a), 1.001f, 0.01f);
    const float ext_y = fmaf(sqrtf(r2 * c), 1.001f, 0.01f);
    const float fx0 = ceilf(u - ext_x - 0.5f), fx1 = floorf(u + ext_x - 0.5f);
    const float fy0 = ceilf(v - ext_y - 0.5f), fy1 = floorf(v + ext_y - 0.5f);
    if (!(fx0 <= fx1) || !(fy0 <= fy1) || !(fx0 <= (float)(W - 1)) || !(fx1 >= 0.0f) ||
        !(fy0 <= (float)(H - 1)) || !(fy1 >= 0.0f))
        return false;
    P.x0 = (int)fmaxf(fx0, 0.0f);
    P.x1 = (int)fminf(fx1, (float)(W - 1));
    P.y0 = (int)fmaxf(fy0, 0.0f);
    P.y1 = (int)fminf(fy1, (float)(H - 1));
    P.A = make_float4(u, v, ex * kHalfLog2e_sqrt, ey * kHalfLog2e_sqrt);
    P.B = make_float4(fy * kHalfLog2e_sqrt, o, 0.0f, 0.0f);
    // alpha >= 1/255 needs q <= log2(255 o); margin for FP32 rounding
    const float tau = fmaf(log2f(o * 255.0f), 1.001f, 0.002f);
    P.C = make_float4(0.0f, z, tau, 0.0f);
    return true;
}

// Per-pixel state of the front-to-back walk: U = kAlphaMax x the
// transmittance T. The sign of U carries the stop flag: U > 0 while the
// pixel is live; a stop negates it, keeping |U| / kAlphaMax as the final
// transmittance.
struct Pixel {
    float U, r, g, b, zw;
};

// LDS form of a record: R0 = (ex, ey, fy, log2(0.99) - log2(opacity)),
// R1 = (r, g, b, z),
// and per wave (E0, F0) = (ex Xw + ey Yw, fy Yw) with (Xw, Yw) = the wave's
// 8x8 block origin + 0.5 - (u, v). For the pixel at (lx, ly) in the block
// (integers 0..7) the conic factor terms are e = ex lx + ey ly + E0 and
// f = fy ly + F0, and opacity * exp2(-(e^2 + f^2)) / 0.99 =
// exp2(-(e^2 + f^2 + R0.w)). The blocks form the same 8x8 grid for every
// tile shape, so a pixel's arithmetic does not depend on the tiling.
//
// One step of the walk for one (pixel, Gaussian) pair: alpha clamped to
// 0.99; skipped below 1/255; the walk stops (without this Gaussian) when the
// new transmittance would fall under 1e-4; otherwise weight alpha T is
// accumulated into colour and depth. In the scaled form a = alpha / 0.99 =
// min(1, exp2(-q)) (the clamp is the exponential's own output clamp), the
// weight is alpha T = a U and the new U is U - 0.99 a U, with the thresholds
// scaled alike: one instruction fewer per pair than clamping alpha itself.
// Branch-free: a pair that does not accumulate adds a zero weight, which
// leaves every sum bitwise unchanged; once stopped, U < 0 makes every later
// Un negative, so nothing accumulates. Returns whether the pair was
// accumulated.
__device__ __forceinline__ bool composite(Pixel &s, float lx, float ly, float4 R0, float4 R1,
                                          float E0, float F0)
{
    const float e = fmaf(R0.x, lx, fmaf(R0.y, ly, E0));
    const float f = fmaf(R0.z, ly, F0);
    const float q = fmaf(e, e, fmaf(f, f, R0.w));
    const float a = __builtin_amdgcn_fmed3f(__builtin_amdgcn_exp2f(-q), 0.0f, 1.0f);
    const bool hit = a >= kScaledAlphaMin;
    const float wt = a * s.U;
    const float Un = fmaf(-kAlphaMax, wt, s.U);
    const bool acc = hit & (Un >= kScaledTMin);
    const float w = acc ? wt : 0.0f;
    s.r = fmaf(w, R1.x, s.r);
    s.g = fmaf(w, R1.y, s.g);
    s.b = fmaf(w, R1.z, s.b);
    s.zw = fmaf(w, R1.w, s.zw);
    s.U = acc ? Un : (hit ? -fabsf(s.U) : s.U);
    return acc;
}

}  // namespace gs
