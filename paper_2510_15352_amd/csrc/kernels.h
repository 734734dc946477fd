// Host-side launchers of the renderer's HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gs {

struct CamParams;
struct SceneDev;
struct ProjItem;

// Device flags of one render: instance-buffer overflow, largest instance
// count of a chunk, and visible pairs / instances summed over the chunks.
struct RenderFlags {
    int32_t overflow;
    uint32_t max_inst;
    unsigned long long visible;
    unsigned long long instances;
    unsigned long long pairs_contrib;  // filled by the counting raster only
    unsigned long long pairs_eval;
    unsigned long long pairs_issued;
};

// What the device reports about finished renders, in mapped host memory:
// monotonic counts (never reset, so a render finishing while the host reads
// cannot undo an earlier report) and the counts of the last finished render.
struct RenderStatus {
    unsigned long long renders;    // renders finished
    unsigned long long overflows;  // of which overflowed an instance buffer
    unsigned long long max_inst;   // largest instance count of one chunk seen
    unsigned long long pad;
    RenderFlags last;              // the last finished render (all its lanes)
};

struct ScanTemp {
    uint32_t *partial;  // >= 4096 entries
};

struct SegSortTemp {
    uint32_t *hist;      // >= seg_sort_hist_entries(n_max, n_seg) entries
    uint32_t *tp;        // >= n_seg + 1 entries (tiles per segment, scanned)
    uint32_t *hist_len;  // 1 entry
    ScanTemp scan;
};

struct RasterArgs {
    const uint2 *ranges;   // [n_cams * tiles_per_cam] (start, end) into ivals
    const uint32_t *ivals; // tile-sorted instance values (record slots)
    const float4 *rec;          // 48-byte records by slot: A, B, C
    const int32_t *cam_global;  // chunk-local -> batch camera index
    const uint32_t *cam_mask;   // batch order, nullable: frames of cameras with 0 are not written
    int tiles_x, tiles_per_cam, W, H;
    float bg_r, bg_g, bg_b;
    float *rgb, *depth, *alpha;
    // 0: write the frame. 1, 2: a sub-frame of a blended frame, written (1)
    // or added (2) as rgb += blend_w * rgb_k, depth += sum of w z (before the
    // division), alpha += accumulated weight (alpha is then required).
    int blend;
    float blend_w;
};

// Backward pass (16x16 tiles: four 8x8 waves per tile; ten screen-space
// gradient values per record: u, v, conic xx, xy, yy, opacity, r, g, b, z).
constexpr int kBwdWaves = 4;
constexpr int kBwdVals = 10;
constexpr int kBwdBatch = 64;

struct BwdArgs {
    const uint2 *ranges;        // [n_cams * tiles_per_cam] into ivals
    const uint32_t *ivals;      // tile-sorted instance values (record slots)
    const float4 *rec;          // records by slot
    const uint2 *rect;          // pixel boxes by slot
    const uint32_t *inst_base;  // emission position of each slot's first instance
    const int32_t *cam_global;  // chunk-local -> batch camera index
    int tiles_x, tiles_per_cam, W, H;
    float bg_r, bg_g, bg_b;
    const float *g_rgb, *g_depth, *g_alpha;  // upstream gradients (nullable)
    float *partial;             // [instance][wave][10]
};

struct BwdGaussArgs {
    const float4 *pos_op, *m01, *m23;
    const float2 *m8r;
    const float *sh;            // planar [(deg+1)^2 * 3][n]
    const float4 *quat;         // unit quaternion (w, x, y, z)
    const float4 *scale;        // (sx, sy, sz, 1 / |q| as given)
    const int32_t *perm;        // caller's index of each stored Gaussian
    int64_t n;
    const CamParams *cams;      // the chunk's cameras
    const uint32_t *cam_slot;   // slot base of each chunk camera
    const uint64_t *vis;        // visibility words by slot / 64
    const float *rgrad;         // [slot][10]
    int n_cams;
    float *d_means, *d_scales, *d_quats, *d_opacity, *d_sh;  // caller order, added to
};

void launch_bwd_emission(const uint2 *srect, const uint32_t *dvals, const uint32_t *counts,
                         uint32_t n_max, uint32_t *cnt, uint32_t *base, uint32_t *inst_base,
                         float *partial, uint32_t cap, const ScanTemp &tmp, hipStream_t st);
void launch_bwd_raster(const BwdArgs &a, int n_cams, hipStream_t st);
void launch_bwd_record(const uint32_t *dvals, const uint32_t *base, const uint32_t *cnt,
                       const uint32_t *counts, uint32_t n_max, const float *partial, float *rgrad,
                       hipStream_t st);
void launch_bwd_gauss(int deg, const BwdGaussArgs &a, hipStream_t st);

// Sub-frame camera poses of a motion-blurred frame: for every camera i and
// sub-frame k < K, the pose with centre C_i - v_i * offs[k] (rotation kept),
// written as out[k][i][3][4].
void launch_blur_poses(const float *poses, const float *vel, int n_cams, const float *offs, int K,
                       float *out, hipStream_t st);
// Final pass of a blended frame: depth = (sum w z) / (sum of weights), or 0;
// alpha = (sum of weights) * inv_k.
void launch_blur_finalize(float *depth, float *alpha_sum, float *alpha_out, int64_t n_px,
                          float inv_k, hipStream_t st);

// quat / scale (nullable): the unit quaternion and (scales, 1 / |q|) kept
// for the backward pass.
void launch_scene_prep(const float *means, const float *scales, const float *quats,
                       const float *opacity, const float *sh, int64_t n, int ncoef, float4 *pos_op,
                       float4 *m01, float4 *m23, float2 *m8r, float *sh_planar, float4 *quat,
                       float4 *scale, int *bad, hipStream_t st);
// mask (nullable, batch order): cameras whose entry is 0 see nothing and
// their frames are left as they are.
void launch_camera_setup(const float *poses, const float *intr, const int32_t *cam_global,
                         int n_cams, int W, int H, CamParams *out, hipStream_t st,
                         const uint32_t *mask = nullptr);
void launch_project(int deg, const ProjItem *items, int n_items, const SceneDev *scenes,
                    const CamParams *cams, const uint32_t *cam_slot, float near, int W, int H,
                    float4 *rec, uint2 *rect, uint32_t *zbits,
                    uint64_t *vis, hipStream_t st);
void launch_debug_project(const SceneDev &sc, const int32_t *perm, const CamParams *cam,
                          float near, int W, int H, float *out, hipStream_t st);

void scan_u32(const uint32_t *in, const uint32_t *n_dev, uint32_t n_max, uint32_t *out,
              uint32_t *total_out, const ScanTemp &tmp, hipStream_t st);
// Order-preserving compaction of the set bits of the visibility words into
// (z bits, slot) pairs, camera-major; *n_vis_out receives their number and
// seg_start[c] (c <= n_cams) the first position of camera c.
void compact_visible(const uint64_t *vis, uint32_t n_words, const uint32_t *cam_slot, int n_cams,
                     const uint32_t *zbits, uint32_t *keys, uint32_t *vals, uint32_t *n_vis_out,
                     uint32_t *seg_start, const ScanTemp &tmp, hipStream_t st);
// Tile instances of the depth-sorted records (slots dvals, pixel boxes rect,
// both in sorted order), keyed by the tile index inside the camera:
// counts[1] = instances, counts[2] = min(instances, cap), flags
// updated; entries past cap dropped; inst_start[c] (c <= n_cams) = first
// instance of camera c.
void emit_instances(const uint32_t *dvals, const uint32_t *n_vis, uint32_t n_max,
                    const uint32_t *vis_start, int n_cams, const uint2 *rect, int tw, int th,
                    int tiles_x, uint32_t cap, uint32_t *ikeys, uint32_t *ivals,
                    uint32_t *inst_start, uint32_t *counts, RenderFlags *flags,
                    const ScanTemp &tmp, hipStream_t st);
// Stable sort of u32 keys by their low `bits` bits inside the segments
// [seg[c], seg[c+1]) (on the device; seg[0] = 0, n_seg <= 4096, the segments
// tile [0, seg[n_seg]) and seg[n_seg] <= n_max). The last pass adds
// c * seg_key_stride to the keys of segment c; with pay_dst set it writes
// pay_dst[i] = pay_src[value i * pay_stride] in sorted order instead of the
// keys. With ranges set (key output only), the last pass also folds every
// output key's [first, last + 1) position into ranges[key] with atomic min
// and max (the caller fills ranges with (~0, 0) first: fill_ranges). Returns
// 0 if the result is in (k0, v0), 1 if in (k1, v1).
int seg_sort_u32(uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1, const uint32_t *seg,
                 int n_seg, uint32_t n_max, int bits, uint32_t seg_key_stride,
                 const SegSortTemp &tmp, hipStream_t st, const uint2 *pay_src = nullptr,
                 uint2 *pay_dst = nullptr, uint32_t pay_stride = 1, uint2 *ranges = nullptr);
// ranges[0 .. n) = (~0, 0): every tile's range empty until the tile sort
// folds its instances in.
void fill_ranges(uint2 *ranges, uint64_t n, hipStream_t st);
uint64_t seg_sort_hist_entries(uint32_t n_max, int n_seg);

// Calibration kernels (kind 0: FMA chains, 1: v_exp_f32 chains, 2: copy of
// n float4 from src to dst); `blocks` blocks of 256 threads.
void launch_probe(int kind, float *scratch, int64_t n, int iters, const float4 *src, float4 *dst,
                  int blocks, hipStream_t st);

void launch_finalize_counts(uint32_t *counts, uint32_t cap, RenderFlags *flags, hipStream_t st);
void launch_zero_u32(uint32_t *p, uint64_t n, hipStream_t st);
bool raster_supported(int tw, int th, int b);
int raster_occupancy(int tw, int th, int b);
// count != nullptr selects the instrumented (pair-counting) grid kernel.
void launch_raster(int tw, int th, int b, bool persistent, const RasterArgs &a, int n_cams,
                   uint32_t *queue, int persistent_blocks, RenderFlags *count, hipStream_t st);

}  // namespace gs
