// Host runtime behind include/gs.h: scene store, camera-batch planner,
// workspace with device-side capacity checks, HIP-graph cache, autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <set>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/gs.h"
#include "gs_device.h"
#include "kernels.h"
#include "up_kernels.h"

using namespace gs;

namespace {

// A roctx range for the lifetime of the object (shown by rocprofv3
// --marker-trace; a no-op when no tool is attached).
struct TraceRange {
    explicit TraceRange(const char *name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

struct GsError : std::runtime_error {
    int code;
    GsError(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define HIP_CHECK(expr)                                                                      \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            throw GsError(e_ == hipErrorOutOfMemory ? GS_ERR_OOM : GS_ERR_HIP,               \
                          std::string(#expr) + ": " + hipGetErrorString(e_));                \
    } while (0)

template <typename T>
struct DevBuf {
    T *p = nullptr;
    size_t n = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    // Grow to at least `count` elements (contents are not preserved).
    bool reserve(size_t count)
    {
        if (count <= n && p) return false;
        release();
        size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
        HIP_CHECK(hipMalloc((void **)&p, bytes));
        n = std::max<size_t>(count, 1);
        return true;
    }
};

struct Scene {
    int64_t n = 0;
    int deg = 0;
    DevBuf<int32_t> perm;  // caller's index of each stored Gaussian
    DevBuf<float4> pos_op, m01, m23;
    DevBuf<float2> m8r;
    DevBuf<float> sh;
    DevBuf<float4> quat, scale;  // unit quaternion, (scales, 1/|q|): read by the backward pass
    int graph_refs = 0;
};

using DevFlags = RenderFlags;

struct Choice {
    int tw = 16, th = 16, batch = 128, chunk = 512, persistent = 0;
};

struct Chunk {
    int start = 0, count = 0;  // positions in the plan's camera order
    uint64_t slots = 0;        // visibility slots (sum of per-camera scene sizes, 64-aligned)
    int item_off[4] = {0, 0, 0, 0}, item_cnt[4] = {0, 0, 0, 0};
};

struct Plan {
    int n_cams = 0, W = 0, H = 0;
    Choice ch;
    int tiles_x = 0, tiles_y = 0, tiles_per_cam = 0;
    std::vector<int32_t> order;     // batch camera indices sorted by (scene, index)
    std::vector<uint32_t> cam_slot; // per order position, slot base inside its chunk
    std::vector<ProjItem> items;    // per chunk, grouped by SH degree
    std::vector<Chunk> chunks;
    std::vector<int32_t> scenes_used;
    uint64_t max_slots = 0;
    int max_chunk_cams = 0;
    DevBuf<int32_t> d_order;
    DevBuf<uint32_t> d_cam_slot;
    DevBuf<ProjItem> d_items;
};

// Buffers of one chunk pipeline.
struct Lane {
    DevBuf<float4> rec;  // 48-byte records by slot (A, B, C)
    DevBuf<uint2> rect, srect;  // pixel boxes by slot, and in depth order
    DevBuf<uint32_t> zbits;
    DevBuf<uint64_t> vis;
    DevBuf<uint32_t> dkeys[2], dvals[2];
    DevBuf<uint32_t> ikeys[2], ivals[2];
    DevBuf<uint32_t> vis_start, inst_start;  // per-camera segment starts (+ end)
    DevBuf<uint2> ranges;
    DevBuf<uint32_t> counts;  // [0] visible, [1] instances, [2] kept
    DevBuf<RenderFlags> flags;
    DevBuf<uint32_t> queue;
    DevBuf<uint32_t> scan_partial, sort_hist, sort_tp, sort_len;
};

constexpr int kLanes = 4;  // chunk pipelines, one stream each

struct LaneFlagPtrs {
    const RenderFlags *p[kLanes];
};

// End of a render (one thread): the render's counts over its lanes, folded
// into the monotonic device status, which is then written to the host's
// mapped copy (the host reads it after the render's event, or without
// waiting to look at renders that have finished).
__global__ void k_status_merge(LaneFlagPtrs lanes, int n_lanes, RenderStatus *dev,
                               RenderStatus *host)
{
    RenderFlags f{};
    for (int l = 0; l < n_lanes; ++l) {
        const RenderFlags &x = *lanes.p[l];
        f.overflow |= x.overflow;
        f.max_inst = max(f.max_inst, x.max_inst);
        f.visible += x.visible;
        f.instances += x.instances;
        f.pairs_contrib += x.pairs_contrib;
        f.pairs_eval += x.pairs_eval;
        f.pairs_issued += x.pairs_issued;
    }
    RenderStatus s = *dev;
    s.renders += 1;
    s.overflows += f.overflow ? 1ull : 0ull;
    if ((unsigned long long)f.max_inst > s.max_inst) s.max_inst = f.max_inst;
    s.last = f;
    *dev = s;
    *host = s;
    __threadfence_system();
}

// How the raster stores a frame: as the frame itself, or as sub-frame k of a
// blended (motion-blurred) frame (mode 1 for the first, 2 for the others).
struct Blend {
    int mode = 0;
    float w = 1.0f;
};
constexpr int kMaxChunkCams = 4096;  // segments of one segmented sort
constexpr int kMaxBlurSub = 16;      // sub-frames of a motion-blurred frame
// instance buffer entries per chunk: keeps every sort histogram index in 32 bits
constexpr uint64_t kMaxInstCap = uint64_t(1) << 31;

// Learned upsampler: FP32 master weights [cout][9][32] (layer 1's four input
// channels zero-padded to 32), Adam moments, BF16 packed copies, buffers.
constexpr int kUpCin[4] = {4, 32, 32, 32};
constexpr int kUpCout[4] = {32, 32, 32, 64};
constexpr int kUpCinM = 32;
constexpr int kUpChunk = 512;  // cameras per network pass of an upsampled render

struct Upsampler {
    bool ready = false;
    bool packed = false;
    int step = 0;
    DevBuf<float> w[4], b[4], mw[4], vw[4], mb[4], vb[4], gw[4], gb[4];
    DevBuf<uint16_t> wf[4], wd[4];
    // activations of up to `cap` images of h x w
    DevBuf<float> x0f, y4, lpart, wpart, bpart, scalar;
    DevBuf<uint16_t> x0b, a1, a2, a3, dy4, da3, da2, da1;
    // renders used by training and the upsampled form
    DevBuf<float> lo_rgb, lo_depth, hi_rgb, hi_depth, intr_lo, score;
    // fallback flags of the upsampled form (one per camera) and their count
    DevBuf<uint32_t> flags, n_flagged;
};

// Scratch of gs_upsampler_forward_noalloc: the FP32 four-channel input and
// the three BF16 32-channel activations of as many frames as fit (208 bytes
// per low-resolution pixel, each buffer 256-byte aligned). One copy per GPU
// for the life of the process; host code reaches it only through the
// address hipGetSymbolAddress returns for the current device.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
constexpr size_t kNoAllocBytesPerPixel = 4 * 4 + 3 * 32 * 2;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

struct GraphEntry {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<int32_t> scenes;
    std::unique_ptr<Plan> plan;
};

}  // namespace

struct gs_ctx {
    int device = 0;
    int cu_count = 0;
    std::string arch;  // gcnArchName of the device (autotune cache key)
    bool trace = false;  // GS_TRACE set: one line per render on stderr
    bool debug = false;  // GS_DEBUG set: eager renders check every stage
    unsigned char *scratch = nullptr;  // this device's copy of the scratch array
    std::string err;
    std::vector<std::unique_ptr<Scene>> scenes;
    DevBuf<SceneDev> d_scenes;
    bool scenes_dirty = true;

    // workspace: kLanes lanes (one per hardware queue), so that chunks'
    // rasters overlap other chunks' projection and sorts on other streams
    Lane lanes[kLanes];
    DevBuf<CamParams> cams;
    DevBuf<float> dbg_pose;
    // motion blur: sub-frame poses, time offsets, summed weights
    DevBuf<float> blur_poses, blur_offs, blur_asum;
    uint64_t inst_cap = 0;
    int generation = 0;  // bumps whenever a workspace buffer moves
    // Visibility slots of one camera chunk: the lanes' slot-indexed buffers
    // (record 48 B, two pixel boxes 16 B, depth key 4 B, two key/value pairs
    // 16 B) take at most a third of the device memory.
    uint64_t slot_budget = uint64_t(1) << 27;

    // device status of finished renders and its mapped host copy
    RenderStatus *status_host = nullptr;
    RenderStatus *status_host_dev = nullptr;  // device address of status_host
    DevBuf<RenderStatus> status_dev;
    unsigned long long acked_overflows = 0;   // overflows already acted on
    hipEvent_t ev_done = nullptr;             // recorded after every render
    bool pending = false;                     // an asynchronous render may still run
    bool last_deferred = false;               // the last render returned before finishing
    int capacity_errors = 0;                  // overflowed renders not yet reported
    // configurations (cameras, scenes, size, choice, pipelines) rendered once
    // with a wait, which sized the instance buffers for them
    std::set<std::string> sized;
    hipStream_t capture_stream = nullptr;
    // streams of the lanes after the first, for captured and eager renders
    hipStream_t capture_aux[kLanes - 1] = {};
    hipStream_t aux_stream[kLanes - 1] = {};
    hipEvent_t ev_fork = nullptr, ev_join[kLanes - 1] = {};

    Upsampler up;
    // backward pass: per-record tile counts, their scan, emission base by
    // slot, screen-space record gradients, per (instance, wave) partial sums
    DevBuf<uint32_t> bw_cnt, bw_base, bw_inst_base;
    DevBuf<float> bw_rgrad, bw_partial;
    std::vector<hipEvent_t> events;  // pool for stage timing
    std::map<std::string, std::unique_ptr<GraphEntry>> graphs;
    std::map<std::string, Choice> tuned;
    gs_stats last{};
    int graph_captures = 0;
};

namespace {

int fail(gs_ctx *ctx, int code, const std::string &msg)
{
    if (ctx) ctx->err = msg;
    return code;
}

template <class F>
int guarded(gs_ctx *ctx, F &&f)
{
    try {
        return f();
    } catch (const GsError &e) {
        return fail(ctx, e.code, e.what());
    } catch (const std::bad_alloc &) {
        return fail(ctx, GS_ERR_OOM, "host allocation failed");
    } catch (const std::exception &e) {
        return fail(ctx, GS_ERR_HIP, e.what());
    } catch (...) {
        return fail(ctx, GS_ERR_HIP, "unknown failure");
    }
}

uint64_t round64(uint64_t x) { return (x + 63) & ~uint64_t(63); }

int bits_for(uint64_t n_values)
{
    int b = 0;
    while (b < 63 && (uint64_t(1) << b) < n_values) ++b;
    return b;
}

void sync_scene_table(gs_ctx *ctx)
{
    if (!ctx->scenes_dirty) return;
    std::vector<SceneDev> tab(std::max<size_t>(ctx->scenes.size(), 1));
    for (size_t i = 0; i < ctx->scenes.size(); ++i) {
        SceneDev d{};
        if (ctx->scenes[i]) {
            Scene &s = *ctx->scenes[i];
            d.pos_op = s.pos_op.p;
            d.m01 = s.m01.p;
            d.m23 = s.m23.p;
            d.m8r = s.m8r.p;
            d.sh = s.sh.p;
            d.n = s.n;
            d.deg = s.deg;
        }
        tab[i] = d;
    }
    if (ctx->d_scenes.reserve(tab.size())) ++ctx->generation;
    HIP_CHECK(hipMemcpy(ctx->d_scenes.p, tab.data(), tab.size() * sizeof(SceneDev),
                        hipMemcpyHostToDevice));
    ctx->scenes_dirty = false;
}

Choice resolve_choice(gs_ctx *ctx, const gs_render_opts &o, int n_cams, int W, int H,
                      uint64_t total_gauss)
{
    Choice c;
    char key[128];
    snprintf(key, sizeof key, "%d:%d:%d:%d", W, H, n_cams, bits_for(total_gauss + 1));
    auto it = ctx->tuned.find(key);
    if (it != ctx->tuned.end()) c = it->second;
    if (o.tile_w > 0) c.tw = o.tile_w;
    if (o.tile_h > 0) c.th = o.tile_h;
    if (o.lds_batch > 0) c.batch = o.lds_batch;
    if (o.chunk_cams > 0) c.chunk = o.chunk_cams;
    if (o.persistent >= 0) c.persistent = o.persistent;
    if (o.mode == GS_MODE_PLAIN) {
        c.chunk = 1;
        c.persistent = 0;
    }
    return c;
}

std::string choice_key(const Choice &c)
{
    char b[96];
    snprintf(b, sizeof b, "%dx%d/b%d/c%d/p%d", c.tw, c.th, c.batch, c.chunk, c.persistent);
    return b;
}

// Cameras are grouped by scene (stable in batch order) and cut into chunks of
// at most `chunk` cameras and ~2^27 visibility slots; each chunk's projection
// is split into items of 256 Gaussians x up to 16 cameras of one scene.
std::unique_ptr<Plan> make_plan(gs_ctx *ctx, int n_cams, const int32_t *scene_ids, int W, int H,
                                const Choice &ch, const std::vector<int32_t> *subset = nullptr)
{
    // a subset renders only the listed batch cameras into their own slots
    if (subset) n_cams = (int)subset->size();
    constexpr int kCamGroup = kProjCams;
    const uint64_t kSlotBudget = ctx->slot_budget;
    auto P = std::make_unique<Plan>();
    P->n_cams = n_cams;
    P->W = W;
    P->H = H;
    P->ch = ch;
    P->tiles_x = (W + ch.tw - 1) / ch.tw;
    P->tiles_y = (H + ch.th - 1) / ch.th;
    P->tiles_per_cam = P->tiles_x * P->tiles_y;
    P->order.resize(n_cams);
    for (int i = 0; i < n_cams; ++i) P->order[i] = subset ? (*subset)[i] : i;
    std::stable_sort(P->order.begin(), P->order.end(),
                     [&](int a, int b) { return scene_ids[a] < scene_ids[b]; });
    P->cam_slot.resize(n_cams);
    int pos = 0;
    while (pos < n_cams) {
        Chunk c;
        c.start = pos;
        uint64_t slots = 0;
        while (pos < n_cams && c.count < ch.chunk) {
            const Scene &s = *ctx->scenes[scene_ids[P->order[pos]]];
            const uint64_t need = round64((uint64_t)s.n);
            if (c.count > 0 && slots + need > kSlotBudget) break;
            P->cam_slot[pos] = (uint32_t)slots;
            slots += need;
            ++c.count;
            ++pos;
        }
        c.slots = slots;
        // items, grouped by SH degree
        std::vector<ProjItem> per_deg[4];
        int run = c.start;
        while (run < c.start + c.count) {
            const int sid = scene_ids[P->order[run]];
            int end = run;
            while (end < c.start + c.count && scene_ids[P->order[end]] == sid) ++end;
            const Scene &s = *ctx->scenes[sid];
            for (int64_t g0 = 0; g0 < s.n; g0 += 256)
                for (int c0 = run; c0 < end; c0 += kCamGroup) {
                    ProjItem it;
                    it.scene = sid;
                    it.g0 = (int32_t)g0;
                    it.cam0 = c0 - c.start;
                    it.ncam = std::min(kCamGroup, end - c0);
                    per_deg[s.deg].push_back(it);
                }
            run = end;
        }
        for (int d = 0; d < 4; ++d) {
            c.item_off[d] = (int)P->items.size();
            c.item_cnt[d] = (int)per_deg[d].size();
            P->items.insert(P->items.end(), per_deg[d].begin(), per_deg[d].end());
        }
        P->max_slots = std::max(P->max_slots, slots);
        P->max_chunk_cams = std::max(P->max_chunk_cams, c.count);
        P->chunks.push_back(c);
    }
    for (int i = 0; i < n_cams; ++i) {
        const int sid = scene_ids[P->order[i]];
        if (std::find(P->scenes_used.begin(), P->scenes_used.end(), sid) == P->scenes_used.end())
            P->scenes_used.push_back(sid);
    }
    P->d_order.reserve(n_cams);
    P->d_cam_slot.reserve(n_cams);
    P->d_items.reserve(std::max<size_t>(P->items.size(), 1));
    HIP_CHECK(hipMemcpy(P->d_order.p, P->order.data(), n_cams * sizeof(int32_t),
                        hipMemcpyHostToDevice));
    HIP_CHECK(hipMemcpy(P->d_cam_slot.p, P->cam_slot.data(), n_cams * sizeof(uint32_t),
                        hipMemcpyHostToDevice));
    if (!P->items.empty())
        HIP_CHECK(hipMemcpy(P->d_items.p, P->items.data(), P->items.size() * sizeof(ProjItem),
                            hipMemcpyHostToDevice));
    return P;
}

// Grow the workspace of `n_lanes` lanes for a plan; returns true if any
// buffer moved.
bool ensure_workspace(gs_ctx *ctx, const Plan &P, int n_lanes)
{
    bool moved = false;
    const uint64_t slots = std::max<uint64_t>(P.max_slots, 64);
    if (ctx->inst_cap == 0) ctx->inst_cap = std::max<uint64_t>(uint64_t(1) << 20, slots / 2);
    ctx->inst_cap = std::min<uint64_t>(ctx->inst_cap, kMaxInstCap);
    for (int l = 0; l < n_lanes; ++l) {
        Lane &L = ctx->lanes[l];
        moved |= L.rec.reserve(slots * 3);
        moved |= L.rect.reserve(slots);
        moved |= L.srect.reserve(slots);
        moved |= L.zbits.reserve(slots);
        moved |= L.vis.reserve(slots / 64);
        for (int i = 0; i < 2; ++i) {
            moved |= L.dkeys[i].reserve(slots);
            moved |= L.dvals[i].reserve(slots);
            moved |= L.ikeys[i].reserve(ctx->inst_cap);
            moved |= L.ivals[i].reserve(ctx->inst_cap);
        }
        moved |= L.vis_start.reserve((uint64_t)P.max_chunk_cams + 1);
        moved |= L.inst_start.reserve((uint64_t)P.max_chunk_cams + 1);
        moved |= L.ranges.reserve((uint64_t)P.max_chunk_cams * P.tiles_per_cam);
        moved |= L.counts.reserve(4);
        moved |= L.flags.reserve(1);
        moved |= L.queue.reserve(1);
        moved |= L.scan_partial.reserve(4096);
        moved |= L.sort_hist.reserve(
            std::max(seg_sort_hist_entries((uint32_t)slots, P.max_chunk_cams),
                     seg_sort_hist_entries((uint32_t)ctx->inst_cap, P.max_chunk_cams)));
        moved |= L.sort_tp.reserve((uint64_t)P.max_chunk_cams + 1);
        moved |= L.sort_len.reserve(1);
    }
    moved |= ctx->cams.reserve(std::max(P.n_cams, 1));
    if (moved) ++ctx->generation;
    return moved;
}

// HIP events around each stage of an eager render.
struct StageTimer {
    gs_ctx *ctx;
    hipStream_t st;
    bool on;
    size_t used = 0;
    std::vector<std::array<size_t, 3>> marks;  // stage, begin event, end event
    size_t record()
    {
        if (used == ctx->events.size()) {
            hipEvent_t e;
            HIP_CHECK(hipEventCreate(&e));
            ctx->events.push_back(e);
        }
        HIP_CHECK(hipEventRecord(ctx->events[used], st));
        return used++;
    }
    size_t begin() { return on ? record() : 0; }
    void end(int stage, size_t b)
    {
        if (on) marks.push_back({(size_t)stage, b, record()});
    }
    void collect(gs_stats &s)
    {
        for (auto &m : marks) {
            float ms = 0.0f;
            HIP_CHECK(hipEventElapsedTime(&ms, ctx->events[m[1]], ctx->events[m[2]]));
            s.stage_ms[m[0]] += ms;
            s.stage_launches[m[0]] += 1;
        }
    }
};

void clear_graphs(gs_ctx *ctx);

// End of a render on `st` (after the join): fold the lanes' flags into the
// status block and record the render's event. Also used under capture.
void enqueue_status(gs_ctx *ctx, int n_lanes, hipStream_t st)
{
    LaneFlagPtrs lp{};
    for (int l = 0; l < n_lanes && l < kLanes; ++l) lp.p[l] = ctx->lanes[l].flags.p;
    hipLaunchKernelGGL(k_status_merge, dim3(1), dim3(1), 0, st, lp, std::min(n_lanes, kLanes),
                       ctx->status_dev.p, ctx->status_host_dev);
}

// GS_DEBUG: wait for stream s after a stage of an eager render and turn a
// device error into an error that names the stage (not while capturing).
void debug_check(gs_ctx *ctx, hipStream_t s, const char *stage)
{
    if (!ctx->debug) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) return;
    hipError_t e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess)
        throw GsError(GS_ERR_HIP, std::string("stage ") + stage + ": " + hipGetErrorString(e));
}

// Projection, compaction, depth sort, tile emission, tile sort and ranges
// of one chunk on lane L (stream s); returns which half of the instance
// ping-pong holds the tile-sorted instances (the depth-sorted records are
// in L.dvals[depth_half] when depth_half is given).
int enqueue_chunk_bins(gs_ctx *ctx, const Plan &P, const Chunk &c, Lane &L, hipStream_t s,
                       float near, uint32_t cap, StageTimer &T, int *depth_half = nullptr)
{
    const Choice &ch = P.ch;
    size_t t0;
    ScanTemp scan{L.scan_partial.p};
    SegSortTemp sort{L.sort_hist.p, L.sort_tp.p, L.sort_len.p, scan};
    const CamParams *cams = ctx->cams.p + c.start;
    const uint32_t *cam_slot = P.d_cam_slot.p + c.start;
    const uint32_t n_words = (uint32_t)(c.slots / 64);
    t0 = T.begin();
    for (int d = 0; d < 4; ++d)
        if (c.item_cnt[d])
            launch_project(d, P.d_items.p + c.item_off[d], c.item_cnt[d], ctx->d_scenes.p, cams,
                           cam_slot, near, P.W, P.H, L.rec.p, L.rect.p,
                           L.zbits.p, L.vis.p, s);
    T.end(GS_STAGE_PROJECT, t0);
    debug_check(ctx, s, "project");
    // visible count, order-preserving compaction, per-camera segments
    t0 = T.begin();
    compact_visible(L.vis.p, n_words, cam_slot, c.count, L.zbits.p, L.dkeys[0].p,
                    L.dvals[0].p, L.counts.p + 0, L.vis_start.p, scan, s);
    T.end(GS_STAGE_COMPACT, t0);
    debug_check(ctx, s, "compact");
    // depth sort inside each camera's segment: key = z bits (z > 0)
    t0 = T.begin();
    const int r = seg_sort_u32(L.dkeys[0].p, L.dvals[0].p, L.dkeys[1].p, L.dvals[1].p,
                               L.vis_start.p, c.count, (uint32_t)c.slots, 31, 0u, sort, s,
                               L.rect.p, L.srect.p);
    T.end(GS_STAGE_DEPTH_SORT, t0);
    debug_check(ctx, s, "depth sort");
    // tile instances in (camera, depth, index) order, keyed by tile
    t0 = T.begin();
    emit_instances(L.dvals[r].p, L.counts.p + 0, (uint32_t)c.slots, L.vis_start.p, c.count,
                   L.srect.p, ch.tw, ch.th, P.tiles_x, cap, L.ikeys[0].p, L.ivals[0].p,
                   L.inst_start.p, L.counts.p, L.flags.p, scan, s);
    T.end(GS_STAGE_EMIT, t0);
    debug_check(ctx, s, "emit");
    // stable sort by tile inside each camera keeps the depth order in
    // each tile
    const uint64_t n_tiles = (uint64_t)c.count * P.tiles_per_cam;
    const int tbits = std::max(1, bits_for((uint64_t)P.tiles_per_cam));
    // radix passes inside each camera's segment, the last one turning
    // the keys into camera * tiles + tile and folding each tile's first and
    // last instance into its range (every range empty before it)
    t0 = T.begin();
    fill_ranges(L.ranges.p, n_tiles, s);
    T.end(GS_STAGE_RANGES, t0);
    t0 = T.begin();
    const int r2 = seg_sort_u32(L.ikeys[0].p, L.ivals[0].p, L.ikeys[1].p, L.ivals[1].p,
                                L.inst_start.p, c.count, cap, tbits, (uint32_t)P.tiles_per_cam,
                                sort, s, nullptr, nullptr, 1, L.ranges.p);
    T.end(GS_STAGE_TILE_SORT, t0);
    debug_check(ctx, s, "tile sort and ranges");
    if (depth_half) *depth_half = r;
    return r2;
}

// Enqueue the whole render of a plan on `st` (also used under capture).
// With several lanes, chunk ci runs on lane ci mod n_lanes: lane 0 on `st`,
// lane l > 0 on aux[l - 1], forked from `st` after the camera setup and
// joined back at the end; each lane's chunks are serial on its stream, so a
// lane's buffers are reused only after its previous raster.
void enqueue_render(gs_ctx *ctx, const Plan &P, const float *poses, const float *intr, float near,
                    const float bg[3], float *rgb, float *depth, float *alpha, hipStream_t st,
                    const hipStream_t *aux, int n_lanes, StageTimer *tm = nullptr,
                    bool count_pairs = false, Blend blend = Blend{},
                    const uint32_t *cam_mask = nullptr)
{
    StageTimer off{ctx, st, false};
    StageTimer &T = tm ? *tm : off;
    const Choice &ch = P.ch;
    const uint32_t cap = (uint32_t)ctx->inst_cap;
    size_t t0 = T.begin();
    for (int l = 0; l < n_lanes; ++l)
        launch_zero_u32((uint32_t *)ctx->lanes[l].flags.p, sizeof(DevFlags) / 4, st);
    launch_camera_setup(poses, intr, P.d_order.p, P.n_cams, P.W, P.H, ctx->cams.p, st, cam_mask);
    T.end(GS_STAGE_SETUP, t0);
    if (n_lanes > 1) {
        HIP_CHECK(hipEventRecord(ctx->ev_fork, st));
        for (int l = 1; l < n_lanes; ++l) HIP_CHECK(hipStreamWaitEvent(aux[l - 1], ctx->ev_fork, 0));
    }
    int persistent_blocks = 0;
    if (ch.persistent)
        persistent_blocks = raster_occupancy(ch.tw, ch.th, ch.batch) * std::max(ctx->cu_count, 1);
    for (size_t ci = 0; ci < P.chunks.size(); ++ci) {
        const Chunk &c = P.chunks[ci];
        Lane &L = ctx->lanes[ci % n_lanes];
        const int lane = (int)(ci % (size_t)n_lanes);
        const hipStream_t s = lane ? aux[lane - 1] : st;
        T.st = s;
        const int r2 = enqueue_chunk_bins(ctx, P, c, L, s, near, cap, T);
        RasterArgs a;
        a.ranges = L.ranges.p;
        a.ivals = L.ivals[r2].p;
        a.rec = L.rec.p;
        a.cam_global = P.d_order.p + c.start;
        a.cam_mask = cam_mask;
        a.tiles_x = P.tiles_x;
        a.tiles_per_cam = P.tiles_per_cam;
        a.W = P.W;
        a.H = P.H;
        a.bg_r = bg[0];
        a.bg_g = bg[1];
        a.bg_b = bg[2];
        a.rgb = rgb;
        a.depth = depth;
        a.alpha = alpha;
        a.blend = blend.mode;
        a.blend_w = blend.w;
        t0 = T.begin();
        launch_raster(ch.tw, ch.th, ch.batch, ch.persistent != 0, a, c.count, L.queue.p,
                      persistent_blocks, count_pairs ? L.flags.p : nullptr, s);
        T.end(GS_STAGE_RASTER, t0);
        debug_check(ctx, s, "raster");
    }
    for (int l = 1; l < n_lanes; ++l) {
        HIP_CHECK(hipEventRecord(ctx->ev_join[l - 1], aux[l - 1]));
        HIP_CHECK(hipStreamWaitEvent(st, ctx->ev_join[l - 1], 0));
    }
    enqueue_status(ctx, n_lanes, st);
    HIP_CHECK(hipGetLastError());
}

// Wait for the last render and return its counts.
void wait_status(gs_ctx *ctx, DevFlags &out)
{
    HIP_CHECK(hipEventSynchronize(ctx->ev_done));
    ctx->pending = false;
    const volatile RenderStatus *h = ctx->status_host;
    out.overflow = h->last.overflow;
    out.max_inst = h->last.max_inst;
    out.visible = h->last.visible;
    out.instances = h->last.instances;
    out.pairs_contrib = h->last.pairs_contrib;
    out.pairs_eval = h->last.pairs_eval;
    out.pairs_issued = h->last.pairs_issued;
    // overflows of earlier renders on the stream that no call has reported yet
    const unsigned long long seen = h->overflows;
    const unsigned long long mine = out.overflow ? 1ull : 0ull;
    if (seen > ctx->acked_overflows + mine)
        ctx->capacity_errors += (int)(seen - ctx->acked_overflows - mine);
    ctx->acked_overflows = std::max(ctx->acked_overflows, seen);
}

// Grow the instance buffers past `need` instances per chunk (at least
// doubling); false when they are already at the 2^31 limit.
bool grow_instances(gs_ctx *ctx, uint64_t need)
{
    uint64_t want = std::max<uint64_t>(need + need / 4 + 1024, ctx->inst_cap * 2);
    if (want > kMaxInstCap) want = kMaxInstCap;
    if (want <= ctx->inst_cap) return false;
    ctx->inst_cap = want;
    return true;
}

// Without waiting: act on renders that have finished since the last look.
// An overflow grows the buffers and is kept for gs_render_status; a chunk
// that came within a fifth of the capacity grows them ahead of time. Either
// drops the captured graphs (their buffers move).
void poll_status(gs_ctx *ctx)
{
    const volatile RenderStatus *h = ctx->status_host;
    const unsigned long long seen = h->overflows, max_inst = h->max_inst;
    bool grow = false;
    if (seen > ctx->acked_overflows) {
        ctx->capacity_errors += (int)(seen - ctx->acked_overflows);
        ctx->acked_overflows = seen;
        grow = true;
    }
    if (max_inst * 5 > (unsigned long long)ctx->inst_cap * 4) grow = true;
    if (grow && grow_instances(ctx, max_inst)) clear_graphs(ctx);
}

void clear_graphs(gs_ctx *ctx)
{
    for (auto &kv : ctx->graphs) {
        GraphEntry &g = *kv.second;
        for (int32_t s : g.scenes)
            if (s >= 0 && s < (int)ctx->scenes.size() && ctx->scenes[s]) --ctx->scenes[s]->graph_refs;
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.graph) (void)hipGraphDestroy(g.graph);
    }
    ctx->graphs.clear();
}

int check_scene_ids(gs_ctx *ctx, int n_cams, const int32_t *scene_ids, uint64_t *total)
{
    uint64_t t = 0;
    std::vector<char> seen(ctx->scenes.size(), 0);
    for (int i = 0; i < n_cams; ++i) {
        const int32_t s = scene_ids[i];
        if (s < 0 || s >= (int)ctx->scenes.size() || !ctx->scenes[s])
            return fail(ctx, GS_ERR_INVALID_ARG, "scene_ids[" + std::to_string(i) + "] = " +
                                                     std::to_string(s) + " is not a live scene");
        if (!seen[s]) {
            seen[s] = 1;
            t += ctx->scenes[s]->n;
        }
    }
    *total = t;
    return GS_OK;
}

std::string graph_key(int n_cams, const int32_t *scene_ids, int W, int H, const Choice &ch,
                      float near, const float *bg, const void *poses, const void *intr,
                      const void *rgb, const void *depth, const void *alpha, int generation,
                      uint64_t cap, const std::vector<int32_t> *subset)
{
    uint64_t h = 1469598103934665603ull;
    for (int i = 0; i < n_cams; ++i) {
        h ^= (uint32_t)scene_ids[i];
        h *= 1099511628211ull;
    }
    if (subset) {
        h ^= 0x5bd1e995u;
        for (int32_t c : *subset) {
            h ^= (uint32_t)c + 1u;
            h *= 1099511628211ull;
        }
    }
    char b[512];
    snprintf(b, sizeof b, "%d|%llx|%dx%d|%s|%a|%a,%a,%a|%p|%p|%p|%p|%p|g%d|c%llu", n_cams,
             (unsigned long long)h, W, H, choice_key(ch).c_str(), near, bg[0], bg[1], bg[2], poses,
             intr, rgb, depth, alpha, generation, (unsigned long long)cap);
    return b;
}

int render_impl(gs_ctx *ctx, int32_t n_cams, const int32_t *scene_ids, const float *poses,
                const float *intr, int32_t W, int32_t H, float *rgb, float *depth, float *alpha,
                const gs_render_opts &o, hipStream_t st, const Choice *forced,
                const std::vector<int32_t> *subset = nullptr, Blend blend = Blend{},
                bool may_defer = false, const uint32_t *cam_mask = nullptr)
{
    uint64_t total = 0;
    int rc = check_scene_ids(ctx, n_cams, scene_ids, &total);
    if (rc) return rc;
    const int n_render = subset ? (int)subset->size() : n_cams;
    Choice ch = forced ? *forced : resolve_choice(ctx, o, n_render, W, H, total);
    if (!raster_supported(ch.tw, ch.th, ch.batch))
        return fail(ctx, GS_ERR_INVALID_ARG, "unsupported tile/batch choice " + choice_key(ch));
    if (ch.chunk < 1 || ch.chunk > kMaxChunkCams)
        return fail(ctx, GS_ERR_INVALID_ARG, "chunk_cams must be in [1, 4096]");
    const bool batched = o.mode != GS_MODE_PLAIN;
    const bool use_graph = batched && o.use_graph;
    // up to kLanes overlapped chunk pipelines for batched renders, except
    // when timing stages (their durations are measured one kernel at a time)
    const int n_lanes =
        (batched && !o.timing) ? (o.streams > 0 ? std::min<int>(o.streams, kLanes) : kLanes) : 1;
    sync_scene_table(ctx);
    poll_status(ctx);
    // renders share the context's work buffers: one enqueued on another
    // stream than the last one starts after it on the device
    if (ctx->pending) HIP_CHECK(hipStreamWaitEvent(st, ctx->ev_done, 0));
    char mask_key[32];
    snprintf(mask_key, sizeof mask_key, "|m%p", (const void *)cam_mask);
    const std::string tail = "|l" + std::to_string(n_lanes) + "|b" +
                             std::to_string(blend.mode) + ":" + std::to_string(blend.w) + mask_key;
    // the configuration without buffer addresses: the first render of it waits
    const std::string config = graph_key(n_cams, scene_ids, W, H, ch, o.near_plane, o.bg, nullptr,
                                         nullptr, nullptr, nullptr, nullptr, 0, 0, subset) + tail;
    const bool wait = !may_defer || o.sync || o.timing || o.count_pairs ||
                      ctx->sized.count(config) == 0;
    ctx->last = gs_stats{};
    int regrows = 0;
    size_t n_chunks = 0;
    bool captured = false;
    for (int attempt = 0; attempt < 6; ++attempt) {
        StageTimer timer{ctx, st, o.timing != 0};
        if (!use_graph) {
            // eager: the plain form is the same kernel sequence with one camera per chunk
            std::unique_ptr<Plan> P = make_plan(ctx, n_cams, scene_ids, W, H, ch, subset);
            n_chunks = P->chunks.size();
            if (ensure_workspace(ctx, *P, n_lanes)) clear_graphs(ctx);
            enqueue_render(ctx, *P, poses, intr, o.near_plane, o.bg, rgb, depth, alpha, st,
                           ctx->aux_stream, n_lanes, &timer, o.count_pairs != 0, blend, cam_mask);
        } else {
            std::string key = graph_key(n_cams, scene_ids, W, H, ch, o.near_plane, o.bg, poses,
                                        intr, rgb, depth, alpha, ctx->generation, ctx->inst_cap,
                                        subset) +
                              tail;
            auto it = ctx->graphs.find(key);
            if (it == ctx->graphs.end()) {
                TraceRange tr("gs capture");
                captured = true;
                auto g = std::make_unique<GraphEntry>();
                g->plan = make_plan(ctx, n_cams, scene_ids, W, H, ch, subset);
                if (ensure_workspace(ctx, *g->plan, n_lanes)) {
                    clear_graphs(ctx);
                    key = graph_key(n_cams, scene_ids, W, H, ch, o.near_plane, o.bg, poses, intr,
                                    rgb, depth, alpha, ctx->generation, ctx->inst_cap, subset) +
                          tail;
                }
                HIP_CHECK(hipStreamBeginCapture(ctx->capture_stream,
                                                hipStreamCaptureModeThreadLocal));
                try {
                    enqueue_render(ctx, *g->plan, poses, intr, o.near_plane, o.bg, rgb, depth,
                                   alpha, ctx->capture_stream, ctx->capture_aux, n_lanes, nullptr,
                                   false, blend, cam_mask);
                } catch (...) {
                    hipGraph_t junk = nullptr;
                    (void)hipStreamEndCapture(ctx->capture_stream, &junk);
                    if (junk) (void)hipGraphDestroy(junk);
                    throw;
                }
                HIP_CHECK(hipStreamEndCapture(ctx->capture_stream, &g->graph));
                HIP_CHECK(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
                g->scenes = g->plan->scenes_used;
                for (int32_t s : g->scenes) ++ctx->scenes[s]->graph_refs;
                ++ctx->graph_captures;
                it = ctx->graphs.emplace(key, std::move(g)).first;
            }
            n_chunks = it->second->plan->chunks.size();
            HIP_CHECK(hipGraphLaunch(it->second->exec, st));
        }
        HIP_CHECK(hipEventRecord(ctx->ev_done, st));
        ctx->pending = true;
        if (!wait) break;
        DevFlags f;
        wait_status(ctx, f);
        ctx->last = gs_stats{};
        ctx->last.visible = (int64_t)f.visible;
        ctx->last.instances = (int64_t)f.instances;
        ctx->last.pairs_contrib = (int64_t)f.pairs_contrib;
        ctx->last.pairs_evaluated = (int64_t)f.pairs_eval;
        ctx->last.pairs_issued = (int64_t)f.pairs_issued;
        timer.collect(ctx->last);
        if (!f.overflow) {
            ctx->sized.insert(config);
            break;
        }
        // grow the instance buffers past the largest chunk's need and retry
        ++regrows;
        if (!grow_instances(ctx, f.max_inst))
            return fail(ctx, GS_ERR_CAPACITY, "instance count per chunk exceeds 2^31");
        clear_graphs(ctx);
        if (attempt == 5) return fail(ctx, GS_ERR_CAPACITY, "instance buffers kept overflowing");
    }
    ctx->last.instance_capacity = (int64_t)ctx->inst_cap;
    ctx->last.regrows = regrows;
    ctx->last.graph_captures = ctx->graph_captures;
    ctx->last.tile_w = ch.tw;
    ctx->last.tile_h = ch.th;
    ctx->last.lds_batch = ch.batch;
    ctx->last.chunk_cams = ch.chunk;
    ctx->last.persistent = ch.persistent;
    ctx->last_deferred = !wait;
    if (ctx->trace)
        fprintf(stderr,
                "[gs] render: %d cameras %dx%d, choice %s, %zu chunks on %d pipelines, %s%s, "
                "%s, instance capacity %llu, regrows %d\n",
                n_render, W, H, choice_key(ch).c_str(), n_chunks, n_lanes,
                use_graph ? (captured ? "graph captured" : "graph replayed") : "eager",
                batched ? "" : " (plain)", wait ? "waited" : "returned before finishing",
                (unsigned long long)ctx->inst_cap, regrows);
    return GS_OK;
}

// Backward pass of the render of n_cams cameras of one scene: the forward
// binning of every chunk, then the gradient kernels (k_backward.hip), all on
// one stream so that the per-Gaussian sums are added chunk after chunk.
int render_backward_impl(gs_ctx *ctx, int32_t scene_id, int32_t n_cams, const float *poses,
                         const float *intr, int32_t W, int32_t H, const float *g_rgb,
                         const float *g_depth, const float *g_alpha, const gs_render_opts &o,
                         float *d_means, float *d_scales, float *d_quats, float *d_opacity,
                         float *d_sh, hipStream_t st)
{
    Scene &sc = *ctx->scenes[scene_id];
    const int nc = (sc.deg + 1) * (sc.deg + 1);
    std::vector<int32_t> ids((size_t)n_cams, scene_id);
    Choice ch;
    ch.tw = 16;
    ch.th = 16;
    ch.batch = kBwdBatch;
    ch.chunk = o.chunk_cams > 0 ? std::min(o.chunk_cams, kMaxChunkCams) : 512;
    ch.persistent = 0;
    sync_scene_table(ctx);
    if (ctx->pending) HIP_CHECK(hipStreamWaitEvent(st, ctx->ev_done, 0));
    ctx->last = gs_stats{};
    int regrows = 0;
    for (int attempt = 0; attempt < 6; ++attempt) {
        std::unique_ptr<Plan> P = make_plan(ctx, n_cams, ids.data(), W, H, ch);
        if (ensure_workspace(ctx, *P, 1)) clear_graphs(ctx);
        const uint64_t slots = std::max<uint64_t>(P->max_slots, 64);
        ctx->bw_cnt.reserve(slots);
        ctx->bw_base.reserve(slots);
        ctx->bw_inst_base.reserve(slots);
        ctx->bw_rgrad.reserve(slots * kBwdVals);
        ctx->bw_partial.reserve(ctx->inst_cap * kBwdWaves * kBwdVals);
        const uint32_t cap = (uint32_t)ctx->inst_cap;
        const int64_t n = sc.n;
        launch_zero_u32(reinterpret_cast<uint32_t *>(d_means), (uint64_t)n * 3, st);
        launch_zero_u32(reinterpret_cast<uint32_t *>(d_scales), (uint64_t)n * 3, st);
        launch_zero_u32(reinterpret_cast<uint32_t *>(d_quats), (uint64_t)n * 4, st);
        launch_zero_u32(reinterpret_cast<uint32_t *>(d_opacity), (uint64_t)n, st);
        launch_zero_u32(reinterpret_cast<uint32_t *>(d_sh), (uint64_t)n * nc * 3, st);
        Lane &L = ctx->lanes[0];
        launch_zero_u32(reinterpret_cast<uint32_t *>(L.flags.p), sizeof(DevFlags) / 4, st);
        launch_camera_setup(poses, intr, P->d_order.p, P->n_cams, W, H, ctx->cams.p, st);
        StageTimer off{ctx, st, false};
        for (const Chunk &c : P->chunks) {
            int r = 0;
            const int r2 = enqueue_chunk_bins(ctx, *P, c, L, st, o.near_plane, cap, off, &r);
            ScanTemp scan{L.scan_partial.p};
            launch_bwd_emission(L.srect.p, L.dvals[r].p, L.counts.p, (uint32_t)c.slots,
                                ctx->bw_cnt.p, ctx->bw_base.p, ctx->bw_inst_base.p,
                                ctx->bw_partial.p, cap, scan, st);
            BwdArgs a;
            a.ranges = L.ranges.p;
            a.ivals = L.ivals[r2].p;
            a.rec = L.rec.p;
            a.rect = L.rect.p;
            a.inst_base = ctx->bw_inst_base.p;
            a.cam_global = P->d_order.p + c.start;
            a.tiles_x = P->tiles_x;
            a.tiles_per_cam = P->tiles_per_cam;
            a.W = W;
            a.H = H;
            a.bg_r = o.bg[0];
            a.bg_g = o.bg[1];
            a.bg_b = o.bg[2];
            a.g_rgb = g_rgb;
            a.g_depth = g_depth;
            a.g_alpha = g_alpha;
            a.partial = ctx->bw_partial.p;
            launch_bwd_raster(a, c.count, st);
            launch_bwd_record(L.dvals[r].p, ctx->bw_base.p, ctx->bw_cnt.p, L.counts.p,
                              (uint32_t)c.slots, ctx->bw_partial.p, ctx->bw_rgrad.p, st);
            BwdGaussArgs b;
            b.pos_op = sc.pos_op.p;
            b.m01 = sc.m01.p;
            b.m23 = sc.m23.p;
            b.m8r = sc.m8r.p;
            b.sh = sc.sh.p;
            b.quat = sc.quat.p;
            b.scale = sc.scale.p;
            b.perm = sc.perm.p;
            b.n = n;
            b.cams = ctx->cams.p + c.start;
            b.cam_slot = P->d_cam_slot.p + c.start;
            b.vis = L.vis.p;
            b.rgrad = ctx->bw_rgrad.p;
            b.n_cams = c.count;
            b.d_means = d_means;
            b.d_scales = d_scales;
            b.d_quats = d_quats;
            b.d_opacity = d_opacity;
            b.d_sh = d_sh;
            launch_bwd_gauss(sc.deg, b, st);
        }
        enqueue_status(ctx, 1, st);
        HIP_CHECK(hipGetLastError());
        HIP_CHECK(hipEventRecord(ctx->ev_done, st));
        DevFlags f;
        wait_status(ctx, f);
        ctx->last.visible = (int64_t)f.visible;
        ctx->last.instances = (int64_t)f.instances;
        if (!f.overflow) break;
        ++regrows;
        if (!grow_instances(ctx, f.max_inst))
            return fail(ctx, GS_ERR_CAPACITY, "instance count per chunk exceeds 2^31");
        clear_graphs(ctx);
        if (attempt == 5) return fail(ctx, GS_ERR_CAPACITY, "instance buffers kept overflowing");
    }
    ctx->last.instance_capacity = (int64_t)ctx->inst_cap;
    ctx->last.regrows = regrows;
    ctx->last.tile_w = ch.tw;
    ctx->last.tile_h = ch.th;
    ctx->last.lds_batch = ch.batch;
    ctx->last.chunk_cams = ch.chunk;
    return GS_OK;
}

int validate_render_args(gs_ctx *ctx, int32_t n_cams, const int32_t *scene_ids, const float *poses,
                         const float *intr, int32_t W, int32_t H, const float *rgb,
                         const float *depth)
{
    if (!ctx) return GS_ERR_INVALID_ARG;
    if (n_cams < 1) return fail(ctx, GS_ERR_INVALID_ARG, "n_cams must be >= 1");
    if (!scene_ids || !poses || !intr || !rgb || !depth)
        return fail(ctx, GS_ERR_INVALID_ARG, "null scene_ids/poses/intrinsics/rgb/depth");
    if (W < 1 || H < 1 || W > 65535 || H > 65535)
        return fail(ctx, GS_ERR_INVALID_ARG, "width/height must be in [1, 65535]");
    return GS_OK;
}

}  // namespace


namespace {

// ------------------------------------------------------------- upsampler --

int64_t up_num_params()
{
    int64_t n = 0;
    for (int l = 0; l < 4; ++l) n += (int64_t)kUpCout[l] * 9 * kUpCin[l] + kUpCout[l];
    return n;
}

void up_zero_state(gs_ctx *ctx)
{
    Upsampler &U = ctx->up;
    for (int l = 0; l < 4; ++l) {
        const size_t nw = (size_t)kUpCout[l] * 9 * kUpCinM, nb = kUpCout[l];
        U.w[l].reserve(nw);
        U.b[l].reserve(nb);
        U.mw[l].reserve(nw);
        U.vw[l].reserve(nw);
        U.mb[l].reserve(nb);
        U.vb[l].reserve(nb);
        U.gw[l].reserve(nw);
        U.gb[l].reserve(nb);
        U.wf[l].reserve((size_t)9 * kUpCout[l] * kUpCinM);
        U.wd[l].reserve((size_t)9 * kUpCout[l] * kUpCinM);
        HIP_CHECK(hipMemset(U.mw[l].p, 0, nw * 4));
        HIP_CHECK(hipMemset(U.vw[l].p, 0, nw * 4));
        HIP_CHECK(hipMemset(U.mb[l].p, 0, nb * 4));
        HIP_CHECK(hipMemset(U.vb[l].p, 0, nb * 4));
    }
    U.step = 0;
    U.packed = false;
}

// Parameter-vector layout (host) -> padded FP32 device tensors.
void up_put(DevBuf<float> *wdst, DevBuf<float> *bdst, const float *params)
{
    const float *src = params;
    for (int l = 0; l < 4; ++l) {
        const int ci = kUpCin[l], co = kUpCout[l];
        std::vector<float> w((size_t)co * 9 * kUpCinM, 0.0f);
        for (int o = 0; o < co; ++o)
            for (int t = 0; t < 9; ++t)
                for (int c = 0; c < ci; ++c) w[((size_t)o * 9 + t) * kUpCinM + c] = src[((size_t)o * 9 + t) * ci + c];
        src += (size_t)co * 9 * ci;
        HIP_CHECK(hipMemcpy(wdst[l].p, w.data(), w.size() * 4, hipMemcpyHostToDevice));
        HIP_CHECK(hipMemcpy(bdst[l].p, src, (size_t)co * 4, hipMemcpyHostToDevice));
        src += co;
    }
}

// Parameter vector (oracle layout) -> FP32 master weights; Adam reset.
void up_set(gs_ctx *ctx, const float *params)
{
    Upsampler &U = ctx->up;
    up_zero_state(ctx);
    up_put(U.w, U.b, params);
    U.ready = true;
}

// FP32 master tensors (weights or their gradients) -> oracle layout.
void up_get(gs_ctx *ctx, DevBuf<float> *wsrc, DevBuf<float> *bsrc, float *params)
{
    float *dst = params;
    for (int l = 0; l < 4; ++l) {
        const int ci = kUpCin[l], co = kUpCout[l];
        std::vector<float> w((size_t)co * 9 * kUpCinM);
        HIP_CHECK(hipMemcpy(w.data(), wsrc[l].p, w.size() * 4, hipMemcpyDeviceToHost));
        for (int o = 0; o < co; ++o)
            for (int t = 0; t < 9; ++t)
                for (int c = 0; c < ci; ++c) dst[((size_t)o * 9 + t) * ci + c] = w[((size_t)o * 9 + t) * kUpCinM + c];
        dst += (size_t)co * 9 * ci;
        HIP_CHECK(hipMemcpy(dst, bsrc[l].p, (size_t)co * 4, hipMemcpyDeviceToHost));
        dst += co;
    }
}

void up_pack(gs_ctx *ctx, hipStream_t st)
{
    Upsampler &U = ctx->up;
    for (int l = 0; l < 4; ++l)
        launch_pack_weights(U.w[l].p, kUpCout[l], kUpCinM, kUpCinM, U.wf[l].p,
                            l > 0 ? U.wd[l].p : nullptr, st);
    U.packed = true;
}

void up_alloc(gs_ctx *ctx, int n, int h, int w, bool train)
{
    Upsampler &U = ctx->up;
    const size_t px = (size_t)n * h * w;
    U.x0f.reserve(px * 4);
    U.x0b.reserve(px * 32);
    U.a1.reserve(px * 32);
    U.a2.reserve(px * 32);
    U.a3.reserve(px * 32);
    U.y4.reserve(px * 64);
    U.scalar.reserve(4);
    if (train) {
        U.dy4.reserve(px * 64);
        U.da3.reserve(px * 32);
        U.da2.reserve(px * 32);
        U.da1.reserve(px * 32);
        U.lpart.reserve((size_t)up_head_blocks(n, h, w));
        U.wpart.reserve((size_t)up_conv_blocks(n, h, w) * 64 * 9 * 32);
        U.bpart.reserve((size_t)up_conv_blocks(n, h, w) * 64);
    }
}

// x0b / x0f of n images must be filled; writes y4.
// Network forward. With rgb / depth set (inference) the last layer's
// epilogue is the head and writes the full-resolution frames; otherwise the
// last layer writes y4 (FP32) for the training head.
// Inference network on given buffers: x0f (n h w FP32 four-channel input)
// -> a1 -> a2 -> a3 (BF16, 32 channels) -> the head, which writes the
// full-resolution frames.
void up_infer(gs_ctx *ctx, int n, int h, int w, hipStream_t st, const float *x0f, uint16_t *a1,
              uint16_t *a2, uint16_t *a3, float *rgb, float *depth)
{
    Upsampler &U = ctx->up;
    launch_up_conv(32, 32, UP_EPI_RELU_BF16_IN4, nullptr, U.wf[0].p, U.b[0].p, n, h, w, nullptr,
                   a1, st, x0f);
    launch_up_conv(32, 32, UP_EPI_RELU_BF16, a1, U.wf[1].p, U.b[1].p, n, h, w, nullptr, a2, st);
    launch_up_conv(32, 32, UP_EPI_RELU_BF16, a2, U.wf[2].p, U.b[2].p, n, h, w, nullptr, a3, st);
    launch_up_conv(32, 64, UP_EPI_HEAD, a3, U.wf[3].p, U.b[3].p, n, h, w, nullptr, nullptr, st,
                   x0f, rgb, depth);
}

void up_forward(gs_ctx *ctx, int n, int h, int w, hipStream_t st, float *rgb = nullptr,
                float *depth = nullptr)
{
    Upsampler &U = ctx->up;
    if (rgb) {  // inference: the first layer reads x0f directly
        up_infer(ctx, n, h, w, st, U.x0f.p, U.a1.p, U.a2.p, U.a3.p, rgb, depth);
        return;
    }
    launch_up_conv(32, 32, UP_EPI_RELU_BF16, U.x0b.p, U.wf[0].p, U.b[0].p, n, h, w, nullptr,
                   U.a1.p, st);
    launch_up_conv(32, 32, UP_EPI_RELU_BF16, U.a1.p, U.wf[1].p, U.b[1].p, n, h, w, nullptr, U.a2.p, st);
    launch_up_conv(32, 32, UP_EPI_RELU_BF16, U.a2.p, U.wf[2].p, U.b[2].p, n, h, w, nullptr, U.a3.p, st);
    launch_up_conv(32, 64, UP_EPI_F32, U.a3.p, U.wf[3].p, U.b[3].p, n, h, w, nullptr, U.y4.p, st);
}

// dy4 must be filled (training head); writes gw / gb of every layer.
void up_backward(gs_ctx *ctx, int n, int h, int w, hipStream_t st)
{
    Upsampler &U = ctx->up;
    const int nblk = up_conv_blocks(n, h, w);
    const uint16_t *xin[4] = {U.x0b.p, U.a1.p, U.a2.p, U.a3.p};
    uint16_t *dout[4] = {U.da1.p, U.da2.p, U.da3.p, U.dy4.p};  // dL/d(output of layer l)
    for (int l = 3; l >= 0; --l) {
        const int co = kUpCout[l];
        launch_up_wgrad(kUpCinM, co, xin[l], dout[l], n, h, w, U.wpart.p, U.bpart.p, st);
        launch_sum_partials(U.wpart.p, nblk, co * 9 * kUpCinM, U.gw[l].p, st);
        launch_sum_partials(U.bpart.p, nblk, co, U.gb[l].p, st);
        if (l > 0)  // dL/d(input of layer l), masked by ReLU'(previous output)
            launch_up_conv(co, kUpCinM, UP_EPI_MASK_BF16, dout[l], U.wd[l].p, nullptr, n, h, w,
                           xin[l], dout[l - 1], st);
    }
}

float up_loss_and_grads(gs_ctx *ctx, int n, int h, int w, const float *rgb_lo,
                        const float *depth_lo, const float *rgb_hi, const float *depth_hi,
                        hipStream_t st)
{
    Upsampler &U = ctx->up;
    up_alloc(ctx, n, h, w, true);
    if (!U.packed) up_pack(ctx, st);
    launch_up_input(rgb_lo, depth_lo, (int64_t)n * h * w, U.x0f.p, U.x0b.p, st);
    up_forward(ctx, n, h, w, st);
    launch_up_head(true, U.x0f.p, U.y4.p, h, w, n, nullptr, nullptr, rgb_hi, depth_hi, U.lpart.p,
                   U.dy4.p, st);
    up_backward(ctx, n, h, w, st);
    const int nb = up_head_blocks(n, h, w);
    launch_sum_partials(U.lpart.p, nb, 1, U.scalar.p, st);
    float loss = 0.0f;
    HIP_CHECK(hipMemcpyAsync(&loss, U.scalar.p, 4, hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    return loss / (float)((int64_t)n * h * w * 16);
}

void up_adam(gs_ctx *ctx, float lr, hipStream_t st)
{
    Upsampler &U = ctx->up;
    ++U.step;
    for (int l = 0; l < 4; ++l) {
        launch_adam(U.w[l].p, U.mw[l].p, U.vw[l].p, U.gw[l].p, kUpCout[l] * 9 * kUpCinM, lr, U.step, st);
        launch_adam(U.b[l].p, U.mb[l].p, U.vb[l].p, U.gb[l].p, kUpCout[l], lr, U.step, st);
    }
    U.packed = false;
}

// Cosine learning-rate schedule of the optimisation steps: lr0 at step 0,
// lr_min at step steps - 1 (half a cosine period), lr0 throughout for one step.
float up_cosine_lr(int s, int steps, float lr0, float lr_min)
{
    if (steps <= 1) return lr0;
    const double pi = 3.14159265358979323846;
    return (float)((double)lr_min + 0.5 * ((double)lr0 - (double)lr_min) *
                                        (1.0 + std::cos(pi * (double)s / (double)(steps - 1))));
}

// Confidence scores of n low-resolution frames, in chunks of the network's
// activation buffers.
void up_scores(gs_ctx *ctx, int n, int h, int w, const float *rgb_lo, const float *depth_lo,
               float *score, hipStream_t st)
{
    Upsampler &U = ctx->up;
    const int64_t lp = (int64_t)h * w;
    for (int c0 = 0; c0 < n; c0 += kUpChunk) {
        const int m = std::min(kUpChunk, n - c0);
        up_alloc(ctx, m, h, w, false);
        launch_up_input(rgb_lo + c0 * lp * 3, depth_lo + c0 * lp, m * lp, U.x0f.p, nullptr, st);
        launch_up_score(U.x0f.p, m, h, w, score + c0, st);
    }
}

uint64_t splitmix(uint64_t &x)
{
    uint64_t z = (x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

}  // namespace

extern "C" {

int gs_abi_sizes(int32_t *scene_desc, int32_t *render_opts, int32_t *stats)
{
    if (scene_desc) *scene_desc = (int32_t)sizeof(gs_scene_desc);
    if (render_opts) *render_opts = (int32_t)sizeof(gs_render_opts);
    if (stats) *stats = (int32_t)sizeof(gs_stats);
    return GS_OK;
}

void gs_default_opts(gs_render_opts *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->near_plane = 0.2f;
    o->mode = GS_MODE_BATCHED;
    o->persistent = -1;
    o->use_graph = 0;
}

int gs_create(int hip_device, gs_ctx **out)
{
    if (!out) return GS_ERR_INVALID_ARG;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return GS_ERR_HIP;
    if (hip_device < 0 || hip_device >= count) return GS_ERR_INVALID_ARG;
    auto *ctx = new (std::nothrow) gs_ctx();
    if (!ctx) return GS_ERR_OOM;
    int rc = guarded(ctx, [&] {
        ctx->device = hip_device;
        HIP_CHECK(hipSetDevice(hip_device));
        hipDeviceProp_t prop;
        HIP_CHECK(hipGetDeviceProperties(&prop, hip_device));
        ctx->cu_count = prop.multiProcessorCount;
        ctx->arch = prop.gcnArchName;
        const char *tr = std::getenv("GS_TRACE"), *dbg = std::getenv("GS_DEBUG");
        ctx->trace = tr && *tr && std::strcmp(tr, "0") != 0;
        ctx->debug = dbg && *dbg && std::strcmp(dbg, "0") != 0;
        {
            constexpr uint64_t kSlotBytes = 84;
            const uint64_t b = (uint64_t)prop.totalGlobalMem / (3 * kLanes * kSlotBytes);
            ctx->slot_budget = std::min<uint64_t>(std::max<uint64_t>(b, uint64_t(1) << 20),
                                                  uint64_t(1) << 30);
        }
        HIP_CHECK(hipHostMalloc((void **)&ctx->status_host, sizeof(RenderStatus),
                                hipHostMallocMapped));
        std::memset((void *)ctx->status_host, 0, sizeof(RenderStatus));
        HIP_CHECK(hipHostGetDevicePointer((void **)&ctx->status_host_dev, ctx->status_host, 0));
        ctx->status_dev.reserve(1);
        HIP_CHECK(hipMemset(ctx->status_dev.p, 0, sizeof(RenderStatus)));
        HIP_CHECK(hipEventCreateWithFlags(&ctx->ev_done, hipEventDisableTiming));
        HIP_CHECK(hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking));
        for (int l = 0; l < kLanes - 1; ++l) {
            HIP_CHECK(hipStreamCreateWithFlags(&ctx->capture_aux[l], hipStreamNonBlocking));
            HIP_CHECK(hipStreamCreateWithFlags(&ctx->aux_stream[l], hipStreamNonBlocking));
            HIP_CHECK(hipEventCreateWithFlags(&ctx->ev_join[l], hipEventDisableTiming));
        }
        HIP_CHECK(hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming));
        // the scratch array's address on this device (hip_device is current)
        HIP_CHECK(hipGetSymbolAddress((void **)&ctx->scratch, HIP_SYMBOL(scratch)));
        if (!ctx->scratch) throw GsError(GS_ERR_HIP, "no device address for the scratch array");
        return GS_OK;
    });
    if (rc != GS_OK) {
        gs_destroy(ctx);
        return rc;
    }
    *out = ctx;
    return GS_OK;
}

int gs_destroy(gs_ctx *ctx)
{
    if (!ctx) return GS_ERR_INVALID_ARG;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    clear_graphs(ctx);
    for (hipEvent_t e : ctx->events) (void)hipEventDestroy(e);
    if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
    if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
    for (int l = 0; l < kLanes - 1; ++l) {
        if (ctx->ev_join[l]) (void)hipEventDestroy(ctx->ev_join[l]);
        if (ctx->capture_aux[l]) (void)hipStreamDestroy(ctx->capture_aux[l]);
        if (ctx->aux_stream[l]) (void)hipStreamDestroy(ctx->aux_stream[l]);
    }
    if (ctx->ev_done) (void)hipEventDestroy(ctx->ev_done);
    if (ctx->status_host) (void)hipHostFree(ctx->status_host);
    delete ctx;
    return GS_OK;
}

const char *gs_last_error(const gs_ctx *ctx)
{
    if (!ctx) return "null context";
    return ctx->err.c_str();
}

int gs_upload_scene(gs_ctx *ctx, const gs_scene_desc *d, int32_t *scene_id_out)
{
    if (!ctx) return GS_ERR_INVALID_ARG;
    if (!d || !scene_id_out) return fail(ctx, GS_ERR_INVALID_ARG, "null descriptor or id output");
    if (d->n < 1 || d->n > (int64_t(1) << 30))
        return fail(ctx, GS_ERR_BAD_SCENE, "scene size must be in [1, 2^30]");
    if (d->sh_degree < 0 || d->sh_degree > 3)
        return fail(ctx, GS_ERR_BAD_SCENE, "sh_degree must be in 0..3");
    if (!d->means || !d->scales || !d->quats || !d->opacity || !d->sh)
        return fail(ctx, GS_ERR_BAD_SCENE, "null scene array");
    if (d->mem_kind != GS_MEM_HOST && d->mem_kind != GS_MEM_DEVICE)
        return fail(ctx, GS_ERR_INVALID_ARG, "mem_kind must be GS_MEM_HOST or GS_MEM_DEVICE");
    return guarded(ctx, [&] {
        HIP_CHECK(hipSetDevice(ctx->device));
        const int64_t n = d->n;
        const int nc = (d->sh_degree + 1) * (d->sh_degree + 1);
        auto s = std::make_unique<Scene>();
        s->n = n;
        s->deg = d->sh_degree;
        s->pos_op.reserve(n);
        s->m01.reserve(n);
        s->m23.reserve(n);
        s->m8r.reserve(n);
        s->sh.reserve((size_t)n * nc * 3);
        s->quat.reserve(n);
        s->scale.reserve(n);
        DevBuf<float> tmp;
        DevBuf<int> bad;
        bad.reserve(1);
        HIP_CHECK(hipMemset(bad.p, 0, sizeof(int)));
        // Host copies of the arrays, stored in Morton order of the means so that
        // the Gaussians of one wave are spatial neighbours (coherent culling).
        const size_t counts[5] = {(size_t)n * 3, (size_t)n * 3, (size_t)n * 4, (size_t)n,
                                  (size_t)n * nc * 3};
        const size_t widths[5] = {3, 3, 4, 1, (size_t)nc * 3};
        const float *src[5] = {d->means, d->scales, d->quats, d->opacity, d->sh};
        std::vector<std::vector<float>> host(5);
        for (int i = 0; i < 5; ++i) {
            host[i].resize(counts[i]);
            if (d->mem_kind == GS_MEM_HOST)
                std::memcpy(host[i].data(), src[i], counts[i] * sizeof(float));
            else
                HIP_CHECK(hipMemcpy(host[i].data(), src[i], counts[i] * sizeof(float),
                                    hipMemcpyDeviceToHost));
        }
        const float *hm = host[0].data();
        float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int64_t g = 0; g < n; ++g)
            for (int a = 0; a < 3; ++a) {
                const float v = hm[g * 3 + a];
                if (!std::isfinite(v))
                    return fail(ctx, GS_ERR_BAD_SCENE, "scene has non-finite means");
                lo[a] = std::min(lo[a], v);
                hi[a] = std::max(hi[a], v);
            }
        std::vector<std::pair<uint64_t, int32_t>> code(n);
        for (int64_t g = 0; g < n; ++g) {
            uint64_t c = 0;
            uint32_t qv[3];
            for (int a = 0; a < 3; ++a) {
                const float span = hi[a] - lo[a];
                const float t = span > 0 ? (hm[g * 3 + a] - lo[a]) / span : 0.0f;
                qv[a] = (uint32_t)std::min(2097151.0f, std::max(0.0f, t * 2097151.0f));
            }
            for (int bit = 20; bit >= 0; --bit)
                for (int a = 0; a < 3; ++a) c = (c << 1) | ((qv[a] >> bit) & 1u);
            code[g] = {c, (int32_t)g};
        }
        std::sort(code.begin(), code.end());
        std::vector<float> packed;
        size_t total = 0;
        for (size_t c : counts) total += c;
        packed.resize(total);
        size_t off[5];
        {
            size_t o = 0;
            for (int i = 0; i < 5; ++i) {
                off[i] = o;
                o += counts[i];
            }
        }
        std::vector<int32_t> perm(n);
        for (int64_t g = 0; g < n; ++g) {
            const int32_t from = code[g].second;
            perm[g] = from;
            for (int i = 0; i < 5; ++i)
                std::memcpy(packed.data() + off[i] + (size_t)g * widths[i],
                            host[i].data() + (size_t)from * widths[i], widths[i] * sizeof(float));
        }
        tmp.reserve(total);
        HIP_CHECK(hipMemcpy(tmp.p, packed.data(), total * sizeof(float), hipMemcpyHostToDevice));
        s->perm.reserve(n);
        HIP_CHECK(hipMemcpy(s->perm.p, perm.data(), n * sizeof(int32_t), hipMemcpyHostToDevice));
        const float *m = tmp.p + off[0], *sc = tmp.p + off[1], *q = tmp.p + off[2],
                    *op = tmp.p + off[3], *sh = tmp.p + off[4];
        launch_scene_prep(m, sc, q, op, sh, n, nc, s->pos_op.p, s->m01.p, s->m23.p, s->m8r.p,
                          s->sh.p, s->quat.p, s->scale.p, bad.p, nullptr);
        HIP_CHECK(hipGetLastError());
        int hbad = 0;
        HIP_CHECK(hipMemcpy(&hbad, bad.p, sizeof(int), hipMemcpyDeviceToHost));
        if (hbad)
            return fail(ctx, GS_ERR_BAD_SCENE,
                        "scene has non-finite values, non-positive scales, opacity outside "
                        "[0,1] or zero quaternions");
        int32_t id = -1;
        for (size_t i = 0; i < ctx->scenes.size(); ++i)
            if (!ctx->scenes[i]) {
                id = (int32_t)i;
                break;
            }
        if (id < 0) {
            id = (int32_t)ctx->scenes.size();
            ctx->scenes.emplace_back();
        }
        ctx->scenes[id] = std::move(s);
        ctx->scenes_dirty = true;
        ctx->sized.clear();
        *scene_id_out = id;
        return GS_OK;
    });
}

int gs_release_scene(gs_ctx *ctx, int32_t scene_id)
{
    if (!ctx) return GS_ERR_INVALID_ARG;
    if (scene_id < 0 || scene_id >= (int)ctx->scenes.size() || !ctx->scenes[scene_id])
        return fail(ctx, GS_ERR_INVALID_ARG, "no such scene");
    if (ctx->scenes[scene_id]->graph_refs > 0)
        return fail(ctx, GS_ERR_BUSY, "a captured graph still references the scene");
    return guarded(ctx, [&] {
        HIP_CHECK(hipSetDevice(ctx->device));
        HIP_CHECK(hipDeviceSynchronize());
        ctx->scenes[scene_id].reset();
        ctx->scenes_dirty = true;
        ctx->sized.clear();
        return GS_OK;
    });
}

int64_t gs_scene_size(gs_ctx *ctx, int32_t scene_id)
{
    if (!ctx) return GS_ERR_INVALID_ARG;
    if (scene_id < 0 || scene_id >= (int)ctx->scenes.size() || !ctx->scenes[scene_id])
        return fail(ctx, GS_ERR_INVALID_ARG, "no such scene");
    return ctx->scenes[scene_id]->n;
}

int gs_render_batch(gs_ctx *ctx, int32_t n_cams, const int32_t *scene_ids, const float *poses,
                    const float *intrinsics, int32_t width, int32_t height, float *rgb,
                    float *depth, float *alpha, const gs_render_opts *opts, void *stream)
{
    TraceRange trace_range("gs_render_batch");
    int rc = validate_render_args(ctx, n_cams, scene_ids, poses, intrinsics, width, height, rgb,
                                  depth);
    if (rc) return rc;
    gs_render_opts o;
    if (opts) o = *opts; else gs_default_opts(&o);
    if (o.mode != GS_MODE_PLAIN && o.mode != GS_MODE_BATCHED)
        return fail(ctx, GS_ERR_INVALID_ARG, "mode must be GS_MODE_PLAIN or GS_MODE_BATCHED");
    if (!(o.near_plane > 0.0f) || !std::isfinite(o.near_plane))
        return fail(ctx, GS_ERR_INVALID_ARG, "near_plane must be a positive finite value");
    return guarded(ctx, [&] {
        HIP_CHECK(hipSetDevice(ctx->device));
        return render_impl(ctx, n_cams, scene_ids, poses, intrinsics, width, height, rgb, depth,
                           alpha, o, (hipStream_t)stream, nullptr, nullptr, Blend{}, true);
    });
}

int gs_render_backward(gs_ctx *ctx, int32_t scene_id, int32_t n_cams, const float *poses,
                       const float *intrinsics, int32_t width, int32_t height,
                       const float *grad_rgb, const float *grad_depth, const float *grad_alpha,
                       const gs_render_opts *opts, float *d_means, float *d_scales,
                       float *d_quats, float *d_opacity, float *d_sh, void *stream)
{
    TraceRange trace_range("gs_render_backward");
    if (!ctx) return GS_ERR_INVALID_ARG;
    if (scene_id < 0 || scene_id >= (int)ctx->scenes.size() || !ctx->scenes[scene_id])
        return fail(ctx, GS_ERR_INVALID_ARG, "no such scene");
    if (n_cams < 1) return fail(ctx, GS_ERR_INVALID_ARG, "n_cams must be >= 1");
    if (!poses || !intrinsics)
        return fail(ctx, GS_ERR_INVALID_ARG, "null poses/intrinsics");
    if (!grad_rgb && !grad_depth && !grad_alpha)
        return fail(ctx, GS_ERR_INVALID_ARG, "no upstream gradient given");
    if (!d_means || !d_scales || !d_quats || !d_opacity || !d_sh)
        return fail(ctx, GS_ERR_INVALID_ARG, "null gradient output");
    if (width < 1 || height < 1 || width > 65535 || height > 65535)
        return fail(ctx, GS_ERR_INVALID_ARG, "width/height must be in [1, 65535]");
    gs_render_opts o;
    gs_default_opts(&o);
    if (opts) o = *opts;
    return guarded(ctx, [&] {
        HIP_CHECK(hipSetDevice(ctx->device));
        return render_backward_impl(ctx, scene_id, n_cams, poses, intrinsics, width, height,
                                    grad_rgb, grad_depth, grad_alpha, o, d_means, d_scales,
                                    d_quats, d_opacity, d_sh, (hipStream_t)stream);
    });
}

int gs_render_due(gs_ctx *ctx, int32_t n_cams, const int32_t *scene_ids, const float *poses,
                  const float *intrinsics, int32_t width, int32_t height, int64_t sim_step,
                  int32_t period, const int32_t *phase, float *rgb, float *depth, float *alpha,
                  const gs_render_opts *opts, int32_t *n_due_out, void *stream)
{
    TraceRange trace_range("gs_render_due");
    int rc = validate_render_args(ctx, n_cams, scene_ids, poses, intrinsics, width, height, rgb,
                                  depth);
    if (rc) return rc;
    if (period < 1) return fail(ctx, GS_ERR_INVALID_ARG, "period must be >= 1");
    if (sim_step < 0) return fail(ctx, GS_ERR_INVALID_ARG, "sim_step must be >= 0");
    gs_render_opts o;
    if (opts) o = *opts; else gs_default_opts(&o);
    if (o.mode != GS_MODE_PLAIN && o.mode != GS_MODE_BATCHED)
        return fail(ctx, GS_ERR_INVALID_ARG, "mode must be GS_MODE_PLAIN or GS_MODE_BATCHED");
    if (!(o.near_plane > 0.0f) || !std::isfinite(o.near_plane))
        return fail(ctx, GS_ERR_INVALID_ARG, "near_plane must be a positive finite value");
    // camera i is due when (sim_step + phase_i) is a multiple of the period
    std::vector<int32_t> due;
    for (int32_t i = 0; i < n_cams; ++i) {
        const int64_t ph = phase ? (int64_t)phase[i] : (int64_t)i;
        if (ph < 0) return fail(ctx, GS_ERR_INVALID_ARG, "phase values must be >= 0");
        if ((sim_step + ph) % period == 0) due.push_back(i);
    }
    if (n_due_out) *n_due_out = (int32_t)due.size();
    if (due.empty()) {
        ctx->last = gs_stats{};
        return GS_OK;
    }
    return guarded(ctx, [&] {
        HIP_CHECK(hipSetDevice(ctx->device));
        return render_impl(ctx, n_cams, scene_ids, poses, intrinsics, width, height, rgb, depth,
                           alpha, o, (hipStream_t)stream, nullptr, &due);
    });
}

int gs_render_batch_motion_blur(gs_ctx *ctx, int32_t n_cams, const int32_t *scene_ids,
                                const float *poses, const float *velocities,
                                const float *intrinsics, int32_t width, int32_t height,
                                float shutter, int32_t n_sub, float *rgb, float *depth,
                                float *alpha, const gs_render_opts *opts, void *stream)
{
    TraceRange trace_range("gs_render_batch_motion_blur");
    int rc = validate_render_args(ctx, n_cams, scene_ids, poses, intrinsics, width, height, rgb,
                                  depth);
    if (rc) return rc;
    if (!velocities) return fail(ctx, GS_ERR_INVALID_ARG, "null velocities");
    if (n_sub < 1 || n_sub > kMaxBlurSub)
        return fail(ctx, GS_ERR_INVALID_ARG, "n_sub must be in [1, 16]");
    if (!(shutter >= 0.0f) || !std::isfinite(shutter))
        return fail(ctx, GS_ERR_INVALID_ARG, "shutter must be a finite value >= 0");
    gs_render_opts o;
    if (opts) o = *opts; else gs_default_opts(&o);
    if (o.mode != GS_MODE_PLAIN && o.mode != GS_MODE_BATCHED)
        return fail(ctx, GS_ERR_INVALID_ARG, "mode must be GS_MODE_PLAIN or GS_MODE_BATCHED");
    if (!(o.near_plane > 0.0f) || !std::isfinite(o.near_plane))
        return fail(ctx, GS_ERR_INVALID_ARG, "near_plane must be a positive finite value");
    return guarded(ctx, [&] {
        HIP_CHECK(hipSetDevice(ctx->device));
        const hipStream_t st = (hipStream_t)stream;
        const int64_t n_px = (int64_t)n_cams * width * height;
        // sub-frame k sits at the middle of the k-th of n_sub equal parts of
        // the exposure [t - shutter, t]
        float offs[kMaxBlurSub];
        for (int k = 0; k < n_sub; ++k) offs[k] = (float)((double)shutter * (k + 0.5) / n_sub);
        bool moved = ctx->blur_poses.reserve((size_t)n_sub * n_cams * 12);
        moved |= ctx->blur_offs.reserve(kMaxBlurSub);
        float *asum = alpha;
        if (!alpha) {
            moved |= ctx->blur_asum.reserve((size_t)n_px);
            asum = ctx->blur_asum.p;
        }
        if (moved) {
            // graphs captured with the old addresses of these buffers
            clear_graphs(ctx);
            ++ctx->generation;
        }
        HIP_CHECK(hipMemcpyAsync(ctx->blur_offs.p, offs, sizeof(float) * n_sub,
                                 hipMemcpyHostToDevice, st));
        launch_blur_poses(poses, velocities, n_cams, ctx->blur_offs.p, n_sub, ctx->blur_poses.p, st);
        const float w = 1.0f / (float)n_sub;
        // an instance-buffer regrow inside a sub-frame re-runs that sub-frame
        // on top of its partial sums: start the blend over (capacity only
        // grows, so this ends)
        int64_t regrows = 0;
        for (int attempt = 0; attempt < 4; ++attempt) {
            bool clean = true;
            for (int k = 0; k < n_sub && clean; ++k) {
                Blend b;
                b.mode = k == 0 ? 1 : 2;
                b.w = w;
                int r = render_impl(ctx, n_cams, scene_ids, ctx->blur_poses.p + (size_t)k * n_cams * 12,
                                    intrinsics, width, height, rgb, depth, asum, o, st, nullptr,
                                    nullptr, b);
                if (r) return r;
                if (ctx->last.regrows > 0) {
                    regrows += ctx->last.regrows;
                    clean = false;
                }
            }
            if (clean) {
                launch_blur_finalize(depth, asum, alpha, n_px, w, st);
                HIP_CHECK(hipGetLastError());
                ctx->last.regrows = regrows;
                return GS_OK;
            }
        }
        return fail(ctx, GS_ERR_CAPACITY, "instance buffers kept overflowing");
    });
}

int gs_peak_probe(gs_ctx *ctx, int32_t kind, double *rate_out)
{
    if (!ctx || !rate_out) return GS_ERR_INVALID_ARG;
    if (kind < 0 || kind > 2) return fail(ctx, GS_ERR_INVALID_ARG, "kind must be 0, 1 or 2");
    return guarded(ctx, [&] {
        HIP_CHECK(hipSetDevice(ctx->device));
        hipStream_t st = nullptr;
        HIP_CHECK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        hipEvent_t e0 = nullptr, e1 = nullptr;
        HIP_CHECK(hipEventCreate(&e0));
        HIP_CHECK(hipEventCreate(&e1));
        const int blocks = std::max(ctx->cu_count, 1) * 32;  // 8 waves per SIMD
        const int iters = 4096;
        const int64_t n = int64_t(1) << 26;                   // 1 GiB of float4
        DevBuf<float> scratch;
        DevBuf<float4> src, dst;
        scratch.reserve((size_t)blocks * 256);
        if (kind == 2) {
            src.reserve((size_t)n);
            dst.reserve((size_t)n);
            HIP_CHECK(hipMemsetAsync(src.p, 0, (size_t)n * sizeof(float4), st));
        }
        float best = 1e30f;
        for (int rep = 0; rep < 4; ++rep) {  // the first run warms up
            HIP_CHECK(hipEventRecord(e0, st));
            launch_probe(kind, scratch.p, n, iters, src.p, dst.p, kind == 2 ? blocks * 4 : blocks,
                         st);
            HIP_CHECK(hipEventRecord(e1, st));
            HIP_CHECK(hipEventSynchronize(e1));
            float ms = 0.0f;
            HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
            if (rep > 0) best = std::min(best, ms);
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        (void)hipStreamDestroy(st);
        const double sec = (double)best * 1e-3;
        if (kind == 2)
            *rate_out = 2.0 * (double)n * sizeof(float4) / sec;  // bytes read + written
        else
            *rate_out = (double)blocks * 256.0 * iters * 8.0 / sec;  // lane-ops
        return GS_OK;
    });
}

int gs_last_stats(gs_ctx *ctx, gs_stats *out)
{
    if (!ctx || !out) return GS_ERR_INVALID_ARG;
    return guarded(ctx, [&] {
        if (ctx->last_deferred) {
            // the last render returned before it finished: wait for its counts
            HIP_CHECK(hipSetDevice(ctx->device));
            DevFlags f;
            wait_status(ctx, f);
            ctx->last.visible = (int64_t)f.visible;
            ctx->last.instances = (int64_t)f.instances;
            ctx->last.pairs_contrib = (int64_t)f.pairs_contrib;
            ctx->last.pairs_evaluated = (int64_t)f.pairs_eval;
            ctx->last.pairs_issued = (int64_t)f.pairs_issued;
            ctx->last_deferred = false;
        }
        *out = ctx->last;
        out->instance_capacity = (int64_t)ctx->inst_cap;
        return GS_OK;
    });
}

int gs_render_status(gs_ctx *ctx, int32_t wait)
{
    if (!ctx) return GS_ERR_INVALID_ARG;
    return guarded(ctx, [&] {
        HIP_CHECK(hipSetDevice(ctx->device));
        if (wait && ctx->pending) {
            HIP_CHECK(hipEventSynchronize(ctx->ev_done));
            ctx->pending = false;
        } else if (ctx->pending) {
            const hipError_t q = hipEventQuery(ctx->ev_done);
            if (q != hipSuccess && q != hipErrorNotReady)
                throw GsError(GS_ERR_HIP, std::string("render failed: ") + hipGetErrorString(q));
        }
        poll_status(ctx);
        if (ctx->capacity_errors > 0) {
            const int n = ctx->capacity_errors;
            ctx->capacity_errors = 0;
            return fail(ctx, GS_ERR_CAPACITY,
                        std::to_string(n) + " render(s) overflowed the instance buffers and are "
                        "incomplete; the buffers now hold " + std::to_string(ctx->inst_cap) +
                        " instances per chunk: render again");
        }
        return GS_OK;
    });
}

int gs_set_instance_capacity(gs_ctx *ctx, int64_t cap)
{
    if (!ctx) return GS_ERR_INVALID_ARG;
    if (cap < 1 || cap > (int64_t)kMaxInstCap)
        return fail(ctx, GS_ERR_INVALID_ARG, "capacity out of range [1, 2^31]");
    return guarded(ctx, [&] {
        HIP_CHECK(hipSetDevice(ctx->device));
        HIP_CHECK(hipDeviceSynchronize());
        clear_graphs(ctx);
        ctx->sized.clear();
        // the largest chunk seen so far no longer drives the buffer size (the
        // device is idle here, so the status can be rewritten)
        RenderStatus st{};
        HIP_CHECK(hipMemcpy(&st, ctx->status_dev.p, sizeof st, hipMemcpyDeviceToHost));
        st.max_inst = 0;
        HIP_CHECK(hipMemcpy(ctx->status_dev.p, &st, sizeof st, hipMemcpyHostToDevice));
        ctx->status_host->max_inst = 0;
        for (Lane &L : ctx->lanes)
            for (int i = 0; i < 2; ++i) {
                L.ikeys[i].release();
                L.ivals[i].release();
            }
        ctx->inst_cap = (uint64_t)cap;
        ++ctx->generation;
        return GS_OK;
    });
}

int gs_clear_graphs(gs_ctx *ctx)
{
    if (!ctx) return GS_ERR_INVALID_ARG;
    return guarded(ctx, [&] {
        HIP_CHECK(hipSetDevice(ctx->device));
        HIP_CHECK(hipDeviceSynchronize());
        clear_graphs(ctx);
        return GS_OK;
    });
}

int gs_debug_project(gs_ctx *ctx, int32_t scene_id, const float *pose, const float *intrinsics,
                     int32_t width, int32_t height, float near_plane, float *out)
{
    if (!ctx) return GS_ERR_INVALID_ARG;
    if (!pose || !intrinsics || !out) return fail(ctx, GS_ERR_INVALID_ARG, "null argument");
    if (scene_id < 0 || scene_id >= (int)ctx->scenes.size() || !ctx->scenes[scene_id])
        return fail(ctx, GS_ERR_INVALID_ARG, "no such scene");
    if (width < 1 || height < 1 || width > 65535 || height > 65535)
        return fail(ctx, GS_ERR_INVALID_ARG, "width/height must be in [1, 65535]");
    return guarded(ctx, [&] {
        HIP_CHECK(hipSetDevice(ctx->device));
        sync_scene_table(ctx);
        ctx->dbg_pose.reserve(16);
        ctx->cams.reserve(1);
        float h[16];
        std::memcpy(h, pose, 12 * sizeof(float));
        std::memcpy(h + 12, intrinsics, 4 * sizeof(float));
        HIP_CHECK(hipMemcpy(ctx->dbg_pose.p, h, sizeof h, hipMemcpyHostToDevice));
        launch_camera_setup(ctx->dbg_pose.p, ctx->dbg_pose.p + 12, nullptr, 1, width, height,
                            ctx->cams.p, nullptr);
        const Scene &s = *ctx->scenes[scene_id];
        SceneDev sd{};
        sd.pos_op = s.pos_op.p;
        sd.m01 = s.m01.p;
        sd.m23 = s.m23.p;
        sd.m8r = s.m8r.p;
        sd.sh = s.sh.p;
        sd.n = s.n;
        sd.deg = s.deg;
        launch_debug_project(sd, s.perm.p, ctx->cams.p, near_plane, width, height, out, nullptr);
        HIP_CHECK(hipGetLastError());
        HIP_CHECK(hipDeviceSynchronize());
        return GS_OK;
    });
}

int gs_autotune(gs_ctx *ctx, int32_t n_cams, const int32_t *scene_ids, const float *poses,
                const float *intrinsics, int32_t width, int32_t height, float *rgb, float *depth,
                const char *cache_path, void *stream)
{
    TraceRange trace_range("gs_autotune");
    int rc = validate_render_args(ctx, n_cams, scene_ids, poses, intrinsics, width, height, rgb,
                                  depth);
    if (rc) return rc;
    return guarded(ctx, [&] {
        HIP_CHECK(hipSetDevice(ctx->device));
        hipStream_t st = (hipStream_t)stream;
        uint64_t total = 0;
        int r = check_scene_ids(ctx, n_cams, scene_ids, &total);
        if (r) return r;
        char key[128];
        snprintf(key, sizeof key, "%d:%d:%d:%d", width, height, n_cams, bits_for(total + 1));
        // the cache key adds the GPU (architecture and compute units)
        const std::string ckey = ctx->arch.substr(0, ctx->arch.find(':')) + ":" +
                                 std::to_string(ctx->cu_count) + "cu:" + key;
        if (cache_path) {
            // the last entry for this key in the cache file, if any, is used as is
            FILE *f = fopen(cache_path, "r");
            bool found = false;
            Choice cached;
            if (f) {
                char line[8192];
                const std::string want = "\"key\": \"" + ckey + "\"";
                while (fgets(line, sizeof line, f)) {
                    if (!strstr(line, want.c_str())) continue;
                    const char *b = strstr(line, "\"best\": \"");
                    Choice c;
                    if (b && sscanf(b + 9, "%dx%d/b%d/c%d/p%d", &c.tw, &c.th, &c.batch, &c.chunk,
                                    &c.persistent) == 5 &&
                        raster_supported(c.tw, c.th, c.batch) && c.chunk >= 1 &&
                        c.chunk <= kMaxChunkCams) {
                        cached = c;
                        found = true;
                    }
                }
                fclose(f);
            }
            if (found) {
                ctx->tuned[key] = cached;
                ctx->last = gs_stats{};
                ctx->last.tile_w = cached.tw;
                ctx->last.tile_h = cached.th;
                ctx->last.lds_batch = cached.batch;
                ctx->last.chunk_cams = cached.chunk;
                ctx->last.persistent = cached.persistent;
                return GS_OK;
            }
        }
        gs_render_opts o;
        gs_default_opts(&o);
        // candidates in order of preference, the library default first:
        // among choices timed within 2% of the fastest the earliest wins, so
        // timing noise does not flip the pick between near-equal choices
        std::vector<Choice> cands;
        cands.push_back(Choice{});
        const int shapes[][2] = {{16, 16}, {32, 8}, {16, 8}, {8, 8}, {32, 16}};
        const int batches[] = {128, 64, 256};
        const int chunks[] = {512, 1024, 256, 128, 64};
        for (auto &s : shapes)
            for (int b : batches)
                if (raster_supported(s[0], s[1], b))
                    for (int p = 0; p < 2; ++p) {
                        Choice c;
                        c.tw = s[0];
                        c.th = s[1];
                        c.batch = b;
                        c.chunk = 512;
                        c.persistent = p;
                        if (choice_key(c) != choice_key(cands[0])) cands.push_back(c);
                    }
        constexpr float kTie = 1.02f;
        hipEvent_t e0, e1;
        HIP_CHECK(hipEventCreate(&e0));
        HIP_CHECK(hipEventCreate(&e1));
        auto time_choice = [&](const Choice &c, int reps) -> float {
            int rr = render_impl(ctx, n_cams, scene_ids, poses, intrinsics, width, height, rgb,
                                 depth, nullptr, o, st, &c);
            if (rr) throw GsError(rr, ctx->err);
            float best = 1e30f;
            for (int rep = 0; rep < reps; ++rep) {
                HIP_CHECK(hipEventRecord(e0, st));
                rr = render_impl(ctx, n_cams, scene_ids, poses, intrinsics, width, height, rgb,
                                 depth, nullptr, o, st, &c);
                if (rr) throw GsError(rr, ctx->err);
                HIP_CHECK(hipEventRecord(e1, st));
                HIP_CHECK(hipEventSynchronize(e1));
                float ms = 0;
                HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
                best = std::min(best, ms);
            }
            return best;
        };
        std::vector<std::pair<Choice, float>> table;
        auto pick = [&](size_t from) {
            float fastest = 1e30f;
            for (size_t i = from; i < table.size(); ++i) fastest = std::min(fastest, table[i].second);
            for (size_t i = from; i < table.size(); ++i)
                if (table[i].second <= fastest * kTie) return table[i];
            return table[from];
        };
        for (const Choice &c : cands) table.push_back({c, time_choice(c, 2)});
        // the chunk sizes differ by a few percent: the picked shape and its
        // chunk variants are timed again over more replays
        const Choice shape = pick(0).first;
        const size_t second = table.size();
        for (int ck : chunks) {
            Choice c = shape;
            c.chunk = ck;
            table.push_back({c, time_choice(c, 6)});
        }
        const std::pair<Choice, float> chosen = pick(second);
        const Choice best = chosen.first;
        const float best_ms = chosen.second;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        ctx->tuned[key] = best;
        if (cache_path) {
            FILE *f = fopen(cache_path, "a");
            if (f) {
                fprintf(f, "{\"key\": \"%s\", \"best\": \"%s\", \"best_ms\": %.4f, \"table\": {", ckey.c_str(),
                        choice_key(best).c_str(), best_ms);
                for (size_t i = 0; i < table.size(); ++i)
                    fprintf(f, "%s\"%s\": %.4f", i ? ", " : "", choice_key(table[i].first).c_str(),
                            table[i].second);
                fprintf(f, "}}\n");
                fclose(f);
            }
        }
        return GS_OK;
    });
}

int64_t gs_upsampler_num_params(void) { return up_num_params(); }

int gs_upsampler_init(gs_ctx *ctx, uint64_t seed)
{
    if (!ctx) return GS_ERR_INVALID_ARG;
    return guarded(ctx, [&] {
        HIP_CHECK(hipSetDevice(ctx->device));
        std::vector<float> p((size_t)up_num_params(), 0.0f);
        uint64_t st = seed * 0x2545F4914F6CDD1Dull + 1;
        float *dst = p.data();
        for (int l = 0; l < 4; ++l) {
            const int ci = kUpCin[l], co = kUpCout[l];
            const double bound = std::sqrt(6.0 / (9.0 * ci));
            for (size_t i = 0; i < (size_t)co * 9 * ci; ++i) {
                const double u = (double)(splitmix(st) >> 11) * (1.0 / 9007199254740992.0);
                dst[i] = l == 3 ? 0.0f : (float)((2.0 * u - 1.0) * bound);
            }
            dst += (size_t)co * 9 * ci + co;  // biases stay zero
        }
        up_set(ctx, p.data());
        return GS_OK;
    });
}

int gs_upsampler_set_weights(gs_ctx *ctx, const float *params, int64_t n)
{
    if (!ctx) return GS_ERR_INVALID_ARG;
    if (!params || n != up_num_params())
        return fail(ctx, GS_ERR_INVALID_ARG, "parameter vector must hold gs_upsampler_num_params() values");
    return guarded(ctx, [&] {
        HIP_CHECK(hipSetDevice(ctx->device));
        up_set(ctx, params);
        return GS_OK;
    });
}

int gs_upsampler_get_weights(gs_ctx *ctx, float *params, int64_t n)
{
    if (!ctx) return GS_ERR_INVALID_ARG;
    if (!params || n != up_num_params())
        return fail(ctx, GS_ERR_INVALID_ARG, "parameter vector must hold gs_upsampler_num_params() values");
    if (!ctx->up.ready) return fail(ctx, GS_ERR_NOT_TRAINED, "upsampler not initialised");
    return guarded(ctx, [&] {
        HIP_CHECK(hipSetDevice(ctx->device));
        HIP_CHECK(hipDeviceSynchronize());
        up_get(ctx, ctx->up.w, ctx->up.b, params);
        return GS_OK;
    });
}

// Checkpoint file: magic, version, parameter count, Adam step, then the
// parameter vector and Adam's first and second moments in the same layout.
static const char kUpMagic[8] = {'G', 'S', 'U', 'P', 'C', 'K', 'P', 'T'};
constexpr uint32_t kUpVersion = 1;

int gs_upsampler_save(gs_ctx *ctx, const char *path)
{
    if (!ctx) return GS_ERR_INVALID_ARG;
    if (!path) return fail(ctx, GS_ERR_INVALID_ARG, "null path");
    if (!ctx->up.ready) return fail(ctx, GS_ERR_NOT_TRAINED, "upsampler not initialised");
    return guarded(ctx, [&] {
        HIP_CHECK(hipSetDevice(ctx->device));
        HIP_CHECK(hipDeviceSynchronize());
        Upsampler &U = ctx->up;
        const size_t np = (size_t)up_num_params();
        std::vector<float> buf(3 * np);
        up_get(ctx, U.w, U.b, buf.data());
        up_get(ctx, U.mw, U.mb, buf.data() + np);
        up_get(ctx, U.vw, U.vb, buf.data() + 2 * np);
        FILE *f = fopen(path, "wb");
        if (!f) return fail(ctx, GS_ERR_INVALID_ARG, std::string("cannot open ") + path);
        const int64_t n64 = (int64_t)np;
        const int32_t step = U.step, pad = 0;
        bool ok = fwrite(kUpMagic, 1, 8, f) == 8 && fwrite(&kUpVersion, 4, 1, f) == 1 &&
                  fwrite(&pad, 4, 1, f) == 1 && fwrite(&n64, 8, 1, f) == 1 &&
                  fwrite(&step, 4, 1, f) == 1 && fwrite(&pad, 4, 1, f) == 1 &&
                  fwrite(buf.data(), 4, buf.size(), f) == buf.size();
        ok = (fclose(f) == 0) && ok;
        if (!ok) return fail(ctx, GS_ERR_INVALID_ARG, std::string("write failed: ") + path);
        return GS_OK;
    });
}

int gs_upsampler_load(gs_ctx *ctx, const char *path)
{
    if (!ctx) return GS_ERR_INVALID_ARG;
    if (!path) return fail(ctx, GS_ERR_INVALID_ARG, "null path");
    return guarded(ctx, [&] {
        FILE *f = fopen(path, "rb");
        if (!f) return fail(ctx, GS_ERR_INVALID_ARG, std::string("cannot open ") + path);
        char magic[8];
        uint32_t version = 0;
        int32_t pad = 0, step = 0;
        int64_t n64 = 0;
        const size_t np = (size_t)up_num_params();
        std::vector<float> buf(3 * np);
        bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, kUpMagic, 8) == 0 &&
                  fread(&version, 4, 1, f) == 1 && version == kUpVersion &&
                  fread(&pad, 4, 1, f) == 1 && fread(&n64, 8, 1, f) == 1 &&
                  n64 == (int64_t)np && fread(&step, 4, 1, f) == 1 && step >= 0 &&
                  fread(&pad, 4, 1, f) == 1 && fread(buf.data(), 4, buf.size(), f) == buf.size();
        fclose(f);
        if (!ok) return fail(ctx, GS_ERR_INVALID_ARG, std::string("not an upsampler checkpoint: ") + path);
        HIP_CHECK(hipSetDevice(ctx->device));
        up_set(ctx, buf.data());
        Upsampler &U = ctx->up;
        up_put(U.mw, U.mb, buf.data() + np);
        up_put(U.vw, U.vb, buf.data() + 2 * np);
        U.step = step;
        return GS_OK;
    });
}

int gs_upsampler_forward(gs_ctx *ctx, int32_t n, int32_t h, int32_t w, const float *rgb_lo,
                         const float *depth_lo, float *rgb_out, float *depth_out, void *stream)
{
    if (!ctx) return GS_ERR_INVALID_ARG;
    if (n < 1 || h < 1 || w < 1 || !rgb_lo || !depth_lo || !rgb_out || !depth_out)
        return fail(ctx, GS_ERR_INVALID_ARG, "bad upsampler forward arguments");
    if (!ctx->up.ready) return fail(ctx, GS_ERR_NOT_TRAINED, "upsampler not initialised");
    return guarded(ctx, [&] {
        HIP_CHECK(hipSetDevice(ctx->device));
        hipStream_t st = (hipStream_t)stream;
        Upsampler &U = ctx->up;
        if (!U.packed) up_pack(ctx, st);
        for (int c0 = 0; c0 < n; c0 += kUpChunk) {
            const int m = std::min(kUpChunk, n - c0);
            up_alloc(ctx, m, h, w, false);
            const int64_t lp = (int64_t)h * w, hp = lp * 16;
            launch_up_input(rgb_lo + c0 * lp * 3, depth_lo + c0 * lp, m * lp, U.x0f.p, nullptr, st);
            up_forward(ctx, m, h, w, st, rgb_out + c0 * hp * 3, depth_out + c0 * hp);
        }
        HIP_CHECK(hipGetLastError());
        return GS_OK;
    });
}

int gs_upsampler_forward_noalloc(gs_ctx *ctx, int32_t n, int32_t h, int32_t w,
                                 const float *rgb_lo, const float *depth_lo, float *rgb_out,
                                 float *depth_out, void *stream)
{
    if (!ctx) return GS_ERR_INVALID_ARG;
    if (n < 1 || h < 1 || w < 1 || !rgb_lo || !depth_lo || !rgb_out || !depth_out)
        return fail(ctx, GS_ERR_INVALID_ARG, "bad upsampler forward arguments");
    if (!ctx->up.ready) return fail(ctx, GS_ERR_NOT_TRAINED, "upsampler not initialised");
    if (!ctx->scratch) return fail(ctx, GS_ERR_HIP, "scratch array has no device address");
    // frames per pass: whole frames of activations in the scratch array
    // (three alignment gaps of at most 255 bytes between the four buffers)
    const uint64_t frame_bytes = (uint64_t)h * (uint64_t)w * kNoAllocBytesPerPixel;
    const uint64_t fit = (kNoAllocScratchBytes - 3 * 256) / frame_bytes;
    if (fit < 1)
        return fail(ctx, GS_ERR_INVALID_ARG,
                    "frame of " + std::to_string(w) + "x" + std::to_string(h) +
                        " needs " + std::to_string(frame_bytes) +
                        " bytes of activations, more than the " +
                        std::to_string(kNoAllocScratchBytes) + "-byte scratch array");
    return guarded(ctx, [&] {
        HIP_CHECK(hipSetDevice(ctx->device));
        hipStream_t st = (hipStream_t)stream;
        if (!ctx->up.packed) up_pack(ctx, st);
        const int per = (int)std::min<uint64_t>(fit, (uint64_t)kUpChunk);
        const int64_t lp = (int64_t)h * w, hp = lp * 16;
        auto align = [](size_t b) { return (b + 255) & ~size_t(255); };
        for (int c0 = 0; c0 < n; c0 += per) {
            const int m = std::min(per, n - c0);
            const size_t px = (size_t)m * lp;
            unsigned char *base = ctx->scratch;
            float *x0f = reinterpret_cast<float *>(base);
            uint16_t *act[3];
            size_t off = align(px * 16);
            for (int i = 0; i < 3; ++i) {
                act[i] = reinterpret_cast<uint16_t *>(base + off);
                off += align(px * 64);
            }
            launch_up_input(rgb_lo + c0 * lp * 3, depth_lo + c0 * lp, m * lp, x0f, nullptr, st);
            up_infer(ctx, m, h, w, st, x0f, act[0], act[1], act[2], rgb_out + c0 * hp * 3,
                     depth_out + c0 * hp);
        }
        HIP_CHECK(hipGetLastError());
        return GS_OK;
    });
}

int gs_upsampler_grads(gs_ctx *ctx, int32_t n, int32_t h, int32_t w, const float *rgb_lo,
                       const float *depth_lo, const float *rgb_hi, const float *depth_hi,
                       float *loss_out, float *grads_out, void *stream)
{
    if (!ctx) return GS_ERR_INVALID_ARG;
    if (n < 1 || h < 1 || w < 1 || !rgb_lo || !depth_lo || !rgb_hi || !depth_hi)
        return fail(ctx, GS_ERR_INVALID_ARG, "bad upsampler gradient arguments");
    if (!ctx->up.ready) return fail(ctx, GS_ERR_NOT_TRAINED, "upsampler not initialised");
    return guarded(ctx, [&] {
        HIP_CHECK(hipSetDevice(ctx->device));
        hipStream_t st = (hipStream_t)stream;
        const float loss = up_loss_and_grads(ctx, n, h, w, rgb_lo, depth_lo, rgb_hi, depth_hi, st);
        if (loss_out) *loss_out = loss;
        if (grads_out) up_get(ctx, ctx->up.gw, ctx->up.gb, grads_out);
        return GS_OK;
    });
}

int gs_upsampler_step(gs_ctx *ctx, int32_t n, int32_t h, int32_t w, const float *rgb_lo,
                      const float *depth_lo, const float *rgb_hi, const float *depth_hi,
                      float lr, float *loss_out, void *stream)
{
    if (!ctx) return GS_ERR_INVALID_ARG;
    if (n < 1 || h < 1 || w < 1 || !rgb_lo || !depth_lo || !rgb_hi || !depth_hi)
        return fail(ctx, GS_ERR_INVALID_ARG, "bad upsampler step arguments");
    if (!(lr >= 0.0f) || !std::isfinite(lr))
        return fail(ctx, GS_ERR_INVALID_ARG, "lr must be a finite value >= 0");
    if (!ctx->up.ready) return fail(ctx, GS_ERR_NOT_TRAINED, "upsampler not initialised");
    return guarded(ctx, [&] {
        HIP_CHECK(hipSetDevice(ctx->device));
        hipStream_t st = (hipStream_t)stream;
        const float loss = up_loss_and_grads(ctx, n, h, w, rgb_lo, depth_lo, rgb_hi, depth_hi, st);
        up_adam(ctx, lr, st);
        HIP_CHECK(hipGetLastError());
        HIP_CHECK(hipStreamSynchronize(st));
        if (loss_out) *loss_out = loss;
        return GS_OK;
    });
}

int gs_upsampler_apply_grads(gs_ctx *ctx, const float *grads, int64_t n, float lr)
{
    if (!ctx) return GS_ERR_INVALID_ARG;
    if (!grads || n != up_num_params())
        return fail(ctx, GS_ERR_INVALID_ARG, "gradient vector must hold gs_upsampler_num_params() values");
    if (!(lr >= 0.0f) || !std::isfinite(lr))
        return fail(ctx, GS_ERR_INVALID_ARG, "lr must be a finite value >= 0");
    if (!ctx->up.ready) return fail(ctx, GS_ERR_NOT_TRAINED, "upsampler not initialised");
    return guarded(ctx, [&] {
        HIP_CHECK(hipSetDevice(ctx->device));
        HIP_CHECK(hipDeviceSynchronize());
        up_put(ctx->up.gw, ctx->up.gb, grads);
        up_adam(ctx, lr, nullptr);
        HIP_CHECK(hipGetLastError());
        HIP_CHECK(hipDeviceSynchronize());
        return GS_OK;
    });
}

int gs_upsampler_get_state(gs_ctx *ctx, float *m, float *v, int64_t n, int32_t *step)
{
    if (!ctx) return GS_ERR_INVALID_ARG;
    if (n != up_num_params())
        return fail(ctx, GS_ERR_INVALID_ARG, "moment vectors must hold gs_upsampler_num_params() values");
    if (!ctx->up.ready) return fail(ctx, GS_ERR_NOT_TRAINED, "upsampler not initialised");
    return guarded(ctx, [&] {
        HIP_CHECK(hipSetDevice(ctx->device));
        HIP_CHECK(hipDeviceSynchronize());
        if (m) up_get(ctx, ctx->up.mw, ctx->up.mb, m);
        if (v) up_get(ctx, ctx->up.vw, ctx->up.vb, v);
        if (step) *step = ctx->up.step;
        return GS_OK;
    });
}

float gs_upsampler_lr(int32_t step, int32_t steps, float lr0, float lr_min)
{
    return up_cosine_lr(step, steps, lr0, lr_min);
}

int gs_upsampler_score(gs_ctx *ctx, int32_t n, int32_t h, int32_t w, const float *rgb_lo,
                       const float *depth_lo, float *score_out, void *stream)
{
    if (!ctx) return GS_ERR_INVALID_ARG;
    if (n < 1 || h < 1 || w < 1 || !rgb_lo || !depth_lo || !score_out)
        return fail(ctx, GS_ERR_INVALID_ARG, "bad score arguments");
    return guarded(ctx, [&] {
        HIP_CHECK(hipSetDevice(ctx->device));
        up_scores(ctx, n, h, w, rgb_lo, depth_lo, score_out, (hipStream_t)stream);
        HIP_CHECK(hipGetLastError());
        return GS_OK;
    });
}

int gs_upsampler_train(gs_ctx *ctx, const gs_train_opts *opts, int32_t n_pairs,
                       const int32_t *scene_ids, const float *poses, const float *intrinsics,
                       int32_t width, int32_t height, float *loss_curve, void *stream)
{
    TraceRange trace_range("gs_upsampler_train");
    if (!ctx) return GS_ERR_INVALID_ARG;
    if (!opts || !scene_ids || !poses || !intrinsics || n_pairs < 1 || width % 4 || height % 4 ||
        width < 4 || height < 4)
        return fail(ctx, GS_ERR_INVALID_ARG, "bad training arguments (sizes must be multiples of 4)");
    if (!ctx->up.ready) return fail(ctx, GS_ERR_NOT_TRAINED, "upsampler not initialised");
    const int batch = opts->batch > 0 ? opts->batch : 32;
    if (batch > n_pairs) return fail(ctx, GS_ERR_INVALID_ARG, "batch larger than the camera set");
    return guarded(ctx, [&] {
        HIP_CHECK(hipSetDevice(ctx->device));
        hipStream_t st = (hipStream_t)stream;
        Upsampler &U = ctx->up;
        const int h = height / 4, w = width / 4;
        U.lo_rgb.reserve((size_t)batch * h * w * 3);
        U.lo_depth.reserve((size_t)batch * h * w);
        U.hi_rgb.reserve((size_t)batch * width * height * 3);
        U.hi_depth.reserve((size_t)batch * width * height);
        U.intr_lo.reserve((size_t)batch * 4);
        gs_render_opts ro;
        gs_default_opts(&ro);
        const float lr0 = opts->lr > 0 ? opts->lr : 1e-3f;
        const float lr1 = opts->lr_min > 0 ? opts->lr_min : lr0 * 0.05f;
        for (int s = 0; s < opts->steps; ++s) {
            int c0 = (int)(((int64_t)s * batch) % n_pairs);
            if (c0 + batch > n_pairs) c0 = 0;
            launch_quarter_intr(intrinsics + (int64_t)c0 * 4, batch, U.intr_lo.p, st);
            int rc = render_impl(ctx, batch, scene_ids + c0, poses + (int64_t)c0 * 12, U.intr_lo.p,
                                 w, h, U.lo_rgb.p, U.lo_depth.p, nullptr, ro, st, nullptr);
            if (rc) return rc;
            rc = render_impl(ctx, batch, scene_ids + c0, poses + (int64_t)c0 * 12,
                             intrinsics + (int64_t)c0 * 4, width, height, U.hi_rgb.p, U.hi_depth.p,
                             nullptr, ro, st, nullptr);
            if (rc) return rc;
            const float loss = up_loss_and_grads(ctx, batch, h, w, U.lo_rgb.p, U.lo_depth.p,
                                                 U.hi_rgb.p, U.hi_depth.p, st);
            up_adam(ctx, up_cosine_lr(s, opts->steps, lr0, lr1), st);
            if (loss_curve) loss_curve[s] = loss;
        }
        HIP_CHECK(hipStreamSynchronize(st));
        return GS_OK;
    });
}

int gs_render_batch_upsampled(gs_ctx *ctx, int32_t n_cams, const int32_t *scene_ids,
                              const float *poses, const float *intrinsics, int32_t width,
                              int32_t height, float *rgb, float *depth, float *score_out,
                              float fallback_threshold, int32_t *n_fallback_out,
                              const gs_render_opts *opts, void *stream)
{
    TraceRange trace_range("gs_render_batch_upsampled");
    int rc = validate_render_args(ctx, n_cams, scene_ids, poses, intrinsics, width, height, rgb,
                                  depth);
    if (rc) return rc;
    if (width % 4 || height % 4)
        return fail(ctx, GS_ERR_INVALID_ARG, "width and height must be multiples of 4");
    if (!ctx->up.ready) return fail(ctx, GS_ERR_NOT_TRAINED, "upsampler not initialised");
    gs_render_opts o;
    if (opts) o = *opts; else gs_default_opts(&o);
    return guarded(ctx, [&] {
        HIP_CHECK(hipSetDevice(ctx->device));
        hipStream_t st = (hipStream_t)stream;
        Upsampler &U = ctx->up;
        const int h = height / 4, w = width / 4;
        const int64_t lp = (int64_t)h * w, hp = lp * 16;
        U.lo_rgb.reserve((size_t)n_cams * lp * 3);
        U.lo_depth.reserve((size_t)n_cams * lp);
        U.intr_lo.reserve((size_t)n_cams * 4);
        U.score.reserve((size_t)n_cams);
        U.flags.reserve((size_t)n_cams);
        U.n_flagged.reserve(1);
        launch_quarter_intr(intrinsics, n_cams, U.intr_lo.p, st);
        int r = render_impl(ctx, n_cams, scene_ids, poses, U.intr_lo.p, w, h, U.lo_rgb.p,
                            U.lo_depth.p, nullptr, o, st, nullptr, nullptr, Blend{}, true);
        if (r) return r;
        if (!U.packed) up_pack(ctx, st);
        for (int c0 = 0; c0 < n_cams; c0 += kUpChunk) {
            const int m = std::min(kUpChunk, n_cams - c0);
            up_alloc(ctx, m, h, w, false);
            launch_up_input(U.lo_rgb.p + c0 * lp * 3, U.lo_depth.p + c0 * lp, m * lp, U.x0f.p,
                            nullptr, st);
            launch_up_score(U.x0f.p, m, h, w, U.score.p + c0, st);
            up_forward(ctx, m, h, w, st, rgb + c0 * hp * 3, depth + c0 * hp);
        }
        if (score_out)
            HIP_CHECK(hipMemcpyAsync(score_out, U.score.p, (size_t)n_cams * 4,
                                     hipMemcpyDeviceToDevice, st));
        // fallback: the cameras whose score exceeds the threshold are flagged
        // on the device and rendered at full resolution straight into their
        // frames of the batch outputs (over the network's images); the
        // render of the others projects nothing and writes nothing
        launch_zero_u32(U.n_flagged.p, 1, st);
        launch_up_flag(U.score.p, n_cams, fallback_threshold, U.flags.p, U.n_flagged.p, st);
        r = render_impl(ctx, n_cams, scene_ids, poses, intrinsics, width, height, rgb, depth,
                        nullptr, o, st, nullptr, nullptr, Blend{}, true, U.flags.p);
        if (r) return r;
        if (n_fallback_out) {
            uint32_t nf = 0;
            HIP_CHECK(hipMemcpyAsync(&nf, U.n_flagged.p, 4, hipMemcpyDeviceToHost, st));
            HIP_CHECK(hipStreamSynchronize(st));
            *n_fallback_out = (int32_t)nf;
        }
        return GS_OK;
    });
}

int gs_frame_psnr(gs_ctx *ctx, int32_t n, int64_t npix, const float *a, const float *b, float *out,
                  void *stream)
{
    if (!ctx) return GS_ERR_INVALID_ARG;
    if (n < 1 || npix < 1 || !a || !b || !out) return fail(ctx, GS_ERR_INVALID_ARG, "bad PSNR arguments");
    return guarded(ctx, [&] {
        HIP_CHECK(hipSetDevice(ctx->device));
        launch_frame_psnr(a, b, n, npix, out, (hipStream_t)stream);
        HIP_CHECK(hipGetLastError());
        return GS_OK;
    });
}

}  // extern "C"
