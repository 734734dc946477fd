// Device-wide scans and a stable LSD radix sort segmented by camera, with
// element counts read from device memory so that a captured graph needs no
// host read-back.
//
// The scans use a fixed number of blocks `nb`, each owning one contiguous
// range of ceil(n / nb) elements (reduce-then-scan), so the output order is
// determined by the input alone, never by scheduling.
//
// Two scans end in fused writers instead of an offsets array:
//   * compaction: exclusive scan of the popcounts of the visibility words,
//     then each wave writes the set bits of its 64 words, one word at a time,
//     to consecutive positions (coalesced), as depth keys, camera-major, and
//     records where each camera's segment starts;
//   * instance emission: exclusive scan of the tile counts of the
//     depth-sorted records, then each wave expands its 64 records into
//     their tile instances with one lane per output position (load-balanced,
//     coalesced), finding each position's record by a binary search over the
//     wave's offsets, and writes each camera's instance segment start where
//     it meets the camera's first record.
#include <stdexcept>

#include "gs_device.h"
#include "kernels.h"

namespace gs {

constexpr int kBS = 256;          // block size of scan / sort kernels
constexpr int kWaves = kBS / 64;  // waves per block
constexpr uint32_t kMaxBlocks = 4096;  // blocks of a scan or sort pass

// v plus the value of a lane chosen by a DPP pattern (0 where the pattern
// has no source lane or the row is masked off).
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ uint32_t dpp_add_u32(uint32_t v)
{
    return v + (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROW_MASK, 0xF, true);
}

// Inclusive scan over the wave with DPP moves (no LDS round trips): shifts
// by 1, 2, 4 and 8 lanes inside each row of 16, then row 0's total into
// row 1 and row 2's into row 3, then rows 0-1's total into rows 2 and 3.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v)
{
    v = dpp_add_u32<0x111>(v);       // row_shr 1
    v = dpp_add_u32<0x112>(v);       // row_shr 2
    v = dpp_add_u32<0x114>(v);       // row_shr 4
    v = dpp_add_u32<0x118>(v);       // row_shr 8
    v = dpp_add_u32<0x142, 0xA>(v);  // row_bcast 15 into rows 1 and 3
    v = dpp_add_u32<0x143, 0xC>(v);  // row_bcast 31 into rows 2 and 3
    return v;
}

// Inclusive max-scan over the wave (same DPP pattern as wave_incl_scan).
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ uint32_t dpp_max_u32(uint32_t v)
{
    return max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROW_MASK, 0xF, true));
}

__device__ __forceinline__ uint32_t wave_incl_max(uint32_t v)
{
    v = dpp_max_u32<0x111>(v);
    v = dpp_max_u32<0x112>(v);
    v = dpp_max_u32<0x114>(v);
    v = dpp_max_u32<0x118>(v);
    v = dpp_max_u32<0x142, 0xA>(v);
    v = dpp_max_u32<0x143, 0xC>(v);
    return v;
}

// Exclusive scan across the block (NW waves); `total` gets the block sum.
template <int NW>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t &total, uint32_t *s_wave)
{
    const uint32_t inc = wave_incl_scan(v);
    const int wave = threadIdx.x >> 6;
    if (__lane_id() == 63) s_wave[wave] = inc;
    __syncthreads();
    uint32_t wbase = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        const uint32_t t = s_wave[w];
        wbase += (w < wave) ? t : 0u;
        tot += t;
    }
    __syncthreads();
    total = tot;
    return wbase + inc - v;
}

__device__ __forceinline__ void block_range(uint32_t n, int nb, uint32_t &start, uint32_t &end)
{
    const uint32_t per = (n + (uint32_t)nb - 1) / (uint32_t)nb;
    start = min(n, per * blockIdx.x);
    end = min(n, start + per);
}

__device__ __forceinline__ uint32_t count_of(const uint32_t *n_dev, uint32_t n_host)
{
    return n_dev ? *n_dev : n_host;
}

// ----------------------------------------------------------------- loaders --

struct LoadU32 {
    const uint32_t *p;
    __device__ uint32_t operator()(uint32_t i) const { return p[i]; }
};

struct LoadPopc {
    const uint64_t *p;
    __device__ uint32_t operator()(uint32_t i) const { return (uint32_t)__popcll(p[i]); }
};

// Tiles of the footprint box of the i-th depth-sorted record (boxes stored
// in sorted order by the depth sort's last pass).
struct LoadTiles {
    const uint2 *rect;
    int lw, lh;  // log2 of the tile width and height
    __device__ uint32_t operator()(uint32_t i) const
    {
        const TileBox b = tile_box(rect[i], lw, lh);
        return (uint32_t)(b.bw * b.bh);
    }
};

// ------------------------------------------------------------------- scan --

template <class Load>
__global__ __launch_bounds__(kBS) void k_scan_reduce(Load ld, const uint32_t *n_dev,
                                                     uint32_t n_host, int nb,
                                                     uint32_t *__restrict__ partial)
{
    __shared__ unsigned long long s_sum[kWaves];
    uint32_t start, end;
    block_range(count_of(n_dev, n_host), nb, start, end);
    // 64-bit sums: a block's total saturates at 2^32 - 1 instead of wrapping
    // (the emission then sees a count past any capacity and flags it)
    unsigned long long s = 0;
    // eight loads in flight per thread (indices past the end read the last
    // element, which is then not counted, so no load sits under a branch)
    for (uint32_t i0 = start + threadIdx.x; i0 < end; i0 += 8u * kBS) {
        uint32_t v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = ld(min(i0 + (uint32_t)u * kBS, end - 1u));
#pragma unroll
        for (int u = 0; u < 8; ++u) s += i0 + (uint32_t)u * kBS < end ? v[u] : 0u;
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) s += __shfl_down(s, d, 64);
    if (__lane_id() == 0) s_sum[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) t += s_sum[w];
        partial[blockIdx.x] = t > 0xffffffffull ? 0xffffffffu : (uint32_t)t;
    }
}

// Exclusive scan of the nb (<= 4096) block sums by one 1024-thread block,
// four consecutive sums per thread.
__global__ __launch_bounds__(1024) void k_scan_partials(uint32_t *__restrict__ partial, int nb,
                                                        uint32_t *__restrict__ total_out)
{
    // in 64 bits, saturated at 2^32 - 1 when stored (never wraps to a small count)
    __shared__ unsigned long long s_wave[16];
    uint32_t v[4];
    unsigned long long sum = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int i = (int)threadIdx.x * 4 + q;
        v[q] = i < nb ? partial[i] : 0u;
        sum += v[q];
    }
    const uint32_t lane = __lane_id();
    unsigned long long inc = sum;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const unsigned long long t = __shfl_up(inc, d, 64);
        if (lane >= (uint32_t)d) inc += t;
    }
    const int wave = (int)threadIdx.x >> 6;
    if (lane == 63) s_wave[wave] = inc;
    __syncthreads();
    unsigned long long ex = 0, total = 0;
#pragma unroll
    for (int w = 0; w < 16; ++w) {
        const unsigned long long t = s_wave[w];
        ex += w < wave ? t : 0ull;
        total += t;
    }
    ex += inc - sum;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int i = (int)threadIdx.x * 4 + q;
        if (i < nb) partial[i] = ex > 0xffffffffull ? 0xffffffffu : (uint32_t)ex;
        ex += v[q];
    }
    if (threadIdx.x == 0 && total_out)
        *total_out = total > 0xffffffffull ? 0xffffffffu : (uint32_t)total;
}

template <class Load>
__global__ __launch_bounds__(kBS) void k_scan_down(Load ld, const uint32_t *n_dev,
                                                   uint32_t n_host, int nb,
                                                   const uint32_t *__restrict__ partial,
                                                   uint32_t *__restrict__ out)
{
    __shared__ uint32_t s_wave[kWaves];
    uint32_t start, end;
    block_range(count_of(n_dev, n_host), nb, start, end);
    uint32_t base = partial[blockIdx.x];
    for (uint32_t t0 = start; t0 < end; t0 += kBS) {
        const uint32_t i = t0 + threadIdx.x;
        const uint32_t v = i < end ? ld(i) : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan<kWaves>(v, tot, s_wave);
        if (i < end) out[i] = base + ex;
        base += tot;
    }
}

static int scan_blocks(uint32_t n_max, uint32_t per_block = 2048)
{
    uint32_t nb = (n_max + per_block - 1) / per_block;
    return (int)(nb < 1 ? 1 : (nb > kMaxBlocks ? kMaxBlocks : nb));
}

template <class Load>
static int scan_reduce(Load ld, const uint32_t *n_dev, uint32_t n_max, uint32_t *total_out,
                       const ScanTemp &tmp, hipStream_t st, uint32_t per_block = 2048)
{
    const int nb = scan_blocks(n_max, per_block);
    hipLaunchKernelGGL(k_scan_reduce<Load>, dim3(nb), dim3(kBS), 0, st, ld, n_dev, n_max, nb,
                       tmp.partial);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, st, tmp.partial, nb, total_out);
    return nb;
}

void scan_u32(const uint32_t *in, const uint32_t *n_dev, uint32_t n_max, uint32_t *out,
              uint32_t *total_out, const ScanTemp &tmp, hipStream_t st)
{
    const int nb = scan_reduce(LoadU32{in}, n_dev, n_max, total_out, tmp, st);
    hipLaunchKernelGGL(k_scan_down<LoadU32>, dim3(nb), dim3(kBS), 0, st, LoadU32{in}, n_dev,
                       n_max, nb, tmp.partial, out);
}

// ------------------------------------------------------- fused compaction --

constexpr int kCompactMaxCams = 4096;  // cameras of a chunk (segments of the sorts)

__global__ __launch_bounds__(kBS) void k_compact_down(
    const uint64_t *__restrict__ vis, uint32_t n_words, int nb,
    const uint32_t *__restrict__ cam_slot_g, int n_cams, const uint32_t *__restrict__ partial,
    const uint32_t *__restrict__ zbits, uint32_t *__restrict__ keys, uint32_t *__restrict__ vals,
    uint32_t *__restrict__ seg_start)
{
    __shared__ uint32_t s_wave[kWaves];
    // the cameras' first slots, staged once per block: the searches below
    // then wait on LDS rather than on a chain of dependent global loads
    __shared__ uint32_t cam_slot[kCompactMaxCams];
    for (int c = (int)threadIdx.x; c < n_cams; c += kBS) cam_slot[c] = cam_slot_g[c];
    __syncthreads();
    uint32_t start, end;
    block_range(n_words, nb, start, end);
    uint32_t base = partial[blockIdx.x];
    const uint32_t lane = __lane_id();
    const uint64_t lt = lanemask_lt();
    for (uint32_t t0 = start; t0 < end; t0 += kBS) {
        const uint32_t i = t0 + threadIdx.x;
        const uint64_t word = i < end ? vis[i] : 0ull;
        uint32_t tot;
        const uint32_t ex = block_excl_scan<kWaves>((uint32_t)__popcll(word), tot, s_wave);
        const uint32_t w0 = t0 + (threadIdx.x & ~63u);
        if (w0 < end) {
            // camera owning the wave's first word; slots grow with the word index
            int cam;
            {
                int lo = 0, hi = n_cams - 1;
                const uint32_t s0 = w0 << 6;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (cam_slot[mid] <= s0) lo = mid; else hi = mid - 1;
                }
                cam = lo;
            }
            uint32_t first = cam_slot[cam];
            uint32_t next = cam + 1 < n_cams ? cam_slot[cam + 1] : 0xFFFFFFFFu;
            const uint32_t wlo = (uint32_t)word, whi = (uint32_t)(word >> 32);
            // 8 words per round: their depth bits are loaded together
            for (int w8 = 0; w8 < 64; w8 += 8) {
                uint64_t wd[8];
                uint32_t zb[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    wd[q] = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)whi, w8 + q) << 32) |
                            (uint32_t)__builtin_amdgcn_readlane((int)wlo, w8 + q);
                    const uint32_t slot = ((w0 + (uint32_t)(w8 + q)) << 6) | lane;
                    zb[q] = ((wd[q] >> lane) & 1ull) ? zbits[slot] : 0u;
                }
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const uint32_t wi = w0 + (uint32_t)(w8 + q);
                    if (wi >= end) break;
                    while ((wi << 6) >= next) {
                        ++cam;
                        first = next;
                        next = cam + 1 < n_cams ? cam_slot[cam + 1] : 0xFFFFFFFFu;
                    }
                    const uint32_t off = (uint32_t)__builtin_amdgcn_readlane((int)ex, w8 + q);
                    // the camera's first word: its segment starts here
                    if ((wi << 6) == first && lane == 0) seg_start[cam] = base + off;
                    if (wd[q] == 0ull) continue;
                    if ((wd[q] >> lane) & 1ull) {
                        const uint32_t pos = base + off + (uint32_t)__popcll(wd[q] & lt);
                        keys[pos] = zb[q];
                        vals[pos] = (wi << 6) | lane;
                    }
                }
            }
        }
        base += tot;
    }
}

// seg_start[n] = total (the end of the last segment).
__global__ void k_copy_u32(const uint32_t *__restrict__ src, uint32_t *__restrict__ dst)
{
    *dst = *src;
}

void compact_visible(const uint64_t *vis, uint32_t n_words, const uint32_t *cam_slot, int n_cams,
                     const uint32_t *zbits, uint32_t *keys, uint32_t *vals, uint32_t *n_vis_out,
                     uint32_t *seg_start, const ScanTemp &tmp, hipStream_t st)
{
    if (n_words == 0) return;
    if (n_cams < 1 || n_cams > kCompactMaxCams)
        throw std::invalid_argument("compaction: 1..4096 cameras per chunk");
    // one step of kBS words per block where the block limit allows: each
    // word expands into up to 64 records, so small blocks keep enough of
    // them in flight
    const int nb = scan_reduce(LoadPopc{vis}, nullptr, n_words, n_vis_out, tmp, st, kBS);
    hipLaunchKernelGGL(k_compact_down, dim3(nb), dim3(kBS), 0, st, vis, n_words, nb, cam_slot,
                       n_cams, tmp.partial, zbits, keys, vals, seg_start);
    hipLaunchKernelGGL(k_copy_u32, dim3(1), dim3(1), 0, st, n_vis_out, seg_start + n_cams);
}

// --------------------------------------------------------- fused emission --

__global__ __launch_bounds__(kBS) void k_emit_down(
    const uint32_t *__restrict__ dvals, const uint32_t *__restrict__ n_dev, int nb,
    const uint32_t *__restrict__ partial, const uint2 *__restrict__ rect, int lw, int lh,
    int tiles_x, uint32_t cap, uint32_t *__restrict__ ikeys, uint32_t *__restrict__ ivals,
    const uint32_t *__restrict__ vis_start, int n_cams, const uint32_t *__restrict__ counts,
    uint32_t *__restrict__ inst_start)
{
    __shared__ uint32_t s_wave[kWaves];
    __shared__ uint32_t s_idx[kWaves * 64];
    __shared__ int s_cam;
    uint32_t start, end;
    block_range(*n_dev, nb, start, end);
    uint64_t base = partial[blockIdx.x];  // 64-bit: positions past 2^32 stay past cap
    const uint32_t lane = __lane_id();
    // first camera whose records start inside this block's range or later
    // (vis_start is non-decreasing; vis_start[n_cams] = number of records)
    if (threadIdx.x == 0) {
        int lo = 0, hi = n_cams;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (vis_start[mid] >= start) hi = mid; else lo = mid + 1;
        }
        s_cam = lo;
    }
    __syncthreads();
    int cam = s_cam;
    uint32_t cam_first = cam < n_cams ? vis_start[cam] : ~0u;  // reloaded only when passed
    const uint32_t kept = counts[2];
    // the next step's slot and box are loaded before this step's work
    uint32_t nslot = 0;
    uint2 nrect = make_uint2(0, 0);
    if (start + threadIdx.x < end) {
        nslot = dvals[start + threadIdx.x];
        nrect = rect[start + threadIdx.x];
    }
    for (uint32_t t0 = start; t0 < end; t0 += kBS) {
        const uint32_t i = t0 + threadIdx.x;
        uint32_t slot = 0, kbase = 0, cnt = 0;
        TileBox tb{0, 0, 1, 1};
        const uint32_t cslot = nslot;
        const uint2 crect = nrect;
        if (i + kBS < end) {
            nslot = dvals[i + kBS];
            nrect = rect[i + kBS];
        }
        if (i < end) {
            slot = cslot;
            tb = tile_box(crect, lw, lh);
            kbase = (uint32_t)tb.ty0 * (uint32_t)tiles_x + (uint32_t)tb.tx0;
            cnt = (uint32_t)(tb.bw * tb.bh);
        }
        uint32_t tot;
        const uint32_t ex = block_excl_scan<kWaves>(cnt, tot, s_wave);
        // instance segment of every camera whose first record is in this
        // step: the first instance of that record (cameras without records
        // share the offset of the next camera's first record)
        const uint32_t lim = min(t0 + (uint32_t)kBS, end);
        while (cam_first < lim) {
            if (i == cam_first) inst_start[cam] = (uint32_t)min(base + ex, (uint64_t)kept);
            ++cam;
            cam_first = cam < n_cams ? vis_start[cam] : ~0u;
        }
        // every lane is active here: lane 0 and lane 63 are read directly
        const uint32_t first = (uint32_t)__builtin_amdgcn_readlane((int)ex, 0);
        const uint32_t wave_total = (uint32_t)__builtin_amdgcn_readlane((int)ex, 63) +
                                    (uint32_t)__builtin_amdgcn_readlane((int)cnt, 63) - first;
        const uint32_t lex = ex - first;
        // all lanes stay active through the shuffles; only the stores are masked
        uint32_t *sidx = s_idx + (threadIdx.x >> 6) * 64;
        for (uint32_t k0 = 0; k0 < wave_total; k0 += 64) {
            const uint32_t k = k0 + lane;
            // record of output position k: the last lane with instances whose
            // first output position is at most k. The window's record starts
            // are marked at their positions, the lane covering k0 at 0, and an
            // inclusive max-scan over the window carries each start forward.
            const uint64_t le = __ballot(cnt > 0u && lex <= k0);
            const uint32_t cover = 63u - (uint32_t)__builtin_clzll(le);
            sidx[lane] = 0u;
            __builtin_amdgcn_wave_barrier();
            if (cnt > 0u && lex > k0 && lex - k0 < 64u) sidx[lex - k0] = lane;
            __builtin_amdgcn_wave_barrier();
            uint32_t rr = sidx[lane];
            if (lane == 0u) rr = cover;
            rr = wave_incl_max(rr);
            __builtin_amdgcn_wave_barrier();
            const int r = (int)rr;
            const uint32_t j = k - __shfl(lex, r, 64);
            const uint32_t bw = (uint32_t)__shfl(tb.bw, r, 64);
            const uint32_t key0 = __shfl(kbase, r, 64);
            const uint32_t sl = __shfl(slot, r, 64);
            const uint32_t ty = j / bw, tx = j - ty * bw;
            const uint64_t o = base + first + k;
            if (k < wave_total && o < cap) {
                ikeys[o] = key0 + ty * (uint32_t)tiles_x + tx;
                ivals[o] = sl;
            }
        }
        base += tot;
    }
}

// Instance segment starts, first all set to the number of kept instances
// (what cameras after the last record keep, and the closing boundary); the
// emission then writes those of cameras whose first record it meets.
__global__ void k_inst_starts(int n_cams, const uint32_t *__restrict__ counts,
                              uint32_t *__restrict__ inst_start)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c > n_cams) return;
    inst_start[c] = counts[2];
}

void emit_instances(const uint32_t *dvals, const uint32_t *n_vis, uint32_t n_max,
                    const uint32_t *vis_start, int n_cams, const uint2 *rect, int tw, int th,
                    int tiles_x, uint32_t cap, uint32_t *ikeys, uint32_t *ivals,
                    uint32_t *inst_start, uint32_t *counts, RenderFlags *flags,
                    const ScanTemp &tmp, hipStream_t st)
{
    // tile sizes are powers of two (the raster's tile shapes): shifts, not divisions
    const int lw = __builtin_ctz((unsigned)tw), lh = __builtin_ctz((unsigned)th);
    if (tw <= 0 || th <= 0 || (1 << lw) != tw || (1 << lh) != th)
        throw std::invalid_argument("tile sizes must be powers of two");
    const int nb = scan_reduce(LoadTiles{rect, lw, lh}, n_vis, n_max, counts + 1, tmp, st);
    launch_finalize_counts(counts, cap, flags, st);
    hipLaunchKernelGGL(k_inst_starts, dim3((n_cams + 1 + 255) / 256), dim3(256), 0, st, n_cams,
                       counts, inst_start);
    hipLaunchKernelGGL(k_emit_down, dim3(nb), dim3(kBS), 0, st, dvals, n_vis, nb, tmp.partial,
                       rect, lw, lh, tiles_x, cap, ikeys, ivals, vis_start, n_cams, counts,
                       inst_start);
}

// ------------------------------------------------------ segmented radix sort --
// Stable LSD sort of (key, value) pairs inside segments [seg[c], seg[c+1]).
// Each segment is cut into tiles of kSegTile keys; block b handles tile
// b - tp[c] of segment c (tp = exclusive scan of tiles per segment). The
// digit histograms are laid out [segment][digit][tile of segment], so one
// plain exclusive scan over them yields every (segment, digit, tile)'s output
// position, stable inside the segment.
constexpr int kSegKPT = 16;
constexpr int kSegTile = kBS * kSegKPT;

// tp[c] for c <= n_seg (n_seg <= 4096) and hist_len = tp[n_seg] * R.
__global__ __launch_bounds__(1024) void k_seg_tiles(const uint32_t *__restrict__ seg, int n_seg,
                                                    int R, uint32_t *__restrict__ tp,
                                                    uint32_t *__restrict__ hist_len)
{
    __shared__ uint32_t s_wave[16];
    uint32_t v[4], sum = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int c = (int)threadIdx.x * 4 + q;
        v[q] = c < n_seg ? (seg[c + 1] - seg[c] + kSegTile - 1) / kSegTile : 0u;
        sum += v[q];
    }
    uint32_t total;
    uint32_t ex = block_excl_scan<16>(sum, total, s_wave);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int c = (int)threadIdx.x * 4 + q;
        if (c < n_seg) tp[c] = ex;
        ex += v[q];
    }
    if (threadIdx.x == 0) {
        tp[n_seg] = total;
        *hist_len = total * (uint32_t)R;
    }
}

struct SegTile {
    int c;            // segment
    uint32_t t, nt;   // tile index inside the segment, tiles of the segment
    uint32_t start, end;
    uint32_t hbase;   // tp[c] * R
};

// Blocks are dealt to the 8 XCDs round-robin (block i -> XCD i mod 8). Of
// the `total` tiles, XCD x takes the contiguous run [x * per, (x + 1) * per),
// per = ceil(total / 8), so whole segments are written through one XCD's L2
// (their scattered output lines are completed there) while every XCD gets
// the same number of tiles. The grid is a multiple of 8 and >= total.
template <int R>
__device__ __forceinline__ bool seg_tile(const uint32_t *seg, const uint32_t *tp, int n_seg,
                                         SegTile &st)
{
    const uint32_t total = tp[n_seg];
    const uint32_t per = (total + 7u) >> 3;
    const uint32_t j = blockIdx.x >> 3;
    if (j >= per) return false;
    const uint32_t b = (blockIdx.x & 7u) * per + j;
    if (b >= total) return false;
    int lo = 0, hi = n_seg - 1;
    while (lo < hi) {  // last segment with tp[c] <= b (skips empty segments)
        const int mid = (lo + hi + 1) >> 1;
        if (tp[mid] <= b) lo = mid; else hi = mid - 1;
    }
    st.c = lo;
    st.t = b - tp[lo];
    st.nt = tp[lo + 1] - tp[lo];
    st.start = seg[lo] + st.t * kSegTile;
    st.end = min(seg[lo + 1], st.start + kSegTile);
    st.hbase = tp[lo] * R;
    return true;
}

// copies of each digit counter per wave in the histogram kernel
constexpr int kHistCopies = 4;

template <typename K, int RB>
__global__ __launch_bounds__(kBS) void k_seg_hist(const K *__restrict__ keys,
                                                  const uint32_t *__restrict__ seg,
                                                  const uint32_t *__restrict__ tp, int n_seg,
                                                  int shift, uint32_t *__restrict__ hist)
{
    constexpr int R = 1 << RB;
    // kHistCopies counters per digit and wave, lane l counting into copy
    // l mod kHistCopies (rows padded to an odd stride): lanes with the same
    // digit mostly hit different addresses and banks (one shared set of
    // counters serialised the atomics: 8-11 bank conflicts per access)
    constexpr int NC = kWaves * kHistCopies, STRIDE = R + 1;
    __shared__ uint32_t h[NC * STRIDE];
    SegTile st;
    if (!seg_tile<R>(seg, tp, n_seg, st)) return;
    // every key of the thread is loaded before the first atomic, so a tile
    // waits for one memory latency rather than one per key
    K key[kSegKPT];
#pragma unroll
    for (int k = 0; k < kSegKPT; ++k) {
        const uint32_t i = st.start + (uint32_t)(k * kBS) + threadIdx.x;
        key[k] = i < st.end ? keys[i] : K(0);
    }
    for (int d = threadIdx.x; d < NC * STRIDE; d += kBS) h[d] = 0;
    __syncthreads();
    uint32_t *hc = h + ((threadIdx.x >> 6) * kHistCopies + (__lane_id() % kHistCopies)) * STRIDE;
#pragma unroll
    for (int k = 0; k < kSegKPT; ++k)
        if (st.start + (uint32_t)(k * kBS) + threadIdx.x < st.end)
            atomicAdd(&hc[(uint32_t)(key[k] >> shift) & (uint32_t)(R - 1)], 1u);
    __syncthreads();
    for (int d = threadIdx.x; d < R; d += kBS) {
        uint32_t c = 0;
#pragma unroll
        for (int q = 0; q < NC; ++q) c += h[q * STRIDE + d];
        hist[st.hbase + d * st.nt + st.t] = c;
    }
}

// Wave-private ranking: wave w ranks keys [w*64*KPT, (w+1)*64*KPT) of the
// tile, 64 at a time, against its own digit counters in LDS (no barrier per
// step); one barrier then turns the per-wave counts into wave offsets and
// tile offsets per digit. The tile is reordered by digit in LDS and written
// out in that order.
template <typename K, int RB>
__global__ __launch_bounds__(kBS) void k_seg_scatter(
    const K *__restrict__ kin, const uint32_t *__restrict__ vin, K *__restrict__ kout,
    uint32_t *__restrict__ vout, const uint32_t *__restrict__ seg,
    const uint32_t *__restrict__ tp, int n_seg, int shift, const uint32_t *__restrict__ hist,
    uint32_t seg_key_stride, const uint2 *__restrict__ pay_src, uint2 *__restrict__ pay_dst,
    uint32_t pay_stride, uint2 *__restrict__ ranges)
{
    constexpr int R = 1 << RB;
    constexpr int DPT = R >= kBS ? R / kBS : 1;  // digits owned by each thread
    __shared__ K s_keys[kSegTile];
    __shared__ uint32_t s_vals[kSegTile];
    __shared__ uint32_t s_cnt[kWaves][R];
    __shared__ uint32_t s_toff[R], s_base[R];
    __shared__ uint32_t s_wave[kWaves];
    SegTile st;
    if (!seg_tile<R>(seg, tp, n_seg, st)) return;
    const uint32_t tid = threadIdx.x;
    const int wave = tid >> 6;
    const uint32_t lane = __lane_id();
    const uint64_t lt = lanemask_lt();
    const uint32_t mask = (uint32_t)(R - 1);
#pragma unroll
    for (int q = 0; q < DPT; ++q) {
        const int d = tid * DPT + q;
        if (d < R) {
            s_base[d] = hist[st.hbase + d * st.nt + st.t];
#pragma unroll
            for (int w = 0; w < kWaves; ++w) s_cnt[w][d] = 0;
        }
    }
    __syncthreads();
    K key[kSegKPT];
    uint32_t val[kSegKPT], dig[kSegKPT], lrank[kSegKPT];
    uint32_t *cnt = s_cnt[wave];
    // all of the thread's keys and values first: one memory latency per tile
#pragma unroll
    for (int k = 0; k < kSegKPT; ++k) {
        const uint32_t i = st.start + (uint32_t)(wave * 64 * kSegKPT + k * 64) + lane;
        key[k] = 0;
        val[k] = 0;
        if (i < st.end) {
            key[k] = kin[i];
            val[k] = vin[i];
        }
    }
#pragma unroll
    for (int k = 0; k < kSegKPT; ++k) {
        const uint32_t i = st.start + (uint32_t)(wave * 64 * kSegKPT + k * 64) + lane;
        const bool valid = i < st.end;
        dig[k] = (uint32_t)(key[k] >> shift) & mask;
        // lanes with the same digit: for every digit bit keep the lanes
        // whose bit equals this lane's, i.e. AND with ~(ballot ^ t), t = 0
        // or all ones as the bit is clear or set (one 3-input bit operation
        // per 32-bit half)
        const uint64_t vm = __ballot(valid);
        uint32_t plo = (uint32_t)vm, phi = (uint32_t)(vm >> 32);
#pragma unroll
        for (int bit = 0; bit < RB; ++bit) {
            const uint32_t t = (uint32_t)((int32_t)(dig[k] << (31 - bit)) >> 31);
            const uint64_t m = __ballot(t != 0u);
            plo &= ~((uint32_t)m ^ t);
            phi &= ~((uint32_t)(m >> 32) ^ t);
        }
        const uint64_t peers = ((uint64_t)phi << 32) | plo;
        const uint32_t rank = (uint32_t)__popcll(peers & lt);
        const uint32_t before = valid ? cnt[dig[k]] : 0u;
        lrank[k] = before + rank;
        __builtin_amdgcn_wave_barrier();
        if (valid && rank == 0) cnt[dig[k]] = before + (uint32_t)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // per digit: offsets of the waves, then exclusive scan of the tile totals
    {
        uint32_t tot_d[DPT], sum = 0;
#pragma unroll
        for (int q = 0; q < DPT; ++q) {
            const int d = tid * DPT + q;
            uint32_t run = 0;
            if (d < R) {
#pragma unroll
                for (int w = 0; w < kWaves; ++w) {
                    const uint32_t c = s_cnt[w][d];
                    s_cnt[w][d] = run;
                    run += c;
                }
            }
            tot_d[q] = run;
            sum += run;
        }
        uint32_t tot;
        uint32_t ex = block_excl_scan<kWaves>(sum, tot, s_wave);
#pragma unroll
        for (int q = 0; q < DPT; ++q) {
            if (tid * DPT + q < R) s_toff[tid * DPT + q] = ex;
            ex += tot_d[q];
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kSegKPT; ++k) {
        const uint32_t i = st.start + (uint32_t)(wave * 64 * kSegKPT + k * 64) + lane;
        if (i < st.end) {
            const uint32_t p = s_toff[dig[k]] + s_cnt[wave][dig[k]] + lrank[k];
            s_keys[p] = key[k];
            s_vals[p] = val[k];
        }
    }
    __syncthreads();
    const uint32_t n_tile = st.end - st.start;
    const K add = (K)((uint32_t)st.c * seg_key_stride);
    for (uint32_t p = tid; p < n_tile; p += kBS) {
        const K kk = s_keys[p];
        const uint32_t d = (uint32_t)(kk >> shift) & mask;
        const uint32_t g = s_base[d] + p - s_toff[d];
        const uint32_t v = s_vals[p];
        if (pay_dst)
            pay_dst[g] = pay_src[(size_t)v * pay_stride];  // keys not needed after this pass
        else
            kout[g] = kk + add;
        vout[g] = v;
        if (ranges) {
            // Last pass: inside the run of digit d the keys are sorted (the
            // earlier passes ordered the tile by the lower digits), and the
            // run lands at consecutive positions. The first and last element
            // of each key in the run bound that key's range; a key whose run
            // continues in another tile's run is completed there, so the
            // bounds are folded in with min / max.
            const uint32_t run0 = s_toff[d];
            const uint32_t run1 = d + 1u < (uint32_t)R ? s_toff[d + 1] : n_tile;
            if (p == run0 || s_keys[p - 1] != kk) atomicMin(&ranges[kk + add].x, g);
            if (p + 1u == run1 || s_keys[p + 1] != kk) atomicMax(&ranges[kk + add].y, g + 1u);
        }
    }
}

// Tile ranges before the tile sort folds its bounds in: start ~0, end 0 (an
// empty range for every tile no instance reaches).
__global__ void k_fill_ranges(uint2 *__restrict__ ranges, uint64_t n)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        ranges[i] = make_uint2(~0u, 0u);
}

void fill_ranges(uint2 *ranges, uint64_t n, hipStream_t st)
{
    if (n == 0) return;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_fill_ranges, dim3((unsigned)blocks), dim3(256), 0, st, ranges, n);
}

template <typename K, int RB>
static int seg_sort_rb(K *k0, uint32_t *v0, K *k1, uint32_t *v1, const uint32_t *seg, int n_seg,
                       uint32_t n_max, int bits, uint32_t stride, const uint2 *pay_src,
                       uint2 *pay_dst, uint32_t pay_stride, const SegSortTemp &tmp,
                       hipStream_t st, uint2 *ranges)
{
    constexpr int R = 1 << RB;
    const uint32_t max_tiles =
        ((uint32_t)(((uint64_t)n_max + kSegTile - 1) / kSegTile) + (uint32_t)n_seg + 7u) & ~7u;
    hipLaunchKernelGGL(k_seg_tiles, dim3(1), dim3(1024), 0, st, seg, n_seg, R, tmp.tp,
                       tmp.hist_len);
    int cur = 0;
    for (int shift = 0; shift < bits; shift += RB) {
        K *ki = cur ? k1 : k0;
        K *ko = cur ? k0 : k1;
        uint32_t *vi = cur ? v1 : v0;
        uint32_t *vo = cur ? v0 : v1;
        hipLaunchKernelGGL((k_seg_hist<K, RB>), dim3(max_tiles), dim3(kBS), 0, st, ki, seg, tmp.tp,
                           n_seg, shift, tmp.hist);
        scan_u32(tmp.hist, tmp.hist_len, max_tiles * (uint32_t)R, tmp.hist, nullptr, tmp.scan, st);
        const bool last = shift + RB >= bits;
        hipLaunchKernelGGL((k_seg_scatter<K, RB>), dim3(max_tiles), dim3(kBS), 0, st, ki, vi, ko,
                           vo, seg, tmp.tp, n_seg, shift, tmp.hist, last ? stride : 0u,
                           last ? pay_src : nullptr, last ? pay_dst : nullptr, pay_stride,
                           last ? ranges : nullptr);
        cur ^= 1;
    }
    return cur;
}

uint64_t seg_sort_hist_entries(uint32_t n_max, int n_seg)
{
    return (((uint64_t)n_max + kSegTile - 1) / kSegTile + (uint64_t)n_seg + 7u) * 256u;
}

int seg_sort_u32(uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1, const uint32_t *seg,
                 int n_seg, uint32_t n_max, int bits, uint32_t seg_key_stride,
                 const SegSortTemp &tmp, hipStream_t st, const uint2 *pay_src, uint2 *pay_dst,
                 uint32_t pay_stride, uint2 *ranges)
{
    if (ranges && pay_dst)
        throw std::invalid_argument("segmented sort: ranges are for key output, not a payload");
    if (bits <= 0) return 0;
    // as many 8-bit passes as needed, with the bits spread evenly over them
    // (narrower digits: fewer ballots per rank, longer runs per write)
    const int passes = (bits + 7) / 8;
    const int rb = (bits + passes - 1) / passes;
#define GS_SEG(RB_)                                                                               \
    return seg_sort_rb<uint32_t, RB_>(k0, v0, k1, v1, seg, n_seg, n_max, bits, seg_key_stride,   \
                                      pay_src, pay_dst, pay_stride, tmp, st, ranges);
    switch (rb) {
    case 1: case 2: case 3: case 4: GS_SEG(4)
    case 5: GS_SEG(5)
    case 6: GS_SEG(6)
    case 7: GS_SEG(7)
    default: GS_SEG(8)
    }
#undef GS_SEG
}

}  // namespace gs
