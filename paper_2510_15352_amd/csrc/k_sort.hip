// Device-wide scans and a stable LSD radix sort, with element counts read
// from device memory so that a captured graph needs no host read-back.
//
// All of them use a fixed number of blocks `nb`, each owning one contiguous
// range of ceil(n / nb) elements (reduce-then-scan), so the output order is
// determined by the input alone, never by scheduling.
//
// Two scans end in fused writers instead of an offsets array:
//   * compaction: exclusive scan of the popcounts of the visibility words,
//     then each wave writes the set bits of its 64 words, one word at a time,
//     to consecutive positions (coalesced), as (camera, depth) keys;
//   * instance emission: exclusive scan of the tile counts of the
//     depth-sorted records, then each wave expands its 64 records into
//     their tile instances with one lane per output position (load-balanced,
//     coalesced), finding each position's record by a binary search over the
//     wave's offsets.
#include "gs_device.h"
#include "kernels.h"

namespace gs {

constexpr int kBS = 256;          // block size of scan / sort kernels
constexpr int kWaves = kBS / 64;  // waves per block
constexpr uint32_t kMaxBlocks = 4096;  // blocks of a scan or sort pass

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v)
{
    const uint32_t lane = __lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t t = __shfl_up(v, d, 64);
        if (lane >= (uint32_t)d) v += t;
    }
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

__device__ __forceinline__ uint64_t shfl64(uint64_t v, int src)
{
    const uint32_t lo = __shfl((uint32_t)v, src, 64);
    const uint32_t hi = __shfl((uint32_t)(v >> 32), src, 64);
    return ((uint64_t)hi << 32) | lo;
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

// Tiles of the footprint box of the i-th depth-sorted record.
struct LoadTiles {
    const uint32_t *vals;
    const uint2 *rect;
    int tw, th;
    __device__ uint32_t operator()(uint32_t i) const
    {
        const TileBox b = tile_box(rect[vals[i]], tw, th);
        return (uint32_t)(b.bw * b.bh);
    }
};

// ------------------------------------------------------------------- scan --

template <class Load>
__global__ __launch_bounds__(kBS) void k_scan_reduce(Load ld, const uint32_t *n_dev,
                                                     uint32_t n_host, int nb,
                                                     uint32_t *__restrict__ partial)
{
    __shared__ uint32_t s_wave[kWaves];
    uint32_t start, end;
    block_range(count_of(n_dev, n_host), nb, start, end);
    uint32_t s = 0;
    for (uint32_t i = start + threadIdx.x; i < end; i += kBS) s += ld(i);
    uint32_t t;
    block_excl_scan<kWaves>(s, t, s_wave);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// Exclusive scan of the nb (<= 4096) block sums by one 1024-thread block,
// four consecutive sums per thread.
__global__ __launch_bounds__(1024) void k_scan_partials(uint32_t *__restrict__ partial, int nb,
                                                        uint32_t *__restrict__ total_out)
{
    __shared__ uint32_t s_wave[16];
    uint32_t v[4], sum = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int i = (int)threadIdx.x * 4 + q;
        v[q] = i < nb ? partial[i] : 0u;
        sum += v[q];
    }
    uint32_t total;
    uint32_t ex = block_excl_scan<16>(sum, total, s_wave);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int i = (int)threadIdx.x * 4 + q;
        if (i < nb) partial[i] = ex;
        ex += v[q];
    }
    if (threadIdx.x == 0 && total_out) *total_out = total;
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

static int scan_blocks(uint32_t n_max)
{
    const uint32_t per_block = 2048;
    uint32_t nb = (n_max + per_block - 1) / per_block;
    return (int)(nb < 1 ? 1 : (nb > kMaxBlocks ? kMaxBlocks : nb));
}

template <class Load>
static int scan_reduce(Load ld, const uint32_t *n_dev, uint32_t n_max, uint32_t *total_out,
                       const ScanTemp &tmp, hipStream_t st)
{
    const int nb = scan_blocks(n_max);
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

__global__ __launch_bounds__(kBS) void k_compact_down(
    const uint64_t *__restrict__ vis, uint32_t n_words, int nb,
    const uint32_t *__restrict__ partial, const uint32_t *__restrict__ cam_slot, int n_cams,
    const uint32_t *__restrict__ zbits, uint64_t *__restrict__ keys, uint32_t *__restrict__ vals)
{
    __shared__ uint32_t s_wave[kWaves];
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
                    if (wd[q] == 0ull) continue;
                    const uint32_t wi = w0 + (uint32_t)(w8 + q);
                    while ((wi << 6) >= next) {
                        ++cam;
                        next = cam + 1 < n_cams ? cam_slot[cam + 1] : 0xFFFFFFFFu;
                    }
                    const uint32_t off = (uint32_t)__builtin_amdgcn_readlane((int)ex, w8 + q);
                    if ((wd[q] >> lane) & 1ull) {
                        const uint32_t pos = base + off + (uint32_t)__popcll(wd[q] & lt);
                        keys[pos] = ((uint64_t)cam << 31) | (uint64_t)zb[q];
                        vals[pos] = (wi << 6) | lane;
                    }
                }
            }
        }
        base += tot;
    }
}

void compact_visible(const uint64_t *vis, uint32_t n_words, const uint32_t *cam_slot, int n_cams,
                     const uint32_t *zbits, uint64_t *keys, uint32_t *vals, uint32_t *n_vis_out,
                     const ScanTemp &tmp, hipStream_t st)
{
    if (n_words == 0) return;
    const int nb = scan_reduce(LoadPopc{vis}, nullptr, n_words, n_vis_out, tmp, st);
    hipLaunchKernelGGL(k_compact_down, dim3(nb), dim3(kBS), 0, st, vis, n_words, nb, tmp.partial,
                       cam_slot, n_cams, zbits, keys, vals);
}
// --------------------------------------------------------- fused emission --

__global__ __launch_bounds__(kBS) void k_emit_down(
    const uint64_t *__restrict__ dkeys, const uint32_t *__restrict__ dvals,
    const uint32_t *__restrict__ n_dev, int nb, const uint32_t *__restrict__ partial,
    const uint2 *__restrict__ rect, int tw, int th, int tiles_x, int tiles_per_cam, uint32_t cap,
    uint32_t *__restrict__ ikeys, uint32_t *__restrict__ ivals)
{
    __shared__ uint32_t s_wave[kWaves];
    uint32_t start, end;
    block_range(*n_dev, nb, start, end);
    uint32_t base = partial[blockIdx.x];
    const uint32_t lane = __lane_id();
    for (uint32_t t0 = start; t0 < end; t0 += kBS) {
        const uint32_t i = t0 + threadIdx.x;
        uint32_t slot = 0, kbase = 0, cnt = 0;
        TileBox tb{0, 0, 1, 1};
        if (i < end) {
            slot = dvals[i];
            tb = tile_box(rect[slot], tw, th);
            kbase = (uint32_t)(dkeys[i] >> 31) * (uint32_t)tiles_per_cam +
                    (uint32_t)tb.ty0 * (uint32_t)tiles_x + (uint32_t)tb.tx0;
            cnt = (uint32_t)(tb.bw * tb.bh);
        }
        uint32_t tot;
        const uint32_t ex = block_excl_scan<kWaves>(cnt, tot, s_wave);
        const uint32_t first = __shfl(ex, 0, 64);
        const uint32_t wave_total = __shfl(ex, 63, 64) + __shfl(cnt, 63, 64) - first;
        const uint32_t lex = ex - first;
        // all lanes stay active through the shuffles; only the stores are masked
        for (uint32_t k0 = 0; k0 < wave_total; k0 += 64) {
            const uint32_t k = k0 + lane;
            // record of output position k: largest lane r with lex[r] <= k
            int r = 0;
#pragma unroll
            for (int step = 32; step >= 1; step >>= 1)
                if (__shfl(lex, r + step, 64) <= k) r += step;
            const uint32_t j = k - __shfl(lex, r, 64);
            const uint32_t bw = (uint32_t)__shfl(tb.bw, r, 64);
            const uint32_t key0 = __shfl(kbase, r, 64);
            const uint32_t sl = __shfl(slot, r, 64);
            const uint32_t ty = j / bw, tx = j - ty * bw;
            const uint32_t o = base + first + k;
            if (k < wave_total && o < cap) {
                ikeys[o] = key0 + ty * (uint32_t)tiles_x + tx;
                ivals[o] = sl;
            }
        }
        base += tot;
    }
}

void emit_instances(const uint64_t *dkeys, const uint32_t *dvals, const uint32_t *n_vis,
                    uint32_t n_max, const uint2 *rect, int tw, int th, int tiles_x,
                    int tiles_per_cam, uint32_t cap, uint32_t *ikeys, uint32_t *ivals,
                    uint32_t *counts, RenderFlags *flags, const ScanTemp &tmp, hipStream_t st)
{
    const int nb = scan_reduce(LoadTiles{dvals, rect, tw, th}, n_vis, n_max, counts + 1, tmp, st);
    launch_finalize_counts(counts, cap, flags, st);
    hipLaunchKernelGGL(k_emit_down, dim3(nb), dim3(kBS), 0, st, dkeys, dvals, n_vis, nb,
                       tmp.partial, rect, tw, th, tiles_x, tiles_per_cam, cap, ikeys, ivals);
}

// ------------------------------------------------------------- radix sort --

template <typename K, int RB>
__global__ __launch_bounds__(kBS) void k_radix_hist(const K *__restrict__ keys,
                                                    const uint32_t *n_dev, int shift, int nb,
                                                    uint32_t *__restrict__ hist)
{
    constexpr int R = 1 << RB;
    __shared__ uint32_t h[R];
    for (int d = threadIdx.x; d < R; d += kBS) h[d] = 0;
    __syncthreads();
    uint32_t start, end;
    block_range(*n_dev, nb, start, end);
    for (uint32_t i = start + threadIdx.x; i < end; i += kBS)
        atomicAdd(&h[(uint32_t)(keys[i] >> shift) & (uint32_t)(R - 1)], 1u);
    __syncthreads();
    for (int d = threadIdx.x; d < R; d += kBS) hist[d * nb + blockIdx.x] = h[d];
}

// Stable scatter of one RB-bit digit pass. A block walks its range in tiles
// of 256 * KPT keys. Keys of a tile are ranked sub-tile by sub-tile (256 keys
// in index order): the rank among equal digits is the count in earlier
// sub-tiles and waves plus the count of lower lanes of the same wave (peer
// mask from RB ballots). The tile is then reordered by digit in LDS and
// written out in that order, so each digit's run goes to consecutive
// addresses.
template <typename K, int RB, int KPT>
__global__ __launch_bounds__(kBS) void k_radix_scatter(
    const K *__restrict__ kin, const uint32_t *__restrict__ vin, K *__restrict__ kout,
    uint32_t *__restrict__ vout, const uint32_t *n_dev, int shift, int nb,
    const uint32_t *__restrict__ hist_scanned)
{
    constexpr int R = 1 << RB;
    constexpr int DPT = R / kBS;  // digits owned by each thread
    constexpr int TILE = kBS * KPT;
    __shared__ K s_keys[TILE];
    __shared__ uint32_t s_vals[TILE];
    __shared__ uint32_t s_cnt[kWaves][R];
    __shared__ uint32_t s_run[R], s_toff[R], s_base[R];
    __shared__ uint32_t s_wave[kWaves];
    const uint32_t tid = threadIdx.x;
    const int wave = tid >> 6;
    const uint64_t lt = lanemask_lt();
    const uint32_t mask = (uint32_t)(R - 1);
#pragma unroll
    for (int q = 0; q < DPT; ++q) s_base[tid * DPT + q] = hist_scanned[(tid * DPT + q) * nb + blockIdx.x];
    uint32_t start, end;
    block_range(*n_dev, nb, start, end);
    for (uint32_t t0 = start; t0 < end; t0 += TILE) {
        K key[KPT];
        uint32_t val[KPT], dig[KPT], lrank[KPT];
#pragma unroll
        for (int k = 0; k < KPT; ++k) {
            const uint32_t i = t0 + k * kBS + tid;
            key[k] = 0;
            val[k] = 0;
            if (i < end) {
                key[k] = kin[i];
                val[k] = vin[i];
            }
            dig[k] = (uint32_t)(key[k] >> shift) & mask;
        }
#pragma unroll
        for (int q = 0; q < DPT; ++q) s_run[tid * DPT + q] = 0;
#pragma unroll
        for (int k = 0; k < KPT; ++k) {
            const bool valid = t0 + k * kBS + tid < end;
#pragma unroll
            for (int q = 0; q < DPT; ++q)
#pragma unroll
                for (int w = 0; w < kWaves; ++w) s_cnt[w][tid * DPT + q] = 0;
            __syncthreads();
            uint64_t peers = __ballot(valid);
#pragma unroll
            for (int bit = 0; bit < RB; ++bit) {
                const bool on = (dig[k] >> bit) & 1u;
                const uint64_t m = __ballot(on);
                peers &= on ? m : ~m;
            }
            const uint32_t rank = (uint32_t)__popcll(peers & lt);
            if (valid && rank == 0) s_cnt[wave][dig[k]] = (uint32_t)__popcll(peers);
            __syncthreads();
#pragma unroll
            for (int q = 0; q < DPT; ++q) {
                const int d = tid * DPT + q;
                uint32_t run = s_run[d];
#pragma unroll
                for (int w = 0; w < kWaves; ++w) {
                    const uint32_t c = s_cnt[w][d];
                    s_cnt[w][d] = run;
                    run += c;
                }
                s_run[d] = run;
            }
            __syncthreads();
            lrank[k] = valid ? s_cnt[wave][dig[k]] + rank : 0u;
            __syncthreads();
        }
        // tile digit offsets: exclusive scan of the tile's digit counts
        {
            uint32_t local[DPT], sum = 0;
#pragma unroll
            for (int q = 0; q < DPT; ++q) {
                local[q] = sum;
                sum += s_run[tid * DPT + q];
            }
            uint32_t tot;
            const uint32_t ex = block_excl_scan<kWaves>(sum, tot, s_wave);
#pragma unroll
            for (int q = 0; q < DPT; ++q) s_toff[tid * DPT + q] = ex + local[q];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < KPT; ++k)
            if (t0 + k * kBS + tid < end) {
                const uint32_t p = s_toff[dig[k]] + lrank[k];
                s_keys[p] = key[k];
                s_vals[p] = val[k];
            }
        __syncthreads();
        const uint32_t n_tile = min((uint32_t)TILE, end - t0);
        for (uint32_t p = tid; p < n_tile; p += kBS) {
            const K kk = s_keys[p];
            const uint32_t d = (uint32_t)(kk >> shift) & mask;
            const uint32_t g = s_base[d] + p - s_toff[d];
            kout[g] = kk;
            vout[g] = s_vals[p];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < DPT; ++q) s_base[tid * DPT + q] += s_run[tid * DPT + q];
        __syncthreads();
    }
}

static int sort_blocks(uint32_t n_max)
{
    const uint32_t per_block = 8192;
    uint32_t nb = (n_max + per_block - 1) / per_block;
    return (int)(nb < 1 ? 1 : (nb > kMaxBlocks ? kMaxBlocks : nb));
}

template <typename K, int RB>
static int radix_sort_rb(K *k0, uint32_t *v0, K *k1, uint32_t *v1, const uint32_t *n_dev,
                         uint32_t n_max, int bits, const SortTemp &tmp, hipStream_t st)
{
    constexpr int KPT = sizeof(K) == 8 ? 8 : 8;
    const int nb = sort_blocks(n_max);
    int cur = 0;
    for (int shift = 0; shift < bits; shift += RB) {
        K *ki = cur ? k1 : k0;
        K *ko = cur ? k0 : k1;
        uint32_t *vi = cur ? v1 : v0;
        uint32_t *vo = cur ? v0 : v1;
        hipLaunchKernelGGL((k_radix_hist<K, RB>), dim3(nb), dim3(kBS), 0, st, ki, n_dev, shift, nb,
                           tmp.hist);
        scan_u32(tmp.hist, nullptr, (uint32_t)((1 << RB) * nb), tmp.hist, nullptr, tmp.scan, st);
        hipLaunchKernelGGL((k_radix_scatter<K, RB, KPT>), dim3(nb), dim3(kBS), 0, st, ki, vi, ko,
                           vo, n_dev, shift, nb, tmp.hist);
        cur ^= 1;
    }
    return cur;
}

// 10-bit digits when they need fewer passes than 8-bit ones.
template <typename K>
static int radix_sort(K *k0, uint32_t *v0, K *k1, uint32_t *v1, const uint32_t *n_dev,
                      uint32_t n_max, int bits, const SortTemp &tmp, hipStream_t st)
{
    if ((bits + 9) / 10 < (bits + 7) / 8)
        return radix_sort_rb<K, 10>(k0, v0, k1, v1, n_dev, n_max, bits, tmp, st);
    return radix_sort_rb<K, 8>(k0, v0, k1, v1, n_dev, n_max, bits, tmp, st);
}

int radix_sort_u64(uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1, const uint32_t *n_dev,
                   uint32_t n_max, int bits, const SortTemp &tmp, hipStream_t st)
{
    return radix_sort<uint64_t>(k0, v0, k1, v1, n_dev, n_max, bits, tmp, st);
}

int radix_sort_u32(uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1, const uint32_t *n_dev,
                   uint32_t n_max, int bits, const SortTemp &tmp, hipStream_t st)
{
    return radix_sort<uint32_t>(k0, v0, k1, v1, n_dev, n_max, bits, tmp, st);
}

}  // namespace gs
