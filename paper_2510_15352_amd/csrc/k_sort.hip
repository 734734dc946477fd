// Device-wide exclusive scan and stable LSD radix sort (8-bit digits) with
// element counts read from device memory, so a captured graph needs no host
// read-back between stages.
//
// Both use a fixed number of blocks `nb`, each owning one contiguous range
// of ceil(n / nb) elements (reduce-then-scan): the output order is fully
// determined by the input, independent of scheduling.
#include "gs_device.h"
#include "kernels.h"

namespace gs {

constexpr int kBS = 256;          // block size of scan / sort kernels
constexpr int kWaves = kBS / 64;  // waves per block

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

__device__ __forceinline__ uint32_t block_reduce(uint32_t v, uint32_t *s_wave)
{
    uint32_t total;
    block_excl_scan<kWaves>(v, total, s_wave);
    return total;
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

// ------------------------------------------------------------------ scan --

struct LoadU32 {
    const uint32_t *p;
    __device__ uint32_t operator()(uint32_t i) const { return p[i]; }
};

struct LoadPopc {
    const uint64_t *p;
    __device__ uint32_t operator()(uint32_t i) const { return (uint32_t)__popcll(p[i]); }
};

// Tiles overlapped by the footprint box of the i-th depth-sorted record.
struct LoadTiles {
    const uint32_t *vals;
    const uint2 *rect;
    int tw, th;
    __device__ uint32_t operator()(uint32_t i) const
    {
        const uint2 r = rect[vals[i]];
        const uint32_t x0 = r.x & 0xffffu, x1 = r.x >> 16, y0 = r.y & 0xffffu, y1 = r.y >> 16;
        return (x1 / tw - x0 / tw + 1) * (y1 / th - y0 / th + 1);
    }
};

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
    const uint32_t t = block_reduce(s, s_wave);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// Exclusive scan of the nb (<= 1024) block sums by one 1024-thread block.
__global__ __launch_bounds__(1024) void k_scan_partials(uint32_t *__restrict__ partial, int nb,
                                                        uint32_t *__restrict__ total_out)
{
    __shared__ uint32_t s_wave[16];
    const uint32_t v = (int)threadIdx.x < nb ? partial[threadIdx.x] : 0u;
    uint32_t total;
    const uint32_t ex = block_excl_scan<16>(v, total, s_wave);
    if ((int)threadIdx.x < nb) partial[threadIdx.x] = ex;
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
    const uint32_t per_block = 8192;
    uint32_t nb = (n_max + per_block - 1) / per_block;
    return (int)(nb < 1 ? 1 : (nb > 1024 ? 1024 : nb));
}

template <class Load>
static void scan_with(Load ld, const uint32_t *n_dev, uint32_t n_max, uint32_t *out,
                      uint32_t *total_out, const ScanTemp &tmp, hipStream_t st)
{
    const int nb = scan_blocks(n_max);
    hipLaunchKernelGGL(k_scan_reduce<Load>, dim3(nb), dim3(kBS), 0, st, ld, n_dev, n_max, nb,
                       tmp.partial);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, st, tmp.partial, nb, total_out);
    hipLaunchKernelGGL(k_scan_down<Load>, dim3(nb), dim3(kBS), 0, st, ld, n_dev, n_max, nb,
                       tmp.partial, out);
}

void scan_u32(const uint32_t *in, const uint32_t *n_dev, uint32_t n_max, uint32_t *out,
              uint32_t *total_out, const ScanTemp &tmp, hipStream_t st)
{
    scan_with(LoadU32{in}, n_dev, n_max, out, total_out, tmp, st);
}

void scan_popcount(const uint64_t *words, uint32_t n_words, uint32_t *out, uint32_t *total_out,
                   const ScanTemp &tmp, hipStream_t st)
{
    scan_with(LoadPopc{words}, nullptr, n_words, out, total_out, tmp, st);
}

void scan_tile_counts(const uint32_t *vals, const uint2 *rect, int tw, int th,
                      const uint32_t *n_dev, uint32_t n_max, uint32_t *out, uint32_t *total_out,
                      const ScanTemp &tmp, hipStream_t st)
{
    scan_with(LoadTiles{vals, rect, tw, th}, n_dev, n_max, out, total_out, tmp, st);
}

// ------------------------------------------------------------ radix sort --

template <typename K>
__global__ __launch_bounds__(kBS) void k_radix_hist(const K *__restrict__ keys,
                                                    const uint32_t *n_dev, int shift, int nb,
                                                    uint32_t *__restrict__ hist)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    uint32_t start, end;
    block_range(*n_dev, nb, start, end);
    for (uint32_t i = start + threadIdx.x; i < end; i += kBS)
        atomicAdd(&h[(uint32_t)(keys[i] >> shift) & 255u], 1u);
    __syncthreads();
    hist[threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter of one digit pass. Each block walks its range in tiles of
// 256 keys; within a tile, the rank of a key among equal digits is the
// count in earlier waves plus the count of lower lanes in its own wave
// (peer mask from 8 ballots, one per digit bit).
template <typename K>
__global__ __launch_bounds__(kBS) void k_radix_scatter(
    const K *__restrict__ kin, const uint32_t *__restrict__ vin, K *__restrict__ kout,
    uint32_t *__restrict__ vout, const uint32_t *n_dev, int shift, int nb,
    const uint32_t *__restrict__ hist_scanned)
{
    __shared__ uint32_t s_cnt[kWaves][256];
    __shared__ uint32_t s_base[256];
    const uint32_t tid = threadIdx.x;
    const int wave = tid >> 6;
    s_base[tid] = hist_scanned[tid * nb + blockIdx.x];
    uint32_t start, end;
    block_range(*n_dev, nb, start, end);
    const uint64_t lt = lanemask_lt();
    for (uint32_t t0 = start; t0 < end; t0 += kBS) {
        const uint32_t i = t0 + tid;
        const bool valid = i < end;
        K key = 0;
        uint32_t val = 0;
        if (valid) {
            key = kin[i];
            val = vin[i];
        }
        const uint32_t d = (uint32_t)(key >> shift) & 255u;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) s_cnt[w][tid] = 0;
        __syncthreads();
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const bool on = (d >> bit) & 1u;
            const uint64_t m = __ballot(on);
            peers &= on ? m : ~m;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lt);
        if (valid && rank == 0) s_cnt[wave][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        {
            uint32_t run = s_base[tid];
#pragma unroll
            for (int w = 0; w < kWaves; ++w) {
                const uint32_t c = s_cnt[w][tid];
                s_cnt[w][tid] = run;
                run += c;
            }
            s_base[tid] = run;
        }
        __syncthreads();
        if (valid) {
            const uint32_t pos = s_cnt[wave][d] + rank;
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
    }
}

static int sort_blocks(uint32_t n_max)
{
    const uint32_t per_block = 16384;
    uint32_t nb = (n_max + per_block - 1) / per_block;
    return (int)(nb < 1 ? 1 : (nb > 1024 ? 1024 : nb));
}

template <typename K>
static int radix_sort(K *k0, uint32_t *v0, K *k1, uint32_t *v1, const uint32_t *n_dev,
                      uint32_t n_max, int bits, const SortTemp &tmp, hipStream_t st)
{
    const int nb = sort_blocks(n_max);
    int cur = 0;
    for (int shift = 0; shift < bits; shift += 8) {
        K *ki = cur ? k1 : k0;
        K *ko = cur ? k0 : k1;
        uint32_t *vi = cur ? v1 : v0;
        uint32_t *vo = cur ? v0 : v1;
        hipLaunchKernelGGL(k_radix_hist<K>, dim3(nb), dim3(kBS), 0, st, ki, n_dev, shift, nb,
                           tmp.hist);
        scan_u32(tmp.hist, nullptr, (uint32_t)(256 * nb), tmp.hist, nullptr, tmp.scan, st);
        hipLaunchKernelGGL(k_radix_scatter<K>, dim3(nb), dim3(kBS), 0, st, ki, vi, ko, vo, n_dev,
                           shift, nb, tmp.hist);
        cur ^= 1;
    }
    return cur;
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
