// Ray ordering for coherent traversal.
//
// Rays are ordered by the Morton code of their origin inside the scene's
// root box (8 bits per axis, a 24-bit key), so that the 64 rays of a wave
// start close together and share the upper levels of the tree and their
// cache lines. The order is the stable result of a least-significant-digit
// radix sort with 8-bit digits (three passes). The traversal then takes rays
// in this order and writes every result at the ray's own index: results do
// not depend on the order, only the time does.
//
// One pass over m keys, tiles of 4096 keys per 256-thread block:
//   digit_hist_kernel   per-tile digit counts, stored digit-major
//   scan_*              exclusive prefix sum over the 256 x tiles counts
//   digit_scatter_kernel  stable scatter: a key's place is its digit's offset
//                       for the tile, plus the keys with the same digit before
//                       it in the tile (earlier rounds, earlier waves, lower
//                       lanes, counted with ballots)
#include "internal.h"

namespace sc {
namespace {

constexpr uint32_t kSortThreads = 256;
constexpr uint32_t kSortItems = 16;
constexpr uint32_t kSortTile = kSortThreads * kSortItems;  // keys per tile
constexpr uint32_t kDigits = 256;
constexpr uint32_t kScanTile = kSortThreads * kSortItems;  // counts per scan block
constexpr uint32_t kSortWaves = kSortThreads / 64;

// bits 0..7 of x moved to bits 0, 3, 6, ..., 21
__device__ inline uint32_t spread3(uint32_t x) {
    x &= 0xFFu;
    x = (x | (x << 16)) & 0x030000FFu;
    x = (x | (x << 8)) & 0x0300F00Fu;
    x = (x | (x << 4)) & 0x030C30C3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}

__device__ inline uint32_t cell8(float p, float lo, float scale) {
    const float u = (p - lo) * scale;
    if (!(u > 0.0f)) return 0u;  // below the box, or NaN
    if (u >= 255.0f) return 255u;
    return (uint32_t)u;
}

__global__ __launch_bounds__(256) void ray_key_kernel(const float* __restrict__ rays, uint32_t n, float lox,
                                                      float loy, float loz, float sx, float sy, float sz,
                                                      uint32_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float4 o = reinterpret_cast<const float4*>(rays)[2 * (size_t)i];
    keys[i] = (spread3(cell8(o.x, lox, sx)) << 2) | (spread3(cell8(o.y, loy, sy)) << 1) |
              spread3(cell8(o.z, loz, sz));
    vals[i] = i;
}

// batched launches: key = item index (bits 24..31) | Morton code of the origin in the item's bounds
__global__ __launch_bounds__(256) void batch_ray_key_kernel(const BatchItem* __restrict__ items, uint32_t n_items,
                                                            uint32_t n, uint32_t* __restrict__ keys,
                                                            uint32_t* __restrict__ vals) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t lo = 0, hi = n_items;  // the last item whose first ray is <= i
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (items[mid].ray_begin <= i) lo = mid;
        else hi = mid;
    }
    const BatchItem& it = items[lo];
    const float4 o = reinterpret_cast<const float4*>(it.rays)[2 * (size_t)(i - it.ray_begin)];
    keys[i] = (lo << 24) | (spread3(cell8(o.x, it.key_lo[0], it.key_scale[0])) << 2) |
              (spread3(cell8(o.y, it.key_lo[1], it.key_scale[1])) << 1) |
              spread3(cell8(o.z, it.key_lo[2], it.key_scale[2]));
    vals[i] = i;
}

__global__ __launch_bounds__(kSortThreads) void digit_hist_kernel(const uint32_t* __restrict__ keys, uint32_t n,
                                                                  uint32_t shift, uint32_t ntiles,
                                                                  uint32_t* __restrict__ counts) {
    __shared__ uint32_t h[kDigits];
    const uint32_t tid = threadIdx.x;
    h[tid] = 0u;
    __syncthreads();
    const size_t base = (size_t)blockIdx.x * kSortTile;
    for (uint32_t k = 0; k < kSortItems; ++k) {
        const size_t i = base + (size_t)k * kSortThreads + tid;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & (kDigits - 1)], 1u);
    }
    __syncthreads();
    counts[(size_t)tid * ntiles + blockIdx.x] = h[tid];
}

// Exclusive scan of one block's values held one per thread; returns the
// block total through *total.
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t* wave_tot, uint32_t* total) {
    const uint32_t tid = threadIdx.x, lane = tid & 63u, w = tid >> 6;
    uint32_t x = v;
#pragma unroll
    for (uint32_t d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) wave_tot[w] = x;
    __syncthreads();
    uint32_t before = 0, all = 0;
    for (uint32_t j = 0; j < kSortWaves; ++j) {
        if (j < w) before += wave_tot[j];
        all += wave_tot[j];
    }
    __syncthreads();
    *total = all;
    return before + x - v;
}

// Exclusive scan of each kScanTile-long block of `a` in place; block totals to `sums`.
__global__ __launch_bounds__(kSortThreads) void scan_blocks_kernel(uint32_t* __restrict__ a, size_t m,
                                                                   uint32_t* __restrict__ sums) {
    __shared__ uint32_t wave_tot[kSortWaves];
    const uint32_t tid = threadIdx.x;
    const size_t base = (size_t)blockIdx.x * kScanTile + (size_t)tid * kSortItems;
    uint32_t v[kSortItems];
    uint32_t s = 0;
    for (uint32_t k = 0; k < kSortItems; ++k) {
        v[k] = (base + k < m) ? a[base + k] : 0u;
        s += v[k];
    }
    uint32_t total;
    uint32_t run = block_exclusive_scan(s, wave_tot, &total);
    for (uint32_t k = 0; k < kSortItems; ++k) {
        if (base + k < m) a[base + k] = run;
        run += v[k];
    }
    if (tid == 0) sums[blockIdx.x] = total;
}

// Exclusive scan of the block totals by one block, in order.
__global__ __launch_bounds__(kSortThreads) void scan_sums_kernel(uint32_t* __restrict__ sums, uint32_t nb) {
    __shared__ uint32_t wave_tot[kSortWaves];
    uint32_t carry = 0;
    for (uint32_t b0 = 0; b0 < nb; b0 += kSortThreads) {
        const uint32_t i = b0 + threadIdx.x;
        const uint32_t v = i < nb ? sums[i] : 0u;
        uint32_t total;
        const uint32_t ex = block_exclusive_scan(v, wave_tot, &total);
        if (i < nb) sums[i] = carry + ex;
        carry += total;
    }
}

__global__ __launch_bounds__(kSortThreads) void scan_add_kernel(uint32_t* __restrict__ a, size_t m,
                                                                const uint32_t* __restrict__ sums) {
    const size_t base = (size_t)blockIdx.x * kScanTile + (size_t)threadIdx.x * kSortItems;
    const uint32_t add = sums[blockIdx.x];
    for (uint32_t k = 0; k < kSortItems; ++k)
        if (base + k < m) a[base + k] += add;
}

__global__ __launch_bounds__(kSortThreads) void digit_scatter_kernel(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin, uint32_t n, uint32_t shift,
    uint32_t ntiles, const uint32_t* __restrict__ offsets, uint32_t* __restrict__ kout, uint32_t* __restrict__ vout) {
    __shared__ uint32_t running[kDigits];             // next place of each digit in this tile
    __shared__ uint32_t wcount[kSortWaves][kDigits];  // this round's count per wave and digit
    const uint32_t tid = threadIdx.x, lane = tid & 63u, w = tid >> 6;
    running[tid] = offsets[(size_t)tid * ntiles + blockIdx.x];
    for (uint32_t j = 0; j < kSortWaves; ++j) wcount[j][tid] = 0u;
    __syncthreads();
    const uint64_t below = (1ull << lane) - 1ull;
    const size_t base = (size_t)blockIdx.x * kSortTile;
    for (uint32_t k = 0; k < kSortItems; ++k) {
        const size_t i = base + (size_t)k * kSortThreads + tid;
        const bool valid = i < n;
        const uint32_t key = valid ? kin[i] : 0u;
        const uint32_t val = valid ? vin[i] : 0u;
        const uint32_t d = (key >> shift) & (kDigits - 1);
        uint64_t match = __ballot(valid);
#pragma unroll
        for (uint32_t b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t m = __ballot(bit);
            match &= bit ? m : ~m;
        }
        const uint32_t rank = (uint32_t)__popcll(match & below);
        if (valid && rank == 0) wcount[w][d] = (uint32_t)__popcll(match);
        __syncthreads();
        if (valid) {
            uint32_t off = running[d] + rank;
            for (uint32_t j = 0; j < w; ++j) off += wcount[j][d];
            kout[off] = key;
            vout[off] = val;
        }
        __syncthreads();
        uint32_t add = 0;
        for (uint32_t j = 0; j < kSortWaves; ++j) {
            add += wcount[j][tid];
            wcount[j][tid] = 0u;
        }
        running[tid] += add;
        __syncthreads();
    }
}

}  // namespace

size_t ray_order_workspace_bytes(uint32_t n) {
    const size_t ntiles = ((size_t)n + kSortTile - 1) / kSortTile;
    const size_t m = ntiles * kDigits;
    const size_t nb = (m + kScanTile - 1) / kScanTile;
    return 16 * (size_t)n + 4 * m + 4 * nb;
}

namespace {

// LSD radix sort of the n (key, value) pairs in the first two workspace arrays, 8 bits per pass
// from bit 0; returns the sorted values (in the second or the fourth array)
uint32_t* sort_pairs(void* workspace, uint32_t n, uint32_t passes, hipStream_t s) {
    const size_t ntiles = ((size_t)n + kSortTile - 1) / kSortTile;
    const size_t m = ntiles * kDigits;
    const size_t nb = (m + kScanTile - 1) / kScanTile;
    auto* k0 = static_cast<uint32_t*>(workspace);
    uint32_t* v0 = k0 + n;
    uint32_t* k1 = v0 + n;
    uint32_t* v1 = k1 + n;
    uint32_t* counts = v1 + n;
    uint32_t* sums = counts + m;
    uint32_t *kin = k0, *vin = v0, *kout = k1, *vout = v1;
    for (uint32_t p = 0; p < passes; ++p) {
        const uint32_t shift = 8 * p;
        hipLaunchKernelGGL(digit_hist_kernel, dim3((uint32_t)ntiles), dim3(kSortThreads), 0, s, kin, n, shift,
                           (uint32_t)ntiles, counts);
        hipLaunchKernelGGL(scan_blocks_kernel, dim3((uint32_t)nb), dim3(kSortThreads), 0, s, counts, m, sums);
        hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(kSortThreads), 0, s, sums, (uint32_t)nb);
        hipLaunchKernelGGL(scan_add_kernel, dim3((uint32_t)nb), dim3(kSortThreads), 0, s, counts, m, sums);
        hipLaunchKernelGGL(digit_scatter_kernel, dim3((uint32_t)ntiles), dim3(kSortThreads), 0, s, kin, vin, n,
                           shift, (uint32_t)ntiles, counts, kout, vout);
        uint32_t* t = kin; kin = kout; kout = t;
        t = vin; vin = vout; vout = t;
    }
    return vin;
}

}  // namespace

uint32_t* sort_pairs_u32(void* workspace, uint32_t n, uint32_t passes, hipStream_t s) {
    return sort_pairs(workspace, n, passes, s);
}

size_t scan_u32_sums(size_t m) { return (m + kScanTile - 1) / kScanTile; }

hipError_t exclusive_scan_u32(uint32_t* a, size_t m, uint32_t* sums, hipStream_t s) {
    if (m == 0) return hipSuccess;
    const size_t nb = scan_u32_sums(m);
    if (nb > 0xFFFFFFFFull) return hipErrorInvalidValue;
    hipLaunchKernelGGL(scan_blocks_kernel, dim3((uint32_t)nb), dim3(kSortThreads), 0, s, a, m, sums);
    hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(kSortThreads), 0, s, sums, (uint32_t)nb);
    hipLaunchKernelGGL(scan_add_kernel, dim3((uint32_t)nb), dim3(kSortThreads), 0, s, a, m, sums);
    return hipGetLastError();
}

namespace {

bool sort_fits(uint32_t n) {
    const size_t ntiles = ((size_t)n + kSortTile - 1) / kSortTile;
    const size_t nb = (ntiles * kDigits + kScanTile - 1) / kScanTile;
    return nb <= 0xFFFFFFFFull && ntiles <= 0xFFFFFFFFull;
}

}  // namespace

hipError_t launch_ray_order(const float* rays, uint32_t n, const float lo[3], const float hi[3], void* workspace,
                            uint32_t** order, hipStream_t s) {
    if (n == 0) return hipSuccess;
    if (!sort_fits(n)) return hipErrorInvalidValue;
    float sc[3];
    for (int j = 0; j < 3; ++j) {
        const float e = hi[j] - lo[j];
        const float q = 256.0f / e;
        sc[j] = (e > 0.0f && q < __builtin_inff()) ? q : 0.0f;
    }
    auto* k0 = static_cast<uint32_t*>(workspace);
    hipLaunchKernelGGL(ray_key_kernel, dim3((n + 255) / 256), dim3(256), 0, s, rays, n, lo[0], lo[1], lo[2],
                       sc[0], sc[1], sc[2], k0, k0 + n);
    *order = sort_pairs(workspace, n, 3, s);  // 24-bit keys
    return hipGetLastError();
}

hipError_t launch_batch_order(const BatchItem* items, uint32_t n_items, uint32_t n, void* workspace,
                              uint32_t** order, hipStream_t s) {
    if (n == 0) return hipSuccess;
    if (!sort_fits(n) || n_items == 0 || n_items > kBatchSortItems) return hipErrorInvalidValue;
    auto* k0 = static_cast<uint32_t*>(workspace);
    hipLaunchKernelGGL(batch_ray_key_kernel, dim3((n + 255) / 256), dim3(256), 0, s, items, n_items, n, k0, k0 + n);
    *order = sort_pairs(workspace, n, 4, s);  // item index above the 24-bit Morton code
    return hipGetLastError();
}

}  // namespace sc
