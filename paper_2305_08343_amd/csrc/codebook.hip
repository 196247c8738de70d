// Compression-LUT (codebook) selection on the device (Sect. 3.2.2).
//
// The paper ranks object masks by the importance SA(N) * O_m(N) / R^3 of its masked SAH
// (Eq. 2) and keeps the most important ones. Here, for the S child slots:
//  - importance per slot in float64: (SA * popcount) / R^3, SA = 2((dx*dy + dy*dz) + dz*dx) of
//    the slot's float32 box (the box the binary node holds for it);
//  - the slots are put in order of their mask's value (a mask read as an unsigned integer whose
//    last word is the most significant) by a stable radix sort, so the slots of one mask stay in
//    ascending slot order;
//  - equal masks add their importances in that order, one thread per distinct mask (the same
//    sequence of float64 additions as one pass over the slots);
//  - the distinct masks other than the full one are ordered by importance descending with ties
//    by value ascending (a stable sort of the value-ordered list), and the first K-1 are chosen.
// finish_codebook (codebook.cpp) then appends the full mask up to K entries and sorts the codebook
// by (set bits ascending, value ascending), which makes the lowest conservative index the tightest
// one (Sect. 3.2.3).
#include <hip/hip_runtime.h>

#include <cstring>

#include "internal.h"

namespace sc {
namespace {

constexpr uint32_t kThreads = 256;

uint32_t blocks(size_t n) { return (uint32_t)((n + kThreads - 1) / kThreads); }

template <int W>
__device__ __forceinline__ uint32_t mask_popcount(const uint64_t* m) {
    uint32_t c = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) c += (uint32_t)__popcll(m[w]);
    return c;
}

// importance of slot s; its box is child (s & 1) of binary node s >> 1: lo xyz, hi xyz at float 6 (s & 1)
template <int R>
__global__ __launch_bounds__(kThreads) void slot_importance_kernel(const unsigned char* __restrict__ nodes,
                                                                   uint32_t stride, const uint64_t* __restrict__ masks,
                                                                   uint32_t S, double* __restrict__ imp) {
    constexpr int W = (R * R * R + 63) / 64;
    const uint32_t s = blockIdx.x * kThreads + threadIdx.x;
    if (s >= S) return;
    const float* b = reinterpret_cast<const float*>(nodes + (size_t)(s >> 1) * stride) + 6 * (s & 1u);
    const double dx = (double)b[3] - (double)b[0];
    const double dy = (double)b[4] - (double)b[1];
    const double dz = (double)b[5] - (double)b[2];
    const double sa = 2.0 * ((dx * dy + dy * dz) + dz * dx);
    imp[s] = (sa * (double)mask_popcount<W>(masks + (size_t)s * W)) / (double)(R * R * R);
}

__global__ __launch_bounds__(kThreads) void iota_kernel(uint32_t* __restrict__ v, uint32_t n) {
    const uint32_t i = blockIdx.x * kThreads + threadIdx.x;
    if (i < n) v[i] = i;
}

// one 32-bit round of the value sort: half h of word w of the mask of slot order[i]
__global__ __launch_bounds__(kThreads) void mask_key_kernel(const uint64_t* __restrict__ masks, uint32_t W,
                                                            const uint32_t* __restrict__ order, uint32_t n,
                                                            uint32_t w, uint32_t h, uint32_t* __restrict__ keys) {
    const uint32_t i = blockIdx.x * kThreads + threadIdx.x;
    if (i < n) keys[i] = (uint32_t)(masks[(size_t)order[i] * W + w] >> (32u * h));
}

// head[i] = 1 where the value-sorted slots start a new mask; gid[i] the same flag, to be scanned;
// simp[i] the importance of slot order[i], so each mask's importances lie contiguous in slot order
__global__ __launch_bounds__(kThreads) void group_head_kernel(const uint64_t* __restrict__ masks, uint32_t W,
                                                              const uint32_t* __restrict__ order, uint32_t n,
                                                              const double* __restrict__ imp,
                                                              uint32_t* __restrict__ head, uint32_t* __restrict__ gid,
                                                              double* __restrict__ simp) {
    const uint32_t i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const uint32_t si = order[i];
    uint32_t h = (i == 0) ? 1u : 0u;
    if (i > 0) {
        const uint64_t* a = masks + (size_t)si * W;
        const uint64_t* b = masks + (size_t)order[i - 1] * W;
        for (uint32_t w = 0; w < W; ++w) h |= (a[w] != b[w]) ? 1u : 0u;
    }
    head[i] = h;
    gid[i] = h;
    simp[i] = imp[si];
}

// after the scan gid[i] is the index of the distinct mask at head i: its first place and first slot
__global__ __launch_bounds__(kThreads) void group_start_kernel(const uint32_t* __restrict__ order,
                                                               const uint32_t* __restrict__ head,
                                                               const uint32_t* __restrict__ gid, uint32_t n,
                                                               uint32_t* __restrict__ gstart,
                                                               uint32_t* __restrict__ first) {
    const uint32_t i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= n || !head[i]) return;
    gstart[gid[i]] = i;
    first[gid[i]] = order[i];
}

// one thread per distinct mask adds its slots' importances one after another in slot order, the
// order of a sequential pass over the slots (the loads run ahead of the dependent adds)
__global__ __launch_bounds__(kThreads) void group_sum_kernel(const uint32_t* __restrict__ head,
                                                             const uint32_t* __restrict__ gid, uint32_t n,
                                                             const uint32_t* __restrict__ gstart,
                                                             const double* __restrict__ simp,
                                                             double* __restrict__ gsum) {
    const uint32_t g = blockIdx.x * kThreads + threadIdx.x;
    const uint32_t groups = gid[n - 1] + head[n - 1];
    if (g >= groups) return;
    const uint32_t a = gstart[g];
    const uint32_t b = (g + 1 < groups) ? gstart[g + 1] : n;
    double t = simp[a];
    uint32_t j = a + 1;
    for (; j + 8 <= b; j += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = simp[j + u];
#pragma unroll
        for (int u = 0; u < 8; ++u) t += v[u];
    }
    for (; j < b; ++j) t += simp[j];
    gsum[g] = t;
}

// one 32-bit round of the importance sort: half h of a key that orders the sums descending
__global__ __launch_bounds__(kThreads) void importance_key_kernel(const double* __restrict__ gsum,
                                                                  const uint32_t* __restrict__ order, uint32_t n,
                                                                  uint32_t h, uint32_t* __restrict__ keys) {
    const uint32_t i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    uint64_t u = (uint64_t)__double_as_longlong(gsum[order[i]]);
    u = (u >> 63) ? ~u : (u | 0x8000000000000000ull);  // ascending in the value of the double
    keys[i] = (uint32_t)(~u >> (32u * h));              // descending
}

// the masks of the chosen distinct masks, most important first
__global__ __launch_bounds__(kThreads) void gather_chosen_kernel(const uint64_t* __restrict__ masks, uint32_t W,
                                                                 const uint32_t* __restrict__ order,
                                                                 const uint32_t* __restrict__ first, uint32_t take,
                                                                 uint64_t* __restrict__ out) {
    const uint32_t k = blockIdx.x * kThreads + threadIdx.x;
    if (k >= take) return;
    const uint64_t* m = masks + (size_t)first[order[k]] * W;
    for (uint32_t w = 0; w < W; ++w) out[(size_t)k * W + w] = m[w];
}

struct Layout {
    size_t sort, imp, simp, head, gid, sums, gstart, gsum, first, chosen, total;
};

Layout layout(uint32_t S, uint32_t W, uint32_t K) {
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    Layout L{};
    size_t o = 0;
    L.sort = o;   o += up(ray_order_workspace_bytes(S));
    L.imp = o;    o += up((size_t)S * 8);
    L.simp = o;   o += up((size_t)S * 8);
    L.head = o;   o += up((size_t)S * 4);
    L.gid = o;    o += up((size_t)S * 4);
    L.sums = o;   o += up(scan_u32_sums(S) * 4);
    L.gstart = o; o += up((size_t)S * 4);
    L.gsum = o;   o += up((size_t)S * 8);
    L.first = o;  o += up((size_t)S * 4);
    L.chosen = o; o += up((size_t)K * W * 8);
    L.total = o;
    return L;
}

}  // namespace

size_t codebook_workspace_bytes(uint32_t S, uint32_t R, uint32_t K) { return layout(S, words_for(R), K).total; }

hipError_t select_codebook_device(const unsigned char* nodes, uint32_t stride, const uint64_t* masks, uint32_t S,
                                  uint32_t R, uint32_t K, void* workspace, std::vector<uint64_t>& chosen,
                                  hipStream_t s) {
    chosen.clear();
    if (S == 0 || K == 0) return hipSuccess;
    if (R != 4 && R != 6) return hipErrorInvalidValue;
    const uint32_t W = words_for(R);
    const Layout L = layout(S, W, K);
    auto* base = static_cast<unsigned char*>(workspace);
    void* ws = base + L.sort;
    auto* keys = static_cast<uint32_t*>(ws);  // the sort's key array, then its value array
    uint32_t* vals = keys + S;
    auto* imp = reinterpret_cast<double*>(base + L.imp);
    auto* simp = reinterpret_cast<double*>(base + L.simp);
    auto* head = reinterpret_cast<uint32_t*>(base + L.head);
    auto* gid = reinterpret_cast<uint32_t*>(base + L.gid);
    auto* sums = reinterpret_cast<uint32_t*>(base + L.sums);
    auto* gstart = reinterpret_cast<uint32_t*>(base + L.gstart);
    auto* gsum = reinterpret_cast<double*>(base + L.gsum);
    auto* first = reinterpret_cast<uint32_t*>(base + L.first);
    auto* out = reinterpret_cast<uint64_t*>(base + L.chosen);

    if (R == 4) hipLaunchKernelGGL(slot_importance_kernel<4>, dim3(blocks(S)), dim3(kThreads), 0, s, nodes, stride,
                                   masks, S, imp);
    else hipLaunchKernelGGL(slot_importance_kernel<6>, dim3(blocks(S)), dim3(kThreads), 0, s, nodes, stride, masks, S,
                            imp);
    // slots by mask value: stable 32-bit rounds from the least significant half word up
    hipLaunchKernelGGL(iota_kernel, dim3(blocks(S)), dim3(kThreads), 0, s, vals, S);
    for (uint32_t w = 0; w < W; ++w)
        for (uint32_t h = 0; h < 2; ++h) {
            hipLaunchKernelGGL(mask_key_kernel, dim3(blocks(S)), dim3(kThreads), 0, s, masks, W, vals, S, w, h, keys);
            if (sort_pairs_u32(ws, S, 4, s) != vals) return hipErrorUnknown;  // 4 passes end in `vals`
        }
    hipLaunchKernelGGL(group_head_kernel, dim3(blocks(S)), dim3(kThreads), 0, s, masks, W, vals, S, imp, head, gid,
                       simp);
    hipError_t e = exclusive_scan_u32(gid, S, sums, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(group_start_kernel, dim3(blocks(S)), dim3(kThreads), 0, s, vals, head, gid, S, gstart, first);
    hipLaunchKernelGGL(group_sum_kernel, dim3(blocks(S)), dim3(kThreads), 0, s, head, gid, S, gstart, simp, gsum);
    // the number of distinct masks, and whether the last (largest value) is the full mask
    uint32_t tail[2] = {0, 0};
    e = hipMemcpyAsync(&tail[0], gid + S - 1, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&tail[1], head + S - 1, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    const uint32_t groups = tail[0] + tail[1];
    uint32_t last_slot = 0;
    std::vector<uint64_t> last(W);
    e = hipMemcpyAsync(&last_slot, first + groups - 1, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(last.data(), masks + (size_t)last_slot * W, (size_t)W * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    bool full = true;
    for (uint32_t w = 0; w < W; ++w) {
        const uint32_t bits = R * R * R - 64 * w;
        const uint64_t want = bits >= 64 ? ~0ull : ((1ull << bits) - 1);
        full = full && last[w] == want;
    }
    const uint32_t cand = groups - (full ? 1u : 0u);  // the full mask sorts last by value: leave it out
    const uint32_t take = cand < K - 1 ? cand : K - 1;
    if (take == 0) return hipSuccess;
    // distinct masks by importance descending; the stable rounds keep ties in value order (the sort of
    // `cand` pairs keeps its values right after its `cand` keys)
    uint32_t* gvals = keys + cand;
    hipLaunchKernelGGL(iota_kernel, dim3(blocks(cand)), dim3(kThreads), 0, s, gvals, cand);
    for (uint32_t h = 0; h < 2; ++h) {
        hipLaunchKernelGGL(importance_key_kernel, dim3(blocks(cand)), dim3(kThreads), 0, s, gsum, gvals, cand, h,
                           keys);
        if (sort_pairs_u32(ws, cand, 4, s) != gvals) return hipErrorUnknown;
    }
    hipLaunchKernelGGL(gather_chosen_kernel, dim3(blocks(take)), dim3(kThreads), 0, s, masks, W, gvals, first, take,
                       out);
    chosen.resize((size_t)take * W);
    e = hipMemcpyAsync(chosen.data(), out, chosen.size() * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? hipGetLastError() : e;
}

}  // namespace sc
