// Traversal with subspace culling (Alg. 4 with Alg. 1 and the mask AND of
// Sect. 3.1.2) for gfx950.
//
// Every ray runs the same canonical sequence as the plain reference
// traversal, so hits and the per-ray test counts are reproducible bit for
// bit:
//  slab test of child box [lo, hi]: per axis x, y, z the near bound n and far
//      bound f are lo and hi, swapped when the reciprocal direction inv is
//      negative; a = (n - o) * inv, b = (f - o) * inv,
//      b = b * (1 + 3*2^-23) (robust far value), t0 = max(a, t0),
//      t1 = min(b, t1), from t0 = tmin, t1 = best_t; hit iff t0 <= t1
//  ray mask (Alg. 1): for p = o + t*d at t0 and at t1, per axis
//      s = R / (hi - lo) (0 if the extent is not positive or s is infinite),
//      u = (p - lo) * s clamped to [0, R-1] (NaN -> 0), cell = (int)u
//  culling: child survives iff (ray mask AND object mask) != 0; skipped for
//      rays whose max|o| exceeds the scene's origin bound and for children
//      whose stored mask is full (or, in the sparse layout, absent)
//  order: both children survive -> the one with the smaller t0 (tie: child
//      0) is visited next and the other pushed with its t0; a popped entry
//      with t0 > best_t is dropped
//  leaf: Moller-Trumbore, two-sided, det == 0 rejects; accept t in
//      [tmin, best_t]; replace iff t < best_t or (t == best_t and the
//      original id is lower)
//
// Ray masks: R = 6 reads the R^6-entry table (1.42 MiB, resident in each
// XCD's L2). R = 4 uses the table's translation invariance instead: the
// entry for cells (b, e) is the pattern of the displacement e - b (x made
// non-negative by the symmetry of the sweep) moved to the componentwise
// minimum corner, so the 196 patterns (1.5 KiB) sit in LDS and the test is
// ((object mask >> corner bit) AND pattern) != 0. Both give the table's bits.
//
// Compressed masks: a codebook of at most 8 KiB (K <= 1024 at R = 4, K <= 256
// at R = 6) is copied into LDS, so with R = 4 a compressed mask test reads no
// memory beyond the node itself.
//
// Scheduling: persistent waves fed by partitioned ray queues (one range of
// consecutive rays per XCD by default; see the kernel). A wave takes
// 64*chunk consecutive rays at a time with one atomic add; whenever lanes
// finish their ray they take the next unstarted ray (ballot + prefix count),
// so lanes stay busy while the slowest rays of a wave finish. This changes
// which lane runs a ray, never the ray's own sequence. The next node of a
// lane stays in registers; postponed far children go to an LDS stack of
// STACK entries per lane and spill to private memory beyond that.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "raymask.h"

// 1: compile the device checks into every traversal kernel (kernels_trace_checked.hip does, for
// the library's checked instances; a failed check sets a bit and skips the access it guards)
#ifndef SC_DEVICE_CHECKS
#define SC_DEVICE_CHECKS 0
#endif

namespace sc {
namespace {

constexpr bool kChecks = SC_DEVICE_CHECKS != 0;

__device__ __forceinline__ void chk_fail(uint32_t* flags, uint32_t bit) {
    if (flags) atomicOr(flags, bit);
}

constexpr int kWave = 64;
constexpr uint32_t kModeNone = SC_MASK_NONE, kModeRaw = SC_MASK_RAW, kModeLut = SC_MASK_LUT,
                   kModeSparse = SC_MASK_SPARSE;
// Compressed masks with the codebook copied into LDS (chosen when it fits).
constexpr uint32_t kModeLutLds = 16;
// Compressed masks tested through the scene's 2-D bit table (one bit per test).
constexpr uint32_t kModeLutBits = 17;
constexpr uint32_t kCbLdsWords = 1024;  // 8 KiB: K <= 1024 at R = 4, K <= 256 at R = 6

__global__ void reset_counters_kernel(uint32_t* c, uint32_t n) {
    if (threadIdx.x < n) c[threadIdx.x] = 0u;
}

__device__ __forceinline__ float mx(float a, float b) { return (a > b) ? a : b; }

__device__ __forceinline__ bool ray_is_valid(float4 r0, float4 r1) {
    const bool fin = isfinite(r0.x) && isfinite(r0.y) && isfinite(r0.z) && isfinite(r0.w) &&
                     isfinite(r1.x) && isfinite(r1.y) && isfinite(r1.z);
    const bool dir = !(r1.x == 0.0f && r1.y == 0.0f && r1.z == 0.0f);
    return fin && dir && !isnan(r1.w) && (r0.w <= r1.w);
}

// R / ext rounded correctly, 0 when ext is not positive or the quotient is infinite. For ext in
// [2^-100, 2^100] the hardware reciprocal and one correction of the quotient by its exact
// residual (fused multiply-add) give the correctly rounded quotient -- checked on gfx950 for
// every float of that range, R = 4 and 6 -- in four operations instead of the full division's
// ten; any other extent takes the full division.
template <int R>
__device__ __forceinline__ float grid_scale_ext(float ext) {
    if (ext >= 0x1p-100f && ext <= 0x1p100f) {
        const float rc = __builtin_amdgcn_rcpf(ext);
        const float q = (float)R * rc;
        const float e = __builtin_fmaf(-ext, q, (float)R);
        return __builtin_fmaf(e, rc, q);
    }
    const float s = (ext > 0.0f) ? (float)R / ext : 0.0f;
    return isinf(s) ? 0.0f : s;
}

template <int R>
__device__ __forceinline__ float grid_scale(float lo, float hi) {
    return grid_scale_ext<R>(hi - lo);
}

template <int R>
__device__ __forceinline__ int cell_of(float lo, float s, float o, float d, float t) {
    const float p = o + t * d;
    float u = (p - lo) * s;
    u = (u > 0.0f) ? u : 0.0f;
    u = (u < (float)(R - 1)) ? u : (float)(R - 1);
    return (int)u;
}

struct Ray {
    float ox, oy, oz, dx, dy, dz, ix, iy, iz, tmin;
    uint32_t neg;  // bit j: the direction's axis-j reciprocal is negative (sign bit set)
};

// Slab interval of a box given by its near and far bound per axis (the lower
// bound is near where the reciprocal direction is non-negative).
__device__ __forceinline__ void slab_nf(const float* nr, const float* fr, const Ray& r, float tmax, float& t0,
                                        float& t1) {
    t0 = r.tmin;
    t1 = tmax;
    const float o[3] = {r.ox, r.oy, r.oz};
    const float inv[3] = {r.ix, r.iy, r.iz};
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const float a = (nr[j] - o[j]) * inv[j];
        float b = (fr[j] - o[j]) * inv[j];
        b = b * 0x1.000006p0f;
        // hardware max/min: with a NaN first operand they keep t0 / t1 as the
        // compare-and-select form does; they may differ from it only in the
        // sign of a zero result, which no comparison, cell index or order sees
        t0 = fmaxf(a, t0);
        t1 = fminf(b, t1);
    }
}

__device__ __forceinline__ void slab(const float* lo, const float* hi, const Ray& r, float tmax,
                                     float& t0, float& t1) {
    const float nr[3] = {(r.neg & 1u) ? hi[0] : lo[0], (r.neg & 2u) ? hi[1] : lo[1], (r.neg & 4u) ? hi[2] : lo[2]};
    const float fr[3] = {(r.neg & 1u) ? lo[0] : hi[0], (r.neg & 2u) ? lo[1] : hi[1], (r.neg & 4u) ? lo[2] : hi[2]};
    slab_nf(nr, fr, r, tmax, t0, t1);
}

// cells of box [lo, hi] holding o + t0 d (b) and o + t1 d (e)
template <int R>
__device__ __forceinline__ void ray_cells(const float* lo, const float* hi, const Ray& r, float t0, float t1,
                                          int& bx, int& by, int& bz, int& ex, int& ey, int& ez) {
    const float sx = grid_scale<R>(lo[0], hi[0]);
    const float sy = grid_scale<R>(lo[1], hi[1]);
    const float sz = grid_scale<R>(lo[2], hi[2]);
    bx = cell_of<R>(lo[0], sx, r.ox, r.dx, t0);
    by = cell_of<R>(lo[1], sy, r.oy, r.dy, t0);
    bz = cell_of<R>(lo[2], sz, r.oz, r.dz, t0);
    ex = cell_of<R>(lo[0], sx, r.ox, r.dx, t1);
    ey = cell_of<R>(lo[1], sy, r.oy, r.dy, t1);
    ez = cell_of<R>(lo[2], sz, r.oz, r.dz, t1);
}

// the same cells from a box given by its near and far bound per axis (sign bit j of `neg` set:
// the far bound is the lower one); hi - lo is |far - near|, exactly, as a difference and its
// negation round alike
template <int R>
__device__ __forceinline__ void ray_cells_nf(const float* nr, const float* fr, uint32_t neg, const Ray& r, float t0,
                                             float t1, int& bx, int& by, int& bz, int& ex, int& ey, int& ez) {
    const float lo[3] = {(neg & 1u) ? fr[0] : nr[0], (neg & 2u) ? fr[1] : nr[1], (neg & 4u) ? fr[2] : nr[2]};
    const float sx = grid_scale_ext<R>(fabsf(fr[0] - nr[0]));
    const float sy = grid_scale_ext<R>(fabsf(fr[1] - nr[1]));
    const float sz = grid_scale_ext<R>(fabsf(fr[2] - nr[2]));
    bx = cell_of<R>(lo[0], sx, r.ox, r.dx, t0);
    by = cell_of<R>(lo[1], sy, r.oy, r.dy, t0);
    bz = cell_of<R>(lo[2], sz, r.oz, r.dz, t0);
    ex = cell_of<R>(lo[0], sx, r.ox, r.dx, t1);
    ey = cell_of<R>(lo[1], sy, r.oy, r.dy, t1);
    ez = cell_of<R>(lo[2], sz, r.oz, r.dz, t1);
}

// the 2-D bit table answers (ray mask of key) AND (codebook entry idx) != 0 with one bit
template <int R>
__device__ __forceinline__ bool bit_overlap(const float* lo, const float* hi, const Ray& r, float t0, float t1,
                                            const uint32_t* table, uint32_t K, uint32_t idx) {
    int bx, by, bz, ex, ey, ez;
    ray_cells<R>(lo, hi, r, t0, t1, bx, by, bz, ex, ey, ez);
    const uint32_t row = bit_row((uint32_t)((bx * R + by) * R + bz), (uint32_t)((ex * R + ey) * R + ez));
    return (table[row * (K >> 5) + (idx >> 5)] >> (idx & 31u)) & 1u;
}

// R = 4: the ray mask of cells (b, e) is displacement pattern pidx (x made
// non-negative by the symmetry of the sweep) moved to the componentwise minimum
// corner, bit `shift`: the test is ((mask >> shift) AND pattern) != 0
__device__ __forceinline__ void r4_pattern(int bx, int by, int bz, int ex, int ey, int ez, uint32_t& pidx,
                                           uint32_t& shift) {
    int qx = bx, qy = by, qz = bz, fx = ex, fy = ey, fz = ez;
    if (fx < qx) {
        qx = ex; qy = ey; qz = ez; fx = bx; fy = by; fz = bz;
    }
    pidx = (uint32_t)(((fx - qx) * 7 + (fy - qy + 3)) * 7 + (fz - qz + 3));
    const int my = qy < fy ? qy : fy, mz = qz < fz ? qz : fz;
    shift = (uint32_t)(qx + 4 * my + 16 * mz);
}

// (ray mask of cells b, e) AND (object mask om) != 0
template <int R>
__device__ __forceinline__ bool mask_overlap_cells(int bx, int by, int bz, int ex, int ey, int ez,
                                                   const uint64_t* om, const uint64_t* lut, const uint64_t* lds_pat) {
    constexpr int W = (R * R * R + 63) / 64;
    uint64_t ob[W];
    load_mask<W>(om, ob);
    if constexpr (R == 4) {
        // displacement pattern (LDS) against the mask moved to its corner
        uint32_t pidx, shift;
        r4_pattern(bx, by, bz, ex, ey, ez, pidx, shift);
        return ((ob[0] >> shift) & lds_pat[pidx]) != 0;
    } else {
        const uint32_t key = (uint32_t)(((((bx * R + by) * R + bz) * R + ex) * R + ey) * R + ez);
        uint64_t rm[W];
        load_mask<W>(lut + (size_t)key * W, rm);
        uint64_t acc = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) acc |= rm[w] & ob[w];
        return acc != 0;
    }
}

// (ray mask of the cells holding o + t0 d and o + t1 d) AND (object mask om) != 0
template <int R>
__device__ __forceinline__ bool mask_overlap(const float* lo, const float* hi, const Ray& r, float t0, float t1,
                                             const uint64_t* om, const uint64_t* lut, const uint64_t* lds_pat) {
    int bx, by, bz, ex, ey, ez;
    ray_cells<R>(lo, hi, r, t0, t1, bx, by, bz, ex, ey, ez);
    return mask_overlap_cells<R>(bx, by, bz, ex, ey, ez, om, lut, lds_pat);
}

// order by (key, id): swap when b comes first
__device__ __forceinline__ void order2(float& ka, uint32_t& ia, uint32_t& ra, float& kb, uint32_t& ib,
                                       uint32_t& rb) {
    const bool sw = (kb < ka) || (kb == ka && ib < ia);
    const float k = sw ? kb : ka;
    const uint32_t i = sw ? ib : ia, q = sw ? rb : ra;
    kb = sw ? ka : kb;
    ib = sw ? ia : ib;
    rb = sw ? ra : rb;
    ka = k;
    ia = i;
    ra = q;
}

// LDS of one block of the traversal kernel: its stack, the R = 4 ray-mask
// patterns and the codebook copy where the mode keeps them in LDS.
template <uint32_t MODE, int R, int BLOCK, int STACK>
constexpr uint32_t trace_lds_bytes() {
    const bool pat = (R == 4) && (MODE != kModeNone) && (MODE != kModeLutBits);
    return (uint32_t)(STACK * BLOCK) * 8u + (pat ? (uint32_t)kPatterns<4> * 8u : 8u) +
           (MODE == kModeLutLds ? kCbLdsWords * 8u : 16u);
}
constexpr uint32_t kLdsPerCu = 160u * 1024u;  // gfx950

// Minimum waves per SIMD the register allocation must allow (1 = no constraint).
// Held to 80 VGPRs (6 waves): the plain 4-wide kernel, the bit-table kernels, the
// R = 4 raw kernel on float boxes and the R = 6 raw kernel on quantised boxes
// (their few spilled registers sit in the ray set-up, not in the traversal
// step). The other 4-wide mask kernels -- among them the quantised R = 4 raw
// kernel, whose four in-flight mask reads need the room -- spill inside the
// step at 80 and are held to 96 VGPRs (5 waves). Batched launches keep each
// lane's scene pointers in registers as well: their mask kernels are held to 96
// VGPRs, the float-box R = 6 ones to 128 (4 waves). Where LDS already allows fewer
// waves than that, the target is what LDS allows: registers beyond it would buy
// nothing.
template <uint32_t MODE, int R, int WIDTH, int BLOCK, int STACK, bool QUANT = false, bool BATCH = false>
struct MinWaves {
    static constexpr int target =
        (WIDTH == 4 && BATCH && MODE != kModeNone && R == 6 && !QUANT) ? 4
        : (WIDTH == 4 && BATCH && MODE != kModeNone)                   ? 5
        : (WIDTH == 4 && (MODE == kModeNone || (MODE == kModeRaw && (R == 4) != QUANT) || MODE == kModeLutBits)) ? 6
        : (WIDTH == 4) ? 5
                       : 1;
    static constexpr int lds_waves =
        (int)((kLdsPerCu / trace_lds_bytes<MODE, R, BLOCK, STACK>()) * (uint32_t)(BLOCK / kWave) / 4u);
    static constexpr int value = (lds_waves < target) ? (lds_waves > 1 ? lds_waves : 1) : target;
};

template <uint32_t MODE, int R, int BLOCK, int STACK, bool BATCH, int WIDTH, bool QUANT = false>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(MinWaves<MODE, R, WIDTH, BLOCK, STACK, QUANT, BATCH>::value)))
void trace_kernel(TraceLaunch a) {
    static_assert(WIDTH == 2 || (WIDTH == 4 && MODE != kModeSparse), "4-wide: no sparse masks");
    static_assert(!BATCH || (MODE != kModeLutLds && MODE != kModeLutBits), "batches read each scene's codebook");
    constexpr int W = (R * R * R + 63) / 64;
    constexpr uint32_t kStride = (MODE == kModeRaw) ? kRawNodeBytes : kNodeBytes;
    constexpr bool kPatLds = (R == 4) && (MODE != kModeNone) && (MODE != kModeLutBits);
    constexpr bool kCbLds = (MODE == kModeLutLds);
    // 4-wide nodes: issue the mask reads of several children before deciding any
    // (where a test reads one word: the bit table, or an R = 4 mask; an R = 6 test reads two 32-byte
    // rows, and holding them for several children costs more waves than the overlap gains)
    constexpr bool kPhased = (WIDTH == 4) && (MODE == kModeLutBits || (R == 4 && MODE != kModeNone));
    __shared__ uint2 lds_stack[STACK * BLOCK];
    __shared__ uint64_t lds_pat[kPatLds ? kPatterns<4> : 1];
    __shared__ __attribute__((aligned(16))) uint64_t lds_cb[kCbLds ? kCbLdsWords : 2];

    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & (kWave - 1);
    if constexpr (kPatLds) {
        for (int k = tid; k < kPatterns<4>; k += BLOCK) lds_pat[k] = a.patterns[k];
    }
    if constexpr (kCbLds) {
        for (uint32_t k = tid; k < a.K * W; k += BLOCK) lds_cb[k] = a.codebook[k];
    }
    if constexpr (kPatLds || kCbLds) __syncthreads();
    const uint64_t lanes_below = (1ull << lane) - 1ull;
    const uint32_t chunk_rays = kWave * a.chunk;
    const bool use_flags = (a.flags & (SC_TRACE_CULL | SC_TRACE_SHADOW)) != 0;
    const bool cull = (a.flags & SC_TRACE_CULL) != 0;
    const bool shadow_flag = (a.flags & SC_TRACE_SHADOW) != 0;

    // deeper stack entries: a binary traversal holds at most depth + 1 <= 65,
    // a 4-wide one at most kMaxStack4 (checked when the scene is built)
    constexpr int kSpill = (WIDTH == 2) ? (int)kMaxDepth - STACK + 1 : (int)kMaxStack4 - STACK;
    uint2 spill[kSpill];

    // The scene of the lane's current ray: uniform for a single scene, per
    // lane in a batch (set when the lane takes a ray).
    const unsigned char* s_nodes = a.nodes;
    const float* s_tris = a.tris;
    const uint64_t* s_codebook = a.codebook;
    const uint64_t* s_side = a.side_masks;
    const float* s_rays = a.rays;
    uint32_t s_full = a.full_start, s_root = a.root;
    float s_bound = a.origin_bound;
    sc_hit* s_hits = a.hits;
    uint32_t* s_extra = a.extra;
    uint32_t* s_fp = a.slot_fp;
    const uint32_t* s_src4 = a.src4;
    uint32_t s_nlim = a.chk_nodes, s_tlim = a.chk_tris;  // device checks: the lane's scene's limits

    // The rays are split into a.parts contiguous partitions, one queue counter
    // each. Workgroups are dispatched round-robin over the XCDs, so a wave
    // starts on partition (block % parts) -- its own XCD's share when parts is
    // the XCD count -- and moves on to the others once that one is empty.
    const uint32_t parts = a.parts;
    const uint32_t home = blockIdx.x % parts;
    uint32_t exhausted = 0;        // wave-uniform bit per partition
    uint32_t cursor = 0, end = 0;  // wave-uniform range of unstarted rays
    bool more = true;
    // next range of rays for this wave; false when every partition is empty
    auto fetch = [&]() -> bool {
        for (uint32_t t = 0; t < parts; ++t) {
            const uint32_t p = (home + t) % parts;
            if (exhausted & (1u << p)) continue;
            const uint32_t lo = (uint32_t)(((uint64_t)a.n * p) / parts);
            const uint32_t hi = (uint32_t)(((uint64_t)a.n * (p + 1)) / parts);
            uint32_t base = 0;
            if (lane == 0) base = atomicAdd(a.queue + p, chunk_rays);
            base = __shfl(base, 0, kWave);
            if (base < hi - lo) {
                cursor = lo + base;
                end = min(hi, cursor + chunk_rays);
                return true;
            }
            exhausted |= 1u << p;
        }
        return false;
    };
    {
        bool has = false;
        uint32_t ray_id = 0;
        Ray r;
        float best_t = 0.0f;
        uint32_t best = kNoHit, box_tests = 0, tri_tests = 0, mask_tests = 0, mask_culls = 0;
        bool use_mask = false;
        int sp = 0;
        uint32_t ref = 0;
        uint32_t waited = 0;  // steps the leaf lanes have waited in a row
        while (true) {
            // refill idle lanes with unstarted rays, once a.refill of them are idle or
            // none is busy: the refill (ray load, validity test, set-up) costs the
            // wave the same for one lane as for many; a ray that starts a few steps
            // later traverses exactly as before
            const uint64_t idle = __ballot(!has);
            if (idle != 0 && ((uint32_t)__popcll(idle) >= a.refill || idle == __ballot(true))) {
                if (cursor >= end && more) more = fetch();
                if (cursor < end) {
                    if (!has) {
                        const uint32_t gid = cursor + (uint32_t)__popcll(idle & lanes_below);
                        if (gid < end) {
                            uint32_t id = a.order ? a.order[gid] : gid;
                            if constexpr (BATCH) {
                                // item holding this ray: the last one whose first ray is <= its index
                                const uint32_t g = id;
                                uint32_t lo = 0, hi = a.n_items;
                                while (hi - lo > 1) {
                                    const uint32_t mid = (lo + hi) >> 1;
                                    if (a.items[mid].ray_begin <= g) lo = mid;
                                    else hi = mid;
                                }
                                const BatchItem& it = a.items[lo];
                                s_nodes = it.nodes; s_tris = it.tris; s_codebook = it.codebook;
                                s_side = it.side_masks; s_rays = it.rays; s_full = it.full_start;
                                s_root = it.root; s_bound = it.origin_bound; s_hits = it.hits;
                                s_extra = it.extra; s_fp = it.slot_fp; s_src4 = it.src4;
                                if constexpr (kChecks) {
                                    s_nlim = min(a.chk_nodes, it.n_nodes);
                                    s_tlim = min(a.chk_tris, it.n_tris);
                                }
                                id = g - it.ray_begin;
                            }
                            const float4 r0 = reinterpret_cast<const float4*>(s_rays)[2 * (size_t)id];
                            const float4 r1 = reinterpret_cast<const float4*>(s_rays)[2 * (size_t)id + 1];
                            ray_id = id;
                            if (ray_is_valid(r0, r1) && s_root != kEmptyRef) {
                                r.ox = r0.x; r.oy = r0.y; r.oz = r0.z; r.tmin = r0.w;
                                r.dx = r1.x; r.dy = r1.y; r.dz = r1.z;
                                r.ix = 1.0f / r.dx; r.iy = 1.0f / r.dy; r.iz = 1.0f / r.dz;
                                r.neg = (signbit(r.ix) ? 1u : 0u) | (signbit(r.iy) ? 2u : 0u) |
                                        (signbit(r.iz) ? 4u : 0u);
                                best_t = r1.w;
                                best = kNoHit;
                                box_tests = tri_tests = mask_tests = mask_culls = 0;
                                use_mask = (MODE != kModeNone) && use_flags &&
                                           !(mx(mx(fabsf(r.ox), fabsf(r.oy)), fabsf(r.oz)) > s_bound);
                                sp = 0;
                                ref = s_root;
                                has = true;
                            } else {
                                reinterpret_cast<uint4*>(s_hits)[id] =
                                    make_uint4(kNoHit, __float_as_uint(__builtin_inff()), 0u, 0u);
                                if (s_extra) reinterpret_cast<uint2*>(s_extra)[id] = make_uint2(0u, 0u);
                            }
                        }
                    }
                    cursor += (uint32_t)__popcll(idle);
                }
            }
            if (__ballot(has) == 0) {
                if (!more && cursor >= end) break;  // no ray left for this wave
                continue;                           // every refilled ray finished at once (invalid rays)
            }
            {
                // Leaf gathering: a wave runs the triangle tests as soon as one lane needs
                // them, for the price of all. A lane whose ray stands at a leaf therefore
                // waits (its ray does not advance) while fewer than a.gather lanes do and
                // some lane still stands at an inner node, at most a.gather / 2 steps in a
                // row. Every ray keeps its own sequence of visits, so no result or count
                // changes; the wait ends at the latest when the inner lanes run out, which
                // they do once the ray queue is empty.
                const bool at_leaf = has && (ref & kLeafBit) != 0;
                const uint64_t leaves = __ballot(at_leaf);
                const uint64_t inner = __ballot(has && (ref & kLeafBit) == 0);
                const bool gather = inner != 0 && (uint32_t)__popcll(leaves) < a.gather && waited < a.gather / 2;
                waited = gather ? waited + 1u : 0u;  // the same in every lane
                if (gather && at_leaf) continue;
            }
            if (!has) continue;

            // one traversal step of this lane's ray
            bool pop = true;
            bool bad = false;  // device checks: the node or leaf reference is out of range
            if constexpr (kChecks) {
                if (ref & kLeafBit) {
                    const uint32_t first = ref & 0x1FFFFFFFu, count = ((ref >> 29) & 3u) + 1u;
                    bad = first >= s_tlim || count > s_tlim - first;
                    if (bad) chk_fail(a.chk_flags, kChkTri);
                } else if (ref >= s_nlim) {
                    bad = true;
                    chk_fail(a.chk_flags, kChkNode);
                }
                if (bad) sp = 0;  // the ray ends with the hit it has
            }
            if (bad) {
                // nothing is read
            } else if (ref & kLeafBit) {
                const uint32_t first = ref & 0x1FFFFFFFu;
                const uint32_t count = ((ref >> 29) & 3u) + 1u;
                for (uint32_t k = 0; k < count; ++k) {
                    ++tri_tests;
                    const float4* tp = reinterpret_cast<const float4*>(
                        reinterpret_cast<const unsigned char*>(s_tris) + (size_t)(first + k) * kTriBytes);
                    const float4 q0 = tp[0], q1 = tp[1], q2 = tp[2];
                    const float v0x = q0.x, v0y = q0.y, v0z = q0.z;
                    const float e1x = q0.w, e1y = q1.x, e1z = q1.y;
                    const float e2x = q1.z, e2y = q1.w, e2z = q2.x;
                    const uint32_t id = __float_as_uint(q2.y);
                    const float px = r.dy * e2z - r.dz * e2y;
                    const float py = r.dz * e2x - r.dx * e2z;
                    const float pz = r.dx * e2y - r.dy * e2x;
                    const float det = (e1x * px + e1y * py) + e1z * pz;
                    if (det == 0.0f) continue;
                    const float idet = 1.0f / det;
                    const float sx = r.ox - v0x, sy = r.oy - v0y, sz = r.oz - v0z;
                    const float u = ((sx * px + sy * py) + sz * pz) * idet;
                    if (u < 0.0f || u > 1.0f) continue;
                    const float qx = sy * e1z - sz * e1y;
                    const float qy = sz * e1x - sx * e1z;
                    const float qz = sx * e1y - sy * e1x;
                    const float v = ((r.dx * qx + r.dy * qy) + r.dz * qz) * idet;
                    if (v < 0.0f || u + v > 1.0f) continue;
                    const float t = ((e2x * qx + e2y * qy) + e2z * qz) * idet;
                    if (t < r.tmin || t > best_t) continue;
                    if (t < best_t || (t == best_t && id < best)) {
                        best_t = t;
                        best = id;
                    }
                }
            } else if constexpr (WIDTH == 4) {
                // 4-wide node: SoA boxes lo.x[4] lo.y[4] lo.z[4] hi.x[4] hi.y[4] hi.z[4], refs[4], aux;
                // quantised: corner, step exponents, refs, 8-bit planes, aux in 64 bytes
                const float4* np4 =
                    reinterpret_cast<const float4*>(s_nodes + (size_t)ref * (QUANT ? kNode4QBytes : kNode4Bytes));
                const uint32_t sx = r.neg & 1u, sy = (r.neg >> 1) & 1u, sz = (r.neg >> 2) & 1u;
                float4 nx, ny, nz, fx, fy, fz;
                uint4 cr;
                uint32_t ax0 = 0u, ax1 = 0u;  // LUT modes: the four 16-bit codebook indices
                if constexpr (QUANT) {
                    // four line pieces: corner + exponents, refs, qlo.xyz qhi.x, qhi.yz aux
                    const uint4 h = reinterpret_cast<const uint4*>(np4)[0];
                    cr = reinterpret_cast<const uint4*>(np4)[1];
                    const uint4 q0 = reinterpret_cast<const uint4*>(np4)[2];
                    const uint4 q1 = reinterpret_cast<const uint4*>(np4)[3];
                    const float cx = __uint_as_float(h.x), cy = __uint_as_float(h.y), cz = __uint_as_float(h.z);
                    // step 2^(b - 127) from its biased exponent b (1..254): a normal float
                    const float ux = __uint_as_float((h.w & 0xFFu) << 23);
                    const float uy = __uint_as_float(((h.w >> 8) & 0xFFu) << 23);
                    const float uz = __uint_as_float(((h.w >> 16) & 0xFFu) << 23);
                    // near / far plane words of each axis, picked by the ray's direction signs
                    const uint32_t wnx = sx ? q0.w : q0.x, wfx = sx ? q0.x : q0.w;
                    const uint32_t wny = sy ? q1.x : q0.y, wfy = sy ? q0.y : q1.x;
                    const uint32_t wnz = sz ? q1.y : q0.z, wfz = sz ? q0.z : q1.y;
                    // corner + q * step: the product is exact, so one fused multiply-add rounds the
                    // sum exactly as a multiply then an add would
                    auto dq = [](uint32_t w, float c, float u) {
                        return make_float4(__builtin_fmaf((float)(w & 0xFFu), u, c),
                                           __builtin_fmaf((float)((w >> 8) & 0xFFu), u, c),
                                           __builtin_fmaf((float)((w >> 16) & 0xFFu), u, c),
                                           __builtin_fmaf((float)(w >> 24), u, c));
                    };
                    nx = dq(wnx, cx, ux); ny = dq(wny, cy, uy); nz = dq(wnz, cz, uz);
                    fx = dq(wfx, cx, ux); fy = dq(wfy, cy, uy); fz = dq(wfz, cz, uz);
                    ax0 = q1.z;  // the aux words ride in the last piece
                    ax1 = q1.w;
                } else {
                    // near and far bounds of the four children, picked by address from the
                    // lo / hi rows (row j holds lo, row j + 3 hi, of axis j)
                    nx = np4[3 * sx]; ny = np4[1 + 3 * sy]; nz = np4[2 + 3 * sz];
                    fx = np4[3 - 3 * sx]; fy = np4[4 - 3 * sy]; fz = np4[5 - 3 * sz];
                    cr = reinterpret_cast<const uint4*>(np4)[6];
                }
                // aux words at byte 112, for the LUT modes' four 16-bit codebook indices; raw
                // nodes keep their full-mask flags in bit 28 of the refs, so they load one line
                // piece less per visit (each lane's load costs the address path a line access)
                if constexpr (!QUANT && MODE != kModeNone && MODE != kModeRaw) {  // raw: flags in the refs
                    const uint2 a2 = reinterpret_cast<const uint2*>(np4)[14];
                    ax0 = a2.x;
                    ax1 = a2.y;
                }
                const float cnx[4] = {nx.x, nx.y, nx.z, nx.w}, cny[4] = {ny.x, ny.y, ny.z, ny.w};
                const float cnz[4] = {nz.x, nz.y, nz.z, nz.w}, cfx[4] = {fx.x, fx.y, fx.z, fx.w};
                const float cfy[4] = {fy.x, fy.y, fy.z, fy.w}, cfz[4] = {fz.x, fz.y, fz.z, fz.w};
                const uint32_t crf[4] = {cr.x, cr.y, cr.z, cr.w};
                // surviving children as (t0, child index, ref); dead ones sort last. The
                // loop keeps a flag instead of leaving an iteration early: a form with
                // `continue` in the mask branch was compiled into code that dropped every
                // child whose mask was tested.
                float key[4];
                uint32_t kid[4], kref[4];
                uint32_t alive = 0;
                // Slab tests of all four children first, without a branch (an unused child's
                // result is computed and dropped), so the node's pieces are waited for once on
                // every path. Where a mask read takes one load (the bit table, R = 4 masks), the
                // reads of all tested children are then issued together before any is decided,
                // instead of one round trip after another; otherwise each tested child reads and
                // decides in turn. Children are still decided in order and every count is the same.
                bool ckeep[4], cneed[4];
                float ct0[4], ct1[4];
                uint32_t cidx4[4];  // LUT modes: codebook index per child
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    kref[c] = (crf[c] == kEmptyRef) ? kEmptyRef : (crf[c] & ~kRef4Full);
                    const bool used = crf[c] != kEmptyRef;
                    float t0, t1;
                    const float nr[3] = {cnx[c], cny[c], cnz[c]}, fr[3] = {cfx[c], cfy[c], cfz[c]};
                    slab_nf(nr, fr, r, best_t, t0, t1);
                    box_tests += used ? 1u : 0u;
                    ckeep[c] = used && t0 <= t1;
                    ct0[c] = t0;
                    ct1[c] = t1;
                    // whether the child's mask is tested (reads the refs' full flags or the
                    // codebook indices here, before any mask read is in flight)
                    bool test = false;
                    cidx4[c] = 0u;
                    if constexpr (MODE == kModeRaw) {
                        test = !(crf[c] & kRef4Full);
                    } else if constexpr (MODE != kModeNone) {
                        cidx4[c] = ((c < 2 ? ax0 : ax1) >> (16 * (c & 1))) & 0xFFFFu;
                        test = cidx4[c] < s_full;
                    }
                    cneed[c] = (MODE != kModeNone) && ckeep[c] && use_mask && test;
                    if constexpr (kChecks && !BATCH && MODE != kModeNone && MODE != kModeRaw) {
                        if (cneed[c] && cidx4[c] >= a.K) {
                            chk_fail(a.chk_flags, kChkIndex);
                            cneed[c] = false;
                        }
                    }
                }
                uint32_t pw[4], pb[4], pp[4];  // phased: bit table word + bit; R = 4 pattern + shift
                uint64_t pm[4];                // phased R = 4: the object mask
                if constexpr (kPhased) {
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        pw[c] = 0u;
                        pb[c] = 0u;
                        pp[c] = 0u;
                        pm[c] = 0u;
                        const uint32_t idx = cidx4[c];
                        if (cneed[c]) {
                            const float nr[3] = {cnx[c], cny[c], cnz[c]}, fr[3] = {cfx[c], cfy[c], cfz[c]};
                            int bx, by, bz, ex, ey, ez;
                            ray_cells_nf<R>(nr, fr, r.neg, r, ct0[c], ct1[c], bx, by, bz, ex, ey, ez);
                            if constexpr (MODE == kModeLutBits) {
                                const uint32_t row = bit_row((uint32_t)((bx * R + by) * R + bz),
                                                             (uint32_t)((ex * R + ey) * R + ez));
                                // R^3 (R^3 + 1) / 2 rows of K / 32 words: below 2^22 words for R <= 6, K <= 4096
                                pw[c] = a.bit_table[row * (a.K >> 5) + (idx >> 5)];
                                pb[c] = idx & 31u;
                            } else {
                                if constexpr (MODE == kModeRaw) pm[c] = s_side[(size_t)ref * 4 + c];
                                if constexpr (MODE == kModeLut) pm[c] = s_codebook[idx];
                                if constexpr (MODE == kModeLutLds) pm[c] = lds_cb[idx];
                                r4_pattern(bx, by, bz, ex, ey, ez, pp[c], pb[c]);
                            }
                        }
                    }
                }
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    bool keep = ckeep[c];
                    if constexpr (MODE != kModeNone) {
                        if (cneed[c]) {
                            ++mask_tests;
                            bool any;
                            if constexpr (kPhased) {
                                if constexpr (MODE == kModeLutBits) any = ((pw[c] >> pb[c]) & 1u) != 0u;
                                else any = ((pm[c] >> pb[c]) & lds_pat[pp[c]]) != 0;
                            } else {
                                const uint64_t* om = nullptr;
                                if constexpr (MODE == kModeRaw) om = s_side + ((size_t)ref * 4 + c) * W;
                                if constexpr (MODE == kModeLutLds) om = lds_cb + cidx4[c] * W;
                                if constexpr (MODE == kModeLut) om = s_codebook + (size_t)cidx4[c] * W;
                                const float nr[3] = {cnx[c], cny[c], cnz[c]}, fr[3] = {cfx[c], cfy[c], cfz[c]};
                                int bx, by, bz, ex, ey, ez;
                                ray_cells_nf<R>(nr, fr, r.neg, r, ct0[c], ct1[c], bx, by, bz, ex, ey, ez);
                                any = mask_overlap_cells<R>(bx, by, bz, ex, ey, ez, om, a.lut, lds_pat);
                            }
                            if (!any) {
                                ++mask_culls;
                                if (shadow_flag && s_fp) atomicAdd(&s_fp[s_src4[(size_t)ref * 4 + c]], 1u);
                                keep = !cull;
                            }
                        }
                    }
                    key[c] = __builtin_inff();
                    kid[c] = 4u + (uint32_t)c;
                    if (keep) {
                        key[c] = ct0[c];
                        kid[c] = (uint32_t)c;
                        ++alive;
                    }
                }
                // sorting network for four (t0, child) pairs
                order2(key[0], kid[0], kref[0], key[1], kid[1], kref[1]);
                order2(key[2], kid[2], kref[2], key[3], kid[3], kref[3]);
                order2(key[0], kid[0], kref[0], key[2], kid[2], kref[2]);
                order2(key[1], kid[1], kref[1], key[3], kid[3], kref[3]);
                order2(key[1], kid[1], kref[1], key[2], kid[2], kref[2]);
                if (alive > 0) {
                    // farther survivors go on the stack, the second nearest on top
#pragma unroll
                    for (int j = 3; j >= 1; --j) {
                        if ((uint32_t)j < alive) {
                            const uint2 e = make_uint2(kref[j], __float_as_uint(key[j]));
                            if (kChecks && (uint32_t)sp >= a.chk_stack) {
                                chk_fail(a.chk_flags, kChkStack);
                            } else {
                                if (sp < STACK) lds_stack[sp * BLOCK + tid] = e;
                                else spill[sp - STACK] = e;
                                ++sp;
                            }
                        }
                    }
                    ref = kref[0];
                    pop = false;
                }
            } else {
                const unsigned char* np = s_nodes + (size_t)ref * kStride;
                const float4 n0 = reinterpret_cast<const float4*>(np)[0];
                const float4 n1 = reinterpret_cast<const float4*>(np)[1];
                const float4 n2 = reinterpret_cast<const float4*>(np)[2];
                const uint4 n3 = reinterpret_cast<const uint4*>(np)[3];
                const float lo0[3] = {n0.x, n0.y, n0.z}, hi0[3] = {n0.w, n1.x, n1.y};
                const float lo1[3] = {n1.z, n1.w, n2.x}, hi1[3] = {n2.y, n2.z, n2.w};
                float t00, t10, t01, t11;
                box_tests += 2;
                slab(lo0, hi0, r, best_t, t00, t10);
                slab(lo1, hi1, r, best_t, t01, t11);
                bool h0 = t00 <= t10, h1 = t01 <= t11;
                if constexpr (MODE != kModeNone) {
                    if (use_mask) {
#pragma unroll
                        for (int c = 0; c < 2; ++c) {
                            // a full mask cannot cull (the ray mask holds its entry cell): no test
                            bool test;
                            const uint64_t* om = nullptr;
                            uint32_t idx = 0;
                            if constexpr (MODE == kModeRaw) {
                                test = !((n3.z >> c) & 1u);
                                om = reinterpret_cast<const uint64_t*>(np + 64) + c * W;
                            } else if constexpr (MODE == kModeLut || MODE == kModeLutLds || MODE == kModeLutBits) {
                                idx = c ? (n3.z >> 16) : (n3.z & 0xFFFFu);
                                test = idx < s_full;
                                if constexpr (kChecks && !BATCH) {
                                    if (test && idx >= a.K) {
                                        chk_fail(a.chk_flags, kChkIndex);
                                        test = false;
                                    }
                                }
                                if constexpr (MODE == kModeLut) om = s_codebook + (size_t)idx * W;
                                if constexpr (MODE == kModeLutLds) om = lds_cb + (test ? idx : 0u) * W;
                            } else {
                                const uint32_t ms = c ? n3.w : n3.z;
                                test = ms != kNoMask;
                                om = s_side + (size_t)(test ? ms : 0u) * W;
                            }
                            if ((c ? h1 : h0) && test) {
                                ++mask_tests;
                                const float* lo = c ? lo1 : lo0;
                                const float* hi = c ? hi1 : hi0;
                                const float t0 = c ? t01 : t00, t1 = c ? t11 : t10;
                                bool any;
                                if constexpr (MODE == kModeLutBits) any = bit_overlap<R>(lo, hi, r, t0, t1, a.bit_table, a.K, idx);
                                else any = mask_overlap<R>(lo, hi, r, t0, t1, om, a.lut, lds_pat);
                                if (!any) {
                                    ++mask_culls;
                                    if (shadow_flag && s_fp) atomicAdd(&s_fp[2 * (size_t)ref + c], 1u);
                                    if (cull) {
                                        if (c) h1 = false;
                                        else h0 = false;
                                    }
                                }
                            }
                        }
                    }
                }
                if (h0 && h1) {
                    const bool near1 = t01 < t00;
                    const uint2 e = make_uint2(near1 ? n3.x : n3.y, __float_as_uint(near1 ? t00 : t01));
                    if (kChecks && (uint32_t)sp >= a.chk_stack) {
                        chk_fail(a.chk_flags, kChkStack);
                    } else {
                        if (sp < STACK) lds_stack[sp * BLOCK + tid] = e;
                        else spill[sp - STACK] = e;
                        ++sp;
                    }
                    ref = near1 ? n3.y : n3.x;
                    pop = false;
                } else if (h0 || h1) {
                    ref = h0 ? n3.x : n3.y;
                    pop = false;
                }
            }
            if (pop) {
                bool found = false;
                while (sp > 0) {
                    --sp;
                    const uint2 e = (sp < STACK) ? lds_stack[sp * BLOCK + tid] : spill[sp - STACK];
                    if (__uint_as_float(e.y) > best_t) continue;
                    ref = e.x;
                    found = true;
                    break;
                }
                if (!found) {
                    const float tout = (best == kNoHit) ? __builtin_inff() : best_t;
                    reinterpret_cast<uint4*>(s_hits)[ray_id] =
                        make_uint4(best, __float_as_uint(tout), box_tests, tri_tests);
                    if (s_extra) reinterpret_cast<uint2*>(s_extra)[ray_id] = make_uint2(mask_tests, mask_culls);
                    has = false;
                }
            }
        }
    }
}

template <uint32_t MODE, int R, int BLOCK, int STACK, bool BATCH, int WIDTH, bool QUANT = false>
hipError_t launch_one(const TraceLaunch& a, hipStream_t s) {
    // blocks per CU that fit, and CUs: queried once per instance (on the device current at
    // the first launch; every GPU of an MI355X node is the same part), thread-safe
    struct Occupancy {
        int per_cu, cus;
    };
    static const Occupancy occ = [] {
        int dev = 0, c = 0, p = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev);
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&p, trace_kernel<MODE, R, BLOCK, STACK, BATCH, WIDTH, QUANT>,
                                                           BLOCK, 0);
        return Occupancy{p > 0 ? p : 4, c > 0 ? c : 256};
    }();
    const int per_cu = occ.per_cu, cus = occ.cus;
    uint32_t blocks_per_cu = (uint32_t)per_cu;
    if (a.waves > 0) {
        // 4 SIMDs per CU: waves per SIMD * 4 / waves per block, at least one block
        uint32_t cap = (a.waves * 4u) / (BLOCK / kWave);
        cap = cap > 0 ? cap : 1u;
        blocks_per_cu = cap < blocks_per_cu ? cap : blocks_per_cu;
    }
    const uint32_t resident = (uint32_t)cus * blocks_per_cu;
    const uint32_t waves = (a.n + kWave - 1) / kWave;
    uint32_t blocks = (waves + BLOCK / kWave - 1) / (BLOCK / kWave);
    blocks = blocks < resident ? blocks : resident;
    hipLaunchKernelGGL(reset_counters_kernel, dim3(1), dim3(kQueueParts), 0, s, a.queue, kQueueParts);
    hipLaunchKernelGGL((trace_kernel<MODE, R, BLOCK, STACK, BATCH, WIDTH, QUANT>), dim3(blocks), dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

template <int BLOCK, int STACK, bool BATCH>
hipError_t launch_cfg(const TraceLaunch& a, hipStream_t s) {
    switch (a.mode) {
        case SC_MASK_NONE: return launch_one<kModeNone, 6, BLOCK, STACK, BATCH, 2>(a, s);
        case SC_MASK_RAW:
            return a.R == 4 ? launch_one<kModeRaw, 4, BLOCK, STACK, BATCH, 2>(a, s)
                            : launch_one<kModeRaw, 6, BLOCK, STACK, BATCH, 2>(a, s);
        case SC_MASK_LUT:
            if (!BATCH && a.bit_table)
                return a.R == 4 ? launch_one<kModeLutBits, 4, BLOCK, STACK, false, 2>(a, s)
                                : launch_one<kModeLutBits, 6, BLOCK, STACK, false, 2>(a, s);
            if (!BATCH && !a.cb_global && (size_t)a.K * (a.R == 4 ? 1 : 4) <= kCbLdsWords)
                return a.R == 4 ? launch_one<kModeLutLds, 4, BLOCK, STACK, false, 2>(a, s)
                                : launch_one<kModeLutLds, 6, BLOCK, STACK, false, 2>(a, s);
            return a.R == 4 ? launch_one<kModeLut, 4, BLOCK, STACK, BATCH, 2>(a, s)
                            : launch_one<kModeLut, 6, BLOCK, STACK, BATCH, 2>(a, s);
        case SC_MASK_SPARSE:
            return a.R == 4 ? launch_one<kModeSparse, 4, BLOCK, STACK, BATCH, 2>(a, s)
                            : launch_one<kModeSparse, 6, BLOCK, STACK, BATCH, 2>(a, s);
        default: return hipErrorInvalidValue;
    }
}

template <int BLOCK, int STACK, bool BATCH, bool QUANT>
hipError_t launch_cfg4q(const TraceLaunch& a, hipStream_t s) {
    switch (a.mode) {
        case SC_MASK_NONE: return launch_one<kModeNone, 6, BLOCK, STACK, BATCH, 4, QUANT>(a, s);
        case SC_MASK_RAW:
            return a.R == 4 ? launch_one<kModeRaw, 4, BLOCK, STACK, BATCH, 4, QUANT>(a, s)
                            : launch_one<kModeRaw, 6, BLOCK, STACK, BATCH, 4, QUANT>(a, s);
        case SC_MASK_LUT:
            if constexpr (!BATCH) {
                // single scene: the 2-D bit table, or the codebook copied into LDS when it fits
                if (a.bit_table)
                    return a.R == 4 ? launch_one<kModeLutBits, 4, BLOCK, STACK, false, 4, QUANT>(a, s)
                                    : launch_one<kModeLutBits, 6, BLOCK, STACK, false, 4, QUANT>(a, s);
                if (!a.cb_global && (size_t)a.K * (a.R == 4 ? 1 : 4) <= kCbLdsWords)
                    return a.R == 4 ? launch_one<kModeLutLds, 4, BLOCK, STACK, false, 4, QUANT>(a, s)
                                    : launch_one<kModeLutLds, 6, BLOCK, STACK, false, 4, QUANT>(a, s);
            }
            return a.R == 4 ? launch_one<kModeLut, 4, BLOCK, STACK, BATCH, 4, QUANT>(a, s)
                            : launch_one<kModeLut, 6, BLOCK, STACK, BATCH, 4, QUANT>(a, s);
        default: return hipErrorInvalidValue;
    }
}

template <int BLOCK, int STACK, bool BATCH>
hipError_t launch_cfg4(const TraceLaunch& a, hipStream_t s) {
    return a.quant ? launch_cfg4q<BLOCK, STACK, BATCH, true>(a, s) : launch_cfg4q<BLOCK, STACK, BATCH, false>(a, s);
}

template <bool BATCH>
hipError_t launch_any(const TraceLaunch& a, hipStream_t s) {
    if (a.width == 4) {
        if (a.block == 256 && a.stack == 8) return launch_cfg4<256, 8, BATCH>(a, s);
        if (a.block == 128 && a.stack == 8) return launch_cfg4<128, 8, BATCH>(a, s);
        if (a.block == 256 && a.stack == 12) return launch_cfg4<256, 12, BATCH>(a, s);
        if (a.block == 256 && a.stack == 4) return launch_cfg4<256, 4, BATCH>(a, s);
        if (a.block == 128 && a.stack == 16) return launch_cfg4<128, 16, BATCH>(a, s);
        return hipErrorInvalidValue;
    }
    if (a.width != 2) return hipErrorInvalidValue;
    if (a.block == 256 && a.stack == 8) return launch_cfg<256, 8, BATCH>(a, s);
    if (a.block == 128 && a.stack == 8) return launch_cfg<128, 8, BATCH>(a, s);
    if (a.block == 256 && a.stack == 12) return launch_cfg<256, 12, BATCH>(a, s);
    if (a.block == 256 && a.stack == 4) return launch_cfg<256, 4, BATCH>(a, s);
    if (a.block == 128 && a.stack == 16) return launch_cfg<128, 16, BATCH>(a, s);
    return hipErrorInvalidValue;
}

}  // namespace

#if !SC_DEVICE_CHECKS
bool trace_config_supported(uint32_t block, uint32_t stack) {
    for (const auto& c : kTraceConfigs)
        if (c[0] == block && c[1] == stack) return true;
    return false;
}

#endif

#if SC_DEVICE_CHECKS
hipError_t launch_trace_checked(const TraceLaunch& a, hipStream_t s) {
#else
hipError_t launch_trace(const TraceLaunch& a, hipStream_t s) {
#endif
    if (a.n == 0) return hipSuccess;
    if (a.chunk < 1 || !a.queue || a.parts < 1 || a.parts > kQueueParts) return hipErrorInvalidValue;
    return a.items ? launch_any<true>(a, s) : launch_any<false>(a, s);
}

}  // namespace sc
