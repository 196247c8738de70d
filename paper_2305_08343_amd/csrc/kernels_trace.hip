// Traversal with subspace culling (Alg. 4 with Alg. 1 and the mask AND of
// Sect. 3.1.2) for gfx950.
//
// One lane per ray in wave64. Every ray runs the same canonical sequence as
// the plain reference traversal, so hits and the per-ray test counts are
// reproducible bit for bit:
//  slab test of child box [lo, hi]: per axis x, y, z
//      a = (lo - o) * inv, b = (hi - o) * inv, swap if a > b,
//      b = b * (1 + 3*2^-23) (robust far value), t0 = (a > t0) ? a : t0,
//      t1 = (b < t1) ? b : t1, from t0 = tmin, t1 = best_t; hit iff t0 <= t1
//  ray mask (Alg. 1): for p = o + t*d at t0 and at t1, per axis
//      s = R / (hi - lo) (0 if the extent is not positive or s is infinite),
//      u = (p - lo) * s clamped to [0, R-1] (NaN -> 0), cell = (int)u;
//      ray mask = LUT[(((((bx*R+by)*R+bz)*R+ex)*R+ey)*R+ez)]
//  culling: child survives iff (ray mask AND object mask) != 0; skipped for
//      rays whose max|o| exceeds the scene's origin bound
//  order: both children survive -> the one with the smaller t0 (tie: child
//      0) is visited next and the other pushed with its t0; a popped entry
//      with t0 > best_t is dropped
//  leaf: Moller-Trumbore, two-sided, det == 0 rejects; accept t in
//      [tmin, best_t]; replace iff t < best_t or (t == best_t and the
//      original id is lower)
// The next node of a lane is carried in registers instead of being pushed
// and popped (its pop test could never fail: its t0 <= best_t by the slab
// test), so the stack holds only postponed far children; it lives in LDS
// (kLdsStack entries per lane) and spills the rest to private memory.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace sc {
namespace {

constexpr int kBlock = 128;
constexpr int kLdsStack = 16;
constexpr uint32_t kModeNone = SC_MASK_NONE, kModeRaw = SC_MASK_RAW, kModeLut = SC_MASK_LUT,
                   kModeSparse = SC_MASK_SPARSE;

__device__ __forceinline__ float mx(float a, float b) { return (a > b) ? a : b; }

__device__ __forceinline__ bool ray_is_valid(float4 r0, float4 r1) {
    const bool fin = isfinite(r0.x) && isfinite(r0.y) && isfinite(r0.z) && isfinite(r0.w) &&
                     isfinite(r1.x) && isfinite(r1.y) && isfinite(r1.z);
    const bool dir = !(r1.x == 0.0f && r1.y == 0.0f && r1.z == 0.0f);
    return fin && dir && !isnan(r1.w) && (r0.w <= r1.w);
}

template <int R>
__device__ __forceinline__ int cell_of(float lo, float hi, float o, float d, float t) {
    const float ext = hi - lo;
    float s = (ext > 0.0f) ? (float)R / ext : 0.0f;
    if (isinf(s)) s = 0.0f;
    const float p = o + t * d;
    float u = (p - lo) * s;
    u = (u > 0.0f) ? u : 0.0f;
    u = (u < (float)(R - 1)) ? u : (float)(R - 1);
    return (int)u;
}

struct Ray {
    float ox, oy, oz, dx, dy, dz, ix, iy, iz, tmin;
};

template <int R>
__device__ __forceinline__ uint32_t lut_key(const float* lo, const float* hi, const Ray& r, float t0,
                                            float t1) {
    const int bx = cell_of<R>(lo[0], hi[0], r.ox, r.dx, t0);
    const int by = cell_of<R>(lo[1], hi[1], r.oy, r.dy, t0);
    const int bz = cell_of<R>(lo[2], hi[2], r.oz, r.dz, t0);
    const int ex = cell_of<R>(lo[0], hi[0], r.ox, r.dx, t1);
    const int ey = cell_of<R>(lo[1], hi[1], r.oy, r.dy, t1);
    const int ez = cell_of<R>(lo[2], hi[2], r.oz, r.dz, t1);
    return (uint32_t)(((((bx * R + by) * R + bz) * R + ex) * R + ey) * R + ez);
}

__device__ __forceinline__ void slab(const float* lo, const float* hi, const Ray& r, float tmax,
                                     float& t0, float& t1) {
    t0 = r.tmin;
    t1 = tmax;
    const float o[3] = {r.ox, r.oy, r.oz};
    const float inv[3] = {r.ix, r.iy, r.iz};
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        float a = (lo[j] - o[j]) * inv[j];
        float b = (hi[j] - o[j]) * inv[j];
        if (a > b) {
            const float t = a;
            a = b;
            b = t;
        }
        b = b * 0x1.000006p0f;
        t0 = (a > t0) ? a : t0;
        t1 = (b < t1) ? b : t1;
    }
}

// Loads the W words of a mask; the layout keeps every mask 8-byte aligned
// and, for W = 4, 32-byte aligned.
template <int W>
__device__ __forceinline__ void load_mask(const uint64_t* p, uint64_t* m) {
    if constexpr (W == 4) {
        const uint4 a = reinterpret_cast<const uint4*>(p)[0];
        const uint4 b = reinterpret_cast<const uint4*>(p)[1];
        m[0] = ((uint64_t)a.y << 32) | a.x;
        m[1] = ((uint64_t)a.w << 32) | a.z;
        m[2] = ((uint64_t)b.y << 32) | b.x;
        m[3] = ((uint64_t)b.w << 32) | b.z;
    } else {
#pragma unroll
        for (int w = 0; w < W; ++w) m[w] = p[w];
    }
}

template <uint32_t MODE, int R>
__global__ __launch_bounds__(kBlock) void trace_kernel(TraceLaunch a) {
    constexpr int W = (R * R * R + 63) / 64;
    constexpr uint32_t kStride = (MODE == kModeRaw) ? kRawNodeBytes : kNodeBytes;
    __shared__ uint2 lds_stack[kLdsStack * kBlock];

    const uint32_t tid = threadIdx.x;
    const uint32_t i = blockIdx.x * kBlock + tid;
    if (i >= a.n) return;
    const float4 r0 = reinterpret_cast<const float4*>(a.rays)[2 * (size_t)i];
    const float4 r1 = reinterpret_cast<const float4*>(a.rays)[2 * (size_t)i + 1];

    uint32_t box_tests = 0, tri_tests = 0, mask_tests = 0, mask_culls = 0;
    uint32_t best = kNoHit;
    float best_t = __builtin_inff();

    if (ray_is_valid(r0, r1) && a.root != kEmptyRef) {
        Ray r;
        r.ox = r0.x; r.oy = r0.y; r.oz = r0.z; r.tmin = r0.w;
        r.dx = r1.x; r.dy = r1.y; r.dz = r1.z;
        r.ix = 1.0f / r.dx; r.iy = 1.0f / r.dy; r.iz = 1.0f / r.dz;
        best_t = r1.w;
        bool use_mask = false;
        if constexpr (MODE != kModeNone) {
            use_mask = (a.flags & (SC_TRACE_CULL | SC_TRACE_SHADOW)) != 0 &&
                       !(mx(mx(fabsf(r.ox), fabsf(r.oy)), fabsf(r.oz)) > a.origin_bound);
        }
        const bool cull = (a.flags & SC_TRACE_CULL) != 0;
        const bool shadow = (a.flags & SC_TRACE_SHADOW) != 0 && a.slot_fp != nullptr;

        uint2 spill[kMaxDepth - kLdsStack + 1];
        int sp = 0;
        uint32_t ref = a.root;
        while (true) {
            if (ref & kLeafBit) {
                const uint32_t first = ref & 0x1FFFFFFFu;
                const uint32_t count = ((ref >> 29) & 3u) + 1u;
                for (uint32_t k = 0; k < count; ++k) {
                    ++tri_tests;
                    const float4* tp = reinterpret_cast<const float4*>(
                        reinterpret_cast<const unsigned char*>(a.tris) + (size_t)(first + k) * kTriBytes);
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
            } else {
                const unsigned char* np = a.nodes + (size_t)ref * kStride;
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
                            const bool hit = c ? h1 : h0;
                            if (!hit) continue;
                            const uint64_t* om;
                            if constexpr (MODE == kModeRaw) {
                                om = reinterpret_cast<const uint64_t*>(np + 64) + c * W;
                            } else if constexpr (MODE == kModeLut) {
                                const uint32_t idx = c ? (n3.z >> 16) : (n3.z & 0xFFFFu);
                                om = a.codebook + (size_t)idx * W;
                            } else {
                                const uint32_t ms = c ? n3.w : n3.z;
                                if (ms == kNoMask) continue;
                                om = a.side_masks + (size_t)ms * W;
                            }
                            ++mask_tests;
                            const uint32_t key = c ? lut_key<R>(lo1, hi1, r, t01, t11)
                                                   : lut_key<R>(lo0, hi0, r, t00, t10);
                            uint64_t rm[W], ob[W];
                            load_mask<W>(a.lut + (size_t)key * W, rm);
                            load_mask<W>(om, ob);
                            uint64_t any = 0;
#pragma unroll
                            for (int w = 0; w < W; ++w) any |= rm[w] & ob[w];
                            if (any == 0) {
                                ++mask_culls;
                                if (shadow) atomicAdd(&a.slot_fp[2 * (size_t)ref + c], 1u);
                                if (cull) {
                                    if (c) h1 = false;
                                    else h0 = false;
                                }
                            }
                        }
                    }
                }
                if (h0 && h1) {
                    const bool near1 = t01 < t00;
                    const uint32_t far_ref = near1 ? n3.x : n3.y;
                    const float far_t = near1 ? t00 : t01;
                    const uint2 e = make_uint2(far_ref, __float_as_uint(far_t));
                    if (sp < kLdsStack) lds_stack[sp * kBlock + tid] = e;
                    else spill[sp - kLdsStack] = e;
                    ++sp;
                    ref = near1 ? n3.y : n3.x;
                    continue;
                }
                if (h0) { ref = n3.x; continue; }
                if (h1) { ref = n3.y; continue; }
            }
            // pop, dropping entries that start beyond the current closest hit
            bool found = false;
            while (sp > 0) {
                --sp;
                const uint2 e = (sp < kLdsStack) ? lds_stack[sp * kBlock + tid] : spill[sp - kLdsStack];
                if (__uint_as_float(e.y) > best_t) continue;
                ref = e.x;
                found = true;
                break;
            }
            if (!found) break;
        }
    }
    const float tout = (best == kNoHit) ? __builtin_inff() : best_t;
    reinterpret_cast<uint4*>(a.hits)[i] = make_uint4(best, __float_as_uint(tout), box_tests, tri_tests);
    if (a.extra) reinterpret_cast<uint2*>(a.extra)[i] = make_uint2(mask_tests, mask_culls);
}

}  // namespace

hipError_t launch_trace(const TraceLaunch& a, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    const dim3 grid((a.n + kBlock - 1) / kBlock), block(kBlock);
    switch (a.mode) {
        case SC_MASK_NONE:
            hipLaunchKernelGGL((trace_kernel<kModeNone, 6>), grid, block, 0, s, a);
            break;
        case SC_MASK_RAW:
            if (a.R == 4) hipLaunchKernelGGL((trace_kernel<kModeRaw, 4>), grid, block, 0, s, a);
            else hipLaunchKernelGGL((trace_kernel<kModeRaw, 6>), grid, block, 0, s, a);
            break;
        case SC_MASK_LUT:
            if (a.R == 4) hipLaunchKernelGGL((trace_kernel<kModeLut, 4>), grid, block, 0, s, a);
            else hipLaunchKernelGGL((trace_kernel<kModeLut, 6>), grid, block, 0, s, a);
            break;
        case SC_MASK_SPARSE:
            if (a.R == 4) hipLaunchKernelGGL((trace_kernel<kModeSparse, 4>), grid, block, 0, s, a);
            else hipLaunchKernelGGL((trace_kernel<kModeSparse, 6>), grid, block, 0, s, a);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace sc
