// Build-time kernels for gfx950: ray-mask LUT, exact object masks,
// requirement LUTs, Alg. 3 compression and node packing.
//
// All float32 arithmetic follows the exact expression order stated at each
// kernel; the library is compiled with -ffp-contract=off so no product is
// fused into an add, and divisions are correctly rounded.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "raymask.h"

namespace sc {
namespace {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Ray masks (Sect. 3.1.1, Alg. 1). The LUT entry for cells (beg, end) holds
// voxel v iff a unit cell swept from cell beg to cell end overlaps v with
// positive volume at some time s in [0,1]: per axis the overlap times form
// the open interval between (v-1-beg)/D and (v+1-beg)/D (D = end-beg != 0),
// or all of [0,1] when D = 0 and v = beg. Times are scaled by 60 so every
// bound is an integer for R <= 6.
// ---------------------------------------------------------------------------
template <int R>
__device__ void sweep_mask(const int* beg, const int* end, uint64_t* m) {
    constexpr int W = (R * R * R + 63) / 64;
    constexpr int T = 60;
    constexpr int kBig = 1 << 20;
    int tlo[3][R], thi[3][R];
    bool ok[3][R];
    for (int i = 0; i < 3; ++i) {
        const int D = end[i] - beg[i];
        for (int v = 0; v < R; ++v) {
            if (D == 0) {
                ok[i][v] = (v == beg[i]);
                tlo[i][v] = -kBig;
                thi[i][v] = kBig;
            } else {
                const int a = T * (v - 1 - beg[i]) / D;
                const int b = T * (v + 1 - beg[i]) / D;
                tlo[i][v] = a < b ? a : b;
                thi[i][v] = a < b ? b : a;
                ok[i][v] = true;
            }
        }
    }
    for (int w = 0; w < W; ++w) m[w] = 0;
    for (int z = 0; z < R; ++z)
        for (int y = 0; y < R; ++y)
            for (int x = 0; x < R; ++x) {
                if (!(ok[0][x] && ok[1][y] && ok[2][z])) continue;
                int lo = tlo[0][x];
                lo = tlo[1][y] > lo ? tlo[1][y] : lo;
                lo = tlo[2][z] > lo ? tlo[2][z] : lo;
                int hi = thi[0][x];
                hi = thi[1][y] < hi ? thi[1][y] : hi;
                hi = thi[2][z] < hi ? thi[2][z] : hi;
                if (lo < hi && lo < T && hi > 0) {
                    const int bit = x + R * y + R * R * z;
                    m[bit >> 6] |= 1ull << (bit & 63);
                }
            }
}

// One thread per displacement (dx in [0,R-1], dy, dz in [-(R-1), R-1]):
// the sweep of the cell pair with that displacement whose minimum corner is
// the origin.
template <int R>
__global__ void raymask_pattern_kernel(uint64_t* __restrict__ out) {
    constexpr int W = (R * R * R + 63) / 64;
    constexpr int S = 2 * R - 1;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kPatterns<R>) return;
    const int D[3] = {p / (S * S), (p / S) % S - (R - 1), p % S - (R - 1)};
    int beg[3], end[3];
    for (int i = 0; i < 3; ++i) {
        beg[i] = D[i] < 0 ? -D[i] : 0;
        end[i] = beg[i] + D[i];
    }
    uint64_t m[W];
    sweep_mask<R>(beg, end, m);
    for (int w = 0; w < W; ++w) out[(size_t)p * W + w] = m[w];
}

// The full R^6 table, expanded through the traversal's own pattern lookup;
// key ((((bx*R+by)*R+bz)*R+ex)*R+ey)*R+ez.
template <int R>
__global__ void raymask_lut_kernel(const uint64_t* __restrict__ pat, uint64_t* __restrict__ out) {
    constexpr int R3 = R * R * R;
    constexpr int W = (R3 + 63) / 64;
    const int key = blockIdx.x * blockDim.x + threadIdx.x;
    if (key >= R3 * R3) return;
    const int kb = key / R3, ke = key % R3;
    uint64_t m[W];
    ray_mask_from_patterns<R>(pat, kb / (R * R), (kb / R) % R, kb % R, ke / (R * R), (ke / R) % R, ke % R, m);
    for (int w = 0; w < W; ++w) out[(size_t)key * W + w] = m[w];
}

// ---------------------------------------------------------------------------
// Triangle / voxel overlap: separating axis test on the triangle translated
// to the voxel centre c with half-size h (3 box normals, the 9 products of a
// box axis with an edge, the triangle normal). On each axis the three
// projected vertices are compared with +-r, r the box's projected radius;
// separated iff all three lie above r or all below -r.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float mn2(float a, float b) { return (a < b) ? a : b; }
__device__ __forceinline__ float mx2(float a, float b) { return (a > b) ? a : b; }
__device__ __forceinline__ bool outside(float p0, float p1, float p2, float r) {
    return mn2(mn2(p0, p1), p2) > r || mx2(mx2(p0, p1), p2) < -r;
}

__device__ __forceinline__ bool tri_voxel_overlap(const float* v, float cx, float cy, float cz,
                                                  const float* h) {
    const float ax = v[0] - cx, ay = v[1] - cy, az = v[2] - cz;
    const float bx = v[3] - cx, by = v[4] - cy, bz = v[5] - cz;
    const float qx = v[6] - cx, qy = v[7] - cy, qz = v[8] - cz;
    if (outside(ax, bx, qx, h[0]) || outside(ay, by, qy, h[1]) || outside(az, bz, qz, h[2]))
        return false;
    const float ex[3] = {bx - ax, qx - bx, ax - qx};
    const float ey[3] = {by - ay, qy - by, ay - qy};
    const float ez[3] = {bz - az, qz - bz, az - qz};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float fx = ex[k], fy = ey[k], fz = ez[k];
        float r = h[1] * fabsf(fz) + h[2] * fabsf(fy);
        if (outside(fy * az - fz * ay, fy * bz - fz * by, fy * qz - fz * qy, r)) return false;
        r = h[0] * fabsf(fz) + h[2] * fabsf(fx);
        if (outside(fz * ax - fx * az, fz * bx - fx * bz, fz * qx - fx * qz, r)) return false;
        r = h[0] * fabsf(fy) + h[1] * fabsf(fx);
        if (outside(fx * ay - fy * ax, fx * by - fy * bx, fx * qy - fy * qx, r)) return false;
    }
    const float nx = ey[0] * ez[1] - ez[0] * ey[1];
    const float ny = ez[0] * ex[1] - ex[0] * ez[1];
    const float nz = ex[0] * ey[1] - ey[0] * ex[1];
    const float r = (h[0] * fabsf(nx) + h[1] * fabsf(ny)) + h[2] * fabsf(nz);
    const float p0 = (nx * ax + ny * ay) + nz * az;
    const float p1 = (nx * bx + ny * by) + nz * bz;
    const float p2 = (nx * qx + ny * qy) + nz * qz;
    return !outside(p0, p1, p2, r);
}

// Voxels of box (lo, hi) that triangle v overlaps; voxel k on axis j has
// centre lo + (k + 0.5f) * w and half-size 0.5f * w + delta, w = (hi-lo)/R.
// Candidate voxels are those passing the box-normal tests of the same
// overlap test (separable per axis), so the result is the full test's.
template <int R>
__device__ void voxelize(const float* v, const float* lo, const float* hi, float delta,
                         uint64_t* bits) {
    float w[3], h[3];
    uint32_t pass[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        w[j] = (hi[j] - lo[j]) / (float)R;
        h[j] = 0.5f * w[j] + delta;
        pass[j] = 0;
        for (int k = 0; k < R; ++k) {
            const float c = lo[j] + ((float)k + 0.5f) * w[j];
            if (!outside(v[j] - c, v[3 + j] - c, v[6 + j] - c, h[j])) pass[j] |= 1u << k;
        }
    }
    for (uint32_t pz = pass[2]; pz; pz &= pz - 1) {
        const int z = __builtin_ctz(pz);
        const float cz = lo[2] + ((float)z + 0.5f) * w[2];
        for (uint32_t py = pass[1]; py; py &= py - 1) {
            const int y = __builtin_ctz(py);
            const float cy = lo[1] + ((float)y + 0.5f) * w[1];
            for (uint32_t px = pass[0]; px; px &= px - 1) {
                const int x = __builtin_ctz(px);
                const float cx = lo[0] + ((float)x + 0.5f) * w[0];
                if (tri_voxel_overlap(v, cx, cy, cz, h)) {
                    const int bit = x + R * y + R * R * z;
                    bits[bit >> 6] |= 1ull << (bit & 63);
                }
            }
        }
    }
}

__device__ __forceinline__ uint64_t shfl_down64(uint64_t x, int off) {
    const uint32_t lo = __shfl_down((uint32_t)x, off, kWave);
    const uint32_t hi = __shfl_down((uint32_t)(x >> 32), off, kWave);
    return ((uint64_t)hi << 32) | lo;
}

// ---------------------------------------------------------------------------
// Object masks from triangles (Sect. 3.2.1): one thread per triangle in leaf
// order. The thread walks from the root to its leaf; at every level it
// voxelizes its triangle into the child box that contains it. Threads of a
// wave hold consecutive triangles, so the lanes sharing a child slot are
// contiguous: a segmented OR across the wave leaves one value per slot, and
// the first lane of each segment ORs it into global memory. With levels = 0
// every slot on the path gets the triangle (the exact mask, L = infinity);
// with levels = L only the slots at most L levels above the triangle's leaf
// do (the triangle part of the approximation; the rest comes from fills).
// ---------------------------------------------------------------------------
template <int R>
__global__ __launch_bounds__(256) void object_mask_kernel(
    const float* __restrict__ tris, const uint32_t* __restrict__ perm, uint32_t n,
    const unsigned char* __restrict__ nodes, uint32_t stride, const uint32_t* __restrict__ range,
    uint32_t root, float delta, uint32_t levels, unsigned long long* __restrict__ masks) {
    constexpr int W = (R * R * R + 63) / 64;
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & (kWave - 1);
    bool active = (j < n) && !(root & kLeafBit);
    float v[9];
    if (active) {
        const float* src = tris + 9 * (size_t)perm[j];
#pragma unroll
        for (int k = 0; k < 9; ++k) v[k] = src[k];
    }
    // depth of the triangle's leaf slot (root children at depth 1)
    uint32_t leaf_depth = 0;
    if (active && levels > 0) {
        uint32_t nd = root;
        while (true) {
            const uint32_t* nu = reinterpret_cast<const uint32_t*>(nodes + (size_t)nd * stride);
            const uint32_t ref0 = nu[12];
            const uint32_t lcount = (ref0 & kLeafBit) ? ((ref0 >> 29) & 3u) + 1u : range[2 * (size_t)ref0 + 1];
            const int c = (j < range[2 * (size_t)nd] + lcount) ? 0 : 1;
            ++leaf_depth;
            const uint32_t ref = nu[12 + c];
            if (ref & kLeafBit) break;
            nd = ref;
        }
    }
    uint32_t depth = 0;
    uint32_t node = root;
    while (__ballot(active) != 0) {
        ++depth;
        uint32_t slot = 0xFFFFFFFFu;
        uint64_t bits[W];
#pragma unroll
        for (int w = 0; w < W; ++w) bits[w] = 0;
        uint32_t next = 0;
        bool leaf = true;
        if (active) {
            const float* nf = reinterpret_cast<const float*>(nodes + (size_t)node * stride);
            const uint32_t* nu = reinterpret_cast<const uint32_t*>(nf);
            const uint32_t ref0 = nu[12];
            const uint32_t lcount = (ref0 & kLeafBit) ? ((ref0 >> 29) & 3u) + 1u : range[2 * (size_t)ref0 + 1];
            const int c = (j < range[2 * (size_t)node] + lcount) ? 0 : 1;
            slot = 2u * node + (uint32_t)c;
            if (levels == 0 || depth + levels >= leaf_depth) voxelize<R>(v, nf + 6 * c, nf + 6 * c + 3, delta, bits);
            const uint32_t ref = nu[12 + c];
            leaf = (ref & kLeafBit) != 0;
            next = ref;
        }
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const uint32_t s2 = __shfl_down(slot, off, kWave);
#pragma unroll
            for (int w = 0; w < W; ++w) {
                const uint64_t b2 = shfl_down64(bits[w], off);
                if (lane + off < kWave && s2 == slot) bits[w] |= b2;
            }
        }
        const uint32_t prev = __shfl_up(slot, 1, kWave);
        if (slot != 0xFFFFFFFFu && (lane == 0 || prev != slot)) {
#pragma unroll
            for (int w = 0; w < W; ++w)
                if (bits[w]) atomicOr(&masks[(size_t)slot * W + w], (unsigned long long)bits[w]);
        }
        active = active && !leaf;
        node = next;
    }
}

// ---------------------------------------------------------------------------
// Approximate masks, fill part (Alg. 2): for each slot s of one depth whose
// node is inner, every inner node exactly L levels below contributes its own
// (already final) mask: a set child voxel fills the parent voxels its extent
// plus a 2 delta margin projects to (float64, floor, clamped to [0, R-1]; a
// parent axis of zero extent is filled whole). The box of voxels is built
// from bit runs instead of read from the filling-pattern table; both give
// the same bits. One thread per slot; slots of deeper levels are done first.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int clamp_floor(double u, int R) {
    const double f = floor(u);
    if (!(f > 0.0)) return 0;
    if (f > (double)(R - 1)) return R - 1;
    return (int)f;
}

template <int R>
__device__ void or_box(uint64_t* m, int x0, int y0, int z0, int x1, int y1, int z1) {
    const uint64_t row = ((1ull << (x1 + 1)) - 1ull) & ~((1ull << x0) - 1ull);
    for (int z = z0; z <= z1; ++z)
        for (int y = y0; y <= y1; ++y) {
            const int bit = R * y + R * R * z;
            const int w = bit >> 6, sh = bit & 63;
            m[w] |= row << sh;
            if (sh + R > 64) m[w + 1] |= row >> (64 - sh);
        }
}

template <int R>
__global__ __launch_bounds__(256) void approx_fill_kernel(const uint32_t* __restrict__ slots, uint32_t count,
                                                          const float* __restrict__ cbox,
                                                          const uint32_t* __restrict__ cref, uint32_t levels,
                                                          float delta, uint64_t* __restrict__ masks) {
    constexpr int W = (R * R * R + 63) / 64;
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    const uint32_t s = slots[t];
    const uint32_t r = cref[s];
    if (r & kLeafBit) return;
    const float* P = cbox + 6 * (size_t)s;
    uint64_t m[W];
#pragma unroll
    for (int w = 0; w < W; ++w) m[w] = 0;
    uint32_t st[65];
    uint32_t lev[65];
    int sp = 0;
    st[sp] = 2u * r + 1u; lev[sp] = 1; ++sp;
    st[sp] = 2u * r; lev[sp] = 1; ++sp;
    while (sp > 0) {
        --sp;
        const uint32_t d = st[sp], k = lev[sp];
        const uint32_t rd = cref[d];
        if (rd & kLeafBit) continue;  // its triangles came in the triangle part
        if (k < levels) {
            st[sp] = 2u * rd + 1u; lev[sp] = k + 1; ++sp;
            st[sp] = 2u * rd; lev[sp] = k + 1; ++sp;
            continue;
        }
        const float* Cb = cbox + 6 * (size_t)d;
        int lo_idx[3][R + 1], hi_idx[3][R + 1];
        for (int j = 0; j < 3; ++j) {
            const double pl = (double)P[j], pe = (double)P[3 + j] - (double)P[j];
            const double cl = (double)Cb[j], ce = (double)Cb[3 + j] - (double)Cb[j];
            for (int i = 0; i <= R; ++i) {
                if (!(pe > 0.0)) {
                    lo_idx[j][i] = 0;
                    hi_idx[j][i] = R - 1;
                    continue;
                }
                const double b = cl + ((double)i * ce) / (double)R;
                lo_idx[j][i] = clamp_floor(((double)R * ((b - 2.0 * (double)delta) - pl)) / pe, R);
                hi_idx[j][i] = clamp_floor(((double)R * ((b + 2.0 * (double)delta) - pl)) / pe, R);
            }
        }
        const uint64_t* cm = masks + (size_t)d * W;
        for (int w = 0; w < W; ++w) {
            for (uint64_t bits = cm[w]; bits; bits &= bits - 1) {
                const int bit = 64 * w + __builtin_ctzll(bits);
                const int x = bit % R, y = (bit / R) % R, z = bit / (R * R);
                or_box<R>(m, lo_idx[0][x], lo_idx[1][y], lo_idx[2][z], hi_idx[0][x + 1], hi_idx[1][y + 1],
                          hi_idx[2][z + 1]);
            }
        }
    }
#pragma unroll
    for (int w = 0; w < W; ++w) masks[(size_t)s * W + w] |= m[w];
}

// ---------------------------------------------------------------------------
// Requirement LUTs (Sect. 3.2.3): table i, row p, word w has bit b set iff
// codebook entry k = 64w + b contains every bit of p in its chunk i (mask
// bits [8i, 8i+8)). One thread per (table, row, word).
// ---------------------------------------------------------------------------
__global__ void req_lut_kernel(const uint64_t* __restrict__ cb, uint32_t K, uint32_t W,
                               uint32_t nch, uint64_t* __restrict__ req) {
    const uint32_t KW = K / 64;
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (size_t)nch * 256 * KW) return;
    const uint32_t w = gid % KW;
    const uint32_t p = (gid / KW) % 256;
    const uint32_t i = (uint32_t)(gid / ((size_t)KW * 256));
    const uint32_t bit = 8 * i;
    uint64_t out = 0;
    for (uint32_t b = 0; b < 64; ++b) {
        const uint32_t k = 64 * w + b;
        const uint32_t chunk = (uint32_t)((cb[(size_t)k * W + (bit >> 6)] >> (bit & 63)) & 0xFFu);
        if ((chunk & p) == p) out |= 1ull << b;
    }
    req[gid] = out;
}

// ---------------------------------------------------------------------------
// Alg. 3 (Sect. 3.2.3): one wave per mask; lane l owns the 64 codebook
// entries of word l. The rows picked by the mask's 8-bit chunks are ANDed,
// the first lane with a non-zero word is found by a ballot, and its lowest
// set bit is the index of the tightest conservative entry.
// ---------------------------------------------------------------------------
template <int R>
__global__ __launch_bounds__(256) void compress_kernel(const uint64_t* __restrict__ masks, uint32_t n,
                                                       const uint64_t* __restrict__ req, uint32_t K,
                                                       uint16_t* __restrict__ idx) {
    constexpr int W = (R * R * R + 63) / 64;
    constexpr int NCH = (R * R * R + 7) / 8;
    const uint32_t KW = K / 64;
    const size_t wave = ((size_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint32_t lane = threadIdx.x & (kWave - 1);
    if (wave >= n) return;
    uint64_t m[W];
#pragma unroll
    for (int w = 0; w < W; ++w) m[w] = masks[wave * W + w];
    uint64_t acc = ~0ull;
    if (lane < KW) {
#pragma unroll
        for (int i = 0; i < NCH; ++i) {
            const uint32_t bit = 8 * i;
            const uint32_t p = (uint32_t)((m[bit >> 6] >> (bit & 63)) & 0xFFu);
            acc &= req[((size_t)i * 256 + p) * KW + lane];
        }
    }
    const uint64_t nz = __ballot(lane < KW && acc != 0);
    if (nz == 0) {
        if (lane == 0) idx[wave] = 0xFFFFu;
        return;
    }
    const int first = __builtin_ctzll(nz);
    const uint32_t lo = __shfl((uint32_t)acc, first, kWave);
    const uint32_t hi = __shfl((uint32_t)(acc >> 32), first, kWave);
    const uint64_t word = ((uint64_t)hi << 32) | lo;
    if (lane == 0) idx[wave] = (uint16_t)(first * 64 + __builtin_ctzll(word));
}

// Copy each inner node's two raw masks into bytes [64, 64 + 2*W*8) of its
// 128-byte node, and set bit c of the node's aux word when child c's mask has
// more than test_max set bits (a full mask at the default R^3 - 1: it can never
// cull), so the traversal skips its test.
template <int R>
__global__ void pack_raw_kernel(const uint64_t* __restrict__ masks, uint32_t n_inner, uint32_t test_max,
                                unsigned char* __restrict__ nodes) {
    constexpr int W = (R * R * R + 63) / 64;
    const size_t node = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (node >= n_inner) return;
    uint32_t flags = 0;
    uint64_t* dst = reinterpret_cast<uint64_t*>(nodes + node * kRawNodeBytes + 64);
    for (int c = 0; c < 2; ++c) {
        int pc = 0;
        for (int w = 0; w < W; ++w) {
            const uint64_t m = masks[(node * 2 + c) * W + w];
            dst[c * W + w] = m;
            pc += __popcll(m);
        }
        if ((uint32_t)pc > test_max) flags |= 1u << c;
    }
    reinterpret_cast<uint32_t*>(nodes + node * kRawNodeBytes)[14] = flags;
}

__global__ void pack_lut_kernel(const uint16_t* __restrict__ idx, uint32_t n_inner,
                                unsigned char* __restrict__ nodes) {
    const size_t node = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (node >= n_inner) return;
    const uint32_t v = (uint32_t)idx[2 * node] | ((uint32_t)idx[2 * node + 1] << 16);
    reinterpret_cast<uint32_t*>(nodes + node * kNodeBytes)[14] = v;
}

// 4-wide node m, child c from binary slot src4[4m + c]: the raw mask goes to
// masks4[4m + c] and bit c of aux word 0 (byte 112) and bit 28 of the child's ref
// mark a mask with more than test_max set bits (untested); a codebook index goes
// to the 16-bit aux entry c.
template <int R>
__global__ void pack4_kernel(uint32_t mode, const uint32_t* __restrict__ src4, uint32_t n4,
                             const uint64_t* __restrict__ masks, const uint16_t* __restrict__ cidx,
                             uint32_t test_max, unsigned char* __restrict__ nodes4, uint64_t* __restrict__ masks4,
                             uint32_t stride, uint32_t refs_at, uint32_t aux_at) {
    constexpr int W = (R * R * R + 63) / 64;
    const size_t m = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n4) return;
    uint32_t* aux = reinterpret_cast<uint32_t*>(nodes4 + m * stride + aux_at);
    uint32_t full = 0, idx01 = 0, idx23 = 0;
    for (int c = 0; c < 4; ++c) {
        const uint32_t s = src4[4 * m + c];
        if (s == kEmptyRef) continue;
        if (mode == SC_MASK_RAW) {
            int pc = 0;
            for (int w = 0; w < W; ++w) {
                const uint64_t v = masks[(size_t)s * W + w];
                masks4[(4 * m + c) * W + w] = v;
                pc += __popcll(v);
            }
            if ((uint32_t)pc > test_max) full |= 1u << c;
        } else {
            const uint32_t v = cidx[s];
            if (c < 2) idx01 |= v << (16 * c);
            else idx23 |= v << (16 * (c - 2));
        }
    }
    aux[0] = (mode == SC_MASK_RAW) ? full : idx01;
    aux[1] = (mode == SC_MASK_RAW) ? 0u : idx23;
    if (mode == SC_MASK_RAW) {
        // the full flags again in the refs (bit 28), where the traversal reads them
        uint32_t* refs = reinterpret_cast<uint32_t*>(nodes4 + m * stride + refs_at);
        for (int c = 0; c < 4; ++c)
            if (((full >> c) & 1u) && refs[c] != kEmptyRef) refs[c] |= kRef4Full;
    }
}

// 2-D bit table (Sect. 3.2.2), stored by unordered cell pair (bit_row): one thread per (row,
// 32 codebook entries); the row of cells lo <= hi reads the LUT entry of key lo * R^3 + hi.
template <int R>
__global__ __launch_bounds__(256) void bit_table_kernel(const uint64_t* __restrict__ lut,
                                                        const uint64_t* __restrict__ cb, uint32_t K,
                                                        uint32_t* __restrict__ out) {
    constexpr int W = (R * R * R + 63) / 64;
    constexpr uint32_t kCells = R * R * R;
    const uint32_t kw = K / 32;
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (size_t)kBitRows<R> * kw) return;
    const uint32_t row = (uint32_t)(gid / kw);
    const uint32_t w = (uint32_t)(gid % kw);
    // hi: the largest h with h (h + 1) / 2 <= row (a float guess, then exact integer steps)
    uint32_t hi = (uint32_t)((sqrtf(8.0f * (float)row + 1.0f) - 1.0f) * 0.5f);
    while (hi > 0 && ((hi * (hi + 1u)) >> 1) > row) --hi;
    while ((((hi + 1u) * (hi + 2u)) >> 1) <= row) ++hi;
    const uint32_t lo = row - ((hi * (hi + 1u)) >> 1);
    const size_t key = (size_t)lo * kCells + hi;
    uint64_t rm[W];
#pragma unroll
    for (int q = 0; q < W; ++q) rm[q] = lut[key * W + q];
    uint32_t word = 0;
    for (uint32_t b = 0; b < 32; ++b) {
        const uint64_t* e = cb + (size_t)(32 * w + b) * W;
        uint64_t any = 0;
#pragma unroll
        for (int q = 0; q < W; ++q) any |= rm[q] & e[q];
        if (any) word |= 1u << b;
    }
    out[gid] = word;
}

// Slot s = 2*node + c keeps its mask only when child c is a leaf; an inner child's
// slot gets the full mask (all R^3 bits), which no traversal tests.
template <int R>
__global__ void full_inner_slots_kernel(const unsigned char* __restrict__ nodes, uint32_t stride, uint32_t n_inner,
                                        uint64_t* __restrict__ masks) {
    constexpr int W = (R * R * R + 63) / 64;
    const size_t s = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= 2 * (size_t)n_inner) return;
    const uint32_t ref = reinterpret_cast<const uint32_t*>(nodes + (s >> 1) * stride + 48)[s & 1];
    if ((ref & kLeafBit) || ref == kEmptyRef) return;
    for (int w = 0; w < W; ++w) {
        const int bits = R * R * R - 64 * w;
        masks[s * W + w] = bits >= 64 ? ~0ull : ((1ull << bits) - 1ull);
    }
}

inline unsigned blocks_for(size_t n, unsigned b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

hipError_t launch_raymask_patterns(uint32_t R, uint64_t* patterns, hipStream_t s) {
    if (R == 4) hipLaunchKernelGGL(raymask_pattern_kernel<4>, dim3(blocks_for(kPatterns<4>, 64)), dim3(64), 0, s, patterns);
    else if (R == 6) hipLaunchKernelGGL(raymask_pattern_kernel<6>, dim3(blocks_for(kPatterns<6>, 64)), dim3(64), 0, s, patterns);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_raymask_lut(uint32_t R, const uint64_t* patterns, uint64_t* out, hipStream_t s) {
    const size_t n = (size_t)R * R * R * R * R * R;
    if (R == 4) hipLaunchKernelGGL(raymask_lut_kernel<4>, dim3(blocks_for(n, 256)), dim3(256), 0, s, patterns, out);
    else if (R == 6) hipLaunchKernelGGL(raymask_lut_kernel<6>, dim3(blocks_for(n, 256)), dim3(256), 0, s, patterns, out);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_object_masks(uint32_t R, const float* tris_orig, const uint32_t* perm, uint32_t n,
                               const unsigned char* nodes, uint32_t node_stride,
                               const uint32_t* range, uint32_t root, float delta, uint32_t levels,
                               uint64_t* masks, hipStream_t s) {
    if (n == 0) return hipSuccess;
    auto* m = reinterpret_cast<unsigned long long*>(masks);
    if (R == 4)
        hipLaunchKernelGGL(object_mask_kernel<4>, dim3(blocks_for(n, 256)), dim3(256), 0, s, tris_orig,
                           perm, n, nodes, node_stride, range, root, delta, levels, m);
    else if (R == 6)
        hipLaunchKernelGGL(object_mask_kernel<6>, dim3(blocks_for(n, 256)), dim3(256), 0, s, tris_orig,
                           perm, n, nodes, node_stride, range, root, delta, levels, m);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_approx_fill(uint32_t R, const uint32_t* slots, uint32_t count, const float* cbox,
                              const uint32_t* cref, uint32_t levels, float delta, uint64_t* masks, hipStream_t s) {
    if (count == 0) return hipSuccess;
    if (levels < 1 || levels > 64) return hipErrorInvalidValue;
    if (R == 4)
        hipLaunchKernelGGL(approx_fill_kernel<4>, dim3(blocks_for(count, 256)), dim3(256), 0, s, slots, count, cbox,
                           cref, levels, delta, masks);
    else if (R == 6)
        hipLaunchKernelGGL(approx_fill_kernel<6>, dim3(blocks_for(count, 256)), dim3(256), 0, s, slots, count, cbox,
                           cref, levels, delta, masks);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_req_luts(uint32_t R, const uint64_t* cb, uint32_t K, uint64_t* req, hipStream_t s) {
    const uint32_t W = words_for(R), nch = (R * R * R + 7) / 8;
    const size_t n = (size_t)nch * 256 * (K / 64);
    hipLaunchKernelGGL(req_lut_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, cb, K, W, nch, req);
    return hipGetLastError();
}

hipError_t launch_compress(uint32_t R, const uint64_t* masks, uint32_t n, const uint64_t* req,
                           uint32_t K, uint16_t* idx, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const size_t threads = (size_t)n * kWave;
    if (R == 4)
        hipLaunchKernelGGL(compress_kernel<4>, dim3(blocks_for(threads, 256)), dim3(256), 0, s, masks, n,
                           req, K, idx);
    else if (R == 6)
        hipLaunchKernelGGL(compress_kernel<6>, dim3(blocks_for(threads, 256)), dim3(256), 0, s, masks, n,
                           req, K, idx);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_pack_raw(uint32_t R, const uint64_t* masks, uint32_t n_inner, uint32_t test_max,
                           unsigned char* nodes, hipStream_t s) {
    if (n_inner == 0) return hipSuccess;
    if (R == 4)
        hipLaunchKernelGGL(pack_raw_kernel<4>, dim3(blocks_for(n_inner, 256)), dim3(256), 0, s, masks, n_inner,
                           test_max, nodes);
    else if (R == 6)
        hipLaunchKernelGGL(pack_raw_kernel<6>, dim3(blocks_for(n_inner, 256)), dim3(256), 0, s, masks, n_inner,
                           test_max, nodes);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_full_inner_slots(uint32_t R, const unsigned char* nodes, uint32_t stride, uint32_t n_inner,
                                   uint64_t* masks, hipStream_t s) {
    if (n_inner == 0) return hipSuccess;
    const size_t S = 2 * (size_t)n_inner;
    if (R == 4)
        hipLaunchKernelGGL(full_inner_slots_kernel<4>, dim3(blocks_for(S, 256)), dim3(256), 0, s, nodes, stride,
                           n_inner, masks);
    else if (R == 6)
        hipLaunchKernelGGL(full_inner_slots_kernel<6>, dim3(blocks_for(S, 256)), dim3(256), 0, s, nodes, stride,
                           n_inner, masks);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_pack4(uint32_t mode, uint32_t R, const uint32_t* src4, uint32_t n4, const uint64_t* masks,
                        const uint16_t* cidx, uint32_t test_max, unsigned char* nodes4, uint64_t* masks4,
                        uint32_t quant, hipStream_t s) {
    if (n4 == 0) return hipSuccess;
    if (mode != SC_MASK_RAW && mode != SC_MASK_LUT) return hipErrorInvalidValue;
    const uint32_t stride = quant ? kNode4QBytes : kNode4Bytes;
    const uint32_t refs_at = quant ? kNode4QRefs : 96u, aux_at = quant ? kNode4QAux : 112u;
    if (R == 4)
        hipLaunchKernelGGL(pack4_kernel<4>, dim3(blocks_for(n4, 256)), dim3(256), 0, s, mode, src4, n4, masks, cidx,
                           test_max, nodes4, masks4, stride, refs_at, aux_at);
    else if (R == 6)
        hipLaunchKernelGGL(pack4_kernel<6>, dim3(blocks_for(n4, 256)), dim3(256), 0, s, mode, src4, n4, masks, cidx,
                           test_max, nodes4, masks4, stride, refs_at, aux_at);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_bit_table(uint32_t R, const uint64_t* lut, const uint64_t* cb, uint32_t K, uint32_t* out,
                            hipStream_t s) {
    if (K == 0 || K % 32) return hipErrorInvalidValue;
    const size_t n = (size_t)(R == 4 ? kBitRows<4> : kBitRows<6>) * (K / 32);
    if (R == 4) hipLaunchKernelGGL(bit_table_kernel<4>, dim3(blocks_for(n, 256)), dim3(256), 0, s, lut, cb, K, out);
    else if (R == 6) hipLaunchKernelGGL(bit_table_kernel<6>, dim3(blocks_for(n, 256)), dim3(256), 0, s, lut, cb, K, out);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_pack_lut(const uint16_t* idx, uint32_t n_inner, unsigned char* nodes, hipStream_t s) {
    if (n_inner == 0) return hipSuccess;
    hipLaunchKernelGGL(pack_lut_kernel, dim3(blocks_for(n_inner, 256)), dim3(256), 0, s, idx, n_inner, nodes);
    return hipGetLastError();
}

}  // namespace sc
