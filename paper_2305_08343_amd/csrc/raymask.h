// Device helpers for ray masks (Alg. 1), shared by the build kernels and
// the traversal so that the exported LUT is produced by the traversal's own
// code path.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sc {

// Number of displacement patterns: dx in [0, R-1], dy, dz in [-(R-1), R-1].
template <int R>
constexpr int kPatterns = R * (2 * R - 1) * (2 * R - 1);

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

// m <<= k for a W-word little-endian bit string (k < 64*W; no set bit leaves it).
template <int W>
__device__ __forceinline__ void shift_left(uint64_t* m, uint32_t k) {
    if constexpr (W == 1) {
        m[0] <<= k;
    } else {
        static_assert(W == 4, "masks are one or four words");
        const uint32_t q = k >> 6, r = k & 63;
        if (q & 2) {
            m[3] = m[1]; m[2] = m[0]; m[1] = 0; m[0] = 0;
        }
        if (q & 1) {
            m[3] = m[2]; m[2] = m[1]; m[1] = m[0]; m[0] = 0;
        }
        if (r) {
            m[3] = (m[3] << r) | (m[2] >> (64 - r));
            m[2] = (m[2] << r) | (m[1] >> (64 - r));
            m[1] = (m[1] << r) | (m[0] >> (64 - r));
            m[0] = m[0] << r;
        }
    }
}

// Ray mask of the cell pair (b, e). The sweep that defines the LUT is
// invariant under translation and symmetric in its two cells, so the entry
// equals the pattern of the displacement e - b (x made non-negative by the
// symmetry) moved to the componentwise minimum corner, i.e. shifted left by
// that corner's bit index x + R*y + R^2*z. Patterns are stored with their
// minimum corner at the origin.
template <int R>
__device__ __forceinline__ void ray_mask_from_patterns(const uint64_t* pat, int bx, int by, int bz, int ex,
                                                       int ey, int ez, uint64_t* m) {
    constexpr int W = (R * R * R + 63) / 64;
    constexpr int S = 2 * R - 1;
    if (ex < bx) {
        int t = bx; bx = ex; ex = t;
        t = by; by = ey; ey = t;
        t = bz; bz = ez; ez = t;
    }
    const int pidx = ((ex - bx) * S + (ey - by + R - 1)) * S + (ez - bz + R - 1);
    const int my = by < ey ? by : ey, mz = bz < ez ? bz : ez;
    load_mask<W>(pat + (size_t)pidx * W, m);
    shift_left<W>(m, (uint32_t)(bx + R * my + R * R * mz));
}

}  // namespace sc
