// Learned mask placement on gfx950: per-slot features, a small MLP
// (12 -> 64 -> 64 -> 1, ReLU) with forward, backward and Adam kernels, and
// the prefix scan the features use.
//
// The MLP predicts, from a child slot's geometry, how many false-positive
// box hits its object mask would remove (the would-be culls of the shadow
// trace). Masks are then placed on the slots with the highest predictions
// under a memory budget; a slot without a mask is traversed as in plain
// BVH traversal, so any placement keeps the exact hits.
//
// Parameter layout (5,057 floats): W1 [64][12], b1 [64], W2 [64][64],
// b2 [64], W3 [64], b3.
// All reductions over the batch run in a fixed order (one thread per
// parameter summing samples in index order), so training is deterministic.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace sc {
namespace {

constexpr int kIn = 12, kHid = 64;
constexpr int oW1 = 0, oB1 = oW1 + kHid * kIn, oW2 = oB1 + kHid, oB2 = oW2 + kHid * kHid, oW3 = oB2 + kHid,
              oB3 = oW3 + kHid;
static_assert(oB3 + 1 == kMlpParams, "parameter layout");

inline unsigned blocks_for(size_t n, unsigned b) { return (unsigned)((n + b - 1) / b); }

// ---------------------------------------------------------------- features
// Per triangle (leaf order, from the traversal's records v0, e1 = v1 - v0,
// e2 = v2 - v0): thinness 1 - 4*sqrt(3)*area / (sum of squared edge
// lengths), 0 for an equilateral triangle, 1 when degenerate.
__global__ void tri_shape_kernel(const float* __restrict__ rec, uint32_t n, double* __restrict__ out /*[n]*/) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float* r = rec + 12 * (size_t)i;
    float e[3][3];
    for (int j = 0; j < 3; ++j) {
        e[0][j] = r[3 + j];              // v1 - v0
        e[1][j] = r[6 + j] - r[3 + j];   // v2 - v1
        e[2][j] = -r[6 + j];             // v0 - v2
    }
    float l2[3];
    for (int k = 0; k < 3; ++k) l2[k] = e[k][0] * e[k][0] + e[k][1] * e[k][1] + e[k][2] * e[k][2];
    const float cx = e[0][1] * e[1][2] - e[0][2] * e[1][1];
    const float cy = e[0][2] * e[1][0] - e[0][0] * e[1][2];
    const float cz = e[0][0] * e[1][1] - e[0][1] * e[1][0];
    const float area = 0.5f * sqrtf(cx * cx + cy * cy + cz * cz);
    const float s = l2[0] + l2[1] + l2[2];
    const float thin = (s > 0.0f) ? 1.0f - 4.0f * 1.7320508075688772f * area / s : 1.0f;
    out[i] = fminf(fmaxf(thin, 0.0f), 1.0f);
}

// Inclusive prefix sums of `rows` arrays of n doubles, in place, three
// passes with a fixed summation order: block sums, a single-block scan of
// the block sums, then each block's local scan plus its offset.
constexpr int kScanBlock = 256, kScanItems = 8, kScanTile = kScanBlock * kScanItems;

__global__ void scan_block_sums(const double* __restrict__ a, uint32_t n, double* __restrict__ sums) {
    const uint32_t row = blockIdx.y;
    const double* x = a + (size_t)row * n;
    __shared__ double part[kScanBlock];
    const size_t base = (size_t)blockIdx.x * kScanTile + (size_t)threadIdx.x * kScanItems;
    double acc = 0.0;
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < n) acc += x[base + k];
    part[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < kScanBlock; ++k) t += part[k];
        sums[(size_t)row * gridDim.x + blockIdx.x] = t;
    }
}

__global__ void scan_sums_exclusive(double* __restrict__ sums, uint32_t nb) {
    const uint32_t row = blockIdx.x;
    if (threadIdx.x != 0) return;
    double t = 0.0;
    for (uint32_t b = 0; b < nb; ++b) {
        const double v = sums[(size_t)row * nb + b];
        sums[(size_t)row * nb + b] = t;
        t += v;
    }
}

__global__ void scan_apply(double* __restrict__ a, uint32_t n, const double* __restrict__ sums) {
    const uint32_t row = blockIdx.y;
    double* x = a + (size_t)row * n;
    __shared__ double part[kScanBlock];
    const size_t base = (size_t)blockIdx.x * kScanTile + (size_t)threadIdx.x * kScanItems;
    double loc[kScanItems];
    double acc = 0.0;
    for (int k = 0; k < kScanItems; ++k) {
        const double v = (base + k < n) ? x[base + k] : 0.0;
        acc += v;
        loc[k] = acc;
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {  // exclusive scan of the thread totals, fixed order
        double t = sums[(size_t)row * gridDim.x + blockIdx.x];
        for (int k = 0; k < kScanBlock; ++k) {
            const double v = part[k];
            part[k] = t;
            t += v;
        }
    }
    __syncthreads();
    const double off = part[threadIdx.x];
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < n) x[base + k] = off + loc[k];
}

__device__ __forceinline__ double box_area(const float* lo, const float* hi) {
    const double dx = (double)hi[0] - lo[0], dy = (double)hi[1] - lo[1], dz = (double)hi[2] - lo[2];
    return 2.0 * ((dx * dy + dy * dz) + dz * dx);
}

// 12 features per child slot s = 2*node + c (see the header for the list).
template <int W>
__global__ void slot_feature_kernel(const unsigned char* __restrict__ nodes, uint32_t stride,
                                    const uint32_t* __restrict__ range, const uint8_t* __restrict__ depth,
                                    uint32_t max_depth, const uint64_t* __restrict__ masks, uint32_t R3,
                                    const double* __restrict__ prefix /*[n] inclusive*/, RootBox root,
                                    uint32_t n_inner, float* __restrict__ out) {
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= 2 * n_inner) return;
    const uint32_t node = s >> 1, c = s & 1;
    const float* nb = reinterpret_cast<const float*>(nodes + (size_t)node * stride);
    const uint32_t ref = reinterpret_cast<const uint32_t*>(nb)[12 + c];
    const float* lo = nb + 6 * c;
    const float* hi = lo + 3;
    float plo[3], phi[3];
    for (int j = 0; j < 3; ++j) {
        plo[j] = fminf(nb[j], nb[6 + j]);
        phi[j] = fmaxf(nb[3 + j], nb[9 + j]);
    }
    float* f = out + (size_t)s * 12;
    for (int j = 0; j < 3; ++j) {
        const float pe = phi[j] - plo[j];
        f[j] = (pe > 0.0f) ? (hi[j] - lo[j]) / pe : 0.0f;
    }
    const double ratio = box_area(lo, hi) / root.area;
    f[3] = (float)(log2(fmax(ratio, 0x1p-40)) / 32.0);
    f[4] = (float)depth[node] / (float)max_depth;
    uint32_t first, count;
    if (ref & kLeafBit) {
        first = ref & 0x1FFFFFFFu;
        count = ((ref >> 29) & 3u) + 1u;
    } else {
        first = range[2 * (size_t)ref];
        count = range[2 * (size_t)ref + 1];
    }
    f[5] = (float)(log2(1.0 + (double)count) / 24.0);
    int pc = 0;
    for (int w = 0; w < W; ++w) pc += __popcll(masks[(size_t)s * W + w]);
    f[6] = (float)pc / (float)R3;
    const double sum = prefix[first + count - 1] - (first ? prefix[first - 1] : 0.0);
    f[7] = (float)(sum / (double)count);
    // where the child sits in the scene: its box centre relative to the root box
    for (int j = 0; j < 3; ++j) {
        const double ext = root.hi[j] - root.lo[j];
        const double mid = ((double)lo[j] + (double)hi[j]) * 0.5;
        f[8 + j] = (ext > 0.0) ? (float)((mid - root.lo[j]) / ext) : 0.0f;
    }
    f[11] = (ref & kLeafBit) ? 1.0f : 0.0f;
}

// ---------------------------------------------------------------- the MLP
// act [n][128]: z1 (pre-activation of layer 1) then z2 (layer 2).
__global__ __launch_bounds__(256) void mlp_forward_kernel(const float* __restrict__ prm, const float* __restrict__ x,
                                                          uint32_t n, float* __restrict__ y, float* __restrict__ act) {
    __shared__ float w[kMlpParams];
    for (int k = threadIdx.x; k < kMlpParams; k += blockDim.x) w[k] = prm[k];
    __syncthreads();
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    float xin[kIn], h1[kHid];
    for (int q = 0; q < kIn; ++q) xin[q] = x[(size_t)s * kIn + q];
    for (int k = 0; k < kHid; ++k) {
        float z = w[oB1 + k];
        for (int q = 0; q < kIn; ++q) z += w[oW1 + k * kIn + q] * xin[q];
        if (act) act[(size_t)s * 128 + k] = z;
        h1[k] = z > 0.0f ? z : 0.0f;
    }
    float out = w[oB3];
    for (int j = 0; j < kHid; ++j) {
        float z = w[oB2 + j];
        for (int k = 0; k < kHid; ++k) z += w[oW2 + j * kHid + k] * h1[k];
        if (act) act[(size_t)s * 128 + 64 + j] = z;
        out += w[oW3 + j] * (z > 0.0f ? z : 0.0f);
    }
    y[s] = out;
}

// Per sample: dy = 2 (y - t) / n, dz2 = dy W3 [z2 > 0], dz1 = (dz2 W2) [z1 > 0].
// delta [n][128] = dz1, dz2; dyv [n].
__global__ __launch_bounds__(256) void mlp_delta_kernel(const float* __restrict__ prm, const float* __restrict__ act,
                                                        const float* __restrict__ y, const float* __restrict__ t,
                                                        uint32_t n, float* __restrict__ delta,
                                                        float* __restrict__ dyv, float* __restrict__ sqerr) {
    __shared__ float w[kMlpParams];
    for (int k = threadIdx.x; k < kMlpParams; k += blockDim.x) w[k] = prm[k];
    __syncthreads();
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const float e = y[s] - t[s];
    const float dy = 2.0f * e / (float)n;
    dyv[s] = dy;
    sqerr[s] = e * e;
    float dz2[kHid];
    for (int j = 0; j < kHid; ++j) {
        dz2[j] = act[(size_t)s * 128 + 64 + j] > 0.0f ? dy * w[oW3 + j] : 0.0f;
        delta[(size_t)s * 128 + 64 + j] = dz2[j];
    }
    for (int k = 0; k < kHid; ++k) {
        float d = 0.0f;
        for (int j = 0; j < kHid; ++j) d += dz2[j] * w[oW2 + j * kHid + k];
        delta[(size_t)s * 128 + k] = act[(size_t)s * 128 + k] > 0.0f ? d : 0.0f;
    }
}

// One thread per (parameter, range of samples): the samples of range blockIdx.y (SC_MLP_GRAD_PARTS
// contiguous ranges) summed in index order into part[range][parameter].
__global__ void mlp_grad_kernel(const float* __restrict__ x, const float* __restrict__ act,
                                const float* __restrict__ delta, const float* __restrict__ dyv, uint32_t n,
                                float* __restrict__ part) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kMlpParams) return;
    const uint32_t r = blockIdx.y;
    const uint32_t s0 = (uint32_t)(((uint64_t)n * r) / SC_MLP_GRAD_PARTS);
    const uint32_t s1 = (uint32_t)(((uint64_t)n * (r + 1)) / SC_MLP_GRAD_PARTS);
    float g = 0.0f;
    if (p < oB1) {
        const int k = p / kIn, q = p % kIn;
        for (uint32_t s = s0; s < s1; ++s) g += delta[(size_t)s * 128 + k] * x[(size_t)s * kIn + q];
    } else if (p < oW2) {
        const int k = p - oB1;
        for (uint32_t s = s0; s < s1; ++s) g += delta[(size_t)s * 128 + k];
    } else if (p < oB2) {
        const int j = (p - oW2) / kHid, k = (p - oW2) % kHid;
        for (uint32_t s = s0; s < s1; ++s) {
            const float z1 = act[(size_t)s * 128 + k];
            g += delta[(size_t)s * 128 + 64 + j] * (z1 > 0.0f ? z1 : 0.0f);
        }
    } else if (p < oW3) {
        const int j = p - oB2;
        for (uint32_t s = s0; s < s1; ++s) g += delta[(size_t)s * 128 + 64 + j];
    } else if (p < oB3) {
        const int j = p - oW3;
        for (uint32_t s = s0; s < s1; ++s) {
            const float z2 = act[(size_t)s * 128 + 64 + j];
            g += dyv[s] * (z2 > 0.0f ? z2 : 0.0f);
        }
    } else {
        for (uint32_t s = s0; s < s1; ++s) g += dyv[s];
    }
    part[(size_t)r * kMlpParams + p] = g;
}

// grad[p] = the ranges' partial sums, added in range order
__global__ void mlp_grad_sum_kernel(const float* __restrict__ part, float* __restrict__ grad) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kMlpParams) return;
    float g = 0.0f;
    for (int r = 0; r < SC_MLP_GRAD_PARTS; ++r) g += part[(size_t)r * kMlpParams + p];
    grad[p] = g;
}

// mean of v[n] in float64: thread t adds samples t, t + 256, ... in order, then a fixed pairwise tree
constexpr int kSumThreads = 256;
__global__ __launch_bounds__(kSumThreads) void sum_kernel(const float* __restrict__ v, uint32_t n,
                                                          float* __restrict__ out) {
    __shared__ double acc[kSumThreads];
    double t = 0.0;
    for (uint32_t s = threadIdx.x; s < n; s += kSumThreads) t += v[s];
    acc[threadIdx.x] = t;
    __syncthreads();
    for (int w = kSumThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) acc[threadIdx.x] += acc[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = (float)(acc[0] / (double)(n ? n : 1));
}

// Adam (Kingma & Ba 2015); bc1 = 1 - beta1^step, bc2 = 1 - beta2^step.
__global__ void adam_kernel(float* __restrict__ prm, const float* __restrict__ grad, float* __restrict__ m,
                            float* __restrict__ v, float lr, float b1, float b2, float eps, float bc1, float bc2) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kMlpParams) return;
    const float g = grad[p];
    const float mm = b1 * m[p] + (1.0f - b1) * g;
    const float vv = b2 * v[p] + (1.0f - b2) * g * g;
    m[p] = mm;
    v[p] = vv;
    prm[p] -= lr * (mm / bc1) / (sqrtf(vv / bc2) + eps);
}

}  // namespace

hipError_t launch_tri_shape(const float* rec, uint32_t n, double* out, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(tri_shape_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, rec, n, out);
    return hipGetLastError();
}

size_t scan_scratch_doubles(uint32_t n, uint32_t rows) {
    return (size_t)rows * ((n + kScanTile - 1) / kScanTile + 1);
}

hipError_t launch_prefix_scan(double* a, uint32_t n, uint32_t rows, double* scratch, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const uint32_t nb = (n + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(scan_block_sums, dim3(nb, rows), dim3(kScanBlock), 0, s, a, n, scratch);
    hipLaunchKernelGGL(scan_sums_exclusive, dim3(rows), dim3(1), 0, s, scratch, nb);
    hipLaunchKernelGGL(scan_apply, dim3(nb, rows), dim3(kScanBlock), 0, s, a, n, scratch);
    return hipGetLastError();
}

hipError_t launch_slot_features(uint32_t R, const unsigned char* nodes, uint32_t stride, const uint32_t* range,
                                const uint8_t* depth, uint32_t max_depth, const uint64_t* masks,
                                const double* prefix, const RootBox& root, uint32_t n_inner, float* out,
                                hipStream_t s) {
    if (n_inner == 0) return hipSuccess;
    const dim3 g(blocks_for(2 * (size_t)n_inner, 256));
    if (R == 4)
        hipLaunchKernelGGL(slot_feature_kernel<1>, g, dim3(256), 0, s, nodes, stride, range, depth, max_depth, masks,
                           64u, prefix, root, n_inner, out);
    else
        hipLaunchKernelGGL(slot_feature_kernel<4>, g, dim3(256), 0, s, nodes, stride, range, depth, max_depth, masks,
                           216u, prefix, root, n_inner, out);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const float* prm, const float* x, uint32_t n, float* y, float* act, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(mlp_forward_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, prm, x, n, y, act);
    return hipGetLastError();
}

hipError_t launch_mlp_backward(const float* prm, const float* x, const float* act, const float* y, const float* t,
                               uint32_t n, float* grad, float* work, float* loss, hipStream_t s) {
    if (n == 0) return hipErrorInvalidValue;
    float* delta = work;                  // [n][128]
    float* dyv = work + (size_t)n * 128;  // [n]
    float* sqerr = dyv + n;               // [n]
    float* part = sqerr + n;              // [SC_MLP_GRAD_PARTS][kMlpParams]
    hipLaunchKernelGGL(mlp_delta_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, prm, act, y, t, n, delta, dyv,
                       sqerr);
    hipLaunchKernelGGL(mlp_grad_kernel, dim3(blocks_for(kMlpParams, 64), SC_MLP_GRAD_PARTS), dim3(64), 0, s, x, act,
                       delta, dyv, n, part);
    hipLaunchKernelGGL(mlp_grad_sum_kernel, dim3(blocks_for(kMlpParams, 256)), dim3(256), 0, s, part, grad);
    if (loss) hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(kSumThreads), 0, s, sqerr, n, loss);
    return hipGetLastError();
}

hipError_t launch_adam(float* prm, const float* grad, float* m, float* v, float lr, float b1, float b2, float eps,
                       float bc1, float bc2, hipStream_t s) {
    hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(kMlpParams, 256)), dim3(256), 0, s, prm, grad, m, v, lr, b1, b2,
                       eps, bc1, bc2);
    return hipGetLastError();
}

}  // namespace sc
