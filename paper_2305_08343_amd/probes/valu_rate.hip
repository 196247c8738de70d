// Vector-ALU issue rate of the GPU, measured: the reference point for the traversal kernels'
// SQ_INSTS_VALU counts (a kernel's wave-level VALU instructions per SIMD per cycle against the
// rate a saturating instruction stream reaches).
//
// Each lane runs eight independent dependency chains of float32 multiply / add, of integer
// add / shift / xor, and of fused multiply-add / max, long enough that the launch (eight waves
// per SIMD on every CU) is bound by instruction issue alone. The loop bodies hold 16, 24 and 16
// VALU instructions (one per chain and operation; the assembly of this file shows them), which
// SQ_INSTS_VALU confirms under rocprofv3.
//
//   valu_rate [iterations]     prints one line per kernel and repetition
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

template <int KIND>
__global__ __launch_bounds__(256) void valu_chains(float* out, int iters) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    float f[8];
    unsigned u[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        f[k] = (float)(t + k) * 1e-7f;
        u[k] = (unsigned)(t * 7 + k);
    }
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if constexpr (KIND == 0) {
                f[k] = f[k] * 0.999f;
                f[k] = f[k] + 1e-6f;
            } else if constexpr (KIND == 1) {
                u[k] = u[k] + 0x9E3779B9u;
                u[k] = u[k] ^ (u[k] >> 7);
            } else {
                f[k] = __builtin_fmaf(f[k], 0.999f, 1e-6f);
                f[k] = fmaxf(f[k], 1e-7f);
            }
        }
    }
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < 8; ++k) s += f[k] + (float)u[k];
    out[t] = s;  // keeps every chain live
}

static void check(hipError_t e, const char* what) {
    if (e != hipSuccess) {
        std::fprintf(stderr, "%s: %s\n", what, hipGetErrorString(e));
        std::exit(1);
    }
}

int main(int argc, char** argv) {
    const int iters = argc > 1 ? std::atoi(argv[1]) : 20000;
    int dev = 0, cus = 0;
    check(hipGetDevice(&dev), "hipGetDevice");
    check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "hipDeviceGetAttribute");
    const int simds = cus * 4;
    const int blocks = simds * 8 / 4;  // eight 64-lane waves per SIMD, four waves a block
    float* d = nullptr;
    check(hipMalloc(&d, sizeof(float) * (size_t)blocks * 256), "hipMalloc");
    hipEvent_t a, b;
    check(hipEventCreate(&a), "hipEventCreate");
    check(hipEventCreate(&b), "hipEventCreate");
    const char* names[3] = {"f32 mul+add", "u32 add+shift+xor", "f32 fma+max"};
    const double per_iter[3] = {16.0, 24.0, 16.0};
    for (int kind = 0; kind < 3; ++kind) {
        for (int rep = 0; rep < 3; ++rep) {
            check(hipEventRecord(a, 0), "hipEventRecord");
            if (kind == 0) hipLaunchKernelGGL(valu_chains<0>, dim3(blocks), dim3(256), 0, 0, d, iters);
            if (kind == 1) hipLaunchKernelGGL(valu_chains<1>, dim3(blocks), dim3(256), 0, 0, d, iters);
            if (kind == 2) hipLaunchKernelGGL(valu_chains<2>, dim3(blocks), dim3(256), 0, 0, d, iters);
            check(hipGetLastError(), "launch");
            check(hipEventRecord(b, 0), "hipEventRecord");
            check(hipEventSynchronize(b), "hipEventSynchronize");
            float ms = 0.0f;
            check(hipEventElapsedTime(&ms, a, b), "hipEventElapsedTime");
            const double instrs = (double)blocks * 4.0 * iters * per_iter[kind];
            std::printf("%-18s rep %d: %.3f ms, %.4e wave instructions, %.3f per SIMD per ns\n", names[kind], rep, ms,
                        instrs, instrs / simds / (ms * 1e6));
        }
    }
    check(hipFree(d), "hipFree");
    return 0;
}
