// Device probes: a read-only stream over device memory, the rate that
// read-dominated kernels are compared with (the copy probe sits beside the
// exact kernels), and a vector-ALU issue probe, the rate of binary64 additions
// that instruction-bound kernels are compared with.

#include "pip_common.h"

namespace pip {
namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Every 16-byte word of src read once (nontemporal); the XOR of a thread's
// words is stored only if it equals a fixed value, so the loads must happen
// and at most one word of sink is ever written.
__global__ __launch_bounds__(256) void k_read16(const u32x4 *__restrict__ src, int64_t n16, unsigned *sink)
{
    u32x4 acc = {0u, 0u, 0u, 0u};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16;
         i += (int64_t)gridDim.x * blockDim.x)
        acc ^= __builtin_nontemporal_load(&src[i]);
    const unsigned v = acc.x ^ acc.y ^ acc.z ^ acc.w;
    if (v == 0x9e3779b9u)
        sink[0] = v;
}

constexpr int kValuChains = 8;   // independent binary64 addition chains per thread
constexpr int kValuBlocksPerCu = 8;   // eight wavefronts per SIMD

// Every thread runs `iters` rounds of kValuChains independent binary64
// additions of the uniform `step` (one full-rate vector instruction each, no
// fused or packed forms); the sum is stored only if it equals a value it
// cannot reach from these inputs, so the additions must happen and at most
// one word of sink is written.
__global__ __launch_bounds__(256) void k_valu_probe(double *sink, int iters, double step)
{
    double a[kValuChains];
#pragma unroll
    for (int c = 0; c < kValuChains; ++c)
        a[c] = (double)(threadIdx.x * kValuChains + c);
#pragma unroll 4
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < kValuChains; ++c)
            a[c] += step;
    }
    double t = 0.0;
#pragma unroll
    for (int c = 0; c < kValuChains; ++c)
        t += a[c];
    if (t == -1.0)
        sink[0] = t;
}

}  // namespace

int launch_valu_probe(int iters, double *sink, int cu_count, int64_t *lane_ops, hipStream_t stream)
{
    const unsigned g = (unsigned)(cu_count > 0 ? cu_count : 1) * kValuBlocksPerCu;
    *lane_ops = (int64_t)g * 256 * (int64_t)iters * kValuChains;
    // a step the additions cannot be folded over (a power of two: every sum is exact)
    hipLaunchKernelGGL(k_valu_probe, dim3(g), dim3(256), 0, stream, sink, iters, 0.5);
    PIP_HIP_TRY(hipGetLastError());
    return PIP_OK;
}

int launch_read(const void *src, int64_t nbytes, unsigned *sink, hipStream_t stream)
{
    const int64_t n16 = nbytes / 16;
    int64_t g = (n16 + 255) / 256;
    g = g > 65536 ? 65536 : (g < 1 ? 1 : g);
    hipLaunchKernelGGL(k_read16, dim3((unsigned)g), dim3(256), 0, stream, (const u32x4 *)src, n16, sink);
    PIP_HIP_TRY(hipGetLastError());
    return PIP_OK;
}

}  // namespace pip
