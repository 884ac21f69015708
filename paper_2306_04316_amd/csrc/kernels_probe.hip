// Bandwidth probe: a read-only stream over device memory, the rate that
// read-dominated kernels are compared with (the copy probe sits beside the
// exact kernels).

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

}  // namespace

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
