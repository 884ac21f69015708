// Device-wide exclusive scan of uint32 counts into int64 offsets (n + 1
// outputs, the last one the total): per-tile sums, one workgroup scanning the
// tile sums, then per-tile prefixes.  Kernels only (no memset), so it can be
// captured in a graph.
#include "pip_common.h"

namespace pip {
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanPer = 16;
constexpr int kScanTile = kScanThreads * kScanPer;

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const uint32_t *__restrict__ in, int64_t n,
                                                              int64_t *__restrict__ block_sums)
{
    __shared__ int64_t s[kScanThreads];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    int64_t acc = 0;
    for (int k = 0; k < kScanPer; ++k) {
        const int64_t i = base + (int64_t)k * kScanThreads + threadIdx.x;
        if (i < n)
            acc += in[i];
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int off = kScanThreads / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off)
            s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        block_sums[blockIdx.x] = s[0];
}

// Block-level inclusive scan of one value per thread (LDS, Hillis-Steele).
__device__ __forceinline__ int64_t block_inclusive_scan(int64_t v, int64_t *s)
{
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        const int64_t add = (int)threadIdx.x >= off ? s[threadIdx.x - off] : 0;
        __syncthreads();
        s[threadIdx.x] += add;
        __syncthreads();
    }
    return s[threadIdx.x];
}

// One workgroup: exclusive scan of the nb block sums in place (any nb).
__global__ __launch_bounds__(kScanThreads) void k_scan_blocks(int64_t *__restrict__ sums, int64_t nb)
{
    __shared__ int64_t s[kScanThreads];
    int64_t carry = 0;
    for (int64_t c0 = 0; c0 < nb; c0 += kScanThreads) {
        const int64_t i = c0 + threadIdx.x;
        const int64_t v = i < nb ? sums[i] : 0;
        const int64_t inc = block_inclusive_scan(v, s);
        if (i < nb)
            sums[i] = carry + inc - v;
        const int64_t total = s[kScanThreads - 1];
        __syncthreads();
        carry += total;
    }
}

// out[i] = block offset + exclusive prefix within the tile; out[n] = total.
__global__ __launch_bounds__(kScanThreads) void k_scan_down(const uint32_t *__restrict__ in, int64_t n,
                                                            const int64_t *__restrict__ block_off,
                                                            int64_t *__restrict__ out)
{
    __shared__ int64_t s[kScanThreads];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
    uint32_t v[kScanPer];
    int64_t acc = 0;
    for (int k = 0; k < kScanPer; ++k) {
        const int64_t i = base + k;
        v[k] = i < n ? in[i] : 0u;
        acc += v[k];
    }
    const int64_t inc = block_inclusive_scan(acc, s);
    int64_t run = block_off[blockIdx.x] + inc - acc;
    for (int k = 0; k < kScanPer; ++k) {
        const int64_t i = base + k;
        if (i < n)
            out[i] = run;
        run += v[k];
        if (i == n - 1)
            out[n] = run;
    }
}

__global__ void k_scan_zero(int64_t *out) { *out = 0; }

}  // namespace

int64_t scan_ws_entries(int64_t n) { return (n > 0 ? (n + kScanTile - 1) / kScanTile : 1) + 1; }

int launch_scan_u32(const uint32_t *in, int64_t n, int64_t *out, int64_t *block_ws, hipStream_t s)
{
    if (n <= 0) {
        hipLaunchKernelGGL(k_scan_zero, dim3(1), dim3(1), 0, s, out);
        PIP_HIP_TRY(hipGetLastError());
        return PIP_OK;
    }
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, n, block_ws);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(kScanThreads), 0, s, block_ws, nb);
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, n, block_ws, out);
    PIP_HIP_TRY(hipGetLastError());
    return PIP_OK;
}

}  // namespace pip
