// The binary32 filter's bound constants, its eligibility test for edge
// normals, and the list of undecided pairs that the binary64 recheck re-runs.
// Shared by the filtered kernels; the bound itself is derived where the
// filtered kernels are (paper, Method section, constraint 1: the side value
// whose sign the filter decides).  Include only from .hip files compiled with
// -ffp-contract=off.
#pragma once

#include "pip_common.h"

namespace pip {
namespace {

constexpr float kBoundK = 12.0f * 5.9604644775390625e-8f;   // 12 * 2^-24
constexpr float kEta4 = 4.0f * 1.1754943508222875e-38f;       // 4 * 2^-126
constexpr float kN1 = 1.0f + 2.384185791015625e-7f;            // 1 + 2^-22 >= |NX| + |NY|
constexpr double kLim = 1.152921504606846976e18;              // 2^60
constexpr double kTiny = 8.673617379884035e-19;               // 2^-60

constexpr float kLimF = 1.152921504606846976e18f;   // 2^60
constexpr unsigned kRingBad = 0xffffffffu;         // M marker: an edge outside the filter's range

__device__ __forceinline__ bool normal_ok(double v)
{
    const double a = fabs(v);
    return a == 0.0 || (a >= kTiny && a <= kLim);
}

// The filtered record (NX, NY, -C, 0) of edge (a, b) re-centred on c, and
// max(|a_x - c_x|, |a_y - c_y|) rounded up (or kRingBad when the edge is
// outside the filter's range).
__device__ __forceinline__ float4 filtered_record(double ax, double ay, double bx, double by, double cx, double cy,
                                                  unsigned *m_bits)
{
    double nx = by - ay;
    double ny = ax - bx;
    if (nx < 0.0) {
        nx = -nx;
        ny = -ny;
    }
    const double sn = nx + fabs(ny);
    // exact scaling by 2^-e, 1 <= sn 2^-e < 2 (sn = 0: a horizontal edge, never straddling)
    const int e = sn > 0.0 ? ilogb(sn) : 0;
    const double nxs = ldexp(nx, -e), nys = ldexp(ny, -e);
    const double dx = ax - cx, dy = ay - cy;
    const double c = dx * nxs + dy * nys;   // separately rounded (no contraction in this unit)
    const double m = fmax(fabs(dx), fabs(dy));
    const bool ok = normal_ok(nx) && normal_ok(ny) && m <= kLim;
    *m_bits = ok ? __float_as_uint(__double2float_ru(m)) : kRingBad;
    return make_float4((float)nxs, (float)nys, (float)(-c), 0.0f);
}

// The item's undecided pairs join the recheck list with one global atomic per
// item (not one per wavefront and row: with many undecided pairs those
// same-address atomics serialise): every wavefront reserves its share in an
// LDS counter, thread 0 reserves the item's total in the list, then every
// lane writes its own entries.  rows[u] is the wavefront's ballot of row u.
// Must be called by the whole workgroup; s_cnt, s_base: LDS words, s_cnt
// zeroed (and a barrier passed) since the last call.  An item with no
// undecided pair passes one barrier and touches no global memory.
template <int U>
__device__ __forceinline__ void append_recheck_item(const uint64_t (&rows)[U], int64_t p0, int32_t *list,
                                                    unsigned *count, unsigned *s_cnt, unsigned *s_base)
{
    const int lane = threadIdx.x & 63;
    unsigned mine = 0;
#pragma unroll
    for (int u = 0; u < U; ++u)
        mine += (unsigned)__builtin_popcountll(rows[u]);
    unsigned wbase = 0;
    if (lane == 0 && mine)
        wbase = atomicAdd(s_cnt, mine);
    wbase = __builtin_amdgcn_readfirstlane(wbase);
    __syncthreads();
    const unsigned tot = *s_cnt;   // the same for every thread: most items end here
    if (tot == 0)
        return;
    if (threadIdx.x == 0)
        *s_base = atomicAdd(count, tot);
    __syncthreads();
    unsigned at = *s_base + wbase;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const uint64_t m = rows[u];
        if ((m >> lane) & 1u) {
            const unsigned below = (unsigned)__builtin_popcountll(m & ((1ull << lane) - 1ull));
            list[at + below] = (int32_t)(p0 + u * 256 + threadIdx.x);
        }
        at += (unsigned)__builtin_popcountll(m);
    }
}

}  // namespace
}  // namespace pip
