// Wavefront-per-large-ring form of the filtered batched step (paper, Method
// section, constraint 1, and Algorithm 1, with the half-open straddle
// reading): lanes are edges and the point is wave-uniform.
//
// The batched kernel leaves the pairs of rings with at least wave_k vertices
// to this kernel and lists each such ring once per work item, with the
// item's pair range (WaveTask).  A workgroup takes one task at a time from a
// queue.  Its pairs of the ring (point_poly equal to the ring) are compacted
// into an LDS table of binary64 p_y and binary32 P = fl32(fl64(p - c)), c the
// ring's first vertex.  The ring's 64-edge chunks are cut into groups of up
// to kGroup held in registers, and the four wavefronts share the (group,
// point slice) units.  Lane l of chunk j holds edge e = 64 j + l, from vertex e-1
// (the last vertex for e = 0) to vertex e: both endpoints' y in binary64 and
// the batched kernel's filtered record (NX, NY, -C).  For each point:
//   above bits (y_a > p_y), (y_b > p_y): the sign bits of the binary64
//   differences p_y - y (exact), so the edge straddles when they differ
//   (half-open rule);
//   S = fma(P_x, NX, fma(P_y, NY, -C)) on every lane;
//   a lane's crossing bit (straddles and S < 0) folds into its XOR word, and
//   the popcount parity of the ballot of those words is the group's
//   contribution;
//   a straddling edge with |S| <= B_p, B_p = fma(M, k_B, e_B) and M =
//   max(the group's M, |P_x|, |P_y|), makes the pair undecided.
// A group's parity and undecided flag go into the point's LDS word by one
// lane; when every unit is done the workgroup writes each decided pair's
// byte and lists the undecided ones for the binary64 recheck.  The error
// bound and its proof are the batched kernel's: a group's M bounds |a - c|
// over the anchors its tests use, and the same eligibility limits apply.
// Edges that cannot straddle (horizontal, or lanes past the ring's end) carry
// y_a = y_b and a record whose S is 2^100, so they never count.
//
// This translation unit must be compiled with -ffp-contract=off.

#include "filter_bound.h"
#include "pip_common.h"
#include "ring_walk.h"

namespace pip {
namespace {

constexpr int kGroup = 5;   // 64-edge chunks per register group (80 VGPRs: six wavefronts per SIMD)
constexpr float kFar = 1.2676506002282294e30f;   // 2^100: the offset of a record that never counts

struct WaveArgs {
    const double *px, *py;
    int64_t n;
    const int64_t *offsets;
    int64_t n_polys;
    const double *vx, *vy;
    int64_t nv;
    const int32_t *point_poly;
    uint8_t *inside;
    const WaveTask *tasks;
    const unsigned *task_count;
    unsigned max_tasks;
    unsigned *cursor;
    float bound_k, bound_eta;
    int force_recheck;
    int32_t *recheck;
    unsigned *recheck_count;
    unsigned long long *stats;   // [256][2]: point-edge tests, undecided side tests
};

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v = max(v, (uint32_t)__shfl_xor((int)v, o));
    return v;
}

// One unit: the group's NJ chunks (in registers) against the points m =
// slice, slice + nslices, ... of the table.  Per chunk and point, on every
// lane (edge): the sign bits of p_y - y_a and p_y - y_b (binary64; with p_y
// + 0.0, never -0, the difference is negative exactly when y > p_y, and x - x
// is +0), their XOR (bit 31: the edge straddles), S, then two three-input bit operations: the lane's
// crossing word x ^= straddle & S (bit 31: S < 0) and its undecided word
// u |= straddle & (|S| - B') with B' the float after B (bit 31: |S| <= B).
// The point's parity is the popcount parity of ballot(x bit 31) and it is
// undecided when any lane's u has bit 31; both go into the point's LDS word.
template <int NJ, bool STATS>
__device__ __forceinline__ void wave_unit(const double (&ya)[kGroup], const double (&yb)[kGroup],
                                          const float (&nx)[kGroup], const float (&ny)[kGroup],
                                          const float (&cc)[kGroup], uint32_t bgb, bool bad, int M, int slice,
                                          int nslices, const double2 *s_pp, const float *s_bp, unsigned *s_acc,
                                          uint32_t &n_und)
{
    const int lane = threadIdx.x & 63;
    for (int m = slice; m < M; m += nslices) {
        const double2 pp = s_pp[m];   // p_y + 0.0; (P_x, P_y) as two binary32 in the second word
        const double p = pp.x;
        const float px = __uint_as_float((uint32_t)__double_as_longlong(pp.y));
        const float py = __uint_as_float((uint32_t)(__double_as_longlong(pp.y) >> 32));
        // B = fma(max(group M, |P|), k_B, e_B) = max(the group's B, the point's B)
        // (the rounding is monotone); non-negative floats order as their bits.
        // B' = the float after B: |S| < B' iff |S| <= B.
        const float bnd1 = __uint_as_float(max(bgb, __float_as_uint(s_bp[m])) + 1u);
        uint32_t x = 0, u = 0;
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const uint32_t ha = (uint32_t)(__double_as_longlong(p - ya[j]) >> 32);
            const uint32_t hb = (uint32_t)(__double_as_longlong(p - yb[j]) >> 32);
            const uint32_t t = ha ^ hb;
            const float sv = __builtin_fmaf(px, nx[j], __builtin_fmaf(py, ny[j], cc[j]));
            x ^= t & __float_as_uint(sv);
            u |= t & __float_as_uint(fabsf(sv) - bnd1);
        }
        const uint64_t xs = __builtin_amdgcn_ballot_w64((int)x < 0);
        const uint64_t us = __builtin_amdgcn_ballot_w64((int)u < 0);
        if (STATS)
            n_und += (uint32_t)__builtin_popcountll(us);
        // bit 0 of the point's word sums (XORs) the groups' parities; an
        // undecided group adds 2^16 (carries from bit 0 stay below it)
        const unsigned r = __builtin_amdgcn_readfirstlane(((unsigned)__builtin_popcountll(xs) & 1u) |
                                                         ((us != 0 || bad) ? 0x10000u : 0u));
        if (r != 0 && lane == 0)
            atomicAdd(&s_acc[m], r);
    }
}

template <bool STATS>
__global__ __launch_bounds__(256) void k_wave_rings(WaveArgs A)
{
    __shared__ double2 s_pp[256];      // p_y + 0.0, and P_x, P_y (binary32) packed in one word
    __shared__ float s_bp[256];        // fma(max(|P_x|, |P_y|), k_B, e_B): the point's part of the bound
    __shared__ int s_off[256];         // the pair's offset in the block
    __shared__ unsigned s_acc[256];    // bit 0: crossing parity; from bit 16: undecided groups
    __shared__ unsigned s_task, s_m, s_rcnt, s_rbase;
    __shared__ unsigned s_stat[2];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform
    const unsigned cnt = *A.task_count;
    const unsigned ntask = cnt < A.max_tasks ? cnt : A.max_tasks;
    uint32_t n_tests = 0, n_und = 0;
    if (STATS && tid < 2)
        s_stat[tid] = 0;

    for (;;) {
        if (tid == 0)
            s_task = atomicAdd(A.cursor, 1u);
        __syncthreads();
        const unsigned t = s_task;
        if (t >= ntask)
            break;
        const WaveTask T = A.tasks[t];
        int64_t b = A.offsets[T.ring], e = A.offsets[T.ring + 1];
        clamp_ring(b, e, A.nv);
        const int k = (int)(e - b);
        const double cx = k > 0 ? A.vx[b] : 0.0, cy = k > 0 ? A.vy[b] : 0.0;
        const int nch = (k + 63) >> 6;
        const int G = (nch + kGroup - 1) / kGroup;
        const int nslices = G >= 4 ? 1 : 4 / G;
        const int64_t pend = T.p_lo + T.count < A.n ? T.p_lo + T.count : A.n;

        for (int64_t q0 = T.p_lo; q0 < pend; q0 += 256) {
            if (tid == 0) {
                s_m = 0;
                s_rcnt = 0;
            }
            __syncthreads();
            // the block's pairs of this ring, compacted into the point table
            const int64_t i = q0 + tid;
            const bool mine = i < pend && (A.point_poly ? A.point_poly[i] : 0) == T.ring;
            double py = 0.0;
            float PX = 0.0f, PY = 0.0f, mp = 0.0f;
            bool elig = false;
            if (mine) {
                const double px = A.px[i];
                py = A.py[i];
                PX = (float)(px - cx);
                PY = (float)(py - cy);
                // |P| < 2^60 (binary32, so |p - c| < 2^60); NaN is ineligible
                elig = fabsf(PX) < kLimF && fabsf(PY) < kLimF;
                mp = fmaxf(fabsf(PX), fabsf(PY));
            }
            const uint64_t bal = __builtin_amdgcn_ballot_w64(mine);
            unsigned wbase = 0;
            if (lane == 0 && bal)
                wbase = atomicAdd(&s_m, (unsigned)__builtin_popcountll(bal));
            wbase = __builtin_amdgcn_readfirstlane(wbase);
            if (mine) {
                const int m = (int)wbase + (int)__builtin_popcountll(bal & ((1ull << lane) - 1ull));
                const uint64_t pxy = (uint64_t)__float_as_uint(PX) | ((uint64_t)__float_as_uint(PY) << 32);
                s_pp[m] = make_double2(py + 0.0, __longlong_as_double((long long)pxy));   // no negative zero
                s_bp[m] = __builtin_fmaf(mp, A.bound_k, A.bound_eta);
                s_off[m] = tid;
                s_acc[m] = (k > 0 && elig) ? 0u : 0x10000u;
            }
            __syncthreads();
            const int M = (int)s_m;

            for (int unit = w; unit < G * nslices; unit += 4) {
                const int g = unit % G;
                const int slice = unit / G;
                const int c0 = g * kGroup;
                const int nj = nch - c0 < kGroup ? nch - c0 : kGroup;
                double ya[kGroup], yb[kGroup];
                float nx[kGroup], ny[kGroup], cc[kGroup];
                uint32_t mb = 0;
#pragma unroll
                for (int j = 0; j < kGroup; ++j) {
                    const int ej = (c0 + j) * 64 + lane;
                    ya[j] = 0.0;
                    yb[j] = 0.0;
                    nx[j] = 0.0f;
                    ny[j] = 0.0f;
                    cc[j] = kFar;
                    if (j < nj && ej < k) {
                        const int ep = ej == 0 ? k - 1 : ej - 1;
                        const double ax = A.vx[b + ep], ay = A.vy[b + ep];
                        const double bx = A.vx[b + ej], by = A.vy[b + ej];
                        if (ay != by) {
                            unsigned mj;
                            const float4 rec = filtered_record(ax, ay, bx, by, cx, cy, &mj);
                            ya[j] = ay;
                            yb[j] = by;
                            nx[j] = rec.x;
                            ny[j] = rec.y;
                            cc[j] = rec.z;
                            mb = max(mb, mj);
                        }
                    }
                    // one edge's loads and record at a time: the group's
                    // registers hold only the finished records
                    __builtin_amdgcn_sched_barrier(0);
                }
                mb = __builtin_amdgcn_readfirstlane(wave_max_u32(mb));
                const bool bad = mb == kRingBad;
                // the group's part of the bound: fma(M_group, k_B, e_B)
                const uint32_t bgb = __float_as_uint(__builtin_fmaf(bad ? 0.0f : __uint_as_float(mb), A.bound_k,
                                                                    A.bound_eta));
                static_assert(kGroup == 5, "one case per group size");
                switch (nj) {
                case 1: wave_unit<1, STATS>(ya, yb, nx, ny, cc, bgb, bad, M, slice, nslices, s_pp, s_bp, s_acc, n_und); break;
                case 2: wave_unit<2, STATS>(ya, yb, nx, ny, cc, bgb, bad, M, slice, nslices, s_pp, s_bp, s_acc, n_und); break;
                case 3: wave_unit<3, STATS>(ya, yb, nx, ny, cc, bgb, bad, M, slice, nslices, s_pp, s_bp, s_acc, n_und); break;
                case 4: wave_unit<4, STATS>(ya, yb, nx, ny, cc, bgb, bad, M, slice, nslices, s_pp, s_bp, s_acc, n_und); break;
                default: wave_unit<5, STATS>(ya, yb, nx, ny, cc, bgb, bad, M, slice, nslices, s_pp, s_bp, s_acc, n_und); break;
                }
            }
            __syncthreads();

            // outputs: decided pairs' bytes; undecided ones join the recheck list
            bool und = false;
            int64_t ip = 0;
            if (tid < M) {
                const unsigned acc = s_acc[tid];
                ip = q0 + s_off[tid];
                und = (acc >> 16) != 0 || A.force_recheck;
                if (!und)
                    A.inside[ip] = (uint8_t)(acc & 1u);
                if (STATS)
                    n_tests += (uint32_t)k;
            }
            const uint64_t ub = __builtin_amdgcn_ballot_w64(und);
            unsigned rb = 0;
            if (lane == 0 && ub)
                rb = atomicAdd(&s_rcnt, (unsigned)__builtin_popcountll(ub));
            rb = __builtin_amdgcn_readfirstlane(rb);
            __syncthreads();
            if (tid == 0 && s_rcnt)
                s_rbase = atomicAdd(A.recheck_count, s_rcnt);
            __syncthreads();
            if (und)
                A.recheck[s_rbase + rb + (unsigned)__builtin_popcountll(ub & ((1ull << lane) - 1ull))] = (int32_t)ip;
            // the next block (or task) rewrites the table only after the barrier at its start
        }
        __syncthreads();   // every thread has read s_task before thread 0 takes the next one
    }
    if (STATS) {
        if (n_tests)
            atomicAdd(&s_stat[0], n_tests);
        if (n_und)
            atomicAdd(&s_stat[1], n_und);
        __syncthreads();
        if (tid == 0) {
            unsigned long long *st = A.stats + (blockIdx.x & 255) * 2;
            atomicAdd(st, (unsigned long long)s_stat[0]);
            atomicAdd(st + 1, (unsigned long long)s_stat[1]);
        }
    }
}

}  // namespace

int launch_wave_rings(const Problem &p, hipStream_t stream, const WaveTask *tasks, const unsigned *task_count,
                      unsigned max_tasks, unsigned *cursor, float bound_k, float bound_eta, int force_recheck,
                      int32_t *recheck, unsigned *recheck_count, unsigned long long *stats, int grid)
{
    if (grid <= 0)
        return PIP_OK;
    WaveArgs A{p.px, p.py, p.n_points, p.offsets, p.n_polys, p.vx, p.vy, p.n_vertices, p.point_poly, p.inside,
               tasks, task_count, max_tasks, cursor, bound_k, bound_eta, force_recheck, recheck, recheck_count,
               stats};
    if (stats)
        PIP_LAUNCH(k_wave_rings<true>, dim3(grid), dim3(256), 0, stream, A);
    else
        PIP_LAUNCH(k_wave_rings<false>, dim3(grid), dim3(256), 0, stream, A);
    PIP_HIP_TRY(hipGetLastError());
    return PIP_OK;
}

}  // namespace pip
