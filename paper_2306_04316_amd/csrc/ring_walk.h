// Device helpers shared by the exact and the filtered kernels: the rule's
// per-edge step in binary64 (paper, Method section, constraint 1, and
// Algorithm 1, half-open straddle reading), in per-lane and lane-mask forms,
// and the wave-uniform ring walks.  Include only from .hip files compiled
// with -ffp-contract=off.
//
// The negation of the normal is never materialised in the per-lane and mask
// steps: with round-to-nearest-even, fl(t * (-d)) = -fl(t * d) and
// fl(-u - v) = -fl(u + v), so the side value with the negated normal is
// exactly -s' where s' uses the unnegated normal.  Under the straddle
// condition n_x < 0 holds exactly when a is the endpoint above the ray, so the
// crossing test becomes (b above ? s' <= 0 : s' >= 0).  Both tests treat +0
// and -0 alike, so the bit is the same as the literal rule's.
#pragma once

#include "pip_common.h"

namespace pip {
namespace {

// Clamp a ring's [b, e) to the vertex array so no access leaves it, and to
// at most INT32_MAX vertices per ring.
__device__ __forceinline__ void clamp_ring(int64_t &b, int64_t &e, int64_t nv)
{
    e = e < 0 ? 0 : (e > nv ? nv : e);
    b = b < 0 ? 0 : (b > e ? e : b);
    e = (e - b > INT32_MAX) ? b + INT32_MAX : e;
}

// Rings [r0, r1) of polygon q: with a ring index (polygons of several rings),
// poly_rings[q] .. poly_rings[q+1]-1 clamped to [0, n_rings]; without one,
// ring q alone (offsets is then the polygon CSR).
__device__ __forceinline__ void poly_ring_range(const int64_t *__restrict__ poly_rings, int64_t n_rings, int64_t q,
                                                int64_t &r0, int64_t &r1)
{
    if (!poly_rings) {
        r0 = q;
        r1 = q + 1;
        return;
    }
    r0 = poly_rings[q];
    r1 = poly_rings[q + 1];
    r0 = r0 < 0 ? 0 : (r0 > n_rings ? n_rings : r0);
    r1 = r1 < r0 ? r0 : (r1 > n_rings ? n_rings : r1);
}

// Which test decides a straddling edge's crossing (paper, Method section):
//   kSide: constraint 1, (p - a) . n <= 0 with the normal oriented n_x > 0
//   kIntersection: constraint 2, lambda = (p_y - a_y) / d_y,
//                  x = a_x + lambda * d_x, crossing iff x >= p_x
enum Predicate : int { kSide = 0, kIntersection = 1 };

// Crossing bit of a straddling edge (a, b); b_above says which endpoint is
// above the ray (so the normal's orientation needs no negation, see above).
template <int PRED>
__device__ __forceinline__ bool straddle_crosses(double x, double y, double ax, double ay, double bx, double by,
                                                 bool b_above)
{
    if (PRED == kIntersection) {
        const double dx = bx - ax;
        const double dy = by - ay;
        const double lam = (y - ay) / dy;
        const double xn = ax + lam * dx;
        return xn >= x;
    }
    const double nx = by - ay;
    const double ny = ax - bx;
    const double t1 = x - ax;
    const double t2 = y - ay;
    const double s = t1 * nx + t2 * ny;
    return b_above ? (s <= 0.0) : (s >= 0.0);
}

// Crossing-parity contribution of edge (a, b) for point (x, y).
template <int PRED>
__device__ __forceinline__ unsigned edge_cross(double x, double y, double ax, double ay, bool a_above,
                                               double bx, double by, bool b_above)
{
    return (a_above != b_above && straddle_crosses<PRED>(x, y, ax, ay, bx, by, b_above)) ? 1u : 0u;
}

// Shift the "vertex above the ray" bit of y_v into the low end of word w.
// y_v > p_y  <=>  fl(p_y - y_v) < 0: the difference of two binary64 values is
// zero only when they are equal (gradual underflow) and otherwise has the
// exact sign, so its sign bit is the comparison -- provided p_y carries no
// negative zero (p_y = -0, y_v = +0 would give -0).  Callers pass
// yq = p_y + 0.0, which maps -0 to +0 and leaves every other value alone.
// One add and one funnel shift, and no condition-mask hazards.
__device__ __forceinline__ uint32_t shift_in_above(uint32_t w, double yq, double yv)
{
    const double d = yq - yv;
    const uint32_t hi = (uint32_t)(__double_as_longlong(d) >> 32);
    return __builtin_amdgcn_alignbit(w, hi, 31);
}

// True on every thread when v is true on every thread of the 256-thread
// workgroup; also a workgroup barrier.  Each wavefront reduces with one
// ballot and posts its verdict to flags (LDS, 4 words, rewritten on every
// call, so nothing needs clearing); one barrier later every thread reads the
// four.  A caller that calls it again must pass another barrier in between.
__device__ __forceinline__ bool block_all(bool v, int *flags)
{
    const bool w = __builtin_amdgcn_ballot_w64(!v) == 0;
    if ((threadIdx.x & 63) == 0)
        flags[threadIdx.x >> 6] = w ? 1 : 0;
    __syncthreads();
    return (flags[0] & flags[1] & flags[2] & flags[3]) != 0;
}

// One 32-edge chunk of a wave-uniform ring of k vertices with compacted side
// tests: edges c0 .. c0+m-1, m = min(32, end - c0) (end <= k: the last edge
// the walk takes, for walks over a part of the ring), i.e. vertices
// v_{c0-1} -> v_{c0} onwards.  The ring's
// y values stream through scalar loads into each lane's 32-bit "above" word
// (two vector instructions per vertex); each member lane then evaluates the
// side value only for its own straddling edges, fetching those two vertices
// itself.  `prev` holds the above bit of v_{c0-1} on entry and of the chunk's
// last vertex on exit.  Returns the lanes with an odd number of crossings in
// the chunk: each lane's own bit of the result is exact; the other bits are
// those of the side-test ballots that lane took part in (the loop is
// divergent), so a caller that needs the whole mask gathers it with one
// ballot of each lane's own bit.
template <int PRED>
__device__ __forceinline__ uint64_t chunk_parity_uniform(double x, double y, double yq, bool member,
                                                         const double *__restrict__ rx,
                                                         const double *__restrict__ ry, int k, int c0,
                                                         uint32_t &prev, int end)
{
    const int m = end - c0 < 32 ? end - c0 : 32;
    uint32_t above = 0;
    if (m == 32) {
#pragma unroll
        for (int t = 0; t < 32; ++t)
            above = shift_in_above(above, yq, ry[c0 + t]);
    } else {
        // partial chunk: batches of 8 (clamped to the ring's last vertex, whose
        // extra bits are masked below), then left-align
        int t = 0;
        for (; t < m; t += 8) {
#pragma unroll
            for (int tt = 0; tt < 8; ++tt)
                above = shift_in_above(above, yq, ry[c0 + (t + tt < m ? t + tt : m - 1)]);
        }
        above <<= (32 - t);
    }
    uint32_t strad = above ^ ((above >> 1) | (prev << 31));
    if (m < 32)
        strad &= ~(0xffffffffu >> m);
    prev = (above >> (32 - m)) & 1u;
    strad = member ? strad : 0u;
    uint64_t par = 0;
    while (strad != 0) {
        const int j = __builtin_clz(strad);
        strad ^= 0x80000000u >> j;
        const int jb = c0 + j;
        const int ja = jb == 0 ? k - 1 : jb - 1;
        const double ax = rx[ja], ay = ry[ja], bx = rx[jb], by = ry[jb];
        const bool b_above = (above >> (31 - j)) & 1u;
        par ^= __builtin_amdgcn_ballot_w64(straddle_crosses<PRED>(x, y, ax, ay, bx, by, b_above));
    }
    return par;
}

// Crossing parity of every lane's point against the wave-uniform ring [b, e),
// chunk by chunk.  Must be called with the whole wavefront active.
template <int PRED>
__device__ __forceinline__ uint64_t ring_parity_compact_uniform(double x, double y, bool member,
                                                                const double *__restrict__ vx,
                                                                const double *__restrict__ vy, int64_t b,
                                                                int64_t e)
{
    const int k = (int)(e - b);
    const double *__restrict__ rx = vx + b;
    const double *__restrict__ ry = vy + b;
    uint64_t par = 0;
    if (k <= 0)
        return 0;
    const double yq = y + 0.0;
    uint32_t prev = shift_in_above(0u, yq, ry[k - 1]);
    for (int c0 = 0; c0 < k; c0 += 32)
        par ^= chunk_parity_uniform<PRED>(x, y, yq, member, rx, ry, k, c0, prev, k);
    return par;
}

// Rows u of a workgroup item whose rings were not staged: lanes that share a
// polygon run together (leader = first unfinished lane), each group walking
// its ring wave-uniformly with compacted side tests.
// Polygons of several rings (MR) XOR their rings' parities (poly_rings as in
// poly_ring_range); without MR ring q is polygon q.
template <int PRED, int U, bool MR = false>
__device__ __forceinline__ void group_walk_rows(int64_t p0, const double (&x)[U], const double (&y)[U],
                                                const int (&q)[U], int64_t n, const int64_t *__restrict__ offsets,
                                                int64_t n_polys, const int64_t *__restrict__ poly_rings,
                                                int64_t n_rings, const double *__restrict__ vx,
                                                const double *__restrict__ vy, int64_t nv,
                                                uint8_t *__restrict__ inside)
{
    const int tid = threadIdx.x;
    const int lane = tid & 63;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t i = p0 + u * 256 + tid;
        const int qv = ((uint32_t)q[u] < (uint64_t)n_polys) ? q[u] : 0;
        uint64_t todo = __builtin_amdgcn_ballot_w64(i < n);
        uint64_t par = 0;
        while (todo) {
            const int leader = __builtin_ctzll(todo);
            const int qu = __builtin_amdgcn_readlane(qv, leader);
            const uint64_t member = todo & __builtin_amdgcn_ballot_w64(qv == qu);
            uint64_t gp = 0;
            if (MR) {
                int64_t r0, r1;
                poly_ring_range(poly_rings, n_rings, qu, r0, r1);
                for (int64_t r = r0; r < r1; ++r) {
                    int64_t b = offsets[r], e = offsets[r + 1];
                    clamp_ring(b, e, nv);
                    gp ^= ring_parity_compact_uniform<PRED>(x[u], y[u], (member >> lane) & 1u, vx, vy, b, e);
                }
            } else {
                int64_t b = offsets[qu], e = offsets[qu + 1];
                clamp_ring(b, e, nv);
                gp = ring_parity_compact_uniform<PRED>(x[u], y[u], (member >> lane) & 1u, vx, vy, b, e);
            }
            par |= gp & member;
            todo &= ~member;
        }
        if (i < n)
            inside[i] = (uint8_t)((par >> lane) & 1u);
    }
}

}  // namespace
}  // namespace pip
