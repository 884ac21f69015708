// Binary32 filtered evaluation with a proven error bound, plus the binary64
// recheck of the pairs the filter cannot decide.
//
// Per workgroup item (256*U consecutive pairs, sorted by polygon) the rings'
// binary64 vertices are first copied to LDS in one coalesced round with the
// ring table; from there one thread per vertex derives, re-centred on the
// ring's bounding-box centre c:
//   YF : fl32(fl64(y_j - c_y)) per vertex (straddle pass)
//   EF : (XI, YI, NX, NY) = fl32 of fl64(a - c) and of the rule's binary64
//        normal n (negated when its x part is negative) scaled by
//        fl64(1 / s), s = fl64(n_x + |n_y|), per edge
// and per ring: c (binary64), M_ring = an upper bound of |v - c| over the
// ring (rounded up to binary32), and an eligibility flag.
//
// For a pair, P = fl32(fl64(p - c)).  Straddle: rounding is monotone, so a
// strict binary32 order between P_y and a vertex's YF implies the same
// strict binary64 order between p_y and y_v; equal values are undecided.
// The order is the sign bit of the difference P_y - YF, which is nonzero
// for unequal values (gradual underflow; a flushed subnormal difference is
// zero, so undecided as well); a zero difference of either sign marks the
// pair undecided.
// Side: S = fl32(fl32(P_x - XI) * NX + fl32(P_y - YI) * NY).  Every edge
// that can straddle has s > 0, and NX, NY have relative error at most
// u (1 + 2^-27) against n_x / s, n_y / s (u = 2^-24: the conversion, plus two
// binary64 roundings), so |NX| + |NY| <= N1 = 1 + 2^-22.  The sign to find
// is that of E = t1 n_x + t2 n_y, the exact value on the binary64 inputs and
// normals, which is the sign of E / s.  With M >= every re-centred
// coordinate of the pair (point and ring),
//   |S - E / s| <= 10.03 u M (|NX| + |NY|) + 4 eta (|NX| + |NY| + 1),
// where eta = 2^-126 covers flushed subnormals.  If |S| > B = 12 u M N1 +
// 4 eta (N1 + 1), one threshold per pair, then |E| > 1.97 u M s, while the
// binary64 value the rule computes differs from E by at most
// 6.02 * 2^-53 M (|n_x| + |n_y|): that value is nonzero with the sign of S
// (the 12 also covers the rounding of B itself and of M).  The bound needs
// every nonzero |n| component in [2^-60, 2^60] (no overflow of s; scaled
// components stay at or above 2^-121, so none underflows in binary32) and
// |p - c|, |v - c| <= 2^60; rings or points outside that range are not
// filtered.  A pair with any undecided straddle or side test is appended to
// a list and re-run in binary64 in the rule's order.
//
// An item whose vertex range does not fit this layout (or whose pairs are
// not sorted by polygon) is classified in binary64 by the exact kernels'
// staged item (staged_exact.h), which walks a large range in LDS tiles.
//
// This translation unit must be compiled with -ffp-contract=off: the bound
// assumes separately rounded binary32 products and sums.

#include "pip_common.h"
#include "ring_walk.h"
#include "staged_exact.h"
#include "filter_bound.h"

namespace pip {

size_t filtered_smem_bytes(int max_edges, int max_rings)
{
    // T int[max_rings+1] | ring table 32 B per ring | YF float[max_edges+max_rings+64] | EF float4[max_edges]
    // | XD, YD double[max_edges] (the staged binary64 vertices) | per ring: four bounding-box keys and a
    // flag | RID: each staged vertex's ring, one byte
    size_t o = (((size_t)(max_rings + 1) * 4 + 15) & ~(size_t)15);
    o += (size_t)max_rings * 32;
    o += ((((size_t)max_edges + max_rings + 64) * 4 + 15) & ~(size_t)15);
    o += (size_t)max_edges * 16;
    o += (size_t)max_edges * 16;
    o += (size_t)max_rings * 36;
    o += ((size_t)max_edges + 15) & ~(size_t)15;
    return o;
}

namespace {

struct RingInfo {
    double cx, cy;
    float m;        // bound on |v - c| (rounded up), or -1 when the ring is not filterable
    int pad[3];
};

// Order-preserving unsigned key of a binary64 value (finite inputs): unsigned
// comparison of keys is the floating-point order, so LDS integer atomics give
// exact minima and maxima.
__device__ __forceinline__ unsigned long long order_key(double v)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__device__ __forceinline__ double from_order_key(unsigned long long k)
{
    const unsigned long long b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
    return __longlong_as_double((long long)b);
}

// Ring of staged vertex e: the r with T[r] <= e < T[r+1]; -1 when the table is
// not sorted around e (offsets not monotone: unspecified results, accesses in
// bounds).
__device__ __forceinline__ int ring_of_vertex(const int *T, int nr, int e)
{
    int lo = 0, hi = nr;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (T[mid] <= e)
            lo = mid;
        else
            hi = mid;
    }
    return (T[lo] <= e && e < T[lo + 1]) ? lo : -1;
}

template <int U>
__device__ __forceinline__ void filtered_item(
    int64_t p0, const double *__restrict__ px, const double *__restrict__ py, int64_t n,
    const int64_t *__restrict__ offsets, int64_t n_polys,
    const double *__restrict__ vx, const double *__restrict__ vy, int64_t nv,
    const int32_t *__restrict__ point_poly, uint8_t *__restrict__ inside, int max_edges, int max_rings,
    int tile_edges, float bound_scale, int force_recheck, int32_t *__restrict__ recheck, unsigned *recheck_count,
    unsigned char *smem)
{
    const int tid = threadIdx.x;
    const int ypad = 64;
    const int y_alloc = max_edges + max_rings + ypad;

    double x[U], y[U];
    int q[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t i = p0 + u * 256 + tid;
        x[u] = 0.0;
        y[u] = 0.0;
        q[u] = -1;
        if (i < n) {
            // read once: streamed past the caches
            x[u] = __builtin_nontemporal_load(px + i);
            y[u] = __builtin_nontemporal_load(py + i);
            q[u] = point_poly ? __builtin_nontemporal_load(point_poly + i) : 0;
        }
    }
    // the workgroup's range (uniform): pair ids, then offsets, while the
    // pairs' own loads are in flight
    const int64_t plast = (p0 + 256 * U < n ? p0 + 256 * U : n) - 1;
    int qf = 0, ql = 0;
    if (point_poly) {
        qf = point_poly[p0];
        ql = point_poly[plast];
    }
    const bool range_ok = (uint32_t)qf < (uint64_t)n_polys && (uint32_t)ql < (uint64_t)n_polys && qf <= ql;
    int64_t vb = 0, ve = 0;
    if (range_ok) {
        vb = offsets[qf];
        ve = offsets[ql + 1];
        clamp_ring(vb, ve, nv);
    }
    const int nr = ql - qf + 1;
    const int nvr = (int)(ve - vb);
    const bool fits = range_ok && nvr <= max_edges && nr <= max_rings;

    int *T = (int *)smem;
    size_t o = (((size_t)(max_rings + 1) * 4 + 15) & ~(size_t)15);
    RingInfo *R = (RingInfo *)(smem + o);
    o += (size_t)max_rings * 32;
    float *YF = (float *)(smem + o);
    o += ((((size_t)max_edges + max_rings + 64) * 4 + 15) & ~(size_t)15);
    float4 *EF = (float4 *)(smem + o);
    o += (size_t)max_edges * 16;
    double *XD = (double *)(smem + o);
    double *YD = XD + max_edges;
    o += (size_t)max_edges * 16;
    unsigned long long *KB = (unsigned long long *)(smem + o);   // per ring: x min, x max, y min, y max keys
    int *BAD = (int *)(KB + 4 * (size_t)max_rings);              // per ring: a normal out of the filter's range
    signed char *RID = (signed char *)(BAD + max_rings);         // per vertex: its ring (max_rings <= 128), or -1
    __shared__ int s_kmax;
    __shared__ unsigned s_rcnt, s_rbase;   // the item's undecided pairs, their list position

    // the ring table and the binary64 vertices in one round of loads
    if (tid == 0) {
        s_kmax = 0;
        s_rcnt = 0;
    }
    if (fits) {
        // YF starts as quiet NaNs: the straddle pass's minimum of |P_y - YF|
        // runs over every slot a lane reads, also past its ring (padding,
        // slots of rings without vertices), and a NaN leaves it unchanged
        for (int j = tid; j < y_alloc; j += 256)
            YF[j] = __int_as_float(0x7fc00000);
        for (int r = tid; r < nr; r += 256) {
            KB[4 * r + 0] = ~0ull;
            KB[4 * r + 1] = 0ull;
            KB[4 * r + 2] = ~0ull;
            KB[4 * r + 3] = 0ull;
            BAD[r] = 0;
        }
        for (int r = tid; r <= nr; r += 256) {
            int64_t ov = offsets[qf + r];
            ov = ov < vb ? vb : (ov > ve ? ve : ov);
            T[r] = (int)(ov - vb);
        }
        for (int e = tid; e < nvr; e += 256) {
            XD[e] = vx[vb + e];
            YD[e] = vy[vb + e];
        }
    }
    bool mine_ok = true;
#pragma unroll
    for (int u = 0; u < U; ++u)
        mine_ok = mine_ok && (q[u] < 0 || (q[u] >= qf && q[u] <= ql));
    __shared__ int s_all[4];
    const bool staged = block_all(fits && mine_ok, s_all);

    if (!staged) {
        // A vertex range larger than the binary32 layout's LDS budget, more
        // rings than its tables hold, or pairs not sorted by polygon: the
        // item is classified exactly in binary64 by the staged exact item,
        // which walks a large range in LDS tiles of tile_edges vertices (and
        // itself takes the scalar-load group walk when its tables cannot
        // hold the item or the pairs are unsorted).  Every thread has passed
        // the vote's barrier, so the LDS is free to be laid out anew.
        ItemRows<U> P;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            P.x[u] = x[u];
            P.y[u] = y[u];
            P.q[u] = q[u];
        }
        ItemRange R;
        R.vb = vb;
        R.rf = qf;
        R.qf = qf;
        R.ql = ql;
        R.nr = range_ok ? nr : 0;
        R.nv = nvr;
        R.ok = range_ok;
        staged_item_fp64<kSide, U, false, true>(p0, P, n, offsets, n_polys, nullptr, n_polys, vx, vy, nv, inside,
                                                tile_edges, max_rings, smem, R);
        return;
    }

    // Per ring: bounding box (LDS atomics on order keys, one thread per
    // vertex; the vertex's ring from a binary search of T, kept for the next
    // pass), then per vertex its binary32 records, each thread deriving the
    // ring's centre from the keys itself; the thread of a ring's first vertex
    // also stores the ring's centre, radius bound and eligibility.  A
    // vertex's predecessor is the ring's last vertex for its first vertex.
    for (int e = tid; e < nvr; e += 256) {
        const int r = ring_of_vertex(T, nr, e);
        RID[e] = (signed char)r;
        if (r < 0)
            continue;
        const double a = XD[e], b = YD[e];
        atomicMin(&KB[4 * r + 0], order_key(a));
        atomicMax(&KB[4 * r + 1], order_key(a));
        atomicMin(&KB[4 * r + 2], order_key(b));
        atomicMax(&KB[4 * r + 3], order_key(b));
        const int ep = e == T[r] ? T[r + 1] - 1 : e - 1;
        const double nx = b - YD[ep], ny = XD[ep] - a;   // the normal before orientation: the same magnitudes
        if (!(normal_ok(nx) && normal_ok(ny)))
            BAD[r] = 1;
    }
    for (int r = tid; r < nr; r += 256) {
        if (T[r + 1] <= T[r]) {   // no vertex: never filtered
            RingInfo ri;
            ri.cx = 0.0;
            ri.cy = 0.0;
            ri.m = -1.0f;
            R[r] = ri;
        }
    }
    __syncthreads();
    for (int e = tid; e < nvr; e += 256) {
        const int r = RID[e];
        if (r < 0)
            continue;
        const int e0 = T[r], e1 = T[r + 1];
        const double xmn = from_order_key(KB[4 * r + 0]), xmx = from_order_key(KB[4 * r + 1]);
        const double ymn = from_order_key(KB[4 * r + 2]), ymx = from_order_key(KB[4 * r + 3]);
        const double cx = 0.5 * xmn + 0.5 * xmx;
        const double cy = 0.5 * ymn + 0.5 * ymx;
        if (e == e0) {
            const double m = fmax(fmax(fabs(xmn - cx), fabs(xmx - cx)), fmax(fabs(ymn - cy), fabs(ymx - cy)));
            const bool ring_ok = !BAD[r] && m <= kLim;
            RingInfo ri;
            ri.cx = cx;
            ri.cy = cy;
            ri.m = ring_ok ? __double2float_ru(m) : -1.0f;
            R[r] = ri;
            atomicMax(&s_kmax, e1 - e0);
        }
        const int ep = e == e0 ? e1 - 1 : e - 1;
        const double ax = XD[ep], ay = YD[ep], bx = XD[e], by = YD[e];
        double nx = by - ay;
        double ny = ax - bx;
        if (nx < 0.0) {
            nx = -nx;
            ny = -ny;
        }
        // scaled to |n_x| + |n_y| = 1 (s > 0 for every edge that can straddle)
        const double sn = nx + fabs(ny);
        const double rs = sn > 0.0 ? 1.0 / sn : 0.0;
        EF[e] = make_float4((float)(ax - cx), (float)(ay - cy), (float)(nx * rs), (float)(ny * rs));
        const float yv = (float)(by - cy);
        YF[e + r + 1] = yv;
        if (e == e1 - 1)
            YF[e0 + r] = yv;
    }
    __syncthreads();
    const int kmax_b = s_kmax;

    const float ks = kBoundK * bound_scale;
    const float eta = kEta4 * bound_scale;
    uint64_t amb_rows[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t i = p0 + u * 256 + tid;
        const int r = (q[u] < 0 ? qf : q[u]) - qf;
        const int e0 = T[r];
        int k = T[r + 1] - e0;
        k = k < 0 ? 0 : k;
        const int yb = e0 + r;
        const RingInfo ri = R[r];
        const double xr = x[u] - ri.cx, yr = y[u] - ri.cy;
        const float PX = (float)xr, PY = (float)yr;
        bool amb = ri.m < 0.0f || !(fabs(xr) <= kLim) || !(fabs(yr) <= kLim) || force_recheck;
        const float mp = fmaxf(ri.m, fmaxf(fabsf(PX), fabsf(PY)));
        const float bnd = (ks * mp + eta) * kN1 + eta;   // B, the pair's threshold
        const float y_last = YF[yb];   // the ring's last vertex: the first edge's start
        uint32_t sgn = 0;   // bit 31: parity of the side values below zero
        uint32_t above_prev = (k > 0 && (__float_as_uint(PY - y_last) >> 31)) ? 1u : 0u;
        // smallest |P_y - YF| over the vertices read: zero when some vertex of
        // the ring has the point's binary32 y (undecided order); slots past
        // the ring hold NaN (ignored) or another ring's values (a zero there
        // only sends the pair to the recheck)
        float zmin = fabsf(PY - y_last);
        for (int c0 = 0; c0 < kmax_b; c0 += 32) {
            if (__builtin_amdgcn_ballot_w64(k > c0) == 0)
                break;
            uint32_t above = 0;   // sign bits of P_y - y_v: vertex above the point
            const int ybase = yb + 1 + c0;
            const float *yp = YF + (ybase < y_alloc - 32 ? ybase : y_alloc - 32);
            int t = 0;
            for (; t < 32; t += 4) {
                if (__builtin_amdgcn_ballot_w64(k > c0 + t) == 0)
                    break;
#pragma unroll
                for (int tt = 0; tt < 4; ++tt) {
                    const float d = PY - yp[t + tt];
                    zmin = fminf(zmin, fabsf(d));
                    above = __builtin_amdgcn_alignbit(above, __float_as_uint(d), 31);
                }
            }
            above = t < 32 ? above << (32 - t) : above;
            const int rem = k - c0;
            const uint32_t keep = rem <= 0 ? 0u : (rem >= 32 ? ~0u : ~(0xffffffffu >> rem));
            // reversed: bit b is the edge ending at chunk vertex b
            uint32_t strad = __builtin_bitreverse32((above ^ ((above >> 1) | (above_prev << 31))) & keep);
            above_prev = rem >= 32 ? (above & 1u) : above_prev;
            const float4 *er = EF + e0 + c0;
            while (strad != 0) {
                const int b = __builtin_ctz(strad);
                strad &= strad - 1u;
                const float4 rec = er[b];
                const float t1 = PX - rec.x;
                const float t2 = PY - rec.y;
                const float p1 = t1 * rec.z;
                const float p2 = t2 * rec.w;
                const float sv = p1 + p2;
                amb = amb || !(fabsf(sv) > bnd);
                // the edge counts when the side value is <= 0; a zero value
                // is undecided (|sv| > bnd fails), so for every decided pair
                // that is the sign bit
                sgn ^= __float_as_uint(sv);
            }
        }
        amb = amb || zmin == 0.0f;
        const bool valid = i < n;
        amb_rows[u] = __builtin_amdgcn_ballot_w64(valid && amb);
        if (valid && !amb)
            inside[i] = (uint8_t)(sgn >> 31);
    }
    append_recheck_item<U>(amb_rows, p0, recheck, recheck_count, &s_rcnt, &s_rbase);
}

// One workgroup per item (QUEUE false: workgroup b takes item order[b], or
// b), or a resident grid taking items from an atomic counter (QUEUE true).
// The two forms are separate kernels, each compiled with only its own
// control flow and registers.  The one-item form runs at eight waves per
// SIMD: at that register budget it keeps its pair loads in flight while the
// ring table and vertices are staged (no spill reload waits on them).
template <int U, bool QUEUE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(QUEUE ? 1 : 8))) void k_filtered_fp32(
    const double *__restrict__ px, const double *__restrict__ py, int64_t n,
    const int64_t *__restrict__ offsets, int64_t n_polys,
    const double *__restrict__ vx, const double *__restrict__ vy, int64_t nv,
    const int32_t *__restrict__ point_poly, uint8_t *__restrict__ inside, int max_edges, int max_rings,
    int tile_edges, float bound_scale, int force_recheck, int32_t *__restrict__ recheck, unsigned *recheck_count,
    const int32_t *__restrict__ order, int n_items, unsigned *queue)
{
    extern __shared__ __align__(16) unsigned char smem[];
    if (!QUEUE) {
        const int item = order ? order[blockIdx.x] : (int)blockIdx.x;
        filtered_item<U>((int64_t)item * (256 * U), px, py, n, offsets, n_polys, vx, vy, nv, point_poly, inside,
                         max_edges, max_rings, tile_edges, bound_scale, force_recheck, recheck, recheck_count, smem);
        return;
    }
    __shared__ int s_item;
    for (;;) {
        if (threadIdx.x == 0)
            s_item = (int)atomicAdd(queue, 1u);
        __syncthreads();
        const int it = s_item;
        __syncthreads();
        if (it >= n_items)
            break;
        const int item = order ? order[it] : it;
        filtered_item<U>((int64_t)item * (256 * U), px, py, n, offsets, n_polys, vx, vy, nv, point_poly, inside,
                         max_edges, max_rings, tile_edges, bound_scale, force_recheck, recheck, recheck_count, smem);
        __syncthreads();
    }
}

// The rule's binary64 crossing test for edge (a, b) against point (x, y):
// half-open straddle, then the side value with the oriented normal, each
// operation separately rounded.
__device__ __forceinline__ unsigned rule_crossing(double x, double y, double ax, double ay, double bx, double by)
{
    if ((ay > y) == (by > y))
        return 0u;
    double nx = by - ay;
    double ny = ax - bx;
    if (nx < 0.0) {
        nx = -nx;
        ny = -ny;
    }
    const double t1 = x - ax;
    const double t2 = y - ay;
    const double s = t1 * nx + t2 * ny;
    return s <= 0.0 ? 1u : 0u;
}

constexpr int64_t kRecheckWide = 64;   // rings longer than this are walked by a whole wavefront

__device__ __forceinline__ int64_t readlane64(int64_t v, int lane)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), lane);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ double readlane_f64(double v, int lane)
{
    return __longlong_as_double(readlane64(__double_as_longlong(v), lane));
}

// Binary64 recheck, in the rule's operation order, of the listed pairs, in
// two kernels over the list with fixed grids (the lengths are read on the
// device, so the launches do not depend on them: graph-safe):
//   1. k_recheck_lanes: every pair whose ring has at most kRecheckWide
//      vertices is walked by one lane, four vertices' loads issued together;
//      a longer ring's pair is appended to a second list in the free tail of
//      the same array (one counter, aggregated per wavefront), or, when the
//      tail is full, walked by its lane as well;
//   2. k_recheck_wide: one wavefront per appended pair, lane l taking edges
//      l, l + 64, ... (coalesced loads, four edges per round), the
//      crossings' parity gathered with one ballot.  (A wavefront taking a run
//      of long pairs in turn took 0.68 ms for 592 pairs of 4096-vertex rings;
//      a wavefront per list entry paid the list's load chain for every entry.)
__device__ __forceinline__ void recheck_ring(const double *__restrict__ px, const double *__restrict__ py,
                                             const int64_t *__restrict__ offsets, int64_t n_polys,
                                             int64_t nv, const int32_t *__restrict__ point_poly, int64_t i,
                                             double &x, double &y, int64_t &b, int64_t &e)
{
    int64_t qq = point_poly ? (int64_t)point_poly[i] : 0;
    qq = ((uint64_t)qq < (uint64_t)n_polys) ? qq : 0;
    b = offsets[qq];
    e = offsets[qq + 1];
    clamp_ring(b, e, nv);
    x = px[i];
    y = py[i];
}

__global__ __launch_bounds__(256) void k_recheck_lanes(
    const double *__restrict__ px, const double *__restrict__ py,
    const int64_t *__restrict__ offsets, int64_t n_polys,
    const double *__restrict__ vx, const double *__restrict__ vy, int64_t nv,
    const int32_t *__restrict__ point_poly, uint8_t *__restrict__ inside,
    int32_t *list, const unsigned *__restrict__ count, unsigned *wide_count, int64_t cap)
{
    int64_t m = (int64_t)*count;
    m = m < cap ? m : cap;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < m; t += stride) {
        const int64_t i = list[t];
        double x, y;
        int64_t b, e;
        recheck_ring(px, py, offsets, n_polys, nv, point_poly, i, x, y, b, e);
        if (e - b > kRecheckWide) {
            const int64_t at = m + (int64_t)atomicAdd(wide_count, 1u);
            if (at < cap) {
                list[at] = (int32_t)i;
                continue;
            }
        }
        unsigned par = 0;
        if (e > b) {
            double ax = vx[e - 1], ay = vy[e - 1];
            int64_t j = b;
            for (; j + 4 <= e; j += 4) {
                double bx[4], by[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    bx[u] = vx[j + u];
                    by[u] = vy[j + u];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    par ^= rule_crossing(x, y, ax, ay, bx[u], by[u]);
                    ax = bx[u];
                    ay = by[u];
                }
            }
            for (; j < e; ++j) {
                const double bx = vx[j], by = vy[j];
                par ^= rule_crossing(x, y, ax, ay, bx, by);
                ax = bx;
                ay = by;
            }
        }
        inside[i] = (uint8_t)par;
    }
}

__global__ __launch_bounds__(256) void k_recheck_wide(
    const double *__restrict__ px, const double *__restrict__ py,
    const int64_t *__restrict__ offsets, int64_t n_polys,
    const double *__restrict__ vx, const double *__restrict__ vy, int64_t nv,
    const int32_t *__restrict__ point_poly, uint8_t *__restrict__ inside,
    const int32_t *__restrict__ list, const unsigned *__restrict__ count,
    const unsigned *__restrict__ wide_count, int64_t cap)
{
    int64_t m = (int64_t)*count;
    m = m < cap ? m : cap;
    int64_t nw = (int64_t)*wide_count;
    nw = nw < cap - m ? nw : cap - m;
    const int lane = threadIdx.x & 63;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    // the loop bound is the same for every lane of a wavefront
    for (int64_t t = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; t < nw; t += nwaves) {
        const int64_t i = list[m + t];
        double x, y;
        int64_t b, e;
        recheck_ring(px, py, offsets, n_polys, nv, point_poly, i, x, y, b, e);
        const int64_t k = e - b;
        unsigned lp = 0;
        int64_t j = lane;
        for (; j + 192 < k; j += 256) {
            double ax[4], ay[4], bx[4], by[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t jj = j + 64 * u;
                const int64_t ja = jj == 0 ? k - 1 : jj - 1;
                ax[u] = vx[b + ja];
                ay[u] = vy[b + ja];
                bx[u] = vx[b + jj];
                by[u] = vy[b + jj];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
                lp ^= rule_crossing(x, y, ax[u], ay[u], bx[u], by[u]);
        }
        for (; j < k; j += 64) {
            const int64_t ja = j == 0 ? k - 1 : j - 1;
            lp ^= rule_crossing(x, y, vx[b + ja], vy[b + ja], vx[b + j], vy[b + j]);
        }
        const unsigned odd = (unsigned)__builtin_popcountll(__builtin_amdgcn_ballot_w64(lp != 0)) & 1u;
        if (lane == 0)
            inside[i] = (uint8_t)odd;
    }
}

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

}  // namespace

int launch_filtered(const Problem &p, hipStream_t stream, int pairs_per_lane, int max_edges, float bound_scale,
                    int force_recheck, int32_t *recheck, unsigned *recheck_count, const int32_t *order,
                    int n_items, unsigned *queue, int grid)
{
    if (p.poly_rings)
        return fail(PIP_ENOTSUP, "the filtered mode takes one ring per polygon");
    const int U = pairs_per_lane == 1 ? 1 : (pairs_per_lane == 4 ? 4 : 2);
    const int max_rings = 256 * U < 128 ? 256 * U : 128;
    const size_t shmem = filtered_smem_bytes(max_edges, max_rings);
    // the exact layout's tile for items beyond the binary32 layout: the
    // largest size (in steps of 16 vertices) whose staged layout fits the
    // same LDS; at 16 edges it needs less than the binary32 layout
    int tile_edges = max_edges;
    while (tile_edges > 16 && staged_smem_bytes(tile_edges, max_rings) > shmem)
        tile_edges -= 16;
    if (staged_smem_bytes(tile_edges, max_rings) > shmem)
        return fail(PIP_EINVAL, "LDS budget of %d edges too small for the filtered mode", max_edges);
    if (!queue)
        grid = n_items;
    if (grid <= 0)
        return PIP_OK;
#define PIP_LAUNCH_F(UU, QQ)                                                                                     \
    PIP_LAUNCH((k_filtered_fp32<UU, QQ>), dim3(grid), dim3(256), shmem, stream, p.px, p.py, p.n_points,             \
               p.offsets, p.n_polys, p.vx, p.vy, p.n_vertices, p.point_poly, p.inside, max_edges, max_rings,       \
               tile_edges, bound_scale, force_recheck, recheck, recheck_count, order, n_items, queue)
    if (U == 1) {
        if (queue)
            PIP_LAUNCH_F(1, true);
        else
            PIP_LAUNCH_F(1, false);
    } else if (U == 4) {
        if (queue)
            PIP_LAUNCH_F(4, true);
        else
            PIP_LAUNCH_F(4, false);
    } else {
        if (queue)
            PIP_LAUNCH_F(2, true);
        else
            PIP_LAUNCH_F(2, false);
    }
#undef PIP_LAUNCH_F
    PIP_HIP_TRY(hipGetLastError());
    return PIP_OK;
}

int filtered_occupancy(int pairs_per_lane, int max_edges, int *blocks_per_cu)
{
    const int U = pairs_per_lane == 1 ? 1 : (pairs_per_lane == 4 ? 4 : 2);
    const int max_rings = 256 * U < 128 ? 256 * U : 128;
    const size_t shmem = filtered_smem_bytes(max_edges, max_rings);
    int nb = 0;
    hipError_t e;
    if (U == 1)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_filtered_fp32<1, true>, 256, shmem);
    else if (U == 4)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_filtered_fp32<4, true>, 256, shmem);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_filtered_fp32<2, true>, 256, shmem);
    if (e != hipSuccess)
        return fail(PIP_EHIP, "occupancy query failed: %s", hipGetErrorString(e));
    *blocks_per_cu = nb < 1 ? 1 : nb;
    return PIP_OK;
}

int launch_recheck(const Problem &p, hipStream_t stream, int32_t *list, const unsigned *count,
                   unsigned *wide_count, int grid)
{
    if (p.poly_rings)
        return fail(PIP_ENOTSUP, "the filtered mode takes one ring per polygon");
    hipLaunchKernelGGL(k_recheck_lanes, dim3(grid), dim3(256), 0, stream, p.px, p.py, p.offsets, p.n_polys, p.vx,
                       p.vy, p.n_vertices, p.point_poly, p.inside, list, count, wide_count, (int64_t)p.n_points);
    hipLaunchKernelGGL(k_recheck_wide, dim3(grid), dim3(256), 0, stream, p.px, p.py, p.offsets, p.n_polys, p.vx,
                       p.vy, p.n_vertices, p.point_poly, p.inside, list, count, wide_count, (int64_t)p.n_points);
    PIP_HIP_TRY(hipGetLastError());
    return PIP_OK;
}

}  // namespace pip
