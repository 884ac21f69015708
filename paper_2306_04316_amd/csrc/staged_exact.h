// The staged binary64 work item shared by the exact kernels and the filtered
// kernel: one workgroup classifies 256*U consecutive pairs (sorted by
// polygon) with their rings staged in LDS, walking vertex ranges larger than
// the LDS budget in tiles (paper, Method section, constraint 1 or 2 per
// edge, and Algorithm 1, half-open straddle reading).  Include only from
// .hip files compiled with -ffp-contract=off.
#pragma once

#include "pip_common.h"
#include "ring_walk.h"

namespace pip {
namespace {

// ---------------------------------------------------------------- staged (rings in LDS, compacted side tests)
// A workgroup owns 256*U consecutive pairs (thread t, row u: pair
// base + 256u + t).  When the pairs are sorted by polygon, the rings they test
// form one contiguous vertex range [vb, ve).  The workgroup stages it once in
// LDS, all threads together (one coalesced load per vertex, edges of every
// ring in parallel):
//   T  : ring starts relative to vb (T[r] .. T[r+1]-1 are ring r's vertices)
//   Y  : y of every vertex of the range (the straddle pass input)
//   XR : x of every vertex (only to build E)
//   E  : per edge j = (v_{j-1}, v_j) of its ring, the record (a_x, a_y, n_x, n_y)
//        with the normal n = (b_y - a_y, a_x - b_x) negated when n_x < 0,
//        computed in binary64 exactly as the rule states (so the side value
//        below is the rule's, bit for bit).  Every vertex's record is first
//        built from the vertex stored before it; then each ring's first
//        record is rebuilt from the ring's last vertex (closing edge).
// Each lane then runs two phases per 32-vertex chunk of its own ring:
//   1. straddle pass: above_j = (y_j > p_y) for every vertex (one compare,
//      exact), shifted into a 32-bit word; straddle bits = above XOR above
//      shifted by one (half-open rule);
//   2. side tests only for its straddling edges, taken one set bit at a time:
//      s = (p_x - a_x) * n_x + (p_y - a_y) * n_y, crossing iff s <= 0.
// Only about 2 of a footprint's edges straddle a given point, so phase 2 is
// short; phase 1 costs two vector instructions per vertex.  A polygon of
// several rings that together fit one chunk takes a single pass over all of
// them (staged_poly_parity1); otherwise its rings are walked one by one.
// A vertex range larger than the LDS budget is walked in tiles (the TILES
// form); in the plain form such an item, like one whose pairs are not sorted
// by polygon, takes the scalar-load group walk.
struct StagedLds {
    int *T;    // ring starts, relative to the range start
    int *PR;   // polygons of several rings: first ring of each polygon (relative)
    double *Y;
    double *XR;
    double4 *E;
};

__device__ __forceinline__ StagedLds staged_lds(unsigned char *smem, int max_edges, int max_rings)
{
    StagedLds L;
    L.T = (int *)smem;
    size_t o = (((size_t)(max_rings + 1) * 4 + 31) & ~(size_t)31);
    L.PR = (int *)(smem + o);
    o += (((size_t)(max_rings + 1) * 4 + 31) & ~(size_t)31);
    L.Y = (double *)(smem + o);
    o += (((size_t)max_edges + 64) * 8 + 31) & ~(size_t)31;
    L.XR = (double *)(smem + o);
    o += ((size_t)max_edges * 8 + 31) & ~(size_t)31;
    L.E = (double4 *)(smem + o);
    return L;
}

// Ring of staged vertex e: the r with T[r] <= e < T[r+1] (T sorted, T[0] = 0,
// T[nr] > e).  Returns -1 when the table is not sorted around e (offsets that
// are not monotone; such inputs have unspecified results, but every access
// stays inside the staged range).
__device__ __forceinline__ int staged_ring_of(const int *T, int nr, int e)
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

// Where a work item's rings lie: the polygons qf..ql of its first and last
// pair (pairs sorted by polygon), their rings rf .. rf+nr-1 and the vertex
// range [vb, vb + nv).  `ok` is false when the ids are out of range or not
// ordered.  Without a ring index (MR false), ring q is polygon q.
struct ItemRange {
    int64_t vb;
    int64_t rf;
    int qf, ql;
    int nr;
    int nv;
    int ok;
};

template <bool MR>
__device__ __forceinline__ ItemRange item_range(int64_t p0, int64_t pairs, int64_t n,
                                                const int64_t *__restrict__ offsets, int64_t n_polys,
                                                const int64_t *__restrict__ poly_rings, int64_t n_rings, int64_t nv,
                                                const int32_t *__restrict__ point_poly)
{
    ItemRange R;
    const int64_t plast = (p0 + pairs < n ? p0 + pairs : n) - 1;
    R.qf = 0;
    R.ql = 0;
    if (point_poly) {
        R.qf = point_poly[p0];
        R.ql = point_poly[plast];
    }
    R.ok = (uint32_t)R.qf < (uint64_t)n_polys && (uint32_t)R.ql < (uint64_t)n_polys && R.qf <= R.ql;
    int64_t vb = 0, ve = 0, rf = 0, rl = 0;
    if (R.ok) {
        if (MR) {
            rf = poly_rings[R.qf];
            rl = poly_rings[R.ql + 1];
            rf = rf < 0 ? 0 : (rf > n_rings ? n_rings : rf);
            rl = rl < rf ? rf : (rl > n_rings ? n_rings : rl);
        } else {
            rf = R.qf;
            rl = (int64_t)R.ql + 1;
        }
        vb = offsets[rf];
        ve = offsets[rl];
        clamp_ring(vb, ve, nv);
    }
    R.vb = vb;
    R.rf = rf;
    R.nr = rl - rf > INT32_MAX ? INT32_MAX : (int)(rl - rf);
    R.nv = (int)(ve - vb);   // clamp_ring keeps it within [0, INT32_MAX]
    return R;
}

// Crossing parity of every lane's point against its staged ring: edges
// e0 .. e0+k-1 (k = 0: nothing).  Two phases per 32-vertex chunk:
//   1. straddle pass: above_j = (y_j > p_y) for every vertex (one compare,
//      exact), shifted into a 32-bit word, vertex j of the chunk at bit 31-j;
//      straddle bits = above XOR above shifted by one (half-open rule);
//   2. side tests only for the lane's straddling edges, taken from the
//      bit-reversed straddle word (bit b: the edge ending at chunk vertex b,
//      so its record sits at a fixed stride from the chunk's first), lowest
//      set bit first (the order of the tests does not matter: only their
//      count's parity).
// Returns the lane's parity (0 or 1).  Must be called by the whole wavefront.
// above_prev: the above bit of the vertex before e0 in the ring (for a whole
// ring, its last vertex); with own_prev set (a whole ring of at most 32
// vertices) it is taken from the straddle pass itself, where the last
// vertex's bit lies at 32-k.
template <int PRED>
__device__ __forceinline__ uint32_t staged_ring_parity(const StagedLds &L, int e0, int k, uint32_t above_prev,
                                                       bool own_prev, double xu, double yu, int max_edges,
                                                       int y_alloc)
{
    const double yq = yu + 0.0;
    uint32_t cnt = 0;
    for (int c0 = 0; c0 < max_edges; c0 += 32) {
        if (__builtin_amdgcn_ballot_w64(k > c0) == 0)
            break;
        // phase 1: above bits of vertices c0 .. c0+31, first vertex in bit 31
        uint32_t above = 0;
        // Lanes whose ring ended read past it (their bits are masked below);
        // the clamp keeps those reads inside the Y allocation.  A lane still
        // inside its ring is never clamped: its chunk starts at most at the
        // last staged vertex, 64 slots before the end.
        const int ybase = e0 + c0;
        const double *yr = L.Y + (ybase < y_alloc - 32 ? ybase : y_alloc - 32);
        int t = 0;
        for (; t < 32; t += 4) {
            if (__builtin_amdgcn_ballot_w64(k > c0 + t) == 0)
                break;
#pragma unroll
            for (int tt = 0; tt < 4; ++tt)
                above = shift_in_above(above, yq, yr[t + tt]);
        }
        above = t < 32 ? above << (32 - t) : above;
        if (c0 == 0 && own_prev)
            above_prev = (above >> ((32 - k) & 31)) & 1u;
        uint32_t strad = above ^ ((above >> 1) | (above_prev << 31));
        // keep the bits of the lane's rem = k - c0 chunk vertices (none when
        // rem <= 0, all when rem >= 32): the top rem bits
        const int rem = k - c0;
        const int rc = rem < 0 ? 0 : (rem > 32 ? 32 : rem);
        strad &= (uint32_t)(0xffffffff00000000ull >> rc);
        above_prev = rem >= 32 ? (above & 1u) : above_prev;
        // phase 2: side tests for this lane's straddling edges only; after
        // the reversal bit b is the edge ending at chunk vertex b
        strad = __builtin_bitreverse32(strad);
        const double4 *er = L.E + (e0 + c0);
        while (strad != 0) {
            const int b = __builtin_ctz(strad);
            strad &= strad - 1u;
            const double4 rec = er[b];
            bool cr;
            if (PRED == kIntersection) {
                const double lam = (yu - rec.y) / rec.w;
                const double xn = rec.x + lam * rec.z;
                cr = xn >= xu;
            } else {
                const double t1 = xu - rec.x;
                const double t2 = yu - rec.y;
                const double sv = t1 * rec.z + t2 * rec.w;
                cr = sv <= 0.0;
            }
            cnt += cr ? 1u : 0u;
        }
    }
    return cnt & 1u;
}

// Classify the 256*U pairs starting at p0 (one workgroup, 256 threads).
// smem: dynamic LDS of staged_smem_bytes(max_edges, max_rings) bytes.
// Edge records: constraint 1 stores (a_x, a_y, n_x, n_y) with the normal
// oriented n_x > 0; constraint 2 stores (a_x, a_y, d_x, d_y), d = b - a.
// MR: polygons of several rings; the lane XORs the parities of its
// polygon's rings (PR[j] .. PR[j+1]-1 in the staged ring table).
// Rings larger than the LDS edge budget are walked in tiles (see below);
// only items with more rings or polygons than the tables hold, or with pairs
// not sorted by polygon, take the scalar-load group walk.
// Crossing parity of every lane's point against all rings of its polygon in
// one pass, when the polygon's rings (rings r0 .. r1-1 of the staged table,
// back to back from staged vertex e0, k <= 32 vertices in all) lie in one
// chunk.  The straddle pass runs along the stored order; the bit of each
// ring's first edge is then corrected to compare the ring's first vertex with
// its own last vertex (its closing edge) instead of the previous ring's last
// vertex.  The records of those closing edges are the ones staged at the
// rings' first vertices, so the side tests are the per-ring walk's.  Returns
// the lane's parity, the XOR over the rings.  Whole wavefront; T_base: the
// staged position of the tile (or range) start.
template <int PRED>
__device__ __forceinline__ uint32_t staged_poly_parity1(const StagedLds &L, int e0, int k, int r0, int r1,
                                                        int T_base, double xu, double yu, int y_alloc)
{
    const double yq = yu + 0.0;
    uint32_t above = 0;
    const double *yr = L.Y + (e0 < y_alloc - 32 ? e0 : y_alloc - 32);
    int t = 0;
    for (; t < 32; t += 4) {
        if (__builtin_amdgcn_ballot_w64(k > t) == 0)
            break;
#pragma unroll
        for (int tt = 0; tt < 4; ++tt)
            above = shift_in_above(above, yq, yr[t + tt]);
    }
    above = t < 32 ? above << (32 - t) : above;
    uint32_t strad = above ^ (above >> 1);   // the first vertex's predecessor: fixed below
    for (int step = 0;; ++step) {
        const int rr = r0 + step;
        const bool act = rr < r1;
        if (__builtin_amdgcn_ballot_w64(act) == 0)
            break;
        if (act) {
            const int s = L.T[rr] - T_base - e0, e = L.T[rr + 1] - T_base - e0;   // ring rr: [s, e)
            if (e > s && s >= 0 && e <= k) {
                const uint32_t last = (above >> (31 - (e - 1))) & 1u;
                const uint32_t before = s > 0 ? (above >> (32 - s)) & 1u : 0u;
                strad ^= (before ^ last) << (31 - s);
            }
        }
    }
    const int kc = k < 0 ? 0 : (k > 32 ? 32 : k);
    strad &= (uint32_t)(0xffffffff00000000ull >> kc);
    uint32_t cnt = 0;
    // after the reversal bit b is the edge ending at chunk vertex b
    strad = __builtin_bitreverse32(strad);
    const double4 *er = L.E + e0;
    while (strad != 0) {
        const int b = __builtin_ctz(strad);
        strad &= strad - 1u;
        const double4 rec = er[b];
        bool cr;
        if (PRED == kIntersection) {
            const double lam = (yu - rec.y) / rec.w;
            const double xn = rec.x + lam * rec.z;
            cr = xn >= xu;
        } else {
            const double t1 = xu - rec.x;
            const double t2 = yu - rec.y;
            const double sv = t1 * rec.z + t2 * rec.w;
            cr = sv <= 0.0;
        }
        cnt += cr ? 1u : 0u;
    }
    return cnt & 1u;
}

// The staged record of edge (a, b): constraint 1 stores (a_x, a_y, n_x, n_y)
// with the normal n = (b_y - a_y, a_x - b_x) negated when n_x < 0, constraint
// 2 stores (a_x, a_y, d_x, d_y), d = b - a; binary64, as the rule states.
template <int PRED>
__device__ __forceinline__ double4 edge_record(double ax, double ay, double bx, double by)
{
    if (PRED == kIntersection)
        return make_double4(ax, ay, bx - ax, by - ay);
    double nx = by - ay;
    double ny = ax - bx;
    if (nx < 0.0) {
        nx = -nx;
        ny = -ny;
    }
    return make_double4(ax, ay, nx, ny);
}

// The thread's pairs of the item starting at p0 (row u: pair p0 + 256u + tid),
// read once and streamed past the caches.  q = -1 past the end.
template <int U>
struct ItemRows {
    double x[U], y[U];
    int q[U];
};

template <int U>
__device__ __forceinline__ ItemRows<U> load_rows(int64_t p0, const double *__restrict__ px,
                                                 const double *__restrict__ py, int64_t n,
                                                 const int32_t *__restrict__ point_poly)
{
    ItemRows<U> P;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t i = p0 + u * 256 + threadIdx.x;
        P.x[u] = 0.0;
        P.y[u] = 0.0;
        P.q[u] = -1;
        if (i < n) {
            P.x[u] = __builtin_nontemporal_load(px + i);
            P.y[u] = __builtin_nontemporal_load(py + i);
            P.q[u] = point_poly ? __builtin_nontemporal_load(point_poly + i) : 0;
        }
    }
    return P;
}

template <int PRED, int U, bool MR, bool TILES>
__device__ __forceinline__ void staged_item_fp64(
    int64_t p0, const ItemRows<U> &P, int64_t n, const int64_t *__restrict__ offsets, int64_t n_polys,
    const int64_t *__restrict__ poly_rings, int64_t n_rings, const double *__restrict__ vx,
    const double *__restrict__ vy, int64_t nv, uint8_t *__restrict__ inside, int max_edges, int max_rings,
    unsigned char *smem, const ItemRange R)
{
    const int tid = threadIdx.x;
    const int ypad = 64;
    const int y_alloc = max_edges + ypad;
    const double(&x)[U] = P.x;
    const double(&y)[U] = P.y;
    const int(&q)[U] = P.q;

    // the workgroup's range (the same for every thread, so `tables` and `fits`
    // are uniform)
    const int qf = R.qf, ql = R.ql;
    const int64_t vb = R.vb, ve = R.vb + R.nv;
    const int np = ql - qf + 1;   // polygons
    const int nr = R.nr;          // rings
    const int nvr = R.nv;
    const bool tables = R.ok && nr <= max_rings && np <= max_rings;
    const bool fits = tables && nvr <= max_edges;

    const StagedLds L = staged_lds(smem, max_edges, max_rings);
    // First round of the ring table and of the vertices: one entry of each
    // per thread, their loads issued together (one memory round trip); larger
    // tables and ranges continue in the loops below.
    {
        const bool hr = tables && tid <= nr;
        const bool hv = fits && tid < nvr;
        int64_t o = 0;
        double ax = 0.0, ay = 0.0;
        if (hr)
            o = offsets[R.rf + tid];
        if (hv) {
            ax = vx[vb + tid];
            ay = vy[vb + tid];
        }
        if (hr) {
            o = o < vb ? vb : (o > ve ? ve : o);
            L.T[tid] = (int)(o - vb);
        }
        if (hv) {
            L.XR[tid] = ax;
            L.Y[tid] = ay;
        }
    }
    if (tables) {
        for (int r = tid + 256; r <= nr; r += 256) {
            int64_t o = offsets[R.rf + r];
            o = o < vb ? vb : (o > ve ? ve : o);
            L.T[r] = (int)(o - vb);
        }
        if (MR) {
            for (int j = tid; j <= np; j += 256) {
                int64_t g = poly_rings[qf + j] - R.rf;
                g = g < 0 ? 0 : (g > nr ? nr : g);
                L.PR[j] = (int)g;
            }
        }
    }
    if (fits) {
        for (int e = tid + 256; e < nvr; e += 256) {
            L.XR[e] = vx[vb + e];
            L.Y[e] = vy[vb + e];
        }
        if (tid < ypad)
            L.Y[nvr + tid] = 0.0;
    }
    // every pair's polygon inside the staged range (the pairs' own loads are
    // first waited for here, after the staging loads went out)
    bool mine_ok = true;
#pragma unroll
    for (int u = 0; u < U; ++u)
        mine_ok = mine_ok && (q[u] < 0 || (q[u] >= qf && q[u] <= ql));
    __shared__ int s_all[4];
    const bool staged = block_all(tables && mine_ok && (TILES || fits), s_all);

    if (staged) {
        // The vertex range in tiles of S = max_edges vertices: one tile when it
        // fits (staged above with coalesced loads), else the workgroup walks it
        // tile by tile.  Per tile: the edge records of the edges ending in the
        // tile (and, for a tiled range, their y values, with endpoints read
        // from global memory, cached by the previous tile's loads); then every
        // lane runs the straddle pass and side tests over the part of its
        // ring(s) inside the tile, starting from the above bit of the part's
        // predecessor in the ring, and accumulates its parity across tiles.
        const int S = max_edges;
        uint32_t mine = 0;   // bit u: this lane's parity for row u
        for (int t0 = 0; t0 < nvr; t0 += S) {
            const int t1 = (!TILES || nvr - t0 < S) ? nvr : t0 + S;
            if (!TILES || fits) {
                // the whole range is staged: every vertex's record takes its
                // stored predecessor, then each ring's first record is redone
                // with the ring's last vertex (no search for a vertex's ring)
                for (int e = tid; e < nvr; e += 256) {
                    const int ep = e > 0 ? e - 1 : 0;
                    L.E[e] = edge_record<PRED>(L.XR[ep], L.Y[ep], L.XR[e], L.Y[e]);
                }
                __syncthreads();
                for (int r = tid; r < nr; r += 256) {
                    const int e0 = L.T[r], e1 = L.T[r + 1];
                    if (e0 < e1)
                        L.E[e0] = edge_record<PRED>(L.XR[e1 - 1], L.Y[e1 - 1], L.XR[e0], L.Y[e0]);
                }
            } else {
                for (int e = t0 + tid; e < t1; e += 256) {
                    const int r = staged_ring_of(L.T, nr, e);
                    if (r < 0)
                        continue;
                    const int e0 = L.T[r];
                    const int ep = e == e0 ? L.T[r + 1] - 1 : e - 1;
                    const double by = vy[vb + e];
                    L.E[e - t0] = edge_record<PRED>(vx[vb + ep], vy[vb + ep], vx[vb + e], by);
                    L.Y[e - t0] = by;
                }
            }
            if (TILES && !fits && tid < ypad)
                L.Y[(t1 - t0) + tid] = 0.0;
            __syncthreads();

#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int j = (q[u] < 0 ? qf : q[u]) - qf;
                // the polygon's rings, in step across the wavefront (lanes
                // whose polygon has fewer rings run the extra steps with k = 0)
                int r0 = j, r1 = j + 1;
                if (MR) {
                    r0 = L.PR[j];
                    r1 = L.PR[j + 1];
                    r1 = r1 < r0 ? r0 : r1;
                }
                uint32_t par = 0;
                if (MR) {
                    // all of the polygon's rings in one chunk of this tile: one pass
                    const int pa = L.T[r0], pb = L.T[r1];
                    const bool one = pb >= pa && pb - pa <= 32 && pa >= t0 && pb <= t1;
                    if (__builtin_amdgcn_ballot_w64(!one) == 0) {
                        par = staged_poly_parity1<PRED>(L, pa - t0, pb - pa, r0, r1, t0, x[u], y[u], y_alloc);
                        mine ^= par << u;
                        continue;
                    }
                }
                for (int step = 0;; ++step) {
                    const int rr = r0 + step;
                    const bool act = rr < r1;
                    if (MR && __builtin_amdgcn_ballot_w64(act) == 0)
                        break;
                    const int rs = act ? rr : 0;
                    const int e0 = L.T[rs], e1 = L.T[rs + 1];
                    // the ring's part in this tile: [a, b)
                    const int a = (TILES && e0 < t0) ? t0 : e0;
                    const int b = (TILES && e1 > t1) ? t1 : e1;
                    const int k = act && b > a ? b - a : 0;
                    // the above bit of the part's predecessor: from the pass itself
                    // for a whole ring within one chunk, else read
                    const bool own = a == e0 && b == e1 && k <= 32;
                    uint32_t prev = 0;
                    if (k > 0 && !own) {
                        const int pred = a == e0 ? e1 - 1 : a - 1;
                        double yp;
                        if (TILES && !(pred >= t0 && pred < t1))
                            yp = vy[vb + pred];
                        else
                            yp = L.Y[pred - t0];
                        prev = yp > y[u] ? 1u : 0u;
                    }
                    par ^= staged_ring_parity<PRED>(L, a - t0, k, prev, own, x[u], y[u], S, y_alloc);
                    if (!MR)
                        break;
                }
                mine ^= par << u;
            }
            if (TILES && t1 < nvr)
                __syncthreads();   // the next tile overwrites Y and E
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = p0 + u * 256 + tid;
            if (i < n)
                inside[i] = (uint8_t)((mine >> u) & 1u);
        }
        return;
    }

    // fallback: groups of lanes sharing a polygon, rings streamed through scalar loads
    group_walk_rows<PRED, U, MR>(p0, x, y, q, n, offsets, n_polys, poly_rings, n_rings, vx, vy, nv, inside);
}

// The range as wave-uniform values (the table entries below are read from
// LDS by every lane at the same address).
__device__ __forceinline__ ItemRange uniform_range(const ItemRange &R)
{
    ItemRange U;
    const uint64_t vb = (uint64_t)R.vb;
    U.vb = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(vb >> 32)) << 32) |
                     (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)vb));
    const uint64_t rf = (uint64_t)R.rf;
    U.rf = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(rf >> 32)) << 32) |
                     (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)rf));
    U.qf = __builtin_amdgcn_readfirstlane(R.qf);
    U.ql = __builtin_amdgcn_readfirstlane(R.ql);
    U.nr = __builtin_amdgcn_readfirstlane(R.nr);
    U.nv = __builtin_amdgcn_readfirstlane(R.nv);
    U.ok = __builtin_amdgcn_readfirstlane(R.ok);
    return U;
}

}  // namespace
}  // namespace pip
