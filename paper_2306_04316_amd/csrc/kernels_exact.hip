// Exact binary64 kernels for the constraint-1 ray-casting test (paper,
// Method section, constraint 1, and Algorithm 1, half-open straddle reading):
// the plain per-pair baseline, the wave-segmented kernel, and the staged
// kernel with rings in LDS.  The per-edge arithmetic is in ring_walk.h.
//
// This translation unit must be compiled with -ffp-contract=off.

#include "pip_common.h"
#include "ring_walk.h"

namespace pip {
namespace {

// ---------------------------------------------------------------- plain per-pair baseline
// One lane per pair.  Each lane walks its own polygon's ring (or rings) with
// ordinary (per-lane) global loads.  No preprocessing, no data sharing beyond
// what the caches give.
template <int PRED>
__global__ __launch_bounds__(256) void k_per_pair_fp64(
    const double *__restrict__ px, const double *__restrict__ py, int64_t n,
    const int64_t *__restrict__ offsets, int64_t n_polys, const int64_t *__restrict__ poly_rings,
    int64_t n_rings, const double *__restrict__ vx, const double *__restrict__ vy, int64_t nv,
    const int32_t *__restrict__ point_poly, uint8_t *__restrict__ inside)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    int64_t q = point_poly ? (int64_t)point_poly[i] : 0;
    q = ((uint64_t)q < (uint64_t)n_polys) ? q : 0;
    int64_t r0, r1;
    poly_ring_range(poly_rings, n_rings, q, r0, r1);
    const double x = px[i], y = py[i];
    unsigned par = 0;
    for (int64_t r = r0; r < r1; ++r) {
        int64_t b = offsets[r], e = offsets[r + 1];
        clamp_ring(b, e, nv);
        if (e <= b)
            continue;
        double ax = vx[e - 1], ay = vy[e - 1];   // closing edge v_{k-1} -> v_0 first
        bool a_above = ay > y;
        for (int64_t j = b; j < e; ++j) {
            const double bx = vx[j], by = vy[j];
            const bool b_above = by > y;
            par ^= edge_cross<PRED>(x, y, ax, ay, a_above, bx, by, b_above);
            ax = bx;
            ay = by;
            a_above = b_above;
        }
    }
    inside[i] = (uint8_t)par;
}

// ---------------------------------------------------------------- segmented (wave-uniform polygon)
// One lane per pair, U pairs per lane: a wavefront owns 64*U consecutive pairs
// (row u holds pairs base + 64u + lane, so every load is coalesced) and issues
// all of their loads before any arithmetic, to keep HBM busy.  Within a row,
// the lanes that test the same polygon run together: the polygon id of the
// first unfinished lane is broadcast (readfirstlane), those lanes walk that
// ring with the vertex stream wave-uniform (scalar loads, 8 vertices per
// batch, shared by all of them), then the next group goes.  With pairs sorted
// by polygon a row sees one or two groups.

template <int PRED, bool HAS_INDEX, int U>
__global__ __launch_bounds__(256) void k_segmented_fp64(
    const double *__restrict__ px, const double *__restrict__ py, int64_t n,
    const int64_t *__restrict__ offsets, int64_t n_polys,
    const double *__restrict__ vx, const double *__restrict__ vy, int64_t nv,
    const int32_t *__restrict__ point_poly, uint8_t *__restrict__ inside)
{
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t base = wave * (64 * U);
    double x[U], y[U];
    int q[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t i = base + u * 64 + lane;
        x[u] = 0.0;
        y[u] = 0.0;
        q[u] = 0;
        if (i < n) {
            x[u] = px[i];
            y[u] = py[i];
            if (HAS_INDEX)
                q[u] = point_poly[i];
        }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t i = base + u * 64 + lane;
        const bool valid = i < n;
        if (HAS_INDEX)
            q[u] = ((uint32_t)q[u] < (uint64_t)n_polys) ? q[u] : 0;
        uint64_t todo = __builtin_amdgcn_ballot_w64(valid);
        uint64_t par = 0;
        while (todo) {
            // Leader = first unfinished lane; its polygon is this round's group.
            const int leader = __builtin_ctzll(todo);
            const int qu = __builtin_amdgcn_readlane(q[u], leader);
            int64_t b = offsets[qu], e = offsets[qu + 1];
            clamp_ring(b, e, nv);
            const uint64_t member = todo & __builtin_amdgcn_ballot_w64(q[u] == qu);
            par |= ring_parity_compact_uniform<PRED>(x[u], y[u], (member >> lane) & 1u, vx, vy, b, e) & member;
            todo &= ~member;
        }
        if (valid)
            inside[i] = (uint8_t)((par >> lane) & 1u);
    }
}

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
//   2. side tests only for the lane's straddling edges, lowest set bit first
//      (the order of the tests does not matter: only their count's parity).
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
        // phase 2: side tests for this lane's straddling edges only; bit b
        // is the edge ending at chunk vertex 31 - b
        const int elast = e0 + c0 + 31;
        while (strad != 0) {
            const int b = __builtin_ctz(strad);
            strad &= strad - 1u;
            const double4 rec = L.E[elast - b];
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
    const int elast = e0 + 31;
    while (strad != 0) {
        const int b = __builtin_ctz(strad);
        strad &= strad - 1u;
        const double4 rec = L.E[elast - b];
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

// Batched form.  Without `persistent`, workgroup b takes item order[b] (or b)
// and finds its polygon range itself: pair ids, then offsets, then the ring
// table and vertices, three dependent loads before any work; the pairs' own
// loads are issued first so that they travel alongside that chain.
// With `persistent`, a grid sized to the resident capacity walks the item
// list with a fixed stride (workgroup b: list positions b, b + G, b + 2G, ..).
// Before each block of 64 of its items, 64 lanes look up all 64 polygon
// ranges at once into an LDS table; each item then issues its point, ring
// table and vertex loads together, so an item waits for one memory round
// trip instead of three.  There is no shared counter to contend for: the
// stride is fixed, and the heaviest-first order (if given) deals the costly
// items out evenly.
// Eight waves per SIMD hide the load latency best; the one-item side-test
// variants fit that register budget (64 VGPRs) without spilling; the
// intersection-test variant (its division) and the persistent form (its
// item table) do not, and keep the compiler's choice rather than spill.
// The persistent and one-item-per-workgroup forms are separate kernels
// (PERS), so each is compiled with only its own control flow and registers;
// so are the forms with and without the tile walk for rings larger than the
// LDS budget (TILES; without it such items take the scalar-load group walk).
template <int PRED, int U, bool MR, bool PERS, bool TILES>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PRED == kSide && !MR && !PERS ? 8 : 1)))
void k_staged_batched_fp64(
    const double *__restrict__ px, const double *__restrict__ py, int64_t n,
    const int64_t *__restrict__ offsets, int64_t n_polys, const int64_t *__restrict__ poly_rings,
    int64_t n_rings, const double *__restrict__ vx, const double *__restrict__ vy, int64_t nv,
    const int32_t *__restrict__ point_poly, uint8_t *__restrict__ inside, int max_edges, int max_rings,
    const int32_t *__restrict__ order, int n_items)
{
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int IP = 256 * U;
    if (!PERS) {
        const int item = order ? order[blockIdx.x] : (int)blockIdx.x;
        const int64_t p0 = (int64_t)item * IP;
        // the pairs' loads go out first, so they overlap the range lookups
        const ItemRows<U> P = load_rows<U>(p0, px, py, n, point_poly);
        const ItemRange R = item_range<MR>(p0, IP, n, offsets, n_polys, poly_rings, n_rings, nv, point_poly);
        staged_item_fp64<PRED, U, MR, TILES>(p0, P, n, offsets, n_polys, poly_rings, n_rings, vx, vy, nv, inside,
                                             max_edges, max_rings, smem, R);
        return;
    }
    __shared__ ItemRange s_range[64];
    __shared__ int s_item[64];
    const int64_t G = gridDim.x;
    for (int64_t first = blockIdx.x; first < n_items; first += 64 * G) {
        __syncthreads();   // the previous block's items are done with the table
        if (threadIdx.x < 64) {
            const int64_t pos = first + (int64_t)threadIdx.x * G;
            int item = -1;
            ItemRange R;
            R.vb = R.rf = 0;
            R.qf = R.ql = R.nr = R.nv = R.ok = 0;
            if (pos < n_items) {
                item = order ? order[pos] : (int)pos;
                R = item_range<MR>((int64_t)item * IP, IP, n, offsets, n_polys, poly_rings, n_rings, nv, point_poly);
            }
            s_item[threadIdx.x] = item;
            s_range[threadIdx.x] = R;
        }
        __syncthreads();
        for (int j = 0; j < 64; ++j) {
            const int item = __builtin_amdgcn_readfirstlane(s_item[j]);
            if (item < 0)
                break;
            const int64_t p0 = (int64_t)item * IP;
            const ItemRows<U> P = load_rows<U>(p0, px, py, n, point_poly);
            staged_item_fp64<PRED, U, MR, TILES>(p0, P, n, offsets, n_polys, poly_rings, n_rings, vx, vy, nv,
                                                 inside, max_edges, max_rings, smem, uniform_range(s_range[j]));
            __syncthreads();   // the next item reuses the staging area
        }
    }
}

// ---------------------------------------------------------------- runs (polygon-aligned rows)
// A workgroup item is 1024 consecutive pairs; wavefront w owns pairs
// item + 64*U*w .. +64*U (row u in registers: pair + 64u + lane, coalesced
// loads, all issued before any arithmetic).  The wavefront parks its points
// and polygon ids in a private LDS region and walks them as runs: a run is at
// most 64 consecutive pairs with the same polygon id (found with one ballot),
// processed with the ring wave-uniform -- its y values stream through scalar
// loads into each lane's straddle bits (two vector instructions per vertex),
// then every lane evaluates the side value for its own straddling edges only.
// A run has a single polygon, so no lane waits for another polygon's ring,
// and the ring's size is the run's cost whatever it is (3 or 10^6 vertices).
template <int PRED, int U>
__device__ __forceinline__ void runs_item_fp64(
    int64_t p0, const double *__restrict__ px, const double *__restrict__ py, int64_t n,
    const int64_t *__restrict__ offsets, int64_t n_polys,
    const double *__restrict__ vx, const double *__restrict__ vy, int64_t nv,
    const int32_t *__restrict__ point_poly, uint8_t *__restrict__ inside, unsigned char *smem)
{
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
    constexpr int WP = 64 * U;   // pairs per wavefront
    const int64_t wbase = p0 + (int64_t)wid * WP;
    double2 *P = (double2 *)smem + wid * WP;
    int *Q = (int *)((double2 *)smem + 4 * WP) + wid * WP;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t i = wbase + u * 64 + lane;
        double xv = 0.0, yv = 0.0;
        int qv = 0;
        if (i < n) {
            xv = px[i];
            yv = py[i];
            if (point_poly) {
                qv = point_poly[i];
                qv = ((uint32_t)qv < (uint64_t)n_polys) ? qv : 0;
            }
        }
        P[u * 64 + lane] = make_double2(xv, yv);
        Q[u * 64 + lane] = qv;
    }
    __builtin_amdgcn_s_waitcnt(0);   // wave-private LDS: own writes visible to own reads
    __builtin_amdgcn_wave_barrier();
    const int64_t left = n - wbase;
    const int wn = left <= 0 ? 0 : (left < WP ? (int)left : WP);
    int s = 0;
    while (s < wn) {
        const int qs = __builtin_amdgcn_readfirstlane(Q[s]);
        const int j = s + lane;
        const bool same = j < wn && Q[j < WP ? j : WP - 1] == qs;
        const uint64_t m = __builtin_amdgcn_ballot_w64(same);
        const int cnt = (~m == 0) ? 64 : __builtin_ctzll(~m);
        const bool member = lane < cnt;
        const double2 pt = P[j < WP ? j : WP - 1];
        int64_t b = offsets[qs], e = offsets[qs + 1];
        clamp_ring(b, e, nv);
        const uint64_t par = ring_parity_compact_uniform<PRED>(pt.x, pt.y, member, vx, vy, b, e);
        if (member)
            inside[wbase + j] = (uint8_t)((par >> lane) & 1u);
        s += cnt;
    }
}

// LDS per workgroup: 4 wavefronts x 64*U pairs x (point 16 B + polygon id 4 B)
inline size_t runs_lds_bytes(int pairs_per_lane) { return (size_t)4 * 64 * pairs_per_lane * (16 + 4); }

template <int PRED, int U>
__global__ __launch_bounds__(256) void k_runs_batched_fp64(
    const double *__restrict__ px, const double *__restrict__ py, int64_t n,
    const int64_t *__restrict__ offsets, int64_t n_polys,
    const double *__restrict__ vx, const double *__restrict__ vy, int64_t nv,
    const int32_t *__restrict__ point_poly, uint8_t *__restrict__ inside,
    const int32_t *__restrict__ order, int n_items, unsigned *queue)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_item;
    if (!queue) {
        const int item = order ? order[blockIdx.x] : (int)blockIdx.x;
        runs_item_fp64<PRED, U>((int64_t)item * (256 * U), px, py, n, offsets, n_polys, vx, vy, nv, point_poly, inside,
                          smem);
        return;
    }
    for (;;) {
        if (threadIdx.x == 0)
            s_item = (int)atomicAdd(queue, 1u);
        __syncthreads();
        const int it = s_item;
        __syncthreads();
        if (it >= n_items)
            break;
        const int item = order ? order[it] : it;
        runs_item_fp64<PRED, U>((int64_t)item * (256 * U), px, py, n, offsets, n_polys, vx, vy, nv, point_poly, inside,
                          smem);
        __syncthreads();
    }
}

// ---------------------------------------------------------------- validation
__global__ __launch_bounds__(256) void k_validate_points(
    const double *__restrict__ px, const double *__restrict__ py, int64_t n,
    const int32_t *__restrict__ point_poly, int64_t n_polys, unsigned *flags)
{
    unsigned f = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (!isfinite(px[i]) || !isfinite(py[i]))
            f |= VALIDATE_EDOM;
        if (point_poly && (uint64_t)(int64_t)point_poly[i] >= (uint64_t)n_polys)
            f |= VALIDATE_ERANGE;
    }
    if (f)
        atomicOr(flags, f);
}

__global__ __launch_bounds__(256) void k_validate_polys(
    const int64_t *__restrict__ offsets, int64_t n_polys,
    const double *__restrict__ vx, const double *__restrict__ vy, int64_t nv, unsigned *flags)
{
    unsigned f = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t q = t0; q < n_polys; q += stride)
        if (offsets[q] > offsets[q + 1])
            f |= VALIDATE_ERANGE;
    if (t0 == 0 && (offsets[0] != 0 || offsets[n_polys] != nv))
        f |= VALIDATE_ERANGE;
    for (int64_t j = t0; j < nv; j += stride)
        if (!isfinite(vx[j]) || !isfinite(vy[j]))
            f |= VALIDATE_EDOM;
    if (f)
        atomicOr(flags, f);
}

// Ring index of polygons of several rings: a monotone CSR over n_rings rings.
__global__ __launch_bounds__(256) void k_validate_rings(const int64_t *__restrict__ poly_rings, int64_t n_polys,
                                                        int64_t n_rings, unsigned *flags)
{
    unsigned f = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t q = t0; q < n_polys; q += stride)
        if (poly_rings[q] > poly_rings[q + 1])
            f |= VALIDATE_ERANGE;
    if (t0 == 0 && (poly_rings[0] != 0 || poly_rings[n_polys] != n_rings))
        f |= VALIDATE_ERANGE;
    if (f)
        atomicOr(flags, f);
}

__global__ void k_clear_word(unsigned *w) { *w = 0u; }

// ---------------------------------------------------------------- HBM calibration copy
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_copy16(u32x4 *__restrict__ dst, const u32x4 *__restrict__ src,
                                                int64_t n16)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = __builtin_nontemporal_load(&src[i]);
}

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

}  // namespace

int launch_per_pair(const Problem &p, hipStream_t stream)
{
    if (p.pred == kIntersection)
        PIP_LAUNCH(k_per_pair_fp64<kIntersection>, dim3(grid_for(p.n_points, 256)), dim3(256), 0, stream,
                           p.px, p.py, p.n_points, p.offsets, p.n_polys, p.poly_rings, p.n_rings, p.vx, p.vy,
                           p.n_vertices, p.point_poly, p.inside);
    else
        PIP_LAUNCH(k_per_pair_fp64<kSide>, dim3(grid_for(p.n_points, 256)), dim3(256), 0, stream, p.px,
                           p.py, p.n_points, p.offsets, p.n_polys, p.poly_rings, p.n_rings, p.vx, p.vy,
                           p.n_vertices, p.point_poly, p.inside);
    PIP_HIP_TRY(hipGetLastError());
    return PIP_OK;
}

template <int PRED, int U>
static int launch_segmented_u(const Problem &p, hipStream_t stream, int block)
{
    const int64_t per_block = (int64_t)block * U;
    const dim3 grid(grid_for(p.n_points, (int)per_block)), blk(block);
    if (p.point_poly)
        PIP_LAUNCH((k_segmented_fp64<PRED, true, U>), grid, blk, 0, stream, p.px, p.py, p.n_points, p.offsets,
                           p.n_polys, p.vx, p.vy, p.n_vertices, p.point_poly, p.inside);
    else
        PIP_LAUNCH((k_segmented_fp64<PRED, false, U>), grid, blk, 0, stream, p.px, p.py, p.n_points,
                           p.offsets, p.n_polys, p.vx, p.vy, p.n_vertices, p.point_poly, p.inside);
    PIP_HIP_TRY(hipGetLastError());
    return PIP_OK;
}

template <int PRED>
static int launch_segmented_p(const Problem &p, hipStream_t stream, int pairs_per_lane, int block)
{
    switch (pairs_per_lane) {
    case 1: return launch_segmented_u<PRED, 1>(p, stream, block);
    case 2: return launch_segmented_u<PRED, 2>(p, stream, block);
    case 8: return launch_segmented_u<PRED, 8>(p, stream, block);
    default: return launch_segmented_u<PRED, 4>(p, stream, block);
    }
}

int launch_segmented(const Problem &p, hipStream_t stream, int pairs_per_lane, int block)
{
    if (p.poly_rings)
        return fail(PIP_ENOTSUP, "the segmented kernel takes one ring per polygon; use the staged or per-pair kernel");
    if (block != 64 && block != 128 && block != 256)
        block = 256;
    return p.pred == kIntersection ? launch_segmented_p<kIntersection>(p, stream, pairs_per_lane, block)
                                   : launch_segmented_p<kSide>(p, stream, pairs_per_lane, block);
}

size_t staged_smem_bytes(int max_edges, int max_rings)
{
    // T | PR | Y (with a 64-slot pad) | XR | E, each 32-byte aligned (as staged_lds lays them out)
    size_t o = 2 * (((size_t)(max_rings + 1) * 4 + 31) & ~(size_t)31);
    o += (((size_t)max_edges + 64) * 8 + 31) & ~(size_t)31;
    o += ((size_t)max_edges * 8 + 31) & ~(size_t)31;
    return o + (size_t)max_edges * 32;
}

int staged_max_rings(int pairs_per_lane)
{
    const int u = pairs_per_lane == 1 ? 1 : (pairs_per_lane == 4 ? 4 : 2);
    return 256 * u < 128 ? 256 * u : 128;
}

template <int PRED, int U, bool MR, bool PERS, bool TILES>
static void staged_launch_one(const Problem &p, hipStream_t stream, int grid, size_t shmem, int max_edges,
                              int max_rings, const int32_t *order, int n_items)
{
    PIP_LAUNCH((k_staged_batched_fp64<PRED, U, MR, PERS, TILES>), dim3(grid), dim3(256), shmem, stream, p.px, p.py,
               p.n_points, p.offsets, p.n_polys, p.poly_rings, p.n_rings, p.vx, p.vy, p.n_vertices, p.point_poly,
               p.inside, max_edges, max_rings, order, n_items);
}

template <int U>
static void staged_dispatch(const Problem &p, hipStream_t stream, int grid, size_t shmem, int max_edges,
                            int max_rings, const int32_t *order, int n_items, bool persistent, bool tiles)
{
    using F = void (*)(const Problem &, hipStream_t, int, size_t, int, int, const int32_t *, int);
    // [predicate][several rings][persistent][tiles]
    static const F table[2][2][2][2] = {
        {{{staged_launch_one<kSide, U, false, false, false>, staged_launch_one<kSide, U, false, false, true>},
          {staged_launch_one<kSide, U, false, true, false>, staged_launch_one<kSide, U, false, true, true>}},
         {{staged_launch_one<kSide, U, true, false, false>, staged_launch_one<kSide, U, true, false, true>},
          {staged_launch_one<kSide, U, true, true, false>, staged_launch_one<kSide, U, true, true, true>}}},
        {{{staged_launch_one<kIntersection, U, false, false, false>,
           staged_launch_one<kIntersection, U, false, false, true>},
          {staged_launch_one<kIntersection, U, false, true, false>,
           staged_launch_one<kIntersection, U, false, true, true>}},
         {{staged_launch_one<kIntersection, U, true, false, false>,
           staged_launch_one<kIntersection, U, true, false, true>},
          {staged_launch_one<kIntersection, U, true, true, false>,
           staged_launch_one<kIntersection, U, true, true, true>}}}};
    table[p.pred == kIntersection ? 1 : 0][p.poly_rings ? 1 : 0][persistent ? 1 : 0][tiles ? 1 : 0](
        p, stream, grid, shmem, max_edges, max_rings, order, n_items);
}

int launch_staged_batched(const Problem &p, hipStream_t stream, int pairs_per_lane, int max_edges,
                          const int32_t *order, int n_items, bool persistent, bool tiles, int grid)
{
    const int U = pairs_per_lane == 1 ? 1 : (pairs_per_lane == 4 ? 4 : 2);
    const int max_rings = staged_max_rings(U);
    const size_t shmem = staged_smem_bytes(max_edges, max_rings);
    if (!persistent)
        grid = n_items;
    if (grid <= 0)
        return PIP_OK;
    if (U == 1)
        staged_dispatch<1>(p, stream, grid, shmem, max_edges, max_rings, order, n_items, persistent, tiles);
    else if (U == 4)
        staged_dispatch<4>(p, stream, grid, shmem, max_edges, max_rings, order, n_items, persistent, tiles);
    else
        staged_dispatch<2>(p, stream, grid, shmem, max_edges, max_rings, order, n_items, persistent, tiles);
    PIP_HIP_TRY(hipGetLastError());
    return PIP_OK;
}

int staged_occupancy(int pairs_per_lane, int max_edges, int *blocks_per_cu)
{
    const int U = pairs_per_lane == 1 ? 1 : (pairs_per_lane == 4 ? 4 : 2);
    const size_t shmem = staged_smem_bytes(max_edges, staged_max_rings(U));
    int nb = 0;
    hipError_t e;
    if (U == 1)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_staged_batched_fp64<kSide, 1, false, true, false>, 256,
                                                         shmem);
    else if (U == 4)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_staged_batched_fp64<kSide, 4, false, true, false>, 256,
                                                         shmem);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_staged_batched_fp64<kSide, 2, false, true, false>, 256,
                                                         shmem);
    if (e != hipSuccess)
        return fail(PIP_EHIP, "occupancy query failed: %s", hipGetErrorString(e));
    *blocks_per_cu = nb < 1 ? 1 : nb;
    return PIP_OK;
}

size_t runs_smem_bytes(int pairs_per_lane) { return runs_lds_bytes(pairs_per_lane); }

int launch_runs_batched(const Problem &p, hipStream_t stream, int pairs_per_lane, const int32_t *order,
                        int n_items, unsigned *queue, int grid)
{
    if (p.poly_rings)
        return fail(PIP_ENOTSUP, "the runs kernel takes one ring per polygon; use the staged or per-pair kernel");
    const int U = pairs_per_lane == 1 ? 1 : (pairs_per_lane == 4 ? 4 : 2);
    const size_t shmem = runs_smem_bytes(U);
    if (!queue)
        grid = n_items;
    if (grid <= 0)
        return PIP_OK;
#define PIP_LAUNCH_R(UU)                                                                                         \
    if (p.pred == kIntersection)                                                                                 \
        PIP_LAUNCH((k_runs_batched_fp64<kIntersection, UU>), dim3(grid), dim3(256), shmem, stream, p.px,  \
                           p.py, p.n_points, p.offsets, p.n_polys, p.vx, p.vy, p.n_vertices, p.point_poly,        \
                           p.inside, order, n_items, queue);                                                       \
    else                                                                                                         \
    PIP_LAUNCH((k_runs_batched_fp64<kSide, UU>), dim3(grid), dim3(256), shmem, stream, p.px, p.py, p.n_points, \
                       p.offsets, p.n_polys, p.vx, p.vy, p.n_vertices, p.point_poly, p.inside, order, n_items, queue)
    if (U == 1)
        PIP_LAUNCH_R(1);
    else if (U == 4)
        PIP_LAUNCH_R(4);
    else
        PIP_LAUNCH_R(2);
#undef PIP_LAUNCH_R
    PIP_HIP_TRY(hipGetLastError());
    return PIP_OK;
}

int runs_occupancy(int pairs_per_lane, int *blocks_per_cu)
{
    const int U = pairs_per_lane == 1 ? 1 : (pairs_per_lane == 4 ? 4 : 2);
    const size_t shmem = runs_smem_bytes(U);
    int nb = 0;
    hipError_t e;
    if (U == 1)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_runs_batched_fp64<kSide, 1>, 256, shmem);
    else if (U == 4)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_runs_batched_fp64<kSide, 4>, 256, shmem);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_runs_batched_fp64<kSide, 2>, 256, shmem);
    if (e != hipSuccess)
        return fail(PIP_EHIP, "occupancy query failed: %s", hipGetErrorString(e));
    *blocks_per_cu = nb < 1 ? 1 : nb;
    return PIP_OK;
}

int launch_staged(const Problem &p, hipStream_t stream, int pairs_per_lane, int lds_slots)
{
    // lds_slots = edges a workgroup can stage (40 bytes each in LDS), already
    // clamped to the device's LDS per workgroup
    const int U = pairs_per_lane == 1 ? 1 : (pairs_per_lane == 4 ? 4 : 2);
    const int n_items = (int)((p.n_points + 256 * U - 1) / (256 * U));
    return launch_staged_batched(p, stream, U, lds_slots, nullptr, n_items, false, true, 0);
}

int launch_validate(const Problem &p, unsigned *flags, hipStream_t stream)
{
    hipLaunchKernelGGL(k_clear_word, dim3(1), dim3(1), 0, stream, flags);
    const int64_t np = p.n_points > 0 ? p.n_points : 1;
    unsigned g = grid_for(np, 256);
    g = g > 4096 ? 4096 : g;
    hipLaunchKernelGGL(k_validate_points, dim3(g), dim3(256), 0, stream, p.px, p.py, p.n_points, p.point_poly,
                       p.n_polys, flags);
    // offsets is the ring CSR (n_rings + 1 entries; n_rings = n_polys without a ring index)
    unsigned g2 = grid_for(p.n_vertices > p.n_rings ? p.n_vertices : p.n_rings, 256);
    g2 = g2 < 1 ? 1 : (g2 > 4096 ? 4096 : g2);
    hipLaunchKernelGGL(k_validate_polys, dim3(g2), dim3(256), 0, stream, p.offsets, p.n_rings, p.vx, p.vy,
                       p.n_vertices, flags);
    if (p.poly_rings) {
        unsigned g3 = grid_for(p.n_polys, 256);
        g3 = g3 < 1 ? 1 : (g3 > 4096 ? 4096 : g3);
        hipLaunchKernelGGL(k_validate_rings, dim3(g3), dim3(256), 0, stream, p.poly_rings, p.n_polys, p.n_rings,
                           flags);
    }
    PIP_HIP_TRY(hipGetLastError());
    return PIP_OK;
}

int launch_copy(void *dst, const void *src, int64_t nbytes, hipStream_t stream)
{
    const int64_t n16 = nbytes / 16;
    unsigned g = grid_for(n16, 256);
    g = g > 65536 ? 65536 : (g < 1 ? 1 : g);
    hipLaunchKernelGGL(k_copy16, dim3(g), dim3(256), 0, stream, (u32x4 *)dst, (const u32x4 *)src, n16);
    PIP_HIP_TRY(hipGetLastError());
    return PIP_OK;
}

}  // namespace pip
