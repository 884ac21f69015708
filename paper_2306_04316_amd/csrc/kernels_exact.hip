// Exact binary64 kernels for the constraint-1 ray-casting test (paper,
// Method section, constraint 1, and Algorithm 1, half-open straddle reading):
// the plain per-pair baseline, the wave-segmented kernel, and the staged
// kernel with rings in LDS.  The per-edge arithmetic is in ring_walk.h.
//
// This translation unit must be compiled with -ffp-contract=off.

#include "pip_common.h"
#include "ring_walk.h"
#include "staged_exact.h"

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

// ---------------------------------------------------------------- one ring, cut into segments
// Every point against the one ring [offsets[0], offsets[1]) (no pair index).
// The ring's edges (by end vertex) are cut into nseg = 8 * ns_hi segments of
// equal length and workgroup b takes 1024 points against one segment:
// s_lo = b % 8, then the point block, then s_hi = b / (8 * blocks).
// Consecutive workgroups go to the eight XCDs in turn, so XCD x walks
// segments s_hi * 8 + x, one s_hi group after the other: its share of the
// ring's y values (about 1 MB per segment) stays in its own L2 while every
// point block passes over it.  A segment's walk is the runs kernel's
// wave-uniform chunk walk started with the above bit of the vertex before the
// segment; the segments' parities of each 64-point run are combined by a
// 64-bit XOR into mask[run] (cleared before, turned into bytes after).  The
// segment length follows the ring size read on the device, so any ring
// (even one that changed since the plan chose nseg) is covered exactly.
template <int PRED>
__global__ __launch_bounds__(256) void k_ring_segments(const double *__restrict__ px, const double *__restrict__ py,
                                                       int64_t n, const int64_t *__restrict__ offsets,
                                                       const double *__restrict__ vx, const double *__restrict__ vy,
                                                       int64_t nv, int ns_hi, int64_t nblk,
                                                       unsigned long long *__restrict__ mask)
{
    const int64_t bid = blockIdx.x;
    const int s_lo = (int)(bid & 7);
    const int64_t r = bid >> 3;
    const int64_t blk = r % nblk;
    const int s = (int)(r / nblk) * 8 + s_lo;
    int64_t b0 = offsets[0], e0 = offsets[1];
    clamp_ring(b0, e0, nv);
    const int k = (int)(e0 - b0);
    const int nseg = 8 * ns_hi;
    const int seg = (int)(((int64_t)k + nseg - 1) / nseg);
    const int c_begin = (int)((int64_t)s * seg);
    const int c_end = c_begin + seg < k ? c_begin + seg : k;
    if (k <= 0 || c_begin >= c_end)
        return;
    const double *rx = vx + b0, *ry = vy + b0;
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
    for (int u = 0; u < 4; ++u) {
        const int64_t i0 = blk * 1024 + (int64_t)(u * 4 + wid) * 64;
        if (i0 >= n)
            break;
        const int64_t i = i0 + lane;
        const bool member = i < n;
        double x = 0.0, y = 0.0;
        if (member) {
            x = px[i];
            y = py[i];
        }
        const double yq = y + 0.0;
        uint32_t prev = shift_in_above(0u, yq, ry[c_begin == 0 ? k - 1 : c_begin - 1]);
        uint64_t par = 0;
        for (int c0 = c_begin; c0 < c_end; c0 += 32)
            par ^= chunk_parity_uniform<PRED>(x, y, yq, member, rx, ry, k, c0, prev, c_end);
        // each lane's copy of par is exact in its own bit only (the side-test
        // loop's ballots reach the lanes still in it), so the run's mask is
        // gathered from every lane's own bit
        const uint64_t run = __builtin_amdgcn_ballot_w64((par >> lane) & 1u);
        if (lane == 0 && run)
            atomicXor(&mask[i0 >> 6], (unsigned long long)run);
    }
}

__global__ __launch_bounds__(256) void k_fill_words(unsigned *__restrict__ p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

__global__ __launch_bounds__(256) void k_mask_bytes(const unsigned long long *__restrict__ mask, int64_t n,
                                                    uint8_t *__restrict__ inside)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        inside[i] = (uint8_t)((mask[i >> 6] >> (i & 63)) & 1ull);
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

int ring_segments_hi(int64_t k)
{
    // segments of at most 131,072 vertices (1 MB of y values) per XCD at a time
    const int64_t per = 8 * (int64_t)kSegmentVertices;
    const int64_t h = (k + per - 1) / per;
    return (int)(h < 1 ? 1 : (h > 4096 ? 4096 : h));
}

int launch_ring_segments(const Problem &p, hipStream_t stream, int ns_hi, unsigned long long *mask)
{
    if (p.poly_rings || p.point_poly || p.n_polys != 1)
        return fail(PIP_EINVAL, "the segmented walk takes one polygon of one ring and no pair index");
    if (!mask || ns_hi < 1)
        return fail(PIP_EINVAL, "the segmented walk needs its mask");
    if (p.n_points <= 0)
        return PIP_OK;
    const int64_t nblk = (p.n_points + 1023) / 1024;
    const int64_t words = (p.n_points + 63) / 64;
    const int64_t grid = nblk * 8 * ns_hi;
    if (grid > 0x7fffffffll)
        return fail(PIP_EINVAL, "too many points for the segmented walk");
    // the main-kernel timer spans the clear, the walk and the bytes
    KernelTimer &kt = kernel_timer();
    const KernelTimer saved = kt;
    kt.stop = nullptr;
    const int64_t g1 = grid_for(words * 2, 256) < 65536 ? grid_for(words * 2, 256) : 65536;
    PIP_LAUNCH(k_fill_words, dim3((unsigned)g1), dim3(256), 0, stream, (unsigned *)mask, words * 2);
    kt = KernelTimer{};
    if (p.pred == kIntersection)
        PIP_LAUNCH(k_ring_segments<kIntersection>, dim3((unsigned)grid), dim3(256), 0, stream, p.px, p.py,
                   p.n_points, p.offsets, p.vx, p.vy, p.n_vertices, ns_hi, nblk, mask);
    else
        PIP_LAUNCH(k_ring_segments<kSide>, dim3((unsigned)grid), dim3(256), 0, stream, p.px, p.py, p.n_points,
                   p.offsets, p.vx, p.vy, p.n_vertices, ns_hi, nblk, mask);
    kt.stop = saved.stop;
    const int64_t g2 = grid_for(p.n_points, 256) < 65536 ? grid_for(p.n_points, 256) : 65536;
    PIP_LAUNCH(k_mask_bytes, dim3((unsigned)g2), dim3(256), 0, stream, (const unsigned long long *)mask, p.n_points,
               p.inside);
    kt = saved;
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
