// y-index for one large polygon tested by many points (beyond the paper's
// O(n)-per-point sweep; the results are the rule's bits, unchanged).
//
// The ring's edges are grouped into a three-level tree of y ranges: a level-0
// node covers 32 consecutive edges, a level-1 node 32 level-0 nodes, a
// level-2 node 32 level-1 nodes.  A node's range [lo, hi] spans every endpoint
// of its edges, so a point with p_y < lo (every endpoint above the ray) or
// p_y >= hi (every endpoint at or below it) has no straddling edge in the node
// -- a decision taken by comparisons only, hence exact -- and the above bit of
// the node's last vertex is simply (p_y < lo).  The points are reordered by a
// counting sort on a y bucket, so that the 64 points of a wavefront share a
// narrow y band and whole subtrees are skipped by every lane together; a node
// that some lane's band meets is descended, down to level-0 chunks walked
// exactly as in the unindexed kernel.

#include "pip_common.h"
#include "ring_walk.h"
#include "sort_staged.h"

namespace pip {
namespace {

constexpr int kYBuckets = 65536;

// Level-0 bounds: node c covers edges 32c .. 32c+31, endpoints v_{32c-1} .. v_{32c+31}.
__global__ __launch_bounds__(256) void k_bounds_l0(const double *__restrict__ ry, int k, double2 *__restrict__ b0,
                                                   int n0)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n0)
        return;
    double lo = INFINITY, hi = -INFINITY;
    const int j0 = 32 * c - 1;
    const int j1 = 32 * c + 31 < k - 1 ? 32 * c + 31 : k - 1;
    for (int j = j0; j <= j1; ++j) {
        const double v = ry[j < 0 ? k - 1 : j];
        lo = fmin(lo, v);
        hi = fmax(hi, v);
    }
    b0[c] = make_double2(lo, hi);
}

// Next level: node c covers input nodes 32c .. 32c+31.
__global__ __launch_bounds__(256) void k_bounds_up(const double2 *__restrict__ in, int n_in,
                                                   double2 *__restrict__ out, int n_out)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_out)
        return;
    double lo = INFINITY, hi = -INFINITY;
    const int i1 = 32 * c + 32 < n_in ? 32 * c + 32 : n_in;
    for (int i = 32 * c; i < i1; ++i) {
        lo = fmin(lo, in[i].x);
        hi = fmax(hi, in[i].y);
    }
    out[c] = make_double2(lo, hi);
}

// Whole-ring range: one workgroup reduces the top level.
__global__ __launch_bounds__(256) void k_bounds_root(const double2 *__restrict__ in, int n_in,
                                                     double2 *__restrict__ root)
{
    __shared__ double slo[256], shi[256];
    double lo = INFINITY, hi = -INFINITY;
    for (int i = threadIdx.x; i < n_in; i += 256) {
        lo = fmin(lo, in[i].x);
        hi = fmax(hi, in[i].y);
    }
    slo[threadIdx.x] = lo;
    shi[threadIdx.x] = hi;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            slo[threadIdx.x] = fmin(slo[threadIdx.x], slo[threadIdx.x + o]);
            shi[threadIdx.x] = fmax(shi[threadIdx.x], shi[threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        *root = make_double2(slo[0], shi[0]);
}

__device__ __forceinline__ int ybucket(double y, double lo, double scale)
{
    const double f = (y - lo) * scale;
    return !(f >= 0.0) ? 0 : (f >= (double)(kYBuckets - 1) ? kYBuckets - 1 : (int)f);
}

// The points are counting-sorted by y bucket in two levels (sort_staged.h):
// 512 coarse digits of 128 fine digits each.  The coarse pass orders pieces
// of 4096 points, so that a digit leaves a piece as a run of about eight
// points (whole memory lines rather than single scattered points); the fine
// pass, one workgroup per coarse digit, orders pieces of 2048.
struct YKey {
    static constexpr bool kUsesX = false;
    const double2 *root;
    struct Ready {
        double lo, scale;
        __device__ __forceinline__ int operator()(double, double y) const { return ybucket(y, lo, scale); }
    };
    __device__ __forceinline__ Ready ready() const
    {
        const double lo = root->x, hi = root->y;
        return Ready{lo, hi > lo ? (double)kYBuckets / (hi - lo) : 0.0};
    }
};
constexpr int kCoarse = 512;
constexpr int kFine = kYBuckets / kCoarse;
constexpr int kSortPer = 16;   // points per thread of a sorted piece, pass 1
constexpr int kFinePer = 8;    // the same, pass 2

struct Tree {
    const double2 *b0, *b1, *b2;
    int n0, n1, n2;
};

// The bounds of nodes g0 .. g0+cnt-1 (cnt <= 64) of one tree level, node
// g0+j in lane j (zeros past cnt).  Issued ahead of their use (see below).
__device__ __forceinline__ double2 group_load(const double2 *__restrict__ b, int g0, int cnt)
{
    const int lane = threadIdx.x & 63;
    return lane < cnt ? b[g0 + lane] : make_double2(0.0, 0.0);
}

// Which of those nodes may hold a straddling edge for some lane: the node's
// [lo, hi) against the wavefront's y range [ylo, yhi] (a superset of the
// lanes' exact tests: a node whose range misses it has every lane's y below
// lo or at or above hi, so none of its edges straddles).
__device__ __forceinline__ uint64_t group_mask(const double2 &mine, int cnt, double ylo, double yhi)
{
    const int lane = threadIdx.x & 63;
    return __builtin_amdgcn_ballot_w64(lane < cnt && mine.x <= yhi && mine.y > ylo);
}

// Above bit of the last vertex of a skipped node (bounds held by lane j of
// `mine`): every lane's y lies below its lo (all above) or at or above its hi.
__device__ __forceinline__ uint32_t prev_after_skip(double y, const double2 &mine, int j)
{
    const uint64_t bits = (uint64_t)__double_as_longlong(mine.x);
    const uint32_t lo_lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)bits, j);
    const uint32_t lo_hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(bits >> 32), j);
    const double lo = __longlong_as_double((long long)(((uint64_t)lo_hi << 32) | lo_lo));
    return y < lo ? 1u : 0u;
}

constexpr int kLeafBatch = 4;   // leaves staged per wavefront at a time
constexpr int kLeafSlot = 40;   // doubles per staged leaf and coordinate (33 used)

// Stage up to kLeafBatch hit leaves of one level-0 group (leaf ids c[b],
// b < nb) in the wavefront's LDS slice: leaf b's vertices c0-1 .. c0+m-1
// (c0 = 32 c[b], the ring's last vertex before vertex 0) at slot b.  All
// loads are issued before any is stored, so a batch costs one memory round
// trip.
__device__ __forceinline__ void stage_leaves(const double *__restrict__ rx, const double *__restrict__ ry, int k,
                                             const int (&c)[kLeafBatch], int nb, double *sx, double *sy)
{
    const int lane = threadIdx.x & 63;
    double lx[kLeafBatch], ly[kLeafBatch];
#pragma unroll
    for (int b = 0; b < kLeafBatch; ++b) {
        lx[b] = 0.0;
        ly[b] = 0.0;
        const int c0 = 32 * c[b];
        const int m = k - c0 < 32 ? k - c0 : 32;
        if (b < nb && lane <= m) {
            const int j = c0 - 1 + lane;
            const int jj = j < 0 ? k - 1 : j;
            lx[b] = rx[jj];
            ly[b] = ry[jj];
        }
    }
#pragma unroll
    for (int b = 0; b < kLeafBatch; ++b) {
        const int c0 = 32 * c[b];
        const int m = k - c0 < 32 ? k - c0 : 32;
        if (b < nb && lane <= m) {
            sx[b * kLeafSlot + lane] = lx[b];
            sy[b * kLeafSlot + lane] = ly[b];
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One staged 32-edge leaf (edges ending at vertices c0 .. c0+m-1, m <= 32;
// sx, sy: its slot, entry 0 = vertex c0-1) for the wavefront's points: the
// straddle pass and each lane's side tests read the slot.  `prev`: the above
// bit of vertex c0-1 on entry, of the leaf's last vertex on exit.
template <int PRED>
__device__ __forceinline__ uint64_t leaf_parity_lds(double x, double y, double yq, bool member, int m, uint32_t &prev,
                                                    const double *sx, const double *sy)
{
    uint32_t above = 0;
    int t = 0;
    for (; t < m; t += 4) {
#pragma unroll
        for (int tt = 0; tt < 4; ++tt)
            above = shift_in_above(above, yq, sy[1 + (t + tt < m ? t + tt : m - 1)]);
    }
    above = t < 32 ? above << (32 - t) : above;
    uint32_t strad = above ^ ((above >> 1) | (prev << 31));
    strad &= (uint32_t)(0xffffffff00000000ull >> m);
    prev = (above >> (32 - m)) & 1u;
    strad = member ? strad : 0u;
    uint64_t par = 0;
    while (strad != 0) {
        const int j = __builtin_clz(strad);   // edge (vertex c0+j-1, vertex c0+j)
        strad ^= 0x80000000u >> j;
        const bool b_above = (above >> (31 - j)) & 1u;
        par ^= __builtin_amdgcn_ballot_w64(straddle_crosses<PRED>(x, y, sx[j], sy[j], sx[j + 1], sy[j + 1], b_above));
    }
    return par;
}

// Rows of 64 y-ordered points against the one ring, walked through the tree:
// at each level a wavefront tests up to 64 sibling nodes with one vector load
// and one ballot, then descends into the hit ones in ring order; before a hit
// node whose predecessor was skipped (and after a skipped last node) each
// lane's "above" bit is set from the skipped node's bounds.
template <int PRED>
__global__ __launch_bounds__(256) void k_runs_indexed_fp64(const double2 *__restrict__ spt,
                                                           const int32_t *__restrict__ sidx, int64_t n,
                                                           const double *__restrict__ rx,
                                                           const double *__restrict__ ry, int k, Tree tr,
                                                           uint8_t *__restrict__ inside)
{
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool member = i < n;
    double2 p = make_double2(0.0, 0.0);
    int32_t idx = 0;
    if (member) {
        p = spt[i];
        idx = sidx[i];
    }
    __shared__ double s_leaf[4][2][kLeafBatch * kLeafSlot];   // per wavefront: staged leaves' x and y
    double *sx = s_leaf[threadIdx.x >> 6][0], *sy = s_leaf[threadIdx.x >> 6][1];
    // the top level's bounds and the ring's last y do not depend on the points:
    // their loads go out with the points'
    double2 m2 = group_load(tr.b2, 0, tr.n2 < 64 ? tr.n2 : 64);
    const double ylast = k > 0 ? ry[k - 1] : 0.0;
    uint64_t par = 0;
    if (k > 0) {
        const double yq = p.y + 0.0;
        uint32_t prev = shift_in_above(0u, yq, ylast);
        double ylo = member ? p.y : INFINITY, yhi = member ? p.y : -INFINITY;
        for (int o = 32; o > 0; o >>= 1) {
            ylo = fmin(ylo, __shfl_xor(ylo, o, 64));
            yhi = fmax(yhi, __shfl_xor(yhi, o, 64));
        }
        for (int a2 = 0; a2 < tr.n2; a2 += 64) {
            const int c2 = tr.n2 - a2 < 64 ? tr.n2 - a2 : 64;
            uint64_t h2 = group_mask(m2, c2, ylo, yhi);
            // the children of the next hit node are loaded while the current
            // one's subtree is walked (one level at a time, in ring order)
            int s1n = 0, c1n = 0;
            double2 m1n = make_double2(0.0, 0.0);
            if (h2) {
                s1n = 32 * (a2 + __builtin_ctzll(h2));
                c1n = tr.n1 - s1n < 32 ? tr.n1 - s1n : 32;
                m1n = group_load(tr.b1, s1n, c1n);
            }
            int v2 = -1;   // last visited node of the group
            while (h2) {
                const int j2 = __builtin_ctzll(h2);
                h2 &= h2 - 1;
                if (j2 > 0 && v2 != j2 - 1)
                    prev = prev_after_skip(p.y, m2, j2 - 1);
                const int s1 = s1n, c1 = c1n;
                const double2 m1 = m1n;
                if (h2) {
                    s1n = 32 * (a2 + __builtin_ctzll(h2));
                    c1n = tr.n1 - s1n < 32 ? tr.n1 - s1n : 32;
                    m1n = group_load(tr.b1, s1n, c1n);
                }
                uint64_t h1 = group_mask(m1, c1, ylo, yhi);
                int s0n = 0, c0n = 0;
                double2 m0n = make_double2(0.0, 0.0);
                if (h1) {
                    s0n = 32 * (s1 + __builtin_ctzll(h1));
                    c0n = tr.n0 - s0n < 32 ? tr.n0 - s0n : 32;
                    m0n = group_load(tr.b0, s0n, c0n);
                }
                int v1 = -1;
                while (h1) {
                    const int j1 = __builtin_ctzll(h1);
                    h1 &= h1 - 1;
                    if (j1 > 0 && v1 != j1 - 1)
                        prev = prev_after_skip(p.y, m1, j1 - 1);
                    const int s0 = s0n, c0 = c0n;
                    const double2 m0 = m0n;
                    if (h1) {
                        s0n = 32 * (s1 + __builtin_ctzll(h1));
                        c0n = tr.n0 - s0n < 32 ? tr.n0 - s0n : 32;
                        m0n = group_load(tr.b0, s0n, c0n);
                    }
                    uint64_t h0 = group_mask(m0, c0, ylo, yhi);
                    int v0 = -1;
                    while (h0) {
                        // the next (up to) kLeafBatch hit leaves, staged together
                        int ids[kLeafBatch], cs[kLeafBatch];
                        int nb = 0;
#pragma unroll
                        for (int b = 0; b < kLeafBatch; ++b) {
                            ids[b] = 0;
                            if (h0) {
                                ids[b] = __builtin_ctzll(h0);
                                h0 &= h0 - 1;
                                nb = b + 1;
                            }
                            cs[b] = s0 + ids[b];
                        }
                        stage_leaves(rx, ry, k, cs, nb, sx, sy);
                        for (int b = 0; b < nb; ++b) {
                            const int j0 = ids[b];
                            if (j0 > 0 && v0 != j0 - 1)
                                prev = prev_after_skip(p.y, m0, j0 - 1);
                            const int lc0 = 32 * cs[b];
                            const int m = k - lc0 < 32 ? k - lc0 : 32;
                            par ^= leaf_parity_lds<PRED>(p.x, p.y, yq, member, m, prev, sx + b * kLeafSlot,
                                                         sy + b * kLeafSlot);
                            v0 = j0;
                        }
                        // every lane is done with the slice before the next batch rewrites it
                        __builtin_amdgcn_wave_barrier();
                    }
                    if (v0 != c0 - 1)
                        prev = prev_after_skip(p.y, m0, c0 - 1);
                    v1 = j1;
                }
                if (v1 != c1 - 1)
                    prev = prev_after_skip(p.y, m1, c1 - 1);
                v2 = j2;
            }
            if (v2 != c2 - 1)
                prev = prev_after_skip(p.y, m2, c2 - 1);
            // the next group of top-level nodes (rings of more than 2^21 vertices)
            if (a2 + 64 < tr.n2)
                m2 = group_load(tr.b2, a2 + 64, tr.n2 - a2 - 64 < 64 ? tr.n2 - a2 - 64 : 64);
        }
    }
    if (member)
        inside[idx] = (uint8_t)((par >> lane) & 1u);
}

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

}  // namespace

IndexLayout index_layout(int64_t n_points, int64_t k)
{
    IndexLayout L;
    L.n0 = (int)((k + 31) / 32);
    L.n1 = (L.n0 + 31) / 32;
    L.n2 = (L.n1 + 31) / 32;
    size_t o = 0;
    auto take = [&](size_t b) {
        const size_t at = o;
        o = (o + b + 255) & ~(size_t)255;
        return at;
    };
    L.o_b0 = take((size_t)(L.n0 > 0 ? L.n0 : 1) * 16);
    L.o_b1 = take((size_t)(L.n1 > 0 ? L.n1 : 1) * 16);
    L.o_b2 = take((size_t)(L.n2 > 0 ? L.n2 : 1) * 16);
    L.o_root = take(16);
    const int64_t np = n_points > 0 ? n_points : 1;
    L.nb = (int)((np + kSortChunk - 1) / kSortChunk);
    const int64_t tn = (int64_t)kCoarse * L.nb;
    L.o_hist = take((size_t)tn * 4);                       // (coarse digit, chunk) counts
    L.o_cursor = take((size_t)(tn + 1) * 8);               // their exclusive scan
    L.o_base = take((size_t)scan_ws_entries(tn) * 8);      // scan workspace
    L.o_txy = take((size_t)np * 16);                       // coarse-sorted points
    L.o_tidx = take((size_t)np * 4);
    L.o_spt = take((size_t)np * 16);
    L.o_sidx = take((size_t)np * 4);
    L.bytes = o;
    return L;
}

int launch_index_prep(const Problem &p, hipStream_t s, const IndexLayout &L, unsigned char *ws)
{
    if (p.poly_rings)
        return fail(PIP_ENOTSUP, "the y-index takes one ring");
    // one polygon: its ring is the whole vertex array (offsets = {0, n_vertices})
    const int k = (int)p.n_vertices;
    double2 *b0 = (double2 *)(ws + L.o_b0), *b1 = (double2 *)(ws + L.o_b1), *b2 = (double2 *)(ws + L.o_b2);
    double2 *root = (double2 *)(ws + L.o_root);
    uint32_t *table = (uint32_t *)(ws + L.o_hist);
    int64_t *off = (int64_t *)(ws + L.o_cursor);
    int64_t *scan_ws = (int64_t *)(ws + L.o_base);
    if (k <= 0 || p.n_points <= 0)
        return PIP_OK;
    hipLaunchKernelGGL(k_bounds_l0, dim3(grid_for(L.n0, 256)), dim3(256), 0, s, p.vy, k, b0, L.n0);
    hipLaunchKernelGGL(k_bounds_up, dim3(grid_for(L.n1, 256)), dim3(256), 0, s, b0, L.n0, b1, L.n1);
    hipLaunchKernelGGL(k_bounds_up, dim3(grid_for(L.n2, 256)), dim3(256), 0, s, b1, L.n1, b2, L.n2);
    hipLaunchKernelGGL(k_bounds_root, dim3(1), dim3(256), 0, s, b2, L.n2, root);
    PIP_TRY((launch_sort_staged<YKey, kCoarse, kFine, kSortPer, kFinePer>(
        p.px, p.py, p.n_points, YKey{root}, L.nb, table, off, scan_ws, (double2 *)(ws + L.o_txy),
        (int32_t *)(ws + L.o_tidx), (double2 *)(ws + L.o_spt), (int32_t *)(ws + L.o_sidx), nullptr, s)));
    PIP_HIP_TRY(hipGetLastError());
    return PIP_OK;
}

int launch_runs_indexed(const Problem &p, hipStream_t s, const IndexLayout &L, unsigned char *ws)
{
    if (p.poly_rings)
        return fail(PIP_ENOTSUP, "the y-index takes one ring");
    if (p.n_points <= 0)
        return PIP_OK;
    Tree tr;
    tr.b0 = (const double2 *)(ws + L.o_b0);
    tr.b1 = (const double2 *)(ws + L.o_b1);
    tr.b2 = (const double2 *)(ws + L.o_b2);
    tr.n0 = L.n0;
    tr.n1 = L.n1;
    tr.n2 = L.n2;
    if (p.pred == kIntersection)
        PIP_LAUNCH(k_runs_indexed_fp64<kIntersection>, dim3(grid_for(p.n_points, 256)), dim3(256), 0, s,
                           (const double2 *)(ws + L.o_spt), (const int32_t *)(ws + L.o_sidx), p.n_points, p.vx,
                           p.vy, (int)p.n_vertices, tr, p.inside);
    else
        PIP_LAUNCH(k_runs_indexed_fp64<kSide>, dim3(grid_for(p.n_points, 256)), dim3(256), 0, s,
                           (const double2 *)(ws + L.o_spt), (const int32_t *)(ws + L.o_sidx), p.n_points, p.vx,
                           p.vy, (int)p.n_vertices, tr, p.inside);
    PIP_HIP_TRY(hipGetLastError());
    return PIP_OK;
}

}  // namespace pip
