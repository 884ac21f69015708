// Per-execution preparation for the batched launch: work-item costs and a
// heaviest-first order, plus the counter resets.
//
// A work item is a run of item_pairs consecutive pairs.  With pairs sorted by
// polygon its rings are those of polygons point_poly[first]..point_poly[last],
// and its cost is estimated as pairs x (edges in that range / rings in that
// range).  Items are bucketed by floor(log2(cost)) and listed from the heaviest
// bucket down, so that a persistent grid that pulls items in list order starts
// the long items first (longest-processing-time-first scheduling); the order
// inside a bucket does not matter for the results.

#include "pip_common.h"
#include "staged_exact.h"

namespace pip {
namespace {

constexpr int kBuckets = 32;

__global__ __launch_bounds__(256) void k_fill_u32(unsigned *p, int n, unsigned v)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        p[i] = v;
}

__device__ __forceinline__ int item_bucket(int it, const int32_t *__restrict__ pp, int64_t n,
                                           const int64_t *__restrict__ offsets, int64_t n_polys,
                                           const int64_t *__restrict__ poly_rings, int64_t n_rings, int item_pairs)
{
    const int64_t p0 = (int64_t)it * item_pairs;
    const int64_t p1 = (p0 + item_pairs < n ? p0 + item_pairs : n) - 1;
    int64_t qa = pp[p0], qb = pp[p1];
    qa = (uint64_t)qa < (uint64_t)n_polys ? qa : 0;
    qb = (uint64_t)qb < (uint64_t)n_polys ? qb : 0;
    if (qa > qb) {
        const int64_t t = qa;
        qa = qb;
        qb = t;
    }
    int64_t ra = qa, rb = qb + 1;   // the rings of polygons qa..qb
    if (poly_rings) {
        ra = poly_rings[qa];
        rb = poly_rings[qb + 1];
        ra = ra < 0 ? 0 : (ra > n_rings ? n_rings : ra);
        rb = rb < ra ? ra : (rb > n_rings ? n_rings : rb);
    }
    int64_t span = offsets[rb] - offsets[ra];
    span = span < 1 ? 1 : span;
    const int64_t nr = qb - qa + 1;
    int64_t kavg = span / nr;
    kavg = kavg < 1 ? 1 : kavg;
    const uint64_t cost = (uint64_t)(p1 - p0 + 1) * (uint64_t)kavg;
    return 63 - __builtin_clzll(cost | 1ull) > kBuckets - 1 ? kBuckets - 1 : 63 - __builtin_clzll(cost | 1ull);
}

// Largest vertex range of a work item (pairs sorted by polygon: the rings of
// the polygons of its first and last pair), clamped to 2^32 - 1.
// out[0]: the largest span; out[1 + b]: items with floor(log2(span)) = b.
__global__ __launch_bounds__(256) void k_item_span(const int32_t *__restrict__ pp, int64_t n,
                                                   const int64_t *__restrict__ offsets, int64_t n_polys,
                                                   const int64_t *__restrict__ poly_rings, int64_t n_rings,
                                                   int item_pairs, int n_items, unsigned *out)
{
    __shared__ unsigned h[32];
    if (threadIdx.x < 32)
        h[threadIdx.x] = 0;
    __syncthreads();
    unsigned m = 0;
    for (int it = blockIdx.x * blockDim.x + threadIdx.x; it < n_items; it += gridDim.x * blockDim.x) {
        const int64_t p0 = (int64_t)it * item_pairs;
        const int64_t p1 = (p0 + item_pairs < n ? p0 + item_pairs : n) - 1;
        int64_t qa = pp ? pp[p0] : 0, qb = pp ? pp[p1] : 0;
        qa = (uint64_t)qa < (uint64_t)n_polys ? qa : 0;
        qb = (uint64_t)qb < (uint64_t)n_polys ? qb : 0;
        if (qa > qb) {
            const int64_t t = qa;
            qa = qb;
            qb = t;
        }
        int64_t ra = qa, rb = qb + 1;
        if (poly_rings) {
            ra = poly_rings[qa];
            rb = poly_rings[qb + 1];
            ra = ra < 0 ? 0 : (ra > n_rings ? n_rings : ra);
            rb = rb < ra ? ra : (rb > n_rings ? n_rings : rb);
        }
        const int64_t span = offsets[rb] - offsets[ra];
        const unsigned s = span <= 0 ? 0u : (span > 0xffffffffll ? 0xffffffffu : (unsigned)span);
        m = s > m ? s : m;
        atomicAdd(&h[s ? 31 - __builtin_clz(s) : 0], 1u);
    }
    if (m)
        atomicMax(out, m);
    __syncthreads();
    if (threadIdx.x < 32 && h[threadIdx.x])
        atomicAdd(&out[1 + threadIdx.x], h[threadIdx.x]);
}

// counters[0..31] histogram, [32..63] scatter cursors (both zeroed first)
__global__ __launch_bounds__(256) void k_item_hist(const int32_t *__restrict__ pp, int64_t n,
                                                   const int64_t *__restrict__ offsets, int64_t n_polys,
                                                   const int64_t *__restrict__ poly_rings, int64_t n_rings,
                                                   int item_pairs, int n_items, uint8_t *__restrict__ bucket,
                                                   unsigned *counters)
{
    __shared__ unsigned h[kBuckets];
    if (threadIdx.x < kBuckets)
        h[threadIdx.x] = 0;
    __syncthreads();
    for (int it = blockIdx.x * blockDim.x + threadIdx.x; it < n_items; it += gridDim.x * blockDim.x) {
        const int b = item_bucket(it, pp, n, offsets, n_polys, poly_rings, n_rings, item_pairs);
        bucket[it] = (uint8_t)b;
        atomicAdd(&h[b], 1u);
    }
    __syncthreads();
    if (threadIdx.x < kBuckets && h[threadIdx.x])
        atomicAdd(&counters[threadIdx.x], h[threadIdx.x]);
}

// Descriptor of every work item (the range the batched kernel would find
// from the item's first and last pair), and with bucket set its cost bucket
// and the bucket histogram (counters[0..31], zeroed first).
template <bool LPT>
__global__ __launch_bounds__(256) void k_item_desc(const int32_t *__restrict__ pp, int64_t n,
                                                   const int64_t *__restrict__ offsets, int64_t n_polys, int64_t nv,
                                                   int item_pairs, int n_items, ItemDesc *__restrict__ desc,
                                                   uint8_t *__restrict__ bucket, unsigned *counters)
{
    __shared__ unsigned h[kBuckets];
    if (LPT) {
        if (threadIdx.x < kBuckets)
            h[threadIdx.x] = 0;
        __syncthreads();
    }
    for (int it = blockIdx.x * blockDim.x + threadIdx.x; it < n_items; it += gridDim.x * blockDim.x) {
        const int64_t p0 = (int64_t)it * item_pairs;
        const ItemRange R = item_range<false>(p0, item_pairs, n, offsets, n_polys, nullptr, n_polys, nv, pp);
        ItemDesc d;
        d.vb = R.vb;
        d.item = it;
        d.qf = R.qf;
        d.ql = R.ql;
        d.nv = R.ok ? R.nv : -1;
        desc[it] = d;
        if (LPT) {
            const int b = item_bucket(it, pp, n, offsets, n_polys, nullptr, n_polys, item_pairs);
            bucket[it] = (uint8_t)b;
            atomicAdd(&h[b], 1u);
        }
    }
    if (LPT) {
        __syncthreads();
        if (threadIdx.x < kBuckets && h[threadIdx.x])
            atomicAdd(&counters[threadIdx.x], h[threadIdx.x]);
    }
}

// Each workgroup handles a contiguous chunk of items: counts them per bucket
// in LDS, reserves a range per bucket with one global atomic, then places them
// (and, with desc set, their descriptors in the same order).
__global__ __launch_bounds__(256) void k_item_scatter(const uint8_t *__restrict__ bucket, int n_items,
                                                      int chunk, unsigned *counters, int32_t *__restrict__ order,
                                                      const ItemDesc *__restrict__ desc, ItemDesc *__restrict__ sdesc)
{
    __shared__ unsigned h[kBuckets], base[kBuckets], pos[kBuckets];
    const int t = threadIdx.x;
    if (t < kBuckets) {
        // heaviest bucket first: base[b] = items in buckets above b
        unsigned s = 0;
        for (int b = kBuckets - 1; b > t; --b)
            s += counters[b];
        base[t] = s;
        h[t] = 0;
        pos[t] = 0;
    }
    __syncthreads();
    const int i0 = blockIdx.x * chunk;
    const int i1 = i0 + chunk < n_items ? i0 + chunk : n_items;
    for (int it = i0 + t; it < i1; it += blockDim.x)
        atomicAdd(&h[bucket[it]], 1u);
    __syncthreads();
    if (t < kBuckets && h[t])
        base[t] += atomicAdd(&counters[kBuckets + t], h[t]);
    __syncthreads();
    for (int it = i0 + t; it < i1; it += blockDim.x) {
        const int b = bucket[it];
        const unsigned at = base[b] + atomicAdd(&pos[b], 1u);
        order[at] = it;
        if (desc)
            sdesc[at] = desc[it];
    }
}

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

}  // namespace

int launch_fill(unsigned *p, int n, unsigned v, hipStream_t stream)
{
    if (n <= 0)
        return PIP_OK;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 256)), dim3(256), 0, stream, p, n, v);
    PIP_HIP_TRY(hipGetLastError());
    return PIP_OK;
}

int launch_item_span(const Problem &p, hipStream_t stream, int item_pairs, int n_items, unsigned *out)
{
    if (n_items <= 0)
        return PIP_OK;
    unsigned g = grid_for(n_items, 256);
    g = g > 1024 ? 1024 : g;
    hipLaunchKernelGGL(k_item_span, dim3(g), dim3(256), 0, stream, p.point_poly, p.n_points, p.offsets, p.n_polys,
                       p.poly_rings, p.n_rings, item_pairs, n_items, out);
    PIP_HIP_TRY(hipGetLastError());
    return PIP_OK;
}

int launch_item_order(const Problem &p, hipStream_t stream, int item_pairs, int n_items, uint8_t *bucket,
                      unsigned *counters, int32_t *order)
{
    if (n_items <= 0 || !p.point_poly)
        return PIP_OK;
    PIP_TRY(launch_fill(counters, 2 * kBuckets, 0u, stream));
    unsigned g = grid_for(n_items, 256);
    g = g > 1024 ? 1024 : g;
    hipLaunchKernelGGL(k_item_hist, dim3(g), dim3(256), 0, stream, p.point_poly, p.n_points, p.offsets, p.n_polys,
                       p.poly_rings, p.n_rings, item_pairs, n_items, bucket, counters);
    const int chunk = 2048;
    hipLaunchKernelGGL(k_item_scatter, dim3(grid_for(n_items, chunk)), dim3(256), 0, stream, bucket, n_items, chunk,
                       counters, order, nullptr, nullptr);
    PIP_HIP_TRY(hipGetLastError());
    return PIP_OK;
}

int launch_item_desc(const Problem &p, hipStream_t stream, int item_pairs, int n_items, ItemDesc *desc,
                     uint8_t *bucket, unsigned *counters, int32_t *order, ItemDesc *sdesc)
{
    if (n_items <= 0)
        return PIP_OK;
    if (p.poly_rings)
        return fail(PIP_ENOTSUP, "item descriptors take one ring per polygon");
    unsigned g = grid_for(n_items, 256);
    g = g > 1024 ? 1024 : g;
    const bool lpt = order && p.point_poly;
    if (lpt) {
        PIP_TRY(launch_fill(counters, 2 * kBuckets, 0u, stream));
        hipLaunchKernelGGL(k_item_desc<true>, dim3(g), dim3(256), 0, stream, p.point_poly, p.n_points, p.offsets,
                           p.n_polys, p.n_vertices, item_pairs, n_items, desc, bucket, counters);
        const int chunk = 2048;
        hipLaunchKernelGGL(k_item_scatter, dim3(grid_for(n_items, chunk)), dim3(256), 0, stream, bucket, n_items,
                           chunk, counters, order, desc, sdesc);
    } else {
        hipLaunchKernelGGL(k_item_desc<false>, dim3(g), dim3(256), 0, stream, p.point_poly, p.n_points, p.offsets,
                           p.n_polys, p.n_vertices, item_pairs, n_items, desc, nullptr, nullptr);
    }
    PIP_HIP_TRY(hipGetLastError());
    return PIP_OK;
}

}  // namespace pip
