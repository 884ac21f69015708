// Exact binary64 kernels for the constraint-1 ray-casting test.
//
// Per edge (a, b) of a ring and point p (paper, Method section, constraint 1;
// Algorithm 1, with the half-open straddle reading):
//   straddle  : (a_y > p_y) != (b_y > p_y)                 comparisons only, exact
//   normal    : n = (b_y - a_y, a_x - b_x), negated when n_x < 0
//   side      : s = (p_x - a_x) * n_x + (p_y - a_y) * n_y  each op rounded (no FMA)
//   crossing  : s <= 0
// Parity of the crossing count gives the inside bit.
//
// The negation of n is never materialised: with round-to-nearest-even,
// fl(t * (-d)) = -fl(t * d) and fl(-u - v) = -fl(u + v), so the side value with
// the negated normal is exactly -s' where s' uses the unnegated normal.  Under
// the straddle condition n_x < 0 holds exactly when a is the endpoint above the
// ray, so the crossing test becomes (b above ? s' <= 0 : s' >= 0).  Both tests
// treat +0 and -0 alike, so the bit is the same as the literal rule's.
//
// This translation unit must be compiled with -ffp-contract=off.

#include "pip_common.h"

namespace pip {
namespace {

// Clamp a ring's [b, e) to the vertex array so no access leaves it.
__device__ __forceinline__ void clamp_ring(int64_t &b, int64_t &e, int64_t nv)
{
    e = e < 0 ? 0 : (e > nv ? nv : e);
    b = b < 0 ? 0 : (b > e ? e : b);
}

// Make a value the compiler can prove wave-uniform (it is, by construction).
__device__ __forceinline__ int64_t uniform64(int64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Crossing-parity contribution of edge (a, b) for point (x, y).
__device__ __forceinline__ unsigned edge_cross(double x, double y, double ax, double ay, bool a_above,
                                               double bx, double by, bool b_above)
{
    unsigned c = 0;
    if (a_above != b_above) {
        const double nx = by - ay;
        const double ny = ax - bx;
        const double t1 = x - ax;
        const double t2 = y - ay;
        const double s = t1 * nx + t2 * ny;
        c = b_above ? (s <= 0.0) : (s >= 0.0);
    }
    return c;
}

// ---------------------------------------------------------------- plain per-pair baseline
// One lane per pair.  Each lane walks its own polygon's ring with ordinary
// (per-lane) global loads.  No preprocessing, no data sharing beyond what the
// caches give.
__global__ __launch_bounds__(256) void k_per_pair_fp64(
    const double *__restrict__ px, const double *__restrict__ py, int64_t n,
    const int64_t *__restrict__ offsets, int64_t n_polys,
    const double *__restrict__ vx, const double *__restrict__ vy, int64_t nv,
    const int32_t *__restrict__ point_poly, uint8_t *__restrict__ inside)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    int64_t q = point_poly ? (int64_t)point_poly[i] : 0;
    q = ((uint64_t)q < (uint64_t)n_polys) ? q : 0;
    int64_t b = offsets[q], e = offsets[q + 1];
    clamp_ring(b, e, nv);
    const double x = px[i], y = py[i];
    unsigned par = 0;
    if (e > b) {
        double ax = vx[e - 1], ay = vy[e - 1];   // closing edge v_{k-1} -> v_0 first
        bool a_above = ay > y;
        for (int64_t j = b; j < e; ++j) {
            const double bx = vx[j], by = vy[j];
            const bool b_above = by > y;
            par ^= edge_cross(x, y, ax, ay, a_above, bx, by, b_above);
            ax = bx;
            ay = by;
            a_above = b_above;
        }
    }
    inside[i] = (uint8_t)par;
}

// ---------------------------------------------------------------- segmented (wave-uniform polygon)
// One lane per pair.  Within a wavefront, the lanes that test the same polygon
// run together: the polygon id of the first unfinished lane is broadcast
// (readfirstlane), those lanes walk that ring with the vertex stream
// wave-uniform (scalar loads, shared by all of them), then the next group
// goes.  With pairs sorted by polygon a wavefront sees one or two groups.
template <bool HAS_INDEX>
__global__ __launch_bounds__(256) void k_segmented_fp64(
    const double *__restrict__ px, const double *__restrict__ py, int64_t n,
    const int64_t *__restrict__ offsets, int64_t n_polys,
    const double *__restrict__ vx, const double *__restrict__ vy, int64_t nv,
    const int32_t *__restrict__ point_poly, uint8_t *__restrict__ inside)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < n;
    double x = 0.0, y = 0.0;
    int q = 0;
    if (valid) {
        x = px[i];
        y = py[i];
        if (HAS_INDEX) {
            q = point_poly[i];
            q = ((uint32_t)q < (uint64_t)n_polys) ? q : 0;
        }
    }
    unsigned par = 0;
    bool todo = valid;
    while (todo) {
        // Everything about the group's polygon is derived from the broadcast id
        // before the divergent branch, so it stays in scalar registers.
        const int qu = __builtin_amdgcn_readfirstlane(q);
        int64_t b = offsets[qu], e = offsets[qu + 1];
        clamp_ring(b, e, nv);
        b = uniform64(b);
        e = uniform64(e);
        if (q == qu) {
            todo = false;
            if (e > b) {
                double ax = vx[e - 1], ay = vy[e - 1];
                bool a_above = ay > y;
                for (int64_t j = b; j < e; ++j) {
                    const double bx = vx[j], by = vy[j];
                    const bool b_above = by > y;
                    par ^= edge_cross(x, y, ax, ay, a_above, bx, by, b_above);
                    ax = bx;
                    ay = by;
                    a_above = b_above;
                }
            }
        }
    }
    if (valid)
        inside[i] = (uint8_t)par;
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
    hipLaunchKernelGGL(k_per_pair_fp64, dim3(grid_for(p.n_points, 256)), dim3(256), 0, stream, p.px, p.py,
                       p.n_points, p.offsets, p.n_polys, p.vx, p.vy, p.n_vertices, p.point_poly, p.inside);
    PIP_HIP_TRY(hipGetLastError());
    return PIP_OK;
}

int launch_segmented(const Problem &p, hipStream_t stream)
{
    const dim3 grid(grid_for(p.n_points, 256)), block(256);
    if (p.point_poly)
        hipLaunchKernelGGL(k_segmented_fp64<true>, grid, block, 0, stream, p.px, p.py, p.n_points, p.offsets,
                           p.n_polys, p.vx, p.vy, p.n_vertices, p.point_poly, p.inside);
    else
        hipLaunchKernelGGL(k_segmented_fp64<false>, grid, block, 0, stream, p.px, p.py, p.n_points, p.offsets,
                           p.n_polys, p.vx, p.vy, p.n_vertices, p.point_poly, p.inside);
    PIP_HIP_TRY(hipGetLastError());
    return PIP_OK;
}

int launch_validate(const Problem &p, unsigned *flags, hipStream_t stream)
{
    hipLaunchKernelGGL(k_clear_word, dim3(1), dim3(1), 0, stream, flags);
    const int64_t np = p.n_points > 0 ? p.n_points : 1;
    unsigned g = grid_for(np, 256);
    g = g > 4096 ? 4096 : g;
    hipLaunchKernelGGL(k_validate_points, dim3(g), dim3(256), 0, stream, p.px, p.py, p.n_points, p.point_poly,
                       p.n_polys, flags);
    unsigned g2 = grid_for(p.n_vertices > p.n_polys ? p.n_vertices : p.n_polys, 256);
    g2 = g2 < 1 ? 1 : (g2 > 4096 ? 4096 : g2);
    hipLaunchKernelGGL(k_validate_polys, dim3(g2), dim3(256), 0, stream, p.offsets, p.n_polys, p.vx, p.vy,
                       p.n_vertices, flags);
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
