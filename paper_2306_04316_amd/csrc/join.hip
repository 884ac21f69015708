// Candidate pairs by bounding box: the step before classification.
//
// The paper prepares its input by keeping only the points inside the
// polygon's bounding box (Simulation section).  For many polygons at once the
// same filter is a join: pair (i, q) is a candidate when point i lies in the
// closed box [min x, max x] x [min y, max y] of polygon q's vertices (all its
// rings).  Comparisons only, so the candidate set is exact; it is produced
// grouped by polygon in ascending order, which is the order the staged
// classification kernels want.
//
// Device pipeline (one stream, no host round trip until the pair count):
//   1. extent of the points (two-pass min/max) and a uniform grid of about
//      n/4 cells over it, row-major, cell (x) = floor((x - x0) * sx) clamped
//      -- monotone in x, so a box [a, b] maps to the cell range
//      [cell(a), cell(b)] that holds every point with a <= x <= b;
//   2. counting sort of the points by cell (two levels with LDS counters and
//      LDS-staged writes, sort_staged.h), so the points of cells cx0..cx1 of
//      one grid row are one contiguous run;
//   3. per polygon (one wavefront each): its box and cell range; its rows
//      become work units (a unit = one polygon x one grid row);
//   4. per unit (one wavefront): the lanes test the run's points against
//      the box; count pass, scan, then the fill pass writes the pairs with
//      ballot prefix positions.
// Within a polygon the pairs come in grid order (row, then the cell sort's
// order, which depends on LDS atomics): the set is exact, the order inside a
// polygon is not specified.
#include <mutex>
#include <unordered_map>

#include "pip_common.h"
#include "ring_walk.h"
#include "sort_staged.h"

#include <algorithm>

namespace pip {
namespace {

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

struct GridParams {
    double x0, y0;   // extent origin
    double x1, y1;   // extent end (inclusive)
    double sx, sy;   // cells per unit length
    int gx, gy;      // cells per row, rows
};

__device__ __forceinline__ int cell_1d(double v, double v0, double s, int g)
{
    const double t = (v - v0) * s;
    // NaN and values below the origin land in cell 0, values past the end in g-1
    return t >= 0.0 ? (t < (double)g ? (int)t : g - 1) : 0;
}

// ---------------------------------------------------------------- 1. extent and grid
__global__ __launch_bounds__(256) void k_extent_partial(const double *__restrict__ px, const double *__restrict__ py,
                                                        int64_t n, double4 *__restrict__ part)
{
    __shared__ double4 s[256];
    double x0 = INFINITY, x1 = -INFINITY, y0 = INFINITY, y1 = -INFINITY;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const double x = px[i], y = py[i];
        x0 = fmin(x0, x);
        x1 = fmax(x1, x);
        y0 = fmin(y0, y);
        y1 = fmax(y1, y);
    }
    s[threadIdx.x] = make_double4(x0, x1, y0, y1);
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            const double4 a = s[threadIdx.x], b = s[threadIdx.x + off];
            s[threadIdx.x] = make_double4(fmin(a.x, b.x), fmax(a.y, b.y), fmin(a.z, b.z), fmax(a.w, b.w));
        }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        part[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(256) void k_extent_final(const double4 *__restrict__ part, int nparts, int64_t cells,
                                                      GridParams *__restrict__ g)
{
    __shared__ double4 s[256];
    double4 a = make_double4(INFINITY, -INFINITY, INFINITY, -INFINITY);
    for (int k = threadIdx.x; k < nparts; k += 256) {
        const double4 b = part[k];
        a = make_double4(fmin(a.x, b.x), fmax(a.y, b.y), fmin(a.z, b.z), fmax(a.w, b.w));
    }
    s[threadIdx.x] = a;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            const double4 p = s[threadIdx.x], q = s[threadIdx.x + off];
            s[threadIdx.x] = make_double4(fmin(p.x, q.x), fmax(p.y, q.y), fmin(p.z, q.z), fmax(p.w, q.w));
        }
        __syncthreads();
    }
    if (threadIdx.x != 0)
        return;
    const double4 e = s[0];
    GridParams G;
    G.x0 = e.x;
    G.x1 = e.y;
    G.y0 = e.z;
    G.y1 = e.w;
    double w = e.y - e.x, h = e.w - e.z;
    w = (w > 0.0 && w < INFINITY) ? w : 0.0;   // also NaN -> 0
    h = (h > 0.0 && h < INFINITY) ? h : 0.0;
    int gx = 1, gy = 1;
    if (w > 0.0 && h > 0.0) {
        double fx = sqrt((double)cells * w / h);
        fx = fx < 1.0 ? 1.0 : (fx > (double)cells ? (double)cells : fx);
        gx = (int)fx;
        gy = (int)(cells / gx);
        gy = gy < 1 ? 1 : gy;
    } else if (w > 0.0) {
        gx = (int)cells;
    } else if (h > 0.0) {
        gy = (int)cells;
    }
    G.gx = gx;
    G.gy = gy;
    G.sx = w > 0.0 ? (double)gx / w : 0.0;
    G.sy = h > 0.0 ? (double)gy / h : 0.0;
    if (!(G.x0 <= G.x1)) {   // no finite point: everything in cell 0
        G.x0 = G.y0 = 0.0;
        G.sx = G.sy = 0.0;
    }
    *g = G;
}

// ---------------------------------------------------------------- 2. points sorted by cell
// The grid cell of a point as the sort key (cells of at most 2^22, as the
// join sizes the grid: 2048 coarse digits of 2048 fine digits).
struct CellKey {
    static constexpr bool kUsesX = true;
    const GridParams *g;
    struct Ready {
        GridParams G;
        __device__ __forceinline__ int operator()(double x, double y) const
        {
            return cell_1d(y, G.y0, G.sy, G.gy) * G.gx + cell_1d(x, G.x0, G.sx, G.gx);
        }
    };
    __device__ __forceinline__ Ready ready() const { return Ready{*g}; }
};
constexpr int kCellCoarse = 2048;
constexpr int kCellFine = 2048;
// points per thread of a sorted piece in the coarse and the fine pass (pieces
// of 4096 and 2048 points: longer runs per digit, fewer partial lines written)
constexpr int kCellPer = 16;
constexpr int kCellFinePer = 8;

// ---------------------------------------------------------------- 3. polygon boxes and their rows
struct PolyCells {
    double4 box;   // x0, x1, y0, y1
    int cx0, cx1, cy0, cy1;
};

__device__ __forceinline__ double wave_min(double v)
{
    for (int off = 32; off > 0; off >>= 1)
        v = fmin(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ __forceinline__ double wave_max(double v)
{
    for (int off = 32; off > 0; off >>= 1)
        v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// One wavefront per polygon.  rows[q] = grid rows its box covers (0 when the
// box is empty or misses the points' extent).
__global__ __launch_bounds__(256) void k_poly_cells(const int64_t *__restrict__ offsets, int64_t n_polys,
                                                    const int64_t *__restrict__ poly_rings, int64_t n_rings,
                                                    const double *__restrict__ vx, const double *__restrict__ vy,
                                                    int64_t nv, const GridParams *__restrict__ gp,
                                                    PolyCells *__restrict__ pc, uint32_t *__restrict__ rows)
{
    const GridParams G = *gp;
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * 4;
    for (int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); q < n_polys; q += waves) {
        int64_t r0, r1;
        poly_ring_range(poly_rings, n_rings, q, r0, r1);
        int64_t b = offsets[r0], e = offsets[r1];
        clamp_ring(b, e, nv);
        double x0 = INFINITY, x1 = -INFINITY, y0 = INFINITY, y1 = -INFINITY;
        for (int64_t v = b + lane; v < e; v += 64) {
            const double x = vx[v], y = vy[v];
            x0 = fmin(x0, x);
            x1 = fmax(x1, x);
            y0 = fmin(y0, y);
            y1 = fmax(y1, y);
        }
        x0 = wave_min(x0);
        x1 = wave_max(x1);
        y0 = wave_min(y0);
        y1 = wave_max(y1);
        if (lane == 0) {
            PolyCells P;
            P.box = make_double4(x0, x1, y0, y1);
            const bool live = x0 <= x1 && y0 <= y1 && !(x1 < G.x0) && !(x0 > G.x1) && !(y1 < G.y0) && !(y0 > G.y1);
            P.cx0 = cell_1d(x0, G.x0, G.sx, G.gx);
            P.cx1 = cell_1d(x1, G.x0, G.sx, G.gx);
            P.cy0 = cell_1d(y0, G.y0, G.sy, G.gy);
            P.cy1 = cell_1d(y1, G.y0, G.sy, G.gy);
            pc[q] = P;
            rows[q] = live && P.cy1 >= P.cy0 && P.cx1 >= P.cx0 ? (uint32_t)(P.cy1 - P.cy0 + 1) : 0u;
        }
    }
}

// unit_poly[u] = q for the units (rows) of polygon q: unit_start[q] .. unit_start[q+1]-1
__global__ __launch_bounds__(256) void k_unit_owner(const int64_t *__restrict__ unit_start, int64_t n_polys,
                                                    int32_t *__restrict__ unit_poly)
{
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < n_polys; q += (int64_t)gridDim.x * 256)
        for (int64_t u = unit_start[q]; u < unit_start[q + 1]; ++u)
            unit_poly[u] = (int32_t)q;
}

// ---------------------------------------------------------------- 4. units: count, then fill
// Unit u = (polygon q, grid row cy): the sorted points of cells cx0..cx1 of
// row cy, tested against q's box by the 64 lanes of one wavefront.
template <bool FILL>
__global__ __launch_bounds__(256) void k_units(const int64_t *__restrict__ unit_start,
                                               const int32_t *__restrict__ unit_poly, int64_t n_units,
                                               const PolyCells *__restrict__ pc, const GridParams *__restrict__ gp,
                                               const int64_t *__restrict__ cell_start,
                                               const int32_t *__restrict__ spt, const double2 *__restrict__ sxy,
                                               uint32_t *__restrict__ unit_count, const int64_t *__restrict__ unit_off,
                                               int64_t *__restrict__ pair_point, int32_t *__restrict__ pair_poly,
                                               double *__restrict__ pair_px, double *__restrict__ pair_py)
{
    const int gx = gp->gx;
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * 4;
    for (int64_t u = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); u < n_units; u += waves) {
        const int q = __builtin_amdgcn_readfirstlane(unit_poly[u]);
        const PolyCells P = pc[q];
        const int cy = P.cy0 + (int)(u - unit_start[q]);
        const int64_t c0 = (int64_t)cy * gx + P.cx0;
        const int64_t a = cell_start[c0], b = cell_start[c0 + (P.cx1 - P.cx0) + 1];
        int64_t out = FILL ? unit_off[u] : 0;
        uint32_t cnt = 0;
        for (int64_t k0 = a; k0 < b; k0 += 64) {
            const int64_t k = k0 + lane;
            bool hit = false;
            double2 p = make_double2(0.0, 0.0);
            if (k < b) {
                p = sxy[k];
                hit = P.box.x <= p.x && p.x <= P.box.y && P.box.z <= p.y && p.y <= P.box.w;
            }
            const uint64_t m = __builtin_amdgcn_ballot_w64(hit);
            if (FILL && hit) {
                const int64_t at = out + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                if (pair_point)
                    pair_point[at] = spt[k];
                if (pair_poly)
                    pair_poly[at] = q;
                if (pair_px)
                    pair_px[at] = p.x;
                if (pair_py)
                    pair_py[at] = p.y;
            }
            out += __builtin_popcountll(m);
            cnt += (uint32_t)__builtin_popcountll(m);
        }
        if (!FILL && lane == 0)
            unit_count[u] = cnt;
    }
}

}  // namespace
}  // namespace pip

using namespace pip;

struct pip_join {
    Problem p;              // points and polygons (inside unused)
    int device = -1;
    void *ws = nullptr;     // points grid and per-polygon arrays
    void *ws2 = nullptr;    // per-unit arrays
    bool ws_pooled = false, ws2_pooled = false;
    GridParams *grid = nullptr;
    int64_t cells = 0;
    int64_t n_units = 0;
    int64_t n_pairs = 0;
    PolyCells *pc = nullptr;
    int64_t *cell_start = nullptr, *unit_start = nullptr, *unit_off = nullptr;
    int32_t *spt = nullptr, *unit_poly = nullptr;
    double2 *sxy = nullptr;
    // device timestamps: [0, 1] the first phase's kernels (grid, sort, boxes, unit
    // count), [2, 3] the second's (unit owners, pair count), [4, 5] the fill
    hipEvent_t ev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    bool filled = false;
};

extern "C" {

int pip_join_destroy(pip_join *j)
{
    clear_error();
    if (!j)
        return PIP_OK;
    (void)hipDeviceSynchronize();   // no enqueued work may still use the workspace
    pool_release(j->ws, j->ws_pooled);
    pool_release(j->ws2, j->ws2_pooled);
    for (auto &e : j->ev)
        if (e)
            (void)hipEventDestroy(e);
    delete j;
    return PIP_OK;
}

int pip_join_create(pip_join **out, const double *px, const double *py, int64_t n_points,
                    const int64_t *poly_rings, int64_t n_polys, const int64_t *offsets, int64_t n_rings,
                    const double *vx, const double *vy, int64_t n_vertices, int64_t *n_pairs, void *stream)
{
    clear_error();
    if (!out || !n_pairs)
        return fail(PIP_EINVAL, "out or n_pairs is NULL");
    *out = nullptr;
    *n_pairs = 0;
    if (n_points < 0 || n_polys < 0 || n_vertices < 0 || (poly_rings && n_rings < 0))
        return fail(PIP_EINVAL, "negative count");
    if (n_points > INT32_MAX || n_polys > INT32_MAX || (poly_rings && n_rings > INT32_MAX))
        return fail(PIP_EINVAL, "the join takes fewer than 2^31 points and polygons");
    if (n_polys > 0 && !offsets)
        return fail(PIP_EINVAL, "offsets is NULL");
    if (n_points > 0 && (!px || !py))
        return fail(PIP_EINVAL, "px/py is NULL");
    if (n_vertices > 0 && (!vx || !vy))
        return fail(PIP_EINVAL, "vx/vy is NULL");
    DeviceInfo *dev = nullptr;
    PIP_TRY(current_device(&dev));
    hipStream_t s = (hipStream_t)stream;

    pip_join *j = new pip_join;
    Problem &p = j->p;
    p = Problem{px, py, n_points, offsets, n_polys, vx, vy, n_vertices, nullptr, nullptr};
    p.poly_rings = poly_rings;
    p.n_rings = poly_rings ? n_rings : n_polys;
    j->device = dev->device;
    for (auto &ev : j->ev) {
        if (hipEventCreate(&ev) != hipSuccess) {
            (void)hipGetLastError();
            pip_join_destroy(j);
            return fail(PIP_EHIP, "join: hipEventCreate failed");
        }
    }
    if (n_points == 0 || n_polys == 0) {
        *out = j;
        return PIP_OK;
    }

    // about four points per cell, at most 2^22 cells (the sort's key range)
    j->cells = std::max<int64_t>(1, std::min<int64_t>(n_points / 4, (int64_t)kCellCoarse * kCellFine));
    const int64_t C = j->cells, N = n_points, P = n_polys;
    const int nparts = (int)std::min<int64_t>(1024, grid_for(N, 256));
    const int nb = (int)((N + kSortChunk - 1) / kSortChunk);
    const int64_t tn = (int64_t)kCellCoarse * nb;
    const int64_t scan_blocks = scan_ws_entries(std::max<int64_t>(tn, P));
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = (off + bytes + 255) & ~(size_t)255;
        return at;
    };
    const size_t o_grid = take(sizeof(GridParams));
    const size_t o_part = take((size_t)nparts * sizeof(double4));
    const size_t o_table = take((size_t)tn * 4);
    const size_t o_toff = take((size_t)(tn + 1) * 8);
    const size_t o_txy = take((size_t)N * 16);
    const size_t o_tidx = take((size_t)N * 4);
    const size_t o_cstart = take(((size_t)kCellCoarse * kCellFine + 1) * 8);
    const size_t o_spt = take((size_t)N * 4);
    const size_t o_sxy = take((size_t)N * 16);
    const size_t o_pc = take((size_t)P * sizeof(PolyCells));
    const size_t o_rows = take((size_t)P * 4);
    const size_t o_ustart = take((size_t)(P + 1) * 8);
    const size_t o_scan = take((size_t)scan_blocks * 8);
    hipError_t e = pool_alloc(&j->ws, off, j->device, s, &j->ws_pooled);
    if (e != hipSuccess) {
        delete j;
        (void)hipGetLastError();
        return fail(PIP_ENOMEM, "join workspace of %zu bytes: %s", off, hipGetErrorString(e));
    }
    unsigned char *w = (unsigned char *)j->ws;
    j->grid = (GridParams *)(w + o_grid);
    double4 *part = (double4 *)(w + o_part);
    uint32_t *table = (uint32_t *)(w + o_table);
    int64_t *toff = (int64_t *)(w + o_toff);
    j->cell_start = (int64_t *)(w + o_cstart);
    j->spt = (int32_t *)(w + o_spt);
    j->sxy = (double2 *)(w + o_sxy);
    j->pc = (PolyCells *)(w + o_pc);
    uint32_t *rows = (uint32_t *)(w + o_rows);
    j->unit_start = (int64_t *)(w + o_ustart);
    int64_t *scan_ws = (int64_t *)(w + o_scan);

    int rc = PIP_OK;
    auto step = [&](int r) {
        if (rc == PIP_OK)
            rc = r;
    };
    if (hipEventRecord(j->ev[0], s) != hipSuccess)
        rc = fail(PIP_EHIP, "join: hipEventRecord failed");
    if (rc == PIP_OK) {
        hipLaunchKernelGGL(k_extent_partial, dim3(nparts), dim3(256), 0, s, px, py, N, part);
        hipLaunchKernelGGL(k_extent_final, dim3(1), dim3(256), 0, s, part, nparts, C, j->grid);
        if (hipGetLastError() != hipSuccess)
            rc = fail(PIP_EHIP, "join grid kernels failed to launch");
    }
    // points sorted by cell; cell_start[c] = first position of cell c
    step(launch_sort_staged<CellKey, kCellCoarse, kCellFine, kCellPer, kCellFinePer>(
        px, py, N, CellKey{j->grid}, nb, table, toff, scan_ws, (double2 *)(w + o_txy), (int32_t *)(w + o_tidx),
        j->sxy, j->spt, j->cell_start, s));
    if (rc == PIP_OK) {
        const unsigned gq = std::min<unsigned>(grid_for(P, 4), 65536u);
        hipLaunchKernelGGL(k_poly_cells, dim3(gq), dim3(256), 0, s, offsets, P, poly_rings, p.n_rings, vx, vy,
                           n_vertices, j->grid, j->pc, rows);
        if (hipGetLastError() != hipSuccess)
            rc = fail(PIP_EHIP, "join polygon kernels failed to launch");
    }
    step(launch_scan_u32(rows, P, j->unit_start, scan_ws, s));
    if (rc == PIP_OK && hipEventRecord(j->ev[1], s) != hipSuccess)
        rc = fail(PIP_EHIP, "join: hipEventRecord failed");
    int64_t U = 0;
    if (rc == PIP_OK) {
        e = hipMemcpyAsync(&U, j->unit_start + P, sizeof U, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess)
            e = hipStreamSynchronize(s);
        if (e != hipSuccess)
            rc = fail(PIP_EHIP, "join unit count: %s", hipGetErrorString(e));
    }
    j->n_units = U;
    if (rc == PIP_OK && U > 0) {
        size_t off2 = 0;
        auto take2 = [&](size_t bytes) {
            const size_t at = off2;
            off2 = (off2 + bytes + 255) & ~(size_t)255;
            return at;
        };
        const size_t o_upoly = take2((size_t)U * 4);
        const size_t o_ucount = take2((size_t)U * 4);
        const size_t o_uoff = take2((size_t)(U + 1) * 8);
        const size_t o_uscan = take2((size_t)scan_ws_entries(U) * 8);
        e = pool_alloc(&j->ws2, off2, j->device, s, &j->ws2_pooled);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            rc = fail(PIP_ENOMEM, "join unit workspace of %zu bytes: %s", off2, hipGetErrorString(e));
        } else {
            unsigned char *w2 = (unsigned char *)j->ws2;
            j->unit_poly = (int32_t *)(w2 + o_upoly);
            uint32_t *ucount = (uint32_t *)(w2 + o_ucount);
            j->unit_off = (int64_t *)(w2 + o_uoff);
            const unsigned gq = std::min<unsigned>(grid_for(P, 256), 8192u);
            if (hipEventRecord(j->ev[2], s) != hipSuccess)
                rc = fail(PIP_EHIP, "join: hipEventRecord failed");
            hipLaunchKernelGGL(k_unit_owner, dim3(gq), dim3(256), 0, s, j->unit_start, P, j->unit_poly);
            const unsigned gu = std::min<unsigned>(grid_for(U, 4), 65536u);
            hipLaunchKernelGGL((k_units<false>), dim3(gu), dim3(256), 0, s, j->unit_start, j->unit_poly, U, j->pc,
                               j->grid, j->cell_start, j->spt, j->sxy, ucount, nullptr, nullptr, nullptr, nullptr,
                               nullptr);
            if (hipGetLastError() != hipSuccess)
                rc = fail(PIP_EHIP, "join count kernels failed to launch");
            step(launch_scan_u32(ucount, U, j->unit_off, (int64_t *)(w2 + o_uscan), s));
            if (rc == PIP_OK && hipEventRecord(j->ev[3], s) != hipSuccess)
                rc = fail(PIP_EHIP, "join: hipEventRecord failed");
            int64_t M = 0;
            if (rc == PIP_OK) {
                e = hipMemcpyAsync(&M, j->unit_off + U, sizeof M, hipMemcpyDeviceToHost, s);
                if (e == hipSuccess)
                    e = hipStreamSynchronize(s);
                if (e != hipSuccess)
                    rc = fail(PIP_EHIP, "join pair count: %s", hipGetErrorString(e));
            }
            j->n_pairs = M;
        }
    }
    if (rc != PIP_OK) {
        pip_join_destroy(j);
        return rc;
    }
    *n_pairs = j->n_pairs;
    *out = j;
    return PIP_OK;
}

int pip_join_fill(pip_join *j, int64_t *pair_point, int32_t *pair_poly, double *pair_px, double *pair_py,
                  void *stream)
{
    clear_error();
    if (!j)
        return fail(PIP_EINVAL, "join is NULL");
    int dev = -1;
    PIP_HIP_TRY(hipGetDevice(&dev));
    if (dev != j->device)
        return fail(PIP_EINVAL, "join belongs to device %d, current device is %d", j->device, dev);
    if (j->n_pairs == 0)
        return PIP_OK;
    const int64_t U = j->n_units;
    const unsigned gu = std::min<unsigned>(grid_for(U, 4), 65536u);
    PIP_HIP_TRY(hipEventRecord(j->ev[4], (hipStream_t)stream));
    hipLaunchKernelGGL((k_units<true>), dim3(gu), dim3(256), 0, (hipStream_t)stream, j->unit_start, j->unit_poly, U,
                       j->pc, j->grid, j->cell_start, j->spt, j->sxy, nullptr, j->unit_off, pair_point, pair_poly,
                       pair_px, pair_py);
    PIP_HIP_TRY(hipGetLastError());
    PIP_HIP_TRY(hipEventRecord(j->ev[5], (hipStream_t)stream));
    j->filled = true;
    return PIP_OK;
}

int pip_join_timing(pip_join *j, float *ms_count, float *ms_fill)
{
    clear_error();
    if (!j || !ms_count || !ms_fill)
        return fail(PIP_EINVAL, "NULL argument");
    *ms_count = *ms_fill = 0.f;
    if (j->n_pairs == 0 || !j->filled)
        return j->filled || j->n_pairs == 0 ? PIP_OK : fail(PIP_EINVAL, "pip_join_fill has not run");
    float a = 0.f, b = 0.f, c = 0.f;
    PIP_HIP_TRY(hipEventSynchronize(j->ev[5]));
    PIP_HIP_TRY(hipEventElapsedTime(&a, j->ev[0], j->ev[1]));
    PIP_HIP_TRY(hipEventElapsedTime(&b, j->ev[2], j->ev[3]));
    PIP_HIP_TRY(hipEventElapsedTime(&c, j->ev[4], j->ev[5]));
    *ms_count = a + b;
    *ms_fill = c;
    return PIP_OK;
}

}  // extern "C"
