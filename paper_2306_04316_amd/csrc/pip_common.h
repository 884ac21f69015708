// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pip.h"

namespace pip {

// ---------------------------------------------------------------- errors
int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();
// Diagnostics to stderr when the environment variable PIP_LOG is set (and not "0").
void log_msg(const char *fmt, ...) __attribute__((format(printf, 1, 2)));

#define PIP_HIP_TRY(expr)                                                              \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return ::pip::fail(PIP_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

#define PIP_TRY(expr)            \
    do {                         \
        int r_ = (expr);         \
        if (r_ != PIP_OK)        \
            return r_;           \
    } while (0)

// ---------------------------------------------------------------- kernel timestamps
// Events that the next main-kernel launch on this thread records with its own
// dispatch (the start and end of the kernel's execution, the timestamps a
// profiler reports), set by a timed plan execution around its main phase.
struct KernelTimer {
    hipEvent_t start = nullptr, stop = nullptr;
};
KernelTimer &kernel_timer();

// Launch a main kernel, with the thread's kernel timer when one is set.
#define PIP_LAUNCH(kernel, grid, block, shmem, stream, ...)                                          \
    do {                                                                                             \
        const ::pip::KernelTimer &kt_ = ::pip::kernel_timer();                                       \
        if (kt_.start || kt_.stop)                                                                   \
            hipExtLaunchKernelGGL(kernel, grid, block, shmem, stream, kt_.start, kt_.stop, 0u, __VA_ARGS__); \
        else                                                                                         \
            hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__);                     \
    } while (0)

// ---------------------------------------------------------------- device facts
struct DeviceInfo {
    int device = -1;
    int cu_count = 0;
    bool gfx950 = false;
    unsigned *validate_flags = nullptr;   // address of the __device__ flag word
    unsigned char *scratch = nullptr;     // address of this device's copy of the static scratch array
    size_t lds_per_block = 0;             // largest dynamic LDS a workgroup may request
};
// Largest edge budget (lds_slots) whose staging fits the device's LDS per workgroup.
int clamp_lds_slots(int lds_slots, bool filtered, int pairs_per_lane, const DeviceInfo *dev);
// Largest LDS tile of the batched kernel (vertices, halved from the request)
// whose layout fits a workgroup's LDS.
int clamp_batched_tile(int tile, bool filtered, int pairs_per_lane, const DeviceInfo *dev);
// Info for the current device (cached per device); PIP_ENOTSUP if not gfx950.
int current_device(DeviceInfo **out);

// ---------------------------------------------------------------- device-memory pool
// Stream-ordered workspace from a pool of the library's own, one per device,
// that keeps released memory for later calls (no device-memory mapping and
// unmapping per call); plain hipMalloc where the pool cannot be created
// (*pooled = false).
hipError_t pool_alloc(void **p, size_t bytes, int dev, hipStream_t s, bool *pooled);
// Release p: a pooled block in stream order on s (no host wait: the pool
// orders its reuse after the work enqueued on s so far); a plain allocation
// after synchronising s.
void pool_release(void *p, bool pooled, hipStream_t s = nullptr);

// ---------------------------------------------------------------- problem description
struct Problem {
    const double *px, *py;
    int64_t n_points;
    const int64_t *offsets;
    int64_t n_polys;
    const double *vx, *vy;
    int64_t n_vertices;
    const int32_t *point_poly;
    uint8_t *inside;
    int pred = 0;   // pip_predicate
    // polygons of several rings: polygon q owns rings poly_rings[q] .. poly_rings[q+1]-1
    // and offsets (n_rings + 1 entries) is the ring CSR; NULL: one ring per polygon
    const int64_t *poly_rings = nullptr;
    int64_t n_rings = 0;   // = n_polys when poly_rings is NULL
};

int check_host_args(const Problem &p);
// Device-side validation (synchronises `stream`): PIP_ERANGE / PIP_EDOM.
int validate_on_device(const Problem &p, DeviceInfo *dev, hipStream_t stream);

// ---------------------------------------------------------------- kernel launchers (exact binary64)
int launch_per_pair(const Problem &p, hipStream_t stream);
int launch_segmented(const Problem &p, hipStream_t stream, int pairs_per_lane, int block);
int launch_staged(const Problem &p, hipStream_t stream, int pairs_per_lane, int lds_slots);
size_t staged_smem_bytes(int max_edges, int max_rings);
size_t runs_smem_bytes(int pairs_per_lane);
int runs_occupancy(int pairs_per_lane, int *blocks_per_cu);
int launch_runs_batched(const Problem &p, hipStream_t stream, int pairs_per_lane, const int32_t *order,
                        int n_items, unsigned *queue, int grid);
// One polygon of one ring for every point (no pair index), its edges walked in
// segments laid out over the XCDs (kernels_exact.hip): plans use it from
// kSegmentMinVertices vertices on.  ring_segments_hi: segment groups for a
// ring of k vertices; mask: (n_points + 63) / 64 64-bit words of workspace.
constexpr int kSegmentVertices = 131072;
constexpr int64_t kSegmentMinVertices = 65536;
int ring_segments_hi(int64_t k);
int launch_ring_segments(const Problem &p, hipStream_t stream, int ns_hi, unsigned long long *mask);
int staged_max_rings(int pairs_per_lane);
int staged_occupancy(int pairs_per_lane, int max_edges, int *blocks_per_cu);
// tiles: use the form that walks rings larger than max_edges in LDS tiles
int launch_staged_batched(const Problem &p, hipStream_t stream, int pairs_per_lane, int max_edges,
                          const int32_t *order, int n_items, bool persistent, bool tiles, int grid);
// Vertex ranges of the work items of item_pairs pairs (all the rings of the
// item's polygons): out[0] = the largest, out[1 + b] = items whose range has
// floor(log2) = b (33 device words, cleared first by the caller).
int launch_item_span(const Problem &p, hipStream_t stream, int item_pairs, int n_items, unsigned *out);

// ---------------------------------------------------------------- filtered binary32 path
size_t filtered_smem_bytes(int max_edges, int max_rings);
int filtered_occupancy(int pairs_per_lane, int max_edges, int *blocks_per_cu);
int launch_filtered(const Problem &p, hipStream_t stream, int pairs_per_lane, int max_edges, float bound_scale,
                    int force_recheck, int32_t *recheck, unsigned *recheck_count, const int32_t *order,
                    int n_items, unsigned *queue, int grid);
// list: count[0] undecided pair ids, the rest of the n_points entries free
// (used for the pairs of long rings); wide_count zeroed before the launch.
int launch_recheck(const Problem &p, hipStream_t stream, int32_t *list, const unsigned *count,
                   unsigned *wide_count, int grid);

// ---------------------------------------------------------------- batched kernel (both modes, LDS tiles)
// A work item's place in the inputs, written once per execution by the
// preparation: item id, the polygons qf..ql of its first and last pair and
// their vertex range [vb, vb + nv); nv = -1 when the ids are out of range or
// not ordered (one ring per polygon).
struct ItemDesc {
    int64_t vb;
    int32_t item;
    int32_t qf, ql;
    int32_t nv;
};
// A ring whose pairs in one work item the wavefront-per-large-ring kernel
// classifies: pairs p_lo .. p_lo+count-1 with point_poly equal to `ring`.
struct WaveTask {
    int64_t p_lo;
    int32_t ring;
    int32_t count;
};
// Where the batched kernel leaves the pairs of rings of at least wave_k
// vertices (filtered mode; wave_k = 0: none): tasks, their count (zeroed
// before the launch), at most max_tasks of them, and the queue cursor of the
// wave kernel (zeroed).
struct WaveOut {
    int wave_k = 0;
    WaveTask *tasks = nullptr;
    unsigned *task_count = nullptr;
    unsigned max_tasks = 0;
    unsigned *cursor = nullptr;
    int grid = 0;   // workgroups of the wave kernel
};
size_t batched_smem_bytes(int tile, int max_rings, bool filtered);
// stats: NULL, or [256][2] counters (point-edge tests, undecided side tests) added to.
// desc: one descriptor per workgroup, in launch order (launch_item_desc).
int launch_batched(const Problem &p, hipStream_t stream, bool filtered, int pairs_per_lane, int tile,
                   float bound_scale, int force_recheck, int32_t *recheck, unsigned *recheck_count,
                   unsigned long long *stats, const ItemDesc *desc, int n_items, const WaveOut &wave = WaveOut());
int launch_wave_rings(const Problem &p, hipStream_t stream, const WaveTask *tasks, const unsigned *task_count,
                      unsigned max_tasks, unsigned *cursor, float bound_k, float bound_eta, int force_recheck,
                      int32_t *recheck, unsigned *recheck_count, unsigned long long *stats, int grid);

// ---------------------------------------------------------------- y-index for one large ring
struct IndexLayout {
    int n0 = 0, n1 = 0, n2 = 0;   // tree nodes per level
    int nb = 0;                   // point chunks of the coarse sorting pass
    size_t o_b0 = 0, o_b1 = 0, o_b2 = 0, o_root = 0, o_hist = 0, o_cursor = 0, o_base = 0, o_txy = 0, o_tidx = 0,
           o_spt = 0, o_sidx = 0;
    size_t bytes = 0;             // workspace bytes
};
IndexLayout index_layout(int64_t n_points, int64_t k);
int launch_index_prep(const Problem &p, hipStream_t s, const IndexLayout &L, unsigned char *ws);
int launch_runs_indexed(const Problem &p, hipStream_t s, const IndexLayout &L, unsigned char *ws);

// ---------------------------------------------------------------- preparation
int launch_fill(unsigned *p, int n, unsigned v, hipStream_t stream);
int launch_item_order(const Problem &p, hipStream_t stream, int item_pairs, int n_items, uint8_t *bucket,
                      unsigned *counters, int32_t *order);
// Descriptors of the work items (one ring per polygon); with `order` set also
// the heaviest-first order, and sdesc the descriptors in that order.
int launch_item_desc(const Problem &p, hipStream_t stream, int item_pairs, int n_items, ItemDesc *desc,
                     uint8_t *bucket, unsigned *counters, int32_t *order, ItemDesc *sdesc);
int launch_copy(void *dst, const void *src, int64_t nbytes, hipStream_t stream);
int launch_read(const void *src, int64_t nbytes, unsigned *sink, hipStream_t stream);
int launch_valu_probe(int iters, double *sink, int cu_count, int64_t *lane_ops, hipStream_t stream);
// Exclusive scan of n uint32 counts into out[0..n] (int64; out[n] = total);
// block_ws holds scan_ws_entries(n) int64 entries.  Kernels only.
int64_t scan_ws_entries(int64_t n);
int launch_scan_u32(const uint32_t *in, int64_t n, int64_t *out, int64_t *block_ws, hipStream_t stream);
int launch_validate(const Problem &p, unsigned *flags, hipStream_t stream);

enum : unsigned { VALIDATE_ERANGE = 1u, VALIDATE_EDOM = 2u };

}  // namespace pip
