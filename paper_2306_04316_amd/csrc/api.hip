// C ABI entry points: argument checks, device checks, kernel selection.
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <unordered_map>
#include <vector>

#include "pip_common.h"

namespace pip {

namespace {
thread_local char g_err[512] = "";

// Flag word written by the validation kernels (one per device; concurrent
// validating calls on one device share it).
__device__ unsigned g_validate_word;

// The workspace of pip_classify_noalloc, laid out as batched_ws below for
// PIP_NOALLOC_MAX_POINTS pairs: count words (padded to 256 bytes), the item
// descriptors of the batched kernel (one item per 256 pairs at most), the
// list of undecided pairs.  Host code uses only the address
// hipGetSymbolAddress gives for the current device (DeviceInfo::scratch),
// never the array's name.
constexpr size_t kScratchHead = 256;
constexpr size_t kScratchDesc = (((size_t)PIP_NOALLOC_MAX_POINTS + 255) / 256 * sizeof(ItemDesc) + 255) & ~(size_t)255;
__device__ __align__(256) unsigned char
    scratch[kScratchHead + kScratchDesc + (size_t)PIP_NOALLOC_MAX_POINTS * sizeof(int32_t)];

std::mutex g_dev_mu;
std::vector<DeviceInfo *> g_devs;
}  // namespace

KernelTimer &kernel_timer()
{
    static thread_local KernelTimer t;
    return t;
}

int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

void clear_error() { g_err[0] = '\0'; }

void log_msg(const char *fmt, ...)
{
    static const bool on = [] {
        const char *e = getenv("PIP_LOG");
        return e && e[0] && e[0] != '0';
    }();
    if (!on)
        return;
    va_list ap;
    va_start(ap, fmt);
    fputs("[pip] ", stderr);
    vfprintf(stderr, fmt, ap);
    fputc('\n', stderr);
    va_end(ap);
}

int current_device(DeviceInfo **out)
{
    int dev = 0;
    PIP_HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_dev_mu);
    if ((int)g_devs.size() <= dev)
        g_devs.resize(dev + 1, nullptr);
    if (!g_devs[dev]) {
        hipDeviceProp_t prop;
        PIP_HIP_TRY(hipGetDeviceProperties(&prop, dev));
        auto *d = new DeviceInfo;
        d->device = dev;
        d->cu_count = prop.multiProcessorCount;
        d->gfx950 = strncmp(prop.gcnArchName, "gfx950", 6) == 0;
        d->lds_per_block = prop.sharedMemPerBlock > 1024 ? prop.sharedMemPerBlock - 1024 : prop.sharedMemPerBlock;
        void *sym = nullptr;
        hipError_t e = hipGetSymbolAddress(&sym, HIP_SYMBOL(g_validate_word));
        if (e != hipSuccess) {
            delete d;
            return fail(PIP_EHIP, "hipGetSymbolAddress(validate word) failed: %s", hipGetErrorString(e));
        }
        d->validate_flags = (unsigned *)sym;
        void *scr = nullptr;
        e = hipGetSymbolAddress(&scr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) {
            delete d;
            return fail(PIP_EHIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        }
        d->scratch = (unsigned char *)scr;
        g_devs[dev] = d;
    }
    if (!g_devs[dev]->gfx950)
        return fail(PIP_ENOTSUP, "device %d is not gfx950", dev);
    *out = g_devs[dev];
    return PIP_OK;
}

int clamp_lds_slots(int lds_slots, bool filtered, int pairs_per_lane, const DeviceInfo *dev)
{
    lds_slots = lds_slots < 16 ? 16 : (lds_slots > 2048 ? 2048 : lds_slots);
    const int rings = staged_max_rings(pairs_per_lane);
    while (lds_slots > 16 && (filtered ? filtered_smem_bytes(lds_slots, rings) : staged_smem_bytes(lds_slots, rings)) >
                                 dev->lds_per_block)
        lds_slots /= 2;
    return lds_slots;
}

// Largest LDS tile (vertices, halved from the request) whose batched layout
// fits a workgroup's LDS.
int clamp_batched_tile(int tile, bool filtered, int pairs_per_lane, const DeviceInfo *dev)
{
    tile = tile < 32 ? 32 : (tile > 2048 ? 2048 : tile);
    const int rings = staged_max_rings(pairs_per_lane);
    while (tile > 32 && batched_smem_bytes(tile, rings, filtered) > dev->lds_per_block)
        tile /= 2;
    return tile;
}

int check_host_args(const Problem &p)
{
    if (p.n_points < 0 || p.n_polys < 1 || p.n_vertices < 0)
        return fail(PIP_EINVAL, "negative count or n_polys < 1 (n_points=%lld n_polys=%lld n_vertices=%lld)",
                    (long long)p.n_points, (long long)p.n_polys, (long long)p.n_vertices);
    if (p.n_polys > INT32_MAX)
        return fail(PIP_EINVAL, "n_polys exceeds the int32 pair index range");
    if (!p.offsets)
        return fail(PIP_EINVAL, "offsets is NULL");
    if (p.poly_rings && (p.n_rings < 0 || p.n_rings > INT32_MAX))
        return fail(PIP_EINVAL, "n_rings=%lld out of range", (long long)p.n_rings);
    if (p.n_vertices > 0 && (!p.vx || !p.vy))
        return fail(PIP_EINVAL, "vx/vy is NULL");
    if (p.n_points > 0 && (!p.px || !p.py || !p.inside))
        return fail(PIP_EINVAL, "px/py/inside is NULL");
    // with no points there is no pair index to read (an empty array may be NULL)
    if (p.n_points > 0 && !p.point_poly && p.n_polys != 1)
        return fail(PIP_EINVAL, "point_poly is NULL but n_polys=%lld (must be 1)", (long long)p.n_polys);
    return PIP_OK;
}

namespace {
std::mutex g_pool_mu;
std::unordered_map<int, hipMemPool_t> g_pools;

hipMemPool_t workspace_pool(int dev)
{
    std::lock_guard<std::mutex> lk(g_pool_mu);
    auto it = g_pools.find(dev);
    if (it != g_pools.end())
        return it->second;
    hipMemPoolProps props = {};
    props.allocType = hipMemAllocationTypePinned;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = dev;
    hipMemPool_t pool = nullptr;
    const hipError_t ce = hipMemPoolCreate(&pool, &props);
    if (ce != hipSuccess) {
        (void)hipGetLastError();
        log_msg("workspace pool unavailable on device %d (%s): plain allocations", dev, hipGetErrorString(ce));
        pool = nullptr;
    } else {
        uint64_t keep = UINT64_MAX;   // never trim on synchronisation
        if (hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep) != hipSuccess)
            (void)hipGetLastError();
    }
    g_pools[dev] = pool;
    return pool;
}
}  // namespace

hipError_t pool_alloc(void **p, size_t bytes, int dev, hipStream_t s, bool *pooled)
{
    hipMemPool_t pool = workspace_pool(dev);
    if (pool) {
        const hipError_t e = hipMallocFromPoolAsync(p, bytes, pool, s);
        if (e == hipSuccess) {
            *pooled = true;
            return e;
        }
        (void)hipGetLastError();
        log_msg("workspace pool allocation of %zu bytes failed (%s): plain allocation", bytes, hipGetErrorString(e));
    }
    *pooled = false;
    return hipMalloc(p, bytes);
}

void pool_release(void *p, bool pooled, hipStream_t s)
{
    if (!p)
        return;
    if (pooled) {
        if (hipFreeAsync(p, s) != hipSuccess)
            (void)hipGetLastError();
        return;
    }
    if (hipStreamSynchronize(s) != hipSuccess)
        (void)hipGetLastError();
    (void)hipFree(p);
}

int validate_on_device(const Problem &p, DeviceInfo *dev, hipStream_t stream)
{
    PIP_TRY(launch_validate(p, dev->validate_flags, stream));
    unsigned flags = 0;
    PIP_HIP_TRY(hipMemcpyAsync(&flags, dev->validate_flags, sizeof flags, hipMemcpyDeviceToHost, stream));
    PIP_HIP_TRY(hipStreamSynchronize(stream));
    if (flags & VALIDATE_ERANGE)
        return fail(PIP_ERANGE, "offsets are not a CSR over n_vertices, or a point_poly entry is out of range");
    if (flags & VALIDATE_EDOM)
        return fail(PIP_EDOM, "non-finite coordinate");
    return PIP_OK;
}

}  // namespace pip

using namespace pip;

extern "C" {

void pip_options_init(pip_options *opts)
{
    if (!opts)
        return;
    memset(opts, 0, sizeof *opts);
    opts->struct_size = sizeof *opts;
    opts->mode = PIP_MODE_EXACT_FP64;
    opts->kernel = PIP_KERNEL_AUTO;
    opts->validate = 0;
    opts->persistent = -1;
    opts->order = -1;
    opts->use_graph = 1;
    opts->tune = 0;
    opts->force_recheck = 0;
    opts->bound_scale = 1.0f;
    opts->tune_cache = NULL;
    opts->timing = 0;
    opts->index = 0;
    opts->predicate = PIP_PRED_SIDE;
    opts->stats = 0;
    opts->wave_k = 0;
}

int pip_abi_version(void) { return PIP_ABI_VERSION; }

const char *pip_last_error(void) { return g_err; }

}  // extern "C"

namespace pip {
namespace {
// The batched kernel in pip_classify: the item descriptors, the kernel (in
// binary32 with its list of undecided pairs, or in binary64), then in the
// filtered mode the binary64 recheck of the list.  Workspace: the list's two
// count words (padded to 256 bytes), the descriptors (padded to 256 bytes),
// the n_points list entries (filtered mode).  It is a pooled, stream-ordered
// allocation, or `fixed` (the static scratch array of pip_classify_noalloc,
// which allocates nothing).
int classify_batched(const Problem &p, DeviceInfo *dev, const pip_options &o, hipStream_t s, bool filtered,
                     unsigned char *fixed)
{
    const int u = o.pairs_per_lane == 1 ? 1 : (o.pairs_per_lane == 4 ? 4 : 2);
    const int tile = clamp_batched_tile(o.lds_slots > 0 ? o.lds_slots : 512, filtered, u, dev);
    const int n_items = (int)((p.n_points + 256 * u - 1) / (256 * u));
    const size_t desc_bytes = ((size_t)n_items * sizeof(ItemDesc) + 255) & ~(size_t)255;
    const size_t bytes = kScratchHead + desc_bytes + (filtered ? (size_t)p.n_points * sizeof(int32_t) : 0);
    void *ws = fixed;
    bool pooled = false;
    if (!fixed) {
        hipError_t e = pool_alloc(&ws, bytes, dev->device, s, &pooled);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(PIP_ENOMEM, "batched workspace of %zu bytes: %s", bytes, hipGetErrorString(e));
        }
    }
    unsigned *count = (unsigned *)ws;
    ItemDesc *desc = (ItemDesc *)((unsigned char *)ws + kScratchHead);
    int32_t *list = (int32_t *)((unsigned char *)ws + kScratchHead + (fixed ? kScratchDesc : desc_bytes));
    int rc = filtered ? launch_fill(count, 2, 0u, s) : PIP_OK;   // list length, long-ring entries
    if (rc == PIP_OK)
        rc = launch_item_desc(p, s, 256 * u, n_items, desc, nullptr, nullptr, nullptr, nullptr);
    if (rc == PIP_OK)
        rc = launch_batched(p, s, filtered, u, tile, filtered ? o.bound_scale : 1.0f, filtered ? o.force_recheck : 0,
                            filtered ? list : nullptr, filtered ? count : nullptr, nullptr, desc, n_items);
    if (rc == PIP_OK && filtered)
        rc = launch_recheck(p, s, list, count, count + 1, dev->cu_count * 8);
    if (!fixed)
        pool_release(ws, pooled, s);
    return rc;
}

int classify_problem(Problem p, const pip_options *opts, void *stream, bool noalloc = false)
{
    pip_options o;
    pip_options_init(&o);
    if (opts) {
        if (opts->struct_size != sizeof(pip_options))
            return fail(PIP_EINVAL, "pip_options.struct_size=%u, expected %zu", opts->struct_size,
                        sizeof(pip_options));
        o = *opts;
    }
    if (o.mode != PIP_MODE_EXACT_FP64 && o.mode != PIP_MODE_FILTERED_FP32)
        return fail(PIP_EINVAL, "unknown mode %d", o.mode);
    if (o.kernel < PIP_KERNEL_AUTO || o.kernel > PIP_KERNEL_BATCHED)
        return fail(PIP_EINVAL, "unknown kernel %d", o.kernel);
    if (o.mode == PIP_MODE_FILTERED_FP32) {
        if (o.kernel != PIP_KERNEL_AUTO && o.kernel != PIP_KERNEL_BATCHED)
            return fail(PIP_EINVAL, "pip_classify runs the filtered mode on the batched kernel only");
        if (p.poly_rings)
            return fail(PIP_ENOTSUP, "the filtered mode takes one ring per polygon");
        if (o.predicate != PIP_PRED_SIDE)
            return fail(PIP_ENOTSUP, "the filtered mode implements the side test (constraint 1) only");
        if (p.n_points > INT32_MAX)
            return fail(PIP_EINVAL, "n_points=%lld: the filtered mode takes fewer than 2^31 pairs",
                        (long long)p.n_points);
    }
    const bool batched = o.mode == PIP_MODE_FILTERED_FP32 || o.kernel == PIP_KERNEL_BATCHED;
    if (batched && noalloc && p.n_points > PIP_NOALLOC_MAX_POINTS)
        return fail(PIP_EINVAL, "n_points=%lld exceeds the static scratch of pip_classify_noalloc (%d points)",
                    (long long)p.n_points, PIP_NOALLOC_MAX_POINTS);
    if (batched && p.n_points > INT32_MAX)
        return fail(PIP_EINVAL, "n_points=%lld: the batched kernel takes fewer than 2^31 pairs",
                    (long long)p.n_points);
    if (o.kernel == PIP_KERNEL_BATCHED && (p.poly_rings || o.predicate != PIP_PRED_SIDE))
        return fail(PIP_ENOTSUP, "the batched kernel takes one ring per polygon and the side test only");
    if (o.predicate != PIP_PRED_SIDE && o.predicate != PIP_PRED_INTERSECTION)
        return fail(PIP_EINVAL, "unknown predicate %d", o.predicate);
    p.pred = o.predicate;
    PIP_TRY(check_host_args(p));
    DeviceInfo *dev = nullptr;
    PIP_TRY(current_device(&dev));
    hipStream_t s = (hipStream_t)stream;
    if (o.validate)
        PIP_TRY(validate_on_device(p, dev, s));
    if (p.n_points == 0)
        return PIP_OK;
    if (batched)
        return classify_batched(p, dev, o, s, o.mode == PIP_MODE_FILTERED_FP32, noalloc ? dev->scratch : nullptr);
    if (o.kernel == PIP_KERNEL_PER_PAIR)
        return launch_per_pair(p, s);
    if (o.kernel == PIP_KERNEL_SEGMENTED)
        return launch_segmented(p, s, o.pairs_per_lane, o.block);
    const int ppl = o.pairs_per_lane > 0 ? o.pairs_per_lane : 4;
    if (o.kernel == PIP_KERNEL_RUNS || (o.kernel == PIP_KERNEL_AUTO && !p.poly_rings)) {
        const int u = ppl == 1 ? 1 : (ppl == 2 ? 2 : 4);
        return launch_runs_batched(p, s, u, nullptr, (int)((p.n_points + 256 * u - 1) / (256 * u)), nullptr, 0);
    }
    return launch_staged(p, s, ppl, clamp_lds_slots(o.lds_slots > 0 ? o.lds_slots : 256, false, ppl, dev));
}
}  // namespace
}  // namespace pip

extern "C" {

int pip_classify(const double *px, const double *py, int64_t n_points, const int64_t *offsets, int64_t n_polys,
                 const double *vx, const double *vy, int64_t n_vertices, const int32_t *point_poly,
                 uint8_t *inside, const pip_options *opts, void *stream)
{
    clear_error();
    Problem p{px, py, n_points, offsets, n_polys, vx, vy, n_vertices, point_poly, inside};
    p.n_rings = n_polys;
    return classify_problem(p, opts, stream);
}

int pip_classify_noalloc(const double *px, const double *py, int64_t n_points, const int64_t *offsets,
                         int64_t n_polys, const double *vx, const double *vy, int64_t n_vertices,
                         const int32_t *point_poly, uint8_t *inside, const pip_options *opts, void *stream)
{
    clear_error();
    Problem p{px, py, n_points, offsets, n_polys, vx, vy, n_vertices, point_poly, inside};
    p.n_rings = n_polys;
    return classify_problem(p, opts, stream, true);
}

int pip_classify_rings(const double *px, const double *py, int64_t n_points, const int64_t *poly_rings,
                       int64_t n_polys, const int64_t *ring_offsets, int64_t n_rings, const double *vx,
                       const double *vy, int64_t n_vertices, const int32_t *point_poly, uint8_t *inside,
                       const pip_options *opts, void *stream)
{
    clear_error();
    if (!poly_rings)
        return fail(PIP_EINVAL, "poly_rings is NULL");
    Problem p{px, py, n_points, ring_offsets, n_polys, vx, vy, n_vertices, point_poly, inside};
    p.poly_rings = poly_rings;
    p.n_rings = n_rings;
    return classify_problem(p, opts, stream);
}

int pip_probe_copy(void *dst, const void *src, int64_t nbytes, void *stream)
{
    clear_error();
    if (nbytes < 0 || (nbytes % 16) != 0 || (nbytes > 0 && (!dst || !src)))
        return fail(PIP_EINVAL, "pip_probe_copy: NULL pointer or nbytes not a non-negative multiple of 16");
    DeviceInfo *dev = nullptr;
    PIP_TRY(current_device(&dev));
    if (nbytes == 0)
        return PIP_OK;
    return launch_copy(dst, src, nbytes, (hipStream_t)stream);
}

int pip_probe_read(const void *src, int64_t nbytes, uint32_t *sink, void *stream)
{
    clear_error();
    if (nbytes < 0 || (nbytes % 16) != 0 || (nbytes > 0 && (!src || !sink)))
        return fail(PIP_EINVAL, "pip_probe_read: NULL pointer or nbytes not a non-negative multiple of 16");
    DeviceInfo *dev = nullptr;
    PIP_TRY(current_device(&dev));
    if (nbytes == 0)
        return PIP_OK;
    return launch_read(src, nbytes, sink, (hipStream_t)stream);
}

int pip_probe_valu(int64_t iterations, double *sink, int64_t *lane_ops, void *stream)
{
    clear_error();
    if (iterations < 1 || iterations > (1 << 24) || !sink || !lane_ops)
        return fail(PIP_EINVAL, "pip_probe_valu: NULL pointer or iterations outside [1, 2^24]");
    DeviceInfo *dev = nullptr;
    PIP_TRY(current_device(&dev));
    return launch_valu_probe((int)iterations, sink, dev->cu_count, lane_ops, (hipStream_t)stream);
}

}  // extern "C"
