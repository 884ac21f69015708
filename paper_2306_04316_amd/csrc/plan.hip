// Plans: a prepared, repeatable classification of fixed device buffers.
//
// A plan owns its workspace (one device allocation, made at creation and
// released at destruction) and, by default, a HIP graph of its step sequence:
//   counters reset -> item order (heaviest first) -> main kernel -> recheck
// so an execution is a single graph launch.  The main kernel is chosen by the
// options, optionally by timing candidate configurations on the plan's own
// data (the autotuner below), with results kept in a small text cache.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "pip_common.h"

struct pip_plan {
    pip::Problem p;
    pip_options o;               // as requested
    pip_plan_config cfg;         // as resolved (after tuning)
    int device = -1;
    int cu_count = 0;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    unsigned *counters = nullptr;   // [0,64) ordering, [64] queue, [65] recheck count
    uint8_t *bucket = nullptr;
    int32_t *order = nullptr;
    pip::ItemDesc *desc = nullptr;    // batched kernel: item descriptors, and in heaviest-first order
    pip::ItemDesc *sdesc = nullptr;
    int32_t *recheck = nullptr;
    unsigned long long *stats = nullptr;   // [256][2] device counters (plans with stats = 1)
    pip::WaveTask *tasks = nullptr;        // wave kernel tasks (filtered batched plans)
    unsigned max_tasks = 0;
    unsigned char *index_ws = nullptr;
    pip::IndexLayout index;
    unsigned long long *segmask = nullptr;   // one ring, no pair index: segment parities per 64-point run
    int seg_hi = 0;                          // segment groups of that walk (0: the runs kernel's own walk)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    bool executed = false;
    hipStream_t last_stream = nullptr;   // the stream of the last execution
    int timed = 0;   // events of the last execution: 0 none, 1 phases, 2 main kernel only
    unsigned span[33] = {0};   // vertex ranges of the 1024-pair work items at creation: max, log2 histogram
    int64_t n_items4 = 0;
};

namespace pip {
namespace {

constexpr int kQueue = 64;
constexpr int kRecheckCount = 65;
constexpr int kSpan = 66;        // [66, 99): item span maximum and log2 histogram
constexpr int kTaskCount = 100;  // wave kernel: tasks listed, queue cursor
constexpr int kTaskCursor = 101;
constexpr int kRecheckWideCount = 102;   // recheck: pairs of long rings appended to the list
constexpr int kCounters = 103;
constexpr int kStatWords = 1024;   // [256][2] 64-bit counters of the batched kernel's stats variant

int item_pairs_of(const pip_plan_config &c) { return 256 * c.pairs_per_lane; }

// Kernels that take work items (runs of 256 * pairs_per_lane pairs) and so
// support the persistent queue and the heaviest-first order.
bool staged_kind(const pip_plan_config &c)
{
    return c.mode == PIP_MODE_FILTERED_FP32 || c.kernel == PIP_KERNEL_STAGED || c.kernel == PIP_KERNEL_RUNS ||
           c.kernel == PIP_KERNEL_BATCHED || c.kernel == PIP_KERNEL_AUTO;
}

int resolve_grid(pip_plan *pl, pip_plan_config &c)
{
    DeviceInfo *dev = nullptr;
    PIP_TRY(current_device(&dev));
    if (c.kernel == PIP_KERNEL_BATCHED) {
        c.lds_slots = clamp_batched_tile(c.lds_slots, c.mode == PIP_MODE_FILTERED_FP32, c.pairs_per_lane, dev);
        c.persistent = 0;   // one workgroup per item only
    } else {
        c.lds_slots = clamp_lds_slots(c.lds_slots, c.mode == PIP_MODE_FILTERED_FP32, c.pairs_per_lane, dev);
    }
    c.n_items = (int)((pl->p.n_points + item_pairs_of(c) - 1) / item_pairs_of(c));
    if (!staged_kind(c) || !c.persistent) {
        c.grid = c.n_items;
        return PIP_OK;
    }
    int nb = 1;
    if (c.mode == PIP_MODE_FILTERED_FP32)
        PIP_TRY(filtered_occupancy(c.pairs_per_lane, c.lds_slots, &nb));
    else if (c.kernel == PIP_KERNEL_RUNS)
        PIP_TRY(runs_occupancy(c.pairs_per_lane, &nb));
    else
        PIP_TRY(staged_occupancy(c.pairs_per_lane, c.lds_slots, &nb));
    const int64_t g = (int64_t)nb * pl->cu_count;
    c.grid = (int)std::min<int64_t>(g, c.n_items);
    return PIP_OK;
}

// The step sequence, in three phases; eager executions record the plan's
// events between them, graph executions get event-record nodes instead.
enum Phase { kPrep = 0, kMain = 1, kRecheck = 2 };

// The staged kernel's tile walk (for vertex ranges beyond the LDS budget)
// comes in a form of its own; it is used when more than 1% of the work items
// exceed the budget (fewer take the scalar-load group walk inside the plain
// form, which keeps the plain form's registers).  The counts are for
// 1024-pair items, an upper bound for smaller items.
bool use_tiles(const pip_plan *pl, int lds_slots)
{
    if (pl->span[0] <= (unsigned)lds_slots)
        return false;
    uint64_t over = 0;
    for (int b = 0; b < 32; ++b)
        if ((2ull << b) - 1 > (uint64_t)lds_slots)   // bucket b holds spans in [2^b, 2^(b+1))
            over += pl->span[1 + b];
    return over * 100 > (uint64_t)pl->n_items4;
}

bool phase_empty(const pip_plan *pl, const pip_plan_config &c, int ph)
{
    if (pl->p.n_points == 0)
        return true;
    if (c.index)
        return ph == kRecheck;
    if (ph == kPrep) {   // needed for the item order, or the counters (queue, recheck count)
        if (!staged_kind(c))
            return true;
        const bool lpt = c.order == 1 && pl->p.point_poly;
        const bool counters = c.mode == PIP_MODE_FILTERED_FP32 || (c.persistent && c.kernel == PIP_KERNEL_RUNS) ||
                              (pl->stats && c.kernel == PIP_KERNEL_BATCHED);
        return !(lpt || counters || c.kernel == PIP_KERNEL_BATCHED);
    }
    if (ph == kRecheck)
        return c.mode != PIP_MODE_FILTERED_FP32;
    return false;
}

int enqueue_phase(pip_plan *pl, const pip_plan_config &c, hipStream_t s, int ph)
{
    const Problem &p = pl->p;
    if (phase_empty(pl, c, ph))
        return PIP_OK;
    if (c.index)
        return ph == kPrep ? launch_index_prep(p, s, pl->index, pl->index_ws)
                           : launch_runs_indexed(p, s, pl->index, pl->index_ws);
    const bool lpt = staged_kind(c) && c.order == 1 && p.point_poly;
    if (ph == kPrep) {
        PIP_TRY(launch_fill(pl->counters + kQueue, kSpan - kQueue, 0u, s));
        PIP_TRY(launch_fill(pl->counters + kTaskCount, 3, 0u, s));   // tasks, cursor, long-ring rechecks
        if (pl->stats && c.kernel == PIP_KERNEL_BATCHED)
            PIP_TRY(launch_fill((unsigned *)pl->stats, kStatWords, 0u, s));
        if (c.kernel == PIP_KERNEL_BATCHED)
            return launch_item_desc(p, s, item_pairs_of(c), c.n_items, pl->desc, pl->bucket, pl->counters,
                                    lpt ? pl->order : nullptr, pl->sdesc);
        if (lpt)
            PIP_TRY(launch_item_order(p, s, item_pairs_of(c), c.n_items, pl->bucket, pl->counters, pl->order));
        return PIP_OK;
    }
    if (ph == kMain) {
        unsigned *queue = c.persistent ? pl->counters + kQueue : nullptr;
        const int32_t *order = lpt ? pl->order : nullptr;
        if (c.kernel == PIP_KERNEL_BATCHED) {
            WaveOut wave;
            if (c.wave_k > 0 && c.mode == PIP_MODE_FILTERED_FP32) {
                wave.wave_k = c.wave_k;
                wave.tasks = pl->tasks;
                wave.task_count = pl->counters + kTaskCount;
                wave.max_tasks = pl->max_tasks;
                wave.cursor = pl->counters + kTaskCursor;
                wave.grid = pl->cu_count * 6;
            }
            return launch_batched(p, s, c.mode == PIP_MODE_FILTERED_FP32, c.pairs_per_lane, c.lds_slots,
                                  pl->o.bound_scale, pl->o.force_recheck, pl->recheck, pl->counters + kRecheckCount,
                                  pl->stats, lpt ? pl->sdesc : pl->desc, c.n_items, wave);
        }
        if (c.mode == PIP_MODE_FILTERED_FP32)
            return launch_filtered(p, s, c.pairs_per_lane, c.lds_slots, pl->o.bound_scale, pl->o.force_recheck,
                                   pl->recheck, pl->counters + kRecheckCount, order, c.n_items, queue, c.grid);
        if (c.kernel == PIP_KERNEL_PER_PAIR)
            return launch_per_pair(p, s);
        if (c.kernel == PIP_KERNEL_SEGMENTED)
            return launch_segmented(p, s, c.pairs_per_lane, 256);
        if (c.kernel == PIP_KERNEL_RUNS && pl->seg_hi > 0)
            return launch_ring_segments(p, s, pl->seg_hi, pl->segmask);
        if (c.kernel == PIP_KERNEL_RUNS)
            return launch_runs_batched(p, s, c.pairs_per_lane, order, c.n_items, queue, c.grid);
        return launch_staged_batched(p, s, c.pairs_per_lane, c.lds_slots, order, c.n_items, c.persistent != 0,
                                     use_tiles(pl, c.lds_slots), c.grid);
    }
    return launch_recheck(p, s, pl->recheck, pl->counters + kRecheckCount, pl->counters + kRecheckWideCount,
                          pl->cu_count * 8);
}

// Enqueue one eager execution of the step sequence with configuration c,
// with the plan's phase events when `timed`.
// timed: 0 no events; 1 markers before the preparation (ev[0]) and after the
// recheck (ev[3]) plus the main kernel's own start and end timestamps (ev[1],
// ev[2]); 2 the main kernel's timestamps only (no extra commands in the stream).
int enqueue(pip_plan *pl, const pip_plan_config &c, hipStream_t s, int timed)
{
    if (timed == 1)
        PIP_HIP_TRY(hipEventRecord(pl->ev[0], s));
    PIP_TRY(enqueue_phase(pl, c, s, kPrep));
    if (timed && !phase_empty(pl, c, kMain)) {
        KernelTimer &kt = kernel_timer();
        kt.start = pl->ev[1];
        kt.stop = pl->ev[2];
        const int rc = enqueue_phase(pl, c, s, kMain);
        kt = KernelTimer{};
        PIP_TRY(rc);
    } else {
        if (timed)
            PIP_HIP_TRY(hipEventRecord(pl->ev[1], s));
        PIP_TRY(enqueue_phase(pl, c, s, kMain));
        if (timed)
            PIP_HIP_TRY(hipEventRecord(pl->ev[2], s));
    }
    PIP_TRY(enqueue_phase(pl, c, s, kRecheck));
    if (timed == 1)
        PIP_HIP_TRY(hipEventRecord(pl->ev[3], s));
    return PIP_OK;
}

void drop_graph(pip_plan *pl)
{
    if (pl->exec)
        (void)hipGraphExecDestroy(pl->exec);
    if (pl->graph)
        (void)hipGraphDestroy(pl->graph);
    pl->exec = nullptr;
    pl->graph = nullptr;
}

// The graph: the whole step sequence captured from one stream, kernel nodes
// only (event-record nodes would add several microseconds per execution;
// phase timings come from eager executions with timing enabled).
int build_graph(pip_plan *pl)
{
    drop_graph(pl);
    hipStream_t cs = nullptr;
    PIP_HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    int rc = PIP_OK;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        rc = fail(PIP_EHIP, "hipStreamBeginCapture failed: %s", hipGetErrorString(e));
    } else {
        rc = enqueue(pl, pl->cfg, cs, 0);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(cs, &g);
        if (rc == PIP_OK && e != hipSuccess)
            rc = fail(PIP_EHIP, "hipStreamEndCapture failed: %s", hipGetErrorString(e));
        pl->graph = g;
        if (rc == PIP_OK) {
            e = hipGraphInstantiate(&pl->exec, g, nullptr, nullptr, 0);
            if (e != hipSuccess)
                rc = fail(PIP_EHIP, "hipGraphInstantiate failed: %s", hipGetErrorString(e));
        }
    }
    (void)hipStreamDestroy(cs);
    if (rc != PIP_OK)
        drop_graph(pl);
    return rc;
}

// ---------------------------------------------------------------- tuning cache
std::string tune_key(const pip_plan *pl)
{
    auto lg = [](int64_t v) {
        int b = 0;
        while (v > 1) {
            v >>= 1;
            ++b;
        }
        return b;
    };
    char buf[160];
    snprintf(buf, sizeof buf, "gfx950:m%d:k%d:n%d:p%d:v%d:i%d%s%s", pl->o.mode, pl->o.kernel, lg(pl->p.n_points),
             lg(pl->p.n_polys), lg(pl->p.n_vertices), pl->p.point_poly ? 1 : 0,
             pl->o.predicate == PIP_PRED_INTERSECTION ? ":c2" : "", pl->p.poly_rings ? ":rings" : "");
    return buf;
}

const char *cache_path(const pip_plan *pl)
{
    if (pl->o.tune_cache && pl->o.tune_cache[0])
        return pl->o.tune_cache;
    const char *e = getenv("PIP_TUNE_CACHE");
    return (e && e[0]) ? e : nullptr;
}

// Kernels a plan's tuner and cache may choose: the work-item kernels that
// support the plan's mode, predicate and ring index, within the kernel the
// caller asked for (AUTO: any of them).
bool kernel_allowed(const pip_plan *pl, int kern)
{
    if (pl->o.kernel != PIP_KERNEL_AUTO && kern != pl->o.kernel)
        return false;
    if (kern == PIP_KERNEL_BATCHED)
        return !pl->p.poly_rings && pl->o.predicate == PIP_PRED_SIDE;
    if (kern == PIP_KERNEL_STAGED)
        return true;
    if (kern == PIP_KERNEL_RUNS)
        return pl->o.mode == PIP_MODE_EXACT_FP64 && !pl->p.poly_rings;
    return false;
}

// Cache lines: "<key> <kernel> <pairs_per_lane> <lds_slots> <persistent> <order> <use_graph> <ms>
// [<wave_k>]" (lines without the last field keep the wave kernel off).
// A cached choice fills only what the caller left open: the kernel when it
// asked for AUTO, pairs per lane and LDS slots when 0, persistence and order
// when -1, the wave kernel's ring size when 0 (an explicit request is never
// overridden).
bool cache_lookup(const pip_plan *pl, pip_plan_config &c)
{
    const char *path = cache_path(pl);
    if (!path)
        return false;
    FILE *f = fopen(path, "r");
    if (!f)
        return false;
    const std::string key = tune_key(pl);
    char line[512], k[200];
    int kern, u, l, pe, od, gr, wk;
    float ms;
    bool found = false;
    while (fgets(line, sizeof line, f)) {
        wk = 0;
        const int nf = sscanf(line, "%199s %d %d %d %d %d %d %f %d", k, &kern, &u, &l, &pe, &od, &gr, &ms, &wk);
        if (nf < 8)
            continue;
        const bool sane = kernel_allowed(pl, kern) && (u == 1 || u == 2 || u == 4) && l >= 16 && l <= 2048 &&
                          (pe == 0 || pe == 1) && (od == 0 || od == 1) && (gr == 0 || gr == 1) &&
                          (wk == 0 || (wk >= 64 && wk <= (1 << 30)));
        if (key == k && sane) {
            if (pl->o.wave_k == 0 && pl->o.mode == PIP_MODE_FILTERED_FP32 && !pl->p.poly_rings)
                c.wave_k = wk;
            c.kernel = kern;
            if (pl->o.pairs_per_lane <= 0)
                c.pairs_per_lane = u;
            if (pl->o.lds_slots <= 0)
                c.lds_slots = l;
            if (pl->o.persistent < 0)
                c.persistent = pe;
            if (pl->o.order < 0)
                c.order = od;
            c.use_graph = gr && pl->o.use_graph && !pl->o.timing;
            c.tune_ms = ms;
            found = true;   // the last matching line wins
        }
    }
    fclose(f);
    return found;
}

void cache_store(const pip_plan *pl, const pip_plan_config &c)
{
    const char *path = cache_path(pl);
    if (!path)
        return;
    FILE *f = fopen(path, "a");
    if (!f)
        return;
    fprintf(f, "%s %d %d %d %d %d %d %.6f %d\n", tune_key(pl).c_str(), c.kernel, c.pairs_per_lane, c.lds_slots,
            c.persistent, c.order, c.use_graph, c.tune_ms, c.wave_k);
    fclose(f);
}

// Time one candidate: median device time (ms) of the whole step sequence over
// up to `reps` eager executions on stream s (after one untimed execution).
// A candidate whose first timed execution exceeds `cutoff` ms is abandoned
// after it (its time is that execution's), and long steps get fewer reps.
int time_candidate(pip_plan *pl, pip_plan_config &c, hipStream_t s, int reps, float cutoff, float *ms_out)
{
    PIP_TRY(resolve_grid(pl, c));
    std::vector<float> t;
    PIP_TRY(enqueue(pl, c, s, 1));
    PIP_HIP_TRY(hipEventSynchronize(pl->ev[3]));
    for (int r = 0; r < reps; ++r) {
        PIP_TRY(enqueue(pl, c, s, 1));
        PIP_HIP_TRY(hipEventSynchronize(pl->ev[3]));
        float a = 0.f;
        PIP_HIP_TRY(hipEventElapsedTime(&a, pl->ev[0], pl->ev[3]));
        t.push_back(a);
        if (r == 0 && (a > cutoff || a > 50.0f))
            break;   // clearly worse than the best so far, or a long step: one timing is enough
    }
    std::sort(t.begin(), t.end());
    *ms_out = t[t.size() / 2];
    return PIP_OK;
}

// Mean wall time per launch (ms) of `reps` back-to-back executions of the
// plan as configured now (graph launches if it has a graph), between two
// events on stream s.
int time_launches(pip_plan *pl, hipStream_t s, int reps, float *ms_out)
{
    hipEvent_t a = nullptr, b = nullptr;
    PIP_HIP_TRY(hipEventCreate(&a));
    int rc = PIP_OK;
    hipError_t e = hipEventCreate(&b);
    if (e != hipSuccess)
        rc = fail(PIP_EHIP, "hipEventCreate failed: %s", hipGetErrorString(e));
    for (int r = 0; r < 2 && rc == PIP_OK; ++r)
        rc = pl->exec ? (hipGraphLaunch(pl->exec, s) == hipSuccess ? PIP_OK : fail(PIP_EHIP, "graph launch"))
                      : enqueue(pl, pl->cfg, s, 0);
    if (rc == PIP_OK && hipEventRecord(a, s) != hipSuccess)
        rc = fail(PIP_EHIP, "hipEventRecord failed");
    for (int r = 0; r < reps && rc == PIP_OK; ++r)
        rc = pl->exec ? (hipGraphLaunch(pl->exec, s) == hipSuccess ? PIP_OK : fail(PIP_EHIP, "graph launch"))
                      : enqueue(pl, pl->cfg, s, 0);
    if (rc == PIP_OK && hipEventRecord(b, s) != hipSuccess)
        rc = fail(PIP_EHIP, "hipEventRecord failed");
    if (rc == PIP_OK && hipEventSynchronize(b) != hipSuccess)
        rc = fail(PIP_EHIP, "hipEventSynchronize failed");
    float ms = 0.f;
    if (rc == PIP_OK && hipEventElapsedTime(&ms, a, b) != hipSuccess)
        rc = fail(PIP_EHIP, "hipEventElapsedTime failed");
    *ms_out = ms / (reps > 0 ? reps : 1);
    (void)hipEventDestroy(a);
    if (b)
        (void)hipEventDestroy(b);
    return rc;
}

int autotune(pip_plan *pl, hipStream_t s)
{
    pip_plan_config best = pl->cfg;
    float best_ms = 1e30f;
    const int reps = pl->o.tune > 1 ? pl->o.tune : 5;
    std::vector<pip_plan_config> cands;
    const int lds_opts[] = {128, 256, 512, 1024};
    const int ppl_opts[] = {1, 2, 4};
    // the batched kernel's split between lane-per-pair walks and the wave
    // kernel (filtered mode, ring size left open): off, or rings from 256 or
    // from 1024 vertices
    std::vector<int> wave_opts = {0};
    if (pl->o.wave_k == 0 && pl->o.mode == PIP_MODE_FILTERED_FP32 && !pl->p.poly_rings)
        wave_opts = {0, 256, 1024};
    // the plan's own untuned choice first: when steps are long the budget ends
    // the search after a few candidates, and it must not end worse than that
    if (kernel_allowed(pl, pl->cfg.kernel))
        cands.push_back(pl->cfg);
    std::vector<int> kernels;
    for (int kern : {PIP_KERNEL_BATCHED, PIP_KERNEL_STAGED, PIP_KERNEL_RUNS})
        if (kernel_allowed(pl, kern))
            kernels.push_back(kern);
    for (int kern : kernels)
        for (int u : ppl_opts)
            for (int l : lds_opts) {
                if (kern == PIP_KERNEL_RUNS && l != lds_opts[0])
                    continue;   // the runs kernel stages nothing
                for (int pe = 0; pe <= (kern == PIP_KERNEL_BATCHED ? 0 : 1); ++pe)
                    for (int od = 0; od <= (pl->p.point_poly ? 1 : 0); ++od)
                        for (int wk : wave_opts) {
                            if (wk && kern != PIP_KERNEL_BATCHED)
                                continue;
                            pip_plan_config c = pl->cfg;
                            c.kernel = kern;
                            c.pairs_per_lane = u;
                            c.lds_slots = l;
                            c.persistent = pe;
                            c.order = od;
                            if (kern == PIP_KERNEL_BATCHED && pl->o.wave_k == 0)
                                c.wave_k = wk;
                            cands.push_back(c);
                        }
            }
    // total budget: about 2 s of device time, or every candidate once for long steps
    float spent = 0.f;
    for (auto &c : cands) {
        float ms = 0.f;
        PIP_TRY(time_candidate(pl, c, s, reps, 1.5f * best_ms, &ms));
        spent += ms * (ms > 50.0f ? 2.f : (float)reps + 1.f);
        if (ms < best_ms) {
            best_ms = ms;
            best = c;
        }
        if (spent > 2000.f && best_ms < 1e29f && best_ms > 20.0f)
            break;
    }
    best.tuned = 1;
    best.tune_ms = best_ms;
    PIP_TRY(resolve_grid(pl, best));
    pl->cfg = best;
    // graph or eager launches: whichever issues the chosen sequence faster
    if (pl->o.use_graph && !pl->o.timing) {
        float eager = 0.f, graph = 0.f;
        pl->cfg.use_graph = 0;
        drop_graph(pl);
        PIP_TRY(time_launches(pl, s, 4 * reps, &eager));
        if (build_graph(pl) == PIP_OK) {
            PIP_TRY(time_launches(pl, s, 4 * reps, &graph));
            pl->cfg.use_graph = graph < eager ? 1 : 0;
        } else {
            clear_error();
        }
        drop_graph(pl);
        log_msg("tuned: kernel %d ppl %d lds %d persistent %d order %d: %.4f ms/step eager, %.4f graph",
                pl->cfg.kernel, pl->cfg.pairs_per_lane, pl->cfg.lds_slots, pl->cfg.persistent, pl->cfg.order, eager,
                graph);
    }
    cache_store(pl, pl->cfg);
    return PIP_OK;
}

// Phase times of the last (timed) execution; waits for its last event only.
int read_timing(pip_plan *pl, float *ms_prep, float *ms_main, float *ms_recheck)
{
    *ms_prep = *ms_recheck = 0.f;
    PIP_HIP_TRY(hipEventSynchronize(pl->ev[pl->timed == 1 ? 3 : 2]));
    PIP_HIP_TRY(hipEventElapsedTime(ms_main, pl->ev[1], pl->ev[2]));
    if (pl->timed == 1) {
        PIP_HIP_TRY(hipEventElapsedTime(ms_prep, pl->ev[0], pl->ev[1]));
        PIP_HIP_TRY(hipEventElapsedTime(ms_recheck, pl->ev[2], pl->ev[3]));
    }
    return PIP_OK;
}

int check_options(const pip_options *opts, pip_options &o)
{
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
    if (o.mode == PIP_MODE_FILTERED_FP32 &&
        (o.kernel == PIP_KERNEL_PER_PAIR || o.kernel == PIP_KERNEL_SEGMENTED || o.kernel == PIP_KERNEL_RUNS))
        return fail(PIP_EINVAL, "the filtered mode runs on the staged or batched kernel only");
    if (o.kernel == PIP_KERNEL_BATCHED && o.predicate != PIP_PRED_SIDE)
        return fail(PIP_ENOTSUP, "the batched kernel implements the side test (constraint 1) only");
    if (o.stats < 0 || o.stats > 1)
        return fail(PIP_EINVAL, "stats must be 0 or 1");
    if (!(o.bound_scale >= 0.0f))
        return fail(PIP_EINVAL, "bound_scale must be >= 0");
    if (o.index && o.mode != PIP_MODE_EXACT_FP64)
        return fail(PIP_EINVAL, "the y-index runs in the exact mode only");
    if (o.timing < 0 || o.timing > 2)
        return fail(PIP_EINVAL, "timing must be 0, 1 or 2");
    if (o.predicate != PIP_PRED_SIDE && o.predicate != PIP_PRED_INTERSECTION)
        return fail(PIP_EINVAL, "unknown predicate %d", o.predicate);
    if (o.predicate != PIP_PRED_SIDE && o.mode != PIP_MODE_EXACT_FP64)
        return fail(PIP_EINVAL, "the filtered mode implements the side test (constraint 1) only");
    return PIP_OK;
}

}  // namespace
}  // namespace pip

using namespace pip;

namespace pip {
namespace {
int plan_create(pip_plan **out, Problem p, const pip_options *opts, void *stream)
{
    const int64_t n_points = p.n_points, n_vertices = p.n_vertices;
    const int64_t *offsets = p.offsets;
    const int32_t *point_poly = p.point_poly;
    if (!out)
        return fail(PIP_EINVAL, "out is NULL");
    *out = nullptr;
    pip_options o;
    PIP_TRY(check_options(opts, o));
    if (p.poly_rings) {
        if (o.mode != PIP_MODE_EXACT_FP64)
            return fail(PIP_ENOTSUP, "the filtered mode takes one ring per polygon");
        if (o.index)
            return fail(PIP_EINVAL, "the y-index takes one ring");
        if (o.kernel == PIP_KERNEL_SEGMENTED || o.kernel == PIP_KERNEL_RUNS)
            return fail(PIP_ENOTSUP, "polygons of several rings run on the staged or per-pair kernel");
    }
    p.pred = o.predicate;
    PIP_TRY(check_host_args(p));
    // pair ids are int32 in the recheck list and the item order, and items are counted in int
    if (n_points > INT32_MAX)
        return fail(PIP_EINVAL, "n_points=%lld: plans take fewer than 2^31 pairs", (long long)n_points);
    if (o.stats && o.kernel != PIP_KERNEL_BATCHED && o.kernel != PIP_KERNEL_AUTO)
        return fail(PIP_EINVAL, "stats counting needs the batched kernel");
    if (o.wave_k < -1)
        return fail(PIP_EINVAL, "wave_k=%d (0 default, -1 off, else a ring size)", o.wave_k);
    DeviceInfo *dev = nullptr;
    PIP_TRY(current_device(&dev));
    hipStream_t s = (hipStream_t)stream;
    if (o.validate)
        PIP_TRY(validate_on_device(p, dev, s));

    pip_plan *pl = new pip_plan;
    pl->p = p;
    pl->o = o;
    pl->device = dev->device;
    pl->cu_count = dev->cu_count;
    pip_plan_config &c = pl->cfg;
    memset(&c, 0, sizeof c);
    c.struct_size = sizeof c;
    c.mode = o.mode;
    c.kernel = o.kernel;
    if (o.kernel == PIP_KERNEL_AUTO) {
        // rings shared by every pair of a large single polygon stream best through
        // scalar loads; batched small rings best through LDS (the filtered mode:
        // the batched kernel, where it applies)
        c.kernel = (o.mode == PIP_MODE_FILTERED_FP32 && !p.poly_rings) ? PIP_KERNEL_BATCHED : PIP_KERNEL_STAGED;
        if (o.mode == PIP_MODE_EXACT_FP64 && !point_poly && !p.poly_rings && n_points > 0) {
            int64_t o2[2] = {0, 0};
            if (hipMemcpy(o2, offsets, sizeof o2, hipMemcpyDeviceToHost) == hipSuccess && o2[1] - o2[0] > 512)
                c.kernel = PIP_KERNEL_RUNS;
            (void)hipGetLastError();
        }
    }
    c.pairs_per_lane = o.pairs_per_lane > 0 ? o.pairs_per_lane : (c.kernel == PIP_KERNEL_BATCHED ? 2 : 4);
    c.lds_slots = o.lds_slots > 0 ? std::min(o.lds_slots, 2048) : (c.kernel == PIP_KERNEL_BATCHED ? 512 : 256);
    // one workgroup per item unless asked: the hardware dispatcher already
    // starts a new workgroup wherever one finishes
    c.persistent = o.persistent > 0 ? 1 : 0;
    c.order = o.order >= 0 ? (o.order ? 1 : 0) : (point_poly ? 1 : 0);
    c.use_graph = (o.use_graph && !o.timing) ? 1 : 0;
    if (c.pairs_per_lane != 1 && c.pairs_per_lane != 2 && c.pairs_per_lane != 4)
        c.pairs_per_lane = 4;
    // the wave kernel takes the large rings of filtered batched plans
    // (0: left to the tuner or the cache, off until they choose)
    c.wave_k = (o.mode == PIP_MODE_FILTERED_FP32 && o.wave_k > 0 && !p.poly_rings) ? std::max(64, o.wave_k) : 0;

    int rc = PIP_OK;
    // workspace: counters | bucket[n_items max] | order[n_items max] | item descriptors, unsorted and
    // sorted [n_items max] | recheck[n_points]
    const int64_t max_items = (n_points + 255) / 256 + 1;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = (off + bytes + 255) & ~(size_t)255;
        return at;
    };
    const size_t o_cnt = take(kCounters * sizeof(unsigned));
    const size_t o_bkt = take((size_t)max_items);
    const size_t o_ord = take((size_t)max_items * sizeof(int32_t));
    const size_t o_dsc = take((size_t)max_items * sizeof(ItemDesc));
    const size_t o_sds = take((size_t)max_items * sizeof(ItemDesc));
    const size_t o_rck = take(o.mode == PIP_MODE_FILTERED_FP32 ? (size_t)std::max<int64_t>(n_points, 1) * 4 : 0);
    const size_t o_st = take(o.stats ? kStatWords * sizeof(unsigned) : 0);
    // wave kernel tasks: one per (work item, large ring with pairs in it); with
    // pairs sorted by polygon at most items + polygons of them (a list that
    // would overflow leaves the extra rings to the batched kernel itself)
    const bool wave_ws = o.mode == PIP_MODE_FILTERED_FP32 && o.wave_k >= 0 && !p.poly_rings;
    const uint64_t mt = wave_ws ? std::min<uint64_t>((uint64_t)max_items + (uint64_t)p.n_polys, 0x7fffffffull) : 0;
    const size_t o_tsk = take((size_t)mt * sizeof(WaveTask));
    if (o.index) {
        if (point_poly) {
            delete pl;
            return fail(PIP_EINVAL, "the y-index needs one polygon (point_poly NULL)");
        }
        pl->index = index_layout(n_points, n_vertices);
        c.index = 1;
        c.kernel = PIP_KERNEL_RUNS;
        c.persistent = 0;
        c.order = 0;
    }
    const size_t o_idx = take(o.index ? pl->index.bytes : 0);
    // one ring for every point: the segmented walk's run masks, used when the
    // ring (its size read now; a later change only changes which exact walk
    // runs) has at least kSegmentMinVertices vertices
    const bool one_ring = !point_poly && !p.poly_rings && p.n_polys == 1 && n_points > 0 && !o.index;
    int seg_hi = 0;
    if (one_ring) {
        int64_t o2[2] = {0, 0};
        if (hipMemcpy(o2, offsets, sizeof o2, hipMemcpyDeviceToHost) == hipSuccess &&
            o2[1] - o2[0] >= kSegmentMinVertices)
            seg_hi = ring_segments_hi(o2[1] - o2[0]);
        (void)hipGetLastError();
    }
    const size_t o_seg = take(seg_hi > 0 ? (size_t)((n_points + 63) / 64) * 8 : 0);
    pl->ws_bytes = off;
    hipError_t e = hipMalloc(&pl->ws, pl->ws_bytes);
    if (e != hipSuccess) {
        delete pl;
        (void)hipGetLastError();
        return fail(PIP_ENOMEM, "plan workspace of %zu bytes: %s", off, hipGetErrorString(e));
    }
    unsigned char *w = (unsigned char *)pl->ws;
    pl->counters = (unsigned *)(w + o_cnt);
    pl->bucket = w + o_bkt;
    pl->order = (int32_t *)(w + o_ord);
    pl->desc = (ItemDesc *)(w + o_dsc);
    pl->sdesc = (ItemDesc *)(w + o_sds);
    pl->recheck = o.mode == PIP_MODE_FILTERED_FP32 ? (int32_t *)(w + o_rck) : nullptr;
    pl->stats = o.stats ? (unsigned long long *)(w + o_st) : nullptr;
    pl->tasks = mt ? (WaveTask *)(w + o_tsk) : nullptr;
    pl->max_tasks = (unsigned)mt;
    pl->index_ws = o.index ? w + o_idx : nullptr;
    pl->segmask = seg_hi > 0 ? (unsigned long long *)(w + o_seg) : nullptr;
    pl->seg_hi = seg_hi;
    for (int k = 0; k < 4 && rc == PIP_OK; ++k) {
        e = hipEventCreate(&pl->ev[k]);
        if (e != hipSuccess)
            rc = fail(PIP_EHIP, "hipEventCreate failed: %s", hipGetErrorString(e));
    }
    if (rc == PIP_OK)
        rc = launch_fill(pl->counters, kCounters, 0u, s);
    if (rc == PIP_OK && pl->stats)
        rc = launch_fill((unsigned *)pl->stats, kStatWords, 0u, s);
    // the largest vertex range of a work item (for the largest items): the
    // staged kernel walks ranges beyond its LDS budget in tiles, in a separate
    // form used only when some item needs it (the data may change between
    // executions; a stale choice only changes which correct path runs)
    if (rc == PIP_OK && n_points > 0) {
        pl->n_items4 = (n_points + 1023) / 1024;
        rc = launch_item_span(p, s, 1024, (int)pl->n_items4, pl->counters + kSpan);
        if (rc == PIP_OK) {
            e = hipMemcpyAsync(pl->span, pl->counters + kSpan, sizeof pl->span, hipMemcpyDeviceToHost, s);
            if (e == hipSuccess)
                e = hipStreamSynchronize(s);
            if (e != hipSuccess)
                rc = fail(PIP_EHIP, "item span: %s", hipGetErrorString(e));
        }
    }
    if (rc == PIP_OK && staged_kind(c) && n_points > 0 && !c.index) {
        pip_plan_config cached = c;
        if (cache_lookup(pl, cached)) {
            c = cached;
            c.tuned = 2;
        } else if (o.tune) {
            rc = autotune(pl, s);
        }
    }
    if (rc == PIP_OK)
        rc = resolve_grid(pl, c);
    if (rc == PIP_OK && c.use_graph) {
        if (build_graph(pl) != PIP_OK) {
            c.use_graph = 0;   // capture unsupported here: run the same sequence eagerly
            log_msg("graph capture failed, running eagerly: %s", pip_last_error());
            clear_error();
            (void)hipGetLastError();
        }
    }
    if (rc != PIP_OK) {
        pip_plan_destroy(pl);
        return rc;
    }
    *out = pl;
    return PIP_OK;
}
}  // namespace
}  // namespace pip

extern "C" {

int pip_plan_create(pip_plan **out, const double *px, const double *py, int64_t n_points, const int64_t *offsets,
                    int64_t n_polys, const double *vx, const double *vy, int64_t n_vertices,
                    const int32_t *point_poly, uint8_t *inside, const pip_options *opts, void *stream)
{
    clear_error();
    Problem p{px, py, n_points, offsets, n_polys, vx, vy, n_vertices, point_poly, inside};
    p.n_rings = n_polys;
    return plan_create(out, p, opts, stream);
}

int pip_plan_create_rings(pip_plan **out, const double *px, const double *py, int64_t n_points,
                          const int64_t *poly_rings, int64_t n_polys, const int64_t *ring_offsets, int64_t n_rings,
                          const double *vx, const double *vy, int64_t n_vertices, const int32_t *point_poly,
                          uint8_t *inside, const pip_options *opts, void *stream)
{
    clear_error();
    if (!poly_rings) {
        if (out)
            *out = nullptr;
        return fail(PIP_EINVAL, "poly_rings is NULL");
    }
    Problem p{px, py, n_points, ring_offsets, n_polys, vx, vy, n_vertices, point_poly, inside};
    p.poly_rings = poly_rings;
    p.n_rings = n_rings;
    return plan_create(out, p, opts, stream);
}

int pip_plan_execute(pip_plan *pl, pip_stats *stats, void *stream)
{
    clear_error();
    if (!pl)
        return fail(PIP_EINVAL, "plan is NULL");
    int dev = -1;
    PIP_HIP_TRY(hipGetDevice(&dev));
    if (dev != pl->device)
        return fail(PIP_EINVAL, "plan belongs to device %d, current device is %d", pl->device, dev);
    hipStream_t s = (hipStream_t)stream;
    if (pl->exec) {
        PIP_HIP_TRY(hipGraphLaunch(pl->exec, s));
        pl->timed = 0;
    } else {
        PIP_TRY(enqueue(pl, pl->cfg, s, pl->o.timing));
        pl->timed = pl->o.timing;
    }
    pl->executed = true;
    pl->last_stream = s;
    if (stats)
        return pip_plan_stats(pl, stats);
    return PIP_OK;
}

int pip_plan_stats(pip_plan *pl, pip_stats *st)
{
    clear_error();
    if (!pl || !st)
        return fail(PIP_EINVAL, "NULL argument");
    memset(st, 0, sizeof *st);
    st->pairs = (uint64_t)pl->p.n_points;
    if (!pl->executed)
        return PIP_OK;
    // the execution's stream, not the null stream: a non-blocking stream is
    // not ordered with the null stream
    PIP_HIP_TRY(hipStreamSynchronize(pl->last_stream));
    if (pl->timed)
        PIP_TRY(read_timing(pl, &st->ms_prep, &st->ms_main, &st->ms_recheck));
    if (pl->recheck) {
        unsigned cnt = 0;
        PIP_HIP_TRY(hipMemcpy(&cnt, pl->counters + kRecheckCount, sizeof cnt, hipMemcpyDeviceToHost));
        st->rechecked_pairs = cnt;
    }
    if (pl->stats && pl->cfg.kernel == PIP_KERNEL_BATCHED) {
        std::vector<unsigned long long> v(kStatWords / 2);
        PIP_HIP_TRY(hipMemcpy(v.data(), pl->stats, v.size() * sizeof(v[0]), hipMemcpyDeviceToHost));
        for (size_t i = 0; i < v.size(); i += 2) {
            st->tests += v[i];
            st->ambiguous_tests += v[i + 1];
        }
    }
    return PIP_OK;
}

int pip_plan_timing(pip_plan *pl, float *ms_prep, float *ms_main, float *ms_recheck)
{
    clear_error();
    if (!pl || !ms_prep || !ms_main || !ms_recheck)
        return fail(PIP_EINVAL, "NULL argument");
    *ms_prep = *ms_main = *ms_recheck = 0.f;
    if (!pl->executed)
        return PIP_OK;
    if (!pl->timed)
        return fail(PIP_ENOTSUP, "the last execution was not timed (create the plan with timing = 1 or 2)");
    return read_timing(pl, ms_prep, ms_main, ms_recheck);
}

int pip_plan_get_config(const pip_plan *pl, pip_plan_config *cfg)
{
    clear_error();
    if (!pl || !cfg)
        return fail(PIP_EINVAL, "NULL argument");
    *cfg = pl->cfg;
    return PIP_OK;
}

int pip_plan_destroy(pip_plan *pl)
{
    clear_error();
    if (!pl)
        return PIP_OK;
    drop_graph(pl);
    for (auto &e : pl->ev)
        if (e)
            (void)hipEventDestroy(e);
    if (pl->ws) {
        (void)hipDeviceSynchronize();   // no enqueued execution may still use the workspace
        (void)hipFree(pl->ws);
    }
    delete pl;
    return PIP_OK;
}

}  // extern "C"
