/*
 * pip.h -- C ABI of the MI355X (gfx950) ray-casting point-in-polygon library.
 *
 * The operation (paper, Method section, "constraint 1", and Algorithm 1):
 * for a point p and a polygon ring v_0 .. v_{k-1} (closed implicitly: the last
 * edge runs from v_{k-1} back to v_0) cast a ray from p in direction (1, 0).
 * Edge (a, b) = (v_i, v_{i+1}) crosses the ray when exactly one of a_y > p_y,
 * b_y > p_y holds (half-open rule: a vertex level with the ray counts as
 * below) and (p - a) . n <= 0 for the edge normal n = (b_y - a_y, a_x - b_x)
 * oriented so n_x > 0.  p is inside when the number of crossings is odd.
 * Every side value is evaluated in IEEE binary64 with the operation order
 * t1 = p_x - a_x, t2 = p_y - a_y, s = t1*n_x + t2*n_y, each operation rounded
 * separately (no fused multiply-add).  Results are therefore bit-identical to
 * a plain CPU binary64 evaluation of the same rule, in every mode.  The
 * paper's second test (constraint 2, see pip_predicate) is available too.
 *
 * Layout (all arrays are DEVICE pointers, caller-owned, and must stay valid
 * until the work enqueued on `stream` completes):
 *   px, py        double[n_points]      query points (SoA)
 *   offsets       int64_t[n_polys + 1]  CSR ring offsets; offsets[0] = 0,
 *                                        non-decreasing, offsets[n_polys] =
 *                                        n_vertices
 *   vx, vy        double[n_vertices]    ring vertices (SoA), rings back to back
 *   point_poly    int32_t[n_points]     pair index: point i is tested against
 *                                        polygon point_poly[i]; may be NULL,
 *                                        then every point is tested against
 *                                        polygon 0 and n_polys must be 1.
 *                                        Sorted (non-decreasing) indices are
 *                                        fastest; any order is correct.
 *   inside        uint8_t[n_points]     output, 1 = inside, 0 = outside;
 *                                        fully overwritten.
 * A ring may repeat its first vertex at its end or not: both give the same
 * result (the repeated edge is horizontal and never crosses).  Rings with
 * fewer than 3 vertices, repeated vertices and self-intersections are legal
 * and follow the same rule (even-odd semantics).  Coordinates must be finite.
 *
 * Streams: `stream` is a hipStream_t passed as void* (NULL = the null stream).
 * Calls enqueue work and return without waiting, except where stated.
 *
 * Errors: every call returns a pip_status; pip_last_error() gives the text
 * of the calling thread's last failure.  With validate = 1 the library also
 * checks the data on the device (and then waits for the stream):
 *   PIP_EINVAL   NULL required pointer, negative count, point_poly == NULL
 *                with n_points > 0 and n_polys != 1, unknown mode/kernel,
 *                bad struct_size
 *   PIP_ERANGE   offsets not a valid CSR over n_vertices, or a point_poly
 *                entry outside [0, n_polys)       (validate = 1 only)
 *   PIP_EDOM     a non-finite coordinate           (validate = 1 only)
 *   PIP_ENOMEM   device workspace allocation failed
 *   PIP_EHIP     a HIP runtime error (text in pip_last_error())
 *   PIP_ENOTSUP  the current device is not gfx950
 * Without validation, out-of-range indices and offsets are clamped so that
 * no access leaves the arrays; the bits of such pairs are unspecified.
 */
#ifndef PIP_H
#define PIP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PIP_ABI_VERSION 4

#if defined(__GNUC__) || defined(__clang__)
#define PIP_API __attribute__((visibility("default")))
#else
#define PIP_API
#endif

typedef enum {
    PIP_OK = 0,
    PIP_EINVAL = -1,
    PIP_ERANGE = -2,
    PIP_EDOM = -3,
    PIP_ENOMEM = -4,
    PIP_EHIP = -5,
    PIP_ENOTSUP = -6
} pip_status;

/* Arithmetic of the bulk of the edge tests.  Both modes give the same bits. */
typedef enum {
    /* every side value in binary64, in the rule's operation order */
    PIP_MODE_EXACT_FP64 = 0,
    /* binary32 side values on per-polygon re-centred coordinates with a
     * proven forward error bound; a pair with any undecided edge is re-run in
     * binary64 in the rule's operation order */
    PIP_MODE_FILTERED_FP32 = 1
} pip_mode;

/* The test that decides whether a straddling edge is crossed (paper, Method
 * section).  Both evaluate every operation in binary64 (division correctly
 * rounded, no fused multiply-add) and use the half-open straddle rule. */
typedef enum {
    /* constraint 1 (Algorithm 1): (p - a) . n <= 0, n = (b_y - a_y, a_x - b_x)
     * oriented so n_x > 0 -- the default */
    PIP_PRED_SIDE = 0,
    /* constraint 2 (Algorithm 2): lambda = (p_y - a_y) / (b_y - a_y),
     * x = a_x + lambda * (b_x - a_x), crossed when x >= p_x (the Method
     * section's comparison; its listing uses a strict one) */
    PIP_PRED_INTERSECTION = 1
} pip_predicate;

/* Work mapping of the main kernel. */
typedef enum {
    PIP_KERNEL_AUTO = 0,
    /* one lane per pair, every vertex fetched per lane: the plain baseline */
    PIP_KERNEL_PER_PAIR = 1,
    /* one lane per pair; the lanes of a wavefront that share a polygon run
     * together with the polygon's vertices wave-uniform (scalar loads) */
    PIP_KERNEL_SEGMENTED = 2,
    /* one lane per pair; a workgroup copies the rings its (sorted) pairs
     * test into LDS once and every lane walks its own ring from there;
     * workgroups whose rings do not fit fall back to the segmented walk */
    PIP_KERNEL_STAGED = 3,
    /* one lane per pair; each wavefront splits its pairs into runs of equal
     * polygon id (at most 64 pairs each) and walks each run's ring
     * wave-uniformly: an exact straddle pass into per-lane bit words, then
     * side values only for each lane's straddling edges */
    PIP_KERNEL_RUNS = 4,
    /* one lane per pair, both modes; a workgroup walks the vertex range of its
     * (sorted) pairs in LDS tiles, builds every edge's record there once
     * (binary64, or binary32 re-centred on the ring's first vertex in the
     * filtered mode) and each lane walks its own ring: straddle tests exact
     * (binary64 comparisons) in both modes, side values only for straddling
     * edges.  Constraint 1, one ring per polygon. */
    PIP_KERNEL_BATCHED = 5
} pip_kernel;

typedef struct {
    uint32_t struct_size;   /* = sizeof(pip_options) */
    int32_t mode;           /* pip_mode */
    int32_t kernel;         /* pip_kernel */
    int32_t validate;       /* 1: check the data on the device first (synchronises) */
    int32_t pairs_per_lane; /* tuning, segmented kernel: pairs per lane (1, 2, 4, 8); 0 = default */
    int32_t block;          /* tuning: threads per workgroup (64, 128, 256); 0 = default */
    int32_t lds_slots;      /* tuning, staged kernel: edges a workgroup can stage in
                               LDS (48 bytes each exact, 37 filtered; at most 2048);
                               0 = default */
    int32_t persistent;     /* plans: 1 = a resident grid walks the work items
                               (staged exact kernel: fixed stride, polygon ranges
                               looked up 64 items ahead; other kernels: an
                               atomic queue), 0 or -1 = one workgroup per item
                               (default) */
    int32_t order;          /* plans: 1 = items heaviest first (estimated edges x
                               pairs), 0 = natural order, -1 = automatic */
    int32_t use_graph;      /* plans: 1 = capture the step sequence in a HIP graph
                               (ignored with timing = 1) */
    int32_t tune;           /* plans: 0 = no tuning; n > 0 = time the candidate
                               configurations on the plan's data at creation (n
                               timed runs each, n = 1 means 5) and keep the fastest */
    int32_t force_recheck;  /* filtered mode, for testing: re-run every pair in
                               binary64 (results are unchanged) */
    float bound_scale;      /* filtered mode, for testing only: multiplies the proven
                               error bound; 1 is the only value that guarantees
                               bit-exact results (0 disables the bound) */
    const char *tune_cache; /* plans: tuning cache file; NULL = environment variable
                               PIP_TUNE_CACHE, else no cache */
    int32_t timing;         /* plans: 1 = record the phase times of every execution
                               (markers before the preparation and after the
                               recheck, and the main kernel's own start and end
                               timestamps); 2 = the main kernel's timestamps only
                               (no extra commands in the stream).  Timed plans
                               execute eagerly, not as a graph. */
    int32_t predicate;      /* pip_predicate (the filtered mode supports PIP_PRED_SIDE only) */
    int32_t index;          /* plans, exact mode, one polygon (point_poly NULL):
                               1 = build a y-range tree over the ring's edges and
                               visit the points in y order, so whole groups of
                               edges are skipped by comparisons (same bits; work
                               no longer proportional to every edge) */
    int32_t stats;          /* plans, PIP_KERNEL_BATCHED: 1 = count point-edge tests
                               and undecided binary32 side tests on the device at
                               every execution (a kernel variant with counters;
                               pip_stats.tests / ambiguous_tests), 0 = no counts */
    int32_t wave_k;         /* plans, filtered mode, PIP_KERNEL_BATCHED: pairs whose ring
                               has at least wave_k vertices are classified by one
                               workgroup per (ring, work item) whose wavefronts take
                               64 edges per lane group and the point wave-uniform,
                               crossings combined by ballot, popcount and XOR parity
                               (paper, Method section, constraint 1; same bits).
                               0 = left to the tuner (off, 256 or 1024) or the
                               tuning cache, off without them; -1 = off; values
                               below 64 mean 64 */
} pip_options;

/* Configuration a plan runs with (after automatic choices and tuning). */
typedef struct {
    uint32_t struct_size;
    int32_t mode;
    int32_t kernel;
    int32_t pairs_per_lane;
    int32_t lds_slots;
    int32_t persistent;
    int32_t order;
    int32_t use_graph;      /* 1 if executions are graph launches */
    int32_t grid;           /* workgroups of the main kernel */
    int32_t n_items;        /* work items (256 * pairs_per_lane pairs each) */
    int32_t tuned;          /* 0 = defaults/options, 1 = autotuned now, 2 = from the cache */
    float tune_ms;          /* tuned step time (ms), when tuned */
    int32_t index;          /* 1 if the plan runs the y-indexed path */
    int32_t wave_k;         /* ring size from which the wave kernel takes the pairs (0: off) */
} pip_plan_config;

/* Figures of a plan's last execution (see pip_plan_stats). */
typedef struct {
    uint64_t pairs;             /* pairs the plan classifies */
    uint64_t tests;             /* point-edge tests (sum of the tested rings'
                                   vertex counts), counted on the device by plans
                                   created with stats = 1; 0 otherwise */
    uint64_t ambiguous_tests;   /* filtered mode, stats = 1: side tests whose
                                   binary32 value fell inside the error bound (a
                                   pair with any such test is rechecked) */
    uint64_t rechecked_pairs;   /* pairs re-run in binary64 (filtered mode) */
    float ms_prep;              /* device time: counter resets and item ordering */
    float ms_main;              /* device time: main kernel */
    float ms_recheck;           /* device time: binary64 recheck (filtered mode) */
} pip_stats;

typedef struct pip_plan pip_plan;

/* Fills *opts with the defaults (exact binary64, automatic kernel, no validation). */
PIP_API void pip_options_init(pip_options *opts);

/* ABI version of the loaded library (PIP_ABI_VERSION it was built with). */
PIP_API int pip_abi_version(void);

/* Text of the calling thread's last non-OK status ("" if none). */
PIP_API const char *pip_last_error(void);

/*
 * Classify n_points points (see the layout above).  opts may be NULL
 * (defaults).  n_points == 0 is a no-op.  Asynchronous on `stream` unless
 * opts->validate.  The plan-only options (persistent, order, use_graph, tune,
 * tune_cache, timing, stats) are ignored here.
 * PIP_MODE_EXACT_FP64 allocates nothing on the device.
 * PIP_MODE_FILTERED_FP32 runs the batched kernel (PIP_KERNEL_AUTO or
 * PIP_KERNEL_BATCHED; constraint 1, one ring per polygon, n_points below
 * 2^31, else PIP_EINVAL) followed by the binary64 recheck; its list of
 * undecided pairs (4 bytes per point) is a stream-ordered allocation from a
 * device-memory pool of the library's own (one per device, released memory
 * kept for later calls), freed in stream order after the recheck.
 */
PIP_API int pip_classify(const double *px, const double *py, int64_t n_points,
                 const int64_t *offsets, int64_t n_polys,
                 const double *vx, const double *vy, int64_t n_vertices,
                 const int32_t *point_poly, uint8_t *inside,
                 const pip_options *opts, void *stream);

/* Largest n_points that pip_classify_noalloc takes on the batched kernel
   (the filtered mode, or PIP_KERNEL_BATCHED in the exact mode). */
#define PIP_NOALLOC_MAX_POINTS 4194304

/*
 * For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: pip_classify
 * with its workspace taken from a static device array of the library's own
 * instead of an allocation.  The array holds the batched kernel's work-item
 * descriptors and the filtered mode's count words and list of undecided pairs
 * for up to PIP_NOALLOC_MAX_POINTS points (16 MiB + 384 KiB + 256 bytes; one
 * copy per device, held until the process ends); the other exact-mode kernels
 * need none.  Same arguments, results and errors as pip_classify, plus
 * PIP_EINVAL for n_points > PIP_NOALLOC_MAX_POINTS on the batched kernel
 * (checked before any device call).  Calls nothing that allocates device
 * memory.  Every call on one device shares that device's array, which keeps
 * the last call's contents (the count word is cleared by a kernel at the
 * start of each call): calls that overlap on one device -- on different
 * streams or from different threads -- race, and their results are
 * unspecified.
 */
PIP_API int pip_classify_noalloc(const double *px, const double *py, int64_t n_points,
                         const int64_t *offsets, int64_t n_polys,
                         const double *vx, const double *vy, int64_t n_vertices,
                         const int32_t *point_poly, uint8_t *inside,
                         const pip_options *opts, void *stream);

/*
 * Plans: prepare a repeatable classification of fixed device buffers (the
 * arguments are those of pip_classify).  The plan owns a device workspace
 * (allocated here, released by pip_plan_destroy: a few bytes per pair) and,
 * with use_graph, a HIP graph of its step sequence:
 *   counter resets -> work-item ordering -> main kernel -> binary64 recheck
 * so that pip_plan_execute is one graph launch.  Both modes are accepted;
 * the filtered mode (PIP_MODE_FILTERED_FP32) evaluates in binary32 with a
 * proven error bound and re-runs undecided pairs in binary64, with the same
 * bits as the exact mode (work items whose rings exceed its LDS budget are
 * classified in binary64 directly, their rings walked in LDS tiles).  With tune, creation times candidate
 * configurations on the given data (this runs the classification several
 * times on `stream` and waits for it).  The plan reads the buffers' contents
 * at each execution, so new data in the same buffers needs no new plan; new
 * buffer addresses do.  A plan belongs to the device current at creation.
 * Executions of one plan must not overlap (they share its workspace).
 */
PIP_API int pip_plan_create(pip_plan **out,
                    const double *px, const double *py, int64_t n_points,
                    const int64_t *offsets, int64_t n_polys,
                    const double *vx, const double *vy, int64_t n_vertices,
                    const int32_t *point_poly, uint8_t *inside,
                    const pip_options *opts, void *stream);

/*
 * Polygons of several rings (holes, detached parts) -- an extension beyond
 * the paper, whose polygon is one closed ring: the even-odd rule is applied
 * over all edges of all rings of the polygon, each ring closing on itself and
 * no edge joining two rings, i.e. the parity is the XOR of the rings'
 * parities (Method section, constraint 1 or 2 per edge as selected).
 *   poly_rings   [n_polys + 1] int64, device: polygon q owns rings
 *                poly_rings[q] .. poly_rings[q+1]-1 (poly_rings[0] = 0,
 *                monotone, poly_rings[n_polys] = n_rings)
 *   ring_offsets [n_rings + 1] int64, device: ring r owns vertices
 *                ring_offsets[r] .. ring_offsets[r+1]-1 (a CSR over
 *                n_vertices, as `offsets` above)
 * Every other argument, the error behaviour and the ownership rules are those
 * of pip_classify / pip_plan_create (validate = 1 also checks poly_rings).
 * Kernels: PIP_KERNEL_AUTO (= staged), PIP_KERNEL_STAGED, PIP_KERNEL_PER_PAIR;
 * exact mode only; no y-index (PIP_ENOTSUP / PIP_EINVAL otherwise).
 * poly_rings NULL is PIP_EINVAL.  With one ring per polygon the results are
 * those of pip_classify on ring_offsets.
 */
PIP_API int pip_classify_rings(const double *px, const double *py, int64_t n_points,
                       const int64_t *poly_rings, int64_t n_polys,
                       const int64_t *ring_offsets, int64_t n_rings,
                       const double *vx, const double *vy, int64_t n_vertices,
                       const int32_t *point_poly, uint8_t *inside,
                       const pip_options *opts, void *stream);

PIP_API int pip_plan_create_rings(pip_plan **out,
                          const double *px, const double *py, int64_t n_points,
                          const int64_t *poly_rings, int64_t n_polys,
                          const int64_t *ring_offsets, int64_t n_rings,
                          const double *vx, const double *vy, int64_t n_vertices,
                          const int32_t *point_poly, uint8_t *inside,
                          const pip_options *opts, void *stream);

/* Enqueue one execution on `stream`.  stats NULL: asynchronous.  stats
 * non-NULL: waits for the execution to complete on `stream` and fills *stats
 * as pip_plan_stats does. */
PIP_API int pip_plan_execute(pip_plan *plan, pip_stats *stats, void *stream);

/* Waits for the plan's last execution (synchronises the stream it was
 * enqueued on, which must still exist) and reports its figures (the phase
 * times only when the plan was created with timing = 1). */
PIP_API int pip_plan_stats(pip_plan *plan, pip_stats *stats);

/*
 * Device time (ms) of the last execution's phases: preparation (from its
 * start to the main kernel's start), main kernel (its own start and end
 * timestamps), recheck (to its end).  Needs a plan created with timing = 1,
 * or timing = 2 (main kernel only; the other two are 0).  PIP_ENOTSUP
 * otherwise.  Waits only for that execution's end (not for the stream), so it
 * can be called while later work is still queued.
 */
PIP_API int pip_plan_timing(pip_plan *plan, float *ms_prep, float *ms_main, float *ms_recheck);

/* The configuration the plan runs with. */
PIP_API int pip_plan_get_config(const pip_plan *plan, pip_plan_config *cfg);

/* Waits for the device, then releases the plan's workspace and graph. NULL is a no-op. */
PIP_API int pip_plan_destroy(pip_plan *plan);

/*
 * Candidate pairs by bounding box -- the step before classification (the
 * paper's data preparation kept the points inside the polygon's bounding box,
 * Simulation section; here for many polygons at once).  Pair (i, q) is a
 * candidate when point i lies in the closed box [min x, max x] x [min y, max y]
 * of polygon q's vertices (all its rings).  Exact (comparisons only).
 *
 * pip_join_create: points px/py [n_points] and polygons as for pip_classify
 * (offsets [n_polys + 1], poly_rings NULL) or pip_classify_rings (poly_rings
 * [n_polys + 1] and ring offsets [n_rings + 1]); all device pointers, which
 * must stay valid until pip_join_fill's work has completed.  Builds a grid
 * over the points, counts the candidates, synchronises `stream` and returns
 * their number in *n_pairs.  The join owns its workspace (about 40 bytes per
 * point and per polygon).  n_points and n_polys must be below 2^31.
 * Finite coordinates are required (non-finite ones give unspecified pairs).
 * Errors: PIP_EINVAL (NULL or negative arguments), PIP_ENOMEM, PIP_EHIP,
 * PIP_ENOTSUP (not gfx950).
 *
 * pip_join_fill: writes the n_pairs candidates, grouped by polygon in
 * ascending order (the order the classification kernels want; within a
 * polygon the order is not specified): pair_point[k] (int64 point index),
 * pair_poly[k] (int32, usable as point_poly), pair_px/pair_py[k] (the
 * point's coordinates, usable as px/py).  Device pointers with n_pairs
 * entries; any of them may be NULL (not written).  Asynchronous on `stream`.
 */
typedef struct pip_join pip_join;

PIP_API int pip_join_create(pip_join **out, const double *px, const double *py, int64_t n_points,
                    const int64_t *poly_rings, int64_t n_polys,
                    const int64_t *offsets, int64_t n_rings,
                    const double *vx, const double *vy, int64_t n_vertices,
                    int64_t *n_pairs, void *stream);

PIP_API int pip_join_fill(pip_join *join, int64_t *pair_point, int32_t *pair_poly,
                  double *pair_px, double *pair_py, void *stream);

/*
 * Device time (ms) of a join's kernels, without its host synchronisations
 * and allocations: *ms_count covers pip_join_create's two phases of kernels
 * (grid and sort of the points, polygon boxes, unit and pair counts), *ms_fill
 * pip_join_fill's kernel.  Waits for the fill to complete.  PIP_EINVAL when
 * pip_join_fill has not run on a join with pairs (both 0 for a join without
 * pairs).
 */
PIP_API int pip_join_timing(pip_join *join, float *ms_count, float *ms_fill);

/* Waits for the device, then releases the join's workspace.  NULL is a no-op.
 * The workspace comes from a device-memory pool of the library's own (one per
 * device), which keeps released memory for later joins instead of returning
 * it to the driver (at most what the joins alive at one time held). */
PIP_API int pip_join_destroy(pip_join *join);

/*
 * Diagnostic: copy nbytes (a multiple of 16) from src to dst with a plain
 * streaming kernel.  Used to calibrate HBM traffic counters against a
 * kernel of known size.  The pointers may be NULL when nbytes is 0.
 * Asynchronous on `stream`.
 */
PIP_API int pip_probe_copy(void *dst, const void *src, int64_t nbytes, void *stream);

/*
 * Diagnostic: read nbytes (a multiple of 16) of device memory at src once,
 * with a plain streaming kernel, writing at most one 32-bit word of the
 * device buffer sink (>= 4 bytes; its contents are meaningless).  Measures
 * the read-stream bandwidth that read-dominated kernels are compared with.
 * The pointers may be NULL when nbytes is 0.  Asynchronous on `stream`.
 */
PIP_API int pip_probe_read(const void *src, int64_t nbytes, uint32_t *sink, void *stream);

/*
 * Diagnostic: the vector-ALU issue rate.  Launches eight 256-thread
 * workgroups per compute unit (eight wavefronts per SIMD), each thread
 * running `iterations` (1 .. 2^24) rounds of eight independent binary64
 * additions, one full-rate vector instruction each; *lane_ops receives the
 * number of lane operations the launch performs (set before the launch).
 * At most one 8-byte word of the device buffer sink is written (its contents
 * are meaningless).  Time the launch to get lane operations per second, the
 * measured counterpart of the VALU lane peak that instruction-bound kernels
 * are compared with.  Asynchronous on `stream`.
 */
PIP_API int pip_probe_valu(int64_t iterations, double *sink, int64_t *lane_ops, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* PIP_H */
