/*
 * CPU oracle for the ray-casting point-in-polygon test -- TEST INFRASTRUCTURE.
 *
 * This file is the slow, obviously-correct reference that the GPU library is
 * checked against.  It is used only by the tests, by the smoke check and by the
 * benchmark's CPU-baseline leg; the product path never links or calls it, and it
 * shares no code, header or table with the GPU library.
 *
 * What it computes (paper, Method section, "constraint 1", and Algorithm 1):
 *   For a query point p and a closed ring of vertices v_0 .. v_{k-1} (the ring
 *   closes implicitly: the last edge runs from v_{k-1} back to v_0), cast a ray
 *   from p in direction (1, 0).  Edge (a, b) = (v_i, v_{i+1}) is a candidate
 *   crossing when its endpoints lie on opposite sides of the ray's line
 *   y = p_y.  For a candidate, take the edge normal n = (b_y - a_y, a_x - b_x),
 *   negate it if its x component is negative (so n makes an acute angle with
 *   the ray direction), and count the edge when (p - a) . n <= 0, i.e. when p
 *   lies on or to the left of the edge, so the crossing is at or to the right
 *   of p.  The point is inside when the count is odd.
 *
 * Readings taken where the paper is silent or ambiguous:
 *   - Straddle rule: the paper's product test f_i * f_{i+1} <= 0 counts both
 *     edges that meet at a vertex lying exactly on the ray.  We use the
 *     half-open form: the edge straddles iff exactly one endpoint has
 *     y > p_y (a vertex level with the ray counts as below).  Comparisons only,
 *     so it is exact and never underflows.  A horizontal edge never straddles.
 *   - Anchor: a = v_i, the first endpoint in stored order (as the listing).
 *   - Operation order: t1 = p_x - a_x, t2 = p_y - a_y, s = t1*n_x + t2*n_y,
 *     each operation rounded separately in IEEE binary64 round-to-nearest-even
 *     with no fused multiply-add (build with -ffp-contract=off).
 *   - Boundary: s <= 0 counts (a point on an edge counts that edge).
 *   - Degenerate rings (k < 3, repeated vertices, self-intersections) get no
 *     special case: the rule above is applied as is (even-odd semantics).
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -shared -fPIC -pthread
 *
 * PIP_ORACLE_MUTANT (compile-time, tests only): plants one deliberate mistake
 * so the test suite can show that its pins catch it.  0 / undefined = correct.
 */
#include <stdint.h>
#include <stdlib.h>
#include <pthread.h>

#ifndef PIP_ORACLE_MUTANT
#define PIP_ORACLE_MUTANT 0
#endif

/* Whether edge (a, b) counts for the ray from point (x, y): the straddle
 * test, then the side of p against the edge's oriented normal. */
static int edge_counts(double x, double y, double ax, double ay, double bx, double by)
{
    /* candidate crossing: endpoints on opposite sides of y = p_y (half-open) */
#if PIP_ORACLE_MUTANT == 5
    int a_above = ay >= y, b_above = by >= y;
#else
    int a_above = ay > y, b_above = by > y;
#endif
    if (a_above == b_above)
        return 0;

    /* edge normal, oriented to make an acute angle with the ray (1, 0) */
    double nx = by - ay;
#if PIP_ORACLE_MUTANT == 6
    double ny = bx - ax;
#else
    double ny = ax - bx;
#endif
#if PIP_ORACLE_MUTANT != 3
    if (nx < 0) {
        nx = -nx;
        ny = -ny;
    }
#endif
    /* side of p relative to the edge's line, anchored at a */
#if PIP_ORACLE_MUTANT == 2
    double t1 = x - bx, t2 = y - by;
#else
    double t1 = x - ax, t2 = y - ay;
#endif
#if PIP_ORACLE_MUTANT == 7
    double s = t1 * ny + t2 * nx;
#else
    double s = t1 * nx + t2 * ny;
#endif
#if PIP_ORACLE_MUTANT == 1
    return s < 0;
#else
    return s <= 0;
#endif
}

/* Parity of the ray crossings of point (x, y) against the ring vx/vy[0..k). */
static int ring_parity(double x, double y, const double *vx, const double *vy, int64_t k)
{
    int64_t count = 0;
#if PIP_ORACLE_MUTANT == 4
    int64_t nedges = k > 0 ? k - 1 : 0;     /* mutant: closing edge dropped */
#else
    int64_t nedges = k;
#endif
    for (int64_t i = 0; i < nedges; ++i) {
        int64_t j = (i + 1 == k) ? 0 : i + 1;
        count += edge_counts(x, y, vx[i], vy[i], vx[j], vy[j]);
    }
    return (int)(count & 1);
}

/*
 * Constraint 2 (paper, Method section, second way of testing the constraint,
 * eqs. lamda_eq1, lambda, find_x, and Algorithm 2): for a straddling edge
 * (same half-open rule as above) with direction d = b - a, the ray meets the
 * edge's line at lambda = (p_y - a_y) / d_y, x = a_x + lambda * d_x; the edge
 * counts when x >= p_x ("x >= p_x" as the Method section states; Algorithm 2's
 * listing uses a strict comparison -- reading taken: the text's, so that a
 * point on an edge counts that edge as in constraint 1).  Each operation is
 * rounded in binary64, the division correctly rounded, no fused multiply-add.
 */
static int ring_parity_c2(double x, double y, const double *vx, const double *vy, int64_t k)
{
    int64_t count = 0;
    for (int64_t i = 0; i < k; ++i) {
        int64_t j = (i + 1 == k) ? 0 : i + 1;
        double ax = vx[i], ay = vy[i];
        double bx = vx[j], by = vy[j];
        if ((ay > y) == (by > y))
            continue;
        double dx = bx - ax;
        double dy = by - ay;
        double lam = (y - ay) / dy;
        double xn = ax + lam * dx;
        if (xn >= x)
            ++count;
    }
    return (int)(count & 1);
}

typedef struct {
    const double *px, *py;
    const int64_t *poly_rings;   /* NULL: ring q is polygon q */
    const int64_t *offsets;      /* ring vertex ranges */
    const double *vx, *vy;
    const int32_t *point_poly;
    uint8_t *inside;
    int64_t begin, end;
    int predicate;
} oracle_job;

static int one_ring(const oracle_job *j, double x, double y, int64_t r)
{
    int64_t b = j->offsets[r], e = j->offsets[r + 1];
    return j->predicate == 2 ? ring_parity_c2(x, y, j->vx + b, j->vy + b, e - b)
                             : ring_parity(x, y, j->vx + b, j->vy + b, e - b);
}

/*
 * Polygons made of several rings (holes, or several separate parts): the
 * even-odd rule counts the crossings of all edges of all rings, each ring
 * closing on itself and no edge joining two rings, so the parity is the XOR
 * of the rings' parities.  (An extension beyond the paper, whose polygon is a
 * single closed ring; on a one-ring polygon it is exactly the rule above.)
 */
static int poly_parity(const oracle_job *j, double x, double y, int64_t q)
{
    if (!j->poly_rings)
        return one_ring(j, x, y, q);
    int64_t r0 = j->poly_rings[q], r1 = j->poly_rings[q + 1];
#if PIP_ORACLE_MUTANT == 8
    /* mutant: the polygon's rings walked as one chain (edges joining rings) */
    if (r1 <= r0)
        return 0;
    int64_t b = j->offsets[r0], e = j->offsets[r1];
    return ring_parity(x, y, j->vx + b, j->vy + b, e - b);
#else
    int par = 0;
    for (int64_t r = r0; r < r1; ++r)
        par ^= one_ring(j, x, y, r);
    return par;
#endif
}

static void *oracle_worker(void *arg)
{
    oracle_job *j = (oracle_job *)arg;
    for (int64_t i = j->begin; i < j->end; ++i) {
        int64_t q = j->point_poly ? (int64_t)j->point_poly[i] : 0;
        j->inside[i] = (uint8_t)poly_parity(j, j->px[i], j->py[i], q);
    }
    return NULL;
}

static int classify_impl(const double *px, const double *py, int64_t n_points,
                         const int64_t *poly_rings, const int64_t *offsets, int64_t n_polys,
                         const double *vx, const double *vy,
                         const int32_t *point_poly, uint8_t *inside, int nthreads, int predicate)
{
    if (n_points < 0 || n_polys < 1 || !offsets || !inside)
        return -1;
    if (n_points == 0)
        return 0;
    if (!px || !py)
        return -1;
    if (!point_poly && n_polys != 1)
        return -1;
    if (point_poly) {
        for (int64_t i = 0; i < n_points; ++i)
            if (point_poly[i] < 0 || point_poly[i] >= n_polys)
                return -1;
    }
    if (nthreads < 1)
        nthreads = 1;
    if (nthreads > 256)
        nthreads = 256;
    if ((int64_t)nthreads > n_points)
        nthreads = (int)n_points;

    oracle_job jobs[256];
    pthread_t tids[256];
    for (int t = 0; t < nthreads; ++t) {
        jobs[t].px = px; jobs[t].py = py;
        jobs[t].poly_rings = poly_rings;
        jobs[t].offsets = offsets;
        jobs[t].vx = vx; jobs[t].vy = vy;
        jobs[t].point_poly = point_poly;
        jobs[t].inside = inside;
        jobs[t].begin = n_points * t / nthreads;
        jobs[t].end = n_points * (t + 1) / nthreads;
        jobs[t].predicate = predicate;
    }
    int started = 0;
    for (int t = 1; t < nthreads; ++t) {
        if (pthread_create(&tids[t], NULL, oracle_worker, &jobs[t]) != 0)
            break;
        started = t;
    }
    oracle_worker(&jobs[0]);
    for (int t = 1; t <= started; ++t)
        pthread_join(tids[t], NULL);
    for (int t = started + 1; t < nthreads; ++t)   /* threads that failed to start */
        oracle_worker(&jobs[t]);
    return 0;
}

/*
 * Classify n_points points with constraint 1 (the normal-side test; see the
 * top of this file).  Point i is tested against polygon point_poly[i] (or
 * polygon 0 when point_poly is NULL).  Polygon q's ring is
 * vx/vy[offsets[q] .. offsets[q+1]).  All pointers are host pointers.
 * Writes inside[i] = 1 (inside) or 0 (outside).  Uses up to nthreads POSIX
 * threads over contiguous ranges of points (results do not depend on it).
 * Returns 0 on success, -1 on bad arguments.
 */
int pip_oracle_classify(const double *px, const double *py, int64_t n_points,
                        const int64_t *offsets, int64_t n_polys,
                        const double *vx, const double *vy,
                        const int32_t *point_poly, uint8_t *inside, int nthreads)
{
    return classify_impl(px, py, n_points, NULL, offsets, n_polys, vx, vy, point_poly, inside, nthreads, 1);
}

/* The same with constraint 2 (parametric intersection; see ring_parity_c2). */
int pip_oracle_classify_c2(const double *px, const double *py, int64_t n_points,
                           const int64_t *offsets, int64_t n_polys,
                           const double *vx, const double *vy,
                           const int32_t *point_poly, uint8_t *inside, int nthreads)
{
    return classify_impl(px, py, n_points, NULL, offsets, n_polys, vx, vy, point_poly, inside, nthreads, 2);
}

/*
 * Polygons of several rings (see poly_parity): polygon q owns rings
 * poly_rings[q] .. poly_rings[q+1]-1 and ring r the vertices
 * vx/vy[ring_offsets[r] .. ring_offsets[r+1]).  predicate 1 = constraint 1,
 * 2 = constraint 2.  The index arrays must be monotone CSR arrays.
 */
int pip_oracle_classify_rings(const double *px, const double *py, int64_t n_points,
                              const int64_t *poly_rings, int64_t n_polys,
                              const int64_t *ring_offsets, int64_t n_rings,
                              const double *vx, const double *vy,
                              const int32_t *point_poly, uint8_t *inside, int nthreads, int predicate)
{
    if (!poly_rings || n_rings < 0 || (predicate != 1 && predicate != 2))
        return -1;
    if (n_polys >= 1 && (poly_rings[0] < 0 || poly_rings[n_polys] > n_rings))
        return -1;
    return classify_impl(px, py, n_points, poly_rings, ring_offsets, n_polys, vx, vy, point_poly, inside,
                         nthreads, predicate);
}

/*
 * Candidate pairs by bounding box (the paper's data preparation kept only the
 * points inside the polygon's bounding box, Simulation section; here for many
 * polygons at once): pair (i, q) is a candidate when point i lies in the
 * closed axis-aligned box [min x, max x] x [min y, max y] of polygon q's
 * vertices (all its rings).  A polygon without vertices has no candidates.
 * Comparisons only, so the result is exact.  Brute force over all points for
 * every polygon; pairs are listed by polygon, then by point index.
 */
typedef struct {
    const double *px, *py;
    int64_t n_points;
    const int64_t *poly_rings, *offsets;
    const double *vx, *vy;
    int64_t q0, q1;
    int64_t *counts;          /* [n_polys] */
    const int64_t *starts;    /* [n_polys] or NULL (count pass) */
    int64_t *pair_point;
} join_job;

static int poly_bbox(const join_job *j, int64_t q, double *x0, double *x1, double *y0, double *y1)
{
    int64_t r0 = j->poly_rings ? j->poly_rings[q] : q;
    int64_t r1 = j->poly_rings ? j->poly_rings[q + 1] : q + 1;
    int64_t b = j->offsets[r0], e = j->offsets[r1];
    if (e <= b)
        return 0;
    *x0 = *x1 = j->vx[b];
    *y0 = *y1 = j->vy[b];
    for (int64_t v = b + 1; v < e; ++v) {
        if (j->vx[v] < *x0) *x0 = j->vx[v];
        if (j->vx[v] > *x1) *x1 = j->vx[v];
        if (j->vy[v] < *y0) *y0 = j->vy[v];
        if (j->vy[v] > *y1) *y1 = j->vy[v];
    }
    return 1;
}

static void *join_worker(void *arg)
{
    join_job *j = (join_job *)arg;
    for (int64_t q = j->q0; q < j->q1; ++q) {
        double x0, x1, y0, y1;
        int64_t c = 0;
        if (poly_bbox(j, q, &x0, &x1, &y0, &y1)) {
            for (int64_t i = 0; i < j->n_points; ++i) {
                double x = j->px[i], y = j->py[i];
#if PIP_ORACLE_MUTANT == 9
                int in = x0 <= x && x < x1 && y0 <= y && y <= y1;   /* mutant: half-open in x */
#else
                int in = x0 <= x && x <= x1 && y0 <= y && y <= y1;
#endif
                if (in) {
                    if (j->starts)
                        j->pair_point[j->starts[q] + c] = i;
                    ++c;
                }
            }
        }
        j->counts[q] = c;
    }
    return NULL;
}

static void join_run(join_job *proto, int64_t n_polys, int nthreads)
{
    if (nthreads < 1)
        nthreads = 1;
    if (nthreads > 256)
        nthreads = 256;
    join_job jobs[256];
    pthread_t tids[256];
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = *proto;
        jobs[t].q0 = n_polys * t / nthreads;
        jobs[t].q1 = n_polys * (t + 1) / nthreads;
    }
    int started = 0;
    for (int t = 1; t < nthreads; ++t) {
        if (pthread_create(&tids[t], NULL, join_worker, &jobs[t]) != 0)
            break;
        started = t;
    }
    join_worker(&jobs[0]);
    for (int t = 1; t <= started; ++t)
        pthread_join(tids[t], NULL);
    for (int t = started + 1; t < nthreads; ++t)
        join_worker(&jobs[t]);
}

/*
 * counts[q] = number of candidate points of polygon q.  If pair_point is not
 * NULL (capacity = sum of counts), also lists them: polygon 0's points in
 * ascending index order, then polygon 1's, ...  poly_rings may be NULL (one
 * ring per polygon; offsets then has n_polys + 1 entries).  Returns 0, or -1
 * on bad arguments.
 */
int pip_oracle_bbox_join(const double *px, const double *py, int64_t n_points,
                         const int64_t *poly_rings, int64_t n_polys, const int64_t *offsets,
                         const double *vx, const double *vy, int64_t *counts, int64_t *pair_point,
                         int nthreads)
{
    if (n_points < 0 || n_polys < 0 || !offsets || !counts || (n_points > 0 && (!px || !py)))
        return -1;
    join_job proto;
    proto.px = px; proto.py = py; proto.n_points = n_points;
    proto.poly_rings = poly_rings; proto.offsets = offsets;
    proto.vx = vx; proto.vy = vy;
    proto.counts = counts;
    proto.starts = NULL;
    proto.pair_point = NULL;
    join_run(&proto, n_polys, nthreads);
    if (!pair_point)
        return 0;
    int64_t *starts = (int64_t *)malloc((size_t)(n_polys > 0 ? n_polys : 1) * sizeof(int64_t));
    if (!starts)
        return -1;
    int64_t s = 0;
    for (int64_t q = 0; q < n_polys; ++q) {
        starts[q] = s;
        s += counts[q];
    }
    proto.starts = starts;
    proto.pair_point = pair_point;
    join_run(&proto, n_polys, nthreads);
    free(starts);
    return 0;
}

/*
 * Indexed mode for one ring (the parity check of a huge ring against many
 * points, where the plain double loop would take hours): the same rule, with
 * the edges that cannot straddle a point's ray skipped through an exact y
 * index.  Edge (a, b) straddles the ray at p_y exactly when
 * min(a_y, b_y) <= p_y < max(a_y, b_y).  Points and edges are placed in
 * buckets by bucket(y) = floor((y - y_lo) * scale), clamped to [0, nb - 1]:
 * a non-decreasing function of y (every rounded operation in it is monotone),
 * so an edge listed in every bucket from bucket(min) to bucket(max) is listed
 * in the bucket of each point whose ray it straddles.  A point applies the
 * full rule (edge_counts) to the edges of its bucket; the edges it skips are
 * ones that contribute nothing, and the count's parity does not depend on the
 * order, so the result equals pip_oracle_classify's bit for bit.
 */
typedef struct {
    const double *px, *py;
    const double *vx, *vy;
    int64_t k;
    const int64_t *start, *list;
    double ylo, scale;
    int64_t nb;
    uint8_t *out;
    int64_t i0, i1;
} index_job;

static int64_t bucket_of(double y, double ylo, double scale, int64_t nb)
{
    double t = (y - ylo) * scale;
    if (!(t > 0))
        return 0;
    if (t >= (double)nb)
        return nb - 1;
    return (int64_t)t;
}

static void *index_worker(void *arg)
{
    const index_job *j = (const index_job *)arg;
    for (int64_t i = j->i0; i < j->i1; ++i) {
        double x = j->px[i], y = j->py[i];
        int64_t b = bucket_of(y, j->ylo, j->scale, j->nb);
        int64_t count = 0;
        for (int64_t t = j->start[b]; t < j->start[b + 1]; ++t) {
            int64_t e = j->list[t];
            int64_t f = (e + 1 == j->k) ? 0 : e + 1;
            count += edge_counts(x, y, j->vx[e], j->vy[e], j->vx[f], j->vy[f]);
        }
        j->out[i] = (uint8_t)(count & 1);
    }
    return NULL;
}

/* Edges listed per bucket for nb buckets; total entries, or -1 when over cap. */
static int64_t index_entries(const double *vy, int64_t k, double ylo, double scale, int64_t nb, int64_t cap)
{
    int64_t total = 0;
    for (int64_t e = 0; e < k; ++e) {
        int64_t f = (e + 1 == k) ? 0 : e + 1;
        double lo = vy[e] < vy[f] ? vy[e] : vy[f], hi = vy[e] < vy[f] ? vy[f] : vy[e];
        if (!(lo < hi))
            continue;   /* horizontal: never straddles */
        total += bucket_of(hi, ylo, scale, nb) - bucket_of(lo, ylo, scale, nb) + 1;
        if (total > cap)
            return -1;
    }
    return total;
}

int pip_oracle_classify_indexed(const double *px, const double *py, int64_t n_points, const int64_t *offsets,
                                int64_t n_polys, const double *vx, const double *vy, uint8_t *out, int nthreads)
{
    if (n_points < 0 || n_polys != 1 || !offsets || (n_points > 0 && (!px || !py || !out)))
        return -1;
    int64_t b0 = offsets[0], k = offsets[1] - offsets[0];
    if (k < 0 || b0 < 0)
        return -1;
    const double *rx = vx + b0, *ry = vy + b0;
    double ylo = 0.0, yhi = 0.0;
    for (int64_t e = 0; e < k; ++e) {
        if (e == 0 || ry[e] < ylo)
            ylo = ry[e];
        if (e == 0 || ry[e] > yhi)
            yhi = ry[e];
    }
    int64_t nb = k < (1 << 20) ? (k > 0 ? k : 1) : (1 << 20);
    double scale = 0.0;
    int64_t total = -1;
    for (;;) {
        scale = yhi > ylo ? (double)nb / (yhi - ylo) : 0.0;
        if (!(scale < 1e300))
            scale = 0.0;   /* a degenerate y range: one bucket in effect */
        total = index_entries(ry, k, ylo, scale, nb, 16 * k + nb);
        if (total >= 0 || nb == 1)
            break;
        nb /= 2;
    }
    if (total < 0)
        total = index_entries(ry, k, ylo, scale, nb, INT64_MAX);
    int64_t *start = (int64_t *)calloc((size_t)nb + 1, sizeof(int64_t));
    int64_t *list = (int64_t *)malloc((size_t)(total > 0 ? total : 1) * sizeof(int64_t));
    if (!start || !list) {
        free(start);
        free(list);
        return -2;
    }
    for (int64_t e = 0; e < k; ++e) {
        int64_t f = (e + 1 == k) ? 0 : e + 1;
        double lo = ry[e] < ry[f] ? ry[e] : ry[f], hi = ry[e] < ry[f] ? ry[f] : ry[e];
        if (!(lo < hi))
            continue;
        for (int64_t b = bucket_of(lo, ylo, scale, nb); b <= bucket_of(hi, ylo, scale, nb); ++b)
            start[b + 1]++;
    }
    for (int64_t b = 0; b < nb; ++b)
        start[b + 1] += start[b];
    int64_t *fill = (int64_t *)malloc((size_t)nb * sizeof(int64_t));
    if (!fill) {
        free(start);
        free(list);
        return -2;
    }
    for (int64_t b = 0; b < nb; ++b)
        fill[b] = start[b];
    for (int64_t e = 0; e < k; ++e) {
        int64_t f = (e + 1 == k) ? 0 : e + 1;
        double lo = ry[e] < ry[f] ? ry[e] : ry[f], hi = ry[e] < ry[f] ? ry[f] : ry[e];
        if (!(lo < hi))
            continue;
        for (int64_t b = bucket_of(lo, ylo, scale, nb); b <= bucket_of(hi, ylo, scale, nb); ++b)
            list[fill[b]++] = e;
    }
    free(fill);

    if (nthreads < 1)
        nthreads = 1;
    if (nthreads > 256)
        nthreads = 256;
    index_job jobs[256];
    pthread_t th[256];
    int started[256] = {0};
    int64_t chunk = (n_points + nthreads - 1) / nthreads;
    for (int t = 0; t < nthreads; ++t) {
        index_job *j = &jobs[t];
        j->px = px;
        j->py = py;
        j->vx = rx;
        j->vy = ry;
        j->k = k;
        j->start = start;
        j->list = list;
        j->ylo = ylo;
        j->scale = scale;
        j->nb = nb;
        j->out = out;
        j->i0 = (int64_t)t * chunk < n_points ? (int64_t)t * chunk : n_points;
        j->i1 = j->i0 + chunk < n_points ? j->i0 + chunk : n_points;
        if (t > 0 && j->i0 < j->i1)
            started[t] = pthread_create(&th[t], NULL, index_worker, j) == 0;
        if (t > 0 && j->i0 < j->i1 && !started[t])
            index_worker(j);
    }
    index_worker(&jobs[0]);
    for (int t = 1; t < nthreads; ++t)
        if (started[t])
            pthread_join(th[t], NULL);
    free(start);
    free(list);
    return 0;
}
