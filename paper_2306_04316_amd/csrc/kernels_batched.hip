// Batched classification of pairs sorted by polygon, one workgroup per work
// item of 256*U consecutive pairs, in both arithmetic modes (paper, Method
// section, constraint 1, and Algorithm 1, with the half-open straddle
// reading).
//
// The item's vertex range (the rings of its pairs' polygons, back to back) is
// walked in LDS tiles of S vertices.  Per tile the workgroup stages the
// vertices (coalesced binary64 loads) and builds one record per edge, indexed
// by the edge's end vertex; then every lane walks the part of its own ring
// that lies in the tile, for each of its U pairs:
//   1. straddle pass, exact in both modes: above_j = (y_j > p_y), the sign
//      bit of the binary64 difference p_y - y_j, shifted into a 32-bit word
//      per 32 vertices (two vector instructions per vertex); straddle bits =
//      above XOR above shifted by one;
//   2. side values for the lane's straddling edges only.
// Exact mode: records (a_x, a_y, n_x, n_y) in binary64 with the rule's
// oriented normal; s = (p_x - a_x) n_x + (p_y - a_y) n_y, every operation
// rounded separately; the edge counts when s <= 0 (the oracle's bits).
// Filtered mode: binary32 records on coordinates re-centred on the ring's
// first vertex c (binary64).  With n the rule's binary64 normal after
// orientation and 2^e the power of two with 1 <= (n_x + |n_y|) 2^-e < 2, the
// scaled normal N = n 2^-e is exact in binary64; the record holds
//   NX = fl32(N_x), NY = fl32(N_y), -C with C = fl32(fl64(fl64(d_x N_x) +
//   fl64(d_y N_y))), d = fl64(a - c)
// (the line through the anchor a, offset C), so |NX| + |NY| <= N1 =
// 2 + 2^-20.  For a pair P = fl32(fl64(p - c)) the side value is two fused
// multiply-adds, each rounded once:
//   S = fma(P_x, NX, fma(P_y, NY, -C)).
// Every straddling edge has n_x > 0.  E = t1 n_x + t2 n_y, the exact value
// on the binary64 inputs and normal, satisfies E 2^-e = (p - c).N - (a - c).N.
// With M at least |a - c| and the pair's |P_x|, |P_y| (u = 2^-24, w = 2^-53):
// the point's conversions err by at most u (1 + 2^-28) |P|, the normal's by
// u |N|, C by u M |N|_1 (1 + 2^-28) (its binary64 part by 3 w M |N|_1), the
// inner and outer roundings by u (|P_y NY| + |C|) and u (|P_x NX| + |inner|);
// altogether |S - E 2^-e| <= 7.01 u M |N|_1 plus at most eta (2 N1 + 3) from
// binary32 subnormals flushed to zero (eta = 2^-126).  If |S| > B >=
// 8 u M N1 + 4 eta (N1 + 1) -- one threshold per pair, B = fma(M, k_B, e_B)
// with both coefficients rounded up by 2^-20 on the host so that its one
// rounding cannot take it below that -- then |E| 2^-e > 0.98 u M |N|_1, while the
// rule's binary64 value differs from E by at most 6.02 w M |n|_1: that value
// is nonzero and has the sign of S, so the edge counts exactly when S < 0
// (the sign bit of S).  M is taken per pair as max(M_ring rounded up, |P_x|,
// |P_y|), where M_ring bounds |a - c| over the anchors the pair has been tested
// against so far (an LDS maximum per ring, accumulated tile by tile).  The
// bound needs every nonzero normal component in [2^-60, 2^60] (the scaled
// components stay at or above 2^-121, normal in binary32) and |p - c|,
// |a - c| <= 2^60; outside that the pair is undecided.  A pair whose smallest
// |S| over its straddling edges is at most B joins the recheck list and is
// re-run in binary64 in the rule's order (k_recheck_lanes, k_recheck_wide).
//
// Items whose pairs are not sorted by polygon, or whose polygons outnumber
// the ring table, are classified exactly by the staged binary64 item
// (staged_exact.h) in the same LDS.
//
// This translation unit must be compiled with -ffp-contract=off.

#include "filter_bound.h"
#include "pip_common.h"
#include "ring_walk.h"
#include "staged_exact.h"

namespace pip {

namespace {

struct BatchedArgs {
    const double *px, *py;
    int64_t n;
    const int64_t *offsets;
    int64_t n_polys;
    const double *vx, *vy;
    int64_t nv;
    const int32_t *point_poly;
    uint8_t *inside;
    int tile;        // S: vertices per LDS tile
    int max_rings;   // ring table entries
    int fb_tile;     // tile of the staged binary64 item (fallback), fits the same LDS
    float bound_k;     // B = fma(M, bound_k, bound_eta): bound_k >= 8 u N1, bound_eta >= 4 eta (N1 + 1)
    float bound_eta;   // (both times the testing scale; rounded up on the host)
    int force_recheck;
    int32_t *recheck;
    unsigned *recheck_count;
    unsigned long long *stats;   // [256][2]: point-edge tests, undecided side tests (stats kernels)
    const ItemDesc *desc;        // per workgroup, in launch order
    int wave_k;                  // rings of at least wave_k vertices go to the wave kernel (W variants)
    WaveTask *tasks;
    unsigned *task_count;
    unsigned max_tasks;
};

struct BatchedLds {
    int *T;         // ring starts relative to the range start, nr + 1 entries
    double2 *RC;    // filtered: ring centre (the ring's first vertex)
    unsigned *RM;   // filtered: M_ring as binary32 bits (or kRingBad)
    double *XD;     // the tile's x values
    double *YD;     // the tile's y values, 64 padding slots after the tile
    void *REC;      // per edge (indexed by its end vertex): float4 filtered, double4 exact
    int *RF;        // per ring: the item's stamp when a pair of the item has it; minus the stamp once
                    // it is left to the wave kernel
};

}  // namespace

// LDS bytes of the batched item's layout, and its parts' offsets.
__host__ __device__ inline size_t batched_layout(int S, int max_rings, bool F, size_t *o)
{
    size_t x = 0;
    size_t at[7];
    const size_t sizes[7] = {(size_t)(max_rings + 1) * 4,
                             F ? (size_t)max_rings * 16 : 0,
                             F ? (size_t)max_rings * 4 : 0,
                             (size_t)S * 8,
                             ((size_t)S + 64) * 8,
                             (size_t)S * (F ? 16 : 32),
                             F ? (size_t)max_rings * 4 : 0};
    for (int i = 0; i < 7; ++i) {
        at[i] = x;
        x = (x + sizes[i] + 15) & ~(size_t)15;
    }
    if (o)
        for (int i = 0; i < 7; ++i)
            o[i] = at[i];
    return x;
}

size_t batched_smem_bytes(int tile, int max_rings, bool filtered)
{
    return batched_layout(tile, max_rings, filtered, nullptr);
}

namespace {

template <bool F>
__device__ __forceinline__ BatchedLds batched_lds(unsigned char *smem, int S, int max_rings)
{
    size_t o[7];
    batched_layout(S, max_rings, F, o);
    BatchedLds L;
    L.T = (int *)(smem + o[0]);
    L.RC = (double2 *)(smem + o[1]);
    L.RM = (unsigned *)(smem + o[2]);
    L.XD = (double *)(smem + o[3]);
    L.YD = (double *)(smem + o[4]);
    L.REC = (void *)(smem + o[5]);
    L.RF = (int *)(smem + o[6]);
    return L;
}

// A load from LDS through a pointer into the dynamic LDS block, typed for the
// LDS address space so that it cannot become a generic load.
template <typename T>
__device__ __forceinline__ T lds_load(const T *p)
{
    return *(const __attribute__((address_space(3))) T *)p;
}

// Parity contribution of one lane's ring part: edges ending at staged
// vertices base .. base+k-1 of the tile (k = 0: nothing).  prev: the above
// bit of the vertex before the part in the ring; with own set (the whole ring
// in the tile, k <= 32) it is taken from the straddle pass itself.  Exact
// mode: par counts crossings; filtered mode: bit 31 of par is the parity of
// the negative side values, und is set by an undecided side test.  Must be
// called by the whole wavefront.
template <bool F, bool STATS>
__device__ __forceinline__ void walk_part(const BatchedLds &L, int base, int k, uint32_t prev, bool own, double xu,
                                          double yu, float PX, float PY, float bnd, int S, uint32_t &par, bool &und,
                                          uint32_t &n_und)
{
    const double yq = yu + 0.0;   // no negative zero (see shift_in_above)
    // smallest |S| over the part's side tests (filtered), as binary32 bits:
    // non-negative floats order as their bit patterns, so an integer minimum
    // needs no NaN quieting of the running value (a NaN S, never produced for
    // an eligible pair, would read as larger than any finite value)
    uint32_t amin = 0x7f800000u;
    const int y_alloc = S + 64;
    for (int c0 = 0; c0 < S; c0 += 32) {
        if (__builtin_amdgcn_ballot_w64(k > c0) == 0)
            break;
        uint32_t above = 0;   // vertex c0 + j of the part at bit 31 - j
        // lanes past their part read clamped slots (bits masked below); a lane
        // inside its part starts at most at the tile's last vertex, S - 1 <
        // y_alloc - 32, and is never clamped
        const int ybase = base + c0;
        const double *yr = L.YD + (ybase < y_alloc - 32 ? ybase : y_alloc - 32);
        int t = 0;
        for (; t < 32; t += 4) {
            if (__builtin_amdgcn_ballot_w64(k > c0 + t) == 0)
                break;
#pragma unroll
            for (int tt = 0; tt < 4; ++tt)
                above = shift_in_above(above, yq, yr[t + tt]);
        }
        above = t < 32 ? above << (32 - t) : above;
        if (c0 == 0 && own)
            prev = (above >> ((32 - k) & 31)) & 1u;
        uint32_t strad = above ^ ((above >> 1) | (prev << 31));
        const int rem = k - c0;
        const int rc = rem < 0 ? 0 : (rem > 32 ? 32 : rem);
        strad &= (uint32_t)(0xffffffff00000000ull >> rc);
        prev = rem >= 32 ? (above & 1u) : prev;
        // bit j: the edge ending at part vertex c0 + j
        strad = __builtin_bitreverse32(strad);
        if (F) {
            const float4 *er = (const float4 *)L.REC + (base + c0);
            while (strad != 0) {
                const int b = __builtin_ctz(strad);
                strad &= strad - 1u;
                const float4 rec = er[b];
                const float sv = __builtin_fmaf(PX, rec.x, __builtin_fmaf(PY, rec.y, rec.z));
                // finite for every eligible pair (non-finite inputs make the
                // ring or the point ineligible)
                amin = min(amin, __float_as_uint(sv) & 0x7fffffffu);
                if (STATS)
                    n_und += fabsf(sv) > bnd ? 0u : 1u;
                par ^= __float_as_uint(sv);
            }
        } else {
            const double4 *er = (const double4 *)L.REC + (base + c0);
            while (strad != 0) {
                const int b = __builtin_ctz(strad);
                strad &= strad - 1u;
                const double4 rec = er[b];
                const double t1 = xu - rec.x;
                const double t2 = yu - rec.y;
                const double sv = t1 * rec.z + t2 * rec.w;
                par += sv <= 0.0 ? 1u : 0u;
            }
        }
    }
    if (F)
        und = und || !(__uint_as_float(amin) > bnd);
}

template <bool F, int U, bool STATS, bool W>
__device__ __forceinline__ void batched_item(int64_t p0, const ItemRows<U> &P, const ItemRange &R,
                                             const BatchedArgs &A, unsigned char *smem)
{
    const int tid = threadIdx.x;
    const int S = A.tile;
    const int qf = R.qf, ql = R.ql, nr = R.nr, nvr = R.nv;
    const int64_t vb = R.vb;
    const bool tables = R.ok && nr <= A.max_rings;
    const BatchedLds L = batched_lds<F>(smem, S, A.max_rings);
    __shared__ int s_all[4];
    __shared__ unsigned s_rcnt, s_rbase;
    // tiles the item's own walks need (bit per tile of S vertices), when large
    // rings go to the wave kernel; items of more tiles than bits walk them all
    constexpr int kNeedWords = 64;
    __shared__ unsigned s_need[kNeedWords];
    __shared__ unsigned s_stat[2];

    // First round of the ring table and of the first tile: one entry of each
    // per thread, their loads issued together (one memory round trip).
    const int tn0 = nvr < S ? nvr : S;
    {
        const bool hr = tables && tid <= nr;
        const bool hv = tables && tid < tn0;
        int64_t o = 0;
        double ax = 0.0, ay = 0.0;
        if (hr)
            o = A.offsets[R.rf + tid];
        if (hv) {
            ax = A.vx[vb + tid];
            ay = A.vy[vb + tid];
        }
        if (hr) {
            o = o < vb ? vb : (o > vb + nvr ? vb + nvr : o);
            L.T[tid] = (int)(o - vb);
        }
        if (hv) {
            L.XD[tid] = ax;
            L.YD[tid] = ay;
        }
    }
    if (tables) {
        for (int r = tid + 256; r <= nr; r += 256) {
            int64_t o = A.offsets[R.rf + r];
            o = o < vb ? vb : (o > vb + nvr ? vb + nvr : o);
            L.T[r] = (int)(o - vb);
        }
        for (int e = tid + 256; e < tn0; e += 256) {
            L.XD[e] = A.vx[vb + e];
            L.YD[e] = A.vy[vb + e];
        }
        if (F)
            for (int r = tid; r < nr; r += 256)
                L.RM[r] = 0u;
        if (W && tid < kNeedWords)
            s_need[tid] = 0u;
    }
    if (tid == 0) {
        s_rcnt = 0;
        s_stat[0] = 0;
        s_stat[1] = 0;
    }
    bool mine_ok = true;
#pragma unroll
    for (int u = 0; u < U; ++u)
        mine_ok = mine_ok && (P.q[u] < 0 || (P.q[u] >= qf && P.q[u] <= ql));
    // the rings this item's pairs use, marked with a stamp unique to the
    // workgroup (no clearing needed)
    const int stamp = (int)blockIdx.x + 1;
    const bool wave = W && tables;   // W: filtered, with the wave kernel after this one
    if (wave) {
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (P.q[u] >= qf && P.q[u] <= ql)
                L.RF[P.q[u] - qf] = stamp;
    }
    const bool staged = block_all(tables && mine_ok, s_all);

    if (!staged) {
        // pairs not sorted by polygon, or more polygons than the table holds:
        // the staged binary64 item (exact, no recheck needed)
        if (STATS) {
            uint32_t nt = 0;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (P.q[u] >= 0 && (uint64_t)P.q[u] < (uint64_t)A.n_polys) {
                    int64_t b = A.offsets[P.q[u]], e = A.offsets[P.q[u] + 1];
                    clamp_ring(b, e, A.nv);
                    nt += (uint32_t)(e - b);
                }
            }
            atomicAdd(&A.stats[(blockIdx.x & 255) * 2], (unsigned long long)nt);
        }
        staged_item_fp64<kSide, U, false, true>(p0, P, A.n, A.offsets, A.n_polys, nullptr, A.n_polys, A.vx, A.vy,
                                                A.nv, A.inside, A.fb_tile, A.max_rings, smem, R);
        return;
    }

    // Large rings with pairs here go to the wave kernel, one task each; a
    // ring whose task does not fit the list is walked here as any other.
    if (wave && tid < nr) {
        int v = 0;
        const bool has = L.RF[tid] == stamp;
        if (L.T[tid + 1] - L.T[tid] >= A.wave_k && has) {
            const unsigned at = atomicAdd(A.task_count, 1u);
            if (at < A.max_tasks) {
                WaveTask t;
                t.p_lo = p0;
                t.ring = qf + tid;
                t.count = (int)(A.n - p0 < 256 * U ? A.n - p0 : 256 * U);
                A.tasks[at] = t;
                v = -stamp;
            }
        }
        L.RF[tid] = v;   // read by the rows after the next barrier
        // a ring with pairs walked here needs the tiles it spans
        if (L.RF[tid] != -stamp && has && L.T[tid + 1] > L.T[tid]) {
            const int f = L.T[tid] / S, l = (L.T[tid + 1] - 1) / S;
            for (int t = f; t <= l && t < 32 * kNeedWords; ++t)
                atomicOr(&s_need[t >> 5], 1u << (t & 31));
        }
    }
    const bool skip_tiles = wave && (nvr + S - 1) / S <= 32 * kNeedWords;

    uint32_t par[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
        par[u] = 0;
    uint32_t und = 0;   // bit u: row u has an undecided test (filtered)
    uint32_t n_tests = 0, n_und = 0;

    for (int t0 = 0; t0 < nvr; t0 += S) {
        const int t1 = nvr - t0 < S ? nvr : t0 + S;
        const int tn = t1 - t0;
        // a later tile that only rings of the wave kernel (or rings without
        // pairs here) cover is neither staged nor walked (uniform: LDS word)
        if (t0 > 0 && skip_tiles && !((s_need[(t0 / S) >> 5] >> ((t0 / S) & 31)) & 1u))
            continue;
        if (t0 > 0) {
            for (int e = tid; e < tn; e += 256) {
                L.XD[e] = A.vx[vb + t0 + e];
                L.YD[e] = A.vy[vb + t0 + e];
            }
            __syncthreads();
        }
        if (tid < 64)
            L.YD[tn + tid] = 0.0;
        // Records of the edges ending in the tile.  A vertex's predecessor is
        // the previous vertex, or the ring's last vertex for the ring's first;
        // outside the tile it is read from global memory.
        for (int e = t0 + tid; e < t1; e += 256) {
            const int r = staged_ring_of(L.T, nr, e);
            if (r < 0)
                continue;   // offsets not monotone: unspecified results
            const int e0 = L.T[r], e1 = L.T[r + 1];
            const int ep = e == e0 ? e1 - 1 : e - 1;
            const double bx = L.XD[e - t0], by = L.YD[e - t0];
            // the predecessor from LDS, or (outside the tile) from global
            // memory: two loads of fixed address spaces, not one load through
            // a selected generic pointer
            const bool pin = ep >= t0 && ep < t1;
            const int epl = pin ? ep - t0 : 0;
            double ax = lds_load(L.XD + epl), ay = lds_load(L.YD + epl);
            if (!pin) {
                ax = A.vx[vb + ep];
                ay = A.vy[vb + ep];
            }
            if (F) {
                double cx, cy;
                if (e0 >= t0) {
                    cx = L.XD[e0 - t0];
                    cy = L.YD[e0 - t0];
                } else {
                    const double2 c = L.RC[r];   // stored in an earlier tile
                    cx = c.x;
                    cy = c.y;
                }
                if (e == e0)
                    L.RC[r] = make_double2(cx, cy);
                unsigned mb;
                ((float4 *)L.REC)[e - t0] = filtered_record(ax, ay, bx, by, cx, cy, &mb);
                atomicMax(&L.RM[r], mb);
            } else {
                ((double4 *)L.REC)[e - t0] = edge_record<kSide>(ax, ay, bx, by);
            }
        }
        __syncthreads();

#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int r = (P.q[u] < 0 ? qf : P.q[u]) - qf;
            const int e0 = L.T[r], e1 = L.T[r + 1];
            const int a = e0 > t0 ? e0 : t0;
            const int b = e1 < t1 ? e1 : t1;
            const bool dfr = wave && P.q[u] >= 0 && L.RF[r] == -stamp;   // left to the wave kernel
            const int k = (P.q[u] >= 0 && b > a && !dfr) ? b - a : 0;
            const bool own = a == e0 && b == e1 && k <= 32;
            uint32_t prev = 0;
            if (k > 0 && !own) {
                const int pr = a == e0 ? e1 - 1 : a - 1;
                const bool pin = pr >= t0 && pr < t1;
                double yp = lds_load(L.YD + (pin ? pr - t0 : 0));
                if (!pin)
                    yp = A.vy[vb + pr];
                prev = yp > P.y[u] ? 1u : 0u;
            }
            float PX = 0.0f, PY = 0.0f, bnd = 0.0f;
            bool u_und = false;
            if (F && k > 0) {
                const double2 c = L.RC[r];
                PX = (float)(P.x[u] - c.x);
                PY = (float)(P.y[u] - c.y);
                const unsigned mr = L.RM[r];
                // M = max(M_ring, |P_x|, |P_y|); |P| < 2^60 in binary32 implies
                // |p - c| < 2^60 (rounding is monotone), and M_ring <= 2^60
                const float mp = fmaxf(__uint_as_float(mr), fmaxf(fabsf(PX), fabsf(PY)));
                bnd = __builtin_fmaf(mp, A.bound_k, A.bound_eta);
                u_und = mr == kRingBad || !(mp < kLimF);
            }
            walk_part<F, STATS>(L, a - t0, k, prev, own, P.x[u], P.y[u], PX, PY, bnd, S, par[u], u_und, n_und);
            und |= (u_und ? 1u : 0u) << u;
            if (STATS)
                n_tests += (uint32_t)k;
        }
        if (t1 < nvr)
            __syncthreads();   // the next tile overwrites XD, YD and the records
    }

    uint64_t und_rows[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t i = p0 + u * 256 + tid;
        const bool dfr = wave && P.q[u] >= 0 && L.RF[P.q[u] - qf] == -stamp;
        const bool valid = i < A.n && !dfr;
        const bool un = F && (((und >> u) & 1u) || A.force_recheck);
        und_rows[u] = __builtin_amdgcn_ballot_w64(valid && un);
        if (valid && !un)
            A.inside[i] = (uint8_t)(F ? (par[u] >> 31) : (par[u] & 1u));
    }
    if (STATS) {
        if (n_tests)
            atomicAdd(&s_stat[0], n_tests);
        if (n_und)
            atomicAdd(&s_stat[1], n_und);
    }
    if (F)
        append_recheck_item<U>(und_rows, p0, A.recheck, A.recheck_count, &s_rcnt, &s_rbase);
    else if (STATS)
        __syncthreads();
    if (STATS && tid == 0) {
        unsigned long long *st = A.stats + (blockIdx.x & 255) * 2;
        atomicAdd(st, (unsigned long long)s_stat[0]);
        atomicAdd(st + 1, (unsigned long long)s_stat[1]);
    }
}

// One workgroup per item: workgroup b takes descriptor b (the preparation's
// item order).  Eight waves per SIMD for one and two pairs per lane; four
// pairs per lane need more registers than that leaves (they would spill).
template <bool F, int U, bool STATS, bool W>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(U == 4 ? 5 : 8))) void k_batched(BatchedArgs A)
{
    extern __shared__ __align__(16) unsigned char smem[];
    // one scalar load gives the item and its range; the pairs, the ring
    // table and the first tile then load together
    const ItemDesc d = A.desc[blockIdx.x];
    const int64_t p0 = (int64_t)d.item * (256 * U);
    const ItemRows<U> P = load_rows<U>(p0, A.px, A.py, A.n, A.point_poly);
    ItemRange R;
    R.vb = d.vb;
    R.rf = d.qf;
    R.qf = d.qf;
    R.ql = d.ql;
    R.ok = d.nv >= 0;
    R.nr = d.nv >= 0 ? d.ql - d.qf + 1 : 0;
    R.nv = d.nv >= 0 ? d.nv : 0;
    batched_item<F, U, STATS, W>(p0, P, R, A, smem);
}

template <bool F, int U, bool STATS, bool W>
void launch_batched_one(const BatchedArgs &A, int grid, size_t shmem, hipStream_t stream)
{
    PIP_LAUNCH((k_batched<F, U, STATS, W>), dim3(grid), dim3(256), shmem, stream, A);
}

template <bool F, bool STATS, bool W>
void launch_batched_u(const BatchedArgs &A, int U, int grid, size_t shmem, hipStream_t stream)
{
    if (U == 1)
        launch_batched_one<F, 1, STATS, W>(A, grid, shmem, stream);
    else if (U == 2)
        launch_batched_one<F, 2, STATS, W>(A, grid, shmem, stream);
    else
        launch_batched_one<F, 4, STATS, W>(A, grid, shmem, stream);
}

}  // namespace

int launch_batched(const Problem &p, hipStream_t stream, bool filtered, int pairs_per_lane, int tile,
                   float bound_scale, int force_recheck, int32_t *recheck, unsigned *recheck_count,
                   unsigned long long *stats, const ItemDesc *desc, int n_items, const WaveOut &wave)
{
    if (p.poly_rings)
        return fail(PIP_ENOTSUP, "the batched kernel takes one ring per polygon");
    if (p.pred != kSide)
        return fail(PIP_ENOTSUP, "the batched kernel implements the side test (constraint 1)");
    const int U = pairs_per_lane == 1 ? 1 : (pairs_per_lane == 2 ? 2 : 4);
    const int max_rings = staged_max_rings(U);
    tile = tile < 32 ? 32 : tile;
    const size_t shmem = batched_smem_bytes(tile, max_rings, filtered);
    int fb = tile;
    while (fb > 16 && staged_smem_bytes(fb, max_rings) > shmem)
        fb -= 16;
    if (staged_smem_bytes(fb, max_rings) > shmem)
        return fail(PIP_EINVAL, "LDS tile of %d vertices too small for the batched kernel", tile);
    if (filtered && (!recheck || !recheck_count))
        return fail(PIP_EINVAL, "the filtered mode needs a recheck list");
    if (n_items <= 0)
        return PIP_OK;
    if (!desc)
        return fail(PIP_EINVAL, "the batched kernel needs the item descriptors");
    // the threshold's two coefficients, rounded up so that the one rounding of
    // fma(M, k, eta) keeps B at or above 8 u M N1 + 4 eta (N1 + 1)
    const double n1 = 2.0 + 0x1p-20;
    const double kb = 8.0 * 0x1p-24 * n1 * (double)bound_scale * (1.0 + 0x1p-20);
    const double eb = 4.0 * 0x1p-126 * (n1 + 1.0) * (double)bound_scale * (1.0 + 0x1p-20);
    BatchedArgs A{p.px, p.py, p.n_points, p.offsets, p.n_polys, p.vx, p.vy, p.n_vertices, p.point_poly, p.inside,
                  tile, max_rings, fb, (float)kb, (float)eb, force_recheck, recheck, recheck_count, stats, desc,
                  0, nullptr, nullptr, 0};
    if (filtered) {
        const bool w = wave.wave_k > 0 && wave.tasks && wave.task_count && wave.cursor && wave.grid > 0;
        if (w) {
            A.wave_k = wave.wave_k < 64 ? 64 : wave.wave_k;
            A.tasks = wave.tasks;
            A.task_count = wave.task_count;
            A.max_tasks = wave.max_tasks;
        }
        // with the wave kernel after it, the main-kernel timestamps span both
        KernelTimer &kt = kernel_timer();
        const KernelTimer saved = kt;
        if (w)
            kt.stop = nullptr;
        if (w) {
            if (stats)
                launch_batched_u<true, true, true>(A, U, n_items, shmem, stream);
            else
                launch_batched_u<true, false, true>(A, U, n_items, shmem, stream);
        } else {
            if (stats)
                launch_batched_u<true, true, false>(A, U, n_items, shmem, stream);
            else
                launch_batched_u<true, false, false>(A, U, n_items, shmem, stream);
        }
        kt = saved;
        PIP_HIP_TRY(hipGetLastError());
        if (w) {
            kt.start = nullptr;
            const int rc = launch_wave_rings(p, stream, wave.tasks, wave.task_count, wave.max_tasks, wave.cursor,
                                             (float)kb, (float)eb, force_recheck, recheck, recheck_count, stats,
                                             wave.grid);
            kt = saved;
            return rc;
        }
    } else {
        if (stats)
            launch_batched_u<false, true, false>(A, U, n_items, shmem, stream);
        else
            launch_batched_u<false, false, false>(A, U, n_items, shmem, stream);
    }
    PIP_HIP_TRY(hipGetLastError());
    return PIP_OK;
}

}  // namespace pip
