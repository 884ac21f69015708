// Two-level counting sort of points (x, y, index) by an integer key in
// [0, NC * NF), without a global atomic per point and with coalesced writes.
// Pass 1 orders by the coarse digit key / NF: each workgroup counts a chunk of
// kSortChunk points in LDS, the (digit, chunk) count table is scanned, then
// the workgroup writes its chunk out in pieces of points sorted by
// digit in LDS, each digit's points leaving as one contiguous run (256*PER
// points a piece, PER a template parameter: the longer a digit's run in a
// piece, the fewer partial memory lines the scattered writes touch).  Pass 2:
// one workgroup per coarse digit orders its run by the fine digit key % NF
// the same way.  The order inside a key is not specified.  Used for the
// y-index's y buckets and the candidate join's grid cells.
#pragma once

#include "pip_common.h"

namespace pip {
namespace {

constexpr int kSortChunk = 16384;   // points per workgroup in pass 1

// In-place exclusive prefix of a[0..ND) (LDS), by a workgroup of 256 threads;
// returns the total.  Each thread sums its ND/256 entries, the wavefronts
// scan those sums with lane shuffles, and one exchange of the four wavefront
// totals through part (LDS, 4 words) completes it: two barriers in all.
template <int ND>
__device__ __forceinline__ uint32_t lds_exclusive_scan(uint32_t *a, uint32_t *part)
{
    constexpr int PER = ND / 256 > 0 ? ND / 256 : 1;
    const int t = threadIdx.x;
    const int lane = t & 63, w = t >> 6;
    uint32_t loc[PER], sum = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int d = t * PER + k;
        loc[k] = d < ND ? a[d] : 0u;
        sum += loc[k];
    }
    uint32_t incl = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t v = __shfl_up(incl, o, 64);
        incl += lane >= o ? v : 0u;
    }
    if (lane == 63)
        part[w] = incl;
    __syncthreads();
    uint32_t run = incl - sum, total = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t p = part[i];
        run += i < w ? p : 0u;
        total += p;
    }
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int d = t * PER + k;
        if (d < ND)
            a[d] = run;
        run += loc[k];
    }
    __syncthreads();
    return total;
}

// Digits of up to 256*PER points (PER per thread, digit -1 = no point) are
// counted, placed in digit order in LDS and written at cur[digit] onwards
// (cur advanced).  cnt, cur: LDS arrays of ND entries.
template <int ND, int PER>
__device__ __forceinline__ void write_piece_sorted(const double (&x)[PER], const double (&y)[PER],
                                                   const int32_t (&id)[PER], const int (&dg)[PER], uint32_t *cnt,
                                                   uint32_t *cur, uint32_t *part,
                                                   double2 *sxy, int32_t *sid, uint16_t *sdg,
                                                   double2 *__restrict__ oxy, int32_t *__restrict__ oid)
{
    const int t = threadIdx.x;
    for (int d = t; d < ND; d += 256)
        cnt[d] = 0;
    __syncthreads();
    uint32_t rk[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k)
        rk[k] = dg[k] >= 0 ? atomicAdd(&cnt[dg[k]], 1u) : 0u;
    __syncthreads();
    const uint32_t total = lds_exclusive_scan<ND>(cnt, part);   // cnt: each digit's first slot
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        if (dg[k] >= 0) {
            const uint32_t slot = cnt[dg[k]] + rk[k];
            sxy[slot] = make_double2(x[k], y[k]);
            sid[slot] = id[k];
            sdg[slot] = (uint16_t)dg[k];
        }
    }
    __syncthreads();
    for (uint32_t slot = t; slot < total; slot += 256) {
        const int d = sdg[slot];
        const uint32_t g = cur[d] + (slot - cnt[d]);
        oxy[g] = sxy[slot];
        oid[g] = sid[slot];
    }
    __syncthreads();
    for (int d = t; d < ND; d += 256) {
        const uint32_t end = d + 1 < ND ? cnt[d + 1] : total;
        cur[d] += end - cnt[d];
    }
    __syncthreads();
}

// Key::kUsesX: whether the key reads the x coordinate (its loads are skipped
// if not).
template <class Key, int NC, int NF>
__global__ __launch_bounds__(256) void k_sort_coarse_hist(const double *__restrict__ px,
                                                          const double *__restrict__ py, int64_t n, Key key, int nb,
                                                          uint32_t *__restrict__ table)
{
    __shared__ uint32_t h[NC];
    const auto kf = key.ready();
    for (int c = threadIdx.x; c < NC; c += 256)
        h[c] = 0;
    __syncthreads();
    const int64_t c0 = (int64_t)blockIdx.x * kSortChunk;
    const int64_t c1 = c0 + kSortChunk < n ? c0 + kSortChunk : n;
    // four points per thread per round, their loads issued together
    for (int64_t b = c0; b < c1; b += 1024) {
        double x[4], y[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int64_t i = b + k * 256 + threadIdx.x;
            x[k] = Key::kUsesX && i < c1 ? px[i] : 0.0;
            y[k] = i < c1 ? py[i] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (b + k * 256 + threadIdx.x < c1)
                atomicAdd(&h[kf(x[k], y[k]) / NF], 1u);
    }
    __syncthreads();
    for (int c = threadIdx.x; c < NC; c += 256)
        table[(int64_t)c * nb + blockIdx.x] = h[c];
}

template <class Key, int NC, int NF, int PER>
__global__ __launch_bounds__(256) void k_sort_coarse_scatter(const double *__restrict__ px,
                                                             const double *__restrict__ py, int64_t n, Key key,
                                                             int nb, const int64_t *__restrict__ off,
                                                             double2 *__restrict__ txy, int32_t *__restrict__ tidx)
{
    constexpr int PIECE = 256 * PER;
    __shared__ uint32_t cnt[NC], cur[NC];   // positions fit 32 bits (fewer than 2^31 points)
    __shared__ uint32_t part[4];
    __shared__ double2 sxy[PIECE];
    __shared__ int32_t sid[PIECE];
    __shared__ uint16_t sdg[PIECE];
    const auto kf = key.ready();
    for (int c = threadIdx.x; c < NC; c += 256)
        cur[c] = (uint32_t)off[(int64_t)c * nb + blockIdx.x];
    const int64_t c0 = (int64_t)blockIdx.x * kSortChunk;
    const int64_t c1 = c0 + kSortChunk < n ? c0 + kSortChunk : n;
    // pieces of PIECE points; the next piece's loads are issued before the
    // current piece is ordered and written
    double x[PER], y[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int64_t i = c0 + k * 256 + threadIdx.x;
        x[k] = i < c1 ? px[i] : 0.0;
        y[k] = i < c1 ? py[i] : 0.0;
    }
    for (int64_t p0 = c0; p0 < c1; p0 += PIECE) {
        int32_t id[PER];
        int dg[PER];
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int64_t i = p0 + k * 256 + threadIdx.x;
            id[k] = (int32_t)i;
            dg[k] = i < c1 ? (int)(kf(x[k], y[k]) / NF) : -1;
        }
        double nx[PER], ny[PER];
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int64_t i = p0 + PIECE + k * 256 + threadIdx.x;
            nx[k] = i < c1 ? px[i] : 0.0;
            ny[k] = i < c1 ? py[i] : 0.0;
        }
        write_piece_sorted<NC, PER>(x, y, id, dg, cnt, cur, part, sxy, sid, sdg, txy, tidx);
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            x[k] = nx[k];
            y[k] = ny[k];
        }
    }
}

// One workgroup per coarse digit c: its run [off[c*nb], off[(c+1)*nb]).
// key_start (optional, NC*NF + 1 entries): the first position of every key.
template <class Key, int NC, int NF, int PER>
__global__ __launch_bounds__(256) void k_sort_fine(const double2 *__restrict__ txy, const int32_t *__restrict__ tidx,
                                                   Key key, int nb, const int64_t *__restrict__ off,
                                                   double2 *__restrict__ oxy, int32_t *__restrict__ oidx,
                                                   int64_t *__restrict__ key_start)
{
    constexpr int PIECE = 256 * PER;
    __shared__ uint32_t cnt[NF], cur[NF];
    __shared__ uint32_t part[4];
    __shared__ double2 sxy[PIECE];
    __shared__ int32_t sid[PIECE];
    __shared__ uint16_t sdg[PIECE];
    const auto kf = key.ready();
    const int c = blockIdx.x;
    const int64_t s = off[(int64_t)c * nb];
    const int64_t e = off[(int64_t)(c + 1) * nb];   // c + 1 = NC: the total
    const int t = threadIdx.x;
    // the run's fine counts, then their exclusive prefix as the write cursors
    for (int d = t; d < NF; d += 256)
        cur[d] = 0;
    __syncthreads();
    for (int64_t b = s; b < e; b += 1024) {
        double2 v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int64_t i = b + k * 256 + t;
            v[k] = i < e ? txy[i] : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (b + k * 256 + t < e)
                atomicAdd(&cur[kf(v[k].x, v[k].y) % NF], 1u);
    }
    __syncthreads();
    lds_exclusive_scan<NF>(cur, part);
    for (int d = t; d < NF; d += 256) {
        cur[d] += (uint32_t)s;
        if (key_start)
            key_start[(int64_t)c * NF + d] = cur[d];
    }
    if (key_start && c == NC - 1 && t == 0)
        key_start[(int64_t)NC * NF] = e;
    __syncthreads();
    double2 v[PER];
    int32_t id[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int64_t i = s + k * 256 + t;
        v[k] = i < e ? txy[i] : make_double2(0.0, 0.0);
        id[k] = i < e ? tidx[i] : 0;
    }
    for (int64_t p0 = s; p0 < e; p0 += PIECE) {
        double x[PER], y[PER];
        int dg[PER];
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            x[k] = v[k].x;
            y[k] = v[k].y;
            dg[k] = p0 + k * 256 + t < e ? (int)(kf(x[k], y[k]) % NF) : -1;
        }
        int32_t cid[PER];
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            cid[k] = id[k];
            const int64_t i = p0 + PIECE + k * 256 + t;
            v[k] = i < e ? txy[i] : make_double2(0.0, 0.0);
            id[k] = i < e ? tidx[i] : 0;
        }
        write_piece_sorted<NF, PER>(x, y, cid, dg, cnt, cur, part, sxy, sid, sdg, oxy, oidx);
    }
}

// Sort n points (< 2^31) by Key (values in [0, NC*NF)) in pieces of 256*PER
// points in pass 1 and 256*FPER in pass 2.  nb = chunks of
// kSortChunk points; table: NC*nb words; off: NC*nb + 1 int64; scan_ws:
// scan_ws_entries(NC*nb) int64; txy/tidx: n entries of intermediate storage;
// oxy/oidx: the sorted output; key_start: optional NC*NF + 1 first positions.
template <class Key, int NC, int NF, int PER = 4, int FPER = PER>
int launch_sort_staged(const double *px, const double *py, int64_t n, Key key, int nb, uint32_t *table,
                       int64_t *off, int64_t *scan_ws, double2 *txy, int32_t *tidx, double2 *oxy, int32_t *oidx,
                       int64_t *key_start, hipStream_t s)
{
    hipLaunchKernelGGL((k_sort_coarse_hist<Key, NC, NF>), dim3(nb), dim3(256), 0, s, px, py, n, key, nb, table);
    PIP_HIP_TRY(hipGetLastError());
    PIP_TRY(launch_scan_u32(table, (int64_t)NC * nb, off, scan_ws, s));
    hipLaunchKernelGGL((k_sort_coarse_scatter<Key, NC, NF, PER>), dim3(nb), dim3(256), 0, s, px, py, n, key, nb, off,
                       txy, tidx);
    hipLaunchKernelGGL((k_sort_fine<Key, NC, NF, FPER>), dim3(NC), dim3(256), 0, s, (const double2 *)txy,
                       (const int32_t *)tidx, key, nb, (const int64_t *)off, oxy, oidx, key_start);
    PIP_HIP_TRY(hipGetLastError());
    return PIP_OK;
}

}  // namespace
}  // namespace pip
