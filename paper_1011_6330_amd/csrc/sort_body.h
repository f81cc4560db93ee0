// sort_body.h -- per-tile bodies of the scatter pass of the cell sort, shared
// by the single-tube kernels and the batched sort.
//
// A tile is SORT_TILE consecutive source slots, taken by a block of
// SORT_BLOCK threads as SORT_PPT columns of SORT_BLOCK consecutive slots
// (thread t holds slot tile0 + k SORT_BLOCK + t of column k).  For each
// column, the lanes of a run of equal keys take consecutive destination slots
// with one atomic per run on the key's running offset.  The columns' atomics
// are issued together, in source order, so their latencies overlap and the
// particles of a key keep roughly their source order.  That order carries no
// result (every step is per particle or an integer reduction), but between
// sorts it keeps particles with similar histories, and hence similar
// velocities, in the same wave.
#pragma once

#include <math.h>

#include "pcpic_internal.h"
#include "wave.h"

namespace pcpic {

// The two FP32-bulk particle streams of one buffer parity.
struct Streams {
    int *CL;
    float *OL;
    float *UL;
    unsigned *HP;   // high stream: position words, cells of wide groups, group headers
    int *HW;
    int *HG;
    double *UH;
};

// Cell (-1 for a removed slot) and offset of high-stream slot p.
__device__ __forceinline__ int hi_slot(const Streams &s, int64_t p, float &off)
{
    const unsigned w = s.HP[p];
    off = hi_offset(w);
    if (w == HI_DEAD) return -1;
    const int hdr = s.HG[p >> HI_GROUP_LOG2];
    return hdr >= 0 ? hi_cell(w, hdr, 0) : s.HW[p];
}

// Writes a live particle (cell, frac in units of 2^-24) at high-stream slot q
// of a stream being filled in the wide form (the sort, the appends); the first
// slot of each group sets the group's header.
__device__ __forceinline__ void hi_put_wide(const Streams &s, int64_t q, int cell, unsigned frac, double u)
{
    s.HW[q] = cell;
    s.HP[q] = frac;
    s.UH[q] = u;
    if ((q & (HI_GROUP - 1)) == 0) s.HG[q >> HI_GROUP_LOG2] = HI_WIDE;
}

// Destination stream of a particle: the high stream from |u| >= u_hi on.
__device__ __forceinline__ bool goes_high(double u, double u_hi) { return fabs(u) >= u_hi; }

// Item k of a pass over a tube's slots in tiles of SORT_TILE: FP64 has one
// stream; in FP32-bulk mode the low stream's tiles come first, then the high
// stream's.  Returns false for an item past the slots (so ceil(capacity /
// SORT_TILE) items, plus one in FP32-bulk mode, cover any split).
__device__ __forceinline__ bool sort_item(int64_t k, bool f32, const DevCounters *ctr, bool &hi, int64_t &tile0,
                                          int64_t &n)
{
    const int64_t n_lo = ctr->n_slots;
    const int64_t items_lo = (n_lo + SORT_TILE - 1) / SORT_TILE;
    hi = f32 && k >= items_lo;
    tile0 = (hi ? k - items_lo : k) * SORT_TILE;
    n = hi ? ctr->n_slots_hi : n_lo;
    return tile0 < n;
}

// Scatter of the FP64 slots [tile0, tile0 + SORT_TILE) of (X, U), tile0 < n,
// into (Xo, Uo) at the running offsets off[key]; removed slots (x < 0) are
// dropped.  Called by every thread of a block of SORT_BLOCK threads.
__device__ __forceinline__ void scatter_tile_f64(const Consts &c, const double *X, const double *U, double *Xo,
                                                 double *Uo, unsigned long long *off, int64_t n, int64_t tile0)
{
    const int lane = (int)__lane_id();
    double x[SORT_PPT], u[SORT_PPT];
#pragma unroll
    for (int k = 0; k < SORT_PPT; ++k) {
        const int64_t p = tile0 + (int64_t)k * SORT_BLOCK + threadIdx.x;
        x[k] = p < n ? __builtin_nontemporal_load(X + p) : -1.0;
        u[k] = p < n ? __builtin_nontemporal_load(U + p) : 0.0;
    }
    int64_t key[SORT_PPT];
    bool want[SORT_PPT];
    WaveRun r[SORT_PPT];
    unsigned long long f[SORT_PPT];
#pragma unroll
    for (int k = 0; k < SORT_PPT; ++k) {
        want[k] = x[k] >= 0.0;
        key[k] = want[k] ? sort_key_f64(c, x[k]) : 0;
        r[k] = wave_runs(key[k], want[k]);
    }
#pragma unroll
    for (int k = 0; k < SORT_PPT; ++k) {
        f[k] = 0;
        if (want[k] && r[k].is_head) f[k] = atomicAdd(off + key[k], (unsigned long long)(r[k].end - lane));
    }
#pragma unroll
    for (int k = 0; k < SORT_PPT; ++k) {
        f[k] = __shfl(f[k], r[k].head);
        if (want[k]) {
            const int64_t d = (int64_t)f[k] + r[k].rank;
            Xo[d] = x[k];
            Uo[d] = u[k];
        }
    }
}

// Scatter of the FP32-bulk slots [tile0, tile0 + SORT_TILE) of one source
// stream (HI: the high stream), tile0 < n.  The key (sort_key_f32) names the
// destination stream from the particle's momentum, so particles migrate
// between the streams here; tlo is the number of slots of the destination low
// stream (the high stream's keys start there).
template <bool HI>
__device__ __forceinline__ void scatter_tile_f32(const Consts &c, const Streams &src, const Streams &dst,
                                                 double u_hi, int64_t tlo, unsigned long long *off, int64_t n,
                                                 int64_t tile0)
{
    const int lane = (int)__lane_id();
    int cl[SORT_PPT];
    float o[SORT_PPT];
    double u[SORT_PPT];
#pragma unroll
    for (int k = 0; k < SORT_PPT; ++k) {
        const int64_t p = tile0 + (int64_t)k * SORT_BLOCK + threadIdx.x;
        const bool in = p < n;
        if (HI) {
            o[k] = 0.0f;
            cl[k] = in ? hi_slot(src, p, o[k]) : -1;
            u[k] = in ? __builtin_nontemporal_load(src.UH + p) : 0.0;
        } else {
            cl[k] = in ? __builtin_nontemporal_load(src.CL + p) : -1;
            o[k] = in ? __builtin_nontemporal_load(src.OL + p) : 0.0f;
            u[k] = in ? (double)__builtin_nontemporal_load(src.UL + p) : 0.0;
        }
    }
    const int64_t klo = sort_low_keys(c);
    int64_t key[SORT_PPT];
    bool want[SORT_PPT];
    WaveRun r[SORT_PPT];
    unsigned long long f[SORT_PPT];
#pragma unroll
    for (int k = 0; k < SORT_PPT; ++k) {
        want[k] = cl[k] >= 0;
        key[k] = want[k] ? sort_key_f32(c, cl[k], o[k], goes_high(u[k], u_hi)) : 0;
        r[k] = wave_runs(key[k], want[k]);
    }
#pragma unroll
    for (int k = 0; k < SORT_PPT; ++k) {
        f[k] = 0;
        if (want[k] && r[k].is_head) f[k] = atomicAdd(off + key[k], (unsigned long long)(r[k].end - lane));
    }
#pragma unroll
    for (int k = 0; k < SORT_PPT; ++k) {
        f[k] = __shfl(f[k], r[k].head);
        if (want[k]) {
            const int64_t d = (int64_t)f[k] + r[k].rank;
            if (key[k] >= klo) {
                // a low particle reaching the threshold was put on the 2^-24 grid by its push
                int cell = cl[k];
                unsigned frac;
                hi_snap((double)o[k], cell, frac);
                if (cell >= (int)c.N) { cell = (int)c.N - 1; frac = HI_FRAC_MASK; }
                hi_put_wide(dst, d - tlo, cell, frac, u[k]);
            } else {
                dst.CL[d] = cl[k];
                dst.OL[d] = o[k];
                dst.UL[d] = (float)u[k];
            }
        }
    }
}

// Sort-key counts of the slots [tile0, tile0 + SORT_TILE) of one stream (as
// the scatter keys them), one atomic per run of equal keys in a wave.
__device__ __forceinline__ void hist_tile(const Consts &c, bool f32, bool hi, const double *X, const Streams &s,
                                          double u_hi, unsigned long long *count, int64_t n, int64_t tile0)
{
#pragma unroll 1
    for (int q = 0; q < SORT_PPT; ++q) {
        const int64_t p = tile0 + (int64_t)q * SORT_BLOCK + threadIdx.x;
        bool live = false;
        int64_t key = 0;
        if (p < n) {
            if (f32) {
                float off = 0.0f;
                const int cell = hi ? hi_slot(s, p, off) : s.CL[p];
                if (cell >= 0) {
                    const double u = hi ? s.UH[p] : (double)s.UL[p];
                    live = true;
                    key = sort_key_f32(c, cell, hi ? off : s.OL[p], goes_high(u, u_hi));
                }
            } else {
                const double x = X[p];
                if (x >= 0.0) {
                    live = true;
                    key = sort_key_f64(c, x);
                }
            }
        }
        const WaveRun r = wave_runs(key, live);
        if (live && r.is_head) atomicAdd(count + key, (unsigned long long)(r.end - (int)__lane_id()));
    }
}

}  // namespace pcpic
