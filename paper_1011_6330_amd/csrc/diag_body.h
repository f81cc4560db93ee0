// diag_body.h -- per-wave accumulators of the particle passes of the
// diagnostics (CIC node weights for the Gauss residual, the signed-gamma
// profile), shared by the FP64 and FP32-bulk kernels.
//
// Each wave walks a contiguous range of slots (block_range), so between sorts
// its particles sit in one cell or profile bin for long stretches.  It keeps
// a current key: lanes whose particle belongs to it add to per-lane partial
// sums; when a particle of another key appears, the partial sums are reduced
// over the wave and added to memory with one atomic each, and the key of the
// wave's last particle becomes current.  Particles of any other key go out at
// once through the keyed path (one atomic per distinct key).  Every reduction
// is an integer sum, min or max, so the result does not depend on the order.
#pragma once

#include "pcpic_internal.h"
#include "wave.h"

namespace pcpic {

// Slots [lo, hi) of block b of nblocks over n slots: contiguous ranges of
// whole 256-slot rows.
__device__ __forceinline__ void block_range(int64_t n, int64_t nblocks, int64_t b, int64_t &lo, int64_t &hi)
{
    const int64_t per = (((n + nblocks - 1) / nblocks) + 255) & ~(int64_t)255;
    lo = b * per;
    hi = lo + per < n ? lo + per : n;
}

// CIC node weights: 2^P - F to node `cell`, F to node `cell + 1`.
struct WeightAcc {
    int64_t cell = -1;            // current cell (wave-uniform), -1: none
    int64_t w0 = 0, w1 = 0;       // per-lane partial weights of nodes cell, cell + 1

    __device__ __forceinline__ void flush(unsigned long long *w)
    {
        if (cell < 0) return;
        const int64_t s0 = wave_sum_i64(w0), s1 = wave_sum_i64(w1);
        if (__lane_id() == 0) {
            if (s0 != 0) atomicAdd(w + cell, (unsigned long long)s0);
            if (s1 != 0) atomicAdd(w + cell + 1, (unsigned long long)s1);
        }
        w0 = w1 = 0;
    }

    // Called by every lane of the wave; F is the fixed-point offset in the cell.
    __device__ __forceinline__ void add(unsigned long long *w, bool live, int64_t c, int64_t oneP, int64_t F)
    {
        const unsigned long long lm = __ballot(live);
        if (!lm) return;
        bool mine = live && c == cell;
        if (mine) { w0 += oneP - F; w1 += F; }
        bool rest = live && !mine;
        if (!__ballot(rest)) return;
        flush(w);
        cell = __shfl(c, 63 - __clzll(lm));
        mine = rest && c == cell;
        if (mine) { w0 += oneP - F; w1 += F; }
        rest = rest && !mine;
        wave_add_keyed(w, c, oneP - F, rest);
        wave_add_keyed(w, c + 1, F, rest);
    }
};

// Signed-gamma profile: per bin the count, the 128-bit fixed-point sum (integer
// part and 2^-32 fraction summed separately, combined exactly when added to
// memory), min and max of the ordered bit images.
struct ProfOut {
    long long *cnt;
    unsigned long long *lo;
    long long *hi;
    long long *mn, *mx;
};

struct ProfAcc {
    int64_t bin = -1;                                   // current bin (wave-uniform), -1: none
    int64_t c = 0, si = 0, sf = 0;                      // per-lane partial count and sums
    long long mn = 0x7fffffffffffffffLL, mx = (long long)0x8000000000000000ULL;

    __device__ __forceinline__ static void emit(const ProfOut &o, int64_t b, int64_t sc, int64_t si, int64_t sf,
                                                long long smin, long long smax)
    {
        atomicAdd((unsigned long long *)&o.cnt[b], (unsigned long long)sc);
        atomic_add_i128(&o.lo[b], &o.hi[b], ((__int128)si << 32) + (__int128)sf);
        atomicMin(&o.mn[b], smin);
        atomicMax(&o.mx[b], smax);
    }

    __device__ __forceinline__ void take(int64_t gi, int64_t gf, long long ob)
    {
        c += 1;
        si += gi;
        sf += gf;
        mn = ob < mn ? ob : mn;
        mx = ob > mx ? ob : mx;
    }

    __device__ __forceinline__ void flush(const ProfOut &o)
    {
        if (bin < 0) return;
        const int64_t sc = wave_sum_i64(c), ssi = wave_sum_i64(si), ssf = wave_sum_i64(sf);
        const long long smin = wave_min_i64(mn), smax = wave_max_i64(mx);
        if (__lane_id() == 0 && sc > 0) emit(o, bin, sc, ssi, ssf, smin, smax);
        c = si = sf = 0;
        mn = 0x7fffffffffffffffLL;
        mx = (long long)0x8000000000000000ULL;
    }

    // Called by every lane of the wave.
    __device__ __forceinline__ void add(const ProfOut &o, bool want, int64_t b, int64_t gi, int64_t gf, long long ob)
    {
        const unsigned long long wm = __ballot(want);
        if (!wm) return;
        bool mine = want && b == bin;
        if (mine) take(gi, gf, ob);
        bool rest = want && !mine;
        if (!__ballot(rest)) return;
        flush(o);
        bin = __shfl(b, 63 - __clzll(wm));
        mine = rest && b == bin;
        if (mine) take(gi, gf, ob);
        rest = rest && !mine;
        unsigned long long pend = __ballot(rest);
        while (pend) {
            const int leader = __ffsll(pend) - 1;
            const int64_t lb = __shfl(b, leader);
            const bool one = rest && b == lb;
            const int64_t sc = wave_sum_i64(one ? 1 : 0);
            const int64_t ssi = wave_sum_i64(one ? gi : 0);
            const int64_t ssf = wave_sum_i64(one ? gf : 0);
            const long long smin = wave_min_i64(one ? ob : 0x7fffffffffffffffLL);
            const long long smax = wave_max_i64(one ? ob : (long long)0x8000000000000000ULL);
            if ((int)__lane_id() == leader) emit(o, lb, sc, ssi, ssf, smin, smax);
            pend &= ~__ballot(one);
            rest = rest && !one;
        }
    }
};

// Profile bin and the signed gamma sign(u) sqrt(1 + u^2) of a particle at x
// (cell units) as integer part, 2^-32 fraction and ordered bit image.
__device__ __forceinline__ void prof_values(const Consts &c, int nb, double x, double u, int64_t &bin, int64_t &gi,
                                            int64_t &gf, long long &ob)
{
    double t = u * u;
    t = 1.0 + t;
    const double gam = sqrt(t);
    const double sg = u < 0.0 ? -gam : gam;
    bin = (int64_t)floor((x * (double)nb) / (double)c.N);
    if (bin < 0) bin = 0;
    if (bin > nb - 1) bin = nb - 1;
    const double fl = floor(sg);
    gi = (int64_t)fl;
    gf = (int64_t)rint((sg - fl) * 4294967296.0);
    ob = ordered_bits(sg);
}

}  // namespace pcpic
