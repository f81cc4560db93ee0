// wave.h -- 64-lane wavefront helpers for gfx950 (CDNA4 runs wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pcpic {

__device__ __forceinline__ int64_t wave_sum_i64(int64_t v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

__device__ __forceinline__ long long wave_min_i64(long long v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        long long o = __shfl_xor(v, off);
        v = o < v ? o : v;
    }
    return v;
}

__device__ __forceinline__ long long wave_max_i64(long long v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        long long o = __shfl_xor(v, off);
        v = o > v ? o : v;
    }
    return v;
}

// Runs of equal keys over consecutive lanes of the wave.  A lane without
// `want` belongs to no run and ends the run before it.  For a lane with `want`:
// head = first lane of its run, rank = lane - head, end = one past the run's
// last lane; is_head marks the first lane.  With sorted particles a run is a
// cell (or sort key), so one atomic per run replaces one per particle.
struct WaveRun {
    int head, rank, end;
    bool is_head;
};

__device__ __forceinline__ WaveRun wave_runs(long long key, bool want)
{
    const int lane = (int)__lane_id();
    const unsigned long long wm = __ballot(want);
    const long long kprev = __shfl_up(key, 1u);
    const bool prev_want = lane > 0 && ((wm >> (lane - 1)) & 1ull);
    const bool head = want && (!prev_want || kprev != key);
    const unsigned long long hm = __ballot(head);
    const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);   // lanes 0..lane
    const unsigned long long brk = (hm | ~wm) & ~upto;                              // breaks above the lane
    WaveRun r;
    r.is_head = head;
    r.head = 63 - __clzll(hm & upto);
    r.rank = lane - r.head;
    r.end = brk ? __ffsll(brk) - 1 : 64;
    return r;
}

// Add `val` to dst[key] for every lane with `want`, one global atomic per
// distinct key present in the wave: lanes sharing the leader's key are summed
// with a butterfly, the leader lane issues the atomic, and the loop repeats
// over the keys still pending.  Integer addition makes the result independent
// of the order in which waves and lanes arrive.
__device__ __forceinline__ void wave_add_keyed(unsigned long long *dst, int64_t key, int64_t val,
                                               bool want)
{
    unsigned long long pend = __ballot(want);
    while (pend) {
        const int leader = __ffsll((unsigned long long)pend) - 1;
        const int64_t lk = __shfl(key, leader);
        const bool mine = want && key == lk;
        const int64_t v = wave_sum_i64(mine ? val : 0);
        if ((int)__lane_id() == leader && v != 0) atomicAdd(dst + lk, (unsigned long long)v);
        pend &= ~__ballot(mine);
        want = want && !mine;
    }
}

// 128-bit two's-complement accumulation into (lo, hi) words with carry.
__device__ __forceinline__ void atomic_add_i128(unsigned long long *lo, long long *hi, __int128 v)
{
    const unsigned long long vlo = (unsigned long long)v;
    const long long vhi = (long long)(v >> 64);
    const unsigned long long old = atomicAdd(lo, vlo);
    const long long carry = (old + vlo < old) ? 1 : 0;
    if (vhi + carry != 0) atomicAdd((unsigned long long *)hi, (unsigned long long)(vhi + carry));
}

}  // namespace pcpic

namespace pcpic {

// DPP move of a double (two 32-bit halves); lanes whose source is outside the
// pattern read 0.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_f64(double v)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, ROWMASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWMASK, 0xf, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

// Sum over the 64 lanes, valid in lane 63: inclusive scan inside each row of
// 16 lanes (row_shr 1, 2, 4, 8), then row 0 -> row 1 and row 2 -> row 3
// (row_bcast:15), then rows 0-1 -> rows 2-3 (row_bcast:31).  The additions
// come in a fixed order (exact for integer-valued doubles below 2^53).
__device__ __forceinline__ double wave_sum_f64_to63(double v)
{
    v += dpp_f64<0x111, 0xf>(v);
    v += dpp_f64<0x112, 0xf>(v);
    v += dpp_f64<0x114, 0xf>(v);
    v += dpp_f64<0x118, 0xf>(v);
    v += dpp_f64<0x142, 0xa>(v);
    v += dpp_f64<0x143, 0xc>(v);
    return v;
}

// The double of the lane n places lower in the same row of 16 lanes; the
// first n lanes of each row read 0 (bound control, so no old value is kept).
template <int N>
__device__ __forceinline__ double dpp_row_shr_f64(double v)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), 0x110 + N, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x110 + N, 0xf, 0xf, true);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

// Row swaps of a double across two registers (a row is 16 lanes; both 32-bit
// halves move together).  swap_rows32: rows 2-3 of a trade places with rows
// 0-1 of b, so a becomes (a0, a1, b0, b1) and b becomes (a2, a3, b2, b3).
// swap_rows16: the odd rows of a trade places with the even rows of b, so a
// becomes (a0, b0, a2, b2) and b becomes (a1, b1, a3, b3).
__device__ __forceinline__ void swap_rows32_f64(double &a, double &b)
{
    const unsigned long long ua = __builtin_bit_cast(unsigned long long, a);
    const unsigned long long ub = __builtin_bit_cast(unsigned long long, b);
    const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)ua, (unsigned)ub, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(ua >> 32), (unsigned)(ub >> 32), false, false);
    a = __builtin_bit_cast(double, ((unsigned long long)hi[0] << 32) | lo[0]);
    b = __builtin_bit_cast(double, ((unsigned long long)hi[1] << 32) | lo[1]);
}
__device__ __forceinline__ void swap_rows16_f64(double &a, double &b)
{
    const unsigned long long ua = __builtin_bit_cast(unsigned long long, a);
    const unsigned long long ub = __builtin_bit_cast(unsigned long long, b);
    const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)ua, (unsigned)ub, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(ua >> 32), (unsigned)(ub >> 32), false, false);
    a = __builtin_bit_cast(double, ((unsigned long long)hi[0] << 32) | lo[0]);
    b = __builtin_bit_cast(double, ((unsigned long long)hi[1] << 32) | lo[1]);
}

// Sums over the 64 lanes of four values at once: on return row k (lanes
// 16k .. 16k+15) works on the k-th argument, and lane 16k + 15 holds its
// total.  Two row swaps fold the four rows of each value onto one row (every
// lane then holds the sum of its four lanes of equal position in the rows),
// and an inclusive scan inside the row (row_shr 1, 2, 4, 8) leaves the row
// total in its last lane.  For integer-valued doubles whose sums stay below
// 2^53 every addition is exact.
__device__ __forceinline__ double wave_sum4_rows_f64(double v0, double v1, double v2, double v3)
{
    swap_rows32_f64(v0, v2);
    swap_rows32_f64(v1, v3);
    double s = v0 + v2;          // rows 0-1: v0 over rows (r, r+2); rows 2-3: v2
    double t = v1 + v3;          // rows 0-1: v1; rows 2-3: v3
    swap_rows16_f64(s, t);
    double v = s + t;            // row k: value k summed over the four rows
    v += dpp_row_shr_f64<1>(v);
    v += dpp_row_shr_f64<2>(v);
    v += dpp_row_shr_f64<4>(v);
    v += dpp_row_shr_f64<8>(v);
    return v;
}

// Maximum over the 64 lanes of non-negative doubles, valid in lane 63: the DPP
// pattern of wave_sum_f64_to63 with max in place of the sum (a lane without a
// source reads 0, which no non-negative value is below).
__device__ __forceinline__ double wave_max_f64_to63(double v)
{
    v = fmax(v, dpp_f64<0x111, 0xf>(v));
    v = fmax(v, dpp_f64<0x112, 0xf>(v));
    v = fmax(v, dpp_f64<0x114, 0xf>(v));
    v = fmax(v, dpp_f64<0x118, 0xf>(v));
    v = fmax(v, dpp_f64<0x142, 0xa>(v));
    v = fmax(v, dpp_f64<0x143, 0xc>(v));
    return v;
}

// Minimum (maximum) of an int32 over the 64 lanes, returned in every lane: the
// DPP pattern of wave_sum_f64_to63 on int32 with min (max) in place of the sum,
// where a lane without a DPP source keeps its own value, then lane 63 read back.
__device__ __forceinline__ int wave_min_i32(int v)
{
    v = min(v, __builtin_amdgcn_update_dpp(v, v, 0x111, 0xf, 0xf, false));
    v = min(v, __builtin_amdgcn_update_dpp(v, v, 0x112, 0xf, 0xf, false));
    v = min(v, __builtin_amdgcn_update_dpp(v, v, 0x114, 0xf, 0xf, false));
    v = min(v, __builtin_amdgcn_update_dpp(v, v, 0x118, 0xf, 0xf, false));
    v = min(v, __builtin_amdgcn_update_dpp(v, v, 0x142, 0xa, 0xf, false));
    v = min(v, __builtin_amdgcn_update_dpp(v, v, 0x143, 0xc, 0xf, false));
    return __builtin_amdgcn_readlane(v, 63);
}
__device__ __forceinline__ int wave_max_i32(int v)
{
    v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x111, 0xf, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x112, 0xf, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x114, 0xf, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x118, 0xf, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x142, 0xa, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x143, 0xc, 0xf, false));
    return __builtin_amdgcn_readlane(v, 63);
}

// Value of lane - 1 (lane 0 reads 0): DPP wave_shr:1.
__device__ __forceinline__ int wave_shr1_i32(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xf, 0xf, false);
}

// Runs of equal int keys over consecutive lanes, as wave_runs, with the lane
// shift done by DPP instead of a cross-lane permute through LDS.
__device__ __forceinline__ WaveRun wave_runs_i32(int key, bool want)
{
    const int lane = (int)__lane_id();
    const unsigned long long wm = __ballot(want);
    const int kprev = wave_shr1_i32(key);
    const bool prev_want = lane > 0 && ((wm >> (lane - 1)) & 1ull);
    const bool head = want && (!prev_want || kprev != key);
    const unsigned long long hm = __ballot(head);
    const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);   // lanes 0..lane
    const unsigned long long brk = (hm | ~wm) & ~upto;                              // breaks above the lane
    WaveRun r;
    r.is_head = head;
    r.head = 63 - __clzll(hm & upto);
    r.rank = lane - r.head;
    r.end = brk ? __ffsll(brk) - 1 : 64;
    return r;
}

// Sum of v over [head, lane] inside the lane's run (head = lane - rank): a
// segmented inclusive scan on DPP, row_shr 1, 2, 4, 8 inside each row of 16
// lanes, then row_bcast:15 (rows 0 -> 1, 2 -> 3) and row_bcast:31 (row 1 ->
// rows 2, 3), each step taken only where the source lane lies in the same run.
// On a run's last lane it is the run total.  Every lane must call it.  For
// integer-valued doubles below 2^53 (the current) every addition is exact.
__device__ __forceinline__ double run_sum_to_tail(double v, int rank)
{
    const int lane = (int)__lane_id();
    const int head = lane - rank;
    double t;
    t = dpp_f64<0x111, 0xf>(v);
    if (rank >= 1) v += t;
    t = dpp_f64<0x112, 0xf>(v);
    if (rank >= 2) v += t;
    t = dpp_f64<0x114, 0xf>(v);
    if (rank >= 4) v += t;
    t = dpp_f64<0x118, 0xf>(v);
    if (rank >= 8) v += t;
    t = dpp_f64<0x142, 0xa>(v);                 // lane 15 -> row 1, lane 47 -> row 3; rows 0, 2 read 0
    if (head < (lane & ~15)) v += t;
    t = dpp_f64<0x143, 0xc>(v);                 // lane 31 -> rows 2, 3; rows 0, 1 read 0
    if (head < 32) v += t;
    return v;
}

// Inclusive scan of one value per thread over a block of 256 threads (wave
// scan, then the totals of the lower waves through LDS).  s_wave holds 4
// entries of the caller's shared memory; every thread must call it.
__device__ __forceinline__ long long block_scan_incl(long long v, long long *s_wave)
{
    const int lane = (int)__lane_id();
    const int wv = threadIdx.x >> 6;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const long long o = __shfl_up(v, off);
        if (lane >= off) v += o;
    }
    if (lane == 63) s_wave[wv] = v;
    __syncthreads();
    long long add = 0;
    for (int k = 0; k < wv; ++k) add += s_wave[k];
    __syncthreads();
    return v + add;
}

}  // namespace pcpic
