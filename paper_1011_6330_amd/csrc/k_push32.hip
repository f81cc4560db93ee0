// k_push32.hip -- the FP32-bulk particle path.
//
// Particles live in two SoA streams whose positions keep 24 bits of resolution
// inside a cell of a tube of any length:
//   low stream  (gamma below the threshold): cell i32, offset f32 in [0, 1),
//               u = gamma*beta in f32, 12 B/slot; kick from the f32 kick
//               array, v = u * rsqrt(1 + u^2) (never formed from gamma, so
//               nothing cancels near v = c);
//   high stream (gamma at or above the threshold, 1e6 by default): a 32-bit
//               position word (offset in units of 2^-24, cell relative to the
//               base cell of its group of 256 slots) and u in f64, 12 B/slot;
//               kick, gamma and v in f64 as the FP64 path.
// The deposit takes F = rint(2^P offset) of the stored offsets, so charge
// conservation stays exact.  Fields, the Gauss residual and E_surf stay FP64;
// the high stream's kick is (q/m) dt E_z formed in f64 from E_z itself.  The
// cell sort moves particles between the streams.
#include <math.h>

#include "pcpic_internal.h"
#include "push_common.h"
#include "push_body.h"
#include "sort_body.h"
#include "diag_body.h"

namespace pcpic {

template <int BLOCK, int NT>
__global__ __launch_bounds__(BLOCK) void k_push_f32(Consts c, Push32Args a)
{
    push_item_f32<BLOCK, NT>(c, a, blockIdx.x, a.ctr->n_slots, a.ctr->n_slots_hi);
}

// ------------------------------------------------------------------------
// diagnostics, sort and append for the two streams
// ------------------------------------------------------------------------

// Block b's contiguous range of the slots of both streams taken end to end
// (the low stream's, then the high stream's): [lo0, hi0) of the low stream and
// [lo1, hi1) of the high stream, either possibly empty.
__device__ __forceinline__ void stream_ranges(const DevCounters *ctr, int64_t &lo0, int64_t &hi0, int64_t &lo1,
                                              int64_t &hi1)
{
    const int64_t n_lo = ctr->n_slots, n_hi = ctr->n_slots_hi;
    int64_t a, b;
    block_range(n_lo + n_hi, gridDim.x, blockIdx.x, a, b);
    lo0 = a < n_lo ? a : n_lo;
    hi0 = b < n_lo ? b : n_lo;
    lo1 = (a > n_lo ? a : n_lo) - n_lo;
    hi1 = (b > n_lo ? b : n_lo) - n_lo;
}

__global__ __launch_bounds__(256) void k_weights32(Consts c, Streams s, const DevCounters *ctr,
                                                   unsigned long long *w)
{
    int64_t r[4];
    stream_ranges(ctr, r[0], r[1], r[2], r[3]);
    WeightAcc acc;
#pragma unroll 1
    for (int high = 0; high < 2; ++high) {
        const int64_t hi = r[2 * high + 1];
        for (int64_t base = r[2 * high]; base < hi; base += 256) {
            const int64_t p = base + threadIdx.x;
            float off = 0.0f;
            int cell = -1;
            if (p < hi) {
                if (high) cell = hi_slot(s, p, off);
                else { cell = s.CL[p]; off = s.OL[p]; }
            }
            const bool live = cell >= 0;
            int64_t F = 0;
            if (live) F = (int64_t)rint((double)off * c.twoP);
            acc.add(w, live, cell, c.oneP, F);
        }
    }
    acc.flush(w);
}

__global__ __launch_bounds__(256) void k_profile32(Consts c, int nb, Streams s, const DevCounters *ctr, ProfOut o)
{
    int64_t r[4];
    stream_ranges(ctr, r[0], r[1], r[2], r[3]);
    ProfAcc acc;
#pragma unroll 1
    for (int high = 0; high < 2; ++high) {
        const int64_t hi = r[2 * high + 1];
        for (int64_t base = r[2 * high]; base < hi; base += 256) {
            const int64_t p = base + threadIdx.x;
            float off = 0.0f;
            int cell = -1;
            if (p < hi) {
                if (high) cell = hi_slot(s, p, off);
                else { cell = s.CL[p]; off = s.OL[p]; }
            }
            const bool want = cell >= 0;
            int64_t bin = 0, gi = 0, gf = 0;
            long long ob = 0;
            if (want) {
                const double u = high ? s.UH[p] : (double)s.UL[p];
                prof_values(c, nb, (double)cell + (double)off, u, bin, gi, gf, ob);
            }
            acc.add(o, want, bin, gi, gf, ob);
        }
    }
    acc.flush(o);
}

// Histogram for the sort (sort_key_f32: the destination stream's key range),
// one block per tile of either stream (sort_item).
__global__ __launch_bounds__(SORT_BLOCK) void k_hist32(Consts c, Streams s, const DevCounters *ctr, double u_hi,
                                                       unsigned long long *count)
{
    bool hi;
    int64_t tile0, n;
    if (!sort_item(blockIdx.x, true, ctr, hi, tile0, n)) return;
    hist_tile(c, true, hi, nullptr, s, u_hi, count, n, tile0);
}

// Scatter into the other buffer, one block per tile of either stream; tlo is
// the destination low stream's slot count (the offset of the first high key).
__global__ __launch_bounds__(SORT_BLOCK) void k_scatter32(Consts c, Streams src, Streams dst, const DevCounters *ctr,
                                                          double u_hi, unsigned long long *off,
                                                          const long long *total_lo)
{
    bool hi;
    int64_t tile0, n;
    if (!sort_item(blockIdx.x, true, ctr, hi, tile0, n)) return;
    const int64_t tlo = *total_lo;
    if (hi)
        scatter_tile_f32<true>(c, src, dst, u_hi, tlo, off, n, tile0);
    else
        scatter_tile_f32<false>(c, src, dst, u_hi, tlo, off, n, tile0);
}

// Low-destination total = exclusive offset of the first high key; copied before
// the scatter's atomics advance that offset.
__global__ void k_copy_total(const long long *src, long long *dst)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = *src;
}

__global__ void k_sort32_finish(DevCounters *ctr, const long long *total_lo)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const long long lo = *total_lo;
        ctr->n_slots_hi = ctr->n_alive - lo;
        ctr->n_slots = lo;
        ctr->n_removed = 0;
    }
}

// Staged particles (x in cell units, u) -> validity count.
__global__ __launch_bounds__(256) void k_check_staged(Consts c, const double *X, const double *U, int64_t n,
                                                      DevCounters *ctr)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    bool bad = false;
    if (i < n) bad = !(X[i] >= 0.0 && X[i] < (double)c.N) || !isfinite(U[i]);
    const int64_t nb = wave_sum_i64(bad ? 1 : 0);
    if (__lane_id() == 0 && nb) atomicAdd((unsigned long long *)&ctr->bad_inputs, (unsigned long long)nb);
}

// Appending staged particles keeps their order in both streams (so a beam
// loaded in x order needs no sort before it pushes at full rate): block b of
// 256 staged particles counts its high-stream ones (k_stage_count), one block
// turns the counts into exclusive offsets and advances the slot counters
// (k_stage_offsets), and k_append_staged writes each particle at its stream's
// old slot count + its block's offset + its rank in the block.
__global__ __launch_bounds__(256) void k_stage_count(const double *U, int64_t n, double u_hi, long long *blk)
{
    __shared__ int s_w[4];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool high = i < n && goes_high(U[i], u_hi);
    const int cnt = __popcll(__ballot(high));
    if (__lane_id() == 0) s_w[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) blk[blockIdx.x] = s_w[0] + s_w[1] + s_w[2] + s_w[3];
}

// One block: blk[0, nblk) -> exclusive prefix sums in place; base[0], base[1] =
// the low and high slot counts before the append, which then advance.
__global__ __launch_bounds__(256) void k_stage_offsets(long long *blk, int64_t nblk, int64_t n, DevCounters *ctr,
                                                       long long *base)
{
    __shared__ long long s_wave[4];
    __shared__ long long s_carry;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (int64_t b0 = 0; b0 < nblk; b0 += 256) {
        const int64_t i = b0 + threadIdx.x;
        const long long v = i < nblk ? blk[i] : 0;
        const long long inc = block_scan_incl(v, s_wave);
        const long long carry = s_carry;
        if (i < nblk) blk[i] = carry + inc - v;
        __syncthreads();
        if (threadIdx.x == 255) s_carry = carry + inc;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const long long total_hi = s_carry;
        base[0] = ctr->n_slots;
        base[1] = ctr->n_slots_hi;
        ctr->n_slots += n - total_hi;
        ctr->n_slots_hi += total_hi;
    }
}

// Staged particles -> (cell, f32 offset) in the stream their gamma selects; the
// high stream takes them in the wide form (offsets on its 2^-24 grid).  The
// group that held the high stream's last slots before the append is first
// rewritten wide by the thread that writes its first new slot: the only
// thread that touches that group's header here.
__global__ __launch_bounds__(256) void k_append_staged(Consts c, const double *X, const double *U, int64_t n,
                                                       Streams s, double u_hi, const long long *blk,
                                                       const long long *base)
{
    __shared__ int s_hi[4], s_lo[4];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int lane = __lane_id(), wv = threadIdx.x >> 6;
    const bool want = i < n;
    double x = 0.0, u = 0.0;
    if (want) { x = X[i]; u = U[i]; }
    const bool high = want && goes_high(u, u_hi);
    const unsigned long long mh = __ballot(high), ml = __ballot(want && !high);
    if (lane == 0) { s_hi[wv] = __popcll(mh); s_lo[wv] = __popcll(ml); }
    __syncthreads();
    int ph = 0, pl = 0;
    for (int q = 0; q < wv; ++q) { ph += s_hi[q]; pl += s_lo[q]; }
    if (!want) return;
    // 0 <= x < N: the offset in [0, 1), on the stream's grid; one that rounds up to
    // 1 moves into the next cell, except past the last cell, where it stays just below 1
    const double cd = floor(x);
    const int N = (int)c.N;
    int cell = (int)cd;
    const unsigned long long below = (1ull << lane) - 1ull;
    const long long hi_before = blk[blockIdx.x];                           // high particles in earlier blocks
    if (high) {
        unsigned frac;
        hi_snap(x - cd, cell, frac);
        if (cell >= N) { cell = N - 1; frac = HI_FRAC_MASK; }
        const int64_t d = base[1] + hi_before + ph + __popcll(mh & below);
        const int64_t g0 = d & ~(int64_t)(HI_GROUP - 1);
        if (d == base[1] && d != g0) {
            const int hdr = s.HG[d >> HI_GROUP_LOG2];
            if (hdr >= 0) {
                for (int64_t q = g0; q < d; ++q) {
                    const unsigned w = s.HP[q];
                    if (w == HI_DEAD) continue;
                    s.HW[q] = hi_cell(w, hdr, 0);
                    s.HP[q] = w & HI_FRAC_MASK;
                }
                s.HG[d >> HI_GROUP_LOG2] = HI_WIDE;
            }
        }
        hi_put_wide(s, d, cell, frac, u);
    } else {
        float o = (float)(x - cd);
        if (o >= 1.0f) { o = 0.0f; cell += 1; }
        if (cell >= N) { cell = N - 1; o = 0x1.fffffep-1f; }
        const int64_t d = base[0] + ((int64_t)blockIdx.x * 256 - hi_before) + pl + __popcll(ml & below);
        s.CL[d] = cell; s.OL[d] = o; s.UL[d] = (float)u;
    }
}

// ------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------

static Streams streams_of(pic_handle *h, int b)
{
    const Workspace &w = h->ws;
    return Streams{w.cl[b], w.ol[b], w.ul[b], w.hp[b], w.hw[b], w.hg[b], w.uh[b]};
}

template <int BLOCK, int NT>
static hipError_t launch_push32_t(pic_handle *h)
{
    const Workspace &w = h->ws;
    const int b = h->pbuf;
    const int64_t tile_hi = (int64_t)BLOCK * F32_PPT_HI;
    const unsigned items = (unsigned)((h->c.cap + tile_hi - 1) / tile_hi + 1);   // both streams, any split
    Push32Args a{w.cl[b], w.ol[b], w.ul[b], w.hp[b], w.hw[b], w.hg[b], w.uh[b], w.k32, w.ez[h->fbuf],
                 (unsigned long long *)w.j[h->jbuf], w.ctr,
                 h->hist_on ? (unsigned long long *)w.cell_count : nullptr, h->u_hi};
    hipLaunchKernelGGL((k_push_f32<BLOCK, NT>), dim3(items), dim3(BLOCK), 0, h->stream, h->c, a);
    return hipGetLastError();
}

hipError_t launch_push_f32(pic_handle *h)
{
    const int B = h->push_block;
    if (h->push_nt) {
        if (B == 64) return launch_push32_t<64, 1>(h);
        if (B == 128) return launch_push32_t<128, 1>(h);
        if (B == 256) return launch_push32_t<256, 1>(h);
        if (B == 512) return launch_push32_t<512, 1>(h);
    } else {
        if (B == 64) return launch_push32_t<64, 0>(h);
        if (B == 128) return launch_push32_t<128, 0>(h);
        if (B == 256) return launch_push32_t<256, 0>(h);
        if (B == 512) return launch_push32_t<512, 0>(h);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_weights32(pic_handle *h, int64_t *w_out)
{
    hipLaunchKernelGGL(k_weights32, dim3(h->n_cu * 8), dim3(256), 0, h->stream, h->c, streams_of(h, h->pbuf),
                       h->ws.ctr, (unsigned long long *)w_out);
    return hipGetLastError();
}

hipError_t launch_profile32(pic_handle *h, int nbins, const ProfPtrs &p)
{
    const Workspace &w = h->ws;
    hipLaunchKernelGGL(k_profile32, dim3(h->n_cu * 8), dim3(256), 0, h->stream, h->c, nbins, streams_of(h, h->pbuf),
                       w.ctr, ProfOut{p.cnt, p.lo, p.hi, p.mn, p.mx});
    return hipGetLastError();
}

// Blocks of a pass over both streams in tiles of SORT_TILE slots (sort_item).
static unsigned sort_items32(pic_handle *h) { return (unsigned)((h->c.cap + SORT_TILE - 1) / SORT_TILE + 1); }

hipError_t launch_sort32_hist(pic_handle *h)
{
    hipLaunchKernelGGL(k_hist32, dim3(sort_items32(h)), dim3(SORT_BLOCK), 0, h->stream, h->c, streams_of(h, h->pbuf),
                       h->ws.ctr, h->u_hi, (unsigned long long *)h->ws.cell_count);
    return hipGetLastError();
}

hipError_t launch_sort32_scatter(pic_handle *h)
{
    const int src = h->pbuf, dst = 1 - h->pbuf;
    hipLaunchKernelGGL(k_copy_total, dim3(1), dim3(64), 0, h->stream, (const long long *)(h->ws.cell_off + sort_low_keys(h->c)),
                       h->ws.total_lo);
    hipLaunchKernelGGL(k_scatter32, dim3(sort_items32(h)), dim3(SORT_BLOCK), 0, h->stream, h->c, streams_of(h, src),
                       streams_of(h, dst), h->ws.ctr, h->u_hi, (unsigned long long *)h->ws.cell_off,
                       (const long long *)h->ws.total_lo);
    hipLaunchKernelGGL(k_sort32_finish, dim3(1), dim3(64), 0, h->stream, h->ws.ctr,
                       (const long long *)(h->ws.total_lo));
    return hipGetLastError();
}

hipError_t launch_append_staged(pic_handle *h, int64_t n, bool check_only)
{
    const unsigned g = (unsigned)((n + 255) / 256);
    if (check_only) {
        hipLaunchKernelGGL(k_check_staged, dim3(g), dim3(256), 0, h->stream, h->c, h->ws.stage_x, h->ws.stage_u, n,
                           h->ws.ctr);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_stage_count, dim3(g), dim3(256), 0, h->stream, h->ws.stage_u, n, h->u_hi, h->ws.stage_blk);
    hipLaunchKernelGGL(k_stage_offsets, dim3(1), dim3(256), 0, h->stream, h->ws.stage_blk, (int64_t)g, n, h->ws.ctr,
                       h->ws.stage_base);
    hipLaunchKernelGGL(k_append_staged, dim3(g), dim3(256), 0, h->stream, h->c, h->ws.stage_x, h->ws.stage_u, n,
                       streams_of(h, h->pbuf), h->u_hi, (const long long *)h->ws.stage_blk,
                       (const long long *)h->ws.stage_base);
    return hipGetLastError();
}

}  // namespace pcpic
