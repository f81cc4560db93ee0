// k_sort.hip -- counting sort of the particles by cell, dropping removed slots.
//
// histogram (one atomic per distinct cell per wave) -> exclusive scan over the
// N cells -> scatter into the other particle buffer, lanes of a wave that
// share a cell taking consecutive slots.  Every step of the method is per
// particle or an integer reduction, so the order this produces (which varies
// from run to run between waves of the same cell) never changes a result.
#include <math.h>

#include "pcpic_internal.h"
#include "sort_body.h"
#include "wave.h"

namespace pcpic {

constexpr int SCAN_ITEMS = 4;
constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_TILE = SCAN_ITEMS * SCAN_BLOCK;   // keys per scan block
static_assert(SCAN_TILE == SORT_SCAN_TILE, "scan tile and workspace sizing differ");

__global__ __launch_bounds__(256) void k_fill_ll(long long *p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = 0;
}

__global__ __launch_bounds__(256) void k_hist(Consts c, const double *__restrict__ X, const DevCounters *ctr,
                                              long long *count)
{
    const int64_t n = ctr->n_slots;
    for (int64_t base = (int64_t)blockIdx.x * 256; base < n; base += (int64_t)gridDim.x * 256) {
        const int64_t p = base + threadIdx.x;
        const double x = p < n ? X[p] : -1.0;
        const bool live = x >= 0.0;
        const int64_t key = live ? sort_key_f64(c, x) : 0;
        const WaveRun r = wave_runs(key, live);
        if (live && r.is_head) atomicAdd((unsigned long long *)count + key, (unsigned long long)(r.end - (int)__lane_id()));
    }
}

// phase 1: per-block totals of SCAN_TILE cells
__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_totals(const long long *count, int64_t n, long long *blk)
{
    __shared__ long long s_wave[4];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    long long s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) s += (base + k < n) ? count[base + k] : 0;
    const long long inc = block_scan_incl(s, s_wave);
    if (threadIdx.x == SCAN_BLOCK - 1) blk[blockIdx.x] = inc;
}

// phase 2: exclusive scan of the block totals (one block, sequential chunks)
__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_blocks(long long *blk, int64_t nblk, DevCounters *ctr)
{
    __shared__ long long s_wave[4];
    __shared__ long long s_carry;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (int64_t b0 = 0; b0 < nblk; b0 += SCAN_BLOCK) {
        const int64_t i = b0 + threadIdx.x;
        const long long v = i < nblk ? blk[i] : 0;
        const long long inc = block_scan_incl(v, s_wave);
        const long long carry = s_carry;
        if (i < nblk) blk[i] = carry + inc - v;
        __syncthreads();
        if (threadIdx.x == SCAN_BLOCK - 1) s_carry = carry + inc;
        __syncthreads();
    }
    if (threadIdx.x == 0) ctr->n_alive = s_carry;
}

// phase 3: exclusive offsets per cell
__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_apply(const long long *count, int64_t n, const long long *blk,
                                                           long long *off)
{
    __shared__ long long s_wave[4];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    long long v[SCAN_ITEMS];
    long long s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        v[k] = (base + k < n) ? count[base + k] : 0;
        s += v[k];
    }
    const long long inc = block_scan_incl(s, s_wave);
    long long run = blk[blockIdx.x] + inc - s;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        if (base + k < n) off[base + k] = run;
        run += v[k];
    }
}

// Scatter into the other buffer, one block per tile of SORT_TILE slots.
__global__ __launch_bounds__(SORT_BLOCK) void k_scatter(Consts c, const double *__restrict__ X,
                                                        const double *__restrict__ U, double *__restrict__ Xo,
                                                        double *__restrict__ Uo, const DevCounters *ctr,
                                                        unsigned long long *off)
{
    const int64_t n = ctr->n_slots;
    const int64_t tile0 = (int64_t)blockIdx.x * SORT_TILE;
    if (tile0 >= n) return;
    scatter_tile_f64(c, X, U, Xo, Uo, off, n, tile0);
}

__global__ void k_sort_finish(DevCounters *ctr)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ctr->n_slots = ctr->n_alive;
        ctr->n_removed = 0;
    }
}

hipError_t launch_scan(pic_handle *h, int64_t n)
{
    Workspace &w = h->ws;
    const unsigned nblk = (unsigned)((n + SCAN_TILE - 1) / SCAN_TILE);
    hipLaunchKernelGGL(k_scan_totals, dim3(nblk), dim3(SCAN_BLOCK), 0, h->stream, w.cell_count, n, w.blk_sum);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(SCAN_BLOCK), 0, h->stream, w.blk_sum, (int64_t)nblk, w.ctr);
    hipLaunchKernelGGL(k_scan_apply, dim3(nblk), dim3(SCAN_BLOCK), 0, h->stream, w.cell_count, n, w.blk_sum,
                       w.cell_off);
    return hipGetLastError();
}

// Counting sort by cell into the other particle buffer, dropping removed slots;
// in FP32-bulk mode the destination stream follows the particle's gamma.
// Zero the key counts before a step that accumulates them (the step before a sort).
hipError_t launch_clear_hist(pic_handle *h)
{
    const int64_t nkeys = sort_key_count(h->c, h->p.precision == PIC_FP32_BULK);
    hipLaunchKernelGGL(k_fill_ll, dim3((unsigned)((nkeys + 255) / 256)), dim3(256), 0, h->stream, h->ws.cell_count,
                       nkeys);
    return hipGetLastError();
}

hipError_t launch_sort(pic_handle *h, bool hist_ready)
{
    const Consts &c = h->c;
    Workspace &w = h->ws;
    const bool f32 = h->p.precision == PIC_FP32_BULK;
    const int64_t nkeys = sort_key_count(c, f32);
    const int src = h->pbuf, dst = 1 - h->pbuf;
    hipError_t e;
    if (!hist_ready && (e = launch_clear_hist(h)) != hipSuccess) return e;
    if (f32) {
        if (!hist_ready && (e = launch_sort32_hist(h)) != hipSuccess) return e;
        if ((e = launch_scan(h, nkeys)) != hipSuccess) return e;
        if ((e = launch_sort32_scatter(h)) != hipSuccess) return e;
    } else {
        if (!hist_ready)
            hipLaunchKernelGGL(k_hist, dim3(h->n_cu * 8), dim3(256), 0, h->stream, c, w.x[src], w.ctr, w.cell_count);
        if ((e = launch_scan(h, nkeys)) != hipSuccess) return e;
        const unsigned tiles = (unsigned)((c.cap + SORT_TILE - 1) / SORT_TILE);
        hipLaunchKernelGGL(k_scatter, dim3(tiles), dim3(SORT_BLOCK), 0, h->stream, c, w.x[src], w.u[src], w.x[dst],
                           w.u[dst], w.ctr, (unsigned long long *)w.cell_off);
        hipLaunchKernelGGL(k_sort_finish, dim3(1), dim3(64), 0, h->stream, w.ctr);
    }
    h->pbuf = dst;
    return hipGetLastError();
}

}  // namespace pcpic
