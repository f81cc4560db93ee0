// k_batch.hip -- many independent tubes of uneven size stepped together.
//
// Each tube keeps the exact workspace layout of a single tube; a device table
// of TubeDev descriptors points at them.  A step of the whole batch is two
// kernels over a device work list, one block per item:
//   push  -- items = particle tiles of every tube (both streams in FP32-bulk
//            mode); the body is the single-tube push_tile_*;
//   field -- items = cell tiles of every tube; the body is the single-tube
//            field_tile, whose tile-0 block also injects.
// The kernel boundary orders the two phases, so no block ever waits for
// another and nothing depends on how many blocks are resident or on what else
// shares the GPU.  A round of up to sort_every steps plus the batched cell sort
// is captured once in a HIP graph and replayed with a single launch.  A tube
// therefore computes bit for bit what it computes when stepped alone.
#include <math.h>

#include "field_body.h"
#include "pcpic_internal.h"
#include "push_body.h"
#include "sort_body.h"
#include "wave.h"

namespace pcpic {

struct BatchArgs {
    const TubeDev *tubes;
    int n_tubes;
    int64_t *live_pref;          // [n_tubes + 1] prefix of the push items holding particles (k_batch_worklist)
    int64_t *live_counts;        // [2 n_tubes] slots of each tube's low and high stream (FP64: n, 0)
    int32_t *push_map;           // push item -> tube (k_batch_worklist)
    const int64_t *field_pref;   // [n_tubes + 1] prefix of cell tiles
    const int32_t *field_map;    // cell tile -> tube
    int fb, jb, pb;              // field, current and particle buffer parities of the step
    int hist;                    // the step before a sort: the push counts its survivors' sort keys
                                 // and the injection adds the injected particles' key
    int tile_lo, tile_hi;        // slots per push item: FP64 tiles (tile_lo = tile_hi), or the
                                 // FP32-bulk low- and high-stream tiles
};

// Push items of tube t that hold particles (FP64: ceil(n / tile); FP32-bulk:
// the low stream's tiles, then the high stream's).
__device__ __forceinline__ long long tube_items(const BatchArgs &b, int t, int64_t &n_lo, int64_t &n_hi)
{
    const DevCounters *ctr = generic(b.tubes[t].ctr);
    n_lo = ctr->n_slots;
    n_hi = ctr->n_slots_hi;
    return (n_lo + b.tile_lo - 1) / b.tile_lo + (n_hi + b.tile_hi - 1) / b.tile_hi;
}

// The push work list of the coming step, one block per tube t: the block sums
// the items of the tubes below t from their counters (every block recounts
// them; the counters sit in L2), writes the prefix live_pref[t + 1] and t's
// slot counts, and t's index over its items [live_pref[t], live_pref[t + 1])
// of push_map, so a push block finds its tube with one load.  It runs between
// the field update (which appends injected particles) or the sort and the
// next push, so the counts are final.  The push grid keeps its capacity-sized
// upper bound and every block past live_pref[n_tubes] returns at once: the
// idle blocks come last instead of between the tubes' tiles.
__global__ __launch_bounds__(256) void k_batch_worklist(BatchArgs b)
{
    __shared__ long long s_wave[4];
    const int t = blockIdx.x;
    int64_t n_lo, n_hi;
    long long below = 0;
    for (int s = (int)threadIdx.x; s < t; s += 256) below += tube_items(b, s, n_lo, n_hi);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) below += __shfl_xor(below, o);
    if ((threadIdx.x & 63) == 0) s_wave[threadIdx.x >> 6] = below;
    __syncthreads();
    below = s_wave[0] + s_wave[1] + s_wave[2] + s_wave[3];
    const long long mine = tube_items(b, t, n_lo, n_hi);
    if (threadIdx.x == 0) {
        if (t == 0) b.live_pref[0] = 0;
        b.live_pref[t + 1] = below + mine;
        b.live_counts[2 * t] = n_lo;
        b.live_counts[2 * t + 1] = n_hi;
    }
    for (long long it = below + threadIdx.x; it < below + mine; it += 256) b.push_map[it] = t;
}

template <int BLOCK, int PPT, int NT, int F32>
__global__ __launch_bounds__(BLOCK) void k_batch_push(BatchArgs b)
{
    constexpr int TILE = BLOCK * (F32 ? F32_PPT_LO : PPT);
    const int64_t it = blockIdx.x;
    if (it >= b.live_pref[b.n_tubes]) return;
    {
        const int t = b.push_map[it];
        const TubeDev &T = b.tubes[t];
        // the descriptor and the slot counts are read once, before any store, into registers
        const Consts c = T.c;
        const int64_t local = it - b.live_pref[t];
        const int64_t n_lo = b.live_counts[2 * t], n_hi = b.live_counts[2 * t + 1];
        if (F32) {
            Push32Args a{generic(T.cl[b.pb]), generic(T.ol[b.pb]), generic(T.ul[b.pb]), generic(T.hp[b.pb]),
                         generic(T.hw[b.pb]), generic(T.hg[b.pb]), generic(T.uh[b.pb]), generic(T.k32),
                         generic(T.ez[b.fb]),
                         (unsigned long long *)generic(T.j[b.jb]), generic(T.ctr),
                         b.hist ? (unsigned long long *)generic(T.cell_count) : nullptr, T.u_hi};
            push_item_f32<BLOCK, NT>(c, a, local, n_lo, n_hi);
        } else {
            const int64_t tile0 = local * TILE;
            const int64_t n = n_lo;
            if (tile0 >= n) return;
            PushArgs a{generic(T.x[b.pb]), generic(T.u[b.pb]), generic(T.x[b.pb]), generic(T.u[b.pb]),
                       generic(T.ez[b.fb]), (unsigned long long *)generic(T.j[b.jb]), generic(T.ctr),
                       b.hist ? (unsigned long long *)generic(T.cell_count) : nullptr};
            push_tile_f64<BLOCK, PPT, NT>(c, a, n, tile0);
        }
    }
}

template <int BLOCK, int F32>
__global__ __launch_bounds__(BLOCK) void k_batch_field(BatchArgs b)
{
    const int fb = b.fb, g = b.fb ^ 1, jb = b.jb, pb = b.pb;
    const int64_t it = blockIdx.x;
    if (it >= b.field_pref[b.n_tubes]) return;
    {
        const int t = b.field_map[it];
        const TubeDev &T = b.tubes[t];
        const Consts c = T.c;
        const int64_t local = it - b.field_pref[t];
        FieldArgs a{generic(T.ez[fb]), generic(T.er[fb]), generic(T.b[fb]), generic(T.ez[g]), generic(T.er[g]),
                    generic(T.b[g]), generic(T.j[jb]), generic(T.j[jb ^ 1]), F32 ? generic(T.k32) : nullptr, F32 ? nullptr : generic(T.x[pb]),
                    F32 ? nullptr : generic(T.u[pb]), F32 ? generic(T.cl[pb]) : nullptr,
                    F32 ? generic(T.ol[pb]) : nullptr, F32 ? generic(T.ul[pb]) : nullptr, generic(T.ctr),
                    nullptr, 0, 0, b.hist ? (unsigned long long *)generic(T.cell_count) : nullptr,
                    (F32 && 0.0 >= T.u_hi) ? sort_low_keys(c) : 0};
        field_tile(c, a, local, BLOCK);
    }
}

// ------------------------------------------------------------------------
// batched counting sort (per tube: histogram -> scan -> scatter -> finish)
// ------------------------------------------------------------------------

struct BSortArgs {
    const TubeDev *tubes;
    int n_tubes;
    const int64_t *chunk_pref;   // [n_tubes + 1] prefix of sort items (tiles of SORT_TILE slots, sort_item)
    const int64_t *key_pref;     // [n_tubes + 1] prefix of sort keys
    const int64_t *scan_pref;    // [n_tubes + 1] prefix of scan blocks
    const int32_t *chunk_map;    // sort chunk -> tube
    const int32_t *scan_map;     // scan block -> tube
    int f32;
    int src, dst;                // particle buffer parity before / after
};

// One block per scan block of SORT_SCAN_TILE keys (a block never spans two tubes).
__global__ __launch_bounds__(256) void k_bsort_clear(BSortArgs a)
{
    const int t = a.scan_map[blockIdx.x];
    const TubeDev &T = a.tubes[t];
    const int64_t base = (blockIdx.x - a.scan_pref[t]) * SORT_SCAN_TILE;
#pragma unroll
    for (int k = 0; k < SORT_SCAN_TILE / 256; ++k) {
        const int64_t i = base + k * 256 + threadIdx.x;
        if (i < T.n_keys) T.cell_count[i] = 0;
    }
}

// A tube's particle streams of buffer parity b.
__device__ __forceinline__ Streams tube_streams(const TubeDev &T, int b)
{
    return Streams{generic(T.cl[b]), generic(T.ol[b]), generic(T.ul[b]), generic(T.hp[b]), generic(T.hw[b]),
                   generic(T.hg[b]), generic(T.uh[b])};
}

// One block per sort item (a tile of SORT_TILE slots of one stream) of a tube.
__global__ __launch_bounds__(SORT_BLOCK) void k_bsort_hist(BSortArgs a)
{
    const int64_t it = blockIdx.x;
    const int t = a.chunk_map[it];
    const TubeDev &T = a.tubes[t];
    const Consts c = T.c;
    bool hi;
    int64_t tile0, n;
    if (!sort_item(it - a.chunk_pref[t], a.f32 != 0, generic(T.ctr), hi, tile0, n)) return;
    hist_tile(c, a.f32 != 0, hi, generic(T.x[a.src]), tube_streams(T, a.src), T.u_hi,
              (unsigned long long *)generic(T.cell_count), n, tile0);
}

// Exclusive scan of every tube's key counts in three phases over blocks of
// SORT_SCAN_TILE keys (a block never spans two tubes): block totals, a scan of
// each tube's block totals (one block per tube), then the offsets.
__global__ __launch_bounds__(256) void k_bscan_totals(BSortArgs a)
{
    __shared__ long long s_wave[4];
    const int t = a.scan_map[blockIdx.x];
    const TubeDev &T = a.tubes[t];
    const int64_t lb = blockIdx.x - a.scan_pref[t];
    const int64_t base = lb * SORT_SCAN_TILE + (int64_t)threadIdx.x * 4;
    long long s = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) s += base + k < T.n_keys ? T.cell_count[base + k] : 0;
    const long long inc = block_scan_incl(s, s_wave);
    if (threadIdx.x == 255) T.blk_sum[lb] = inc;
}

__global__ __launch_bounds__(256) void k_bscan_blocks(BSortArgs a)
{
    __shared__ long long s_wave[4];
    __shared__ long long s_carry;
    const TubeDev &T = a.tubes[blockIdx.x];
    const int64_t nb = a.scan_pref[blockIdx.x + 1] - a.scan_pref[blockIdx.x];
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (int64_t b0 = 0; b0 < nb; b0 += 256) {
        const int64_t i = b0 + threadIdx.x;
        const long long v = i < nb ? T.blk_sum[i] : 0;
        const long long inc = block_scan_incl(v, s_wave);
        const long long carry = s_carry;
        if (i < nb) T.blk_sum[i] = carry + inc - v;
        __syncthreads();
        if (threadIdx.x == 255) s_carry = carry + inc;
        __syncthreads();
    }
    if (threadIdx.x == 0) T.ctr->n_alive = s_carry;
}

__global__ __launch_bounds__(256) void k_bscan_apply(BSortArgs a)
{
    __shared__ long long s_wave[4];
    const int t = a.scan_map[blockIdx.x];
    const TubeDev &T = a.tubes[t];
    const int64_t lb = blockIdx.x - a.scan_pref[t];
    const int64_t base = lb * SORT_SCAN_TILE + (int64_t)threadIdx.x * 4;
    long long v[4];
    long long s = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        v[k] = base + k < T.n_keys ? T.cell_count[base + k] : 0;
        s += v[k];
    }
    const long long inc = block_scan_incl(s, s_wave);
    long long run = T.blk_sum[lb] + inc - s;
    const int64_t klo = a.f32 ? sort_low_keys(T.c) : -1;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (base + k < T.n_keys) {
            T.cell_off[base + k] = run;
            if (base + k == klo) *T.total_lo = run;   // slots of the low destination stream
        }
        run += v[k];
    }
}

__global__ __launch_bounds__(SORT_BLOCK) void k_bsort_scatter(BSortArgs a)
{
    const int64_t it = blockIdx.x;
    const int t = a.chunk_map[it];
    const TubeDev &T = a.tubes[t];
    const Consts c = T.c;
    bool hi;
    int64_t tile0, n;
    if (!sort_item(it - a.chunk_pref[t], a.f32 != 0, generic(T.ctr), hi, tile0, n)) return;
    unsigned long long *off = (unsigned long long *)generic(T.cell_off);
    if (a.f32) {
        const int64_t tlo = *T.total_lo;
        if (hi)
            scatter_tile_f32<true>(c, tube_streams(T, a.src), tube_streams(T, a.dst), T.u_hi, tlo, off, n, tile0);
        else
            scatter_tile_f32<false>(c, tube_streams(T, a.src), tube_streams(T, a.dst), T.u_hi, tlo, off, n, tile0);
    } else {
        scatter_tile_f64(c, generic(T.x[a.src]), generic(T.u[a.src]), generic(T.x[a.dst]), generic(T.u[a.dst]), off,
                         n, tile0);
    }
}

__global__ __launch_bounds__(64) void k_bsort_finish(BSortArgs a)
{
    const int t = blockIdx.x * 64 + threadIdx.x;
    if (t >= a.n_tubes) return;
    const TubeDev &T = a.tubes[t];
    if (a.f32) {
        const long long lo = *T.total_lo;
        T.ctr->n_slots_hi = T.ctr->n_alive - lo;
        T.ctr->n_slots = lo;
    } else {
        T.ctr->n_slots = T.ctr->n_alive;
    }
    T.ctr->n_removed = 0;
}

// ------------------------------------------------------------------------
// host side
// ------------------------------------------------------------------------

TubeDev tube_dev(pic_handle *t)
{
    TubeDev d{};
    const Workspace &w = t->ws;
    d.c = t->c;
    for (int k = 0; k < 2; ++k) {
        d.x[k] = to_global(w.x[k]);
        d.u[k] = to_global(w.u[k]);
        d.cl[k] = to_global(w.cl[k]);
        d.ol[k] = to_global(w.ol[k]);
        d.ul[k] = to_global(w.ul[k]);
        d.hp[k] = to_global(w.hp[k]);
        d.hw[k] = to_global(w.hw[k]);
        d.hg[k] = to_global(w.hg[k]);
        d.uh[k] = to_global(w.uh[k]);
        d.ez[k] = to_global(w.ez[k]);
        d.er[k] = to_global(w.er[k]);
        d.b[k] = to_global(w.b[k]);
        d.j[k] = to_global(w.j[k]);
    }
    d.k32 = to_global(w.k32);
    d.ctr = to_global(w.ctr);
    d.cell_count = to_global(w.cell_count);
    d.cell_off = to_global(w.cell_off);
    d.total_lo = to_global(w.total_lo);
    d.blk_sum = to_global(w.blk_sum);
    d.rhs = to_global(w.rhs);
    d.cp = to_global(w.cp);
    d.dp = to_global(w.dp);
    d.phi = to_global(w.phi);
    d.u_hi = t->u_hi;
    d.sort_chunks = (t->c.cap + SORT_TILE - 1) / SORT_TILE;
    d.n_keys = sort_key_count(t->c, t->p.precision == PIC_FP32_BULK);
    return d;
}

template <int BLOCK, int PPT, int NT, int F32>
static const void *push_kernel()
{
    return reinterpret_cast<const void *>(&k_batch_push<BLOCK, PPT, NT, F32>);
}

template <int BLOCK, int F32>
static const void *field_kernel()
{
    return reinterpret_cast<const void *>(&k_batch_field<BLOCK, F32>);
}

static const void *pick_push_kernel(pic_handle *h)
{
    const bool f32 = h->tubes[0]->p.precision == PIC_FP32_BULK;
    const int B = h->batch_block, P = h->batch_ppt;
    if (f32) {
        if (B == 64) return push_kernel<64, 4, 1, 1>();
        if (B == 128) return push_kernel<128, 4, 1, 1>();
        if (B == 256) return push_kernel<256, 4, 1, 1>();
        if (B == 512) return push_kernel<512, 4, 1, 1>();
    } else {
        if (B == 64 && P == 2) return push_kernel<64, 2, 1, 0>();
        if (B == 128 && P == 2) return push_kernel<128, 2, 1, 0>();
        if (B == 256 && P == 2) return push_kernel<256, 2, 1, 0>();
        if (B == 512 && P == 2) return push_kernel<512, 2, 1, 0>();
        if (B == 64 && P == 4) return push_kernel<64, 4, 1, 0>();
        if (B == 128 && P == 4) return push_kernel<128, 4, 1, 0>();
        if (B == 256 && P == 4) return push_kernel<256, 4, 1, 0>();
    }
    return nullptr;
}

static const void *pick_field_kernel(pic_handle *h)
{
    const bool f32 = h->tubes[0]->p.precision == PIC_FP32_BULK;
    switch (h->batch_block) {
    case 64: return f32 ? field_kernel<64, 1>() : field_kernel<64, 0>();
    case 128: return f32 ? field_kernel<128, 1>() : field_kernel<128, 0>();
    case 256: return f32 ? field_kernel<256, 1>() : field_kernel<256, 0>();
    case 512: return f32 ? field_kernel<512, 1>() : field_kernel<512, 0>();
    default: return nullptr;
    }
}

bool batch_shape_supported(pic_handle *h) { return pick_push_kernel(h) && pick_field_kernel(h); }

static BSortArgs bsort_args(pic_handle *h)
{
    pic_handle *t0 = h->tubes[0];
    return BSortArgs{h->d_tubes, (int)h->tubes.size(), h->d_sort_pref, h->d_key_pref, h->d_scan_pref,
                     h->d_chunk_map, h->d_scan_map, t0->p.precision == PIC_FP32_BULK ? 1 : 0, t0->pbuf,
                     1 - t0->pbuf};
}

// nsteps steps of every tube: the work-list, push and field kernels per step.
// With hist_last, the key counts are cleared first and the last step's push
// counts the sort keys of its survivors (the sort that follows skips its
// histogram).  With ev (timed runs), four events per step are recorded around
// the work-list, push and field kernels (ev[4s] .. ev[4s + 3], created by the
// caller).
hipError_t launch_batch_steps(pic_handle *h, int nsteps, bool hist_last, hipEvent_t *ev)
{
    const void *kp = pick_push_kernel(h);
    const void *kf = pick_field_kernel(h);
    if (!kp || !kf || h->batch_push_items <= 0 || h->batch_field_items <= 0 ||
        h->batch_push_items > 0x7fffffff || h->batch_field_items > 0x7fffffff || h->batch_push_items > h->push_map_cap)
        return hipErrorInvalidValue;
    pic_handle *t0 = h->tubes[0];
    const unsigned pgrid = (unsigned)h->batch_push_items, fgrid = (unsigned)h->batch_field_items;
    if (hist_last) {
        if (h->batch_scan_blocks <= 0 || h->batch_scan_blocks > 0x7fffffff) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_bsort_clear, dim3((unsigned)h->batch_scan_blocks), dim3(256), 0, h->stream,
                           bsort_args(h));
    }
    const bool f32 = t0->p.precision == PIC_FP32_BULK;
    for (int s = 0; s < nsteps; ++s) {
        BatchArgs a{h->d_tubes, (int)h->tubes.size(), h->d_live_pref, h->d_live_counts, h->d_push_map,
                    h->d_field_pref, h->d_field_map,
                    t0->fbuf ^ (s & 1), t0->jbuf ^ (s & 1), t0->pbuf, (hist_last && s == nsteps - 1) ? 1 : 0,
                    h->batch_block * (f32 ? F32_PPT_LO : h->batch_ppt),
                    h->batch_block * (f32 ? F32_PPT_HI : h->batch_ppt)};
        void *args[] = {&a};
        hipError_t e = ev ? hipEventRecord(ev[4 * s], h->stream) : hipSuccess;
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_batch_worklist, dim3((unsigned)h->tubes.size()), dim3(256), 0, h->stream, a);
        if (ev && (e = hipEventRecord(ev[4 * s + 1], h->stream)) != hipSuccess) return e;
        e = hipLaunchKernel(kp, dim3(pgrid), dim3(h->batch_block), args, 0, h->stream);
        if (e != hipSuccess) return e;
        if (ev && (e = hipEventRecord(ev[4 * s + 2], h->stream)) != hipSuccess) return e;
        e = hipLaunchKernel(kf, dim3(fgrid), dim3(h->batch_block), args, 0, h->stream);
        if (e != hipSuccess) return e;
        if (ev && (e = hipEventRecord(ev[4 * s + 3], h->stream)) != hipSuccess) return e;
    }
    return hipSuccess;
}

// The batched sort; hist_ready: the key counts were taken by the last push.
hipError_t launch_batch_sort(pic_handle *h, bool hist_ready)
{
    const int nt = (int)h->tubes.size();
    const BSortArgs a = bsort_args(h);
    if (h->batch_scan_blocks <= 0 || h->batch_scan_blocks > 0x7fffffff) return hipErrorInvalidValue;
    const unsigned sb = (unsigned)h->batch_scan_blocks;
    if (h->batch_sort_items <= 0 || h->batch_sort_items > 0x7fffffff) return hipErrorInvalidValue;
    const unsigned g = (unsigned)h->batch_sort_items;   // one block per sort item
    if (!hist_ready) {
        hipLaunchKernelGGL(k_bsort_clear, dim3(sb), dim3(256), 0, h->stream, a);
        hipLaunchKernelGGL(k_bsort_hist, dim3(g), dim3(SORT_BLOCK), 0, h->stream, a);
    }
    hipLaunchKernelGGL(k_bscan_totals, dim3(sb), dim3(256), 0, h->stream, a);
    hipLaunchKernelGGL(k_bscan_blocks, dim3(nt), dim3(256), 0, h->stream, a);
    hipLaunchKernelGGL(k_bscan_apply, dim3(sb), dim3(256), 0, h->stream, a);
    hipLaunchKernelGGL(k_bsort_scatter, dim3(g), dim3(SORT_BLOCK), 0, h->stream, a);
    hipLaunchKernelGGL(k_bsort_finish, dim3((nt + 63) / 64), dim3(64), 0, h->stream, a);
    return hipGetLastError();
}

}  // namespace pcpic
