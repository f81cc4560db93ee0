// k_batch.hip -- many independent tubes of uneven size stepped together.
//
// Each tube keeps the exact workspace layout of a single tube; a device table
// of TubeDev descriptors points at them.  A step of the whole batch is two
// kernels, each a fixed grid of resident blocks that walks a device work list:
//   push  -- items = runs of particle tiles of one tube (both streams in
//            FP32-bulk mode); the body is the single-tube push_tile_*;
//   field -- items = runs of cell tiles of one tube; the body is the
//            single-tube field_tile, whose tile-0 block also injects.
// The kernel boundary orders the two phases, so no block ever waits for
// another and nothing depends on how many blocks are resident or on what else
// shares the GPU.  A round of up to sort_every steps plus the batched cell sort
// is captured once in a HIP graph and replayed with a single launch.  A tube
// therefore computes bit for bit what it computes when stepped alone.
#include <math.h>

#include "field_body.h"
#include "pcpic_internal.h"
#include "push_body.h"
#include "wave.h"

namespace pcpic {

struct BatchArgs {
    const TubeDev *tubes;
    int n_tubes;
    const int64_t *push_pref;    // [n_tubes + 1] prefix of push work items
    const int64_t *field_pref;   // [n_tubes + 1] prefix of field work items
    int64_t push_chunk;          // particle tiles per push item
    int64_t field_chunk;         // cell tiles per field item
    int fb, jb, pb;              // field, current and particle buffer parities of the step
};

// Last t with pref[t] <= item (pref is non-decreasing, pref[0] = 0).
__device__ __forceinline__ int find_tube(const int64_t *pref, int n, int64_t item)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pref[mid] <= item) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int BLOCK, int PPT, int NT, int F32>
__global__ __launch_bounds__(BLOCK) void k_batch_push(BatchArgs b)
{
    constexpr int TILE = BLOCK * (F32 ? 4 : PPT);
    const int64_t ptot = b.push_pref[b.n_tubes];
    for (int64_t it = blockIdx.x; it < ptot; it += gridDim.x) {
        const int t = find_tube(b.push_pref, b.n_tubes, it);
        const TubeDev &T = b.tubes[t];
        const int64_t local = it - b.push_pref[t];
        const int64_t per = (T.push_tiles + b.push_chunk - 1) / b.push_chunk;   // items per stream
        const bool hi = F32 && local >= per;
        const int64_t c0 = (hi ? local - per : local) * b.push_chunk;
        const int64_t c1 = c0 + b.push_chunk < T.push_tiles ? c0 + b.push_chunk : T.push_tiles;
        if (F32) {
            const int64_t n = hi ? T.ctr->n_slots_hi : T.ctr->n_slots;
            Push32Args a{T.cl[b.pb], T.ol[b.pb], T.ul[b.pb], T.ch[b.pb], T.oh[b.pb], T.uh[b.pb], T.k32, T.k64,
                         (unsigned long long *)T.j[b.jb], T.ctr, 0u};
            for (int64_t tl = c0; tl < c1 && tl * TILE < n; ++tl) push_tile_f32<BLOCK, NT>(T.c, a, hi, n, tl * TILE);
        } else {
            const int64_t n = T.ctr->n_slots;
            PushArgs a{T.x[b.pb], T.u[b.pb], T.x[b.pb], T.u[b.pb], T.k64, (unsigned long long *)T.j[b.jb], T.ctr};
            for (int64_t tl = c0; tl < c1 && tl * TILE < n; ++tl) push_tile_f64<BLOCK, PPT, NT>(T.c, a, n, tl * TILE);
        }
    }
}

template <int BLOCK, int F32>
__global__ __launch_bounds__(BLOCK) void k_batch_field(BatchArgs b)
{
    const int64_t ftot = b.field_pref[b.n_tubes];
    const int fb = b.fb, g = b.fb ^ 1, jb = b.jb, pb = b.pb;
    for (int64_t it = blockIdx.x; it < ftot; it += gridDim.x) {
        const int t = find_tube(b.field_pref, b.n_tubes, it);
        const TubeDev &T = b.tubes[t];
        const int64_t local = it - b.field_pref[t];
        const int64_t ftiles = (T.c.N + BLOCK - 1) / BLOCK;
        const int64_t c0 = local * b.field_chunk;
        const int64_t c1 = c0 + b.field_chunk < ftiles ? c0 + b.field_chunk : ftiles;
        FieldArgs a{T.ez[fb], T.er[fb], T.b[fb], T.ez[g], T.er[g], T.b[g], T.j[jb], T.j[jb ^ 1],
                    T.k64, F32 ? T.k32 : nullptr, F32 ? nullptr : T.x[pb], F32 ? nullptr : T.u[pb],
                    F32 ? T.cl[pb] : nullptr, F32 ? T.ol[pb] : nullptr, F32 ? T.ul[pb] : nullptr, T.ctr};
        for (int64_t tl = c0; tl < c1; ++tl) field_tile(T.c, a, tl, BLOCK);
    }
}

// ------------------------------------------------------------------------
// batched counting sort (per tube: histogram -> scan -> scatter -> finish)
// ------------------------------------------------------------------------

struct BSortArgs {
    const TubeDev *tubes;
    int n_tubes;
    const int64_t *chunk_pref;   // [n_tubes + 1] prefix of 256-slot chunks (both streams)
    const int64_t *key_pref;     // [n_tubes + 1] prefix of sort keys
    int f32;
    int src, dst;                // particle buffer parity before / after
};

__global__ __launch_bounds__(256) void k_bsort_clear(BSortArgs a)
{
    const int64_t total = a.key_pref[a.n_tubes];
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
        const int t = find_tube(a.key_pref, a.n_tubes, i);
        a.tubes[t].cell_count[i - a.key_pref[t]] = 0;
    }
}

// Slot p of the chunk item, its stream and the stream's slot count.
__device__ __forceinline__ bool chunk_slot(const TubeDev &T, int f32, int64_t local, int64_t &p, int64_t &n)
{
    const bool hi = f32 && local >= T.sort_chunks;
    p = (hi ? local - T.sort_chunks : local) * 256 + threadIdx.x;
    n = hi ? T.ctr->n_slots_hi : T.ctr->n_slots;
    return hi;
}

__global__ __launch_bounds__(256) void k_bsort_hist(BSortArgs a)
{
    const int64_t total = a.chunk_pref[a.n_tubes];
    for (int64_t it = blockIdx.x; it < total; it += gridDim.x) {
        const int t = find_tube(a.chunk_pref, a.n_tubes, it);
        const TubeDev &T = a.tubes[t];
        int64_t p, n;
        const bool hi = chunk_slot(T, a.f32, it - a.chunk_pref[t], p, n);
        bool live = false;
        int64_t key = 0;
        if (p < n) {
            if (a.f32) {
                const int cell = hi ? T.ch[a.src][p] : T.cl[a.src][p];
                if (cell >= 0) {
                    const double u = hi ? T.uh[a.src][p] : (double)T.ul[a.src][p];
                    live = true;
                    key = sort_key_f32(T.c, cell, hi ? T.oh[a.src][p] : T.ol[a.src][p], fabs(u) >= T.u_hi);
                }
            } else {
                const double x = T.x[a.src][p];
                if (x >= 0.0) {
                    live = true;
                    key = sort_key_f64(T.c, x);
                }
            }
        }
        wave_add_keyed((unsigned long long *)T.cell_count, key, 1, live);
    }
}

// One block per tube: exclusive scan of its keys in chunks of 256.
__global__ __launch_bounds__(256) void k_bsort_scan(BSortArgs a)
{
    __shared__ long long s_wave[4];
    __shared__ long long s_carry;
    const TubeDev &T = a.tubes[blockIdx.x];
    const int64_t nk = T.n_keys;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    const int lane = __lane_id(), wv = threadIdx.x >> 6;
    for (int64_t k0 = 0; k0 < nk; k0 += 256) {
        const int64_t k = k0 + threadIdx.x;
        const long long v = k < nk ? T.cell_count[k] : 0;
        long long inc = v;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const long long o = __shfl_up(inc, off);
            if (lane >= off) inc += o;
        }
        if (lane == 63) s_wave[wv] = inc;
        __syncthreads();
        long long add = s_carry;
        for (int q = 0; q < wv; ++q) add += s_wave[q];
        if (k < nk) T.cell_off[k] = add + inc - v;
        __syncthreads();
        if (threadIdx.x == 255) s_carry = add + inc;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        T.ctr->n_alive = s_carry;
        if (a.f32) *T.total_lo = T.cell_off[sort_low_keys(T.c)];
    }
}

__global__ __launch_bounds__(256) void k_bsort_scatter(BSortArgs a)
{
    const int64_t total = a.chunk_pref[a.n_tubes];
    const int lane = __lane_id();
    for (int64_t it = blockIdx.x; it < total; it += gridDim.x) {
        const int t = find_tube(a.chunk_pref, a.n_tubes, it);
        const TubeDev &T = a.tubes[t];
        int64_t p, n;
        const bool hi = chunk_slot(T, a.f32, it - a.chunk_pref[t], p, n);
        bool want = false;
        int64_t key = 0;
        int cell = 0;
        float o = 0.0f;
        double x = 0.0, u = 0.0;
        if (p < n) {
            if (a.f32) {
                cell = hi ? T.ch[a.src][p] : T.cl[a.src][p];
                if (cell >= 0) {
                    o = hi ? T.oh[a.src][p] : T.ol[a.src][p];
                    u = hi ? T.uh[a.src][p] : (double)T.ul[a.src][p];
                    want = true;
                    key = sort_key_f32(T.c, cell, o, fabs(u) >= T.u_hi);
                }
            } else {
                x = T.x[a.src][p];
                if (x >= 0.0) {
                    u = T.u[a.src][p];
                    want = true;
                    key = sort_key_f64(T.c, x);
                }
            }
        }
        const long long tlo = a.f32 ? *T.total_lo : 0;
        unsigned long long pend = __ballot(want);
        while (pend) {
            const int leader = __ffsll(pend) - 1;
            const int64_t lk = __shfl(key, leader);
            const bool mine = want && key == lk;
            const unsigned long long grp = __ballot(mine);
            unsigned long long f0 = 0;
            if (lane == leader) f0 = atomicAdd((unsigned long long *)T.cell_off + lk, (unsigned long long)__popcll(grp));
            f0 = __shfl(f0, leader);
            if (mine) {
                const int64_t d = (int64_t)f0 + __popcll(grp & ((1ull << lane) - 1ull));
                if (a.f32) {
                    if (key >= sort_low_keys(T.c)) {
                        const int64_t q = d - tlo;
                        T.ch[a.dst][q] = cell;
                        T.oh[a.dst][q] = o;
                        T.uh[a.dst][q] = u;
                    } else {
                        T.cl[a.dst][d] = cell;
                        T.ol[a.dst][d] = o;
                        T.ul[a.dst][d] = (float)u;
                    }
                } else {
                    T.x[a.dst][d] = x;
                    T.u[a.dst][d] = u;
                }
            }
            pend &= ~grp;
            want = want && !mine;
        }
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
        d.x[k] = w.x[k];
        d.u[k] = w.u[k];
        d.cl[k] = w.cl[k];
        d.ol[k] = w.ol[k];
        d.ul[k] = w.ul[k];
        d.ch[k] = w.ch[k];
        d.oh[k] = w.oh[k];
        d.uh[k] = w.uh[k];
        d.ez[k] = w.ez[k];
        d.er[k] = w.er[k];
        d.b[k] = w.b[k];
        d.j[k] = w.j[k];
    }
    d.k64 = w.k64;
    d.k32 = w.k32;
    d.ctr = w.ctr;
    d.cell_count = w.cell_count;
    d.cell_off = w.cell_off;
    d.total_lo = w.total_lo;
    d.u_hi = t->u_hi;
    d.sort_chunks = (t->c.cap + 255) / 256;
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

// Resident blocks per CU of the push kernel for the current shape (0 = unsupported).
int batch_occupancy(pic_handle *h)
{
    const void *k = pick_push_kernel(h);
    const void *kf = pick_field_kernel(h);
    if (!k || !kf) return 0;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, h->batch_block, 0) != hipSuccess) return 0;
    return per_cu;
}

// nsteps steps of every tube: a push and a field kernel per step.
hipError_t launch_batch_steps(pic_handle *h, int nsteps)
{
    const void *kp = pick_push_kernel(h);
    const void *kf = pick_field_kernel(h);
    if (!kp || !kf || h->batch_grid <= 0) return hipErrorInvalidValue;
    pic_handle *t0 = h->tubes[0];
    const int64_t fitems = h->batch_field_items;
    const unsigned fgrid = (unsigned)(fitems < h->batch_grid ? fitems : h->batch_grid);
    for (int s = 0; s < nsteps; ++s) {
        BatchArgs a{h->d_tubes, (int)h->tubes.size(), h->d_push_pref, h->d_field_pref, h->batch_push_chunk,
                    h->batch_field_chunk, t0->fbuf ^ (s & 1), t0->jbuf ^ (s & 1), t0->pbuf};
        void *args[] = {&a};
        hipError_t e = hipLaunchKernel(kp, dim3(h->batch_grid), dim3(h->batch_block), args, 0, h->stream);
        if (e != hipSuccess) return e;
        e = hipLaunchKernel(kf, dim3(fgrid > 0 ? fgrid : 1), dim3(h->batch_block), args, 0, h->stream);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_batch_sort(pic_handle *h)
{
    pic_handle *t0 = h->tubes[0];
    const int nt = (int)h->tubes.size();
    BSortArgs a{h->d_tubes, nt, h->d_sort_pref, h->d_key_pref, t0->p.precision == PIC_FP32_BULK ? 1 : 0,
                t0->pbuf, 1 - t0->pbuf};
    const unsigned g = (unsigned)(h->n_cu * 8);
    hipLaunchKernelGGL(k_bsort_clear, dim3(g), dim3(256), 0, h->stream, a);
    hipLaunchKernelGGL(k_bsort_hist, dim3(g), dim3(256), 0, h->stream, a);
    hipLaunchKernelGGL(k_bsort_scan, dim3(nt), dim3(256), 0, h->stream, a);
    hipLaunchKernelGGL(k_bsort_scatter, dim3(g), dim3(256), 0, h->stream, a);
    hipLaunchKernelGGL(k_bsort_finish, dim3((nt + 63) / 64), dim3(64), 0, h->stream, a);
    return hipGetLastError();
}

}  // namespace pcpic
