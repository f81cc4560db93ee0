// k_push.hip -- the particle half of the PIC cycle (sec. 2, Fig. A) in FP64:
// gather E_z at x^n, relativistic kick and move (eq. 1), charge-conserving
// linear current deposit in fixed point, removal at the tube ends, and the
// node-0 weight tally the SCLF injection needs.
//
// Layout and mapping: x and u are SoA FP64 streams (16 B read + 16 B written
// per live particle and step).  One block owns one tile of BLOCK*PPT
// consecutive slots; each thread takes PPT/2 pairs of consecutive slots, a
// wave's pair v being 128 consecutive slots, each pair one 16-byte vector per
// stream.  Between cell sorts consecutive slots sit in the same cell, so a
// thread's current contributions land on the faces around the one or two
// cells of its pair and are summed in four register channels (DepAcc); per
// wave and pair the channels are summed (all four together for a wave in one
// cell, through a per-wave LDS window for a few cells, by segmented scans
// otherwise) into one int64 atomic per face.  The particle arithmetic is
// straight-line code with selects, so lanes that stay in their cell and lanes
// that cross a face share one instruction stream; the rare boundary events
// (exit, return, node-0 tally) are added by the lanes that have them.
#include <math.h>

#include "pcpic_internal.h"
#include "push_common.h"
#include "push_body.h"

namespace pcpic {

template <int BLOCK, int PPT, int NT, int GR = 0>
__global__ __launch_bounds__(BLOCK) void k_push_f64(Consts c, PushArgs a)
{
    const int64_t n = a.ctr->n_slots;
    const int64_t tile0 = (int64_t)blockIdx.x * (BLOCK * PPT);
    if (tile0 >= n) return;                       // whole block idle (uniform)
    push_tile_f64<BLOCK, PPT, NT, GR>(c, a, n, tile0);
}

template <int BLOCK, int PPT, int NT, int GR = 0>
static hipError_t launch_push_t(pic_handle *h)
{
    PushArgs a{h->ws.x[h->pbuf], h->ws.u[h->pbuf], h->ws.x[h->pbuf], h->ws.u[h->pbuf], h->ws.ez[h->fbuf],
               (unsigned long long *)h->ws.j[h->jbuf], h->ws.ctr,
               h->hist_on ? (unsigned long long *)h->ws.cell_count : nullptr};
    const int64_t tile = (int64_t)BLOCK * PPT;
    const unsigned grid = (unsigned)((h->c.cap + tile - 1) / tile);
    hipLaunchKernelGGL((k_push_f64<BLOCK, PPT, NT, GR>), dim3(grid), dim3(BLOCK), 0, h->stream, h->c, a);
    return hipGetLastError();
}

template <int BLOCK, int PPT, int NT>
static hipError_t launch_push_args_t(pic_handle *h, const PushArgs &a)
{
    const int64_t tile = (int64_t)BLOCK * PPT;
    const unsigned grid = (unsigned)((h->c.cap + tile - 1) / tile);
    hipLaunchKernelGGL((k_push_f64<BLOCK, PPT, NT>), dim3(grid), dim3(BLOCK), 0, h->stream, h->c, a);
    return hipGetLastError();
}

// FP64 push reading (X, U) and writing (Xo, Uo) in the field ez (used by the
// adjoint recompute), at the default launch shape.
hipError_t launch_push_f64_ptrs(pic_handle *h, const double *X, const double *U, double *Xo, double *Uo,
                                const double *ez)
{
    PushArgs a{X, U, Xo, Uo, ez, (unsigned long long *)h->ws.j[h->jbuf], h->ws.ctr};
    return launch_push_args_t<128, 2, 1>(h, a);
}

hipError_t launch_push_f64(pic_handle *h)
{
    // PIC_GR_ALPHA: one launch shape (the default), whatever the configured one
    if (h->c.flags & PIC_GR_ALPHA) return launch_push_t<128, 2, 1, 1>(h);
    const int B = h->push_block, P = h->push_ppt;
    if (h->push_nt) {
        if (B == 256 && P == 2) return launch_push_t<256, 2, 1>(h);
        if (B == 128 && P == 2) return launch_push_t<128, 2, 1>(h);
        if (B == 64 && P == 2) return launch_push_t<64, 2, 1>(h);
        if (B == 512 && P == 2) return launch_push_t<512, 2, 1>(h);
        if (B == 256 && P == 4) return launch_push_t<256, 4, 1>(h);
        if (B == 128 && P == 4) return launch_push_t<128, 4, 1>(h);
        if (B == 64 && P == 4) return launch_push_t<64, 4, 1>(h);
        if (B == 128 && P == 8) return launch_push_t<128, 8, 1>(h);
        if (B == 64 && P == 8) return launch_push_t<64, 8, 1>(h);
        return hipErrorInvalidValue;
    }
    if (B == 256 && P == 2) return launch_push_t<256, 2, 0>(h);
    if (B == 128 && P == 2) return launch_push_t<128, 2, 0>(h);
    if (B == 64 && P == 2) return launch_push_t<64, 2, 0>(h);
    if (B == 512 && P == 2) return launch_push_t<512, 2, 0>(h);
    if (B == 256 && P == 4) return launch_push_t<256, 4, 0>(h);
    if (B == 128 && P == 4) return launch_push_t<128, 4, 0>(h);
    if (B == 64 && P == 4) return launch_push_t<64, 4, 0>(h);
    if (B == 128 && P == 8) return launch_push_t<128, 8, 0>(h);
    if (B == 64 && P == 8) return launch_push_t<64, 8, 0>(h);
    return hipErrorInvalidValue;
}

}  // namespace pcpic
