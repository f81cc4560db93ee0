// k_push.hip -- the particle half of the PIC cycle (sec. 2, Fig. A) in FP64:
// gather E_z at x^n, relativistic kick and move (eq. 1), charge-conserving
// linear current deposit in fixed point, removal at the tube ends, and the
// node-0 weight tally the SCLF injection needs.
//
// Layout and mapping: x and u are SoA FP64 streams (16 B read + 16 B written
// per live particle and step).  One block owns one tile of BLOCK*PPT
// consecutive slots and each thread PPT consecutive slots, loaded as 16-byte
// vectors.  Between cell sorts consecutive slots sit in the same cell, so a
// thread's current contributions land on three faces around the cell of its
// first particle and are summed in registers (DepAcc); one DPP reduction per
// wave and face group then issues a single int64 atomic per face.
#include <math.h>

#include "pcpic_internal.h"
#include "push_common.h"

namespace pcpic {

struct PushArgs {
    double *__restrict__ X;
    double *__restrict__ U;
    const double *__restrict__ K;
    unsigned long long *__restrict__ J;
    DevCounters *ctr;
};

template <int BLOCK, int PPT, int NT>
__global__ __launch_bounds__(BLOCK) void k_push_f64(Consts c, PushArgs a)
{
    const int64_t n = a.ctr->n_slots;
    constexpr int TILE = BLOCK * PPT;
    const int64_t tile0 = (int64_t)blockIdx.x * TILE;
    if (tile0 >= n) return;                       // whole block idle (uniform)
    const int N = (int)c.N;
    const double Nd = (double)c.N, Nm1 = (double)(c.N - 1);
    const int64_t p0 = tile0 + (int64_t)threadIdx.x * PPT;
    const bool full = p0 + PPT <= n;

    double xs[PPT], us[PPT];
    if (full) {
#pragma unroll
        for (int k = 0; k < PPT; k += 2) {
            const dvec2 xv = ld16<NT, dvec2>(a.X + p0 + k);
            const dvec2 uv = ld16<NT, dvec2>(a.U + p0 + k);
            xs[k] = xv.x; xs[k + 1] = xv.y;
            us[k] = uv.x; us[k + 1] = uv.y;
        }
    } else {
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            xs[k] = p0 + k < n ? a.X[p0 + k] : -1.0;
            us[k] = p0 + k < n ? a.U[p0 + k] : 0.0;
        }
    }

    DepAcc acc;
    acc.init();
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const double x = xs[k], u = us[k];
        if (!(x >= 0.0)) continue;               // removed slot (-1) or past the end
        // gather: linear interpolation between face values, clamped at the ends
        const double s = x - 0.5;
        const int jj = (int)floor(s);
        const double g = s - (double)jj;
        const int jc = jj < 0 ? 0 : (jj > N - 2 ? N - 2 : jj);
        const double k0 = a.K[jc], k1 = a.K[jc + 1];
        const double Ei = k0 + g * (k1 - k0);
        const double E = s < 0.0 ? k0 : (s >= Nm1 ? k1 : Ei);
        // eq. (1): u = gamma v, du/dt = (q/m) E_z, dz/dt = v
        const double u1 = u + E;
        double tt = u1 * u1;
        tt = 1.0 + tt;
        const double gam = sqrt(tt);
        const double v = u1 / gam;
        const double x1 = x + c.dtdz * v;
        if (!isfinite(u1) || !isfinite(x1)) {
            acc.bad = true;
            acc.nlost += 1.0;
            xs[k] = -1.0;
            continue;
        }
        const double c0d = floor(x);
        const double F0 = rint((x - c0d) * c.twoP);
        const double c1d = floor(x1);
        const int c1 = (int)c1d;
        const double F1 = rint((x1 - c1d) * c.twoP);
        acc.deposit(a.J, N, c.twoP, (int)c0d, F0, c1, F1);
        if (x1 >= Nd) {                          // leaves through z = L
            acc.exit_gamma(gam);
            xs[k] = -1.0;
        } else if (x1 < 0.0) {                   // returns to the star
            acc.nabs += 1.0;
            xs[k] = -1.0;
        } else {
            if (c1 == 0) acc.w0 += c.twoP - F1;
            xs[k] = x1;
            us[k] = u1;
        }
    }

    // write back (removed particles get x = -1; their u is left as it was)
    if (full) {
#pragma unroll
        for (int k = 0; k < PPT; k += 2) {
            st16<NT, dvec2>(a.X + p0 + k, dvec2{xs[k], xs[k + 1]});
            st16<NT, dvec2>(a.U + p0 + k, dvec2{us[k], us[k + 1]});
        }
    } else {
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            if (p0 + k < n) {
                a.X[p0 + k] = xs[k];
                a.U[p0 + k] = us[k];
            }
        }
    }
    acc.flush(a.J, a.ctr);
}

template <int BLOCK, int PPT, int NT>
static hipError_t launch_push_t(pic_handle *h)
{
    PushArgs a{h->ws.x[h->pbuf], h->ws.u[h->pbuf], h->ws.k64,
               (unsigned long long *)h->ws.j[h->jbuf], h->ws.ctr};
    const int64_t tile = (int64_t)BLOCK * PPT;
    const unsigned grid = (unsigned)((h->c.cap + tile - 1) / tile);
    hipLaunchKernelGGL((k_push_f64<BLOCK, PPT, NT>), dim3(grid), dim3(BLOCK), 0, h->stream, h->c, a);
    return hipGetLastError();
}

hipError_t launch_push_f64(pic_handle *h)
{
    const int B = h->push_block, P = h->push_ppt;
    if (h->push_nt) {
        if (B == 256 && P == 2) return launch_push_t<256, 2, 1>(h);
        if (B == 128 && P == 2) return launch_push_t<128, 2, 1>(h);
        if (B == 64 && P == 2) return launch_push_t<64, 2, 1>(h);
        if (B == 512 && P == 2) return launch_push_t<512, 2, 1>(h);
        if (B == 256 && P == 4) return launch_push_t<256, 4, 1>(h);
        if (B == 128 && P == 4) return launch_push_t<128, 4, 1>(h);
        if (B == 64 && P == 4) return launch_push_t<64, 4, 1>(h);
        return hipErrorInvalidValue;
    }
    if (B == 256 && P == 2) return launch_push_t<256, 2, 0>(h);
    if (B == 128 && P == 2) return launch_push_t<128, 2, 0>(h);
    if (B == 64 && P == 2) return launch_push_t<64, 2, 0>(h);
    if (B == 512 && P == 2) return launch_push_t<512, 2, 0>(h);
    if (B == 256 && P == 4) return launch_push_t<256, 4, 0>(h);
    if (B == 128 && P == 4) return launch_push_t<128, 4, 0>(h);
    if (B == 64 && P == 4) return launch_push_t<64, 4, 0>(h);
    return hipErrorInvalidValue;
}

}  // namespace pcpic
