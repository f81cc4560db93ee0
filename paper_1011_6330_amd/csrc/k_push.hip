// k_push.hip -- the particle half of the PIC cycle (sec. 2, Fig. A) in FP64:
// gather E_z at x^n, relativistic kick and move (eq. 1), charge-conserving
// linear current deposit in fixed point, removal at the tube ends, and the
// node-0 weight tally the SCLF injection needs.
//
// Memory: x and u are SoA FP64 streams, 16 B read + 16 B written per live
// particle and step; the kick array (8 B per face) is read through L2.  The
// current goes to an int64 array with one atomic per distinct face per wave
// (sorted particles share faces), so the sum is exact and order-free.
#include <math.h>

#include "pcpic_internal.h"
#include "wave.h"

namespace pcpic {

struct PushArgs {
    double *__restrict__ X;
    double *__restrict__ U;
    const double *__restrict__ K;
    unsigned long long *__restrict__ J;
    DevCounters *ctr;
};

// Logical block index that gives each XCD (blocks are dealt round-robin over
// 8 XCDs) a contiguous range of tiles, so an XCD's L2 sees nearby faces.
__device__ __forceinline__ int xcd_block(int b, int G)
{
    return (G & 7) == 0 ? (b & 7) * (G >> 3) + (b >> 3) : b;
}

template <int BLOCK, int PPT>
__global__ __launch_bounds__(BLOCK) void k_push_f64(Consts c, PushArgs a)
{
    const int64_t n = a.ctr->n_slots;
    constexpr int64_t TILE = (int64_t)BLOCK * PPT;
    const int64_t ntiles = (n + TILE - 1) / TILE;
    const int G = gridDim.x;
    const int lb = xcd_block(blockIdx.x, G);
    const int64_t t_begin = (ntiles * lb) / G, t_end = (ntiles * (lb + 1)) / G;
    const int64_t N = c.N;
    const double Nd = (double)N, Nm1 = (double)(N - 1);

    int64_t w0 = 0, nexit = 0, nabs = 0, nlost = 0, g_int = 0, g_frac = 0;
    unsigned st = 0;

    for (int64_t t = t_begin; t < t_end; ++t) {
        double xs[PPT], us[PPT];
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int64_t idx = t * TILE + k * BLOCK + threadIdx.x;
            xs[k] = idx < n ? a.X[idx] : -1.0;
            us[k] = idx < n ? a.U[idx] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int64_t idx = t * TILE + k * BLOCK + threadIdx.x;
            const double x = xs[k], u = us[k];
            const bool live = x >= 0.0;          // removed slots hold -1
            int64_t fa = 0, fb = 0, va = 0, vb = 0;
            bool da = false, db = false;
            if (live) {
                // gather: linear interpolation between face values, clamped at the ends
                const double s = x - 0.5;
                int64_t jj = (int64_t)floor(s);
                const double g = s - (double)jj;
                const int64_t jc = jj < 0 ? 0 : (jj > N - 2 ? N - 2 : jj);
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
                    st |= PIC_ST_NONFINITE;
                    ++nlost;
                    a.X[idx] = -1.0;
                } else {
                    // charge-conserving current: J_{i+1/2} += S_i(x^n) - S_i(x^{n+1}),
                    // nonzero on the old cell's face and, after a crossing, the new one
                    const double c0d = floor(x);
                    const int64_t c0 = (int64_t)c0d;
                    const int64_t F0 = (int64_t)rint((x - c0d) * c.twoP);
                    const double c1d = floor(x1);
                    const int64_t c1 = (int64_t)c1d;
                    const int64_t F1 = (int64_t)rint((x1 - c1d) * c.twoP);
                    fa = c0;
                    da = true;
                    if (c1 == c0) {
                        va = F1 - F0;
                    } else if (c1 > c0) {
                        va = c.oneP - F0;
                        if (c1 < N) { fb = c1; vb = F1; db = true; }
                    } else {
                        va = -F0;
                        if (c1 >= 0) { fb = c1; vb = F1 - c.oneP; db = true; }
                    }
                    if (x1 >= Nd) {                  // leaves through z = L
                        ++nexit;
                        const double gi = floor(gam);
                        g_int += (int64_t)gi;
                        g_frac += (int64_t)rint((gam - gi) * 4294967296.0);
                        a.X[idx] = -1.0;
                    } else if (x1 < 0.0) {           // returns to the star
                        ++nabs;
                        a.X[idx] = -1.0;
                    } else {
                        if (c1 == 0) w0 += c.oneP - F1;
                        a.X[idx] = x1;
                        a.U[idx] = u1;
                    }
                }
            }
            wave_add_keyed(a.J, fa, va, da && va != 0);
            wave_add_keyed(a.J, fb, vb, db && vb != 0);
        }
    }

    // per-wave tallies -> one atomic each
    DevCounters *ctr = a.ctr;
    const unsigned long long any = __ballot(w0 != 0 || nexit != 0 || nabs != 0 || nlost != 0 || st != 0);
    if (!any) return;
    w0 = wave_sum_i64(w0);
    nexit = wave_sum_i64(nexit);
    nabs = wave_sum_i64(nabs);
    nlost = wave_sum_i64(nlost);
    g_int = wave_sum_i64(g_int);
    g_frac = wave_sum_i64(g_frac);
    unsigned stw = st;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) stw |= (unsigned)__shfl_xor((int)stw, off);
    if (__lane_id() == 0) {
        if (w0) atomicAdd((unsigned long long *)&ctr->w0, (unsigned long long)w0);
        if (nexit) {
            atomicAdd((unsigned long long *)&ctr->n_exit, (unsigned long long)nexit);
            const __int128 s = ((__int128)g_int << 32) + (__int128)g_frac;
            atomic_add_i128(&ctr->exit_lo, &ctr->exit_hi, s);
        }
        if (nabs) atomicAdd((unsigned long long *)&ctr->n_absorb, (unsigned long long)nabs);
        const int64_t rem = nexit + nabs + nlost;
        if (rem) atomicAdd((unsigned long long *)&ctr->n_removed, (unsigned long long)rem);
        if (stw) atomicOr(&ctr->status, (unsigned long long)stw);
    }
}

template <int BLOCK, int PPT>
static hipError_t launch_push_t(pic_handle *h, unsigned grid)
{
    PushArgs a{h->ws.x[h->pbuf], h->ws.u[h->pbuf], h->ws.k64,
               (unsigned long long *)h->ws.j[h->jbuf], h->ws.ctr};
    hipLaunchKernelGGL((k_push_f64<BLOCK, PPT>), dim3(grid), dim3(BLOCK), 0, h->stream, h->c, a);
    return hipGetLastError();
}

hipError_t launch_push_f64(pic_handle *h)
{
    unsigned grid = h->push_grid > 0 ? (unsigned)h->push_grid : (unsigned)(h->n_cu * 8);
    const int B = h->push_block, P = h->push_ppt;
    if (B == 256 && P == 4) return launch_push_t<256, 4>(h, grid);
    if (B == 256 && P == 2) return launch_push_t<256, 2>(h, grid);
    if (B == 256 && P == 8) return launch_push_t<256, 8>(h, grid);
    if (B == 512 && P == 4) return launch_push_t<512, 4>(h, grid);
    if (B == 128 && P == 4) return launch_push_t<128, 4>(h, grid);
    if (B == 256 && P == 1) return launch_push_t<256, 1>(h, grid);
    return hipErrorInvalidValue;
}

}  // namespace pcpic
