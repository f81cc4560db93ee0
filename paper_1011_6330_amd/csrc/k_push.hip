// k_push.hip -- the particle half of the PIC cycle (sec. 2, Fig. A) in FP64:
// gather E_z at x^n, relativistic kick and move (eq. 1), charge-conserving
// linear current deposit in fixed point, removal at the tube ends, and the
// node-0 weight tally the SCLF injection needs.
//
// Layout and mapping: x and u are SoA FP64 streams (16 B read + 16 B written
// per live particle and step).  One block owns one tile of BLOCK*PPT
// consecutive slots and each thread PPT consecutive slots, loaded as 16-byte
// vectors.  Between cell sorts consecutive slots sit in the same cell, so a
// thread's current contributions land on three faces (cf-1, cf, cf+1 around
// the cell cf of its first live particle) and are summed in registers; one
// DPP reduction per wave and face group then issues a single int64 atomic per
// face.  Contributions elsewhere go straight to a global atomic.
//
// Exactness: every current contribution is an integer below 2^34 held in a
// double; sums of up to 2^19 of them stay below 2^53, so the register and DPP
// additions are exact and the int64 atomics make the total order-free.
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

__device__ __forceinline__ void atomic_add_face(unsigned long long *J, int f, double v)
{
    atomicAdd(J + f, (unsigned long long)(long long)v);
}

template <int BLOCK, int PPT>
__global__ __launch_bounds__(BLOCK) void k_push_f64(Consts c, PushArgs a)
{
    const int64_t n = a.ctr->n_slots;
    constexpr int TILE = BLOCK * PPT;
    const int64_t tile0 = (int64_t)blockIdx.x * TILE;
    if (tile0 >= n) return;                       // whole block idle (uniform)
    const int N = (int)c.N;
    const double Nd = (double)c.N, Nm1 = (double)(c.N - 1);
    const int64_t p0 = tile0 + (int64_t)threadIdx.x * PPT;

    double xs[PPT], us[PPT];
    if (p0 + PPT <= n) {
#pragma unroll
        for (int k = 0; k < PPT; k += 2) {
            const double2 xv = *reinterpret_cast<const double2 *>(a.X + p0 + k);
            const double2 uv = *reinterpret_cast<const double2 *>(a.U + p0 + k);
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

    int cf = -2;                                  // cell of the first live particle
    double acc_m = 0.0, acc_0 = 0.0, acc_p = 0.0; // faces cf-1, cf, cf+1
    double w0 = 0.0, nexit = 0.0, nabs = 0.0, nlost = 0.0, g_int = 0.0, g_frac = 0.0;
    bool bad = false;

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
            bad = true;
            nlost += 1.0;
            xs[k] = -1.0;
            continue;
        }
        // charge-conserving current J_{i+1/2} += S_i(x^n) - S_i(x^{n+1}): nonzero on
        // the old cell's face and, after a crossing, on the new cell's face
        const double c0d = floor(x);
        const int c0 = (int)c0d;
        const double F0 = rint((x - c0d) * c.twoP);
        const double c1d = floor(x1);
        const int c1 = (int)c1d;
        const double F1 = rint((x1 - c1d) * c.twoP);
        double va, vb = 0.0;
        bool hb = false;
        if (c1 == c0) {
            va = F1 - F0;
        } else if (c1 > c0) {
            va = c.twoP - F0;
            if (c1 < N) { vb = F1; hb = true; }
        } else {
            va = -F0;
            if (c1 >= 0) { vb = F1 - c.twoP; hb = true; }
        }
        if (cf == -2) cf = c0;
        if (c0 == cf) {
            acc_0 += va;
            if (hb) {
                if (c1 > c0) acc_p += vb;
                else acc_m += vb;
            }
        } else {
            if (va != 0.0) atomic_add_face(a.J, c0, va);
            if (hb && vb != 0.0) atomic_add_face(a.J, c1, vb);
        }
        if (x1 >= Nd) {                          // leaves through z = L
            nexit += 1.0;
            const double gi = floor(gam);
            g_int += gi;
            g_frac += rint((gam - gi) * 4294967296.0);
            xs[k] = -1.0;
        } else if (x1 < 0.0) {                   // returns to the star
            nabs += 1.0;
            xs[k] = -1.0;
        } else {
            if (c1 == 0) w0 += c.twoP - F1;
            xs[k] = x1;
            us[k] = u1;
        }
    }

    // write back (removed particles get x = -1; their u is left as it was)
    if (p0 + PPT <= n) {
#pragma unroll
        for (int k = 0; k < PPT; k += 2) {
            *reinterpret_cast<double2 *>(a.X + p0 + k) = make_double2(xs[k], xs[k + 1]);
            *reinterpret_cast<double2 *>(a.U + p0 + k) = make_double2(us[k], us[k + 1]);
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

    // one atomic per face group and wave: lanes sharing cf are summed together
    const int lane = __lane_id();
    bool want = cf != -2 && (acc_m != 0.0 || acc_0 != 0.0 || acc_p != 0.0);
    unsigned long long pend = __ballot(want);
    while (pend) {
        const int leader = __ffsll(pend) - 1;
        const int lk = __shfl(cf, leader);
        const bool mine = want && cf == lk;
        const double sm = wave_sum_f64_to63(mine ? acc_m : 0.0);
        const double s0 = wave_sum_f64_to63(mine ? acc_0 : 0.0);
        const double sp = wave_sum_f64_to63(mine ? acc_p : 0.0);
        if (lane == 63) {
            if (sm != 0.0) atomic_add_face(a.J, lk - 1, sm);
            if (s0 != 0.0) atomic_add_face(a.J, lk, s0);
            if (sp != 0.0) atomic_add_face(a.J, lk + 1, sp);
        }
        pend &= ~__ballot(mine);
        want = want && !mine;
    }

    // per-wave tallies
    DevCounters *ctr = a.ctr;
    const unsigned long long any = __ballot(w0 != 0.0 || nexit != 0.0 || nabs != 0.0 || nlost != 0.0);
    if (any) {
        w0 = wave_sum_f64_to63(w0);
        nexit = wave_sum_f64_to63(nexit);
        nabs = wave_sum_f64_to63(nabs);
        nlost = wave_sum_f64_to63(nlost);
        g_int = wave_sum_f64_to63(g_int);
        g_frac = wave_sum_f64_to63(g_frac);
        if (lane == 63) {
            if (w0 != 0.0) atomicAdd((unsigned long long *)&ctr->w0, (unsigned long long)(long long)w0);
            if (nexit != 0.0) {
                atomicAdd((unsigned long long *)&ctr->n_exit, (unsigned long long)(long long)nexit);
                const __int128 sum = ((__int128)(long long)g_int << 32) + (__int128)(long long)g_frac;
                atomic_add_i128(&ctr->exit_lo, &ctr->exit_hi, sum);
            }
            if (nabs != 0.0) atomicAdd((unsigned long long *)&ctr->n_absorb, (unsigned long long)(long long)nabs);
            const double rem = nexit + nabs + nlost;
            if (rem != 0.0) atomicAdd((unsigned long long *)&ctr->n_removed, (unsigned long long)(long long)rem);
        }
    }
    if (__ballot(bad) && lane == 0) atomicOr(&ctr->status, (unsigned long long)PIC_ST_NONFINITE);
}

template <int BLOCK, int PPT>
static hipError_t launch_push_t(pic_handle *h)
{
    PushArgs a{h->ws.x[h->pbuf], h->ws.u[h->pbuf], h->ws.k64,
               (unsigned long long *)h->ws.j[h->jbuf], h->ws.ctr};
    const int64_t tile = (int64_t)BLOCK * PPT;
    const unsigned grid = (unsigned)((h->c.cap + tile - 1) / tile);
    hipLaunchKernelGGL((k_push_f64<BLOCK, PPT>), dim3(grid), dim3(BLOCK), 0, h->stream, h->c, a);
    return hipGetLastError();
}

hipError_t launch_push_f64(pic_handle *h)
{
    const int B = h->push_block, P = h->push_ppt;
    if (B == 256 && P == 4) return launch_push_t<256, 4>(h);
    if (B == 256 && P == 2) return launch_push_t<256, 2>(h);
    if (B == 256 && P == 8) return launch_push_t<256, 8>(h);
    if (B == 128 && P == 4) return launch_push_t<128, 4>(h);
    if (B == 512 && P == 4) return launch_push_t<512, 4>(h);
    if (B == 64 && P == 4) return launch_push_t<64, 4>(h);
    if (B == 128 && P == 8) return launch_push_t<128, 8>(h);
    return hipErrorInvalidValue;
}

}  // namespace pcpic
