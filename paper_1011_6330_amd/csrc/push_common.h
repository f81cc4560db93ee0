// push_common.h -- per-thread accumulation of the charge-conserving current and
// of the boundary tallies, shared by the FP64 and FP32-bulk push kernels.
//
// Current contributions are integers below 2^34 held in doubles; every sum
// below stays under 2^53, so all additions are exact and the int64 atomics
// make the result independent of the order of particles, lanes and blocks.
#pragma once

#include <limits.h>
#include <math.h>

#include "pcpic_internal.h"
#include "short_math.h"
#include "wave.h"

namespace pcpic {

__device__ __forceinline__ void atomic_add_face(unsigned long long *J, int f, double v)
{
    atomicAdd(J + f, (unsigned long long)(long long)v);
}

struct DepAcc {
    int cf;                    // cell of the thread's first deposit (-2 = none yet)
    double am, a0, ap, a2;     // faces cf-1, cf, cf+1, cf+2 (particles starting in cf or cf+1)
    DevCounters *ctr;          // the boundary tallies go straight to the counters

    __device__ __forceinline__ void init(DevCounters *counters)
    {
        cf = -2;
        am = a0 = ap = a2 = 0.0;
        ctr = counters;
    }

    // Boundary events are rare (a few hundred particles per step leave or
    // return; only cell 0 feeds the node-0 tally), so each lane adds its own
    // with integer atomics, which keeps the sums independent of order.
    __device__ __forceinline__ void exit_gamma(double gam)
    {
        // exit-gamma sum in units of 2^-32: integer part and fraction kept apart
        const double gi = floor(gam);
        const double gf = rint((gam - gi) * 4294967296.0);
        const __int128 sum = ((__int128)(long long)gi << 32) + (__int128)(long long)gf;
        atomicAdd((unsigned long long *)&ctr->n_exit, 1ull);
        atomicAdd((unsigned long long *)&ctr->n_removed, 1ull);
        atomic_add_i128(&ctr->exit_lo, &ctr->exit_hi, sum);
    }
    __device__ __forceinline__ void absorb()
    {
        atomicAdd((unsigned long long *)&ctr->n_absorb, 1ull);
        atomicAdd((unsigned long long *)&ctr->n_removed, 1ull);
    }
    __device__ __forceinline__ void lost()
    {
        atomicAdd((unsigned long long *)&ctr->n_removed, 1ull);
        atomicOr(&ctr->status, (unsigned long long)PIC_ST_NONFINITE);
    }
    __device__ __forceinline__ void node0(double w)
    {
        atomicAdd((unsigned long long *)&ctr->w0, (unsigned long long)(long long)w);
    }

    // J_{i+1/2} += S_i(x^n) - S_i(x^{n+1}) for a move from (c0, F0) to (c1, F1),
    // |c1 - c0| <= 1, with S_i the fixed-point cumulative linear weight left of
    // face i+1/2 (2^P left of node i, 2^P - F in cell i, 0 right of node i+1):
    // face c0 gets (2^P if c1 > c0, 0 if c1 < c0, F1 if c1 = c0) - F0, and a
    // crossed face c1 inside the tube gets F1 (moving right) or F1 - 2^P (left).
    // Written with selects for a lane that may have nothing to deposit
    // (ok = false): lanes of a wave split between staying in their cell and
    // crossing a face, and selects keep them on one path.  A particle starting
    // in cf or cf+1 lands in the four channels; any other (a thread whose slots
    // span more than two cells) adds its own atomics.
    __device__ __forceinline__ void deposit_sel(unsigned long long *J, int N, double twoP, bool ok, int c0, double F0,
                                                int c1, double F1)
    {
        const bool right = c1 > c0, left = c1 < c0;
        const double va = (right ? twoP : (left ? 0.0 : F1)) - F0;
        const double vb = left ? F1 - twoP : F1;
        const bool hb = (right && c1 < N) || (left && c1 >= 0);
        if (ok && cf == -2) cf = c0;
        const bool in0 = ok && c0 == cf, in1 = ok && c0 == cf + 1;
        const double vl = (hb && left) ? vb : 0.0, vr = (hb && right) ? vb : 0.0;
        am += in0 ? vl : 0.0;
        a0 += in0 ? va : (in1 ? vl : 0.0);
        ap += in0 ? vr : (in1 ? va : 0.0);
        a2 += in1 ? vr : 0.0;
        if (ok && !in0 && !in1) {
            if (va != 0.0) atomic_add_face(J, c0, va);
            if (hb && vb != 0.0) atomic_add_face(J, c1, vb);
        }
    }

    // Wave-collective: must be reached by all 64 lanes of the wave.  A wave
    // whose lanes share their first cell (the common case between sorts) sums
    // its four channels together (row swaps, then a scan inside each row) and
    // adds one atomic per face.  A wave whose first cells span at most 61 cells
    // sums its channels in a per-wave LDS window with integer atomics and adds
    // each touched face once.  Otherwise lanes with the same first cell in
    // consecutive positions form a run, and the run's last lane adds the run's
    // sums (segmented scans).  The channels start afresh.
    __device__ __forceinline__ void flush_current(unsigned long long *J)
    {
        const bool has = cf != -2;
        const int lane = (int)__lane_id();
        const int c_first = __builtin_amdgcn_readfirstlane(cf);
        if (__ballot(has && cf == c_first) == ~0ull) {
            // row k holds face c_first - 1 + k; its total sits in the row's last lane
            const double s = wave_sum4_rows_f64(am, a0, ap, a2);
            if ((lane & 15) == 15 && s != 0.0)
                atomicAdd(J + (c_first - 1 + (lane >> 4)), (unsigned long long)(long long)s);
            cf = -2;
            am = a0 = ap = a2 = 0.0;
            return;
        }
        const int lo = wave_min_i32(has ? cf : INT_MAX);
        if (wave_max_i32(has ? cf : INT_MIN) - lo <= 60) {
            // a few cells: the faces lo-1 .. hi+2 of the wave's first cells lo .. hi
            // in a window of 64 LDS words (word k: face lo-1+k); the lanes add their
            // channels with LDS integer atomics, then each lane adds one face to J
            __shared__ unsigned long long s_win[8][64];   // one window per wave (blocks up to 512)
            unsigned long long *w = s_win[threadIdx.x >> 6];
            w[lane] = 0;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (has) {
                const int k = cf - lo;
                if (am != 0.0) atomicAdd(w + k, (unsigned long long)(long long)am);
                if (a0 != 0.0) atomicAdd(w + k + 1, (unsigned long long)(long long)a0);
                if (ap != 0.0) atomicAdd(w + k + 2, (unsigned long long)(long long)ap);
                if (a2 != 0.0) atomicAdd(w + k + 3, (unsigned long long)(long long)a2);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const unsigned long long v = w[lane];
            if (v != 0) atomicAdd(J + (lo - 1 + lane), v);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        } else {
            const WaveRun r = wave_runs_i32(cf, has);
            double sm = am, s0 = a0, sp = ap, s2 = a2;
            if (__ballot(am != 0.0)) sm = run_sum_to_tail(sm, r.rank);
            if (__ballot(a0 != 0.0)) s0 = run_sum_to_tail(s0, r.rank);
            if (__ballot(ap != 0.0)) sp = run_sum_to_tail(sp, r.rank);
            if (__ballot(a2 != 0.0)) s2 = run_sum_to_tail(s2, r.rank);
            if (has && lane == r.end - 1) {
                if (sm != 0.0) atomic_add_face(J, cf - 1, sm);
                if (s0 != 0.0) atomic_add_face(J, cf, s0);
                if (sp != 0.0) atomic_add_face(J, cf + 1, sp);
                if (s2 != 0.0) atomic_add_face(J, cf + 2, s2);
            }
        }
        cf = -2;
        am = a0 = ap = a2 = 0.0;
    }
};

// gamma = sqrt(tt) and v = u / gamma for tt = 1 + u^2, both correctly rounded.
// Square root: Goldschmidt iteration from the hardware reciprocal square root
// estimate y (g = tt y, h = y/2, one joint correction, then two residual
// corrections g += (tt - g^2) h).  Quotient: Newton-Raphson reciprocal from the
// hardware estimate (two steps), q = u r, and one residual correction
// q += (u - gamma q) r (Markstein).  These are the operations, in order, that
// the general correctly rounded double-precision square root and division
// perform when their range scaling does not apply, which holds for tt >= 1 and
// 2^-400 <= |u| <= 2^400; outside that range (u = 0 included) the general
// routines are called.  Skipping the scaling and special-case steps saves
// about a dozen instructions per particle.
__device__ __forceinline__ void gamma_velocity(double u, double tt, double &gam, double &v)
{
    const double y = __builtin_amdgcn_rsq(tt);
    double g = tt * y, h = 0.5 * y;
    const double r = fma(-h, g, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    double d = fma(-g, g, tt);
    g = fma(d, h, g);
    d = fma(-g, g, tt);
    g = fma(d, h, g);
    double rc = __builtin_amdgcn_rcp(g);
    double e = fma(-g, rc, 1.0);
    rc = fma(rc, e, rc);
    e = fma(-g, rc, 1.0);
    rc = fma(rc, e, rc);
    const double q = u * rc;
    const double rem = fma(-g, q, u);
    gam = g;
    v = fma(rem, rc, q);
    const double au = fabs(u);
    if (!(au >= 0x1p-400 && au <= 0x1p+400)) {
        gam = sqrt(tt);
        v = u / gam;
    }
}

typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef float fvec4 __attribute__((ext_vector_type(4)));
typedef int ivec4 __attribute__((ext_vector_type(4)));
typedef float fvec2 __attribute__((ext_vector_type(2)));
typedef int ivec2 __attribute__((ext_vector_type(2)));
typedef unsigned uvec2 __attribute__((ext_vector_type(2)));
typedef unsigned uvec4 __attribute__((ext_vector_type(4)));

// Particle-stream vector access (16 or 8 bytes, the size of V); NT = 1 marks it
// nontemporal (each value is streamed once per step and should not displace
// the kick array and the current in L2).
template <int NT, typename V>
__device__ __forceinline__ V ld16(const void *p)
{
    if (NT) return __builtin_nontemporal_load(reinterpret_cast<const V *>(p));
    return *reinterpret_cast<const V *>(p);
}
template <int NT, typename V>
__device__ __forceinline__ void st16(void *p, V v)
{
    if (NT) __builtin_nontemporal_store(v, reinterpret_cast<V *>(p));
    else *reinterpret_cast<V *>(p) = v;
}

}  // namespace pcpic
