// field_body.h -- per-tile body of the leap-frog field update and the SCLF
// injection, shared by the single-tube kernel and the batched field kernel.
#pragma once

#include <math.h>

#include "pcpic_internal.h"

namespace pcpic {

struct FieldArgs {
    const double *ezo, *ero, *bo;   // E^n, B^{n-1/2}
    double *ezn, *ern, *bn;         // E^{n+1}, B^{n+1/2}
    const int64_t *j;               // J^{n+1/2} of this step
    int64_t *jnext;                 // cleared for the next step
    float *k32;                     // FP32-bulk: f32 kick array (q/m) dt E_z (else null)
    double *X, *U;                  // FP64: current particle buffer (injection)
    int *CL;                        // FP32-bulk: low stream of the current buffer
    float *OL, *UL;
    DevCounters *ctr;
    const int64_t *sched = nullptr;   // recorded injection counts (device), replayed for
    int64_t sched_first = 0;          // steps [sched_first, sched_first + sched_n)
    int64_t sched_n = 0;
    unsigned long long *hist = nullptr;   // step before a sort: key counts (injected particles added)
    int64_t inj_key = 0;                  // sort key of a particle injected at x = 0, u = 0
};

// Leap-frog update of eq. (3) at face i (the update of face N-1 also owns node N):
//   B_{i+1/2}  <- B - [ (dt/dz)(E_r,i+1 - E_r,i) + (dt/R) E_z,i+1/2 ]
//   E_r,i      <- E_r,i - (dt/dz)(B_{i+1/2} - B_{i-1/2}),  i = 1..N-1 (E_r,0 unchanged, = 0)
//   E_r,N      <- E_r,N + 2 (dt/dz) B_{N-1/2}           (B odd about the mirror x = N)
//   E_z,i+1/2  <- (E_z + (dt/R) B_{i+1/2}) - 4 pi q_m 2^-P J_{i+1/2}
// The neighbour B_{i-1/2} is recomputed from the old fields with the same
// expression instead of being exchanged.  PIC_GR_ALPHA puts the lapse on each
// term (alpha B/R, alpha d(alpha E_r)/dz, alpha d(alpha B)/dz, alpha E_z/R, with
// alpha at faces and nodes as pcpic.h states).  Returns the new E_z.
__device__ __forceinline__ double field_cell(const Consts &c, const FieldArgs &a, int64_t i)
{
    const int64_t N = c.N;
    a.jnext[i] = 0;
    double ez;
    if (c.flags & PIC_FREEZE_FIELDS) {
        ez = a.ezo[i];
        a.bn[i] = a.bo[i];
        a.ern[i] = a.ero[i];
        if (i == N - 1) a.ern[N] = a.ero[N];
    } else if (c.flags & PIC_GR_ALPHA) {
        // the same update with the lapse on each term (alpha at faces af, nodes an)
        const double af = gr_alpha_face(c, i), an0 = gr_alpha_node(c, i), an1 = gr_alpha_node(c, i + 1);
        const double bi = a.bo[i] - (c.dtdz * (af * (an1 * a.ero[i + 1] - an0 * a.ero[i])) + c.dtR * (af * a.ezo[i]));
        a.bn[i] = bi;
        if (i >= 1) {
            const double afm = gr_alpha_face(c, i - 1), anm = gr_alpha_node(c, i - 1);
            const double bm = a.bo[i - 1] - (c.dtdz * (afm * (an0 * a.ero[i] - anm * a.ero[i - 1])) +
                                             c.dtR * (afm * a.ezo[i - 1]));
            a.ern[i] = a.ero[i] - c.dtdz * (an0 * (af * bi - afm * bm));
        } else {
            a.ern[0] = a.ero[0];
        }
        if (i == N - 1) a.ern[N] = a.ero[N] + c.tw * (an1 * (af * bi));
        ez = (a.ezo[i] + c.dtR * (af * bi)) - c.c4 * (double)a.j[i];
    } else {
        const double bi = a.bo[i] - (c.dtdz * (a.ero[i + 1] - a.ero[i]) + c.dtR * a.ezo[i]);
        a.bn[i] = bi;
        if (i >= 1) {
            const double bm = a.bo[i - 1] - (c.dtdz * (a.ero[i] - a.ero[i - 1]) + c.dtR * a.ezo[i - 1]);
            a.ern[i] = a.ero[i] - c.dtdz * (bi - bm);
        } else {
            a.ern[0] = a.ero[0];
        }
        if (i == N - 1) a.ern[N] = a.ero[N] + c.tw * bi;
        ez = (a.ezo[i] + c.dtR * bi) - c.c4 * (double)a.j[i];
    }
    a.ezn[i] = ez;
    if (a.k32) a.k32[i] = (float)(c.qmdt * ez);
    return ez;
}

// Value of lane + 1 (lane 63 reads 0) and of lane - 1 (lane 0 reads 0) of a
// double: DPP wave_shl:1 and wave_shr:1 on its two halves.
__device__ __forceinline__ double lane_next_f64(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x130, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x130, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double lane_prev_f64(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x138, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x138, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double readlane_f64(double v, int l)
{
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                            __builtin_amdgcn_readlane(__double2loint(v), l));
}

// The flat update (no lapse, fields not frozen) of the 4*64 faces [w0, w0 + 256)
// of one wave (w0 a multiple of 256, w0 + 256 <= N), wave-collective.  Lane L
// takes the face pairs w0 + 2L and w0 + 128 + 2L, so that each 16-byte access
// covers one contiguous span of 128 faces.  A pair's new B at its first face
// serves as B_{i-1/2} of its second; B_{i-1/2} of its first face is the new B
// of the previous lane's second face (moved across lanes), of the first pairs'
// last lane for lane 0's second pair, and is recomputed with field_cell's
// expression only at face w0 - 1; E_r after a pair likewise comes from the
// next lane.  Every value has the expression, and so the bits, of field_cell.
// Returns the new E_z of face w0 + 2L.
__device__ __forceinline__ double field_wave_pairs(const Consts &c, const FieldArgs &a, int64_t w0)
{
    typedef double d2 __attribute__((ext_vector_type(2)));
    typedef long long l2 __attribute__((ext_vector_type(2)));
    typedef float f2 __attribute__((ext_vector_type(2)));
    const int lane = (int)__lane_id();
    const int64_t N = c.N;
    d2 ez[2], er[2], bo[2];
    l2 jj[2];
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        const int64_t f = w0 + 128 * p + 2 * lane;
        ez[p] = *(const d2 *)(a.ezo + f);
        er[p] = *(const d2 *)(a.ero + f);
        bo[p] = *(const d2 *)(a.bo + f);
        jj[p] = *(const l2 *)(a.j + f);
    }
    // E_r at the face after each pair
    double err[2];
    err[0] = lane_next_f64(er[0].x);
    err[1] = lane_next_f64(er[1].x);
    const double er_next0 = readlane_f64(er[1].x, 0);
    if (lane == 63) {
        err[0] = er_next0;
        err[1] = a.ero[w0 + 256];
    }
    double b1[2], b2[2];
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        b1[p] = bo[p].x - (c.dtdz * (er[p].y - er[p].x) + c.dtR * ez[p].x);
        b2[p] = bo[p].y - (c.dtdz * (err[p] - er[p].y) + c.dtR * ez[p].y);
    }
    // B_{i-1/2} of each pair's first face
    double bl[2];
    bl[0] = lane_prev_f64(b2[0]);
    bl[1] = lane_prev_f64(b2[1]);
    const double b_last0 = readlane_f64(b2[0], 63);
    if (lane == 0) {
        bl[1] = b_last0;
        bl[0] = w0 >= 1 ? a.bo[w0 - 1] - (c.dtdz * (er[0].x - a.ero[w0 - 1]) + c.dtR * a.ezo[w0 - 1]) : 0.0;
    }
    double ez_first = 0.0;
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        const int64_t f = w0 + 128 * p + 2 * lane;
        const double ern1 = f >= 1 ? er[p].x - c.dtdz * (b1[p] - bl[p]) : er[p].x;
        const double ern2 = er[p].y - c.dtdz * (b2[p] - b1[p]);
        const double ezn1 = (ez[p].x + c.dtR * b1[p]) - c.c4 * (double)jj[p].x;
        const double ezn2 = (ez[p].y + c.dtR * b2[p]) - c.c4 * (double)jj[p].y;
        *(d2 *)(a.bn + f) = d2{b1[p], b2[p]};
        *(d2 *)(a.ern + f) = d2{ern1, ern2};
        *(d2 *)(a.ezn + f) = d2{ezn1, ezn2};
        *(l2 *)(a.jnext + f) = l2{0, 0};
        if (a.k32) *(f2 *)(a.k32 + f) = f2{(float)(c.qmdt * ezn1), (float)(c.qmdt * ezn2)};
        if (p == 0) ez_first = ezn1;
    }
    if (lane == 63 && w0 + 256 == N) a.ern[N] = a.ero[N] + c.tw * b2[1];
    return ez_first;
}

// The field update of the faces [tile*bs*4, (tile+1)*bs*4), 256 faces per wave:
// field_wave_pairs where the flat update applies to the wave's whole span, else
// FIELD_CPT consecutive faces per thread with field_cell face by face; the
// block of tile 0 then applies the SCLF rule.  Called by all threads of a block
// of bs threads (a multiple of 64).
__device__ __forceinline__ void field_tile(const Consts &c, const FieldArgs &a, int64_t tile, int bs)
{
    __shared__ double s_ez0;
    __shared__ long long s_base, s_n;
    const int64_t N = c.N;
    const int64_t i0 = (tile * bs + threadIdx.x) * FIELD_CPT;
    const int64_t w0 = (tile * bs + (threadIdx.x & ~63)) * FIELD_CPT;   // the wave's first face (uniform)
    static_assert(FIELD_CPT == 4, "a wave takes 256 faces");
    if (!(c.flags & (PIC_FREEZE_FIELDS | PIC_GR_ALPHA)) && w0 + 256 <= N) {
        const double ez = field_wave_pairs(c, a, w0);
        if (w0 + 2 * (int)__lane_id() == 0) s_ez0 = ez;
    } else if (i0 < N) {
        const double ez = field_cell(c, a, i0);
        for (int k = 1; k < FIELD_CPT && i0 + k < N; ++k) field_cell(c, a, i0 + k);
        if (i0 == 0) s_ez0 = ez;
    }
    if (tile != 0) return;
    __syncthreads();
    DevCounters *ctr = a.ctr;
    if (threadIdx.x == 0) {
        // surface field from the node-0 Gauss law over the half cell [0, dz/2]
        const int64_t w0 = __hip_atomic_load(&ctr->w0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int64_t slots = __hip_atomic_load(&ctr->n_slots, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // FP32-bulk: the two streams together stay within the capacity, since a
        // sort may move every particle into either one (0 in FP64 mode)
        const int64_t slots_hi = __hip_atomic_load(&ctr->n_slots_hi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const double t1 = c.qmP * (double)w0;
        double t2 = c.rho0 * c.hdz;
        if (c.flags & PIC_GR_ALPHA) t2 = t2 / gr_alpha_node(c, 0);   // rho_GJ,0 / alpha_0 over the half cell
        const double es = s_ez0 - c.fourpi * (t1 - t2);
        int64_t ninj = 0;
        const int64_t ks = ctr->step - a.sched_first;   // index of this step in a replayed schedule
        if (a.sched && ks >= 0 && ks < a.sched_n) {
            const int64_t want = a.sched[ks] > 0 ? a.sched[ks] : 0;
            const int64_t avail = c.cap - slots - slots_hi;
            ninj = want > avail ? avail : want;
            if (want > avail) atomicOr(&ctr->status, (unsigned long long)PIC_ST_CAPACITY);
        } else if (!(c.flags & PIC_NO_AUTO_INJECT)) {
            const double ratio = es / c.fqm;
            if (ratio > 0.0) {
                const double nf = floor(ratio);
                const int64_t avail = c.cap - slots - slots_hi;
                if (nf > (double)avail) {
                    ninj = avail;
                    atomicOr(&ctr->status, (unsigned long long)PIC_ST_CAPACITY);
                } else {
                    ninj = (int64_t)nf;
                }
            }
        }
        if (a.hist && ninj > 0) atomicAdd(a.hist + a.inj_key, (unsigned long long)ninj);
        s_base = slots;
        s_n = ninj;
        ctr->n_slots = slots + ninj;
        ctr->n_injected += ninj;
        ctr->last_ninj = ninj;
        ctr->e_surf = es;
        ctr->w0_last = w0;
        ctr->w0 = 0;
        ctr->step += 1;
    }
    __syncthreads();
    const long long base = s_base, n = s_n;
    for (long long p = threadIdx.x; p < n; p += bs) {
        // electrons leave the surface at rest
        if (a.CL) {
            a.CL[base + p] = 0;
            a.OL[base + p] = 0.0f;
            a.UL[base + p] = 0.0f;
        } else {
            a.X[base + p] = 0.0;
            a.U[base + p] = 0.0;
        }
    }
}

}  // namespace pcpic
