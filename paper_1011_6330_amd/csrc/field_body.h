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

// The flat update (no lapse, fields not frozen) of the four faces i0 .. i0+3
// (i0 a multiple of 4, i0 + 4 <= N) with 16-byte accesses; each face's B is
// computed once and serves as B_{i-1/2} of the next face, with the same
// expressions as field_cell.  Returns the new E_z of face i0.
__device__ __forceinline__ double field_cells4_flat(const Consts &c, const FieldArgs &a, int64_t i0)
{
    typedef double d2 __attribute__((ext_vector_type(2)));
    typedef long long l2 __attribute__((ext_vector_type(2)));
    typedef float f4 __attribute__((ext_vector_type(4)));
    const int64_t N = c.N;
    const d2 ez01 = *(const d2 *)(a.ezo + i0), ez23 = *(const d2 *)(a.ezo + i0 + 2);
    const d2 er01 = *(const d2 *)(a.ero + i0), er23 = *(const d2 *)(a.ero + i0 + 2);
    const d2 bo01 = *(const d2 *)(a.bo + i0), bo23 = *(const d2 *)(a.bo + i0 + 2);
    const l2 j01 = *(const l2 *)(a.j + i0), j23 = *(const l2 *)(a.j + i0 + 2);
    const double er4 = a.ero[i0 + 4];
    const double ez[4] = {ez01.x, ez01.y, ez23.x, ez23.y};
    const double er[5] = {er01.x, er01.y, er23.x, er23.y, er4};
    const double bo[4] = {bo01.x, bo01.y, bo23.x, bo23.y};
    const long long jj[4] = {j01.x, j01.y, j23.x, j23.y};
    double b[5];
    b[0] = 0.0;
    if (i0 >= 1) b[0] = a.bo[i0 - 1] - (c.dtdz * (er[0] - a.ero[i0 - 1]) + c.dtR * a.ezo[i0 - 1]);
#pragma unroll
    for (int k = 0; k < 4; ++k) b[k + 1] = bo[k] - (c.dtdz * (er[k + 1] - er[k]) + c.dtR * ez[k]);
    double ern[4], ezn[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        ern[k] = (i0 + k >= 1) ? er[k] - c.dtdz * (b[k + 1] - b[k]) : er[0];
        ezn[k] = (ez[k] + c.dtR * b[k + 1]) - c.c4 * (double)jj[k];
    }
    *(d2 *)(a.bn + i0) = d2{b[1], b[2]};
    *(d2 *)(a.bn + i0 + 2) = d2{b[3], b[4]};
    *(d2 *)(a.ern + i0) = d2{ern[0], ern[1]};
    *(d2 *)(a.ern + i0 + 2) = d2{ern[2], ern[3]};
    *(d2 *)(a.ezn + i0) = d2{ezn[0], ezn[1]};
    *(d2 *)(a.ezn + i0 + 2) = d2{ezn[2], ezn[3]};
    *(l2 *)(a.jnext + i0) = l2{0, 0};
    *(l2 *)(a.jnext + i0 + 2) = l2{0, 0};
    if (a.k32)
        *(f4 *)(a.k32 + i0) = f4{(float)(c.qmdt * ezn[0]), (float)(c.qmdt * ezn[1]), (float)(c.qmdt * ezn[2]),
                                 (float)(c.qmdt * ezn[3])};
    if (i0 + 4 == N) a.ern[N] = a.ero[N] + c.tw * b[4];
    return ezn[0];
}

// The field update of the faces [tile*bs*4, (tile+1)*bs*4), FIELD_CPT consecutive
// faces per thread (field_cells4_flat where it applies, else field_cell face by
// face); the block of tile 0 then applies the SCLF rule.  Called by all threads
// of a block of bs threads.
__device__ __forceinline__ void field_tile(const Consts &c, const FieldArgs &a, int64_t tile, int bs)
{
    __shared__ double s_ez0;
    __shared__ long long s_base, s_n;
    const int64_t N = c.N;
    const int64_t i0 = (tile * bs + threadIdx.x) * FIELD_CPT;
    if (i0 < N) {
        double ez;
        if (!(c.flags & (PIC_FREEZE_FIELDS | PIC_GR_ALPHA)) && i0 + FIELD_CPT <= N) {
            ez = field_cells4_flat(c, a, i0);
        } else {
            ez = field_cell(c, a, i0);
            for (int k = 1; k < FIELD_CPT && i0 + k < N; ++k) field_cell(c, a, i0 + k);
        }
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
