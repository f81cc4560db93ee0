// push_body.h -- per-tile bodies of the particle push (FP64 and FP32-bulk),
// shared by the single-tube kernels and the batched push kernel so that
// a tube computes the same bits whichever launch runs it.
#pragma once

#include <math.h>

#include "pcpic_internal.h"
#include "push_common.h"

namespace pcpic {

struct PushArgs {
    const double *__restrict__ X;   // slots read
    const double *__restrict__ U;
    double *__restrict__ Xo;        // slots written (== X, U for an in-place step)
    double *__restrict__ Uo;
    const double *__restrict__ EZ;  // E_z^n at the faces (the kick is (q/m) dt E_z)
    unsigned long long *__restrict__ J;
    DevCounters *ctr;
    unsigned long long *hist;       // non-null on the step before a sort: key counts of the survivors
};

// Add the sort keys of a tile's surviving particles to hist (one atomic per run
// of equal keys across the lanes, for each of a thread's PPT slots).
template <int PPT>
__device__ __forceinline__ void hist_add(unsigned long long *hist, const int64_t (&key)[PPT], const bool (&live)[PPT])
{
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const WaveRun r = wave_runs(key[k], live[k]);
        if (live[k] && r.is_head) atomicAdd(hist + key[k], (unsigned long long)(r.end - (int)__lane_id()));
    }
}

// Kick at x: linear interpolation between the face values K = (q/m) dt E_z,
// clamped at the ends.  Also called for an empty slot (x = -1), whose face index
// clamps to 0, so the loads of every slot can be issued together before any
// particle is pushed.
__device__ __forceinline__ double gather_f64(const Consts &c, const double *__restrict__ EZ, double x)
{
    const int N = (int)c.N;
    const double Nm1 = (double)(c.N - 1);
    const double s = x - 0.5;
    const int jj = (int)floor(s);
    const double g = s - (double)jj;
    const int jc = jj < 0 ? 0 : (jj > N - 2 ? N - 2 : jj);
    const double k0 = c.qmdt * EZ[jc], k1 = c.qmdt * EZ[jc + 1];
    const double Ei = k0 + g * (k1 - k0);
    const double lo = s < 0.0 ? k0 : Ei;
    return s >= Nm1 ? k1 : lo;
}

// Push of one particle (x, u) in place with the gathered kick E: kick and move
// (eq. 1), current deposit, removal at the ends (x = -1) and the node-0 tally.
// x < 0 marks an empty slot and is left alone.  Straight-line code with
// selects: every lane computes the step, and the flags say what is kept.
// GR (PIC_GR_ALPHA): du/dt = alpha (q/m) E_z - gamma alpha alpha' with a
// midpoint gamma for the gravity term, dz/dt = alpha^2 v with a midpoint
// alpha^2, as pcpic.h states.
template <int GR>
__device__ __forceinline__ void push_one_f64(const Consts &c, const PushArgs &a, double E, double &xr, double &ur,
                                             DepAcc &acc)
{
    const int N = (int)c.N;
    const double Nd = (double)N;
    const double x = xr, u = ur;
    const bool live = x >= 0.0;                  // not a removed slot (-1) or past the end
    // eq. (1): u = gamma v, du/dt = (q/m) E_z, dz/dt = v
    double u1, gam, v, x1;
    if (GR) {
        // the divisions and square roots take their short forms (nr_div,
        // gs_sqrt: the same bits) when every live lane's operands allow them
        const double zx = x * c.dz;
        const bool fast = c.gr_fast && __all(!live || nr_num_ok(zx));
        double eta, a2, al, kg, g0, gh;
        double t0 = u * u;
        t0 = 1.0 + t0;
        if (fast) {
            const double rr = nr_recip(c.r_star);
            eta = 1.0 + nr_div(zx, c.r_star, rr);
            a2 = 1.0 - nr_div(c.gr_g, eta, nr_recip(eta));
            al = gs_sqrt(a2);
            const double e2 = eta * eta;
            kg = nr_div(c.gr_cg, e2, nr_recip(e2));
            g0 = gs_sqrt(t0);
        } else {
            eta = 1.0 + zx / c.r_star;
            a2 = 1.0 - c.gr_g / eta;
            al = sqrt(a2);
            kg = c.gr_cg / (eta * eta);
            g0 = sqrt(t0);
        }
        const double uh = u + 0.5 * (al * E - kg * g0);
        double th = uh * uh;
        th = 1.0 + th;
        gh = fast ? gs_sqrt(th) : sqrt(th);
        u1 = u + (al * E - kg * gh);
        double tt = u1 * u1;
        tt = 1.0 + tt;
        gamma_velocity(u1, tt, gam, v);
        const double xh = x + 0.5 * (c.dtdz * (a2 * v));
        const double zh = xh * c.dz;
        double a2h;
        if (fast && __all(!live || nr_num_ok(zh))) {
            const double eh = 1.0 + nr_div(zh, c.r_star, nr_recip(c.r_star));
            a2h = 1.0 - nr_div(c.gr_g, eh, nr_recip(eh));
        } else {
            a2h = gr_alpha2(c, zh);
        }
        x1 = x + c.dtdz * (a2h * v);
    } else {
        u1 = u + E;
        double tt = u1 * u1;
        tt = 1.0 + tt;
        gamma_velocity(u1, tt, gam, v);
        x1 = x + c.dtdz * v;
    }
    const bool fin = isfinite(u1) && isfinite(x1);
    const bool ok = live && fin;
    const double c0d = floor(x);
    const double F0 = rint((x - c0d) * c.twoP);
    const double c1d = floor(x1);
    const int c1 = (int)c1d;
    const double F1 = rint((x1 - c1d) * c.twoP);
    acc.deposit_sel(a.J, N, c.twoP, ok, (int)c0d, F0, c1, F1);
    const bool exits = ok && x1 >= Nd;           // leaves through z = L
    const bool absorbed = ok && x1 < 0.0;        // returns to the star
    const bool stays = ok && !exits && !absorbed;
    if (exits) acc.exit_gamma(gam);
    if (absorbed) acc.absorb();
    if (stays && c1 == 0) acc.node0(c.twoP - F1);
    if (live && !fin) acc.lost();
    xr = stays ? x1 : (live ? -1.0 : x);
    ur = stays ? u1 : u;
}

// One tile of BLOCK*PPT consecutive slots starting at tile0 (< n).  Thread t
// takes PPT/2 pairs of consecutive slots, pair v at tile0 + 2 (v BLOCK + t), so
// each pair is one 16-byte vector per stream and a wave's pair v covers 128
// consecutive slots (PPT = 2: the thread's two slots).  Every pair of the
// thread is loaded, and every gather issued, before the first kick.  The
// current of pair v is flushed before pair v+1 is pushed, so a flush sees the
// few cells 128 consecutive slots span.  Called by every thread of a block of
// BLOCK threads; wave-collective.
template <int BLOCK, int PPT, int NT, int GR = 0>
__device__ __forceinline__ void push_tile_f64(const Consts &c, const PushArgs &a, int64_t n, int64_t tile0)
{
    static_assert(PPT % 2 == 0, "slots are taken in pairs");
    constexpr int V = PPT / 2;
    double xs[PPT], us[PPT];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const int64_t e = tile0 + 2 * ((int64_t)v * BLOCK + threadIdx.x);
        if (e + 2 <= n) {
            const dvec2 xv = ld16<NT, dvec2>(a.X + e);
            const dvec2 uv = ld16<NT, dvec2>(a.U + e);
            xs[2 * v] = xv.x; xs[2 * v + 1] = xv.y;
            us[2 * v] = uv.x; us[2 * v + 1] = uv.y;
        } else {
            xs[2 * v] = e < n ? a.X[e] : -1.0;
            us[2 * v] = e < n ? a.U[e] : 0.0;
            xs[2 * v + 1] = e + 1 < n ? a.X[e + 1] : -1.0;
            us[2 * v + 1] = e + 1 < n ? a.U[e + 1] : 0.0;
        }
    }
    double E[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) E[k] = gather_f64(c, a.EZ, xs[k]);

    DepAcc acc;
    acc.init(a.ctr);
#pragma unroll
    for (int v = 0; v < V; ++v) {
        push_one_f64<GR>(c, a, E[2 * v], xs[2 * v], us[2 * v], acc);
        push_one_f64<GR>(c, a, E[2 * v + 1], xs[2 * v + 1], us[2 * v + 1], acc);
        // write back (removed particles get x = -1; their u is left as it was)
        const int64_t e = tile0 + 2 * ((int64_t)v * BLOCK + threadIdx.x);
        if (e + 2 <= n) {
            st16<NT, dvec2>(a.Xo + e, dvec2{xs[2 * v], xs[2 * v + 1]});
            st16<NT, dvec2>(a.Uo + e, dvec2{us[2 * v], us[2 * v + 1]});
        } else {
            if (e < n) { a.Xo[e] = xs[2 * v]; a.Uo[e] = us[2 * v]; }
            if (e + 1 < n) { a.Xo[e + 1] = xs[2 * v + 1]; a.Uo[e + 1] = us[2 * v + 1]; }
        }
        acc.flush_current(a.J);
        if (a.hist) {
            int64_t key[2];
            bool live[2];
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                live[j] = xs[2 * v + j] >= 0.0;
                key[j] = live[j] ? sort_key_f64(c, xs[2 * v + j]) : 0;
            }
            hist_add<2>(a.hist, key, live);
        }
        // one pair at a time: interleaving pairs would cost registers and occupancy
        if (v + 1 < V) __builtin_amdgcn_sched_barrier(0);
    }
}


struct Push32Args {
    int *__restrict__ CL;
    float *__restrict__ OL;
    float *__restrict__ UL;
    unsigned *__restrict__ HP;       // high stream: position words
    int *__restrict__ HW;            //   cells of the slots of wide groups
    int *__restrict__ HG;            //   group headers
    double *__restrict__ UH;
    const float *__restrict__ K32;   // (float)((q/m) dt E_z) at the faces (low stream)
    const double *__restrict__ EZ;   // E_z^n at the faces (high stream: kick (q/m) dt E_z in f64)
    unsigned long long *__restrict__ J;
    DevCounters *ctr;
    unsigned long long *hist = nullptr;   // non-null on the step before a sort: key counts of the survivors
    double u_hi = 0.0;                    // |u| from which a particle belongs to the high stream
};

// Offset update with the carry into the next or previous cell (|move| < 1 cell),
// with selects.  An offset that rounds to 1.0f is stored as (cell + 1, 0).
__device__ __forceinline__ void carry_f32(float &o, int &cell)
{
    const bool up = o >= 1.0f, dn = o < 0.0f;
    const float om = o + 1.0f;
    const bool dn_full = dn && om >= 1.0f;       // -tiny + 1 rounds to 1: stays in the cell at 0
    o = up ? o - 1.0f : (dn ? (dn_full ? 0.0f : om) : o);
    cell += up ? 1 : ((dn && !dn_full) ? -1 : 0);
}

// Face values around x = cell + off (linear interpolation between faces, clamped
// at the ends): the lower face index, clamped, and the weight of the upper one.
// An empty slot (cell = -1) clamps to face 0, so every slot may load.
__device__ __forceinline__ int gather_face_f32(int N, int cell, float off, float &g, int &j)
{
    j = off < 0.5f ? cell - 1 : cell;
    g = off < 0.5f ? off + 0.5f : off - 0.5f;
    return j < 0 ? 0 : (j > N - 2 ? N - 2 : j);
}

// One particle of the low stream (f32 momentum) with its gathered kick E, in
// place; straight-line code with selects, as push_one_f64.  A particle whose
// |u| has reached the high stream's threshold uf (the sort will move it there)
// lands on the 2^-24 offset grid of that stream before it deposits.
__device__ __forceinline__ void push_one_lo(const Consts &c, const Push32Args &a, float E, float uf, int &cr,
                                            float &orf, float &ur, DepAcc &acc)
{
    const int N = (int)c.N;
    const int cell = cr;
    const float off = orf, u = ur;
    const bool live = cell >= 0;
    const float u1 = u + E;
    float t = u1 * u1;
    t = 1.0f + t;
    const float v = u1 * __builtin_amdgcn_rsqf(t);
    float o1 = off + (float)c.dtdz * v;
    int c1 = cell;
    carry_f32(o1, c1);
    if (fabsf(u1) >= uf) {
        const float q = rintf(o1 * 16777216.0f);
        const bool up = q >= 16777216.0f;
        c1 += up ? 1 : 0;
        o1 = up ? 0.0f : q * 0x1p-24f;
    }
    const bool fin = isfinite(u1) && isfinite(o1);
    const bool ok = live && fin;
    const double F0 = rint((double)off * c.twoP);
    const double F1 = rint((double)o1 * c.twoP);
    acc.deposit_sel(a.J, N, c.twoP, ok, cell, F0, c1, F1);
    const bool exits = ok && c1 >= N, absorbed = ok && c1 < 0;
    const bool stays = ok && !exits && !absorbed;
    if (exits) {
        const double ud = (double)u1;
        double tt = ud * ud;
        tt = 1.0 + tt;
        acc.exit_gamma(sqrt(tt));
    }
    if (absorbed) acc.absorb();
    if (stays && c1 == 0) acc.node0(c.twoP - F1);
    if (live && !fin) acc.lost();
    cr = stays ? c1 : (live ? -1 : cell);
    orf = stays ? o1 : off;
    ur = stays ? u1 : u;
}

// One particle of the high stream (f64 momentum, offset frac 2^-24 in the
// cell): kick, gamma and v in f64; the move c dt v / dz is rounded to the
// 2^-24 grid and added to the offset in integers (|move| < 1 cell, so the
// carry is the sign of the sum's high bits), and the deposit takes the stored
// positions, so that the current carries the charge exactly where it is kept.
// BIG (the whole wave has |u| >= 2^19 after the kick): with t = 1/u^2 <=
// 2^-38, v = sign(u) (1 - t/2) and gamma = |u| + 1/(2|u|) leave out terms
// below 2^-77 of v and 2^-58 of gamma; 1/u comes from the hardware estimate
// (good to about 2^-24) and one Newton step, which squares its error, so v and
// gamma are within half an ulp plus 2^-20 of an ulp of their correctly rounded
// values.  Otherwise gamma and v as the FP64 push forms them.  mscale =
// (c dt / dz) 2^24, fscale = 2^(P - 24).
// u1 is the momentum after the kick; a slot that ends removed keeps whatever
// momentum, as nothing reads it.
template <bool BIG>
__device__ __forceinline__ void push_one_hi(const Consts &c, unsigned long long *J, double u1, double mscale,
                                            double fscale, int &cr, unsigned &fr, DepAcc &acc)
{
    const int N = (int)c.N;
    const int cell = cr;
    const unsigned frac = fr;
    const bool live = cell >= 0;
    double gam, v;
    if (BIG) {
        const double r0 = __builtin_amdgcn_rcp(u1);
        const double r = fma(r0, fma(-u1, r0, 1.0), r0);
        const double h = 0.5 * r;
        v = copysign(fma(-h, r, 1.0), u1);
        gam = fabs(u1) + fabs(h);
    } else {
        double tt = u1 * u1;
        tt = 1.0 + tt;
        gamma_velocity(u1, tt, gam, v);
    }
    const int mv = (int)rint(v * mscale);          // |mv| <= 2^24
    const int nf = (int)frac + mv;
    const int c1 = cell + (nf >> HI_FRAC_BITS);    // -1, 0 or +1 cells
    const unsigned f1 = (unsigned)nf & HI_FRAC_MASK;
    const bool fin = isfinite(u1);
    const bool ok = live && fin;
    const double F0 = rint((double)frac * fscale);
    const double F1 = rint((double)f1 * fscale);
    acc.deposit_sel(J, N, c.twoP, ok, cell, F0, c1, F1);
    const bool exits = ok && c1 >= N, absorbed = ok && c1 < 0;
    const bool stays = ok && !exits && !absorbed;
    if (exits) acc.exit_gamma(gam);
    if (absorbed) acc.absorb();
    if (stays && c1 == 0) acc.node0(c.twoP - F1);
    if (live && !fin) acc.lost();
    cr = stays ? c1 : (live ? -1 : cell);
    fr = stays ? f1 : frac;
}

// One tile of BLOCK*F32_PPT_LO consecutive slots of the low stream, starting at
// tile0 (< n): gathers issued before the first kick, one current flush.
// Called by every thread of the block; wave-collective.
template <int BLOCK, int NT>
__device__ __forceinline__ void push_tile_lo(const Consts &c, const Push32Args &a, int64_t n, int64_t tile0)
{
    constexpr int PPT = F32_PPT_LO;
    const int N = (int)c.N;
    const int64_t p0 = tile0 + (int64_t)threadIdx.x * PPT;
    const bool full = p0 + PPT <= n;
    int *C = a.CL;
    float *O = a.OL;
    int cs[PPT];
    float os[PPT], us[PPT];
    if (full) {
        const ivec4 cv = ld16<NT, ivec4>(C + p0);
        const fvec4 ov = ld16<NT, fvec4>(O + p0);
        const fvec4 uv = ld16<NT, fvec4>(a.UL + p0);
        cs[0] = cv.x; cs[1] = cv.y; cs[2] = cv.z; cs[3] = cv.w;
        os[0] = ov.x; os[1] = ov.y; os[2] = ov.z; os[3] = ov.w;
        us[0] = uv.x; us[1] = uv.y; us[2] = uv.z; us[3] = uv.w;
    } else {
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            cs[k] = p0 + k < n ? C[p0 + k] : -1;
            os[k] = p0 + k < n ? O[p0 + k] : 0.0f;
            us[k] = p0 + k < n ? a.UL[p0 + k] : 0.0f;
        }
    }
    float E[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        float g;
        int j;
        const int jc = gather_face_f32(N, cs[k], os[k], g, j);
        const float k0 = a.K32[jc], k1 = a.K32[jc + 1];
        const float Ei = k0 + g * (k1 - k0);
        const float lo = j < 0 ? k0 : Ei;
        E[k] = j >= N - 1 ? k1 : lo;
    }
    DepAcc acc;
    acc.init(a.ctr);
    const float uf = f32_at_least(a.u_hi);
#pragma unroll
    for (int k = 0; k < PPT; ++k) push_one_lo(c, a, E[k], uf, cs[k], os[k], us[k], acc);
    if (full) {
        st16<NT, ivec4>(C + p0, ivec4{cs[0], cs[1], cs[2], cs[3]});
        st16<NT, fvec4>(O + p0, fvec4{os[0], os[1], os[2], os[3]});
        st16<NT, fvec4>(a.UL + p0, fvec4{us[0], us[1], us[2], us[3]});
    } else {
#pragma unroll
        for (int k = 0; k < PPT; ++k)
            if (p0 + k < n) { C[p0 + k] = cs[k]; O[p0 + k] = os[k]; a.UL[p0 + k] = us[k]; }
    }
    acc.flush_current(a.J);
    if (a.hist) {
        int64_t key[PPT];
        bool live[PPT];
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            live[k] = cs[k] >= 0;
            key[k] = live[k] ? sort_key_f32(c, cs[k], os[k], fabs((double)us[k]) >= a.u_hi) : 0;
        }
        hist_add<PPT>(a.hist, key, live);
    }
}

// One tile of BLOCK*F32_PPT_HI consecutive slots of the high stream (f64
// momentum), starting at tile0 (< n).  Wave-collective, as push_tile_lo.  Each
// wave takes one group of HI_GROUP slots: it decodes the positions with the
// group's header (reading the cell array only for a wide group), pushes, and
// writes the group back narrow or wide as its new live cells allow.  Lane L
// takes the slot pairs 2L and 128 + 2L of the group: with four consecutive
// slots per lane, each 16-byte momentum access would cover every other 16
// bytes of the stream, which measured 8% slower.  A group whose old cells span
// more than two cells flushes its current after the first pairs.
template <int BLOCK, int NT>
__device__ __forceinline__ void push_tile_hi(const Consts &c, const Push32Args &a, int64_t n, int64_t tile0)
{
    constexpr int PPT = F32_PPT_HI;
    static_assert(PPT == 4, "the high tile takes two pairs of slots per lane");
    const int N = (int)c.N;
    // the wave's group of HI_GROUP slots; lane L takes the pairs at g0 + 2L and
    // g0 + 128 + 2L, so every load and store instruction covers one contiguous
    // span (128 slots) of each stream
    const int64_t g0 = tile0 + (int64_t)(threadIdx.x >> 6) * HI_GROUP;
    const int64_t q0 = g0 + 2 * (int64_t)__lane_id(), q1 = q0 + HI_GROUP / 2;
    const bool full = g0 + HI_GROUP <= n;   // uniform
    const int grp = __builtin_amdgcn_readfirstlane((int)(g0 >> HI_GROUP_LOG2));
    const bool has = __builtin_amdgcn_readfirstlane((int)(g0 < n)) != 0;   // the wave holds slots below n
    const int hdr = has ? a.HG[grp] : 0;
    unsigned ws[PPT];
    int wc[PPT];
    double us[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) wc[k] = 0;
    if (full) {
        const uvec2 pa = ld16<NT, uvec2>(a.HP + q0), pb = ld16<NT, uvec2>(a.HP + q1);
        const dvec2 ua = ld16<NT, dvec2>(a.UH + q0), ub = ld16<NT, dvec2>(a.UH + q1);
        ws[0] = pa.x; ws[1] = pa.y; ws[2] = pb.x; ws[3] = pb.y;
        us[0] = ua.x; us[1] = ua.y; us[2] = ub.x; us[3] = ub.y;
        if (hdr < 0) {
            const ivec2 ca = ld16<NT, ivec2>(a.HW + q0), cb = ld16<NT, ivec2>(a.HW + q1);
            wc[0] = ca.x; wc[1] = ca.y; wc[2] = cb.x; wc[3] = cb.y;
        }
    } else {
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int64_t p = (k < 2 ? q0 : q1) + (k & 1);
            ws[k] = p < n ? a.HP[p] : HI_DEAD;
            us[k] = p < n ? a.UH[p] : 0.0;
            if (hdr < 0 && p < n) wc[k] = a.HW[p];
        }
    }
    int cs[PPT];
    unsigned fs[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        cs[k] = ws[k] != HI_DEAD ? hi_cell(ws[k], hdr, wc[k]) : -1;
        fs[k] = ws[k] & HI_FRAC_MASK;
    }
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        float g;
        int j;
        const int jc = gather_face_f32(N, cs[k], hi_offset(fs[k]), g, j);
        const double k0 = c.qmdt * a.EZ[jc], k1 = c.qmdt * a.EZ[jc + 1];
        const double Ei = k0 + (double)g * (k1 - k0);
        const double lo = j < 0 ? k0 : Ei;
        us[k] += j >= N - 1 ? k1 : lo;            // the kick: us holds u^{n+1/2} from here on
    }
    DepAcc acc;
    acc.init(a.ctr);
    bool split;
    // the wave's old cells: when they lie in two consecutive cells, every lane
    // takes the lower one as its current channel base, so the flush is one run
    {
        int lo_o = INT_MAX, hi_o = INT_MIN;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            if (cs[k] >= 0) {
                lo_o = cs[k] < lo_o ? cs[k] : lo_o;
                hi_o = cs[k] > hi_o ? cs[k] : hi_o;
            }
        }
        lo_o = hdr >= 0 ? hdr : wave_min_i32(lo_o);
        hi_o = wave_max_i32(hi_o);
        if (hi_o >= lo_o && hi_o - lo_o <= 1) acc.cf = lo_o;
        // wider: the two pairs of a lane lie 128 slots apart, so the current
        // is flushed after the first pair (each flush then sees the cells of
        // 128 consecutive slots)
        split = hi_o >= lo_o && hi_o - lo_o > 1;
    }
    const double mscale = c.dtdz * 16777216.0, fscale = c.twoP * 0x1p-24;
    bool big = true;
#pragma unroll
    for (int k = 0; k < PPT; ++k) big = big && (cs[k] < 0 || fabs(us[k]) >= 0x1p19);
    const bool all_big = __all(big);
#pragma unroll
    for (int pr = 0; pr < 2; ++pr) {
        if (all_big) {
#pragma unroll
            for (int k = 2 * pr; k < 2 * pr + 2; ++k) {
                push_one_hi<true>(c, a.J, us[k], mscale, fscale, cs[k], fs[k], acc);
                __builtin_amdgcn_sched_barrier(0);
            }
        } else {
#pragma unroll
            for (int k = 2 * pr; k < 2 * pr + 2; ++k) {
                push_one_hi<false>(c, a.J, us[k], mscale, fscale, cs[k], fs[k], acc);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        if (pr == 0 && split) acc.flush_current(a.J);
    }
    // the group's new form: narrow, based at its lowest live cell, if the live cells span <= HI_SPAN
    int lo_c = INT_MAX, hi_c = INT_MIN;
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        if (cs[k] >= 0) {
            lo_c = cs[k] < lo_c ? cs[k] : lo_c;
            hi_c = cs[k] > hi_c ? cs[k] : hi_c;
        }
    }
    lo_c = wave_min_i32(lo_c);
    hi_c = wave_max_i32(hi_c);
    const int nh = lo_c == INT_MAX ? 0 : (hi_c - lo_c <= HI_SPAN ? lo_c : HI_WIDE);
#pragma unroll
    for (int k = 0; k < PPT; ++k) ws[k] = cs[k] >= 0 ? hi_word(cs[k], fs[k], nh) : HI_DEAD;
    if (full) {
        st16<NT, uvec2>(a.HP + q0, uvec2{ws[0], ws[1]});
        st16<NT, uvec2>(a.HP + q1, uvec2{ws[2], ws[3]});
        st16<NT, dvec2>(a.UH + q0, dvec2{us[0], us[1]});
        st16<NT, dvec2>(a.UH + q1, dvec2{us[2], us[3]});
        if (nh < 0) {
            st16<NT, ivec2>(a.HW + q0, ivec2{cs[0], cs[1]});
            st16<NT, ivec2>(a.HW + q1, ivec2{cs[2], cs[3]});
        }
    } else {
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int64_t p = (k < 2 ? q0 : q1) + (k & 1);
            if (p < n) {
                a.HP[p] = ws[k];
                a.UH[p] = us[k];
                if (nh < 0) a.HW[p] = cs[k];
            }
        }
    }
    if (__lane_id() == 0 && has) a.HG[grp] = nh;
    acc.flush_current(a.J);
    if (a.hist) {
        int64_t key[PPT];
        bool live[PPT];
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            live[k] = cs[k] >= 0;
            key[k] = live[k] ? sort_key_f32(c, cs[k], hi_offset(fs[k]), fabs(us[k]) >= a.u_hi) : 0;
        }
        hist_add<PPT>(a.hist, key, live);
    }
}

// Item k of a tube's FP32-bulk push, whose streams hold n_lo and n_hi slots:
// the low stream's tiles of BLOCK*F32_PPT_LO slots come first, then the high
// stream's tiles of BLOCK*F32_PPT_HI slots, one tile per item.  Items past
// both streams return at once.  As the two streams together hold at most
// `capacity` slots, ceil(capacity / (BLOCK*F32_PPT_HI)) + 1 items cover any
// split of the slots, with the idle ones at the end.
template <int BLOCK, int NT>
__device__ __forceinline__ void push_item_f32(const Consts &c, const Push32Args &a, int64_t k, int64_t n_lo,
                                              int64_t n_hi)
{
    constexpr int64_t SPAN = (int64_t)BLOCK * F32_PPT_LO;
    const int64_t items_lo = (n_lo + SPAN - 1) / SPAN;
    if (k < items_lo) {
        push_tile_lo<BLOCK, NT>(c, a, n_lo, k * SPAN);
        return;
    }
    const int64_t tile0 = (k - items_lo) * ((int64_t)BLOCK * F32_PPT_HI);
    if (tile0 < n_hi) push_tile_hi<BLOCK, NT>(c, a, n_hi, tile0);
}

}  // namespace pcpic
