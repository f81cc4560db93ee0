// k_adjoint.hip -- reverse-mode gradient of the mean exit Lorentz factor
// through the FP64 PIC step, with every discrete decision frozen (injection
// counts, exits and returns, cell crossings; rint taken as the identity).
//
// One reverse step s, given the adjoints of the state after the step
// (particles lx, lu per slot; fields lez = dL/dE_z^{s+1}, ler = dL/dE_r^{s+1},
// lb = dL/dB^{s+1/2}) and the recorded state before it (slots X_s, U_s, E_z^s),
// plus lbp = dL/dB^{s+1/2} through its uses in E_r^{s+1} and E_z^{s+1}:
//   1. per slot: recompute the push, route the adjoints through the move, the
//      gather (into lk, the adjoint of the kick array) and the fixed-point
//      current (J enters E_z^{s+1} with weight -c4);
//   2. lez, ler, lb <- adjoints of E^s, B^{s-1/2} (transposed leap-frog of
//      eq. 3), and lbp of step s-1 from them.
// After step 0 the field adjoints go through the transposed Poisson problem of
// eq. (4) to dL/d rho_GJ.  Slots keep their particle across steps (no sort in an
// adjoint run), so the particle adjoints are updated in place.
#include <math.h>

#include "pcpic_internal.h"
#include "wave.h"

namespace pcpic {

typedef double dvec2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ double wave_sum_f64(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// ---- order-independent sums --------------------------------------------
//
// Several waves add to the same word (the kick adjoint of a face, the rate
// gradient).  Each wave's partial sum is formed in a fixed lane order, then
// rounded to a multiple of the quantum 2^(e - 60), where the exponent e of the
// reverse step bounds every partial sum of the step by 2^e (adj_exponent), and
// added as an integer below 2^60 split into its low 32 bits and the rest: two
// integer atomics into an unsigned low word and a signed high word, which hold
// the sums of up to 2^32 addends exactly.  The total does not depend on the
// order in which the waves arrive, so the gradient is the same bits on every
// run; the rounding is 2^-60 of the step's bound.

// dst += v (|v| < 2^e) in units of 2^(e - 60), rounded to nearest.
__device__ __forceinline__ void fixed_add(unsigned long long *lo, long long *hi, double v, int e)
{
    const long long t = (long long)rint(ldexp(v, 60 - e));
    const unsigned long long tl = (unsigned long long)t & 0xffffffffull;
    const long long th = t >> 32;
    if (tl) atomicAdd(lo, tl);
    if (th) atomicAdd((unsigned long long *)hi, (unsigned long long)th);
}

// The word pair (lo, hi) in units of 2^(e - 60) as a double.
__device__ __forceinline__ double double_of(unsigned long long lo, long long hi, int e)
{
    return ldexp((double)hi * 0x1p32 + (double)lo, e - 60);
}

// Smallest e with b < 2^e (b >= 0), kept above the subnormal range.
__device__ __forceinline__ int adj_exponent(double b)
{
    int ex = -900;
    if (b > 0.0) (void)frexp(b, &ex);                  // b = f 2^ex, 0.5 <= f < 1
    return ex < -900 ? -900 : ex;
}

__device__ __forceinline__ double max_of_bits(unsigned long long b) { return __builtin_bit_cast(double, b); }

// Wave maximum of |v| into *dst (non-negative doubles order as their bit images).
__device__ __forceinline__ void wave_max_abs(unsigned long long *dst, double v)
{
    const long long m = __builtin_bit_cast(long long, wave_max_f64_to63(fabs(v)));
    if (__lane_id() == 63 && m != 0) atomicMax(dst, (unsigned long long)m);
}

// Block maximum of |a| and |b| (256 threads) into *da and *db: one atomic per
// block and quantity, skipped when the word already holds as much (it only
// grows, so a stale read costs at most a redundant atomic).  Every thread of
// the block must call it.
__device__ __forceinline__ void block_max_abs2(unsigned long long *da, unsigned long long *db, double a, double b)
{
    __shared__ long long s_m[2][4];
    const long long ma = __builtin_bit_cast(long long, wave_max_f64_to63(fabs(a)));
    const long long mb = __builtin_bit_cast(long long, wave_max_f64_to63(fabs(b)));
    const int w = threadIdx.x >> 6;
    if (__lane_id() == 63) {
        s_m[0][w] = ma;
        s_m[1][w] = mb;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        long long m = s_m[threadIdx.x][0];
        for (int k = 1; k < 4; ++k) m = s_m[threadIdx.x][k] > m ? s_m[threadIdx.x][k] : m;
        unsigned long long *d = threadIdx.x == 0 ? da : db;
        if (m != 0 && (unsigned long long)m > __hip_atomic_load(d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            atomicMax(d, (unsigned long long)m);
    }
}

// dst[key] += val for every lane with `want`: lanes with the same key in
// consecutive positions form a run, a segmented DPP scan sums each run in lane
// order, and the run's last lane adds the run total in fixed point.
// Wave-collective.
__device__ __forceinline__ void wave_add_runs_fixed(unsigned long long *lo, long long *hi, int key, double val,
                                                    bool want, int e)
{
    const WaveRun r = wave_runs_i32(key, want);
    const double s = run_sum_to_tail(want ? val : 0.0, r.rank);
    if (want && (int)__lane_id() == r.end - 1 && s != 0.0) fixed_add(lo + key, hi + key, s, e);
}

__global__ __launch_bounds__(256) void k_copy_slots(const double *X, const double *U, double *Xc, double *Uc,
                                                    const DevCounters *ctr)
{
    const int64_t n = ctr->n_slots;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        Xc[i] = X[i];
        Uc[i] = U[i];
    }
}

__global__ void k_record_slots(const DevCounters *ctr, int64_t *dst)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = ctr->n_slots;
}

__global__ __launch_bounds__(256) void k_fill_f64(double *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = 0.0;
}

// The quanta of a reverse step from the maxima of the adjoints it starts from
// (word set k, filled by the step before):
//   |lu1t| <= max(max|lu|, 1/n_exit) + (dt/dz)(max|lx| + 2^P |c4| max|lez|)
// bounds every particle's kick-adjoint addend (gamma >= 1), and a run of the
// wave adds at most 128 of them (two slots per lane); a particle's
// rate-gradient term is at most 2 2^P |c4| max|lez|, 128 of them per wave.  Every block that needs the
// exponents forms them from the same words, so they agree everywhere.  The
// word sets rotate over three: step r reads set r mod 3, fills set r+1 and
// clears set r+2.
__device__ __forceinline__ void step_exponents(const Consts &c, const AdjScale *sc, int k, int64_t n_exit, int &e_k,
                                               int &e_g)
{
    const double mlu = max_of_bits(sc->max_lu[k]), mlx = max_of_bits(sc->max_lx[k]);
    const double mlez = max_of_bits(sc->max_lez[k]);
    const double seed = n_exit > 0 ? 1.0 / (double)n_exit : 0.0;
    const double lj = c.twoP * fabs(c.c4) * mlez;
    const double bound = (mlu > seed ? mlu : seed) + c.dtdz * (mlx + lj);
    e_k = adj_exponent(128.0 * bound);
    e_g = adj_exponent(256.0 * lj);
}

struct AdjPartArgs {
    const double *X, *U;      // slots before the step
    const double *ez;         // E_z^s (the kick array is (q/m) dt E_z^s)
    const int64_t *n_s;       // slots before the step
    const int64_t *n_next;    // slots after the step (injected ones beyond n_s)
    int64_t n_pre;            // slots loaded before the run (injected class from here on)
    int64_t n_exit;           // exits of the whole run (loss normalisation)
    double *lx, *lu;          // slot adjoints, in place
    const double *lez;        // dL/dE_z^{s+1}
    unsigned long long *lk_lo; // dL/dK^s, 128-bit fixed point (accumulated)
    long long *lk_hi;
    AdjScale *sc;             // quanta of the step (word set rot); maxima of the new slot adjoints (set rot + 1)
    int rot;
};

// One slot's reverse step: the forward push recomputed exactly, then its
// transpose.  lx_in, lu_in: the slot's adjoints after the step.  The new slot
// adjoints, the kick-adjoint terms (faces ka, kb) and the rate-gradient term.
struct AdjSlot {
    double nlx, nlu, va, vb, gr;
    int ka, kb;
    bool wa, wb;
};

__device__ __forceinline__ AdjSlot adj_slot(const Consts &c, const AdjPartArgs &a, int64_t p, double x, double u,
                                            double lx_in, double lu_in)
{
    const int N = (int)c.N;
    AdjSlot o{0.0, 0.0, 0.0, 0.0, 0.0, 0, 0, false, false};
    const double s = x - 0.5;
    int clamp = 0, jj = 0;
    double g = 0.0, dEdx = 0.0;
    const double kN1 = c.qmdt * a.ez[N - 1], k0 = c.qmdt * a.ez[0];
    double kj = 0.0, kj1 = 0.0;
    if (s < 0.0) {
        clamp = 1;
    } else if (s >= (double)(N - 1)) {
        clamp = 2;
    } else {
        jj = (int)floor(s);
        g = s - (double)jj;
        kj = c.qmdt * a.ez[jj];
        kj1 = c.qmdt * a.ez[jj + 1];
        dEdx = kj1 - kj;
    }
    const double E = clamp == 1 ? k0 : (clamp == 2 ? kN1 : kj + g * (kj1 - kj));
    const double u1 = u + E;
    double t = u1 * u1;
    t = 1.0 + t;
    const double gam = sqrt(t);
    const double v = u1 / gam;
    const double x1 = x + c.dtdz * v;
    const double c0d = floor(x), c1d = floor(x1);
    const int c0 = (int)c0d, c1 = (int)c1d;
    double lx1 = 0.0, lu1 = 0.0;
    if (x1 >= (double)N) {
        lu1 = a.n_exit > 0 ? (u1 / gam) / (double)a.n_exit : 0.0;   // d gamma/du = u/gamma
    } else if (x1 >= 0.0) {
        lx1 = lx_in;
        lu1 = lu_in;
    }
    // current: J_i = S_i(x) - S_i(x1), dS_i/dx = -2^P in cell i; E_z^{s+1} -= c4 J
    if (c1 >= 0 && c1 < N) lx1 += c.twoP * (-c.c4 * a.lez[c1]);
    const double lx0J = -c.twoP * (-c.c4 * a.lez[c0]);
    if (p >= a.n_pre) {
        // injected class: its deposit times -c4 times the adjoint of E_z^{s+1}
        const double F0 = rint((x - c0d) * c.twoP), F1 = rint((x1 - c1d) * c.twoP);
        double d0, d1 = 0.0;
        if (c1 == c0) {
            d0 = F1 - F0;
        } else if (c1 > c0) {
            d0 = c.twoP - F0;
            d1 = c1 < N ? F1 : 0.0;
        } else {
            d0 = -F0;
            d1 = c1 >= 0 ? F1 - c.twoP : 0.0;
        }
        o.gr += d0 * (-c.c4 * a.lez[c0]);
        if (d1 != 0.0) o.gr += d1 * (-c.c4 * a.lez[c1]);
    }
    // move: x1 = x + (dt/dz) u1/gamma(u1), dv/du = 1/gamma^3
    const double lu1t = lu1 + lx1 * c.dtdz / (gam * gam * gam);
    o.nlx = lx1 + lx0J + lu1t * dEdx;
    o.nlu = lu1t;
    // kick: E = K_j (1 - g) + K_{j+1} g
    if (clamp == 1) { o.ka = 0; o.va = lu1t; o.wa = true; }
    else if (clamp == 2) { o.ka = N - 1; o.va = lu1t; o.wa = true; }
    else { o.ka = jj; o.va = lu1t * (1.0 - g); o.kb = jj + 1; o.vb = lu1t * g; o.wa = true; o.wb = true; }
    return o;
}

// 2. particles: two consecutive slots per thread (16-byte accesses).  A slot
// removed before the step keeps its adjoints; a slot injected at the end of
// the step (n_s <= p < n_next: created at rest, no dependence) gets 0.  The
// two slots' kick-adjoint terms are merged where they fall on the same face
// (the usual case, as consecutive slots sit in the same or the next cell), so
// the wave usually sums two keyed terms per thread instead of four.
__global__ __launch_bounds__(256) void k_adj_particles(Consts c, AdjPartArgs a)
{
    const int64_t ns = *a.n_s, nn = *a.n_next;
    if ((int64_t)blockIdx.x * 512 >= nn) return;      // a block past every slot (uniform): nothing to add
    const int64_t p0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 2;
    int e_k, e_g;
    step_exponents(c, a.sc, a.rot, a.n_exit, e_k, e_g);
    double x[2] = {-1.0, -1.0}, u[2] = {0.0, 0.0}, lxi[2] = {0.0, 0.0}, lui[2] = {0.0, 0.0};
    const bool pair = p0 + 2 <= nn;
    if (pair) {
        const dvec2 xv = *(const dvec2 *)(a.X + p0), uv = *(const dvec2 *)(a.U + p0);
        const dvec2 lxv = *(const dvec2 *)(a.lx + p0), luv = *(const dvec2 *)(a.lu + p0);
        x[0] = xv.x; x[1] = xv.y; u[0] = uv.x; u[1] = uv.y;
        lxi[0] = lxv.x; lxi[1] = lxv.y; lui[0] = luv.x; lui[1] = luv.y;
    } else if (p0 < nn) {
        x[0] = a.X[p0]; u[0] = a.U[p0]; lxi[0] = a.lx[p0]; lui[0] = a.lu[p0];
    }
    AdjSlot o[2];
    double nlx[2], nlu[2], mlx = 0.0, mlu = 0.0;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int64_t p = p0 + k;
        o[k] = AdjSlot{0.0, 0.0, 0.0, 0.0, 0.0, 0, 0, false, false};
        nlx[k] = lxi[k];
        nlu[k] = lui[k];
        if (p < ns) {
            if (x[k] >= 0.0) {
                o[k] = adj_slot(c, a, p, x[k], u[k], lxi[k], lui[k]);
                nlx[k] = o[k].nlx;
                nlu[k] = o[k].nlu;
                mlx = fmax(mlx, fabs(o[k].nlx));
                mlu = fmax(mlu, fabs(o[k].nlu));
            }
        } else {
            nlx[k] = 0.0;
            nlu[k] = 0.0;
        }
    }
    if (pair) {
        *(dvec2 *)(a.lx + p0) = dvec2{nlx[0], nlx[1]};
        *(dvec2 *)(a.lu + p0) = dvec2{nlu[0], nlu[1]};
    } else if (p0 < nn) {
        a.lx[p0] = nlx[0];
        a.lu[p0] = nlu[0];
    }
    // the second slot's terms join the first slot's where the face is the same
    AdjSlot &f = o[0], &h = o[1];
    if (h.wa && !f.wa) { f.ka = h.ka; f.va = h.va; f.wa = true; h.wa = false; }
    if (h.wb && !f.wb && !(f.wa && h.wb && h.kb == f.ka)) { f.kb = h.kb; f.vb = h.vb; f.wb = true; h.wb = false; }
    if (h.wa && h.ka == f.ka) { f.va += h.va; h.wa = false; }
    else if (h.wa && f.wb && h.ka == f.kb) { f.vb += h.va; h.wa = false; }
    if (h.wb && f.wb && h.kb == f.kb) { f.vb += h.vb; h.wb = false; }
    wave_add_runs_fixed(a.lk_lo, a.lk_hi, f.ka, f.va, f.wa, e_k);
    wave_add_runs_fixed(a.lk_lo, a.lk_hi, f.kb, f.vb, f.wb, e_k);
    if (__ballot(h.wa)) wave_add_runs_fixed(a.lk_lo, a.lk_hi, h.ka, h.va, h.wa, e_k);
    if (__ballot(h.wb)) wave_add_runs_fixed(a.lk_lo, a.lk_hi, h.kb, h.vb, h.wb, e_k);
    // the rate gradient: only slots of the injected class have a term
    const double gr = o[0].gr + o[1].gr;
    if (__ballot(gr != 0.0)) {
        const double gs = wave_sum_f64_to63(gr);
        if (__lane_id() == 63 && gs != 0.0) fixed_add(&a.sc->g_lo, &a.sc->g_hi, gs, e_g);
    }
    const int nx = a.rot == 2 ? 0 : a.rot + 1;
    block_max_abs2(&a.sc->max_lx[nx], &a.sc->max_lu[nx], mlx, mlu);
}

// 2. transposed leap-frog of step s: adjoints of E_z^s, E_r^s, B^{s-1/2}, with
//    the kick adjoint taken out of fixed point (and cleared for the next step),
//    then lbp of step s-1: dL/dB^{s-1/2} through its uses in E_r^s and E_z^s.
//    E_r adjoints ping-pong (ler -> lern) since lbp needs the neighbour's new
//    E_r adjoint, which this thread forms again from the old values; lbp
//    ping-pongs for the same reason.  The maxima of the new E_z adjoint go to
//    word set rot + 1, set rot + 2 is cleared for the step after, and thread 0
//    adds the step's rate gradient to the total (one addition per step, in step
//    order) and clears the step's sum.
__device__ __forceinline__ double ler_next(const Consts &c, const double *ler, const double *lbp, int64_t j)
{
    double a = ler[j];
    if (j <= c.N - 1) a += c.dtdz * lbp[j];
    if (j >= 1) a -= c.dtdz * lbp[j - 1];
    return a;
}

__global__ __launch_bounds__(256) void k_adj_fields(Consts c, double *lez, const double *ler, double *lern,
                                                    double *lb, const double *lbp, double *lbpn,
                                                    unsigned long long *lk_lo, long long *lk_hi, AdjScale *sc,
                                                    int rot, int64_t n_exit)
{
    const int64_t N = c.N;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int e_k, e_g;
    step_exponents(c, sc, rot, n_exit, e_k, e_g);
    const int r1 = rot == 2 ? 0 : rot + 1, r2 = r1 == 2 ? 0 : r1 + 1;
    double nez = 0.0;
    if (i <= N) lern[i] = ler_next(c, ler, lbp, i);
    if (i < N) {
        const double lk = double_of(lk_lo[i], lk_hi[i], e_k);
        lk_lo[i] = 0;
        lk_hi[i] = 0;
        nez = lez[i] - c.dtR * lbp[i] + c.qmdt * lk;
        lez[i] = nez;
        const double nb = lbp[i];
        lb[i] = nb;
        double a = nb + c.dtR * nez;
        if (i >= 1 && i <= N - 1) a -= c.dtdz * ler_next(c, ler, lbp, i);
        if (i + 1 <= N - 1) a += c.dtdz * ler_next(c, ler, lbp, i + 1);
        if (i == N - 1) a += c.tw * ler_next(c, ler, lbp, N);
        lbpn[i] = a;
    }
    wave_max_abs(&sc->max_lez[r1], nez);
    if (i == 0) {
        sc->grate += double_of(sc->g_lo, sc->g_hi, e_g);
        sc->g_lo = 0;
        sc->g_hi = 0;
        sc->max_lu[r2] = 0;
        sc->max_lx[r2] = 0;
        sc->max_lez[r2] = 0;
    }
}

// dL/dphi_m from E_z = -dphi/dz (faces) and E_r = phi/R (nodes), m = 1..N.
__global__ __launch_bounds__(256) void k_adj_phi(Consts c, const double *lez, const double *ler, double *g)
{
    const int64_t N = c.N;
    const int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x + 1;
    if (m > N) return;
    double a = -lez[m - 1] / c.dz + ler[m] / c.R;
    if (m <= N - 1) a += lez[m] / c.dz;
    g[m] = a;
}

// Transposed Thomas solve A^T y = g (A: eq. (4) rows 1..N-1 = 1, bdiag, 1 and
// row N = 2, bdiag; A^T carries the 2 on the super-diagonal of row N-1), then
// dL/d rho_GJ,i = 4 pi dz^2 y_i (the right-hand side is -4 pi dz^2 (rho - rho_GJ)).
constexpr int ADJ_CHUNK = 2048;
__global__ __launch_bounds__(256) void k_adj_poisson(Consts c, const double *g, double *cp, double *dp,
                                                     double *g_rho)
{
    __shared__ double sa[ADJ_CHUNK];
    __shared__ double sb[ADJ_CHUNK];
    __shared__ double carry[2];
    const int64_t N = c.N;
    if (threadIdx.x == 0) { carry[0] = 0.0; carry[1] = 0.0; }
    for (int64_t base = 1; base <= N; base += ADJ_CHUNK) {
        const int cnt = (int)((N - base + 1) < ADJ_CHUNK ? (N - base + 1) : ADJ_CHUNK);
        __syncthreads();
        for (int t = threadIdx.x; t < cnt; t += 256) sa[t] = g[base + t];
        __syncthreads();
        if (threadIdx.x == 0) {
            double pc = carry[0], pd = carry[1];
            for (int t = 0; t < cnt; ++t) {
                const int64_t i = base + t;
                const double sup = (i <= N - 1) ? ((i == N - 1) ? 2.0 : 1.0) : 0.0;
                double ci, di;
                if (i == 1) {
                    ci = sup / c.bdiag;
                    di = sa[t] / c.bdiag;
                } else {
                    const double m = c.bdiag - pc;
                    ci = sup / m;
                    di = (sa[t] - pd) / m;
                }
                sa[t] = di;
                sb[t] = ci;
                pc = ci;
                pd = di;
            }
            carry[0] = pc;
            carry[1] = pd;
        }
        __syncthreads();
        for (int t = threadIdx.x; t < cnt; t += 256) { dp[base + t] = sa[t]; cp[base + t] = sb[t]; }
    }
    __syncthreads();
    if (threadIdx.x == 0) carry[0] = 0.0;
    for (int64_t top = N; top >= 1; top -= ADJ_CHUNK) {
        const int64_t lo = top - ADJ_CHUNK + 1 > 1 ? top - ADJ_CHUNK + 1 : 1;
        const int cnt = (int)(top - lo + 1);
        __syncthreads();
        for (int t = threadIdx.x; t < cnt; t += 256) { sa[t] = dp[lo + t]; sb[t] = cp[lo + t]; }
        __syncthreads();
        if (threadIdx.x == 0) {
            double next = carry[0];
            for (int t = cnt - 1; t >= 0; --t) {
                const int64_t i = lo + t;
                const double v = (i == N) ? sa[t] : sa[t] - sb[t] * next;
                sa[t] = v;
                next = v;
            }
            carry[0] = next;
        }
        __syncthreads();
        const double fac = c.fourpi * (c.dz * c.dz);
        for (int t = threadIdx.x; t < cnt; t += 256) g_rho[lo + t] = fac * sa[t];
    }
    if (threadIdx.x == 0) g_rho[0] = 0.0;
}

// dL/d(parameters of rho_GJ) from the node gradient: knots (hat weights times
// -(1 - kappa/eta^3)), kappa (theta(z)/eta^3 per node), amplitude A.
// One block; out[0] = kappa, out[1] = A, out[2 + k] = knot k.
__global__ __launch_bounds__(256) void k_adj_params(Consts c, const double *knots, const double *g_rho, double *out)
{
    __shared__ double s_red[2][4];
    const int64_t N = c.N;
    const int K = c.n_knots;
    double gk = 0.0, ga = 0.0;
    for (int64_t i = threadIdx.x; i <= N; i += 256) {
        const double gr = g_rho[i];
        const double z = (double)i * c.dz;
        if (c.rho_kind == PIC_RHO_UNIFORM) {
            ga += -gr;
            continue;
        }
        const double eta = 1.0 + z / c.r_star;
        const double e3 = eta * eta * eta;
        const double fd = 1.0 - c.kappa / e3;
        if (c.rho_kind == PIC_RHO_FRAME_DRAG) {
            ga += gr * (-fd);
            gk += gr * (c.rho_amp / e3);
        } else if (c.rho_kind == PIC_RHO_GR) {
            const double br = fd + c.gr_s * sqrt(eta);
            const double al = sqrt(1.0 - c.gr_g / eta);
            ga += gr * (-(br / al));
            gk += gr * (c.rho_amp / (e3 * al));
        } else {
            const double s = (z * (double)(K - 1)) / c.length;
            int kk = (int)floor(s);
            if (kk > K - 2) kk = K - 2;
            if (kk < 0) kk = 0;
            const double g = s - (double)kk;
            const double th = knots[kk] + g * (knots[kk + 1] - knots[kk]);
            gk += gr * (th / e3);
        }
    }
    // knot k: its hat weight at the nodes of its two intervals, summed in node
    // order by one thread
    if (c.rho_kind == PIC_RHO_KNOTS) {
        for (int k = threadIdx.x; k < K; k += 256) {
            double acc = 0.0;
            const int64_t i0 = (int64_t)floor(((double)(k - 1) * (double)N) / (double)(K - 1)) - 1;
            const int64_t i1 = (int64_t)ceil(((double)(k + 1) * (double)N) / (double)(K - 1)) + 1;
            for (int64_t i = (i0 > 0 ? i0 : 0); i <= (i1 < N ? i1 : N); ++i) {
                const double z = (double)i * c.dz;
                const double s = (z * (double)(K - 1)) / c.length;
                int kk = (int)floor(s);
                if (kk > K - 2) kk = K - 2;
                if (kk < 0) kk = 0;
                if (kk != k && kk + 1 != k) continue;
                const double g = s - (double)kk;
                const double eta = 1.0 + z / c.r_star;
                const double fd = 1.0 - c.kappa / (eta * eta * eta);
                acc += g_rho[i] * (kk == k ? -(1.0 - g) * fd : -g * fd);
            }
            out[2 + k] = acc;
        }
    }
    gk = wave_sum_f64(gk);
    ga = wave_sum_f64(ga);
    if (__lane_id() == 0) {
        s_red[0][threadIdx.x >> 6] = gk;
        s_red[1][threadIdx.x >> 6] = ga;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        out[0] = s_red[0][0] + s_red[0][1] + s_red[0][2] + s_red[0][3];
        out[1] = s_red[1][0] + s_red[1][1] + s_red[1][2] + s_red[1][3];
    }
}

// ---- launchers ----

static inline unsigned gridn(int64_t n) { return (unsigned)((n + 255) / 256); }

hipError_t launch_copy_slots(pic_handle *h, const double *X, const double *U, double *Xc, double *Uc)
{
    hipLaunchKernelGGL(k_copy_slots, dim3(h->n_cu * 8), dim3(256), 0, h->stream, X, U, Xc, Uc, h->ws.ctr);
    return hipGetLastError();
}

hipError_t launch_record_slots(pic_handle *h, int64_t *dst)
{
    hipLaunchKernelGGL(k_record_slots, dim3(1), dim3(64), 0, h->stream, h->ws.ctr, dst);
    return hipGetLastError();
}

hipError_t launch_zero_f64(pic_handle *h, double *p, int64_t n)
{
    if (n > 0) hipLaunchKernelGGL(k_fill_f64, dim3(gridn(n) < 4096 ? gridn(n) : 4096), dim3(256), 0, h->stream, p, n);
    return hipGetLastError();
}

hipError_t launch_adj_step(pic_handle *h, const AdjStepPtrs &s)
{
    const Consts &c = h->c;
    AdjPartArgs a{s.X, s.U, s.ez, s.n_s, s.n_next, s.n_pre, s.n_exit, s.lx, s.lu, s.lez, s.lk_lo, s.lk_hi,
                  s.scale, s.rot};
    hipLaunchKernelGGL(k_adj_particles, dim3((unsigned)((c.cap + 511) / 512)), dim3(256), 0, h->stream, c, a);
    hipLaunchKernelGGL(k_adj_fields, dim3(gridn(c.N + 1)), dim3(256), 0, h->stream, c, s.lez, s.ler, s.lern, s.lb,
                       s.lbp, s.lbpn, s.lk_lo, s.lk_hi, s.scale, s.rot, s.n_exit);
    return hipGetLastError();
}

hipError_t launch_adj_finish(pic_handle *h, const double *lez, const double *ler, double *gphi, double *cp,
                             double *dp, double *g_rho, double *params)
{
    const Consts &c = h->c;
    hipLaunchKernelGGL(k_adj_phi, dim3(gridn(c.N)), dim3(256), 0, h->stream, c, lez, ler, gphi);
    hipLaunchKernelGGL(k_adj_poisson, dim3(1), dim3(256), 0, h->stream, c, gphi, cp, dp, g_rho);
    hipLaunchKernelGGL(k_adj_params, dim3(1), dim3(256), 0, h->stream, c, h->ws.knots, g_rho, params);
    return hipGetLastError();
}

}  // namespace pcpic
