// k_field.hip -- grid kernels: rho_GJ, Poisson initialisation (eq. 4), the
// leap-frog update of the reduced Maxwell system (eq. 3) fused with the
// space-charge-limited injection at the base (sec. 2).
//
// Every floating-point expression is written with the operand order of the
// step's definition and compiled with -ffp-contract=off, so the results are
// bit-identical to an IEEE double evaluation of the same formulas.
#include <math.h>

#include "diag_body.h"
#include "pcpic_internal.h"
#include "short_math.h"
#include "wave.h"
#include "field_body.h"
#include "sort_body.h"

namespace pcpic {

__global__ __launch_bounds__(256) void k_rho_gj(Consts c, const double *knots, double *rho,
                                                DevCounters *ctr)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double a = 0.0;
    if (i <= c.N) {
        const double r = rho_node(c, knots, i);
        rho[i] = r;
        a = fabs(r);
    }
    // max |rho_GJ| for the Gauss normalisation (non-negative doubles order as integers)
    long long m = wave_max_i64(__builtin_bit_cast(long long, a));
    if (__lane_id() == 0) atomicMax(&ctr->rho_max_bits, (unsigned long long)m);
}

// CIC node weights of the live particles (node weight W_i = S_i - S_{i-1}).
__global__ __launch_bounds__(256) void k_weights(Consts c, const double *__restrict__ X,
                                                 const DevCounters *ctr, unsigned long long *w)
{
    int64_t lo, hi;
    block_range(ctr->n_slots, gridDim.x, blockIdx.x, lo, hi);
    WeightAcc acc;
    for (int64_t base = lo; base < hi; base += 256) {
        const int64_t p = base + threadIdx.x;
        const double x = p < hi ? X[p] : -1.0;
        const bool live = x >= 0.0 && x < (double)c.N;
        int64_t cell = 0, F = 0;
        if (live) {
            const double cd = floor(x);
            cell = (int64_t)cd;
            F = (int64_t)rint((x - cd) * c.twoP);
        }
        acc.add(w, live, cell, c.oneP, F);
    }
    acc.flush(w);
}

// Right-hand side of eq. (4) times dz^2 on nodes 1..N; node N carries the
// mirror-doubled particle weight (phi' = 0 at the tube end: phi, rho even about N).
// PIC_GR_ALPHA: rho_GJ / alpha at the node.
__global__ __launch_bounds__(256) void k_poisson_rhs(Consts c, const int64_t *w, const double *rho_gj,
                                                     double *rhs)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x + 1;
    if (i > c.N) return;
    const int64_t wi = (i == c.N) ? 2 * w[i] : w[i];
    const double rho = (c.qmP * (double)wi) / c.dz;
    const double rg = (c.flags & PIC_GR_ALPHA) ? rho_gj[i] / gr_alpha_node(c, i) : rho_gj[i];
    const double t = rho - rg;
    rhs[i] = -(c.cpois * t);
}

// Thomas algorithm for phi_{i-1} + bdiag phi_i + phi_{i+1} = rhs_i (row N: 2 phi_{N-1}),
// phi_0 = 0: c'_i = 1/m_i and d'_i = (rhs_i - a d'_{i-1})/m_i with m_i = b_i - a c'_{i-1}
// (a = 2 on row N, else 1), then phi_i = d'_i - c'_i phi_{i+1}.  The recurrence is
// sequential: one lane runs it while the block stages the operands through LDS in
// chunks.  The lane takes rows in runs of TH_RUN, two register sets in turn, so the
// next run's operands are on their way from LDS while the current run computes and
// the chain holds only arithmetic:
//  * the divisions use the reciprocal of m_i (hardware estimate, two Newton steps)
//    for both quotients, each with one residual correction: the operations of the
//    general correctly rounded division when its range scaling does not apply, so
//    the bits are the division's; a run whose operands leave that range (ThRange)
//    is done again with plain divisions;
//  * without the lapse every row below N has the same diagonal, so once c'_i equals
//    c'_{i-1} it stays fixed (m and its reciprocal too) and only d' is left to run.
constexpr int TH_CHUNK = 2048;
constexpr int TH_RUN = 16;

// The range in which the division's scaling and special-case steps do nothing:
// denominators within [2^-300, 2^300] and numerators within [2^-600, 2^400] in
// magnitude.  A run tracks the smallest and largest magnitudes it meets (plain
// min/max, off the chain) and is checked once at its end; a NaN anywhere in the
// run reaches its last d'.
struct ThRange {
    double nlo, nhi, mlo, mhi;
    __device__ __forceinline__ void init() { nlo = mlo = INFINITY; nhi = mhi = 0.0; }
    __device__ __forceinline__ void num(double n) { nlo = fmin(nlo, fabs(n)); nhi = fmax(nhi, fabs(n)); }
    __device__ __forceinline__ void den(double m) { mlo = fmin(mlo, fabs(m)); mhi = fmax(mhi, fabs(m)); }
    __device__ __forceinline__ bool ok(double last) const
    {
        return nlo >= 0x1p-600 && nhi <= 0x1p+400 && mlo >= 0x1p-300 && mhi <= 0x1p+300 && isfinite(last);
    }
};

__device__ __forceinline__ double th_diag(const Consts &c, int64_t i)
{
    // PIC_GR_ALPHA: diagonal -(2 + (dz/R)^2 / alpha_i^2)
    return (c.flags & PIC_GR_ALPHA) ? -(2.0 + c.h2 / gr_alpha2(c, (double)i * c.dz)) : c.bdiag;
}

// Lane 0's forward state: c'_{i-1}, d'_{i-1}, and once c' is fixed, m and 1/m.
struct ThFwd {
    double pc, pd, mst, rst;
    bool fixed;
};

// TH_RUN rows with a = 1 (row 1 < i < N) from their operands s and diagonals bd,
// written to od (d') and oc (c'); false (state untouched) if an operand left the
// fast range.
template <bool FIXED>
__device__ __forceinline__ bool th_run_fast(const double (&s)[TH_RUN], const double (&bd)[TH_RUN], ThFwd &f,
                                            bool gr, double *od, double *oc)
{
    double ci[TH_RUN], di[TH_RUN];
    ThRange rg;
    rg.init();
    double pc = f.pc, pd = f.pd;
    if (FIXED) rg.den(f.mst);
#pragma unroll
    for (int k = 0; k < TH_RUN; ++k) {
        const double n = s[k] - pd;
        rg.num(n);
        if (FIXED) {
            pd = nr_div(n, f.mst, f.rst);
        } else {
            const double m = bd[k] - pc;
            const double r = nr_recip(m);
            rg.den(m);
            pc = fma(fma(-m, r, 1.0), r, r);
            pd = nr_div(n, m, r);
        }
        ci[k] = pc;
        di[k] = pd;
    }
    if (!rg.ok(pd)) return false;
#pragma unroll
    for (int k = 0; k < TH_RUN; ++k) {
        od[k] = di[k];
        if (!FIXED) oc[k] = ci[k];   // a fixed c' is filled in by the block afterwards
    }
    if (!FIXED && !gr && ci[TH_RUN - 1] == ci[TH_RUN - 2]) {
        f.fixed = true;
        f.mst = bd[TH_RUN - 1] - pc;
        f.rst = nr_recip(f.mst);
    }
    f.pc = pc;
    f.pd = pd;
    return true;
}

// The same rows with plain divisions.
__device__ __forceinline__ void th_run_plain(const double (&s)[TH_RUN], const double (&bd)[TH_RUN], ThFwd &f,
                                             double *od, double *oc)
{
#pragma unroll
    for (int k = 0; k < TH_RUN; ++k) {
        const double m = bd[k] - f.pc;
        f.pc = 1.0 / m;
        f.pd = (s[k] - f.pd) / m;
        od[k] = f.pd;
        oc[k] = f.pc;
    }
}

__device__ __forceinline__ void th_run(const Consts &c, const double (&s)[TH_RUN], int64_t i0, ThFwd &f,
                                       double *od, double *oc)
{
    const bool gr = (c.flags & PIC_GR_ALPHA) != 0;
    double bd[TH_RUN];
    if (gr) {
#pragma unroll
        for (int k = 0; k < TH_RUN; ++k) bd[k] = th_diag(c, i0 + k);
    } else {
#pragma unroll
        for (int k = 0; k < TH_RUN; ++k) bd[k] = c.bdiag;
    }
    const bool ok = f.fixed ? th_run_fast<true>(s, bd, f, gr, od, oc) : th_run_fast<false>(s, bd, f, gr, od, oc);
    if (!ok) th_run_plain(s, bd, f, od, oc);
}

// One row of any kind (row 1, row N, or a row outside a run), plain divisions.
__device__ __forceinline__ void th_row(const Consts &c, int64_t i, double s, ThFwd &f, double *od, double *oc)
{
    const double bd = th_diag(c, i);
    if (i == 1) {
        f.pc = 1.0 / bd;
        f.pd = s / bd;
    } else {
        const double a = (i == c.N) ? 2.0 : 1.0;
        const double m = bd - a * f.pc;
        f.pc = 1.0 / m;
        f.pd = (s - a * f.pd) / m;
    }
    *od = f.pd;
    *oc = f.pc;
}

__device__ __forceinline__ void thomas_block(const Consts &c, const double *rhs, double *cp, double *dp, double *phi)
{
    __shared__ double sa[TH_CHUNK];      // operands: rhs (forward), d' (backward)
    __shared__ double sb[TH_CHUNK];      // c'
    __shared__ double sd[TH_CHUNK];      // results: d' (forward), phi (backward)
    __shared__ int s_fix[2];             // chunk rows [s_fix[0], s_fix[1]) hold the fixed c'
    __shared__ double s_cfix;
    const int64_t N = c.N;
    ThFwd f{0.0, 0.0, 0.0, 0.0, false};
    // forward elimination, i = 1..N
    for (int64_t base = 1; base <= N; base += TH_CHUNK) {
        const int cnt = (int)((N - base + 1) < TH_CHUNK ? (N - base + 1) : TH_CHUNK);
        __syncthreads();
        for (int t = threadIdx.x; t < cnt; t += 256) sa[t] = rhs[base + t];
        __syncthreads();
        if (threadIdx.x == 0) {
            int t = 0;
            for (; t < cnt && base + t < 2; ++t) th_row(c, base + t, sa[t], f, sd + t, sb + t);
            // runs of rows with a = 1, two register sets in turn
            const int tend = (int)((N - base) < (int64_t)cnt ? (N - base) : (int64_t)cnt);   // rows below N
            double A[TH_RUN], B[TH_RUN];
            int fix_lo = f.fixed ? t : cnt;   // first row of the runs taken with c' fixed
            if (t + TH_RUN <= tend) {
#pragma unroll
                for (int k = 0; k < TH_RUN; ++k) A[k] = sa[t + k];
                while (true) {
                    const bool nb = t + 2 * TH_RUN <= tend;
                    if (nb)
#pragma unroll
                        for (int k = 0; k < TH_RUN; ++k) B[k] = sa[t + TH_RUN + k];
                    th_run(c, A, base + t, f, sd + t, sb + t);
                    t += TH_RUN;
                    if (f.fixed && fix_lo == cnt) fix_lo = t;
                    if (!nb) break;
                    const bool na = t + 2 * TH_RUN <= tend;
                    if (na)
#pragma unroll
                        for (int k = 0; k < TH_RUN; ++k) A[k] = sa[t + TH_RUN + k];
                    th_run(c, B, base + t, f, sd + t, sb + t);
                    t += TH_RUN;
                    if (f.fixed && fix_lo == cnt) fix_lo = t;
                    if (!na) break;
                }
            }
            s_fix[0] = fix_lo < t ? fix_lo : cnt;
            s_fix[1] = fix_lo < t ? t : cnt;
            s_cfix = f.pc;
            for (; t < cnt; ++t) th_row(c, base + t, sa[t], f, sd + t, sb + t);
        }
        __syncthreads();
        const int flo = s_fix[0], fhi = s_fix[1];
        const double cfix = s_cfix;
        for (int t = threadIdx.x; t < cnt; t += 256) {
            dp[base + t] = sd[t];
            cp[base + t] = (t >= flo && t < fhi) ? cfix : sb[t];
        }
    }
    __syncthreads();
    // back substitution, i = N..1
    double next = 0.0;
    for (int64_t top = N; top >= 1; top -= TH_CHUNK) {
        const int64_t lo = top - TH_CHUNK + 1 > 1 ? top - TH_CHUNK + 1 : 1;
        const int cnt = (int)(top - lo + 1);
        __syncthreads();
        for (int t = threadIdx.x; t < cnt; t += 256) { sa[t] = dp[lo + t]; sb[t] = cp[lo + t]; }
        __syncthreads();
        if (threadIdx.x == 0) {
            int t = cnt - 1;
            if (top == N) {
                next = sa[t];             // phi_N = d'_N
                sd[t] = next;
                --t;
            }
            // runs of rows downwards, two register sets in turn
            double DA[TH_RUN], EA[TH_RUN], DB[TH_RUN], EB[TH_RUN];
            if (t >= TH_RUN - 1) {
#pragma unroll
                for (int k = 0; k < TH_RUN; ++k) {
                    DA[k] = sa[t - k];
                    EA[k] = sb[t - k];
                }
                while (true) {
                    const bool nb = t - TH_RUN >= TH_RUN - 1;
                    if (nb)
#pragma unroll
                        for (int k = 0; k < TH_RUN; ++k) {
                            DB[k] = sa[t - TH_RUN - k];
                            EB[k] = sb[t - TH_RUN - k];
                        }
#pragma unroll
                    for (int k = 0; k < TH_RUN; ++k) {
                        next = DA[k] - EA[k] * next;
                        sd[t - k] = next;
                    }
                    t -= TH_RUN;
                    if (!nb) break;
                    const bool na = t - TH_RUN >= TH_RUN - 1;
                    if (na)
#pragma unroll
                        for (int k = 0; k < TH_RUN; ++k) {
                            DA[k] = sa[t - TH_RUN - k];
                            EA[k] = sb[t - TH_RUN - k];
                        }
#pragma unroll
                    for (int k = 0; k < TH_RUN; ++k) {
                        next = DB[k] - EB[k] * next;
                        sd[t - k] = next;
                    }
                    t -= TH_RUN;
                    if (!na) break;
                }
            }
            for (; t >= 0; --t) {
                next = sa[t] - sb[t] * next;
                sd[t] = next;
            }
        }
        __syncthreads();
        for (int t = threadIdx.x; t < cnt; t += 256) phi[lo + t] = sd[t];
    }
    if (threadIdx.x == 0) phi[0] = 0.0;
}

__global__ __launch_bounds__(256) void k_thomas(Consts c, const double *rhs, double *cp, double *dp,
                                                double *phi)
{
    thomas_block(c, rhs, cp, dp, phi);
}

// The same solve for many tubes of a batch at once, one block per listed tube.
__global__ __launch_bounds__(256) void k_thomas_batch(const TubeDev *tubes, const int32_t *list)
{
    const TubeDev &T = tubes[list[blockIdx.x]];
    thomas_block(T.c, generic(T.rhs), generic(T.cp), generic(T.dp), generic(T.phi));
}

// Current of one drift step of the loaded beam, no kick (steady start,
// PIC_B_STEADY_INIT): J_{i+1/2} += S_i(x) - S_i(x + (dt/dz) v), v = u / sqrt(1 + u^2),
// in the push's fixed point.  One atomic per touched face (once per run).
__device__ __forceinline__ void drift_current(const Consts &c, double x, double u, unsigned long long *J)
{
    const int64_t N = c.N;
    double t = u * u;
    t = 1.0 + t;
    const double gam = sqrt(t);
    const double v = u / gam;
    const double x1 = (c.flags & PIC_GR_ALPHA) ? x + c.dtdz * (gr_alpha2(c, x * c.dz) * v) : x + c.dtdz * v;
    const double c0d = floor(x), c1d = floor(x1);
    const int64_t c0 = (int64_t)c0d, c1 = (int64_t)c1d;
    const double F0 = rint((x - c0d) * c.twoP), F1 = rint((x1 - c1d) * c.twoP);
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
    if (va != 0.0) atomicAdd(J + c0, (unsigned long long)(long long)va);
    if (hb && vb != 0.0) atomicAdd(J + c1, (unsigned long long)(long long)vb);
}

__global__ __launch_bounds__(256) void k_drift_current_f64(Consts c, const double *X, const double *U,
                                                           const DevCounters *ctr, unsigned long long *J)
{
    const int64_t n = ctr->n_slots;
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < n; p += (int64_t)gridDim.x * 256) {
        const double x = X[p];
        if (x >= 0.0) drift_current(c, x, U[p], J);
    }
}

__global__ __launch_bounds__(256) void k_drift_current_f32(Consts c, Streams s, const DevCounters *ctr,
                                                           unsigned long long *J)
{
    const int64_t nl = ctr->n_slots, nh = ctr->n_slots_hi;
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < nl + nh; p += (int64_t)gridDim.x * 256) {
        const bool hi = p >= nl;
        const int64_t q = hi ? p - nl : p;
        float off = 0.0f;
        int cell;
        if (hi) cell = hi_slot(s, q, off);
        else { cell = s.CL[q]; off = s.OL[q]; }
        if (cell < 0) continue;
        const double x = (double)cell + (double)off;
        drift_current(c, x, hi ? s.UH[q] : (double)s.UL[q], J);
    }
}

// B_phi = 4 pi R j: (dt/R) B = 4 pi q_m 2^-P J (PIC_GR_ALPHA: divided by alpha at
// the face, from alpha B/R = 4 pi alpha j), then J is cleared.
__global__ __launch_bounds__(256) void k_b_from_current(Consts c, int64_t *J, double *b)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < c.N) {
        const double bi = (c.c4 * (double)J[i]) / c.dtR;
        b[i] = (c.flags & PIC_GR_ALPHA) ? bi / gr_alpha_face(c, i) : bi;
        J[i] = 0;
    }
}

// E_z = -dphi/dz at faces, E_r = phi/R at nodes (PIC_GR_ALPHA: phi/(alpha R)),
// B_phi = 0, J = 0, f32 kick array.
__global__ __launch_bounds__(256) void k_fields_from_phi(Consts c, const double *phi, double *ez,
                                                         double *er, double *b, float *k32, int64_t *j0,
                                                         int64_t *j1)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i > c.N) return;
    er[i] = ((c.flags & PIC_GR_ALPHA) ? phi[i] / gr_alpha_node(c, i) : phi[i]) / c.R;
    if (i < c.N) {
        const double e = -((phi[i + 1] - phi[i]) / c.dz);
        ez[i] = e;
        b[i] = 0.0;
        if (k32) k32[i] = (float)(c.qmdt * e);
        j0[i] = 0;
        j1[i] = 0;
    }
}

__global__ __launch_bounds__(256) void k_fill_i64(int64_t *p, int64_t n, int64_t v)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ __launch_bounds__(256) void k_field_inject(Consts c, FieldArgs a)
{
    field_tile(c, a, blockIdx.x, 256);
}

// FP32-bulk: the f32 kick array from E_z (after the caller overwrote the fields).
__global__ __launch_bounds__(256) void k_kick(Consts c, const double *ez, float *k32)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < c.N) k32[i] = (float)(c.qmdt * ez[i]);
}

// Check appended particles in slots [base, base + n): 0 <= x < N and u finite.
__global__ __launch_bounds__(256) void k_check_append(Consts c, const double *X, const double *U, int64_t base,
                                                      int64_t n, DevCounters *ctr)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    bool bad = false;
    if (i < n) {
        const double x = X[base + i], u = U[base + i];
        bad = !(x >= 0.0 && x < (double)c.N) || !isfinite(u);
    }
    const int64_t nb = wave_sum_i64(bad ? 1 : 0);
    if (__lane_id() == 0 && nb) atomicAdd((unsigned long long *)&ctr->bad_inputs, (unsigned long long)nb);
}

// Commit n appended particles (slots [n_slots, n_slots + n)) unless any failed the check.
__global__ void k_commit_append(DevCounters *ctr, int64_t n)
{
    if (threadIdx.x == 0 && blockIdx.x == 0 && ctr->bad_inputs == 0) {
        ctr->n_slots += n;
        ctr->n_alive += n;
    }
}

static inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

hipError_t launch_rho_gj(pic_handle *h)
{
    const Consts &c = h->c;
    hipLaunchKernelGGL(k_rho_gj, dim3(grid_for(c.N + 1, 256)), dim3(256), 0, h->stream, c, h->ws.knots,
                       h->ws.rho_gj, h->ws.ctr);
    return hipGetLastError();
}

hipError_t launch_weights(pic_handle *h, int64_t *w_out)
{
    const Consts &c = h->c;
    hipLaunchKernelGGL(k_fill_i64, dim3(grid_for(c.N + 1, 256)), dim3(256), 0, h->stream, w_out,
                       c.N + 1, (int64_t)0);
    if (h->p.precision == PIC_FP32_BULK) return launch_weights32(h, w_out);
    hipLaunchKernelGGL(k_weights, dim3(h->n_cu * 8), dim3(256), 0, h->stream, c, h->ws.x[h->pbuf],
                       h->ws.ctr, (unsigned long long *)w_out);
    return hipGetLastError();
}

// Right-hand side of eq. (4) from the loaded charge (before the solve).
hipError_t launch_poisson_rhs(pic_handle *h)
{
    const Consts &c = h->c;
    Workspace &w = h->ws;
    hipError_t e = launch_weights(h, w.w);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_poisson_rhs, dim3(grid_for(c.N, 256)), dim3(256), 0, h->stream, c, w.w,
                       w.rho_gj, w.rhs);
    return hipGetLastError();
}

// E_z, E_r, B_phi = 0, cleared J and the kick arrays from the solved phi.
hipError_t launch_fields_from_phi(pic_handle *h)
{
    const Consts &c = h->c;
    Workspace &w = h->ws;
    const int f = h->fbuf;
    hipLaunchKernelGGL(k_fields_from_phi, dim3(grid_for(c.N + 1, 256)), dim3(256), 0, h->stream, c,
                       w.phi, w.ez[f], w.er[f], w.b[f], h->p.precision == PIC_FP32_BULK ? w.k32 : nullptr,
                       w.j[0], w.j[1]);
    if (c.flags & PIC_B_STEADY_INIT) {
        // steady start: B_phi from the current the loaded beam carries (J is clear here)
        unsigned long long *J = (unsigned long long *)w.j[h->jbuf];
        const unsigned g = (unsigned)(h->n_cu * 8);
        const int b = h->pbuf;
        if (h->p.precision == PIC_FP32_BULK)
            hipLaunchKernelGGL(k_drift_current_f32, dim3(g), dim3(256), 0, h->stream, c,
                               Streams{w.cl[b], w.ol[b], w.ul[b], w.hp[b], w.hw[b], w.hg[b], w.uh[b]}, w.ctr, J);
        else
            hipLaunchKernelGGL(k_drift_current_f64, dim3(g), dim3(256), 0, h->stream, c, w.x[b], w.u[b], w.ctr, J);
        hipLaunchKernelGGL(k_b_from_current, dim3(grid_for(c.N, 256)), dim3(256), 0, h->stream, c, w.j[h->jbuf],
                           w.b[f]);
    }
    return hipGetLastError();
}

hipError_t launch_poisson(pic_handle *h)
{
    hipError_t e = launch_poisson_rhs(h);
    if (e != hipSuccess) return e;
    Workspace &w = h->ws;
    hipLaunchKernelGGL(k_thomas, dim3(1), dim3(256), 0, h->stream, h->c, w.rhs, w.cp, w.dp, w.phi);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return launch_fields_from_phi(h);
}

// Solve eq. (4) for the listed tubes of a batch together (one Thomas block per tube).
hipError_t launch_thomas_batch(pic_handle *b, const int32_t *d_list, int n)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_thomas_batch, dim3((unsigned)n), dim3(256), 0, b->stream, b->d_tubes, d_list);
    return hipGetLastError();
}

hipError_t launch_field_inject(pic_handle *h)
{
    const Consts &c = h->c;
    Workspace &w = h->ws;
    const int f = h->fbuf, g = 1 - h->fbuf;
    const bool f32 = h->p.precision == PIC_FP32_BULK;
    const int b = h->pbuf;
    FieldArgs a{w.ez[f], w.er[f], w.b[f], w.ez[g], w.er[g], w.b[g], w.j[h->jbuf], w.j[1 - h->jbuf],
                f32 ? w.k32 : nullptr, f32 ? nullptr : w.x[b], f32 ? nullptr : w.u[b],
                f32 ? w.cl[b] : nullptr, f32 ? w.ol[b] : nullptr, f32 ? w.ul[b] : nullptr, w.ctr,
                h->d_sched, h->sched_first, h->sched_n,
                h->hist_on ? (unsigned long long *)w.cell_count : nullptr,
                f32 && 0.0 >= h->u_hi ? sort_low_keys(c) : 0};
    hipLaunchKernelGGL(k_field_inject, dim3(grid_for(c.N, 256 * FIELD_CPT)), dim3(256), 0, h->stream, c, a);
    return hipGetLastError();
}

// Field update + injection with explicit field buffers and injection target
// (used by the adjoint recompute; FP64 only).
hipError_t launch_field_ptrs(pic_handle *h, const double *ezo, const double *ero, const double *bo, double *ezn,
                             double *ern, double *bn, double *X, double *U)
{
    Workspace &w = h->ws;
    FieldArgs a{ezo, ero, bo, ezn, ern, bn, w.j[h->jbuf], w.j[1 - h->jbuf], nullptr, X, U,
                nullptr, nullptr, nullptr, w.ctr, h->d_sched, h->sched_first, h->sched_n};
    hipLaunchKernelGGL(k_field_inject, dim3(grid_for(h->c.N, 256 * FIELD_CPT)), dim3(256), 0, h->stream, h->c, a);
    return hipGetLastError();
}

hipError_t launch_check_append(pic_handle *h, int64_t base, int64_t n)
{
    if (n > 0)
        hipLaunchKernelGGL(k_check_append, dim3(grid_for(n, 256)), dim3(256), 0, h->stream, h->c,
                           h->ws.x[h->pbuf], h->ws.u[h->pbuf], base, n, h->ws.ctr);
    return hipGetLastError();
}

hipError_t launch_commit_append(pic_handle *h, int64_t n)
{
    hipLaunchKernelGGL(k_commit_append, dim3(1), dim3(64), 0, h->stream, h->ws.ctr, n);
    return hipGetLastError();
}


hipError_t launch_zero_i64(pic_handle *h, int64_t *p, int64_t n)
{
    if (n > 0)
        hipLaunchKernelGGL(k_fill_i64, dim3(grid_for(n, 256)), dim3(256), 0, h->stream, p, n, (int64_t)0);
    return hipGetLastError();
}

// The f32 kick array of the FP32-bulk low stream from the current E_z (the
// FP64 path and the high stream form the kick from E_z itself: nothing to do).
hipError_t launch_kick(pic_handle *h)
{
    if (h->p.precision != PIC_FP32_BULK) return hipSuccess;
    hipLaunchKernelGGL(k_kick, dim3(grid_for(h->c.N, 256)), dim3(256), 0, h->stream, h->c, h->ws.ez[h->fbuf],
                       h->ws.k32);
    return hipGetLastError();
}

}  // namespace pcpic
