// k_diag.hip -- diagnostics: discrete Gauss residual (divergence equation of
// eq. 2 with d/dr -> 1/R) and the signed-gamma profile of sec. 3 (returning
// electrons counted with negative gamma).  All reductions are integer or
// max/min on ordered bit images, so every result is independent of the
// order in which particles are visited.
#include <math.h>

#include "pcpic_internal.h"
#include "diag_body.h"
#include "wave.h"

namespace pcpic {

// G_i = (E_z,i+1/2 - E_z,i-1/2)/dz + E_r,i/R - 4 pi (rho_i - rho_GJ,i), nodes 1..N-1
// (PIC_GR_ALPHA: the first and the rho term times alpha_i).
__global__ __launch_bounds__(256) void k_gauss(Consts c, const double *ez, const double *er,
                                               const int64_t *w, const double *rho_gj, double *g,
                                               DevCounters *ctr)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double a = 0.0;
    if (i <= c.N) {
        double gi = 0.0;
        if (i >= 1 && i < c.N) {
            double rho = (c.qmP * (double)w[i]) / c.dz;
            double dez = (ez[i] - ez[i - 1]) / c.dz;
            if (c.flags & PIC_GR_ALPHA) {
                // alpha_i dE_z/dz + E_r/R = 4 pi (alpha_i lambda_i - rho_GJ,i)
                const double an = gr_alpha_node(c, i);
                dez = an * dez;
                rho = an * rho;
            }
            const double d = dez + er[i] / c.R;
            gi = d - c.fourpi * (rho - rho_gj[i]);
        }
        g[i] = gi;
        a = fabs(gi);
    }
    const long long m = wave_max_i64(__builtin_bit_cast(long long, a));
    if (__lane_id() == 0 && m != 0) atomicMax(&ctr->gauss_max_bits, (unsigned long long)m);
}

// Clears nb profile bins (and, with ctr, the Gauss maximum of the diagnostics).
__global__ __launch_bounds__(256) void k_profile_clear(int nb, long long *cnt, unsigned long long *lo,
                                                       long long *hi, long long *mn, long long *mx,
                                                       DevCounters *ctr)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < nb) {
        cnt[i] = 0;
        lo[i] = 0;
        hi[i] = 0;
        mn[i] = ordered_bits(INFINITY);
        mx[i] = ordered_bits(-INFINITY);
    }
    if (i == 0 && ctr) ctr->gauss_max_bits = 0;
}

// The accumulated bins in the caller's layout: counts and the 128-bit sums as
// they are, min and max back from their ordered bit images to doubles (an empty
// bin gives +inf and -inf).  Any output may be null.
__global__ __launch_bounds__(256) void k_profile_finish(int nb, ProfPtrs p, int64_t *count, uint64_t *sum_lo,
                                                        int64_t *sum_hi, double *vmin, double *vmax)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= nb) return;
    if (count) count[i] = p.cnt[i];
    if (sum_lo) sum_lo[i] = p.lo[i];
    if (sum_hi) sum_hi[i] = p.hi[i];
    if (vmin) vmin[i] = from_ordered_bits(p.mn[i]);
    if (vmax) vmax[i] = from_ordered_bits(p.mx[i]);
}

// Signed gamma sign(u) sqrt(1 + u^2) binned uniformly in x (ProfAcc): per bin
// count, 128-bit fixed-point sum in units of 2^-32, min and max.  Block b takes
// a contiguous range of the slots.
__global__ __launch_bounds__(256) void k_profile(Consts c, int nb, const double *__restrict__ X,
                                                 const double *__restrict__ U, const DevCounters *ctr, ProfOut o)
{
    int64_t lo, hi;
    block_range(ctr->n_slots, gridDim.x, blockIdx.x, lo, hi);
    ProfAcc acc;
    for (int64_t base = lo; base < hi; base += 256) {
        const int64_t p = base + threadIdx.x;
        const double x = p < hi ? X[p] : -1.0;
        const bool want = x >= 0.0;
        int64_t bin = 0, gi = 0, gf = 0;
        long long ob = 0;
        if (want) prof_values(c, nb, x, U[p], bin, gi, gf, ob);
        acc.add(o, want, bin, gi, gf, ob);
    }
    acc.flush(o);
}

hipError_t launch_gauss(pic_handle *h)
{
    const Consts &c = h->c;
    Workspace &w = h->ws;
    hipError_t e = launch_weights(h, w.w);
    if (e != hipSuccess) return e;
    const int f = h->fbuf;
    hipLaunchKernelGGL(k_gauss, dim3((unsigned)((c.N + 1 + 255) / 256)), dim3(256), 0, h->stream, c,
                       w.ez[f], w.er[f], w.w, w.rho_gj, w.gauss, w.ctr);
    return hipGetLastError();
}

hipError_t launch_profile_into(pic_handle *h, int nb, const ProfPtrs &p, bool clear_gauss)
{
    const Consts &c = h->c;
    Workspace &w = h->ws;
    const int nbk = nb > 0 ? nb : 1;
    hipLaunchKernelGGL(k_profile_clear, dim3((unsigned)((nbk + 255) / 256)), dim3(256), 0, h->stream, nbk,
                       p.cnt, p.lo, p.hi, p.mn, p.mx, clear_gauss ? w.ctr : nullptr);
    if (nb > 0 && h->p.precision == PIC_FP32_BULK) return launch_profile32(h, nb, p);
    if (nb > 0)
        hipLaunchKernelGGL(k_profile, dim3(h->n_cu * 8), dim3(256), 0, h->stream, c, nb, w.x[h->pbuf],
                           w.u[h->pbuf], w.ctr, ProfOut{p.cnt, p.lo, p.hi, p.mn, p.mx});
    return hipGetLastError();
}

hipError_t launch_profile(pic_handle *h, int nb)
{
    Workspace &w = h->ws;
    return launch_profile_into(h, nb, ProfPtrs{w.pcount, w.plo, w.phi128, w.pmin, w.pmax}, true);
}

hipError_t launch_profile_finish(pic_handle *h, int nb, const ProfPtrs &p, int64_t *count, uint64_t *sum_lo,
                                 int64_t *sum_hi, double *vmin, double *vmax)
{
    if (nb > 0)
        hipLaunchKernelGGL(k_profile_finish, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, h->stream, nb, p,
                           count, sum_lo, sum_hi, vmin, vmax);
    return hipGetLastError();
}

}  // namespace pcpic
