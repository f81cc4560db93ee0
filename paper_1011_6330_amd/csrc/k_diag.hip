// k_diag.hip -- diagnostics: discrete Gauss residual (divergence equation of
// eq. 2 with d/dr -> 1/R) and the signed-gamma profile of sec. 3 (returning
// electrons counted with negative gamma).  All reductions are integer or
// max/min on ordered bit images, so every result is independent of the
// order in which particles are visited.
#include <math.h>

#include "pcpic_internal.h"
#include "wave.h"

namespace pcpic {

// G_i = (E_z,i+1/2 - E_z,i-1/2)/dz + E_r,i/R - 4 pi (rho_i - rho_GJ,i), nodes 1..N-1.
__global__ __launch_bounds__(256) void k_gauss(Consts c, const double *ez, const double *er,
                                               const int64_t *w, const double *rho_gj, double *g,
                                               DevCounters *ctr)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double a = 0.0;
    if (i <= c.N) {
        double gi = 0.0;
        if (i >= 1 && i < c.N) {
            const double rho = (c.qmP * (double)w[i]) / c.dz;
            const double d = (ez[i] - ez[i - 1]) / c.dz + er[i] / c.R;
            gi = d - c.fourpi * (rho - rho_gj[i]);
        }
        g[i] = gi;
        a = fabs(gi);
    }
    const long long m = wave_max_i64(__builtin_bit_cast(long long, a));
    if (__lane_id() == 0 && m != 0) atomicMax(&ctr->gauss_max_bits, (unsigned long long)m);
}

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
    if (i == 0) ctr->gauss_max_bits = 0;
}

// Signed gamma sign(u) sqrt(1 + u^2) binned uniformly in x.  Per bin: count,
// 128-bit fixed-point sum in units of 2^-32 (integer part and fraction summed
// separately, then combined exactly), min and max.
__global__ __launch_bounds__(256) void k_profile(Consts c, int nb, const double *__restrict__ X,
                                                 const double *__restrict__ U, const DevCounters *ctr,
                                                 long long *cnt, unsigned long long *lo, long long *hi,
                                                 long long *mn, long long *mx)
{
    const int64_t n = ctr->n_slots;
    for (int64_t base = (int64_t)blockIdx.x * 256; base < n; base += (int64_t)gridDim.x * 256) {
        const int64_t p = base + threadIdx.x;
        const double x = p < n ? X[p] : -1.0;
        bool want = x >= 0.0;
        int64_t bin = 0, gi = 0, gf = 0;
        long long ob = 0;
        if (want) {
            const double u = U[p];
            double t = u * u;
            t = 1.0 + t;
            const double gam = sqrt(t);
            const double sg = u < 0.0 ? -gam : gam;
            bin = (int64_t)floor((x * (double)nb) / (double)c.N);
            if (bin < 0) bin = 0;
            if (bin > nb - 1) bin = nb - 1;
            const double fl = floor(sg);
            gi = (int64_t)fl;
            gf = (int64_t)rint((sg - fl) * 4294967296.0);
            ob = ordered_bits(sg);
        }
        unsigned long long pend = __ballot(want);
        while (pend) {
            const int leader = __ffsll(pend) - 1;
            const int64_t lb = __shfl(bin, leader);
            const bool mine = want && bin == lb;
            const int64_t sc = wave_sum_i64(mine ? 1 : 0);
            const int64_t si = wave_sum_i64(mine ? gi : 0);
            const int64_t sf = wave_sum_i64(mine ? gf : 0);
            const long long smin = wave_min_i64(mine ? ob : 0x7fffffffffffffffLL);
            const long long smax = wave_max_i64(mine ? ob : (long long)0x8000000000000000ULL);
            if ((int)__lane_id() == leader) {
                atomicAdd((unsigned long long *)&cnt[lb], (unsigned long long)sc);
                atomic_add_i128(&lo[lb], &hi[lb], ((__int128)si << 32) + (__int128)sf);
                atomicMin(&mn[lb], smin);
                atomicMax(&mx[lb], smax);
            }
            pend &= ~__ballot(mine);
            want = want && !mine;
        }
    }
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

hipError_t launch_profile(pic_handle *h, int nb)
{
    const Consts &c = h->c;
    Workspace &w = h->ws;
    const int nbk = nb > 0 ? nb : 1;
    hipLaunchKernelGGL(k_profile_clear, dim3((unsigned)((nbk + 255) / 256)), dim3(256), 0, h->stream, nbk,
                       w.pcount, w.plo, w.phi128, w.pmin, w.pmax, w.ctr);
    if (nb > 0 && h->p.precision == PIC_FP32_BULK) return launch_profile32(h, nb);
    if (nb > 0)
        hipLaunchKernelGGL(k_profile, dim3(h->n_cu * 8), dim3(256), 0, h->stream, c, nb, w.x[h->pbuf],
                           w.u[h->pbuf], w.ctr, w.pcount, w.plo, w.phi128, w.pmin, w.pmax);
    return hipGetLastError();
}

}  // namespace pcpic
