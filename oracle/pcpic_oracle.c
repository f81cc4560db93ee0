/*
 * pcpic_oracle.c -- plain FP64 CPU oracle of the 1D polar-cap PIC time step.
 *
 * TEST INFRASTRUCTURE ONLY (see pcpic_oracle.h).  Serial loops, IEEE double,
 * compiled with -ffp-contract=off so that every product and sum is rounded as
 * written.  Each function names the passage of the paper it follows.
 *
 * One PIC cycle (sec. 2, Fig. A), in this order:
 *   1. equation of motion, eq. (1): gather the kick at x^n, u^{n+1/2} = u^{n-1/2} + kick,
 *      x^{n+1} = x^n + (c dt/dz) v  with v = u / sqrt(1 + u^2);
 *   2. weighting particle -> grid: the charge-conserving linear current J of the move;
 *   3. boundaries (conditions under eq. 4): x >= N leaves the tube, x < 0 returns to the star;
 *   4. Maxwell, eq. (3), leap-frog: B_phi, then E_r, then E_z;
 *   5. SCLF injection at the base (sec. 2) while the base charge is not compensated.
 */
#include "pcpic_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---- derived constants ------------------------------------------------ */

typedef struct {
    int64_t N;
    double dz, dt, dtdz, dtR, qmdt, rho0, qm, qmP, fourpi, c4, fqm, hdz, tw, twoP;
    int64_t oneP; /* 2^P as an integer */
} orc_const;

static int orc_check(const orc_cfg *c)
{
    if (!c || c->n_cells < 2 || !(c->length > 0) || !(c->radius > 0)) return -1;
    if (!(c->dt_over_dz > 0 && c->dt_over_dz < 1)) return -1;
    if (!(c->ppc > 0) || c->fp_bits < 8 || c->fp_bits > 40 || c->capacity < 0) return -1;
    if (c->rho_kind == ORC_RHO_KNOTS && (c->n_knots < 2 || !c->knots)) return -1;
    return 0;
}

/* Goldreich-Julian background at node i (eqs. 5-7).
 * Flat space, i = 0: the bracket of eq. (5) is 1 and (R_star/r)^3 is dropped, so rho_GJ = -A.
 * Frame dragging: eq. (6) with Omega replaced by Omega - omega and omega/Omega = kappa/eta^3
 * from eq. (7), alpha = f = H = 1, giving rho_GJ = -A (1 - kappa / eta^3), eta = 1 + z/R_*.
 * Knots: the amplitude A becomes a piecewise-linear theta(z) on uniform knots over [0, L]. */
static double orc_rho_node(const orc_cfg *c, double dz, int64_t i)
{
    double z = (double)i * dz;
    if (c->rho_kind == ORC_RHO_UNIFORM) return -c->rho_amp;
    double eta = 1.0 + z / c->r_star;
    double e3 = eta * eta * eta;
    double fd = 1.0 - c->kappa / e3;
    if (c->rho_kind == ORC_RHO_FRAME_DRAG) return -(c->rho_amp * fd);
    /* hat-function interpolation of the knot values */
    int64_t K = c->n_knots;
    double s = (z * (double)(K - 1)) / c->length;
    int64_t k = (int64_t)floor(s);
    if (k > K - 2) k = K - 2;
    if (k < 0) k = 0;
    double g = s - (double)k;
    double th = c->knots[k] + g * (c->knots[k + 1] - c->knots[k]);
    return -(th * fd);
}

int orc_rho_gj(const orc_cfg *c, double *rho)
{
    if (orc_check(c)) return -1;
    double dz = c->length / (double)c->n_cells;
    for (int64_t i = 0; i <= c->n_cells; ++i) rho[i] = orc_rho_node(c, dz, i);
    return 0;
}

static void orc_consts(const orc_cfg *c, const orc_state *st, orc_const *k)
{
    k->N = c->n_cells;
    k->dz = c->length / (double)c->n_cells;
    k->dtdz = c->dt_over_dz;
    k->dt = k->dtdz * k->dz;
    k->dtR = k->dt / c->radius;
    k->qmdt = c->q_over_m * k->dt;
    k->rho0 = st->rho_gj[0];
    k->qm = (k->rho0 * k->dz) / c->ppc;          /* macro-particle charge (per unit area) */
    k->twoP = ldexp(1.0, c->fp_bits);
    k->oneP = (int64_t)1 << c->fp_bits;
    k->qmP = k->qm / k->twoP;                      /* charge of one weight unit */
    k->fourpi = 4.0 * M_PI;
    k->c4 = k->fourpi * k->qmP;                    /* E_z change per unit of J */
    k->fqm = k->fourpi * k->qm;                    /* surface-field change per injected particle */
    k->hdz = 0.5 * k->dz;
    k->tw = 2.0 * k->dtdz;
}

/* ---- weighting (sec. 2: linear weighting between particles and grid) --- */

/* Cell and fixed-point offset of a position: c = floor(x), F = rint(2^P (x - c)). */
static void orc_cell(double x, int P, int64_t *cell, int64_t *F)
{
    double c = floor(x);
    double f = x - c;
    *cell = (int64_t)c;
    *F = (int64_t)rint(ldexp(f, P));
}

/* Cumulative weight left of face i+1/2: the part of the particle's linear (CIC)
 * charge that sits on nodes 0..i.  2^P if the particle is left of node i,
 * 0 if it is right of node i+1, 2^P - F inside cell i. */
static int64_t orc_S(int64_t i, int64_t cell, int64_t F, int64_t oneP)
{
    if (cell < i) return oneP;
    if (cell > i) return 0;
    return oneP - F;
}

int orc_weights(const orc_cfg *c, const double *x, int64_t n, int64_t *w)
{
    if (orc_check(c)) return -1;
    int64_t N = c->n_cells, oneP = (int64_t)1 << c->fp_bits;
    memset(w, 0, sizeof(int64_t) * (size_t)(N + 1));
    for (int64_t p = 0; p < n; ++p) {
        int64_t cell, F;
        orc_cell(x[p], c->fp_bits, &cell, &F);
        if (cell < 0 || cell >= N) continue;
        w[cell] += oneP - F;   /* node weight W_i = S_i - S_{i-1} */
        w[cell + 1] += F;
    }
    return 0;
}

/* ---- field initialisation, eq. (4) ------------------------------------ */

/* Solve d2phi/dz2 - phi/R^2 = -4 pi (rho - rho_GJ) on nodes 1..N with phi_0 = 0
 * (star surface) and phi'(L) = 0 (ghost phi_{N+1} = phi_{N-1}), by the Thomas
 * algorithm.  Node N carries the mirror-doubled particle weight (the ghost makes
 * phi and rho even about x = N).  Then E_z = -dphi/dz at faces, E_r = phi/R at
 * nodes (from d/dr -> 1/R), B_phi = 0. */
static void orc_solve_fields(const orc_cfg *c, orc_state *st)
{
    orc_const k;
    orc_consts(c, st, &k);
    int64_t N = k.N;
    orc_weights(c, st->x, st->n, st->w);
    double dz2 = k.dz * k.dz;
    double rr = k.dz / c->radius;
    double h2 = rr * rr;
    double bdiag = -(2.0 + h2);
    double cpois = k.fourpi * dz2;
    /* right-hand side d_i = -4 pi dz^2 (rho_i - rho_GJ,i) */
    for (int64_t i = 1; i <= N; ++i) {
        int64_t wi = (i == N) ? 2 * st->w[i] : st->w[i];
        double rho = (k.qmP * (double)wi) / k.dz;
        double t = rho - st->rho_gj[i];
        st->dp[i] = -(cpois * t);
    }
    /* forward sweep: sub-diagonal 1 (2 in row N), diagonal bdiag, super-diagonal 1 */
    st->cp[1] = 1.0 / bdiag;
    st->dp[1] = st->dp[1] / bdiag;
    for (int64_t i = 2; i <= N; ++i) {
        double a = (i == N) ? 2.0 : 1.0;
        double m = bdiag - a * st->cp[i - 1];
        st->cp[i] = 1.0 / m;
        st->dp[i] = (st->dp[i] - a * st->dp[i - 1]) / m;
    }
    /* back substitution */
    st->phi[0] = 0.0;
    st->phi[N] = st->dp[N];
    for (int64_t i = N - 1; i >= 1; --i) st->phi[i] = st->dp[i] - st->cp[i] * st->phi[i + 1];
    for (int64_t i = 0; i < N; ++i) st->ez[i] = -((st->phi[i + 1] - st->phi[i]) / k.dz);
    for (int64_t i = 0; i <= N; ++i) st->er[i] = st->phi[i] / c->radius;
    for (int64_t i = 0; i < N; ++i) { st->b[i] = 0.0; st->j[i] = 0; st->k[i] = k.qmdt * st->ez[i]; }
}

int orc_init(const orc_cfg *c, orc_state *st)
{
    if (orc_check(c) || !st) return -1;
    if (st->n < 0 || st->n > c->capacity) return -1;
    orc_rho_gj(c, st->rho_gj);
    st->step = 0; st->n_injected = 0; st->n_exit = 0; st->n_absorb = 0;
    st->w0 = 0; st->last_ninj = 0; st->status = 0;
    st->exit_sum_lo = 0; st->exit_sum_hi = 0; st->e_surf = 0.0;
    orc_solve_fields(c, st);
    return 0;
}

int orc_inject(const orc_cfg *c, orc_state *st, int64_t n, const double *x, const double *u)
{
    if (orc_check(c) || n < 0) return -1;
    if (st->n + n > c->capacity) return -2;
    for (int64_t p = 0; p < n; ++p) {
        if (!(x[p] >= 0.0 && x[p] < (double)c->n_cells) || !isfinite(u[p])) return -1;
    }
    for (int64_t p = 0; p < n; ++p) { st->x[st->n + p] = x[p]; st->u[st->n + p] = u[p]; }
    st->n += n;
    if (st->step == 0) orc_solve_fields(c, st);
    return 0;
}

/* ---- one PIC cycle ---------------------------------------------------- */

static void orc_add128(uint64_t *lo, int64_t *hi, int64_t v)
{
    __int128 s = ((__int128)(*hi) << 64) | (__int128)(*lo);
    s += (__int128)v;
    *lo = (uint64_t)s;
    *hi = (int64_t)(s >> 64);
}

static void orc_one_step(const orc_cfg *c, orc_state *st)
{
    orc_const k;
    orc_consts(c, st, &k);
    int64_t N = k.N;
    int P = c->fp_bits;

    /* kick array from the current E_z: K = (q/m) dt E_z */
    for (int64_t i = 0; i < N; ++i) st->k[i] = k.qmdt * st->ez[i];
    for (int64_t i = 0; i < N; ++i) st->j[i] = 0;

    int64_t w0 = 0, kept = 0;
    for (int64_t p = 0; p < st->n; ++p) {
        double x = st->x[p], u = st->u[p];
        /* gather: linear interpolation of the face values, clamped at the ends */
        double s = x - 0.5, E;
        if (s < 0.0) {
            E = st->k[0];
        } else if (s >= (double)(N - 1)) {
            E = st->k[N - 1];
        } else {
            int64_t jj = (int64_t)floor(s);
            double g = s - (double)jj;
            E = st->k[jj] + g * (st->k[jj + 1] - st->k[jj]);
        }
        /* eq. (1): d(gamma m v)/dt = q E_z, dz/dt = v, with u = gamma v (c = 1) */
        double u1 = u + E;
        double t = u1 * u1;
        t = 1.0 + t;
        double gam = sqrt(t);
        double v = u1 / gam;
        double x1 = x + k.dtdz * v;
        if (!isfinite(u1) || !isfinite(x1)) { st->status |= ORC_ST_NONFINITE; continue; }

        /* charge-conserving current: J_{i+1/2} += S_i(x^n) - S_i(x^{n+1}) on every face */
        int64_t c0, F0, c1, F1;
        orc_cell(x, P, &c0, &F0);
        orc_cell(x1, P, &c1, &F1);
        int64_t lo = c0 < c1 ? c0 : c1, hi = c0 < c1 ? c1 : c0;
        if (lo < 0) lo = 0;
        if (hi > N - 1) hi = N - 1;
        for (int64_t i = lo; i <= hi; ++i)
            st->j[i] += orc_S(i, c0, F0, k.oneP) - orc_S(i, c1, F1, k.oneP);

        if (x1 >= (double)N) {               /* leaves through the top of the tube */
            st->n_exit += 1;
            orc_add128(&st->exit_sum_lo, &st->exit_sum_hi, (int64_t)rint(ldexp(gam, 32)));
            continue;
        }
        if (x1 < 0.0) {                      /* returns to the star */
            st->n_absorb += 1;
            continue;
        }
        if (c1 == 0) w0 += k.oneP - F1;      /* node-0 weight of the survivors */
        st->x[kept] = x1;
        st->u[kept] = u1;
        ++kept;
    }
    st->n = kept;
    st->w0 = w0;

    if (!(c->flags & ORC_FREEZE_FIELDS)) {
        /* eq. (3), leap-frog: dB/dt = -dE_r/dz - E_z/R, then dE_r/dt = -dB/dz,
         * then dE_z/dt = B/R - 4 pi j.  E_r,0 = 0 (phi = 0 at the star);
         * mirror about x = N (B odd) gives the E_r,N update. */
        for (int64_t i = 0; i < N; ++i)
            st->b[i] = st->b[i] - (k.dtdz * (st->er[i + 1] - st->er[i]) + k.dtR * st->ez[i]);
        for (int64_t i = 1; i < N; ++i)
            st->er[i] = st->er[i] - k.dtdz * (st->b[i] - st->b[i - 1]);
        st->er[N] = st->er[N] + k.tw * st->b[N - 1];
        for (int64_t i = 0; i < N; ++i)
            st->ez[i] = (st->ez[i] + k.dtR * st->b[i]) - k.c4 * (double)st->j[i];
    }

    /* SCLF injection (sec. 2): the field at the surface from the node-0 Gauss law
     * over the half cell [0, dz/2]; electrons are added at x = 0 with u = 0 until
     * the base charge cancels it (never over-injecting). */
    double t1 = k.qmP * (double)w0;
    double t2 = k.rho0 * k.hdz;
    double es = st->ez[0] - k.fourpi * (t1 - t2);
    st->e_surf = es;
    int64_t ninj = 0;
    if (!(c->flags & ORC_NO_AUTO_INJECT)) {
        double ratio = es / k.fqm;
        if (ratio > 0.0) {
            double nf = floor(ratio);
            int64_t avail = c->capacity - st->n;
            if (nf > (double)avail) { ninj = avail; st->status |= ORC_ST_CAPACITY; }
            else ninj = (int64_t)nf;
        }
        for (int64_t p = 0; p < ninj; ++p) { st->x[st->n + p] = 0.0; st->u[st->n + p] = 0.0; }
        st->n += ninj;
        st->n_injected += ninj;
    }
    st->last_ninj = ninj;
    st->step += 1;
}

int orc_step(const orc_cfg *c, orc_state *st, int64_t n_steps)
{
    if (orc_check(c) || !st || n_steps < 0) return -1;
    for (int64_t s = 0; s < n_steps; ++s) orc_one_step(c, st);
    return 0;
}

/* ---- diagnostics ------------------------------------------------------ */

/* Discrete form of the divergence equation of eq. (2) with d/dr -> 1/R:
 * G_i = (E_z,i+1/2 - E_z,i-1/2)/dz + E_r,i/R - 4 pi (rho_i - rho_GJ,i). */
int orc_gauss(const orc_cfg *c, orc_state *st, double *g, double *gmax)
{
    if (orc_check(c)) return -1;
    orc_const k;
    orc_consts(c, st, &k);
    int64_t N = k.N;
    orc_weights(c, st->x, st->n, st->w);
    double rmax = 0.0, m = 0.0;
    for (int64_t i = 0; i <= N; ++i) rmax = fmax(rmax, fabs(st->rho_gj[i]));
    g[0] = 0.0; g[N] = 0.0;
    for (int64_t i = 1; i < N; ++i) {
        double rho = (k.qmP * (double)st->w[i]) / k.dz;
        double d = (st->ez[i] - st->ez[i - 1]) / k.dz + st->er[i] / c->radius;
        g[i] = d - k.fourpi * (rho - st->rho_gj[i]);
        m = fmax(m, fabs(g[i]));
    }
    *gmax = m / (k.fourpi * rmax);
    return 0;
}

/* Signed Lorentz factor sign(u) gamma (returning electrons negative), binned in x. */
int orc_profile(const orc_cfg *c, const orc_state *st, int32_t nb, int64_t *count,
                uint64_t *sum_lo, int64_t *sum_hi, double *gmin, double *gmax)
{
    if (orc_check(c) || nb < 1) return -1;
    int64_t N = c->n_cells;
    for (int32_t b = 0; b < nb; ++b) {
        count[b] = 0; sum_lo[b] = 0; sum_hi[b] = 0;
        gmin[b] = INFINITY; gmax[b] = -INFINITY;
    }
    for (int64_t p = 0; p < st->n; ++p) {
        double x = st->x[p], u = st->u[p];
        double t = u * u;
        t = 1.0 + t;
        double gam = sqrt(t);
        double sg = (u < 0.0) ? -gam : gam;
        int64_t b = (int64_t)floor((x * (double)nb) / (double)N);
        if (b < 0) b = 0;
        if (b > nb - 1) b = nb - 1;
        count[b] += 1;
        orc_add128(&sum_lo[b], &sum_hi[b], (int64_t)rint(ldexp(sg, 32)));
        if (sg < gmin[b]) gmin[b] = sg;
        if (sg > gmax[b]) gmax[b] = sg;
    }
    return 0;
}
