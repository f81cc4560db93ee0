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

#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- derived constants ------------------------------------------------ */

typedef struct {
    int64_t N;
    double dz, dt, dtdz, dtR, qmdt, rho0, qm, qmP, fourpi, c4, fqm, hdz, tw, twoP;
    int64_t oneP; /* 2^P as an integer */
    int gr;       /* ORC_GR_ALPHA */
    double cg;    /* dt (r_g/R_*) / (2 R_*): k_g = cg / eta^2 = dt alpha alpha' */
} orc_const;

static int orc_check(const orc_cfg *c)
{
    if (!c || c->n_cells < 2 || !(c->length > 0) || !(c->radius > 0)) return -1;
    if (!(c->dt_over_dz > 0 && c->dt_over_dz < 1)) return -1;
    if (!(c->ppc > 0) || c->fp_bits < 8 || c->fp_bits > 40 || c->capacity < 0) return -1;
    if (c->rho_kind == ORC_RHO_KNOTS && (c->n_knots < 2 || !c->knots)) return -1;
    if (c->rho_kind == ORC_RHO_GR &&
        (!(c->rg_over_rstar >= 0.0 && c->rg_over_rstar < 1.0) || !(fabs(c->incl) < 1.5) || !(c->r_star > 0)))
        return -1;
    if ((c->flags & ORC_GR_ALPHA) && (!(c->rg_over_rstar >= 0.0 && c->rg_over_rstar < 1.0) || !(c->r_star > 0)))
        return -1;
    return 0;
}

/* alpha^2 = 1 - r_g/r at height z (ORC_GR_ALPHA), r/R_* = eta = 1 + z/R_*. */
static double orc_alpha2(const orc_cfg *c, double z)
{
    double eta = 1.0 + z / c->r_star;
    return 1.0 - c->rg_over_rstar / eta;
}

/* alpha at node i and at face i+1/2. */
static double orc_alpha_node(const orc_cfg *c, double dz, int64_t i)
{
    return sqrt(orc_alpha2(c, (double)i * dz));
}
static double orc_alpha_face(const orc_cfg *c, double dz, int64_t i)
{
    return sqrt(orc_alpha2(c, ((double)i + 0.5) * dz));
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
    if (c->rho_kind == ORC_RHO_GR) {
        /* eq. 6 divided by the flat surface density of an inclined rotator, Omega B cos(i) / (2 pi c)
         * (the paper's n_GJ carries the cos(i)), with (R_star/r)^3 dropped as for eq. 5 and the
         * curved-space factors f = H = 1 (not given):
         *   rho_GJ = -A [ (1 - kappa/eta^3) + (3/2) eta^(1/2) theta_* tan(i) cos(varphi) ] / alpha,
         *   alpha = (1 - r_g / r)^(1/2) = (1 - (r_g/R_*) / eta)^(1/2). */
        double s = ((1.5 * c->theta_star) * tan(c->incl)) * c->cos_phi;
        double br = fd + s * sqrt(eta);
        double al = sqrt(1.0 - c->rg_over_rstar / eta);
        return -((c->rho_amp * br) / al);
    }
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
    /* macro-particle charge (per unit area); an explicit value keeps it fixed when
     * the background is varied (gradients, finite differences) */
    k->qm = c->macro_charge != 0.0 ? c->macro_charge : (k->rho0 * k->dz) / c->ppc;
    k->twoP = ldexp(1.0, c->fp_bits);
    k->oneP = (int64_t)1 << c->fp_bits;
    k->qmP = k->qm / k->twoP;                      /* charge of one weight unit */
    k->fourpi = 4.0 * M_PI;
    k->c4 = k->fourpi * k->qmP;                    /* E_z change per unit of J */
    k->fqm = k->fourpi * k->qm;                    /* surface-field change per injected particle */
    k->hdz = 0.5 * k->dz;
    k->tw = 2.0 * k->dtdz;
    k->gr = (c->flags & ORC_GR_ALPHA) != 0;
    k->cg = ((0.5 * k->dt) * c->rg_over_rstar) / c->r_star;
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
    /* right-hand side d_i = -4 pi dz^2 (rho_i - rho_GJ,i) (GR: rho_GJ,i / alpha_i) */
    for (int64_t i = 1; i <= N; ++i) {
        int64_t wi = (i == N) ? 2 * st->w[i] : st->w[i];
        double rho = (k.qmP * (double)wi) / k.dz;
        double rg = k.gr ? st->rho_gj[i] / orc_alpha_node(c, k.dz, i) : st->rho_gj[i];
        double t = rho - rg;
        st->dp[i] = -(cpois * t);
    }
    /* forward sweep: sub-diagonal 1 (2 in row N), diagonal bdiag (GR: -(2 + h2/alpha_i^2)),
     * super-diagonal 1 */
    {
        double bd = k.gr ? -(2.0 + h2 / orc_alpha2(c, k.dz)) : bdiag;
        st->cp[1] = 1.0 / bd;
        st->dp[1] = st->dp[1] / bd;
    }
    for (int64_t i = 2; i <= N; ++i) {
        double a = (i == N) ? 2.0 : 1.0;
        double bd = k.gr ? -(2.0 + h2 / orc_alpha2(c, (double)i * k.dz)) : bdiag;
        double m = bd - a * st->cp[i - 1];
        st->cp[i] = 1.0 / m;
        st->dp[i] = (st->dp[i] - a * st->dp[i - 1]) / m;
    }
    /* back substitution */
    st->phi[0] = 0.0;
    st->phi[N] = st->dp[N];
    for (int64_t i = N - 1; i >= 1; --i) st->phi[i] = st->dp[i] - st->cp[i] * st->phi[i + 1];
    for (int64_t i = 0; i < N; ++i) st->ez[i] = -((st->phi[i + 1] - st->phi[i]) / k.dz);
    for (int64_t i = 0; i <= N; ++i)
        st->er[i] = (k.gr ? st->phi[i] / orc_alpha_node(c, k.dz, i) : st->phi[i]) / c->radius;
    for (int64_t i = 0; i < N; ++i) { st->b[i] = 0.0; st->j[i] = 0; st->k[i] = k.qmdt * st->ez[i]; }
    if (c->flags & ORC_B_STEADY_INIT) {
        /* Steady start of eq. (3): with dE_z/dt = 0 the E_z update gives B_phi = 4 pi R j.
         * j is the current the loaded beam carries: the charge-conserving current of one
         * drift step with the particles' own velocities and no kick.  In the update's units,
         * (dt/R) B = 4 pi q_m 2^-P J. */
        for (int64_t p = 0; p < st->n; ++p) {
            double x = st->x[p], u = st->u[p];
            double t = u * u;
            t = 1.0 + t;
            double gam = sqrt(t);
            double v = u / gam;
            double x1 = k.gr ? x + k.dtdz * (orc_alpha2(c, x * k.dz) * v) : x + k.dtdz * v;
            int64_t c0, F0, c1, F1;
            orc_cell(x, c->fp_bits, &c0, &F0);
            orc_cell(x1, c->fp_bits, &c1, &F1);
            int64_t lo = c0 < c1 ? c0 : c1, hi = c0 < c1 ? c1 : c0;
            if (lo < 0) lo = 0;
            if (hi > N - 1) hi = N - 1;
            for (int64_t i = lo; i <= hi; ++i) st->j[i] += orc_S(i, c0, F0, k.oneP) - orc_S(i, c1, F1, k.oneP);
        }
        for (int64_t i = 0; i < N; ++i) {
            st->b[i] = (k.c4 * (double)st->j[i]) / k.dtR;
            if (k.gr) st->b[i] = st->b[i] / orc_alpha_face(c, k.dz, i);
            st->j[i] = 0;
        }
    }
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
    for (int64_t p = 0; p < n; ++p) {
        st->x[st->n + p] = x[p];
        st->u[st->n + p] = u[p];
        if (st->cls) st->cls[st->n + p] = 0;
    }
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

/* What the particle half of a step leaves behind over a range of particles. */
typedef struct {
    int64_t *j;           /* [N] current of the range's moves                     */
    int64_t *j_inj;       /* [N] injected-class part of it (NULL: not kept)        */
    int64_t w0, w0_inj;   /* node-0 weight of the survivors (all / injected class) */
    int64_t n_exit, n_absorb, kept, status;
    uint64_t exit_lo;     /* 128-bit sum of rint(gamma 2^32) over the exits        */
    int64_t exit_hi;
} orc_tally;

/* Start of a step: kick array K = (q/m) dt E_z from the current E_z; J cleared. */
static void orc_step_begin(orc_state *st, const orc_const *k)
{
    int64_t N = k->N;
    for (int64_t i = 0; i < N; ++i) st->k[i] = k->qmdt * st->ez[i];
    for (int64_t i = 0; i < N; ++i) st->j[i] = 0;
    if (st->j_inj)
        for (int64_t i = 0; i < N; ++i) st->j_inj[i] = 0;
}

/* Particles p0 .. p1-1 of the state: gather, eq. (1), the charge-conserving
 * current, the boundaries.  Survivors are written, in order, to xo/uo/clso at
 * index t->kept onwards (xo may be st->x itself: the write never passes the read). */
static void orc_push_range(const orc_cfg *c, const orc_state *st, const orc_const *k, int64_t p0, int64_t p1,
                           double *xo, double *uo, unsigned char *clso, orc_tally *t)
{
    int64_t N = k->N;
    int P = c->fp_bits;
    for (int64_t p = p0; p < p1; ++p) {
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
        double u1, gam, v, x1;
        if (k->gr) {
            /* with the lapse alpha (ORC_GR_ALPHA): du/dt = alpha (q/m) E_z - gamma alpha alpha',
             * dz/dt = alpha^2 v; midpoint gamma for gravity, midpoint alpha^2 for the move */
            double eta = 1.0 + (x * k->dz) / c->r_star;
            double a2 = 1.0 - c->rg_over_rstar / eta;
            double al = sqrt(a2);
            double kg = k->cg / (eta * eta);
            double t0 = u * u;
            t0 = 1.0 + t0;
            double g0 = sqrt(t0);
            double uh = u + 0.5 * (al * E - kg * g0);
            double th = uh * uh;
            th = 1.0 + th;
            double gh = sqrt(th);
            u1 = u + (al * E - kg * gh);
            double tt = u1 * u1;
            tt = 1.0 + tt;
            gam = sqrt(tt);
            v = u1 / gam;
            double xh = x + 0.5 * (k->dtdz * (a2 * v));
            double a2h = orc_alpha2(c, xh * k->dz);
            x1 = x + k->dtdz * (a2h * v);
        } else {
            u1 = u + E;
            double tt = u1 * u1;
            tt = 1.0 + tt;
            gam = sqrt(tt);
            v = u1 / gam;
            x1 = x + k->dtdz * v;
        }
        if (!isfinite(u1) || !isfinite(x1)) { t->status |= ORC_ST_NONFINITE; continue; }

        /* charge-conserving current: J_{i+1/2} += S_i(x^n) - S_i(x^{n+1}) on every face */
        int64_t c0, F0, c1, F1;
        orc_cell(x, P, &c0, &F0);
        orc_cell(x1, P, &c1, &F1);
        int64_t lo = c0 < c1 ? c0 : c1, hi = c0 < c1 ? c1 : c0;
        if (lo < 0) lo = 0;
        if (hi > N - 1) hi = N - 1;
        const int injected = st->cls && st->cls[p];
        for (int64_t i = lo; i <= hi; ++i) {
            const int64_t d = orc_S(i, c0, F0, k->oneP) - orc_S(i, c1, F1, k->oneP);
            t->j[i] += d;
            if (injected && t->j_inj) t->j_inj[i] += d;
        }

        if (x1 >= (double)N) {               /* leaves through the top of the tube */
            t->n_exit += 1;
            orc_add128(&t->exit_lo, &t->exit_hi, (int64_t)rint(ldexp(gam, 32)));
            continue;
        }
        if (x1 < 0.0) {                      /* returns to the star */
            t->n_absorb += 1;
            continue;
        }
        if (c1 == 0) {                       /* node-0 weight of the survivors */
            t->w0 += k->oneP - F1;
            if (injected) t->w0_inj += k->oneP - F1;
        }
        xo[t->kept] = x1;
        uo[t->kept] = u1;
        if (clso) clso[t->kept] = st->cls[p];
        t->kept += 1;
    }
}

/* End of a step, once every particle has moved and t holds the whole step's
 * tallies (its current already in st->j): counters, eq. (3), the injection. */
static void orc_step_end(const orc_cfg *c, orc_state *st, const orc_const *k, const orc_tally *t)
{
    int64_t N = k->N;
    const double rate = c->inj_rate > 0.0 ? c->inj_rate : 1.0;
    st->n = t->kept;
    st->w0 = t->w0;
    st->n_exit += t->n_exit;
    st->n_absorb += t->n_absorb;
    st->status |= t->status;
    {
        __int128 s = ((__int128)st->exit_sum_hi << 64) | (__int128)st->exit_sum_lo;
        s += ((__int128)t->exit_hi << 64) | (__int128)t->exit_lo;
        st->exit_sum_lo = (uint64_t)s;
        st->exit_sum_hi = (int64_t)(s >> 64);
    }
    const int64_t w0 = t->w0, w0_inj = t->w0_inj;

    if (!(c->flags & ORC_FREEZE_FIELDS) && k->gr) {
        /* the same leap-frog with the lapse (ORC_GR_ALPHA): alpha at faces (af) and nodes
         * (an) on each term of eq. (3) as in the header; the deposit's J is alpha j */
        const double dz = k->dz;
        for (int64_t i = 0; i < N; ++i) {
            double af = orc_alpha_face(c, dz, i);
            double d = orc_alpha_node(c, dz, i + 1) * st->er[i + 1] - orc_alpha_node(c, dz, i) * st->er[i];
            st->b[i] = st->b[i] - (k->dtdz * (af * d) + k->dtR * (af * st->ez[i]));
        }
        for (int64_t i = 1; i < N; ++i) {
            double d = orc_alpha_face(c, dz, i) * st->b[i] - orc_alpha_face(c, dz, i - 1) * st->b[i - 1];
            st->er[i] = st->er[i] - k->dtdz * (orc_alpha_node(c, dz, i) * d);
        }
        st->er[N] = st->er[N] + k->tw * (orc_alpha_node(c, dz, N) * (orc_alpha_face(c, dz, N - 1) * st->b[N - 1]));
        for (int64_t i = 0; i < N; ++i) {
            const double jw = (rate == 1.0 || !st->j_inj) ? (double)st->j[i]
                                                          : (double)(st->j[i] - st->j_inj[i]) + rate * (double)st->j_inj[i];
            st->ez[i] = (st->ez[i] + k->dtR * (orc_alpha_face(c, dz, i) * st->b[i])) - k->c4 * jw;
        }
    } else if (!(c->flags & ORC_FREEZE_FIELDS)) {
        /* eq. (3), leap-frog: dB/dt = -dE_r/dz - E_z/R, then dE_r/dt = -dB/dz,
         * then dE_z/dt = B/R - 4 pi j.  E_r,0 = 0 (phi = 0 at the star);
         * mirror about x = N (B odd) gives the E_r,N update. */
        for (int64_t i = 0; i < N; ++i)
            st->b[i] = st->b[i] - (k->dtdz * (st->er[i + 1] - st->er[i]) + k->dtR * st->ez[i]);
        for (int64_t i = 1; i < N; ++i)
            st->er[i] = st->er[i] - k->dtdz * (st->b[i] - st->b[i - 1]);
        st->er[N] = st->er[N] + k->tw * st->b[N - 1];
        if (rate == 1.0 || !st->j_inj) {
            for (int64_t i = 0; i < N; ++i)
                st->ez[i] = (st->ez[i] + k->dtR * st->b[i]) - k->c4 * (double)st->j[i];
        } else {
            /* injected particles carry rate * q_m */
            for (int64_t i = 0; i < N; ++i) {
                const double jw = (double)(st->j[i] - st->j_inj[i]) + rate * (double)st->j_inj[i];
                st->ez[i] = (st->ez[i] + k->dtR * st->b[i]) - k->c4 * jw;
            }
        }
    }

    /* SCLF injection (sec. 2): the field at the surface from the node-0 Gauss law
     * over the half cell [0, dz/2]; electrons are added at x = 0 with u = 0 until
     * the base charge cancels it (never over-injecting). */
    double t1 = rate == 1.0 ? k->qmP * (double)w0
                            : k->qmP * ((double)(w0 - w0_inj) + rate * (double)w0_inj);
    double t2 = k->rho0 * k->hdz;
    if (k->gr) t2 = t2 / orc_alpha_node(c, k->dz, 0);    /* rho_GJ,0 / alpha_0 over the half cell */
    double es = st->ez[0] - k->fourpi * (t1 - t2);
    st->e_surf = es;
    int64_t ninj = 0;
    if (c->schedule) {                       /* frozen injection counts of a recorded run */
        ninj = st->step < c->n_schedule ? c->schedule[st->step] : 0;
        int64_t avail = c->capacity - st->n;
        if (ninj > avail) { ninj = avail; st->status |= ORC_ST_CAPACITY; }
        for (int64_t p = 0; p < ninj; ++p) {
            st->x[st->n + p] = 0.0;
            st->u[st->n + p] = 0.0;
            if (st->cls) st->cls[st->n + p] = 1;
        }
        st->n += ninj;
        st->n_injected += ninj;
    } else if (!(c->flags & ORC_NO_AUTO_INJECT)) {
        double ratio = es / k->fqm;
        if (ratio > 0.0) {
            double nf = floor(ratio);
            int64_t avail = c->capacity - st->n;
            if (nf > (double)avail) { ninj = avail; st->status |= ORC_ST_CAPACITY; }
            else ninj = (int64_t)nf;
        }
        for (int64_t p = 0; p < ninj; ++p) {
            st->x[st->n + p] = 0.0;
            st->u[st->n + p] = 0.0;
            if (st->cls) st->cls[st->n + p] = 1;
        }
        st->n += ninj;
        st->n_injected += ninj;
    }
    st->last_ninj = ninj;
    st->step += 1;
}

/* One PIC cycle, serially: every particle in order, survivors compacted in place. */
static void orc_one_step(const orc_cfg *c, orc_state *st)
{
    orc_const k;
    orc_consts(c, st, &k);
    orc_step_begin(st, &k);
    orc_tally t;
    memset(&t, 0, sizeof t);
    t.j = st->j;
    t.j_inj = st->j_inj;
    orc_push_range(c, st, &k, 0, st->n, st->x, st->u, st->cls, &t);
    orc_step_end(c, st, &k, &t);
}

int orc_step(const orc_cfg *c, orc_state *st, int64_t n_steps)
{
    if (orc_check(c) || !st || n_steps < 0) return -1;
    for (int64_t s = 0; s < n_steps; ++s) orc_one_step(c, st);
    return 0;
}

/* The same steps with the particles split over threads (OpenMP), for timing the
 * oracle on every host core.  Thread k takes the k-th contiguous slice of the
 * particles and pushes it with orc_push_range into its own current array and
 * tallies; the slices' survivors are then written back in slice order, the
 * current arrays summed node by node in thread order and the tallies in thread
 * order.  Every sum is over integers, so the state after each step is the
 * serial oracle's, bit for bit.  Fields and injection run serially (O(N)). */
int orc_step_par(const orc_cfg *c, orc_state *st, int64_t n_steps, int32_t n_threads)
{
    if (orc_check(c) || !st || n_steps < 0) return -1;
    int T = 1;
#ifdef _OPENMP
    T = n_threads > 0 ? n_threads : omp_get_max_threads();
#endif
    if (T < 1) T = 1;
    const int64_t N = c->n_cells, cap = c->capacity;
    int64_t *jt = calloc((size_t)T * (size_t)N, sizeof(int64_t));
    int64_t *jit = st->j_inj ? calloc((size_t)T * (size_t)N, sizeof(int64_t)) : NULL;
    double *sx = malloc(sizeof(double) * (size_t)(cap + 1)), *su = malloc(sizeof(double) * (size_t)(cap + 1));
    unsigned char *scl = st->cls ? malloc((size_t)(cap + 1)) : NULL;
    orc_tally *tl = calloc((size_t)T, sizeof(orc_tally));
    int64_t *pre = calloc((size_t)T + 1, sizeof(int64_t));
    if (!jt || (st->j_inj && !jit) || !sx || !su || (st->cls && !scl) || !tl || !pre) {
        free(jt); free(jit); free(sx); free(su); free(scl); free(tl); free(pre);
        return -2;
    }
    for (int64_t s = 0; s < n_steps; ++s) {
        orc_const k;
        orc_consts(c, st, &k);
        orc_step_begin(st, &k);
        const int64_t n = st->n;
#pragma omp parallel num_threads(T)
        {
            int id = 0;
#ifdef _OPENMP
            id = omp_get_thread_num();
#endif
            const int64_t p0 = (n * id) / T, p1 = (n * (id + 1)) / T;
            int64_t *jme = jt + (size_t)id * (size_t)N;
            int64_t *jime = jit ? jit + (size_t)id * (size_t)N : NULL;
            memset(jme, 0, sizeof(int64_t) * (size_t)N);
            if (jime) memset(jime, 0, sizeof(int64_t) * (size_t)N);
            orc_tally *t = &tl[id];
            memset(t, 0, sizeof *t);
            t->j = jme;
            t->j_inj = jime;
            orc_push_range(c, st, &k, p0, p1, sx + p0, su + p0, scl ? scl + p0 : NULL, t);
#pragma omp barrier
#pragma omp single
            {
                pre[0] = 0;
                for (int q = 0; q < T; ++q) pre[q + 1] = pre[q] + tl[q].kept;
            }
            /* survivors back in slice order; current summed node by node in thread order */
            memcpy(st->x + pre[id], sx + p0, sizeof(double) * (size_t)t->kept);
            memcpy(st->u + pre[id], su + p0, sizeof(double) * (size_t)t->kept);
            if (scl) memcpy(st->cls + pre[id], scl + p0, (size_t)t->kept);
            const int64_t i0 = (N * id) / T, i1 = (N * (id + 1)) / T;
            for (int64_t i = i0; i < i1; ++i) {
                int64_t a = 0, b = 0;
                for (int q = 0; q < T; ++q) {
                    a += jt[(size_t)q * (size_t)N + (size_t)i];
                    if (jit) b += jit[(size_t)q * (size_t)N + (size_t)i];
                }
                st->j[i] = a;
                if (jit) st->j_inj[i] = b;
            }
        }
        orc_tally all;
        memset(&all, 0, sizeof all);
        for (int q = 0; q < T; ++q) {
            all.w0 += tl[q].w0;
            all.w0_inj += tl[q].w0_inj;
            all.n_exit += tl[q].n_exit;
            all.n_absorb += tl[q].n_absorb;
            all.kept += tl[q].kept;
            all.status |= tl[q].status;
            __int128 e = ((__int128)all.exit_hi << 64) | (__int128)all.exit_lo;
            e += ((__int128)tl[q].exit_hi << 64) | (__int128)tl[q].exit_lo;
            all.exit_lo = (uint64_t)e;
            all.exit_hi = (int64_t)(e >> 64);
        }
        orc_step_end(c, st, &k, &all);
    }
    free(jt); free(jit); free(sx); free(su); free(scl); free(tl); free(pre);
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
        double dez = (st->ez[i] - st->ez[i - 1]) / k.dz;
        if (k.gr) {
            /* ORC_GR_ALPHA: alpha_i dE_z/dz + E_r/R = 4 pi (alpha_i lambda_i - rho_GJ,i) */
            double an = orc_alpha_node(c, k.dz, i);
            dez = an * dez;
            rho = an * rho;
        }
        double d = dez + st->er[i] / c->radius;
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

/* ---- reverse-mode gradient (test reference) ------------------------------- */

/* Transposed Thomas solve of A^T y = g on nodes 1..N, A the eq. (4) matrix of
 * orc_solve_fields (rows 1..N-1: 1, bdiag, 1; row N: 2, bdiag).  A^T has the 2
 * on the super-diagonal of row N-1. */
static void orc_poisson_transpose(int64_t N, double bdiag, const double *g, double *y, double *cp, double *dp)
{
    /* row i of A^T: sub 1 (i >= 2), diag bdiag, super (i == N-1 ? 2 : 1) (i <= N-1) */
    double sup = (N - 1 == 1) ? 2.0 : 1.0;
    cp[1] = sup / bdiag;
    dp[1] = g[1] / bdiag;
    for (int64_t i = 2; i <= N; ++i) {
        double m = bdiag - 1.0 * cp[i - 1];
        double c = (i <= N - 1) ? ((i == N - 1) ? 2.0 : 1.0) : 0.0;
        cp[i] = c / m;
        dp[i] = (g[i] - 1.0 * dp[i - 1]) / m;
    }
    y[N] = dp[N];
    for (int64_t i = N - 1; i >= 1; --i) y[i] = dp[i] - cp[i] * y[i + 1];
}

/* ---- the linearised kernels of one step (frozen discrete decisions) ------ */

/* Adjoint of B^{s+1/2} through its uses in E_r^{s+1} and E_z^{s+1} (eq. 3):
 * B^{s+1/2} enters E_r,i and E_r,i+1 (the mirror node N with the factor 2) and E_z. */
static void orc_adj_b_uses(int64_t N, const orc_const *k, const double *lb, const double *lez, const double *ler,
                           double *lbp)
{
    for (int64_t i = 0; i < N; ++i) {
        double a = lb[i] + k->dtR * lez[i];
        if (i >= 1 && i <= N - 1) a -= k->dtdz * ler[i];
        if (i + 1 <= N - 1) a += k->dtdz * ler[i + 1];
        if (i == N - 1) a += k->tw * ler[N];
        lbp[i] = a;
    }
}

/* Adjoints of E_z^s, E_r^s and B^{s-1/2} from lbp (above) and the adjoint lk of
 * the kick array K = (q/m) dt E_z^s, in place (E_r's update uses lbp only). */
static void orc_adj_fields_back(int64_t N, const orc_const *k, double *lez, double *ler, double *lb,
                                const double *lbp, const double *lk)
{
    for (int64_t i = 0; i < N; ++i) {
        const double a = lez[i] - k->dtR * lbp[i] + k->qmdt * lk[i];
        lez[i] = a;
    }
    for (int64_t i = N; i >= 0; --i) {
        double a = ler[i];
        if (i <= N - 1) a += k->dtdz * lbp[i];
        if (i >= 1) a -= k->dtdz * lbp[i - 1];
        ler[i] = a;
    }
    for (int64_t i = 0; i < N; ++i) lb[i] = lbp[i];
}

/* The linearised push of one particle at (x, u) in the kick array K: gather,
 * eq. (1), the move and the current J_i = S_i(x) - S_i(x1), with its cells
 * frozen and rint taken as the identity (dS_i/dx = -2^P in cell i).  What it
 * needs of the forward: */
typedef struct {
    int clamp;            /* 1: x below the first face, 2: above the last face, 0: interpolated */
    int64_t jj;           /* lower face of the interpolation */
    double g, dEdx;       /* interpolation weight of the upper face; K_{j+1} - K_j */
    double u1, gam;       /* new momentum and gamma */
    int64_t c0, c1;       /* cells before and after the move (c1 = N: left the tube; < 0: returned) */
    int64_t F0, F1;       /* fixed-point offsets (the rate gradient's deposit) */
    int fate;             /* 0: stays, 1: exits at the top, 2: absorbed by the star */
} orc_lin_pt;

static void orc_lin_point(int64_t N, int P, const orc_const *k, const double *kk, double x, double u, orc_lin_pt *q)
{
    const double sx = x - 0.5;
    q->jj = 0;
    q->g = 0.0;
    q->dEdx = 0.0;
    q->clamp = 0;
    if (sx < 0.0) { q->clamp = 1; }
    else if (sx >= (double)(N - 1)) { q->clamp = 2; }
    else {
        q->jj = (int64_t)floor(sx);
        q->g = sx - (double)q->jj;
        q->dEdx = kk[q->jj + 1] - kk[q->jj];
    }
    const double E = q->clamp == 1 ? kk[0] : (q->clamp == 2 ? kk[N - 1] : kk[q->jj] + q->g * (kk[q->jj + 1] - kk[q->jj]));
    q->u1 = u + E;
    double t = q->u1 * q->u1;
    t = 1.0 + t;
    q->gam = sqrt(t);
    const double v = q->u1 / q->gam;
    const double x1 = x + k->dtdz * v;
    orc_cell(x, P, &q->c0, &q->F0);
    orc_cell(x1, P, &q->c1, &q->F1);
    q->fate = x1 >= (double)N ? 1 : (x1 < 0.0 ? 2 : 0);
}

/* Transpose of the linearised push of one particle: from the adjoints lx1, lu1
 * of its new state (lu1 of an exit is the loss's seed d gamma/du / n_exit) and
 * lj (the adjoint of the current J, already multiplied by the particle's charge
 * factor), the adjoints of its old state and its part of lk (accumulated). */
static void orc_adj_particle(int64_t N, const orc_const *k, const orc_lin_pt *q, double lx1, double lu1,
                             const double *lj, double wcls, double *lx, double *lu, double *lk)
{
    const double twoP = k->twoP;
    /* current: J_i = S_i(x) - S_i(x1), dS_i/dx = -2^P in cell i */
    if (q->c1 >= 0 && q->c1 < N) lx1 += twoP * (wcls * lj[q->c1]);
    const double lx0J = -twoP * (wcls * lj[q->c0]);
    /* move: x1 = x + (dt/dz) u1 / gamma(u1), dv/du = 1/gamma^3 */
    const double gam = q->gam;
    const double lu1t = lu1 + lx1 * k->dtdz / (gam * gam * gam);
    *lx = lx1 + lx0J + lu1t * q->dEdx;
    *lu = lu1t;
    /* kick: E = K_j (1 - g) + K_{j+1} g */
    if (q->clamp == 1) lk[0] += lu1t;
    else if (q->clamp == 2) lk[N - 1] += lu1t;
    else { lk[q->jj] += lu1t * (1.0 - q->g); lk[q->jj + 1] += lu1t * q->g; }
}

/* The same linearised push, forward (tangent): perturbations dx, du of the old
 * state and dk of the kick array give dx1, du1 and the particle's current
 * perturbation (added to dj). */
static void orc_tl_particle(int64_t N, const orc_const *k, const orc_lin_pt *q, double dx, double du, const double *dk,
                            double *dx1, double *du1, double *dj)
{
    const double twoP = k->twoP;
    double dE;
    if (q->clamp == 1) dE = dk[0];
    else if (q->clamp == 2) dE = dk[N - 1];
    else dE = q->dEdx * dx + (1.0 - q->g) * dk[q->jj] + q->g * dk[q->jj + 1];
    const double d1 = du + dE;
    const double gam = q->gam;
    const double dv = d1 / (gam * gam * gam);
    *du1 = d1;
    *dx1 = dx + k->dtdz * dv;
    dj[q->c0] += -twoP * dx;
    if (q->c1 >= 0 && q->c1 < N) dj[q->c1] += twoP * (*dx1);
}

/* Transposed Poisson start (eq. 4): dL/d rho_GJ at the nodes from the adjoints of
 * the start fields E_z = -dphi/dz, E_r = phi/R, A phi = d, d_i = -cpois (rho_i - rho_GJ,i). */
static void orc_adj_poisson(const orc_cfg *c, const orc_const *k, const double *lez, const double *ler, double *g_rho)
{
    const int64_t N = k->N;
    double *gphi = calloc((size_t)(N + 1), sizeof(double)), *y = calloc((size_t)(N + 1), sizeof(double));
    double *cp = calloc((size_t)(N + 1), sizeof(double)), *dp = calloc((size_t)(N + 1), sizeof(double));
    for (int64_t m = 1; m <= N; ++m) {
        double a = -lez[m - 1] / k->dz + ler[m] / c->radius;
        if (m <= N - 1) a += lez[m] / k->dz;
        gphi[m] = a;
    }
    const double rr = k->dz / c->radius;
    orc_poisson_transpose(N, -(2.0 + rr * rr), gphi, y, cp, dp);
    g_rho[0] = 0.0;
    for (int64_t i = 1; i <= N; ++i) g_rho[i] = k->fourpi * (k->dz * k->dz) * y[i];
    free(gphi); free(y); free(cp); free(dp);
}

int orc_adjoint(const orc_cfg *c, orc_state *st, int64_t T, double *g_rho, double *g_rate, double *loss,
                int64_t *n_exit_out)
{
    if (orc_check(c) || !st || T < 1 || !st->cls || !st->j_inj) return -1;
    if (c->flags & (ORC_FREEZE_FIELDS | ORC_GR_ALPHA)) return -1;
    orc_const k;
    orc_consts(c, st, &k);
    const int64_t N = k.N;
    const int P = c->fp_bits;
    const double rate = c->inj_rate > 0.0 ? c->inj_rate : 1.0;

    /* ---- forward, recording every step's starting state ---- */
    int64_t *n_at = malloc(sizeof(int64_t) * (size_t)(T + 1));
    double **X = calloc((size_t)T, sizeof(double *)), **U = calloc((size_t)T, sizeof(double *));
    unsigned char **C = calloc((size_t)T, sizeof(unsigned char *));
    double *EZ = malloc(sizeof(double) * (size_t)(T * N)), *ER = malloc(sizeof(double) * (size_t)(T * (N + 1)));
    double *BB = malloc(sizeof(double) * (size_t)(T * N));
    if (!n_at || !X || !U || !C || !EZ || !ER || !BB) return -2;
    const int64_t ex0 = st->n_exit;
    const __int128 s0 = ((__int128)st->exit_sum_hi << 64) | (__int128)st->exit_sum_lo;
    for (int64_t s = 0; s < T; ++s) {
        const int64_t n = st->n;
        n_at[s] = n;
        X[s] = malloc(sizeof(double) * (size_t)(n + 1));
        U[s] = malloc(sizeof(double) * (size_t)(n + 1));
        C[s] = malloc((size_t)(n + 1));
        if (!X[s] || !U[s] || !C[s]) return -2;
        memcpy(X[s], st->x, sizeof(double) * (size_t)n);
        memcpy(U[s], st->u, sizeof(double) * (size_t)n);
        memcpy(C[s], st->cls, (size_t)n);
        memcpy(EZ + s * N, st->ez, sizeof(double) * (size_t)N);
        memcpy(ER + s * (N + 1), st->er, sizeof(double) * (size_t)(N + 1));
        memcpy(BB + s * N, st->b, sizeof(double) * (size_t)N);
        orc_one_step(c, st);
    }
    n_at[T] = st->n;
    const int64_t nex = st->n_exit - ex0;
    const __int128 s1 = ((__int128)st->exit_sum_hi << 64) | (__int128)st->exit_sum_lo;
    const double L = nex > 0 ? ldexp((double)(s1 - s0), -32) / (double)nex : 0.0;
    if (loss) *loss = L;
    if (n_exit_out) *n_exit_out = nex;

    /* ---- reverse sweep ---- */
    double *lx = calloc((size_t)(n_at[T] + 1), sizeof(double)), *lu = calloc((size_t)(n_at[T] + 1), sizeof(double));
    double *lez = calloc((size_t)N, sizeof(double)), *ler = calloc((size_t)(N + 1), sizeof(double));
    double *lb = calloc((size_t)N, sizeof(double)), *lbp = calloc((size_t)N, sizeof(double));
    double *lk = calloc((size_t)N, sizeof(double)), *kk = calloc((size_t)N, sizeof(double));
    double *lj = calloc((size_t)N, sizeof(double));
    double grate = 0.0;
    for (int64_t s = T - 1; s >= 0; --s) {
        const double *ez = EZ + s * N;
        for (int64_t i = 0; i < N; ++i) { kk[i] = k.qmdt * ez[i]; lk[i] = 0.0; }
        /* adjoint of B^{s+1/2}: its own adjoint plus its uses in E_r and E_z of step s */
        orc_adj_b_uses(N, &k, lb, lez, ler, lbp);
        /* the current enters E_z^{s+1} = ... - c4 J */
        for (int64_t i = 0; i < N; ++i) lj[i] = -k.c4 * lez[i];
        /* particles of step s (in order; survivors keep their order at step s+1) */
        const int64_t n = n_at[s];
        double *nlx = calloc((size_t)(n + 1), sizeof(double)), *nlu = calloc((size_t)(n + 1), sizeof(double));
        int64_t jn = 0;
        for (int64_t p = 0; p < n; ++p) {
            const double wcls = C[s][p] ? rate : 1.0;
            orc_lin_pt q;
            orc_lin_point(N, P, &k, kk, X[s][p], U[s][p], &q);
            double lx1 = 0.0, lu1 = 0.0;
            if (q.fate == 1) {
                lu1 = nex > 0 ? (q.u1 / q.gam) / (double)nex : 0.0;   /* d gamma / du = u / gamma */
            } else if (q.fate == 0) {
                lx1 = lx[jn];
                lu1 = lu[jn];
                ++jn;
            }                                                          /* absorbed: no further influence */
            if (C[s][p]) {
                /* dL/d rate: the particle's deposit times the adjoint of the current */
                int64_t lo = q.c0 < q.c1 ? q.c0 : q.c1, hi = q.c0 < q.c1 ? q.c1 : q.c0;
                if (lo < 0) lo = 0;
                if (hi > N - 1) hi = N - 1;
                for (int64_t i = lo; i <= hi; ++i)
                    grate += (double)(orc_S(i, q.c0, q.F0, k.oneP) - orc_S(i, q.c1, q.F1, k.oneP)) * lj[i];
            }
            orc_adj_particle(N, &k, &q, lx1, lu1, lj, wcls, &nlx[p], &nlu[p], lk);
        }
        free(lx);
        free(lu);
        lx = nlx;
        lu = nlu;
        /* fields of step s: E_z^{s+1} = E_z + dtR B' - c4 J; B' = B - (dtdz (E_r,i+1 - E_r,i) + dtR E_z) */
        orc_adj_fields_back(N, &k, lez, ler, lb, lbp, lk);
    }
    /* Poisson start (eq. 4) */
    if (g_rho) orc_adj_poisson(c, &k, lez, ler, g_rho);
    if (g_rate) *g_rate = grate;
    for (int64_t s = 0; s < T; ++s) { free(X[s]); free(U[s]); free(C[s]); }
    free(X); free(U); free(C); free(EZ); free(ER); free(BB); free(n_at);
    free(lx); free(lu); free(lez); free(ler); free(lb); free(lbp); free(lk); free(kk); free(lj);
    return 0;
}

/* ---- test hooks: the linearised kernels one by one (dot-product pins) ------ */

int orc_tl_fields(const orc_cfg *c, const orc_state *st, const double *dez, const double *der, const double *db,
                  const double *dj, double *dez1, double *der1, double *db1)
{
    if (orc_check(c) || !st) return -1;
    orc_const k;
    orc_consts(c, st, &k);
    const int64_t N = k.N;
    for (int64_t i = 0; i < N; ++i) db1[i] = db[i] - (k.dtdz * (der[i + 1] - der[i]) + k.dtR * dez[i]);
    der1[0] = der[0];
    for (int64_t i = 1; i < N; ++i) der1[i] = der[i] - k.dtdz * (db1[i] - db1[i - 1]);
    der1[N] = der[N] + k.tw * db1[N - 1];
    for (int64_t i = 0; i < N; ++i) dez1[i] = (dez[i] + k.dtR * db1[i]) - k.c4 * dj[i];
    return 0;
}

int orc_ad_fields(const orc_cfg *c, const orc_state *st, const double *lez1, const double *ler1, const double *lb1,
                  double *lez, double *ler, double *lb, double *lj)
{
    if (orc_check(c) || !st) return -1;
    orc_const k;
    orc_consts(c, st, &k);
    const int64_t N = k.N;
    double *lbp = calloc((size_t)N, sizeof(double)), *lk = calloc((size_t)N, sizeof(double));
    if (!lbp || !lk) { free(lbp); free(lk); return -2; }
    orc_adj_b_uses(N, &k, lb1, lez1, ler1, lbp);
    for (int64_t i = 0; i < N; ++i) { lez[i] = lez1[i]; lb[i] = lb1[i]; lj[i] = -k.c4 * lez1[i]; }
    for (int64_t i = 0; i <= N; ++i) ler[i] = ler1[i];
    orc_adj_fields_back(N, &k, lez, ler, lb, lbp, lk);
    free(lbp);
    free(lk);
    return 0;
}

int orc_tl_push(const orc_cfg *c, const orc_state *st, const double *dx, const double *du, const double *dk,
                double *dx1, double *du1, double *dj)
{
    if (orc_check(c) || !st) return -1;
    orc_const k;
    orc_consts(c, st, &k);
    const int64_t N = k.N;
    for (int64_t i = 0; i < N; ++i) dj[i] = 0.0;
    for (int64_t p = 0; p < st->n; ++p) {
        orc_lin_pt q;
        orc_lin_point(N, c->fp_bits, &k, st->k, st->x[p], st->u[p], &q);
        orc_tl_particle(N, &k, &q, dx[p], du[p], dk, &dx1[p], &du1[p], dj);
    }
    return 0;
}

int orc_ad_push(const orc_cfg *c, const orc_state *st, const double *lx1, const double *lu1, const double *lj,
                double *lx, double *lu, double *lk)
{
    if (orc_check(c) || !st) return -1;
    orc_const k;
    orc_consts(c, st, &k);
    const int64_t N = k.N;
    for (int64_t i = 0; i < N; ++i) lk[i] = 0.0;
    for (int64_t p = 0; p < st->n; ++p) {
        orc_lin_pt q;
        orc_lin_point(N, c->fp_bits, &k, st->k, st->x[p], st->u[p], &q);
        orc_adj_particle(N, &k, &q, lx1[p], lu1[p], lj, 1.0, &lx[p], &lu[p], lk);
    }
    return 0;
}

int orc_tl_poisson(const orc_cfg *c, const orc_state *st, const double *drho, double *dez, double *der)
{
    if (orc_check(c) || !st) return -1;
    orc_const k;
    orc_consts(c, st, &k);
    const int64_t N = k.N;
    double *d = calloc((size_t)(N + 1), sizeof(double)), *cp = calloc((size_t)(N + 1), sizeof(double));
    double *phi = calloc((size_t)(N + 1), sizeof(double));
    if (!d || !cp || !phi) { free(d); free(cp); free(phi); return -2; }
    const double rr = k.dz / c->radius;
    const double bdiag = -(2.0 + rr * rr);
    const double cpois = k.fourpi * (k.dz * k.dz);
    for (int64_t i = 1; i <= N; ++i) d[i] = cpois * drho[i];   /* d_i = -cpois (rho_i - rho_GJ,i) */
    cp[1] = 1.0 / bdiag;
    d[1] = d[1] / bdiag;
    for (int64_t i = 2; i <= N; ++i) {
        const double sub = (i == N) ? 2.0 : 1.0;   /* row N: the mirror ghost doubles the sub-diagonal */
        const double m = bdiag - sub * cp[i - 1];
        cp[i] = 1.0 / m;
        d[i] = (d[i] - sub * d[i - 1]) / m;
    }
    phi[0] = 0.0;
    phi[N] = d[N];
    for (int64_t i = N - 1; i >= 1; --i) phi[i] = d[i] - cp[i] * phi[i + 1];
    for (int64_t i = 0; i < N; ++i) dez[i] = -((phi[i + 1] - phi[i]) / k.dz);
    for (int64_t i = 0; i <= N; ++i) der[i] = phi[i] / c->radius;
    free(d); free(cp); free(phi);
    return 0;
}

int orc_ad_poisson(const orc_cfg *c, const orc_state *st, const double *lez, const double *ler, double *lrho)
{
    if (orc_check(c) || !st) return -1;
    orc_const k;
    orc_consts(c, st, &k);
    orc_adj_poisson(c, &k, lez, ler, lrho);
    return 0;
}
