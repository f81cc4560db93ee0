/*
 * pcpic_oracle.h -- plain FP64 CPU oracle of the 1D polar-cap PIC time step.
 *
 * TEST INFRASTRUCTURE ONLY.  This code is the slow, serial, obviously-correct
 * definition that the GPU library is checked against.  Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it.  It shares no
 * code, header or constant with the GPU library.
 *
 * Method (Barzilay, "Full simulation of the open field lines above pulsar's
 * polar cap - Part I"): a conducting tube of radius R along the field line,
 * electrons pushed in E_z by eq. (1), linear weighting between particles and
 * grid (sec. 2, PIC cycle of Fig. A), the transverse-reduced Maxwell system of
 * eq. (3) advanced by leap-frog, fields started from the Poisson problem of
 * eq. (4) with the boundary conditions stated under it, and space-charge-
 * limited electron injection at the base (sec. 2).  The Goldreich-Julian
 * background is the flat form of eq. (5) with i = 0, the frame-dragging form
 * of eqs. (6)-(7) with alpha = f = H = 1 and the sin(i) term dropped, or
 * eq. (6) with the redshift 1/alpha and the sin(i) term (f = H = 1).
 *
 * Discretisation (a reading; the paper gives no discrete scheme):
 *   positions in cell units x = z/dz in [0, N); nodes x = i carry phi, E_r,
 *   rho_GJ and the integer CIC weight W_i; faces x = i + 1/2 carry E_z, B_phi
 *   and the integer current J_i.  x and E live at integer time levels, u = gamma*beta,
 *   B_phi and J at half levels.  Weights are fixed point with P fraction bits.
 */
#ifndef PCPIC_ORACLE_H
#define PCPIC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    ORC_RHO_UNIFORM = 0,    /* rho_GJ = -A                      (eq. 5, i = 0, (R_star/r)^3 dropped) */
    ORC_RHO_FRAME_DRAG = 1, /* rho_GJ = -A (1 - kappa eta^-3)   (eqs. 6-7, alpha = f = H = 1)    */
    ORC_RHO_KNOTS = 2,      /* rho_GJ = -theta(z) (1 - kappa eta^-3), theta piecewise linear      */
    ORC_RHO_GR = 3          /* eq. 6 with f = H = 1: redshift 1/alpha and the sin(i) term (below)  */
};

enum {
    ORC_NO_AUTO_INJECT = 1u, /* skip the SCLF injection                                  */
    ORC_FREEZE_FIELDS = 2u,  /* skip the Maxwell update: fields stay as they are           */
    ORC_B_STEADY_INIT = 4u,  /* start B_phi = 4 pi R j of the loaded beam (steady E_z)     */
    ORC_GR_ALPHA = 8u        /* lapse alpha(z) in Maxwell and the equation of motion (below) */
};

/*
 * ORC_GR_ALPHA -- the full-GR factor alpha = (1 - r_g/r)^(1/2), r = R_* + z, in
 * Maxwell's equations and the equation of motion, which the paper names after
 * eqs. (6)-(7) but does not write out.  Reading (3+1 split of the Schwarzschild
 * metric, fields and momenta measured by static observers, frame dragging kept
 * in rho_GJ only, the tube's constant radius and d/dr -> 1/R as in eq. 3; z is
 * the radial coordinate, t the coordinate time):
 *   (1/c) dE_z/dt = alpha B/R - 4 pi (alpha j)
 *   (1/c) dE_r/dt = -alpha d(alpha B)/dz
 *   (1/c) dB/dt   = -alpha d(alpha E_r)/dz - alpha E_z/R
 *   alpha dE_z/dz + E_r/R = 4 pi (alpha lambda - rho_GJ)
 *   du/dt = alpha (q/m) E_z - gamma alpha alpha',   dz/dt = alpha^2 u/gamma
 * lambda is the charge per unit coordinate length (the CIC weights) and
 * alpha j its coordinate flux, which is what the charge-conserving deposit
 * counts, so the discrete Gauss law below is kept exactly as in flat space.
 * alpha alpha' = (r_g/R_*) / (2 R_* eta^2), eta = r/R_*; a test particle in a
 * static field E_z = -dPhi/dz keeps alpha gamma + (q/m) Phi.
 * Discretisation: alpha at nodes (a_i) and faces (a_{i+1/2}) multiplies the
 * flat leap-frog terms as written above; the push takes alpha at x^n for the
 * kick, a midpoint gamma for the gravity term (u_h = u + (alpha K - k_g gamma(u))/2,
 * u' = u + alpha K - k_g gamma(u_h), k_g = dt alpha alpha'), and a midpoint alpha^2
 * for the move (x_h = x + (c dt/dz) alpha^2(x) v / 2, x' = x + (c dt/dz) alpha^2(x_h) v);
 * the Poisson start solves d2Phi/dz2 - Phi/(alpha R)^2 = -4 pi (lambda - rho_GJ/alpha)
 * with E_z = -dPhi/dz and E_r = Phi/(alpha R), a fixed point of the update; the
 * surface field takes rho_GJ,0/alpha_0 in the half cell.  With r_g = 0 every
 * factor is 1 and the step is the flat one, bit for bit.  Uses r_star and
 * rg_over_rstar (any rho_kind); not with the reverse-mode gradient.
 */

enum {
    ORC_ST_CAPACITY = 1,     /* injection wanted more particles than the capacity allows */
    ORC_ST_NONFINITE = 2     /* a momentum or position became non-finite (particle removed) */
};

typedef struct orc_cfg {
    int64_t n_cells;      /* N                                                    */
    double length;        /* L, tube length                                       */
    double radius;        /* R, tube radius                                       */
    double dt_over_dz;    /* c dt / dz, must be < 1                                */
    double q_over_m;      /* electron charge-to-mass ratio (negative)             */
    double ppc;           /* macro-particles per base cell-charge                 */
    int32_t rho_kind;     /* ORC_RHO_*                                            */
    int32_t n_knots;      /* knot count for ORC_RHO_KNOTS (>= 2)                  */
    double rho_amp;       /* A                                                    */
    double kappa;         /* frame-dragging strength, omega/Omega at eta = 1      */
    double r_star;        /* star radius R_*                                      */
    const double *knots;  /* theta_k, k = 0..n_knots-1, uniform over [0, L]        */
    int32_t fp_bits;      /* P, fixed-point fraction bits of the weights          */
    uint32_t flags;       /* ORC_NO_AUTO_INJECT | ORC_FREEZE_FIELDS | ORC_B_STEADY_INIT | ORC_GR_ALPHA */
    int64_t capacity;     /* particle array capacity                              */
    double macro_charge;  /* q_m; 0 = rho_GJ(0) dz / ppc                          */
    double inj_rate;      /* charge factor of particles injected during the run (0 = 1) */
    const int64_t *schedule; /* if not NULL: particles injected at step n = schedule[n]
                                (replaces the SCLF rule; frozen decisions)         */
    int64_t n_schedule;
    /* ORC_RHO_GR (eq. 6): inclination i (rad), theta_* (rad), cos(varphi) and r_g / R_*;
       ORC_GR_ALPHA uses r_g / R_* and r_star */
    double incl;
    double theta_star;
    double cos_phi;
    double rg_over_rstar;
} orc_cfg;

/* All arrays are owned by the caller; the oracle never allocates them. */
typedef struct orc_state {
    double *x;            /* [capacity] positions, cell units                    */
    double *u;            /* [capacity] momenta u = gamma*beta                    */
    double *rho_gj;       /* [N+1] background charge density at nodes            */
    double *ez;           /* [N]   E_z at faces                                  */
    double *er;           /* [N+1] E_r at nodes                                  */
    double *b;            /* [N]   B_phi at faces                                */
    int64_t *j;           /* [N]   fixed-point current of the last step          */
    double *k;            /* [N]   kick array (q/m) dt E_z                       */
    double *phi;          /* [N+1] potential (Poisson scratch / output)          */
    double *cp;           /* [N+1] Thomas scratch                                */
    double *dp;           /* [N+1] Thomas scratch                                */
    int64_t *w;           /* [N+1] CIC node weights (Poisson / diagnostics)      */
    int64_t n;            /* live particles                                      */
    int64_t step;         /* completed steps                                     */
    int64_t n_injected;   /* particles injected by the SCLF rule so far          */
    int64_t n_exit;       /* particles that left through x = N                   */
    int64_t n_absorb;     /* particles absorbed by the star (x < 0)              */
    int64_t w0;           /* node-0 weight tally of the last step                */
    int64_t last_ninj;    /* injected in the last step                           */
    int64_t status;       /* ORC_ST_* bits                                       */
    uint64_t exit_sum_lo; /* 128-bit sum of rint(gamma * 2^32) over exits        */
    int64_t exit_sum_hi;
    double e_surf;        /* surface field after the last step                   */
    unsigned char *cls;   /* [capacity] 0 = loaded before the first step, 1 = injected */
    int64_t *j_inj;       /* [N] injected-class part of j (in j already)         */
} orc_state;

/* Background charge density at the N+1 nodes. */
int orc_rho_gj(const orc_cfg *cfg, double *rho_gj);
/* CIC node weights of the first n particles, w[N+1] overwritten. */
int orc_weights(const orc_cfg *cfg, const double *x, int64_t n, int64_t *w);
/* Fill rho_gj and solve eq. (4) with the charge of the live particles; set
 * E_z, E_r from phi, B_phi = 0, J = 0.  Particles may be preloaded (st->n). */
int orc_init(const orc_cfg *cfg, orc_state *st);
/* Append particles; before the first step the fields are solved again. */
int orc_inject(const orc_cfg *cfg, orc_state *st, int64_t n, const double *x, const double *u);
/* Advance n_steps PIC cycles. */
int orc_step(const orc_cfg *cfg, orc_state *st, int64_t n_steps);
/* orc_step on n_threads threads (OpenMP; 0 = the default count): the particles
 * are split into contiguous slices, and the state after every step is identical,
 * bit for bit, to orc_step's (all sums are integer sums).  For timing the oracle
 * on every host core; it allocates per-thread scratch for the call.  Returns -2
 * if that allocation fails. */
int orc_step_par(const orc_cfg *cfg, orc_state *st, int64_t n_steps, int32_t n_threads);
/* Discrete Gauss residual at nodes 1..N-1 into g[N+1] (g[0] = g[N] = 0);
 * returns max |G_i| / (4 pi max|rho_GJ|) in *gmax. */
int orc_gauss(const orc_cfg *cfg, orc_state *st, double *g, double *gmax);
/* Signed-gamma profile: sign(u) gamma binned in x over nb uniform bins.
 * Sums are 128-bit fixed point in units of 2^-32 (lo/hi words). */
int orc_profile(const orc_cfg *cfg, const orc_state *st, int32_t nb, int64_t *count,
                uint64_t *sum_lo, int64_t *sum_hi, double *gmin, double *gmax);

/* Reverse-mode gradient of the loss L = (sum of gamma over particles leaving
 * through x = N during n_steps steps) / (their number), with every discrete
 * decision of the recorded run frozen (injection counts, which particle leaves
 * or returns, cell crossings; rint taken as the identity).  The run starts from
 * the state *st0 (fields, particles, counters as after orc_init / orc_inject),
 * which is advanced in place.  Outputs (each may be NULL):
 *   g_rho[N+1]  dL/d rho_GJ at the nodes (through the Poisson start of eq. 4),
 *   g_rate      dL/d inj_rate,
 *   loss, n_exit.
 * The particle states of every step are kept in memory (plain and slow). */
int orc_adjoint(const orc_cfg *cfg, orc_state *st, int64_t n_steps, double *g_rho, double *g_rate,
                double *loss, int64_t *n_exit);

/* Test hooks: the linearised kernels of one step, each as a tangent (tl) and
 * its transpose (ad), for dot-product pins of the reverse sweep: <ad(l), d> must
 * equal <l, tl(d)>.  The ad functions are the ones orc_adjoint applies.
 *  fields  -- the leap-frog of eq. (3), linear: (dez, der, db, dj) -> (dez1, der1,
 *             db1), dj the current in fixed-point units (real-valued);
 *  push    -- gather, eq. (1), move and current of the particles of st in the kick
 *             array st->k, every fate and cell frozen and rint taken as the
 *             identity: (dx, du, dk) -> (dx1, du1, dj); every particle keeps its
 *             new state as an output, including those that leave or return;
 *  poisson -- the start fields of eq. (4) as a function of rho_GJ: drho -> (dez, der). */
int orc_tl_fields(const orc_cfg *cfg, const orc_state *st, const double *dez, const double *der, const double *db,
                  const double *dj, double *dez1, double *der1, double *db1);
int orc_ad_fields(const orc_cfg *cfg, const orc_state *st, const double *lez1, const double *ler1, const double *lb1,
                  double *lez, double *ler, double *lb, double *lj);
int orc_tl_push(const orc_cfg *cfg, const orc_state *st, const double *dx, const double *du, const double *dk,
                double *dx1, double *du1, double *dj);
int orc_ad_push(const orc_cfg *cfg, const orc_state *st, const double *lx1, const double *lu1, const double *lj,
                double *lx, double *lu, double *lk);
int orc_tl_poisson(const orc_cfg *cfg, const orc_state *st, const double *drho, double *dez, double *der);
int orc_ad_poisson(const orc_cfg *cfg, const orc_state *st, const double *lez, const double *ler, double *lrho);

#ifdef __cplusplus
}
#endif
#endif
