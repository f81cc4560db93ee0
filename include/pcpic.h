/*
 * pcpic.h -- C ABI of the MI355X (gfx950) polar-cap PIC library.
 *
 * One time step of the 1D particle-in-cell model of the open field lines above
 * a pulsar's polar cap (Barzilay, "Full simulation of the open field lines above
 * pulsar's polar cap - Part I", sec. 2): electrons in a conducting tube of
 * radius R are pushed along z by E_z (eq. 1), their charge and current are
 * weighted linearly to the grid (sec. 2, Fig. A), the transverse-reduced
 * Maxwell system (eq. 3, d/dr -> 1/R) is advanced by leap-frog, the fields
 * start from the Poisson problem of eq. (4) with phi = 0 at the star and
 * phi' = 0 at the tube end, and electrons are injected at the base while the
 * Goldreich-Julian charge there (eq. 5, or eqs. 6-7 with frame dragging) is
 * not compensated (space-charge-limited flow, sec. 2).
 *
 * Units (sec. 3): c = 1; lengths in the caller's unit (normally R = 1).
 * Grid: N cells of width dz = L/N.  Particle positions are in cell units
 * x = z/dz in [0, N).  Nodes x = i (i = 0..N) carry phi, E_r and rho_GJ;
 * faces x = i + 1/2 (i = 0..N-1) carry E_z, B_phi and the current.
 * x and E live at integer time levels; u = gamma*beta and B_phi at half levels.
 *
 * Conventions of every entry point:
 *  - Plain C types only.  Pointers marked "host" are ordinary CPU memory, read
 *    or written during the call; pointers marked "device" are HIP device memory.
 *  - The caller owns the device workspace and the HIP stream.  The library
 *    never allocates or frees device memory; it carves the workspace.  The
 *    handle itself is a small host object freed by pic_destroy.
 *  - Every call returns a pic_status (0 = PIC_OK).  On failure nothing has been
 *    enqueued and pic_last_error() (per thread) describes the reason.
 *  - pic_step only enqueues work; device-side conditions (capacity overflow,
 *    non-finite momenta) are latched in a device status word and reported by
 *    the next synchronising call (pic_diagnostics, pic_sync, pic_read_*).
 *  - A handle must not be used from two threads at once.
 */
#ifndef PCPIC_H
#define PCPIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PCPIC_ABI_VERSION 4

typedef int32_t pic_status;
enum {
    PIC_OK = 0,
    PIC_EINVAL = -1,     /* invalid argument or parameter                         */
    PIC_EWORKSPACE = -2, /* workspace missing, too small or misaligned            */
    PIC_ECAPACITY = -3,  /* particle capacity exceeded (host-detected)            */
    PIC_ENONFINITE = -4, /* non-finite input particle                             */
    PIC_ECFL = -5,       /* dt_over_dz not in (0, 1)                              */
    PIC_EDEVICE = -6,    /* a HIP runtime call failed                             */
    PIC_ESTATE = -7,     /* call not allowed in the handle's current state        */
    PIC_EABI = -8,       /* pic_params.abi_version != PCPIC_ABI_VERSION            */
    PIC_EDEVSTATUS = -9  /* the device latched a status bit (see pic_diag.status) */
};

/* Device status bits (latched; reported in pic_diag.status). */
enum {
    PIC_ST_CAPACITY = 1,  /* SCLF injection was clipped at the capacity            */
    PIC_ST_NONFINITE = 2, /* a particle's u or x became non-finite; it was removed */
    PIC_ST_GAUSS = 4      /* a diagnostics call found the discrete Gauss residual of eq. (2)
                             above its request's gauss_tol (the deposit or the field update
                             no longer keeps the divergence equation)                     */
};

/* Arithmetic of the particle push. */
enum {
    PIC_FP64 = 0,         /* x, u in FP64; bit-identical to the FP64 CPU oracle            */
    PIC_FP32_BULK = 1     /* (cell, f32 offset) positions; u in f32 below gamma_fp64 and in
                             f64 from it on; fields, Gauss residual and E_surf stay FP64    */
};

/* Goldreich-Julian background (sec. 2, eqs. 5-7), eta = 1 + z/R_*. */
enum {
    PIC_RHO_UNIFORM = 0,    /* -A: eq. (5) with i = 0 and (R_star/r)^3 dropped            */
    PIC_RHO_FRAME_DRAG = 1, /* -A (1 - kappa/eta^3): eq. (6), Omega -> Omega - omega,
                               omega from eq. (7), alpha = f = H = 1, sin(i) term dropped */
    PIC_RHO_KNOTS = 2,      /* -theta(z)(1 - kappa/eta^3), theta piecewise linear on
                               n_knots uniform knots over [0, L]                          */
    PIC_RHO_GR = 3          /* eq. (6) with f = H = 1, in units of the flat surface density
                               Omega B cos(i)/(2 pi c), (R_star/r)^3 dropped:
                               -A [(1 - kappa/eta^3) + (3/2) eta^(1/2) theta_* tan(i) cos(varphi)]
                               / alpha, alpha = (1 - (r_g/R_*)/eta)^(1/2)                   */
};

/* pic_params.flags */
enum {
    PIC_NO_AUTO_INJECT = 1u, /* no SCLF injection (E_surf is still computed)         */
    PIC_FREEZE_FIELDS = 2u,  /* skip the Maxwell update; fields keep their values     */
    PIC_B_STEADY_INIT = 4u,  /* warm start: B_phi = 4 pi R j of the loaded beam, so that
                                dE_z/dt = 0 at t = 0 (eq. 3); j is the current of one
                                drift step at the particles' velocities, without a kick */
    PIC_GR_ALPHA = 8u        /* full GR: the lapse alpha = (1 - r_g/r)^(1/2), r = R_* + z,
                                in Maxwell's equations and the equation of motion, which
                                sec. 2 names after eqs. (6)-(7) without writing them out.
                                Reading (3+1 Schwarzschild form, fields and momenta of
                                static observers, z the radial coordinate):
                                  dE_z/dt = alpha B/R - 4 pi alpha j,
                                  dE_r/dt = -alpha d(alpha B)/dz,
                                  dB/dt = -alpha d(alpha E_r)/dz - alpha E_z/R,
                                  alpha dE_z/dz + E_r/R = 4 pi (alpha lambda - rho_GJ),
                                  du/dt = alpha (q/m) E_z - gamma alpha alpha',
                                  dz/dt = alpha^2 u/gamma,
                                lambda the charge per coordinate length and alpha j its
                                coordinate flux (what the deposit counts); the push takes
                                a midpoint gamma for gravity and a midpoint alpha^2 for
                                the move; the Poisson start solves
                                d2Phi/dz2 - Phi/(alpha R)^2 = -4 pi (lambda - rho_GJ/alpha)
                                with E_z = -dPhi/dz, E_r = Phi/(alpha R).  Uses r_star and
                                rg_over_rstar with any rho_kind (r_g = 0: the flat step, bit
                                for bit).  FP64 single tubes only: PIC_EINVAL with
                                PIC_FP32_BULK, in a batch, and for the adjoint.  The push
                                runs at its default launch shape.                           */
};

/* Tube description.  Copied by pic_init; the knot array is copied too. */
typedef struct pic_params {
    int32_t abi_version;      /* must be PCPIC_ABI_VERSION                                  */
    int32_t precision;        /* PIC_FP64 or PIC_FP32_BULK                                  */
    int64_t n_cells;          /* N >= 2                                                     */
    double length;            /* L > 0                                                      */
    double radius;            /* R > 0                                                      */
    double dt_over_dz;        /* c dt/dz in (0, 1); 0.5 in every standard configuration     */
    double q_over_m;          /* electron charge-to-mass ratio (negative); sets omega_p     */
    double ppc;               /* macro-particles per base cell-charge:
                                 macro charge q_m = rho_GJ(0) dz / ppc                      */
    int32_t rho_kind;         /* PIC_RHO_*                                                  */
    int32_t n_knots;          /* >= 2 for PIC_RHO_KNOTS, else ignored                       */
    double rho_amp;           /* A                                                          */
    double kappa;             /* omega/Omega at the surface (eq. 7): 0.4 r_g/R_*             */
    double r_star;            /* R_* (> 0 for FRAME_DRAG and KNOTS)                          */
    const double *knots;      /* host, n_knots values theta_k (PIC_RHO_KNOTS)               */
    int32_t fp_bits;          /* P, fraction bits of the fixed-point weights: 16..36         */
    int32_t sort_every;       /* cell sort + compaction period in steps (0 = never)          */
    int64_t capacity;         /* particle capacity (live + not yet compacted; FP32-bulk: both
                                 streams together, each holds up to `capacity` slots)        */
    uint32_t flags;           /* PIC_NO_AUTO_INJECT | PIC_FREEZE_FIELDS | PIC_B_STEADY_INIT |
                                 PIC_GR_ALPHA                                                  */
    int32_t max_bins;         /* largest signed-gamma profile pic_diagnostics may request    */
    double gamma_fp64;        /* PIC_FP32_BULK: gamma from which u is kept in f64 (0 = 1e6)  */
    double macro_charge;      /* q_m (per unit area); 0 = rho_GJ(0) dz / ppc.  A fixed value
                                 keeps the particle charge independent of rho_GJ (gradients) */
    /* PIC_RHO_GR only (eq. 6): */
    double incl;              /* inclination i (rad), |i| < 1.5                              */
    double theta_star;        /* magnetic colatitude theta_* of the field line (rad)         */
    double cos_phi;           /* cos(varphi) of the field line's azimuth (1 for varphi = 0)  */
    double rg_over_rstar;     /* r_g / R_* in [0, 1): alpha = (1 - r_g/r)^(1/2)              */
} pic_params;

typedef struct pic_handle pic_handle;

/* Diagnostics request (sec. 3: gamma(z) with returning electrons negative,
 * and the E_z, E_r, B_phi profiles). */
typedef struct pic_diag_req {
    int32_t n_bins;       /* bins of the signed-gamma profile over [0, N); 0 = none, <= max_bins */
    int32_t want_gauss;   /* compute the discrete Gauss residual at nodes 1..N-1              */
    double gauss_tol;     /* with want_gauss: latch PIC_ST_GAUSS when gauss_max exceeds it
                             (0 = no check)                                                 */
} pic_diag_req;

/* Diagnostics result.  Array pointers are host memory provided by the caller
 * (any may be NULL to skip it); the library fills the scalars. */
typedef struct pic_diag {
    int64_t step;          /* completed steps                                              */
    int64_t n_alive;       /* live particles                                               */
    int64_t n_slots;       /* occupied slots (live + removed since the last compaction)    */
    int64_t n_injected;    /* particles injected by the SCLF rule so far                   */
    int64_t n_exit;        /* particles that left through z = L                            */
    int64_t n_absorb;      /* particles that returned to the star                          */
    int64_t last_n_inj;    /* injected at the end of the last step                         */
    int64_t w0;            /* node-0 fixed-point weight of the last step                   */
    int64_t status;        /* latched PIC_ST_* bits                                        */
    double e_surf;         /* surface field of the last step (node-0 Gauss law, before injection) */
    uint64_t exit_sum_lo;  /* sum over exits of rint(gamma 2^32), 128-bit two's complement */
    int64_t exit_sum_hi;
    double exit_gamma_sum; /* the same sum / 2^32 as a double                              */
    double gauss_max;      /* max |G_i| / (4 pi max|rho_GJ|), nodes 1..N-1 (want_gauss)    */
    int64_t n_slots_high;  /* PIC_FP32_BULK: occupied slots of the f64-momentum stream      */
    double gauss_l2;       /* sqrt(mean over nodes 1..N-1 of G_i^2) / (4 pi max|rho_GJ|) (want_gauss) */
    double *ez;            /* [N]   E_z at faces                                           */
    double *er;            /* [N+1] E_r at nodes                                           */
    double *b_phi;         /* [N]   B_phi at faces                                         */
    double *rho_gj;        /* [N+1] background density at nodes                            */
    int64_t *j_last;       /* [N]   fixed-point current of the last step                   */
    int64_t *weights;      /* [N+1] fixed-point CIC node weights of the live particles     */
    double *gauss;         /* [N+1] Gauss residual (0 at nodes 0 and N)                     */
    int64_t *prof_count;   /* [n_bins] particles per bin                                   */
    double *prof_mean;     /* [n_bins] mean of sign(u) gamma (fixed-point sum / count)     */
    double *prof_min;      /* [n_bins] min of sign(u) gamma                                */
    double *prof_max;      /* [n_bins] max of sign(u) gamma                                */
    uint64_t *prof_sum_lo; /* [n_bins] raw 128-bit sums, units of 2^-32                    */
    int64_t *prof_sum_hi;  /* [n_bins]                                                     */
} pic_diag;

/* Library ABI version (PCPIC_ABI_VERSION of the build). */
int32_t pic_abi_version(void);

/* Description of the last failure on the calling thread ("" if none). */
const char *pic_last_error(void);

/* Device workspace bytes pic_init needs for these parameters, or 0 if the
 * parameters are invalid (then pic_last_error says why).  The workspace holds
 * two particle buffers of `capacity` slots (16 B each, FP64), the field arrays
 * twice (leap-frog ping-pong), the current, kick and Poisson arrays, the
 * counters and the sort and profile scratch. */
size_t pic_workspace_bytes(const pic_params *p);

/* Create a tube: validate p, carve the workspace (device, 256-byte aligned,
 * ws_bytes >= pic_workspace_bytes(p)), fill rho_GJ and solve eq. (4) for the
 * empty tube on the device, set E_z = -dphi/dz, E_r = phi/R, B_phi = 0
 * (sec. 2: the tube starts empty, B_phi(0) = 0).  hip_stream is a hipStream_t
 * (NULL = the null stream); all work of this handle is ordered on it.
 * Errors: PIC_EABI, PIC_EINVAL, PIC_ECFL, PIC_EWORKSPACE, PIC_EDEVICE. */
pic_status pic_init(const pic_params *p, void *d_workspace, size_t ws_bytes, void *hip_stream,
                    pic_handle **out);

/* Append n particles (positions x in cell units, 0 <= x < N; momenta u finite).
 * mem: 0 = host arrays, 1 = device arrays.  Before the first step the fields are
 * solved again from eq. (4) with the charge of all loaded particles (warm start);
 * afterwards the particles are added as they are.  Synchronises the stream.
 * Errors: PIC_EINVAL (range), PIC_ENONFINITE, PIC_ECAPACITY, PIC_EDEVICE. */
pic_status pic_inject(pic_handle *h, int64_t n, const double *x, const double *u, int32_t mem);

/* Enqueue n_steps PIC cycles on the stream and return.  Each cycle: push and
 * charge-conserving deposit, boundary removal, leap-frog field update, SCLF
 * injection; every sort_every cycles a cell sort that drops removed particles.
 * Errors: PIC_EINVAL (n_steps < 0), PIC_EDEVICE. */
pic_status pic_step(pic_handle *h, int64_t n_steps);

/* Synchronise the stream and fill *out (scalars always; arrays where non-NULL).
 * Returns PIC_EDEVSTATUS if a status bit is latched (out is still filled). */
pic_status pic_diagnostics(pic_handle *h, const pic_diag_req *req, pic_diag *out);

/* For callers that cannot allocate (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the signed-gamma profile of
 * pic_diagnostics -- n_bins uniform bins over [0, N) with, per bin, the count,
 * the 128-bit sum of sign(u) gamma in units of 2^-32 (low word, signed high
 * word), the min and the max -- written to caller-provided device arrays of
 * n_bins entries (any of them may be NULL).  Asynchronous on the handle's
 * stream: it enqueues kernels only, synchronises nothing and allocates nothing;
 * the bins accumulate in a fixed device array of the library (at most 65,536
 * bins: 2.5 MiB per GPU, held until the process ends) instead of the
 * workspace.  Every call on a GPU reuses that GPU's array and clears the bins
 * it uses first: calls that overlap on one GPU (from different streams or
 * threads) race.  The handle's device must be current.  The values equal, bit
 * for bit, pic_diagnostics' prof_count, prof_sum_lo, prof_sum_hi, prof_min and
 * prof_max (an empty bin has min +inf and max -inf).  Errors: PIC_EINVAL
 * (n_bins outside [1, 65536], a batch handle), PIC_ESTATE (the t = 0 field
 * solve of a batch tube is still pending, or another device is current),
 * PIC_EDEVICE. */
pic_status pic_profile_noalloc(pic_handle *h, int32_t n_bins, int64_t *d_count, uint64_t *d_sum_lo,
                               int64_t *d_sum_hi, double *d_min, double *d_max);

/* Synchronise and copy the live particles, in slot order, to host arrays of
 * `cap` entries; *n_out receives the live count (PIC_ECAPACITY if cap is short). */
pic_status pic_read_particles(pic_handle *h, double *x, double *u, int64_t cap, int64_t *n_out);

/* Overwrite the fields from host arrays (any may be NULL to keep it): E_z [N],
 * E_r [N+1], B_phi [N]; the kick array follows E_z.  For tests that start from
 * a prescribed field.  Synchronises the stream. */
pic_status pic_write_fields(pic_handle *h, const double *ez, const double *er, const double *b_phi);

/* Per-kernel device time of a stepping run. */
typedef struct pic_timing {
    double push_ms;         /* summed device time of the particle push + deposit kernels */
    double field_ms;        /* summed device time of the field update + injection kernels */
    double sort_ms;         /* summed device time of the cell sort / compaction sequences */
    double total_ms;        /* device time from the first to the last kernel              */
    int64_t push_launches;
    int64_t field_launches;
    int64_t sort_launches;
    int64_t particle_steps; /* sum over the steps of the slots the push visited           */
} pic_timing;

/* pic_step(h, n_steps) with a HIP event recorded on the handle's stream around
 * every kernel group; synchronises at the end and fills *out.  Used to measure
 * per-kernel durations; the events add a little launch overhead.
 * Errors: as pic_step, plus PIC_EDEVICE for event failures. */
pic_status pic_step_timed(pic_handle *h, int64_t n_steps, pic_timing *out);

/* pic_set_push_config flags */
enum {
    PIC_PUSH_NONTEMPORAL = 1u /* stream particles with nontemporal loads and stores */
};

/* Launch shape of the particle push: threads per block (64, 128, 256, 512) and
 * particle slots per thread.  FP64: 2, 4 (up to 256 threads) or 8 (up to 128
 * threads); a thread takes per_thread/2 pairs of consecutive slots, 2*block
 * slots apart.  FP32-bulk: 4 (4 consecutive low-stream slots per thread; in
 * the high stream two pairs of slots 128 apart).  pic_init sets 128 x 2 (FP64) or
 * 128 x 4 (FP32-bulk), both with PIC_PUSH_NONTEMPORAL.
 * Results do not depend on the choice (integer deposition); the autotuner
 * picks the fastest.  Errors: PIC_EINVAL for an unsupported shape or flag. */
pic_status pic_set_push_config(pic_handle *h, int32_t block, int32_t per_thread, uint32_t flags);

/* ---- ensembles: many independent tubes stepped by one graph launch per round ----
 *
 * A batch holds n_tubes tubes of any sizes (each tube's parameters as for
 * pic_init; all tubes share the precision and sort_every).  pic_step on the
 * batch handle advances every tube.  Each step is a push kernel and a field
 * kernel over all tubes, over device lists of (tube, tile) work items, one
 * block per item.  No block waits for another;
 * the kernel boundary orders the phases.  Up to sort_every steps plus a batched
 * cell sort form a round, captured once in a HIP graph and replayed with one
 * launch.  A tube of a batch computes exactly what it computes when stepped
 * alone.  Before each push a one-block kernel lists the push items that hold
 * particles, so the blocks of the push grid (sized for every tube at capacity)
 * that find no work are the last ones.  pic_step_timed on a batch reports the
 * batched push kernels under push_ms (push_launches of them), the field kernels
 * and the work-list kernels under field_ms, and the sorts under sort_ms.
 * pic_sync on a batch checks every tube's status. */

/* Device bytes for a batch (header + every tube's workspace), 0 if invalid. */
size_t pic_batch_workspace_bytes(const pic_params *tubes, int32_t n_tubes);

/* Create a batch from n_tubes parameter sets (host array), carving the caller's
 * workspace (device, 256-byte aligned).  Each tube is initialised as by pic_init.
 * Errors: as pic_init; PIC_EINVAL if precision or sort_every differ. */
pic_status pic_init_batch(const pic_params *tubes, int32_t n_tubes, void *d_workspace, size_t ws_bytes,
                          void *hip_stream, pic_handle **out);

/* Borrowed handle of tube t (for pic_inject, pic_diagnostics, pic_read_particles,
 * pic_write_fields); stepping and release go through the batch handle. */
pic_status pic_batch_tube(pic_handle *batch, int32_t t, pic_handle **out);

/* pic_batch_set_config flags */
enum {
    PIC_BATCH_NO_GRAPH = 1u  /* launch every round directly instead of replaying a captured graph */
};

/* Launch shape of the batched kernels: threads per block (64..512) and slots
 * per thread (FP64: 2 or 4; FP32-bulk: 4).  Results do not depend on the
 * choice.  Errors: PIC_EINVAL for an unsupported shape or flag. */
pic_status pic_batch_set_config(pic_handle *batch, int32_t block, int32_t per_thread, uint32_t flags);

/* Current launch shape (any pointer may be NULL): threads per block, slots per
 * thread, and the blocks of one step's push and field kernels (one per tile of
 * every tube, particle tiles counted at capacity). */
pic_status pic_batch_get_config(pic_handle *batch, int32_t *block, int32_t *per_thread, int64_t *push_blocks,
                                int64_t *field_blocks);

/* ---- hand-written adjoint ----
 *
 * Loss L = mean Lorentz factor of the electrons that leave through z = L during
 * n_steps steps.  pic_adjoint_forward advances the tube by n_steps (the same
 * steps pic_step would take) while checkpointing every checkpoint_every steps
 * into the caller's device tape; pic_backward then runs the reverse sweep,
 * recomputing each segment from its checkpoint, and returns dL/d(parameters).  Every discrete
 * decision of the run is held fixed (injection counts, exits and returns, cell
 * crossings; the fixed-point rounding is taken as the identity), and the
 * macro-particle charge is the one pic_params fixes (set macro_charge so that
 * it does not move with rho_GJ).  rho_GJ enters only through the Poisson start
 * of eq. (4), whose transpose closes the sweep.  Requirements: PIC_FP64,
 * sort_every = 0, fields not frozen, a single tube (not a batch).  The device
 * status word is not changed; the tube ends in the state n_steps steps later. */
typedef struct pic_adjoint_out {
    double loss;            /* L                                                        */
    int64_t n_exit;         /* electrons in the mean                                    */
    double g_rate;          /* dL/d(charge factor of electrons injected during the run) */
    double g_kappa;         /* dL/d kappa (PIC_RHO_FRAME_DRAG, PIC_RHO_KNOTS, PIC_RHO_GR) */
    double g_amp;           /* dL/d A (PIC_RHO_UNIFORM, PIC_RHO_FRAME_DRAG, PIC_RHO_GR)  */
    double *g_rho;          /* host [N+1] or NULL: dL/d rho_GJ at the nodes             */
    double *g_knots;        /* host [n_knots] or NULL: dL/d theta_k (PIC_RHO_KNOTS)     */
    double forward_ms;      /* device time of the checkpointed forward                  */
    double backward_ms;     /* device time of the recompute + reverse sweep             */
} pic_adjoint_out;

/* Device bytes of the tape the adjoint needs (checkpoints, the recorded steps
 * of two segments, adjoint arrays), 0 if the handle cannot run the adjoint.
 * The reverse sweep of one segment overlaps the recompute of the previous one
 * on a second stream that pic_backward creates and destroys. */
size_t pic_adjoint_tape_bytes(pic_handle *h, int64_t n_steps, int32_t checkpoint_every);

/* The forward half: advance the tube by n_steps with a checkpoint every
 * checkpoint_every steps in the caller's device tape (256-byte aligned,
 * tape_bytes >= pic_adjoint_tape_bytes) and record the run on the handle; fills
 * out->loss, out->n_exit and out->forward_ms.  Synchronises the stream.
 * Errors: PIC_EINVAL (requirements above), PIC_EWORKSPACE (tape too small or
 * misaligned), PIC_EDEVICE. */
pic_status pic_adjoint_forward(pic_handle *h, int64_t n_steps, int32_t checkpoint_every, void *d_tape,
                               size_t tape_bytes, pic_adjoint_out *out);

/* The reverse half: the gradient of the recorded forward, scaled by dloss (the
 * derivative of the caller's objective with respect to L; 1 for L itself), into
 * out (g_rate, g_kappa, g_amp, and g_rho, g_knots where non-NULL; loss, n_exit,
 * forward_ms as recorded; backward_ms).  The tape must be the forward's and
 * untouched since, and the tube neither stepped nor changed in between
 * (PIC_ESTATE otherwise); it ends in the state the forward left, so the
 * reverse sweep may be run again (the same bits each time: every sum the sweep
 * shares between waves is an integer sum).  Synchronises the stream.
 * Errors: PIC_EINVAL, PIC_ESTATE, PIC_EDEVICE. */
pic_status pic_backward(pic_handle *h, double dloss, pic_adjoint_out *out);

/* pic_adjoint_forward followed by pic_backward with dloss = 1.
 * Errors: as the two. */
pic_status pic_run_adjoint(pic_handle *h, int64_t n_steps, int32_t checkpoint_every, void *d_tape,
                           size_t tape_bytes, pic_adjoint_out *out);

/* Synchronise the stream; PIC_EDEVSTATUS if a status bit is latched. */
pic_status pic_sync(pic_handle *h);

/* Replay recorded SCLF injection counts (the frozen discrete decisions of
 * finite-difference checks of the adjoint, sec. 2 injection rule): during steps
 * [first_step, first_step + n) the number injected is d_counts[step - first_step]
 * (clipped to the free capacity, which latches PIC_ST_CAPACITY) instead of
 * floor(E_surf / (4 pi q_m)).  d_counts is device memory owned by the caller and
 * must stay valid while the schedule is set; n = 0 clears it.  Single tubes
 * only (PIC_ESTATE for a batch or its tubes); pic_run_adjoint honours it too. */
pic_status pic_set_injection_schedule(pic_handle *h, const int64_t *d_counts, int64_t first_step, int64_t n);

/* Checkpoint of a tube's state in caller-provided host memory: completed steps,
 * device counters, E_z, E_r, B_phi, the last step's current and the occupied
 * particle slots.  With buf == NULL only *bytes (the size needed) is set;
 * otherwise cap must be >= that size.  Synchronises the tube's stream.  A tube of
 * a batch can be saved through its pic_batch_tube handle. */
pic_status pic_save(pic_handle *h, void *buf, size_t cap, size_t *bytes);

/* Restore a pic_save state into a single tube created with the same parameters
 * (capacity may differ if the slots fit).  Stepping afterwards continues
 * bit for bit as the saved tube would have.  Errors: PIC_EINVAL for another
 * tube's parameters or a damaged buffer, PIC_ECAPACITY if the slots do not fit,
 * PIC_ESTATE for a batch or its tubes.  Synchronises the stream. */
pic_status pic_load(pic_handle *h, const void *buf, size_t bytes);

/* Measurement helper, not part of the method: copy `bytes` bytes from d_src to
 * d_dst (device memory, both 16-byte aligned, bytes a multiple of 16, the two
 * ranges disjoint) with one 16-byte nontemporal load and store per thread, the
 * simplest stream the HBM can serve.  Its rate is the achievable bandwidth the
 * particle push is compared with.  Asynchronous on hip_stream (NULL: the
 * default stream); PIC_EINVAL for a misaligned, odd-sized or overlapping
 * request or bytes >= 2^40. */
pic_status pic_stream_copy(const void *d_src, void *d_dst, size_t bytes, void *hip_stream);

/* Release the handle (the caller still owns workspace and stream). */
pic_status pic_destroy(pic_handle *h);

#ifdef __cplusplus
}
#endif
#endif /* PCPIC_H */
