// pcpic_internal.h -- private layout shared by the host code and the gfx950 kernels.
//
// Not part of the C ABI.  Everything here lives in the caller-provided device
// workspace; see pcpic.h for the public contract.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "pcpic.h"

namespace pcpic {

// Constants of one tube, computed once on the host in IEEE double (the library
// is built with -ffp-contract=off) and passed to every kernel by value.
// The order of each floating-point operation is fixed: the device code
// evaluates every formula of the step with exactly these operands.
struct Consts {
    int64_t N;        // cells
    int64_t cap;      // particle capacity
    int32_t P;        // fixed-point fraction bits
    uint32_t flags;   // PIC_* flags
    int32_t sub;      // log2 of the sort key's bins per cell
    int32_t gr_fast;  // PIC_GR_ALPHA: the lapse constants lie where the push's short division and square root apply
    int64_t oneP;     // 2^P
    double twoP;      // 2^P as a double
    double dz;        // L / N
    double dtdz;      // c dt / dz
    double dt;        // dtdz * dz
    double dtR;       // dt / R
    double invR;      // unused by the step; kept for diagnostics scaling
    double R;         // tube radius
    double qmdt;      // (q/m) dt
    double rho0;      // rho_GJ at node 0
    double qm;        // macro charge rho0 dz / ppc
    double qmP;       // qm / 2^P (charge of one weight unit)
    double fourpi;    // 4 pi
    double c4;        // fourpi * qmP: E_z change per unit of J
    double fqm;       // fourpi * qm: surface-field change per injected particle
    double hdz;       // dz / 2
    double tw;        // 2 dtdz (mirror update of E_r at node N)
    double cpois;     // fourpi dz^2 (Poisson right-hand side)
    double bdiag;     // -(2 + (dz/R)^2) (Poisson diagonal)
    double h2;        // (dz/R)^2
    // background density
    int32_t rho_kind;
    int32_t n_knots;
    double rho_amp, kappa, r_star, length;
    double gr_s;      // PIC_RHO_GR: (3/2) theta_* tan(i) cos(varphi)
    double gr_g;      // PIC_RHO_GR or PIC_GR_ALPHA: r_g / R_*
    double gr_cg;     // PIC_GR_ALPHA: dt (r_g/R_*) / (2 R_*); dt alpha alpha' = gr_cg / eta^2
};

// Slots per thread of the two FP32-bulk push streams: the low stream loads its
// three 4-byte fields as 16-byte vectors of 4 slots; the high stream takes 4
// slots too, as two pairs 128 slots apart (an 8-byte vector of position words
// and a 16-byte f64 momentum vector per pair, so that each access instruction
// covers one contiguous span), and one wave covers one group of HI_GROUP slots.
constexpr int F32_PPT_LO = 4;
constexpr int F32_PPT_HI = 4;

// Positions of the high stream (FP32-bulk, gamma at or above the threshold):
// 4 bytes per slot beside the 8-byte f64 momentum.  Slots form groups of
// HI_GROUP consecutive slots (the 256 slots one wave of the push takes).  The
// low HI_FRAC_BITS bits of a slot's word hold its offset in the cell in units
// of 2^-24.  A narrow group (header >= 0) keeps the cell minus the header in
// the high 8 bits; a wide group (header HI_WIDE) keeps zero there and the cell
// in the per-slot cell array, which only wide groups touch.  HI_DEAD marks a
// removed slot in both forms.  The push rewrites each group it moves as
// narrow, based at its lowest live cell, when its live cells span at most
// HI_SPAN cells, and as wide otherwise; the sort and the appends write wide
// groups.  Offsets on the 2^-24 grid are exact in f32, so a particle moves
// between the streams without a change of position (the low push snaps a
// particle's offset to the grid once its momentum reaches the threshold).
constexpr int HI_GROUP_LOG2 = 8;
constexpr int HI_GROUP = 1 << HI_GROUP_LOG2;
// Steps per captured round of a tube that never sorts (even: the field and
// current buffers end a round in the parity they started it in).
constexpr int64_t GRAPH_ROUND = 32;

// Faces per thread of the field update (field_body.h): a wave takes 256 faces,
// as two pairs per lane where the flat update applies.
constexpr int FIELD_CPT = 4;

constexpr int HI_FRAC_BITS = 24;
constexpr unsigned HI_FRAC_MASK = (1u << HI_FRAC_BITS) - 1u;
constexpr unsigned HI_DEAD = 0xFFFFFFFFu;
constexpr int HI_WIDE = -1;
constexpr int HI_SPAN = 254;
static_assert(HI_GROUP == 64 * F32_PPT_HI, "a high-stream group is the slots of one wave of the push");

// The least float f with f >= v (v >= 0 finite): for a float x, |x| >= f exactly
// when (double)|x| >= v, so an f32 test picks the same particles as the f64 one.
__host__ __device__ inline float f32_at_least(double v)
{
    float f = (float)v;
    if ((double)f < v) f = __builtin_bit_cast(float, __builtin_bit_cast(unsigned, f) + 1u);
    return f;
}

__host__ __device__ inline int64_t hi_groups(int64_t slots) { return (slots + HI_GROUP - 1) >> HI_GROUP_LOG2; }
// Cell of a live slot from its word, its group's header and (wide groups) the cell array.
__host__ __device__ inline int hi_cell(unsigned w, int hdr, int wide_cell)
{
    return hdr >= 0 ? hdr + (int)(w >> HI_FRAC_BITS) : wide_cell;
}
__host__ __device__ inline float hi_offset(unsigned w) { return (float)(w & HI_FRAC_MASK) * 0x1p-24f; }
// The word of (cell, frac) in a group with header hdr (HI_WIDE: frac alone).
__host__ __device__ inline unsigned hi_word(int cell, unsigned frac, int hdr)
{
    return hdr >= 0 ? ((unsigned)(cell - hdr) << HI_FRAC_BITS) | frac : frac;
}
// An offset in [0, 1) on the 2^-24 grid: (cell, frac), carried into the next
// cell when it rounds up to 1.
__host__ __device__ inline void hi_snap(double off, int &cell, unsigned &frac)
{
    const double q = rint(off * 16777216.0);
    const bool up = q >= 16777216.0;
    cell += up ? 1 : 0;
    frac = up ? 0u : (unsigned)q;
}

// Cell-sort keys.  A live particle's key is its cell refined into 2^sub bins
// (so that a wave's particles sit within a small fraction of a cell and cross
// cell edges together); in FP32-bulk mode the keys of the high stream follow
// those of the low stream, (N + 1) 2^sub of them.
__host__ __device__ inline int64_t sort_key_count(const Consts &c, bool f32)
{
    return (f32 ? 2 * (c.N + 1) : c.N) << c.sub;
}
__host__ __device__ inline int64_t sort_low_keys(const Consts &c) { return (c.N + 1) << c.sub; }
constexpr int SORT_SCAN_TILE = 1024;   // keys per block of the three-phase scan
constexpr int SORT_BLOCK = 256;        // threads per block of the scatter and histogram passes
constexpr int SORT_PPT = 4;            // consecutive slots per thread in those passes
constexpr int SORT_TILE = SORT_BLOCK * SORT_PPT;
__device__ inline int64_t sort_key_f64(const Consts &c, double x)
{
    return (int64_t)floor(x * (double)(1 << c.sub));   // exact scaling by a power of two
}
__device__ inline int64_t sort_key_f32(const Consts &c, int cell, float off, bool high)
{
    const int64_t k = ((int64_t)cell << c.sub) + (int64_t)(off * (float)(1 << c.sub));
    return high ? sort_low_keys(c) + k : k;
}

// Device-side counters (one per tube), 256-byte aligned in the workspace.
struct DevCounters {
    int64_t n_slots;        // occupied particle slots [0, n_slots) (live + removed)
    int64_t n_alive;        // live particles (maintained by sort / inject)
    int64_t n_injected;
    int64_t n_exit;
    int64_t n_absorb;
    int64_t w0;             // node-0 weight tally of the step in progress
    int64_t w0_last;        // node-0 weight of the last completed step
    int64_t last_ninj;
    unsigned long long exit_lo;  // 128-bit exit-gamma sum, units 2^-32
    long long exit_hi;
    unsigned long long status;   // PIC_ST_* bits
    double e_surf;
    int64_t step;
    int64_t n_removed;      // removed since the last compaction (exit + absorb + lost)
    unsigned long long gauss_max_bits;  // diagnostics: max |G| (non-negative double bits)
    unsigned long long rho_max_bits;    // max |rho_GJ| (non-negative double bits)
    int64_t bad_inputs;                 // rejected particles of the last pic_inject
    int64_t n_slots_hi;                 // FP32-bulk: occupied slots of the high-gamma stream
};

struct Workspace {
    double *x[2], *u[2];    // particle double buffer (FP64)
    // FP32-bulk streams (double-buffered): low (cell, offset, u f32); high (position
    // word, u f64, and per group a header; cells of wide groups in hw)
    int *cl[2];
    float *ol[2], *ul[2];
    unsigned *hp[2];
    int *hw[2];
    int *hg[2];
    double *uh[2];
    float *k32;             // f32 kick array (q/m) dt E_z (FP32-bulk low stream)
    double *stage_x, *stage_u;  // FP32-bulk: staging of injected particles
    int64_t stage_cap;
    long long *stage_blk;       // FP32-bulk: per-256-particle block counts of a staged append
    long long *stage_base;      // [2] slot counts of the two streams before the append
    long long *total_lo;    // FP32-bulk sort: low-destination total
    double *ez[2], *er[2], *b[2];
    int64_t *j[2];          // fixed-point current, ping-pong per step
    double *rho_gj;
    int64_t *w;             // CIC node weights (Poisson, diagnostics)
    double *phi, *cp, *dp, *rhs;
    double *knots;
    DevCounters *ctr;
    // profile bins
    long long *pcount;
    unsigned long long *plo;
    long long *phi128;
    long long *pmin, *pmax; // ordered-integer images of doubles
    double *gauss;
    // sort scratch
    long long *cell_count;  // [N + 1]
    long long *cell_off;    // [N + 1]
    long long *blk_sum;     // [scan blocks + 1]
    size_t bytes;
};

// Pointers kept in a device-side descriptor carry the global address space:
// a kernel that reads them from memory then issues global memory instructions,
// as it does for pointers passed as kernel arguments, instead of flat ones
// (which also wait on the LDS counter and cannot use a scalar base).
template <class T>
using gptr = __attribute__((address_space(1))) T *;
template <class T>
__host__ __device__ __forceinline__ gptr<T> to_global(T *p)
{
    return (gptr<T>)p;
}
template <class T>
__host__ __device__ __forceinline__ T *generic(gptr<T> p)
{
    return (T *)p;
}

// Device descriptor of one tube of a batch: constants and the base pointers of
// both parities of every ping-pong array.
struct TubeDev {
    Consts c;
    gptr<double> x[2], u[2];
    gptr<int> cl[2];
    gptr<float> ol[2], ul[2];
    gptr<unsigned> hp[2];
    gptr<int> hw[2];
    gptr<int> hg[2];
    gptr<double> uh[2];
    gptr<double> ez[2], er[2], b[2];
    gptr<int64_t> j[2];
    gptr<float> k32;
    gptr<DevCounters> ctr;
    gptr<long long> cell_count, cell_off, total_lo, blk_sum;
    gptr<double> rhs, cp, dp, phi;   // Poisson solve of eq. (4)
    double u_hi;
    int64_t push_tiles;      // push tiles at capacity (FP32-bulk: of BLOCK*F32_PPT_HI slots)
    int64_t push_tiles_hi;   // FP32-bulk: 1 more item, as the two streams may each end in a partial tile
    int64_t sort_chunks;  // sort tiles (SORT_TILE slots) per particle stream at capacity
    int64_t n_keys;       // sort keys (N, or 2(N+1) in FP32-bulk mode)
};

// Scale of the fixed-point sums of the reverse sweep (see k_adjoint.hip): the
// maxima of the adjoints a reverse step starts from (bit images of
// non-negative doubles, in three word sets that rotate over the steps), the
// step's fixed-point rate-gradient sum and the running total.
struct AdjScale {
    unsigned long long max_lu[3], max_lx[3], max_lez[3];   // word sets rotating over the reverse steps
    unsigned long long g_lo;          // the step's rate-gradient sum, fixed point (low 32-bit parts)
    long long g_hi;                   //   (the rest)
    double grate;                     // dL/d rate summed over the reverse steps done, in step order
};

// Pointers of one reverse step of the adjoint (see k_adjoint.hip).
struct AdjStepPtrs {
    const double *X, *U, *ez;        // recorded slots and E_z before the step
    const int64_t *n_s, *n_next;     // slot counts before / after the step (device)
    int64_t n_pre, n_exit;
    double *lx, *lu, *lez;
    const double *ler;               // E_r adjoint after the step; lern receives the one before it
    double *lern, *lb;
    const double *lbp;               // dL/dB^{s+1/2} through E^{s+1}; lbpn receives that of step s-1
    double *lbpn;
    unsigned long long *lk_lo;       // kick adjoint, fixed point (low 32-bit parts)
    long long *lk_hi;                //   (the rest)
    AdjScale *scale;
    int rot;                         // reverse steps done, mod 3 (the word set of the step's maxima)
};

// Byte layout of the workspace (offsets from the base).  Computing it with a
// null base gives the size.
Workspace carve(const pic_params &p, uint8_t *base);

// log2 of the sort key's bins per cell: about 32 particles per bin at the
// nominal density (ppc per cell), at most 16 bins.
int sort_sub_log2(const pic_params &p);

}  // namespace pcpic

// The recorded forward of an adjoint run (pic_adjoint_forward), which
// pic_backward reverses: the caller's tape and what the sweep needs besides it.
struct AdjRecord {
    bool valid = false;
    void *tape = nullptr;
    size_t tape_bytes = 0;
    int64_t T = 0, K = 0;       // steps, checkpoint period
    int64_t n_pre = 0;          // slots before the run (the injected class starts here)
    int64_t n_exit = 0;         // exits of the run (the loss's normalisation)
    double loss = 0.0, forward_ms = 0.0;
    int64_t step_end = 0;       // the tube's step count after the forward
    int64_t mut = 0;            // the tube's change count after the forward
    int jb_final = 0;           // current buffer parity after the forward
};

struct pic_handle {
    pic_params p{};
    std::vector<double> knots;
    pcpic::Consts c{};
    pcpic::Workspace ws{};
    hipStream_t stream = nullptr;
    int pbuf = 0;       // current particle buffer
    int fbuf = 0;       // field buffer holding E^n, B^{n-1/2}
    int jbuf = 0;       // current buffer that the next step deposits into
    int64_t step = 0;   // steps enqueued
    int push_block = 64;
    int push_ppt = 2;
    int push_nt = 1;    // nontemporal particle-stream access
    double u_hi = 0.0;  // FP32-bulk: |u| from which a particle belongs to the FP64 stream
    int push_grid = 0;  // 0 = derived from the device
    const int64_t *d_sched = nullptr;   // replayed injection counts (caller's device array)
    int64_t sched_first = 0, sched_n = 0;
    bool hist_on = false;               // this step also counts the sort keys (a sort follows)
    bool poisson_pending = false;       // tube of a batch: eq. (4) to be solved with the batch
    int32_t *d_pending = nullptr;       // batch: device list of tubes to solve together
    int n_cu = 256;
    int dev = 0;        // device ordinal current at pic_init
    int64_t mut = 0;    // changes of the tube's state other than steps (inject, load, field or schedule writes)
    AdjRecord adj;      // the last recorded adjoint forward
    // batch (ensemble) handles
    bool is_batch = false;
    pic_handle *parent = nullptr;               // set on the tubes of a batch
    std::vector<pic_handle *> tubes;
    pcpic::TubeDev *d_tubes = nullptr;
    int64_t *d_live_pref = nullptr;             // [n + 1] prefix of the push items holding particles
    int64_t *d_live_counts = nullptr;           // [2n] slots of each tube's two streams (FP64: n, 0)
    int32_t *d_push_map = nullptr;              // push item -> tube of the coming step (k_batch_worklist)
    int64_t push_map_cap = 0;                   // entries of d_push_map (at least the push grid)
    int64_t *d_field_pref = nullptr, *d_sort_pref = nullptr, *d_key_pref = nullptr;
    int64_t *d_scan_pref = nullptr;             // [n + 1] prefix of 1024-key scan blocks
    int32_t *d_field_map = nullptr;             // cell tile -> tube
    int32_t *d_chunk_map = nullptr, *d_scan_map = nullptr;
    int batch_block = 256, batch_ppt = 2;
    int64_t batch_push_items = 0, batch_field_items = 0, batch_sort_items = 0, batch_keys = 0, batch_scan_blocks = 0;
    hipGraphExec_t graph[8] = {};   // one round, keyed by the (field, current, particle) buffer parities
    int64_t graph_steps = 0;
    bool use_graph = true;
};

namespace pcpic {

// ---- kernel launchers (each enqueues on h->stream, returns hipError_t) ----
hipError_t launch_rho_gj(pic_handle *h);
hipError_t launch_weights(pic_handle *h, int64_t *w_out);
hipError_t launch_poisson(pic_handle *h);
hipError_t launch_poisson_rhs(pic_handle *h);
hipError_t launch_fields_from_phi(pic_handle *h);
hipError_t launch_thomas_batch(pic_handle *b, const int32_t *d_list, int n);
hipError_t launch_push_f64(pic_handle *h);
hipError_t launch_push_f32(pic_handle *h);
hipError_t launch_push_f64_ptrs(pic_handle *h, const double *X, const double *U, double *Xo, double *Uo,
                                const double *ez);
hipError_t launch_field_ptrs(pic_handle *h, const double *ezo, const double *ero, const double *bo, double *ezn,
                             double *ern, double *bn, double *X, double *U);
hipError_t launch_weights32(pic_handle *h, int64_t *w_out);
// Profile bins: count, 128-bit sum (low and high words), ordered bit images of min and max.
struct ProfPtrs {
    long long *cnt;
    unsigned long long *lo;
    long long *hi;
    long long *mn, *mx;
};
hipError_t launch_profile32(pic_handle *h, int nbins, const ProfPtrs &p);
// The profile accumulated into the bins p (cleared first; clear_gauss also clears the
// Gauss maximum of the diagnostics), and copied out in the caller's layout.
hipError_t launch_profile_into(pic_handle *h, int nb, const ProfPtrs &p, bool clear_gauss);
hipError_t launch_profile_finish(pic_handle *h, int nb, const ProfPtrs &p, int64_t *count, uint64_t *sum_lo,
                                 int64_t *sum_hi, double *vmin, double *vmax);
hipError_t launch_sort32_hist(pic_handle *h);
hipError_t launch_sort32_scatter(pic_handle *h);
hipError_t launch_append_staged(pic_handle *h, int64_t n, bool check_only);
hipError_t launch_scan(pic_handle *h, int64_t n_keys);
hipError_t launch_batch_steps(pic_handle *h, int nsteps, bool hist_last, hipEvent_t *ev = nullptr);
hipError_t launch_copy_slots(pic_handle *h, const double *X, const double *U, double *Xc, double *Uc);
hipError_t launch_record_slots(pic_handle *h, int64_t *dst);
hipError_t launch_zero_f64(pic_handle *h, double *p, int64_t n);
hipError_t launch_adj_step(pic_handle *h, const AdjStepPtrs &s);
hipError_t launch_adj_finish(pic_handle *h, const double *lez, const double *ler, double *gphi, double *cp,
                             double *dp, double *g_rho, double *params);
hipError_t launch_zero_i64(pic_handle *h, int64_t *p, int64_t n);
hipError_t launch_batch_sort(pic_handle *h, bool hist_ready);
hipError_t launch_stream_copy(const void *src, void *dst, int64_t n16, hipStream_t stream);
bool batch_shape_supported(pic_handle *h);
TubeDev tube_dev(pic_handle *t);
hipError_t launch_field_inject(pic_handle *h);
hipError_t launch_check_append(pic_handle *h, int64_t base, int64_t n);
hipError_t launch_commit_append(pic_handle *h, int64_t n);
hipError_t launch_kick(pic_handle *h);
hipError_t launch_gauss(pic_handle *h);
hipError_t launch_profile(pic_handle *h, int n_bins);
// Counting sort; hist_ready = the key counts were accumulated by the step before.
hipError_t launch_sort(pic_handle *h, bool hist_ready);
hipError_t launch_clear_hist(pic_handle *h);

// The lapse of PIC_GR_ALPHA: alpha^2 = 1 - r_g/r at height z, eta = r/R_* = 1 + z/R_*;
// alpha at node i and at face i + 1/2.
__host__ __device__ inline double gr_alpha2(const Consts &c, double z)
{
    const double eta = 1.0 + z / c.r_star;
    return 1.0 - c.gr_g / eta;
}
__host__ __device__ inline double gr_alpha_node(const Consts &c, int64_t i) { return sqrt(gr_alpha2(c, (double)i * c.dz)); }
__host__ __device__ inline double gr_alpha_face(const Consts &c, int64_t i)
{
    return sqrt(gr_alpha2(c, ((double)i + 0.5) * c.dz));
}

// Goldreich-Julian density at node i (eqs. 5-7; the three kinds are listed in
// pcpic.h).  Used by the device fill and, at node 0, by the host to fix the
// macro charge, so both see the same value.
__host__ __device__ inline double rho_node(const Consts &c, const double *knots, int64_t i)
{
    const double z = (double)i * c.dz;
    if (c.rho_kind == PIC_RHO_UNIFORM) return -c.rho_amp;
    const double eta = 1.0 + z / c.r_star;
    const double e3 = eta * eta * eta;
    const double fd = 1.0 - c.kappa / e3;   // 1 - omega/Omega, eq. (7)
    if (c.rho_kind == PIC_RHO_FRAME_DRAG) return -(c.rho_amp * fd);
    if (c.rho_kind == PIC_RHO_GR) {
        // eq. (6): inclination term growing as eta^(1/2), gravitational redshift 1/alpha
        const double br = fd + c.gr_s * sqrt(eta);
        const double al = sqrt(1.0 - c.gr_g / eta);
        return -((c.rho_amp * br) / al);
    }
    const int64_t K = c.n_knots;
    const double s = (z * (double)(K - 1)) / c.length;
    int64_t k = (int64_t)floor(s);
    if (k > K - 2) k = K - 2;
    if (k < 0) k = 0;
    const double g = s - (double)k;
    const double th = knots[k] + g * (knots[k + 1] - knots[k]);
    return -(th * fd);
}

// Ordered-integer image of a double: monotone in the double's value.
__host__ __device__ inline long long ordered_bits(double d)
{
    long long k = __builtin_bit_cast(long long, d);
    return k < 0 ? (k ^ 0x7fffffffffffffffLL) : k;
}
__host__ __device__ inline double from_ordered_bits(long long k)
{
    long long b = k < 0 ? (k ^ 0x7fffffffffffffffLL) : k;
    return __builtin_bit_cast(double, b);
}

}  // namespace pcpic
