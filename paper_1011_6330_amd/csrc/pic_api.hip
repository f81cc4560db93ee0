// pic_api.hip -- host side of the C ABI declared in include/pcpic.h:
// parameter validation, workspace carve-up, the per-step launch sequence and
// the synchronising read-back calls.  No device memory is ever allocated here.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <new>
#include <vector>

#include "pcpic_internal.h"

using namespace pcpic;

namespace {

thread_local char g_err[512] = "";

pic_status fail(pic_status s, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return s;
}

#define HIP_OK(expr)                                                                    \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) return fail(PIC_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

constexpr size_t ALIGN = 256;
inline size_t align_up(size_t v) { return (v + ALIGN - 1) & ~(ALIGN - 1); }

int effective_bins(const pic_params &p) { return p.max_bins > 0 ? p.max_bins : 1024; }

// ---- the scratch of pic_profile_noalloc ----------------------------------
//
// A fixed device array instead of the handle's workspace, so that the call
// allocates nothing.  Each GPU the library runs on holds its own copy until the
// process ends; every call on a GPU reuses that GPU's copy (calls overlapping on
// one GPU race).  Host code never uses the array's name as an address: the
// device address comes from hipGetSymbolAddress, once per device, with that
// device current.
constexpr int NOALLOC_MAX_BINS = 65536;
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)5 * 8 * NOALLOC_MAX_BINS;   // 2.5 MiB
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[MAX_DEVICES] = {};

// Device address of `scratch` on the current device (looked up once per device).
pic_status scratch_of_current_device(int *dev_out, void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(PIC_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= MAX_DEVICES) return fail(PIC_EDEVICE, "device ordinal %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(PIC_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_dev[dev] = p;
    }
    if (dev_out) *dev_out = dev;
    if (out) *out = g_scratch_dev[dev];
    return PIC_OK;
}

pic_status validate(const pic_params *p)
{
    if (!p) return fail(PIC_EINVAL, "params is NULL");
    if (p->abi_version != PCPIC_ABI_VERSION)
        return fail(PIC_EABI, "abi_version %d, library is %d", p->abi_version, PCPIC_ABI_VERSION);
    if (p->precision != PIC_FP64 && p->precision != PIC_FP32_BULK)
        return fail(PIC_EINVAL, "precision %d not supported", p->precision);
    if (!isfinite(p->macro_charge)) return fail(PIC_EINVAL, "macro_charge must be finite");
    if (!(p->gamma_fp64 == 0.0 || (p->gamma_fp64 >= 1.0 && p->gamma_fp64 < 1e300)))
        return fail(PIC_EINVAL, "gamma_fp64 must be 0 (default 1e6) or >= 1");
    if (p->n_cells < 2 || p->n_cells > ((int64_t)1 << 31))
        return fail(PIC_EINVAL, "n_cells %lld out of range [2, 2^31]", (long long)p->n_cells);
    if (!(p->length > 0) || !isfinite(p->length)) return fail(PIC_EINVAL, "length must be > 0");
    if (!(p->radius > 0) || !isfinite(p->radius)) return fail(PIC_EINVAL, "radius must be > 0");
    if (!(p->dt_over_dz > 0 && p->dt_over_dz < 1))
        return fail(PIC_ECFL, "dt_over_dz = %g violates 0 < c dt/dz < 1", p->dt_over_dz);
    if (!isfinite(p->q_over_m)) return fail(PIC_EINVAL, "q_over_m must be finite");
    if (!(p->ppc > 0) || !isfinite(p->ppc)) return fail(PIC_EINVAL, "ppc must be > 0");
    if (p->rho_kind < PIC_RHO_UNIFORM || p->rho_kind > PIC_RHO_GR)
        return fail(PIC_EINVAL, "rho_kind %d unknown", p->rho_kind);
    if (!isfinite(p->rho_amp)) return fail(PIC_EINVAL, "rho_amp must be finite");
    if (p->rho_kind != PIC_RHO_UNIFORM && (!(p->r_star > 0) || !isfinite(p->kappa)))
        return fail(PIC_EINVAL, "frame dragging needs r_star > 0 and a finite kappa");
    if (p->rho_kind == PIC_RHO_KNOTS && (p->n_knots < 2 || !p->knots))
        return fail(PIC_EINVAL, "PIC_RHO_KNOTS needs n_knots >= 2 and a knot array");
    if (p->rho_kind == PIC_RHO_GR &&
        (!(p->rg_over_rstar >= 0.0 && p->rg_over_rstar < 1.0) || !(fabs(p->incl) < 1.5) ||
         !isfinite(p->theta_star) || !isfinite(p->cos_phi)))
        return fail(PIC_EINVAL, "PIC_RHO_GR needs r_g/R_* in [0, 1), |i| < 1.5 and finite theta_*, cos(varphi)");
    if (p->fp_bits < 16 || p->fp_bits > 36) return fail(PIC_EINVAL, "fp_bits %d not in [16, 36]", p->fp_bits);
    if (p->capacity < 1 || p->capacity > ((int64_t)1 << 40))
        return fail(PIC_EINVAL, "capacity %lld out of range", (long long)p->capacity);
    if (p->sort_every < 0) return fail(PIC_EINVAL, "sort_every must be >= 0");
    if (p->max_bins < 0 || p->max_bins > (1 << 20)) return fail(PIC_EINVAL, "max_bins out of range");
    if (p->flags & ~(PIC_NO_AUTO_INJECT | PIC_FREEZE_FIELDS | PIC_B_STEADY_INIT | PIC_GR_ALPHA))
        return fail(PIC_EINVAL, "unknown flag bits");
    if ((p->flags & PIC_GR_ALPHA) &&
        (p->precision != PIC_FP64 || !(p->rg_over_rstar >= 0.0 && p->rg_over_rstar < 1.0) || !(p->r_star > 0) ||
         !isfinite(p->r_star)))
        return fail(PIC_EINVAL, "PIC_GR_ALPHA needs PIC_FP64, r_g/R_* in [0, 1) and r_star > 0");
    return PIC_OK;
}

Consts make_consts(const pic_params &p, const double *knots)
{
    Consts c{};
    c.N = p.n_cells;
    c.cap = p.capacity;
    c.P = p.fp_bits;
    c.flags = p.flags;
    c.sub = sort_sub_log2(p);
    c.oneP = (int64_t)1 << p.fp_bits;
    c.twoP = ldexp(1.0, p.fp_bits);
    c.dz = p.length / (double)p.n_cells;
    c.dtdz = p.dt_over_dz;
    c.dt = c.dtdz * c.dz;
    c.dtR = c.dt / p.radius;
    c.R = p.radius;
    c.invR = 1.0 / p.radius;
    c.qmdt = p.q_over_m * c.dt;
    c.rho_kind = p.rho_kind;
    c.n_knots = p.rho_kind == PIC_RHO_KNOTS ? p.n_knots : 0;
    c.rho_amp = p.rho_amp;
    c.kappa = p.kappa;
    c.r_star = p.r_star;
    c.length = p.length;
    c.gr_s = p.rho_kind == PIC_RHO_GR ? ((1.5 * p.theta_star) * tan(p.incl)) * p.cos_phi : 0.0;
    c.gr_g = (p.rho_kind == PIC_RHO_GR || (p.flags & PIC_GR_ALPHA)) ? p.rg_over_rstar : 0.0;
    c.gr_cg = ((0.5 * c.dt) * c.gr_g) / p.r_star;
    {
        // the GR push's short forms need its fixed operands where the general
        // division's scaling steps do nothing (push_common.h, nr_div)
        auto num_ok = [](double v) { return v == 0.0 || (fabs(v) >= 0x1p-600 && fabs(v) <= 0x1p+400); };
        auto den_ok = [](double v) { return fabs(v) >= 0x1p-300 && fabs(v) <= 0x1p+300; };
        c.gr_fast = (num_ok(c.gr_g) && num_ok(c.gr_cg) && den_ok(p.r_star) && den_ok(c.dz)) ? 1 : 0;
    }
    c.rho0 = rho_node(c, knots, 0);
    c.qm = p.macro_charge != 0.0 ? p.macro_charge : (c.rho0 * c.dz) / p.ppc;
    c.qmP = c.qm / c.twoP;
    c.fourpi = 4.0 * M_PI;
    c.c4 = c.fourpi * c.qmP;
    c.fqm = c.fourpi * c.qm;
    c.hdz = 0.5 * c.dz;
    c.tw = 2.0 * c.dtdz;
    const double dz2 = c.dz * c.dz;
    c.cpois = c.fourpi * dz2;
    const double rr = c.dz / p.radius;
    const double h2 = rr * rr;
    c.h2 = h2;
    c.bdiag = -(2.0 + h2);
    return c;
}

}  // namespace

namespace pcpic {

int sort_sub_log2(const pic_params &p)
{
    int s = 0;
    while (s < 4 && p.ppc / (double)(1 << s) > 32.0) ++s;
    return s;
}

Workspace carve(const pic_params &p, uint8_t *base)
{
    Workspace w{};
    size_t off = 0;
    auto take = [&](size_t bytes) -> void * {
        const size_t o = align_up(off);
        off = o + bytes;
        return base ? (void *)(base + o) : nullptr;
    };
    const size_t N = (size_t)p.n_cells, cap = (size_t)p.capacity;
    const size_t nb = (size_t)effective_bins(p);
    const bool f32 = p.precision == PIC_FP32_BULK;
    if (!f32) {
        for (int k = 0; k < 2; ++k) {
            w.x[k] = (double *)take(cap * 8);
            w.u[k] = (double *)take(cap * 8);
        }
    } else {
        // each stream can hold every particle (a tube may sit entirely above or below
        // the threshold); 16-byte vector access needs 16-byte aligned streams
        for (int k = 0; k < 2; ++k) {
            w.cl[k] = (int *)take(cap * 4 + 16);
            w.ol[k] = (float *)take(cap * 4 + 16);
            w.ul[k] = (float *)take(cap * 4 + 16);
            w.hp[k] = (unsigned *)take(cap * 4 + 16);
            w.hw[k] = (int *)take(cap * 4 + 16);
            w.hg[k] = (int *)take((size_t)(hi_groups((int64_t)cap) + 16) * 4);
            w.uh[k] = (double *)take(cap * 8 + 32);
        }
        w.k32 = (float *)take(N * 4);
        w.stage_cap = (int64_t)(cap < ((size_t)1 << 22) ? cap : ((size_t)1 << 22));
        w.stage_x = (double *)take((size_t)w.stage_cap * 8);
        w.stage_u = (double *)take((size_t)w.stage_cap * 8);
        w.stage_blk = (long long *)take(((size_t)w.stage_cap / 256 + 1) * 8);
        w.stage_base = (long long *)take(16);
        w.total_lo = (long long *)take(8);
    }
    for (int k = 0; k < 2; ++k) {
        w.ez[k] = (double *)take(N * 8);
        w.er[k] = (double *)take((N + 1) * 8);
        w.b[k] = (double *)take(N * 8);
        w.j[k] = (int64_t *)take(N * 8);
    }
    w.rho_gj = (double *)take((N + 1) * 8);
    w.w = (int64_t *)take((N + 1) * 8);
    w.phi = (double *)take((N + 1) * 8);
    w.cp = (double *)take((N + 1) * 8);
    w.dp = (double *)take((N + 1) * 8);
    w.rhs = (double *)take((N + 1) * 8);
    w.knots = (double *)take((size_t)(p.n_knots > 0 ? p.n_knots : 1) * 8);
    w.ctr = (DevCounters *)take(sizeof(DevCounters));
    w.pcount = (long long *)take(nb * 8);
    w.plo = (unsigned long long *)take(nb * 8);
    w.phi128 = (long long *)take(nb * 8);
    w.pmin = (long long *)take(nb * 8);
    w.pmax = (long long *)take(nb * 8);
    w.gauss = (double *)take((N + 1) * 8);
    const size_t nkeys = (f32 ? 2 * (N + 1) : N + 1) << sort_sub_log2(p);   // sort keys (see sort_key_count)
    w.cell_count = (long long *)take(nkeys * 8);
    w.cell_off = (long long *)take(nkeys * 8);
    w.blk_sum = (long long *)take((nkeys / SORT_SCAN_TILE + 2) * 8);
    w.bytes = align_up(off);
    return w;
}

}  // namespace pcpic

namespace {

hipError_t launch_push(pic_handle *h)
{
    return h->p.precision == PIC_FP32_BULK ? launch_push_f32(h) : launch_push_f64(h);
}

// The first ns slots of the high stream of particle buffer b, decoded on the
// host: cell (-1 for a removed slot), offset (exact in f32) and u.
pic_status read_high_stream(pic_handle *h, int b, int64_t ns, std::vector<int> &cell, std::vector<float> &off,
                            std::vector<double> &u)
{
    const Workspace &w = h->ws;
    const size_t n = (size_t)ns, ng = (size_t)hi_groups(ns);
    std::vector<unsigned> hp(n);
    std::vector<int> hw(n), hg(ng);
    cell.assign(n, -1);
    off.assign(n, 0.0f);
    u.assign(n, 0.0);
    if (n == 0) return PIC_OK;
    HIP_OK(hipMemcpyAsync(hp.data(), w.hp[b], n * 4, hipMemcpyDeviceToHost, h->stream));
    HIP_OK(hipMemcpyAsync(hw.data(), w.hw[b], n * 4, hipMemcpyDeviceToHost, h->stream));
    HIP_OK(hipMemcpyAsync(hg.data(), w.hg[b], ng * 4, hipMemcpyDeviceToHost, h->stream));
    HIP_OK(hipMemcpyAsync(u.data(), w.uh[b], n * 8, hipMemcpyDeviceToHost, h->stream));
    HIP_OK(hipStreamSynchronize(h->stream));
    for (size_t i = 0; i < n; ++i) {
        const unsigned v = hp[i];
        off[i] = hi_offset(v);
        cell[i] = v == HI_DEAD ? -1 : hi_cell(v, hg[i >> HI_GROUP_LOG2], hw[i]);
    }
    return PIC_OK;
}

// Writes ns slots (cell, offset, u) as the high stream of particle buffer b, in
// the wide form; offsets go onto the stream's 2^-24 grid (those it wrote are
// on it already), a cell below 0 marks a removed slot.
pic_status write_high_stream(pic_handle *h, int b, int64_t ns, const int *cell, const float *off, const double *u)
{
    const Workspace &w = h->ws;
    const size_t n = (size_t)ns, ng = (size_t)hi_groups(ns);
    if (n == 0) return PIC_OK;
    std::vector<unsigned> hp(n);
    std::vector<int> hw(n), hg(ng, HI_WIDE);
    const int N = (int)h->c.N;
    for (size_t i = 0; i < n; ++i) {
        int c = cell[i];
        unsigned frac = 0;
        if (c >= 0) {
            hi_snap((double)off[i], c, frac);
            if (c >= N) { c = N - 1; frac = HI_FRAC_MASK; }
        }
        hw[i] = c;
        hp[i] = c >= 0 ? frac : HI_DEAD;
    }
    HIP_OK(hipMemcpyAsync(w.hp[b], hp.data(), n * 4, hipMemcpyHostToDevice, h->stream));
    HIP_OK(hipMemcpyAsync(w.hw[b], hw.data(), n * 4, hipMemcpyHostToDevice, h->stream));
    HIP_OK(hipMemcpyAsync(w.hg[b], hg.data(), ng * 4, hipMemcpyHostToDevice, h->stream));
    HIP_OK(hipMemcpyAsync(w.uh[b], u, n * 8, hipMemcpyHostToDevice, h->stream));
    HIP_OK(hipStreamSynchronize(h->stream));
    return PIC_OK;
}

pic_status read_counters(pic_handle *h, DevCounters *out)
{
    HIP_OK(hipMemcpyAsync(out, h->ws.ctr, sizeof(DevCounters), hipMemcpyDeviceToHost, h->stream));
    HIP_OK(hipStreamSynchronize(h->stream));
    return PIC_OK;
}

double i128_to_double(unsigned long long lo, long long hi)
{
    const __int128 v = ((__int128)hi << 64) | (__int128)lo;
    return (double)v;
}

}  // namespace

extern "C" {

int32_t pic_abi_version(void) { return PCPIC_ABI_VERSION; }

const char *pic_last_error(void) { return g_err; }

size_t pic_workspace_bytes(const pic_params *p)
{
    if (validate(p) != PIC_OK) return 0;
    return carve(*p, nullptr).bytes;
}

// defer_poisson: leave the t = 0 solve of eq. (4) to the batch the tube belongs to.
static pic_status init_tube(const pic_params *p, void *d_workspace, size_t ws_bytes, void *hip_stream, pic_handle **out,
                            bool defer_poisson = false)
{
    if (!out) return fail(PIC_EINVAL, "out is NULL");
    *out = nullptr;
    pic_status s = validate(p);
    if (s != PIC_OK) return s;
    const size_t need = carve(*p, nullptr).bytes;
    if (!d_workspace || ws_bytes < need)
        return fail(PIC_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    if (((uintptr_t)d_workspace) % ALIGN)
        return fail(PIC_EWORKSPACE, "workspace must be %zu-byte aligned", ALIGN);
    pic_handle *h = new (std::nothrow) pic_handle();
    if (!h) return fail(PIC_EINVAL, "out of host memory");
    h->p = *p;
    if (p->rho_kind == PIC_RHO_KNOTS) h->knots.assign(p->knots, p->knots + p->n_knots);
    h->p.knots = nullptr;
    h->c = make_consts(*p, h->knots.empty() ? nullptr : h->knots.data());
    if (!isfinite(h->c.qm) || !isfinite(h->c.rho0)) {
        delete h;
        return fail(PIC_EINVAL, "rho_GJ(0) is not finite");
    }
    h->stream = (hipStream_t)hip_stream;
    h->ws = carve(*p, (uint8_t *)d_workspace);
    {
        // set-up of the fixed scratch of pic_profile_noalloc on this device
        const pic_status ss = scratch_of_current_device(&h->dev, nullptr);
        if (ss != PIC_OK) {
            delete h;
            return ss;
        }
    }
    // the fastest measured push shapes (nontemporal particle streams)
    h->push_block = 128;
    h->push_ppt = p->precision == PIC_FP32_BULK ? 4 : 2;
    h->push_nt = 1;
    {
        const double g = p->gamma_fp64 > 0.0 ? p->gamma_fp64 : 1e6;
        h->u_hi = sqrt(g * g - 1.0);   // gamma >= g  <=>  |u| >= sqrt(g^2 - 1)
    }
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
        h->n_cu = ncu;
    auto bail = [&](hipError_t e, const char *what) {
        delete h;
        return fail(PIC_EDEVICE, "%s: %s", what, hipGetErrorString(e));
    };
    hipError_t e = hipMemsetAsync(h->ws.ctr, 0, sizeof(DevCounters), h->stream);
    if (e != hipSuccess) return bail(e, "clear counters");
    if (!h->knots.empty()) {
        e = hipMemcpyAsync(h->ws.knots, h->knots.data(), h->knots.size() * 8, hipMemcpyHostToDevice, h->stream);
        if (e != hipSuccess) return bail(e, "copy knots");
    }
    if ((e = launch_rho_gj(h)) != hipSuccess) return bail(e, "rho_gj");
    if (defer_poisson) {
        h->poisson_pending = true;
    } else if ((e = launch_poisson(h)) != hipSuccess) {
        return bail(e, "poisson");
    }
    *out = h;
    return PIC_OK;
}

pic_status pic_init(const pic_params *p, void *d_workspace, size_t ws_bytes, void *hip_stream, pic_handle **out)
{
    pic_status s = init_tube(p, d_workspace, ws_bytes, hip_stream, out);
    if (s != PIC_OK) return s;
    hipError_t e = hipStreamSynchronize((*out)->stream);
    if (e != hipSuccess) {
        delete *out;
        *out = nullptr;
        return fail(PIC_EDEVICE, "init sync: %s", hipGetErrorString(e));
    }
    return PIC_OK;
}

pic_status pic_inject(pic_handle *h, int64_t n, const double *x, const double *u, int32_t mem)
{
    if (!h) return fail(PIC_EINVAL, "handle is NULL");
    if (h->is_batch) return fail(PIC_EINVAL, "inject into a tube handle of the batch (pic_batch_tube)");
    if (n < 0 || (n > 0 && (!x || !u)) || (mem != 0 && mem != 1))
        return fail(PIC_EINVAL, "bad arguments to pic_inject");
    if (n == 0) return PIC_OK;
    h->mut += 1;
    if (mem == 0) {
        for (int64_t i = 0; i < n; ++i) {
            if (!isfinite(u[i]) || !isfinite(x[i])) return fail(PIC_ENONFINITE, "particle %lld not finite", (long long)i);
            if (!(x[i] >= 0.0 && x[i] < (double)h->c.N))
                return fail(PIC_EINVAL, "particle %lld at x = %g outside [0, N)", (long long)i, x[i]);
        }
    }
    DevCounters ctr;
    pic_status s = read_counters(h, &ctr);
    if (s != PIC_OK) return s;
    if (h->p.precision == PIC_FP32_BULK) {
        // a sort may move every particle into either stream, so both together
        // stay within the capacity
        if (ctr.n_slots + ctr.n_slots_hi + n > h->c.cap)
            return fail(PIC_ECAPACITY, "%lld + %lld slots used + %lld > capacity %lld", (long long)ctr.n_slots,
                        (long long)ctr.n_slots_hi, (long long)n, (long long)h->c.cap);
        const hipMemcpyKind kind = mem == 0 ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
        const int64_t ch = h->ws.stage_cap;
        HIP_OK(hipMemsetAsync(&h->ws.ctr->bad_inputs, 0, sizeof(int64_t), h->stream));
        for (int64_t o = 0; o < n; o += ch) {          // validate everything first
            const int64_t m = n - o < ch ? n - o : ch;
            HIP_OK(hipMemcpyAsync(h->ws.stage_x, x + o, (size_t)m * 8, kind, h->stream));
            HIP_OK(hipMemcpyAsync(h->ws.stage_u, u + o, (size_t)m * 8, kind, h->stream));
            HIP_OK(launch_append_staged(h, m, true));
        }
        s = read_counters(h, &ctr);
        if (s != PIC_OK) return s;
        if (ctr.bad_inputs)
            return fail(PIC_EINVAL, "%lld particles outside [0, N) or not finite", (long long)ctr.bad_inputs);
        for (int64_t o = 0; o < n; o += ch) {
            const int64_t m = n - o < ch ? n - o : ch;
            HIP_OK(hipMemcpyAsync(h->ws.stage_x, x + o, (size_t)m * 8, kind, h->stream));
            HIP_OK(hipMemcpyAsync(h->ws.stage_u, u + o, (size_t)m * 8, kind, h->stream));
            HIP_OK(launch_append_staged(h, m, false));
        }
        if (h->step == 0) {
            if (h->parent) h->poisson_pending = true;   // solved with the batch's other tubes
            else HIP_OK(launch_poisson(h));
        }
        HIP_OK(hipStreamSynchronize(h->stream));
        return PIC_OK;
    }
    if (ctr.n_slots + n > h->c.cap)
        return fail(PIC_ECAPACITY, "%lld slots used + %lld > capacity %lld", (long long)ctr.n_slots,
                    (long long)n, (long long)h->c.cap);
    const hipMemcpyKind kind = mem == 0 ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    HIP_OK(hipMemcpyAsync(h->ws.x[h->pbuf] + ctr.n_slots, x, (size_t)n * 8, kind, h->stream));
    HIP_OK(hipMemcpyAsync(h->ws.u[h->pbuf] + ctr.n_slots, u, (size_t)n * 8, kind, h->stream));
    HIP_OK(hipMemsetAsync(&h->ws.ctr->bad_inputs, 0, sizeof(int64_t), h->stream));
    HIP_OK(launch_check_append(h, ctr.n_slots, n));
    HIP_OK(launch_commit_append(h, n));
    s = read_counters(h, &ctr);
    if (s != PIC_OK) return s;
    if (ctr.bad_inputs) return fail(PIC_EINVAL, "%lld particles outside [0, N) or not finite", (long long)ctr.bad_inputs);
    if (h->step == 0) {
        if (h->parent) {
            h->poisson_pending = true;                   // solved with the batch's other tubes
        } else {
            HIP_OK(launch_poisson(h));
            HIP_OK(hipStreamSynchronize(h->stream));
        }
    }
    return PIC_OK;
}

static pic_status batch_advance(pic_handle *h, int64_t n, std::vector<hipEvent_t> *ev = nullptr,
                                pic_timing *tim = nullptr, std::vector<int64_t> *round_steps = nullptr);
static pic_status batch_status(pic_handle *h);
static void free_batch_graphs(pic_handle *h);

// One step of a single tube, launched directly: push (counting the sort keys
// on the step before a sort), field update + injection, and the sort.
static pic_status tube_step_direct(pic_handle *h)
{
    const bool sort_after = h->p.sort_every > 0 && (h->step + 1) % h->p.sort_every == 0;
    if (sort_after) HIP_OK(launch_clear_hist(h));
    h->hist_on = sort_after;            // the step counts the sort keys of its survivors
    hipError_t e1 = launch_push(h);
    hipError_t e2 = e1 == hipSuccess ? launch_field_inject(h) : e1;
    h->hist_on = false;
    HIP_OK(e2);
    h->fbuf ^= 1;
    h->jbuf ^= 1;
    h->step += 1;
    if (sort_after) HIP_OK(launch_sort(h, true));
    return PIC_OK;
}

// Captured rounds of a single tube are launch-shape and schedule specific.
static void free_tube_graphs(pic_handle *h)
{
    for (auto &g : h->graph) {
        if (g) (void)hipGraphExecDestroy(g);
        g = nullptr;
    }
}

pic_status pic_step(pic_handle *h, int64_t n_steps)
{
    if (!h) return fail(PIC_EINVAL, "handle is NULL");
    if (n_steps < 0) return fail(PIC_EINVAL, "n_steps < 0");
    if (h->parent) return fail(PIC_ESTATE, "a tube of a batch is stepped through its batch handle");
    if (h->is_batch) return batch_advance(h, n_steps);
    // A whole round of sort_every steps that starts on a round boundary is
    // replayed from a graph captured once per (field, current, particle)
    // buffer-parity state; other steps are launched one by one.  Both issue the
    // same kernels with the same arguments.  A tube that never sorts takes
    // rounds of GRAPH_ROUND steps the same way (an even count, so a round ends
    // in the parity state it started from).
    const bool sorts = h->p.sort_every > 0;
    const int64_t S = sorts ? h->p.sort_every : GRAPH_ROUND;
    while (n_steps > 0) {
        if (S > 1 && h->use_graph && h->step % S == 0 && n_steps >= S) {
            const int key = h->fbuf | (h->jbuf << 1) | (h->pbuf << 2);
            if (!h->graph[key]) {
                const int fb = h->fbuf, jb = h->jbuf, pb = h->pbuf;
                const int64_t st = h->step;
                hipGraph_t g = nullptr;
                bool ok = hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
                if (ok) {
                    pic_status rc = PIC_OK;
                    for (int64_t s = 0; s < S && rc == PIC_OK; ++s) rc = tube_step_direct(h);
                    const hipError_t e = hipStreamEndCapture(h->stream, &g);
                    ok = rc == PIC_OK && e == hipSuccess && g &&
                         hipGraphInstantiate(&h->graph[key], g, nullptr, nullptr, 0) == hipSuccess;
                    if (g) (void)hipGraphDestroy(g);
                }
                // the captured round has not run yet
                h->fbuf = fb;
                h->jbuf = jb;
                h->pbuf = pb;
                h->step = st;
                if (!ok) {
                    (void)hipGetLastError();
                    h->graph[key] = nullptr;
                    h->use_graph = false;   // launch directly from now on
                    continue;
                }
            }
            HIP_OK(hipGraphLaunch(h->graph[key], h->stream));
            h->fbuf ^= (int)(S & 1);
            h->jbuf ^= (int)(S & 1);
            if (sorts) h->pbuf ^= 1;
            h->step += S;
            n_steps -= S;
        } else {
            if (pic_status rc = tube_step_direct(h)) return rc;
            n_steps -= 1;
        }
    }
    return PIC_OK;
}

pic_status pic_step_timed(pic_handle *h, int64_t n_steps, pic_timing *out)
{
    if (!h || !out) return fail(PIC_EINVAL, "handle or out is NULL");
    if (n_steps < 0) return fail(PIC_EINVAL, "n_steps < 0");
    if (h->parent) return fail(PIC_ESTATE, "a tube of a batch is stepped through its batch handle");
    memset(out, 0, sizeof *out);
    if (n_steps == 0) return PIC_OK;
    if (h->is_batch) {
        std::vector<hipEvent_t> ev;
        std::vector<int64_t> rounds;
        pic_status rc = batch_advance(h, n_steps, &ev, out, &rounds);
        if (rc == PIC_OK && hipStreamSynchronize(h->stream) != hipSuccess) rc = fail(PIC_EDEVICE, "sync failed");
        if (rc == PIC_OK) {
            size_t k = 0;
            for (const int64_t r : rounds) {
                for (int64_t s = 0; s < r; ++s, k += 4) {
                    float a = 0, b = 0, c = 0;
                    (void)hipEventElapsedTime(&a, ev[k], ev[k + 1]);       // work list
                    (void)hipEventElapsedTime(&b, ev[k + 1], ev[k + 2]);   // push
                    (void)hipEventElapsedTime(&c, ev[k + 2], ev[k + 3]);   // field update + injection
                    out->push_ms += b;
                    out->field_ms += a + c;
                }
                float d = 0;
                (void)hipEventElapsedTime(&d, ev[k], ev[k + 1]);           // the sort (0 when none)
                out->sort_ms += d;
                k += 2;
            }
            if (!ev.empty()) {
                float tot = 0;
                (void)hipEventElapsedTime(&tot, ev.front(), ev.back());
                out->total_ms = tot;
            }
            int64_t live = 0;
            for (pic_handle *t : h->tubes) {
                DevCounters c;
                if (read_counters(t, &c) == PIC_OK) live += c.n_slots + c.n_slots_hi - c.n_removed;
            }
            out->particle_steps = live * n_steps;
        }
        for (auto &e : ev)
            if (e) (void)hipEventDestroy(e);
        return rc;
    }
    std::vector<hipEvent_t> ev((size_t)n_steps * 4, nullptr);
    std::vector<int64_t> slots_before((size_t)n_steps, 0);
    pic_status rc = PIC_OK;
    for (auto &e : ev) {
        if (hipEventCreate(&e) != hipSuccess) { rc = fail(PIC_EDEVICE, "hipEventCreate failed"); break; }
    }
    DevCounters ctr;
    if (rc == PIC_OK) rc = read_counters(h, &ctr);
    int64_t slots = ctr.n_slots + ctr.n_slots_hi;
    for (int64_t s = 0; s < n_steps && rc == PIC_OK; ++s) {
        hipEvent_t *e = &ev[(size_t)s * 4];
        const bool sort_after = h->p.sort_every > 0 && (h->step + 1) % h->p.sort_every == 0;
        if (sort_after && launch_clear_hist(h) != hipSuccess) { rc = fail(PIC_EDEVICE, "clear launch failed"); break; }
        h->hist_on = sort_after;
        const bool ok = hipEventRecord(e[0], h->stream) == hipSuccess && launch_push(h) == hipSuccess &&
                        hipEventRecord(e[1], h->stream) == hipSuccess && launch_field_inject(h) == hipSuccess &&
                        hipEventRecord(e[2], h->stream) == hipSuccess;
        h->hist_on = false;
        if (!ok) {
            rc = fail(PIC_EDEVICE, "launch failed in pic_step_timed");
            break;
        }
        h->fbuf ^= 1;
        h->jbuf ^= 1;
        h->step += 1;
        const bool sorted = sort_after;
        if (sort_after && launch_sort(h, true) != hipSuccess) { rc = fail(PIC_EDEVICE, "sort launch failed"); break; }
        if (hipEventRecord(e[3], h->stream) != hipSuccess) { rc = fail(PIC_EDEVICE, "event record failed"); break; }
        slots_before[(size_t)s] = sorted ? -1 : 0;
    }
    if (rc == PIC_OK && hipStreamSynchronize(h->stream) != hipSuccess) rc = fail(PIC_EDEVICE, "sync failed");
    if (rc == PIC_OK) {
        for (int64_t s = 0; s < n_steps; ++s) {
            hipEvent_t *e = &ev[(size_t)s * 4];
            float a = 0, b = 0, c = 0;
            (void)hipEventElapsedTime(&a, e[0], e[1]);
            (void)hipEventElapsedTime(&b, e[1], e[2]);
            (void)hipEventElapsedTime(&c, e[2], e[3]);
            out->push_ms += a;
            out->field_ms += b;
            out->push_launches += 1;
            out->field_launches += 1;
            if (slots_before[(size_t)s] < 0) {
                out->sort_ms += c;
                out->sort_launches += 1;
            }
        }
        float tot = 0;
        (void)hipEventElapsedTime(&tot, ev[0], ev[(size_t)n_steps * 4 - 1]);
        out->total_ms = tot;
        DevCounters end;
        if (read_counters(h, &end) == PIC_OK) {
            // slots visited: between sorts the slot count only grows by injection;
            // the average of the start and end counts times the steps
            out->particle_steps = (int64_t)((double)(slots + end.n_slots + end.n_slots_hi) * 0.5 * (double)n_steps);
        }
    }
    for (auto &e : ev)
        if (e) (void)hipEventDestroy(e);
    return rc;
}

pic_status pic_set_push_config(pic_handle *h, int32_t block, int32_t per_thread, uint32_t flags)
{
    if (!h) return fail(PIC_EINVAL, "handle is NULL");
    if (h->is_batch || h->parent) return fail(PIC_EINVAL, "batches take pic_batch_set_config");
    const bool bok = block == 64 || block == 128 || block == 256 || block == 512;
    // FP32-bulk always takes 4 slots per thread (16-byte vectors of 4-byte fields)
    const bool ok = bok && (h->p.precision == PIC_FP32_BULK ? per_thread == 4
                                                              : (per_thread == 2 || (per_thread == 4 && block != 512) ||
                                                                 (per_thread == 8 && block <= 128)));
    if (!ok || (flags & ~PIC_PUSH_NONTEMPORAL))
        return fail(PIC_EINVAL, "unsupported push shape (%d threads, %d per thread, flags %u)", block, per_thread,
                    flags);
    h->push_block = block;
    h->push_ppt = per_thread;
    h->push_nt = (flags & PIC_PUSH_NONTEMPORAL) ? 1 : 0;
    free_tube_graphs(h);
    return PIC_OK;
}

pic_status pic_sync(pic_handle *h)
{
    if (!h) return fail(PIC_EINVAL, "handle is NULL");
    if (h->is_batch) return batch_status(h);
    DevCounters ctr;
    pic_status s = read_counters(h, &ctr);
    if (s != PIC_OK) return s;
    if (ctr.status) return fail(PIC_EDEVSTATUS, "device status bits 0x%llx", (unsigned long long)ctr.status);
    return PIC_OK;
}

}  // extern "C"

static pic_status batch_resolve_pending(pic_handle *b);

// A tube of a batch whose t = 0 solve of eq. (4) is still pending (after
// pic_init_batch or a warm-start pic_inject) gets it now, together with every
// other pending tube of its batch (one batched Thomas launch).
static pic_status resolve_pending(pic_handle *h)
{
    if (!h->poisson_pending) return PIC_OK;
    if (h->parent) return batch_resolve_pending(h->parent);
    HIP_OK(launch_poisson(h));
    HIP_OK(hipStreamSynchronize(h->stream));
    h->poisson_pending = false;
    return PIC_OK;
}

// Every pending tube of a batch: the right-hand sides, one Thomas block per
// tube in a single launch, then the fields.  Same kernels and arithmetic as a
// single tube's solve.
static pic_status batch_resolve_pending(pic_handle *b)
{
    std::vector<int32_t> list;
    for (size_t t = 0; t < b->tubes.size(); ++t)
        if (b->tubes[t]->poisson_pending) list.push_back((int32_t)t);
    if (list.empty()) return PIC_OK;
    for (int32_t t : list) HIP_OK(launch_poisson_rhs(b->tubes[(size_t)t]));
    HIP_OK(hipMemcpyAsync(b->d_pending, list.data(), 4 * list.size(), hipMemcpyHostToDevice, b->stream));
    HIP_OK(launch_thomas_batch(b, b->d_pending, (int)list.size()));
    for (int32_t t : list) HIP_OK(launch_fields_from_phi(b->tubes[(size_t)t]));
    HIP_OK(hipStreamSynchronize(b->stream));
    for (int32_t t : list) b->tubes[(size_t)t]->poisson_pending = false;
    return PIC_OK;
}

extern "C" {

pic_status pic_diagnostics(pic_handle *h, const pic_diag_req *req, pic_diag *out)
{
    if (!h || !out) return fail(PIC_EINVAL, "handle or out is NULL");
    if (h->is_batch) return fail(PIC_EINVAL, "diagnostics are per tube (pic_batch_tube)");
    if (pic_status sp = resolve_pending(h)) return sp;
    const int nb = req ? req->n_bins : 0;
    const bool want_gauss = req && req->want_gauss;
    if (nb < 0 || nb > effective_bins(h->p)) return fail(PIC_EINVAL, "n_bins %d > max_bins", nb);
    if (req && !(req->gauss_tol >= 0.0)) return fail(PIC_EINVAL, "gauss_tol must be >= 0");
    const int64_t N = h->c.N;
    const Workspace &w = h->ws;
    HIP_OK(launch_profile(h, nb));   // also clears the Gauss maximum
    if (want_gauss || out->gauss) HIP_OK(launch_gauss(h));
    else if (out->weights) HIP_OK(launch_weights(h, w.w));
    DevCounters ctr;
    HIP_OK(hipMemcpyAsync(&ctr, w.ctr, sizeof ctr, hipMemcpyDeviceToHost, h->stream));
    const int f = h->fbuf;
    if (out->ez) HIP_OK(hipMemcpyAsync(out->ez, w.ez[f], (size_t)N * 8, hipMemcpyDeviceToHost, h->stream));
    if (out->er) HIP_OK(hipMemcpyAsync(out->er, w.er[f], (size_t)(N + 1) * 8, hipMemcpyDeviceToHost, h->stream));
    if (out->b_phi) HIP_OK(hipMemcpyAsync(out->b_phi, w.b[f], (size_t)N * 8, hipMemcpyDeviceToHost, h->stream));
    if (out->rho_gj) HIP_OK(hipMemcpyAsync(out->rho_gj, w.rho_gj, (size_t)(N + 1) * 8, hipMemcpyDeviceToHost, h->stream));
    if (out->j_last)
        HIP_OK(hipMemcpyAsync(out->j_last, w.j[1 - h->jbuf], (size_t)N * 8, hipMemcpyDeviceToHost, h->stream));
    if (out->weights) HIP_OK(hipMemcpyAsync(out->weights, w.w, (size_t)(N + 1) * 8, hipMemcpyDeviceToHost, h->stream));
    // The L2 norm of the residual is summed on the host in node order, so it
    // does not depend on a device reduction order.
    std::vector<double> gtmp;
    double *gdst = out->gauss;
    if (want_gauss && !gdst) {
        gtmp.resize((size_t)(N + 1));
        gdst = gtmp.data();
    }
    if (gdst) HIP_OK(hipMemcpyAsync(gdst, w.gauss, (size_t)(N + 1) * 8, hipMemcpyDeviceToHost, h->stream));
    std::vector<long long> cnt(nb), hi(nb), mn(nb), mx(nb);
    std::vector<unsigned long long> lo(nb);
    if (nb > 0) {
        HIP_OK(hipMemcpyAsync(cnt.data(), w.pcount, (size_t)nb * 8, hipMemcpyDeviceToHost, h->stream));
        HIP_OK(hipMemcpyAsync(lo.data(), w.plo, (size_t)nb * 8, hipMemcpyDeviceToHost, h->stream));
        HIP_OK(hipMemcpyAsync(hi.data(), w.phi128, (size_t)nb * 8, hipMemcpyDeviceToHost, h->stream));
        HIP_OK(hipMemcpyAsync(mn.data(), w.pmin, (size_t)nb * 8, hipMemcpyDeviceToHost, h->stream));
        HIP_OK(hipMemcpyAsync(mx.data(), w.pmax, (size_t)nb * 8, hipMemcpyDeviceToHost, h->stream));
    }
    HIP_OK(hipStreamSynchronize(h->stream));
    out->step = ctr.step;
    out->n_slots = ctr.n_slots + ctr.n_slots_hi;
    out->n_alive = ctr.n_slots + ctr.n_slots_hi - ctr.n_removed;
    out->n_slots_high = ctr.n_slots_hi;
    out->n_injected = ctr.n_injected;
    out->n_exit = ctr.n_exit;
    out->n_absorb = ctr.n_absorb;
    out->last_n_inj = ctr.last_ninj;
    out->w0 = ctr.w0_last;
    out->status = (int64_t)ctr.status;
    out->e_surf = ctr.e_surf;
    out->exit_sum_lo = ctr.exit_lo;
    out->exit_sum_hi = ctr.exit_hi;
    out->exit_gamma_sum = ldexp(i128_to_double(ctr.exit_lo, ctr.exit_hi), -32);
    const double rmax = __builtin_bit_cast(double, ctr.rho_max_bits);
    const double gmax = __builtin_bit_cast(double, ctr.gauss_max_bits);
    out->gauss_max = (want_gauss || out->gauss) ? gmax / (h->c.fourpi * rmax) : 0.0;
    if (want_gauss && req->gauss_tol > 0.0 && out->gauss_max > req->gauss_tol && !(ctr.status & PIC_ST_GAUSS)) {
        // latch the bit in the device status word (the stream is idle here)
        ctr.status |= PIC_ST_GAUSS;
        HIP_OK(hipMemcpyAsync(&w.ctr->status, &ctr.status, sizeof ctr.status, hipMemcpyHostToDevice, h->stream));
        HIP_OK(hipStreamSynchronize(h->stream));
        out->status = (int64_t)ctr.status;
    }
    out->gauss_l2 = 0.0;
    if (gdst && N > 1) {
        double ss = 0.0;
        for (int64_t i = 1; i < N; ++i) ss += gdst[i] * gdst[i];
        out->gauss_l2 = sqrt(ss / (double)(N - 1)) / (h->c.fourpi * rmax);
    }
    for (int k = 0; k < nb; ++k) {
        if (out->prof_count) out->prof_count[k] = cnt[k];
        if (out->prof_sum_lo) out->prof_sum_lo[k] = lo[k];
        if (out->prof_sum_hi) out->prof_sum_hi[k] = hi[k];
        if (out->prof_mean)
            out->prof_mean[k] = cnt[k] ? ldexp(i128_to_double(lo[k], hi[k]), -32) / (double)cnt[k] : 0.0;
        if (out->prof_min) out->prof_min[k] = from_ordered_bits(mn[k]);
        if (out->prof_max) out->prof_max[k] = from_ordered_bits(mx[k]);
    }
    if (ctr.status) return fail(PIC_EDEVSTATUS, "device status bits 0x%llx", (unsigned long long)ctr.status);
    return PIC_OK;
}

pic_status pic_profile_noalloc(pic_handle *h, int32_t n_bins, int64_t *d_count, uint64_t *d_sum_lo,
                               int64_t *d_sum_hi, double *d_min, double *d_max)
{
    if (!h) return fail(PIC_EINVAL, "handle is NULL");
    if (h->is_batch) return fail(PIC_EINVAL, "the profile is per tube (pic_batch_tube)");
    if (n_bins < 1 || n_bins > NOALLOC_MAX_BINS)
        return fail(PIC_EINVAL, "n_bins %d not in [1, %d] (the fixed scratch holds %d bins)", n_bins,
                    NOALLOC_MAX_BINS, NOALLOC_MAX_BINS);
    if (h->poisson_pending)
        return fail(PIC_ESTATE, "the tube's t = 0 field solve is pending (call pic_diagnostics or pic_step first)");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != h->dev)
        return fail(PIC_ESTATE, "call with the tube's device (%d) current", h->dev);
    void *base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        base = g_scratch_dev[dev];
    }
    if (!base) {
        const pic_status s = scratch_of_current_device(nullptr, &base);
        if (s != PIC_OK) return s;
    }
    long long *p = (long long *)base;
    const size_t nb = (size_t)n_bins;
    const ProfPtrs bins{p, (unsigned long long *)(p + nb), p + 2 * nb, p + 3 * nb, p + 4 * nb};
    HIP_OK(launch_profile_into(h, n_bins, bins, false));
    HIP_OK(launch_profile_finish(h, n_bins, bins, d_count, d_sum_lo, d_sum_hi, d_min, d_max));
    return PIC_OK;
}

pic_status pic_read_particles(pic_handle *h, double *x, double *u, int64_t cap, int64_t *n_out)
{
    if (!h || !n_out) return fail(PIC_EINVAL, "handle or n_out is NULL");
    if (h->is_batch) return fail(PIC_EINVAL, "particles are per tube (pic_batch_tube)");
    if (pic_status sp = resolve_pending(h)) return sp;
    DevCounters ctr;
    pic_status s = read_counters(h, &ctr);
    if (s != PIC_OK) return s;
    if (h->p.precision == PIC_FP32_BULK) {
        const int b = h->pbuf;
        int64_t m = 0;
        for (int st = 0; st < 2; ++st) {
            const int64_t ns = st ? ctr.n_slots_hi : ctr.n_slots;
            std::vector<int> hc((size_t)ns);
            std::vector<float> ho((size_t)ns), hul((size_t)ns);
            std::vector<double> huh((size_t)ns);
            if (st) {
                if (pic_status e = read_high_stream(h, b, ns, hc, ho, huh)) return e;
            } else if (ns > 0) {
                HIP_OK(hipMemcpyAsync(hc.data(), h->ws.cl[b], (size_t)ns * 4, hipMemcpyDeviceToHost, h->stream));
                HIP_OK(hipMemcpyAsync(ho.data(), h->ws.ol[b], (size_t)ns * 4, hipMemcpyDeviceToHost, h->stream));
                HIP_OK(hipMemcpyAsync(hul.data(), h->ws.ul[b], (size_t)ns * 4, hipMemcpyDeviceToHost, h->stream));
                HIP_OK(hipStreamSynchronize(h->stream));
            }
            for (int64_t i = 0; i < ns; ++i) {
                if (hc[(size_t)i] < 0) continue;   // removed slot
                if (m < cap) {
                    if (x) x[m] = (double)hc[(size_t)i] + (double)ho[(size_t)i];
                    if (u) u[m] = st ? huh[(size_t)i] : (double)hul[(size_t)i];
                }
                ++m;
            }
        }
        *n_out = m;
        if (m > cap) return fail(PIC_ECAPACITY, "%lld live particles, room for %lld", (long long)m, (long long)cap);
        return PIC_OK;
    }
    const int64_t ns = ctr.n_slots;
    std::vector<double> hx((size_t)ns), hu((size_t)ns);
    if (ns > 0) {
        HIP_OK(hipMemcpyAsync(hx.data(), h->ws.x[h->pbuf], (size_t)ns * 8, hipMemcpyDeviceToHost, h->stream));
        HIP_OK(hipMemcpyAsync(hu.data(), h->ws.u[h->pbuf], (size_t)ns * 8, hipMemcpyDeviceToHost, h->stream));
        HIP_OK(hipStreamSynchronize(h->stream));
    }
    int64_t m = 0;
    for (int64_t i = 0; i < ns; ++i) {
        if (!(hx[i] >= 0.0)) continue;   // removed slot
        if (m < cap) {
            if (x) x[m] = hx[i];
            if (u) u[m] = hu[i];
        }
        ++m;
    }
    *n_out = m;
    if (m > cap) return fail(PIC_ECAPACITY, "%lld live particles, room for %lld", (long long)m, (long long)cap);
    return PIC_OK;
}

pic_status pic_write_fields(pic_handle *h, const double *ez, const double *er, const double *b_phi)
{
    if (!h) return fail(PIC_EINVAL, "handle is NULL");
    if (h->is_batch) return fail(PIC_EINVAL, "fields are per tube (pic_batch_tube)");
    if (pic_status sp = resolve_pending(h)) return sp;
    const int64_t N = h->c.N;
    const int f = h->fbuf;
    h->mut += 1;
    if (ez) HIP_OK(hipMemcpyAsync(h->ws.ez[f], ez, (size_t)N * 8, hipMemcpyHostToDevice, h->stream));
    if (er) HIP_OK(hipMemcpyAsync(h->ws.er[f], er, (size_t)(N + 1) * 8, hipMemcpyHostToDevice, h->stream));
    if (b_phi) HIP_OK(hipMemcpyAsync(h->ws.b[f], b_phi, (size_t)N * 8, hipMemcpyHostToDevice, h->stream));
    HIP_OK(launch_kick(h));
    HIP_OK(hipStreamSynchronize(h->stream));
    return PIC_OK;
}

pic_status pic_set_injection_schedule(pic_handle *h, const int64_t *d_counts, int64_t first_step, int64_t n)
{
    if (!h) return fail(PIC_EINVAL, "handle is NULL");
    if (h->is_batch || h->parent) return fail(PIC_ESTATE, "injection schedules are for single tubes");
    if (n < 0 || first_step < 0 || (n > 0 && !d_counts)) return fail(PIC_EINVAL, "bad schedule arguments");
    h->mut += 1;
    h->d_sched = n > 0 ? d_counts : nullptr;
    h->sched_first = first_step;
    h->sched_n = n;
    free_tube_graphs(h);
    return PIC_OK;
}

// ---- save / load --------------------------------------------------------
//
// Blob: header, knot values, device counters, E_z, E_r, B_phi, last-step J,
// then the occupied slots of the current particle buffer(s).  Sections are
// 8-byte aligned.  Loading writes into the target's current buffers, so the
// blob does not depend on buffer parities.

}  // extern "C"

namespace {

constexpr char SAVE_MAGIC[8] = {'P', 'C', 'P', 'I', 'C', 'S', 'V', '2'};

struct SaveHead {
    char magic[8];
    int32_t abi, precision;
    int64_t n_cells, n_knots, n_lo, n_hi, step, total_bytes;
    int32_t rho_kind, fp_bits;
    double length, radius, dt_over_dz, q_over_m, ppc, rho_amp, kappa, r_star, gamma_fp64, macro_charge;
    double incl, theta_star, cos_phi, rg_over_rstar;
};

size_t pad8(size_t b) { return (b + 7) & ~(size_t)7; }

struct SaveLayout {
    size_t knots, ctr, ez, er, b, j, p[6], total;
};

SaveLayout save_layout(int64_t N, int64_t nk, int64_t nlo, int64_t nhi, bool f32)
{
    SaveLayout L{};
    size_t off = pad8(sizeof(SaveHead));
    auto take = [&](size_t bytes) { const size_t o = off; off = pad8(off + bytes); return o; };
    L.knots = take((size_t)nk * 8);
    L.ctr = take(sizeof(DevCounters));
    L.ez = take((size_t)N * 8);
    L.er = take((size_t)(N + 1) * 8);
    L.b = take((size_t)N * 8);
    L.j = take((size_t)N * 8);
    if (!f32) {
        L.p[0] = take((size_t)nlo * 8);   // x
        L.p[1] = take((size_t)nlo * 8);   // u
    } else {
        L.p[0] = take((size_t)nlo * 4);   // low: cell, offset, u f32
        L.p[1] = take((size_t)nlo * 4);
        L.p[2] = take((size_t)nlo * 4);
        L.p[3] = take((size_t)nhi * 4);   // high: cell, offset, u f64
        L.p[4] = take((size_t)nhi * 4);
        L.p[5] = take((size_t)nhi * 8);
    }
    L.total = off;
    return L;
}

void fill_head(const pic_handle *h, SaveHead *hd)
{
    memset(hd, 0, sizeof *hd);
    memcpy(hd->magic, SAVE_MAGIC, 8);
    const pic_params &p = h->p;
    hd->abi = PCPIC_ABI_VERSION;
    hd->precision = p.precision;
    hd->n_cells = p.n_cells;
    hd->n_knots = (int64_t)h->knots.size();
    hd->rho_kind = p.rho_kind;
    hd->fp_bits = p.fp_bits;
    hd->length = p.length;
    hd->radius = p.radius;
    hd->dt_over_dz = p.dt_over_dz;
    hd->q_over_m = p.q_over_m;
    hd->ppc = p.ppc;
    hd->rho_amp = p.rho_amp;
    hd->kappa = p.kappa;
    hd->r_star = p.r_star;
    hd->gamma_fp64 = p.gamma_fp64;
    hd->macro_charge = p.macro_charge;
    hd->incl = p.incl;
    hd->theta_star = p.theta_star;
    hd->cos_phi = p.cos_phi;
    hd->rg_over_rstar = p.rg_over_rstar;
}

}  // namespace

extern "C" {

pic_status pic_save(pic_handle *h, void *buf, size_t cap, size_t *bytes)
{
    if (!h || !bytes) return fail(PIC_EINVAL, "handle or bytes is NULL");
    if (h->is_batch) return fail(PIC_EINVAL, "save the tubes of a batch one by one (pic_batch_tube)");
    if (pic_status sp = resolve_pending(h)) return sp;
    DevCounters ctr;
    pic_status s = read_counters(h, &ctr);
    if (s != PIC_OK) return s;
    const bool f32 = h->p.precision == PIC_FP32_BULK;
    const int64_t N = h->c.N, nlo = ctr.n_slots, nhi = f32 ? ctr.n_slots_hi : 0;
    const SaveLayout L = save_layout(N, (int64_t)h->knots.size(), nlo, nhi, f32);
    *bytes = L.total;
    if (!buf) return PIC_OK;
    if (cap < L.total) return fail(PIC_EINVAL, "buffer of %zu bytes, %zu needed", cap, L.total);
    uint8_t *o = (uint8_t *)buf;
    SaveHead hd;
    fill_head(h, &hd);
    hd.n_lo = nlo;
    hd.n_hi = nhi;
    hd.step = h->step;
    hd.total_bytes = (int64_t)L.total;
    memcpy(o, &hd, sizeof hd);
    if (!h->knots.empty()) memcpy(o + L.knots, h->knots.data(), h->knots.size() * 8);
    memcpy(o + L.ctr, &ctr, sizeof ctr);
    const Workspace &w = h->ws;
    const int f = h->fbuf, b = h->pbuf;
    auto d2h = [&](size_t at, const void *src, size_t n) {
        return n ? hipMemcpyAsync(o + at, src, n, hipMemcpyDeviceToHost, h->stream) : hipSuccess;
    };
    HIP_OK(d2h(L.ez, w.ez[f], (size_t)N * 8));
    HIP_OK(d2h(L.er, w.er[f], (size_t)(N + 1) * 8));
    HIP_OK(d2h(L.b, w.b[f], (size_t)N * 8));
    HIP_OK(d2h(L.j, w.j[1 - h->jbuf], (size_t)N * 8));
    if (!f32) {
        HIP_OK(d2h(L.p[0], w.x[b], (size_t)nlo * 8));
        HIP_OK(d2h(L.p[1], w.u[b], (size_t)nlo * 8));
    } else {
        HIP_OK(d2h(L.p[0], w.cl[b], (size_t)nlo * 4));
        HIP_OK(d2h(L.p[1], w.ol[b], (size_t)nlo * 4));
        HIP_OK(d2h(L.p[2], w.ul[b], (size_t)nlo * 4));
        HIP_OK(hipStreamSynchronize(h->stream));
        // the high stream as (cell, offset, u), as the low stream is kept
        std::vector<int> hc;
        std::vector<float> ho;
        std::vector<double> hu;
        if (pic_status e = read_high_stream(h, b, nhi, hc, ho, hu)) return e;
        if (nhi > 0) {
            memcpy(o + L.p[3], hc.data(), (size_t)nhi * 4);
            memcpy(o + L.p[4], ho.data(), (size_t)nhi * 4);
            memcpy(o + L.p[5], hu.data(), (size_t)nhi * 8);
        }
    }
    HIP_OK(hipStreamSynchronize(h->stream));
    return PIC_OK;
}

pic_status pic_load(pic_handle *h, const void *buf, size_t bytes)
{
    if (!h || !buf) return fail(PIC_EINVAL, "handle or buffer is NULL");
    if (h->is_batch || h->parent) return fail(PIC_ESTATE, "load into a single tube (not a batch or its tubes)");
    if (bytes < sizeof(SaveHead)) return fail(PIC_EINVAL, "buffer too small for a saved state");
    SaveHead hd, mine;
    memcpy(&hd, buf, sizeof hd);
    fill_head(h, &mine);
    if (memcmp(hd.magic, SAVE_MAGIC, 8) != 0) return fail(PIC_EINVAL, "not a saved tube state");
    if (hd.abi != mine.abi) return fail(PIC_EABI, "saved with ABI version %d", hd.abi);
    const bool same = hd.precision == mine.precision && hd.n_cells == mine.n_cells && hd.n_knots == mine.n_knots &&
                      hd.rho_kind == mine.rho_kind && hd.fp_bits == mine.fp_bits && hd.length == mine.length &&
                      hd.radius == mine.radius && hd.dt_over_dz == mine.dt_over_dz && hd.q_over_m == mine.q_over_m &&
                      hd.ppc == mine.ppc && hd.rho_amp == mine.rho_amp && hd.kappa == mine.kappa &&
                      hd.r_star == mine.r_star && hd.gamma_fp64 == mine.gamma_fp64 &&
                      hd.macro_charge == mine.macro_charge && hd.incl == mine.incl &&
                      hd.theta_star == mine.theta_star && hd.cos_phi == mine.cos_phi &&
                      hd.rg_over_rstar == mine.rg_over_rstar;
    if (!same) return fail(PIC_EINVAL, "the saved tube has different parameters");
    const bool f32 = h->p.precision == PIC_FP32_BULK;
    const int64_t N = h->c.N;
    if (hd.n_lo < 0 || hd.n_hi < 0 || hd.n_lo + hd.n_hi > h->c.cap || (!f32 && hd.n_hi != 0))
        return fail(PIC_ECAPACITY, "saved state holds %lld + %lld slots, capacity %lld", (long long)hd.n_lo,
                    (long long)hd.n_hi, (long long)h->c.cap);
    const SaveLayout L = save_layout(N, hd.n_knots, hd.n_lo, hd.n_hi, f32);
    if ((int64_t)L.total != hd.total_bytes || bytes < L.total) return fail(PIC_EINVAL, "truncated saved state");
    const uint8_t *in = (const uint8_t *)buf;
    if (hd.n_knots > 0 && memcmp(in + L.knots, h->knots.data(), (size_t)hd.n_knots * 8) != 0)
        return fail(PIC_EINVAL, "the saved tube has different knot values");
    DevCounters ctr;
    memcpy(&ctr, in + L.ctr, sizeof ctr);
    if (ctr.n_slots != hd.n_lo || (f32 && ctr.n_slots_hi != hd.n_hi))
        return fail(PIC_EINVAL, "inconsistent saved state");
    const Workspace &w = h->ws;
    const int f = h->fbuf, b = h->pbuf;
    h->mut += 1;
    auto h2d = [&](void *dst, size_t at, size_t n) {
        return n ? hipMemcpyAsync(dst, in + at, n, hipMemcpyHostToDevice, h->stream) : hipSuccess;
    };
    HIP_OK(h2d(w.ez[f], L.ez, (size_t)N * 8));
    HIP_OK(h2d(w.er[f], L.er, (size_t)(N + 1) * 8));
    HIP_OK(h2d(w.b[f], L.b, (size_t)N * 8));
    HIP_OK(h2d(w.j[1 - h->jbuf], L.j, (size_t)N * 8));
    HIP_OK(launch_zero_i64(h, w.j[h->jbuf], N));        // the next step deposits into a cleared J
    if (!f32) {
        HIP_OK(h2d(w.x[b], L.p[0], (size_t)hd.n_lo * 8));
        HIP_OK(h2d(w.u[b], L.p[1], (size_t)hd.n_lo * 8));
    } else {
        HIP_OK(h2d(w.cl[b], L.p[0], (size_t)hd.n_lo * 4));
        HIP_OK(h2d(w.ol[b], L.p[1], (size_t)hd.n_lo * 4));
        HIP_OK(h2d(w.ul[b], L.p[2], (size_t)hd.n_lo * 4));
        if (hd.n_hi > 0) {
            std::vector<int> hc((size_t)hd.n_hi);
            std::vector<float> ho((size_t)hd.n_hi);
            std::vector<double> hu((size_t)hd.n_hi);
            memcpy(hc.data(), in + L.p[3], (size_t)hd.n_hi * 4);
            memcpy(ho.data(), in + L.p[4], (size_t)hd.n_hi * 4);
            memcpy(hu.data(), in + L.p[5], (size_t)hd.n_hi * 8);
            if (pic_status e = write_high_stream(h, b, hd.n_hi, hc.data(), ho.data(), hu.data())) return e;
        }
    }
    HIP_OK(hipMemcpyAsync(w.ctr, &ctr, sizeof ctr, hipMemcpyHostToDevice, h->stream));
    HIP_OK(launch_kick(h));
    HIP_OK(hipStreamSynchronize(h->stream));
    h->step = hd.step;
    return PIC_OK;
}

pic_status pic_stream_copy(const void *d_src, void *d_dst, size_t bytes, void *hip_stream)
{
    const uintptr_t s = (uintptr_t)d_src, d = (uintptr_t)d_dst;
    if (!d_src || !d_dst) return fail(PIC_EINVAL, "null pointer");
    if (s % 16 || d % 16 || bytes % 16) return fail(PIC_EINVAL, "pointers and size must be multiples of 16 bytes");
    if (bytes >= ((size_t)1 << 40)) return fail(PIC_EINVAL, "copy of %zu bytes is too large", bytes);
    if (s < d + bytes && d < s + bytes) return fail(PIC_EINVAL, "source and destination overlap");
    if (bytes == 0) return PIC_OK;
    HIP_OK(launch_stream_copy(d_src, d_dst, (int64_t)(bytes / 16), (hipStream_t)hip_stream));
    return PIC_OK;
}

pic_status pic_destroy(pic_handle *h)
{
    if (!h) return fail(PIC_EINVAL, "handle is NULL");
    if (h->parent) return fail(PIC_ESTATE, "a tube of a batch is released with its batch");
    (void)hipStreamSynchronize(h->stream);
    if (h->is_batch) {
        free_batch_graphs(h);
        for (pic_handle *t : h->tubes) delete t;
    } else {
        free_tube_graphs(h);
    }
    delete h;
    return PIC_OK;
}

// ------------------------------------------------------------------------
// batches of tubes (ensembles)
// ------------------------------------------------------------------------

// Entries of the work-item -> tube maps, sized for the smallest tiles any
// launch shape uses (64 cells per field tile).
struct BatchMapSizes {
    int64_t push;   // push items at the smallest tile (64 threads x 2 slots), the work list's bound
    int64_t field, chunk, scan;
};

static BatchMapSizes batch_map_sizes(const pic_params *tubes, int n)
{
    BatchMapSizes m{0, 0, 0, 0};
    for (int t = 0; t < n; ++t) {
        const pic_params &p = tubes[t];
        const bool f32 = p.precision == PIC_FP32_BULK;
        m.push += (p.capacity + 127) / 128 + 2;
        m.field += (p.n_cells + 63) / 64;
        m.chunk += (p.capacity + SORT_TILE - 1) / SORT_TILE + (f32 ? 1 : 0);
        const int64_t keys = (f32 ? 2 * (p.n_cells + 1) : p.n_cells) << sort_sub_log2(p);
        m.scan += (keys + SORT_SCAN_TILE - 1) / SORT_SCAN_TILE;
    }
    return m;
}

static size_t batch_header_bytes(const pic_params *tubes, int n)
{
    const BatchMapSizes m = batch_map_sizes(tubes, n);
    size_t off = 0;
    off = align_up(off) + sizeof(TubeDev) * (size_t)n;
    for (int k = 0; k < 5; ++k) off = align_up(off) + sizeof(int64_t) * (size_t)(n + 1);
    off = align_up(off) + sizeof(int64_t) * 2 * (size_t)n;   // per-tube slot counts of the work list
    off = align_up(off) + 4 * (size_t)m.field;
    off = align_up(off) + 4 * (size_t)m.push;
    off = align_up(off) + 4 * (size_t)m.chunk;
    off = align_up(off) + 4 * (size_t)m.scan;
    off = align_up(off) + 4 * (size_t)n;   // tubes to solve together
    return align_up(off);
}

size_t pic_batch_workspace_bytes(const pic_params *tubes, int32_t n_tubes)
{
    if (!tubes || n_tubes < 1) {
        fail(PIC_EINVAL, "need at least one tube");
        return 0;
    }
    for (int t = 0; t < n_tubes; ++t)
        if (validate(&tubes[t]) != PIC_OK) return 0;
    size_t total = batch_header_bytes(tubes, n_tubes);
    for (int t = 0; t < n_tubes; ++t) total += carve(tubes[t], nullptr).bytes;
    return total;
}

static void free_batch_graphs(pic_handle *h)
{
    for (auto &g : h->graph) {
        if (g) (void)hipGraphExecDestroy(g);
        g = nullptr;
    }
}

// Push/field work-item tables for the current launch shape, uploaded to the device.
static pic_status batch_configure(pic_handle *h, int block, int per_thread)
{
    const bool f32 = h->tubes[0]->p.precision == PIC_FP32_BULK;
    const int ppt = f32 ? 4 : per_thread;
    const int saved_b = h->batch_block, saved_p = h->batch_ppt;
    h->batch_block = block;
    h->batch_ppt = ppt;
    if (!batch_shape_supported(h)) {
        h->batch_block = saved_b;
        h->batch_ppt = saved_p;
        return fail(PIC_EINVAL, "unsupported batch launch shape (%d threads, %d per thread)", block, per_thread);
    }
    const int n = (int)h->tubes.size();
    // slots per push item: FP32-bulk items are tiles of the high stream's size
    // (the low stream's are larger), push_item_f32
    const int64_t tile = (int64_t)block * (f32 ? F32_PPT_HI : ppt);
    std::vector<TubeDev> td((size_t)n);
    std::vector<int64_t> pp((size_t)n + 1, 0), fp((size_t)n + 1, 0), sp((size_t)n + 1, 0), kp((size_t)n + 1, 0);
    std::vector<int64_t> cp((size_t)n + 1, 0);
    for (int t = 0; t < n; ++t) {
        pic_handle *s = h->tubes[(size_t)t];
        td[(size_t)t] = tube_dev(s);
        td[(size_t)t].push_tiles = (s->c.cap + tile - 1) / tile;
        td[(size_t)t].push_tiles_hi = f32 ? 1 : 0;
        pp[(size_t)t + 1] = pp[(size_t)t] + td[(size_t)t].push_tiles + td[(size_t)t].push_tiles_hi;
        fp[(size_t)t + 1] = fp[(size_t)t] + (s->c.N + block * FIELD_CPT - 1) / (block * FIELD_CPT);
        sp[(size_t)t + 1] = sp[(size_t)t] + td[(size_t)t].sort_chunks + (f32 ? 1 : 0);   // sort_item
        kp[(size_t)t + 1] = kp[(size_t)t] + td[(size_t)t].n_keys;
        cp[(size_t)t + 1] = cp[(size_t)t] + (td[(size_t)t].n_keys + SORT_SCAN_TILE - 1) / SORT_SCAN_TILE;
    }
    h->batch_push_items = pp[(size_t)n];
    h->batch_field_items = fp[(size_t)n];
    h->batch_sort_items = sp[(size_t)n];
    h->batch_keys = kp[(size_t)n];
    h->batch_scan_blocks = cp[(size_t)n];
    HIP_OK(hipMemcpyAsync(h->d_tubes, td.data(), sizeof(TubeDev) * (size_t)n, hipMemcpyHostToDevice, h->stream));
    HIP_OK(hipMemcpyAsync(h->d_field_pref, fp.data(), 8 * fp.size(), hipMemcpyHostToDevice, h->stream));
    HIP_OK(hipMemcpyAsync(h->d_sort_pref, sp.data(), 8 * sp.size(), hipMemcpyHostToDevice, h->stream));
    HIP_OK(hipMemcpyAsync(h->d_key_pref, kp.data(), 8 * kp.size(), hipMemcpyHostToDevice, h->stream));
    HIP_OK(hipMemcpyAsync(h->d_scan_pref, cp.data(), 8 * cp.size(), hipMemcpyHostToDevice, h->stream));
    // work item -> tube maps (one entry per block of the batched kernels)
    std::vector<int32_t> fm((size_t)fp[(size_t)n]), sm((size_t)sp[(size_t)n]), cm((size_t)cp[(size_t)n]);
    for (int t = 0; t < n; ++t) {
        for (int64_t i = fp[(size_t)t]; i < fp[(size_t)t + 1]; ++i) fm[(size_t)i] = t;
        for (int64_t i = sp[(size_t)t]; i < sp[(size_t)t + 1]; ++i) sm[(size_t)i] = t;
        for (int64_t i = cp[(size_t)t]; i < cp[(size_t)t + 1]; ++i) cm[(size_t)i] = t;
    }
    HIP_OK(hipMemcpyAsync(h->d_field_map, fm.data(), 4 * fm.size(), hipMemcpyHostToDevice, h->stream));
    HIP_OK(hipMemcpyAsync(h->d_chunk_map, sm.data(), 4 * sm.size(), hipMemcpyHostToDevice, h->stream));
    HIP_OK(hipMemcpyAsync(h->d_scan_map, cm.data(), 4 * cm.size(), hipMemcpyHostToDevice, h->stream));
    HIP_OK(hipStreamSynchronize(h->stream));
    free_batch_graphs(h);
    return PIC_OK;
}

pic_status pic_init_batch(const pic_params *tubes, int32_t n_tubes, void *d_workspace, size_t ws_bytes,
                          void *hip_stream, pic_handle **out)
{
    if (!out) return fail(PIC_EINVAL, "out is NULL");
    *out = nullptr;
    const size_t need = pic_batch_workspace_bytes(tubes, n_tubes);
    if (need == 0) return PIC_EINVAL;
    for (int t = 1; t < n_tubes; ++t)
        if (tubes[t].precision != tubes[0].precision || tubes[t].sort_every != tubes[0].sort_every)
            return fail(PIC_EINVAL, "all tubes of a batch need the same precision and sort_every");
    for (int t = 0; t < n_tubes; ++t)
        if (tubes[t].flags & PIC_GR_ALPHA) return fail(PIC_EINVAL, "PIC_GR_ALPHA runs on single tubes only");
    if (!d_workspace || ws_bytes < need) return fail(PIC_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    if (((uintptr_t)d_workspace) % ALIGN) return fail(PIC_EWORKSPACE, "workspace must be %zu-byte aligned", ALIGN);
    pic_handle *h = new (std::nothrow) pic_handle();
    if (!h) return fail(PIC_EINVAL, "out of host memory");
    h->is_batch = true;
    h->p = tubes[0];
    h->p.knots = nullptr;
    h->stream = (hipStream_t)hip_stream;
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
        h->n_cu = ncu;
    uint8_t *base = (uint8_t *)d_workspace;
    size_t off = 0;
    auto take = [&](size_t bytes) -> void * {
        const size_t o = align_up(off);
        off = o + bytes;
        return (void *)(base + o);
    };
    h->d_tubes = (TubeDev *)take(sizeof(TubeDev) * (size_t)n_tubes);
    h->d_live_pref = (int64_t *)take(8 * (size_t)(n_tubes + 1));
    h->d_field_pref = (int64_t *)take(8 * (size_t)(n_tubes + 1));
    h->d_sort_pref = (int64_t *)take(8 * (size_t)(n_tubes + 1));
    h->d_key_pref = (int64_t *)take(8 * (size_t)(n_tubes + 1));
    h->d_scan_pref = (int64_t *)take(8 * (size_t)(n_tubes + 1));
    h->d_live_counts = (int64_t *)take(16 * (size_t)n_tubes);
    {
        const BatchMapSizes m = batch_map_sizes(tubes, n_tubes);
        h->d_field_map = (int32_t *)take(4 * (size_t)m.field);
        h->d_push_map = (int32_t *)take(4 * (size_t)m.push);
        h->push_map_cap = m.push;
        h->d_chunk_map = (int32_t *)take(4 * (size_t)m.chunk);
        h->d_scan_map = (int32_t *)take(4 * (size_t)m.scan);
        h->d_pending = (int32_t *)take(4 * (size_t)n_tubes);
    }
    off = batch_header_bytes(tubes, n_tubes);
    for (int t = 0; t < n_tubes; ++t) {
        const size_t sz = carve(tubes[t], nullptr).bytes;
        pic_handle *sub = nullptr;
        pic_status s = init_tube(&tubes[t], base + off, sz, hip_stream, &sub, true);
        if (s != PIC_OK) {
            pic_destroy(h);
            return s;
        }
        sub->parent = h;
        h->tubes.push_back(sub);
        off += sz;
    }
    const bool f32 = tubes[0].precision == PIC_FP32_BULK;
    pic_status s = batch_configure(h, 256, f32 ? 4 : 2);
    if (s != PIC_OK) {
        pic_destroy(h);
        return s;
    }
    s = batch_resolve_pending(h);
    if (s != PIC_OK) {
        pic_destroy(h);
        return s;
    }
    *out = h;
    return PIC_OK;
}

pic_status pic_batch_tube(pic_handle *h, int32_t t, pic_handle **out)
{
    if (!h || !out || !h->is_batch) return fail(PIC_EINVAL, "not a batch handle");
    if (t < 0 || t >= (int32_t)h->tubes.size()) return fail(PIC_EINVAL, "tube %d out of range", t);
    *out = h->tubes[(size_t)t];
    return PIC_OK;
}

pic_status pic_batch_set_config(pic_handle *h, int32_t block, int32_t per_thread, uint32_t flags)
{
    if (!h || !h->is_batch) return fail(PIC_EINVAL, "not a batch handle");
    if (flags & ~PIC_BATCH_NO_GRAPH) return fail(PIC_EINVAL, "unknown batch flags");
    pic_status s = batch_configure(h, block, per_thread);
    if (s == PIC_OK) h->use_graph = !(flags & PIC_BATCH_NO_GRAPH);
    return s;
}

pic_status pic_batch_get_config(pic_handle *h, int32_t *block, int32_t *per_thread, int64_t *push_blocks,
                                int64_t *field_blocks)
{
    if (!h || !h->is_batch) return fail(PIC_EINVAL, "not a batch handle");
    if (block) *block = h->batch_block;
    if (per_thread) *per_thread = h->batch_ppt;
    if (push_blocks) *push_blocks = h->batch_push_items;
    if (field_blocks) *field_blocks = h->batch_field_items;
    return PIC_OK;
}

// Advance every tube of the batch by n steps in rounds that end at the sort
// period; a whole round (push and field kernels of every step, then the batched
// sort) is replayed from a captured graph.  With `ev`, events bracket each
// round's step kernels and its sort.
static pic_status batch_advance(pic_handle *h, int64_t n, std::vector<hipEvent_t> *ev, pic_timing *tim,
                                std::vector<int64_t> *round_steps)
{
    if (pic_status sp = batch_resolve_pending(h)) return sp;
    pic_handle *t0 = h->tubes[0];
    const int64_t S = t0->p.sort_every;
    while (n > 0) {
        int64_t r;
        if (S > 0) {
            r = S - (t0->step % S);
            if (r > n) r = n;
        } else {
            r = n < 64 ? n : 64;
        }
        const bool to_sort = S > 0 && (t0->step + r) % S == 0;
        const int key = t0->fbuf | (t0->jbuf << 1) | (t0->pbuf << 2);
        const bool round = to_sort && r == S && h->use_graph && !ev;
        if (round && !h->graph[key]) {
            hipGraph_t g = nullptr;
            if (hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal) == hipSuccess) {
                hipError_t e1 = launch_batch_steps(h, (int)r, true);
                hipError_t e2 = launch_batch_sort(h, true);
                hipError_t e3 = hipStreamEndCapture(h->stream, &g);
                if (e1 == hipSuccess && e2 == hipSuccess && e3 == hipSuccess && g &&
                    hipGraphInstantiate(&h->graph[key], g, nullptr, nullptr, 0) == hipSuccess) {
                    h->graph_steps = r;
                } else {
                    h->graph[key] = nullptr;
                    h->use_graph = false;
                }
                if (g) (void)hipGraphDestroy(g);
            } else {
                (void)hipGetLastError();
                h->use_graph = false;
            }
        }
        if (round && h->graph[key]) {
            HIP_OK(hipGraphLaunch(h->graph[key], h->stream));
        } else {
            // timed: four events per step (work list, push, field) and two around the sort
            hipEvent_t *e = nullptr;
            const size_t ne = ev ? (size_t)r * 4 + 2 : 0;
            if (ev) {
                ev->resize(ev->size() + ne, nullptr);
                e = &(*ev)[ev->size() - ne];
                for (size_t k = 0; k < ne; ++k) HIP_OK(hipEventCreate(&e[k]));
            }
            HIP_OK(launch_batch_steps(h, (int)r, to_sort, e));
            if (e) HIP_OK(hipEventRecord(e[ne - 2], h->stream));
            if (to_sort) HIP_OK(launch_batch_sort(h, true));
            if (e) HIP_OK(hipEventRecord(e[ne - 1], h->stream));
            if (tim) {
                tim->push_launches += r;
                tim->field_launches += r;
                if (to_sort) tim->sort_launches += 1;
            }
            if (ev) round_steps->push_back(r);
        }
        for (pic_handle *t : h->tubes) {
            t->fbuf ^= (int)(r & 1);
            t->jbuf ^= (int)(r & 1);
            t->step += r;
            if (to_sort) t->pbuf ^= 1;
        }
        n -= r;
    }
    return PIC_OK;
}

static pic_status batch_status(pic_handle *h)
{
    for (pic_handle *t : h->tubes) {
        DevCounters c;
        pic_status s = read_counters(t, &c);
        if (s != PIC_OK) return s;
        if (c.status) return fail(PIC_EDEVSTATUS, "a tube latched device status bits 0x%llx", (unsigned long long)c.status);
    }
    return PIC_OK;
}

// ------------------------------------------------------------------------
// hand-written adjoint with checkpointing
// ------------------------------------------------------------------------

}  // extern "C"

namespace {

struct Tape {
    int64_t T, K, nck, N, cap;
    std::vector<double *> ck_x, ck_u, ck_ez, ck_er, ck_b;   // checkpoint c: state at step c*K
    std::vector<DevCounters *> ck_ctr;
    int nsets;                                              // segment slot sets (2 when segments overlap)
    std::vector<double *> sg_x[2], sg_u[2], sg_ez[2], sg_er[2], sg_b[2];   // segment slots 1..K
    int64_t *nslots;                                        // [T + 1]
    double *lx, *lu, *lez, *ler[2], *lb, *lbp[2], *gphi, *cp, *dp, *g_rho, *params;
    unsigned long long *lk_lo;                              // kick adjoint, 128-bit fixed point
    long long *lk_hi;
    AdjScale *scale;
    DevCounters *final_ctr;
    int64_t *final_jlast;
    size_t bytes;
};

Tape carve_tape(pic_handle *h, int64_t T, int64_t K, uint8_t *base)
{
    Tape t{};
    t.T = T;
    t.K = K;
    t.nck = (T + K - 1) / K;
    t.N = h->c.N;
    t.cap = h->c.cap;
    size_t off = 0;
    auto take = [&](size_t bytes) -> void * {
        const size_t o = align_up(off);
        off = o + bytes;
        return base ? (void *)(base + o) : nullptr;
    };
    const size_t N = (size_t)t.N, cap = (size_t)t.cap;
    for (int64_t c = 0; c < t.nck; ++c) {
        t.ck_x.push_back((double *)take(cap * 8));
        t.ck_u.push_back((double *)take(cap * 8));
        t.ck_ez.push_back((double *)take(N * 8));
        t.ck_er.push_back((double *)take((N + 1) * 8));
        t.ck_b.push_back((double *)take(N * 8));
        t.ck_ctr.push_back((DevCounters *)take(sizeof(DevCounters)));
    }
    // two sets of segment slots when there are two segments or more: the
    // recompute of one segment fills one set while the reverse sweep of the
    // next reads the other
    t.nsets = t.nck > 1 ? 2 : 1;
    for (int q = 0; q < t.nsets; ++q) {
        t.sg_x[q].push_back(nullptr);   // slot 0 of a segment is its checkpoint
        t.sg_u[q].push_back(nullptr);
        t.sg_ez[q].push_back(nullptr);
        t.sg_er[q].push_back(nullptr);
        t.sg_b[q].push_back(nullptr);
        for (int64_t k = 1; k <= K; ++k) {
            t.sg_x[q].push_back((double *)take(cap * 8));
            t.sg_u[q].push_back((double *)take(cap * 8));
            t.sg_ez[q].push_back((double *)take(N * 8));
            t.sg_er[q].push_back((double *)take((N + 1) * 8));
            t.sg_b[q].push_back((double *)take(N * 8));
        }
    }
    t.nslots = (int64_t *)take((size_t)(T + 1) * 8);
    t.lx = (double *)take(cap * 8);
    t.lu = (double *)take(cap * 8);
    t.lez = (double *)take(N * 8);
    for (int k = 0; k < 2; ++k) {
        t.ler[k] = (double *)take((N + 1) * 8);
        t.lbp[k] = (double *)take(N * 8);
    }
    t.lb = (double *)take(N * 8);
    t.lk_lo = (unsigned long long *)take(N * 8);
    t.lk_hi = (long long *)take(N * 8);
    t.scale = (AdjScale *)take(sizeof(AdjScale));
    t.gphi = (double *)take((N + 1) * 8);
    t.cp = (double *)take((N + 1) * 8);
    t.dp = (double *)take((N + 1) * 8);
    t.g_rho = (double *)take((N + 1) * 8);
    t.params = (double *)take((size_t)(h->c.n_knots + 2) * 8);
    t.final_ctr = (DevCounters *)take(sizeof(DevCounters));
    t.final_jlast = (int64_t *)take(N * 8);
    t.bytes = align_up(off);
    return t;
}

pic_status adjoint_supported(pic_handle *h)
{
    if (!h) return fail(PIC_EINVAL, "handle is NULL");
    if (h->is_batch || h->parent) return fail(PIC_EINVAL, "the adjoint runs on a single tube");
    if (h->p.precision != PIC_FP64) return fail(PIC_EINVAL, "the adjoint needs PIC_FP64");
    if (h->p.sort_every != 0) return fail(PIC_EINVAL, "the adjoint needs sort_every = 0");
    if (h->p.flags & PIC_FREEZE_FIELDS) return fail(PIC_EINVAL, "the adjoint needs evolving fields");
    if (h->p.flags & PIC_GR_ALPHA) return fail(PIC_EINVAL, "the adjoint covers the flat step (not PIC_GR_ALPHA)");
    if (h->c.cap > ((int64_t)1 << 31))
        return fail(PIC_EINVAL, "the adjoint takes at most 2^31 particle slots (its fixed-point sums)");
    return PIC_OK;
}

// The checkpointed forward of n_steps steps (the same steps as pic_step),
// recorded in the tape and in h->adj for the reverse sweep.
pic_status adjoint_forward(pic_handle *h, int64_t T, int64_t K, void *d_tape, size_t tape_bytes, pic_adjoint_out *out)
{
    Tape t = carve_tape(h, T, K, (uint8_t *)d_tape);
    Workspace &w = h->ws;
    const int64_t N = h->c.N;
    h->adj.valid = false;
    hipEvent_t ev[2] = {};
    for (auto &e : ev) HIP_OK(hipEventCreate(&e));
    auto done = [&](pic_status r) {
        for (auto &e : ev) (void)hipEventDestroy(e);
        return r;
    };
#define FWD_OK(expr)                                                                                  \
    do {                                                                                              \
        const hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess) return done(fail(PIC_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_))); \
    } while (0)
    DevCounters c0;
    pic_status s = read_counters(h, &c0);
    if (s != PIC_OK) return done(s);
    FWD_OK(hipEventRecord(ev[0], h->stream));
    for (int64_t st = 0; st < T; ++st) {
        if (st % K == 0) {
            const int64_t ck = st / K;
            const int f = h->fbuf;
            FWD_OK(launch_copy_slots(h, w.x[h->pbuf], w.u[h->pbuf], t.ck_x[ck], t.ck_u[ck]));
            FWD_OK(hipMemcpyAsync(t.ck_ez[ck], w.ez[f], (size_t)N * 8, hipMemcpyDeviceToDevice, h->stream));
            FWD_OK(hipMemcpyAsync(t.ck_er[ck], w.er[f], (size_t)(N + 1) * 8, hipMemcpyDeviceToDevice, h->stream));
            FWD_OK(hipMemcpyAsync(t.ck_b[ck], w.b[f], (size_t)N * 8, hipMemcpyDeviceToDevice, h->stream));
            FWD_OK(hipMemcpyAsync(t.ck_ctr[ck], w.ctr, sizeof(DevCounters), hipMemcpyDeviceToDevice, h->stream));
        }
        FWD_OK(launch_record_slots(h, t.nslots + st));
        FWD_OK(launch_push_f64(h));
        FWD_OK(launch_field_inject(h));
        h->fbuf ^= 1;
        h->jbuf ^= 1;
        h->step += 1;
    }
    FWD_OK(launch_record_slots(h, t.nslots + T));
    // keep what the recompute overwrites: counters and the last step's current
    FWD_OK(hipMemcpyAsync(t.final_ctr, w.ctr, sizeof(DevCounters), hipMemcpyDeviceToDevice, h->stream));
    FWD_OK(hipMemcpyAsync(t.final_jlast, w.j[1 - h->jbuf], (size_t)N * 8, hipMemcpyDeviceToDevice, h->stream));
    FWD_OK(hipEventRecord(ev[1], h->stream));
    DevCounters c1;
    s = read_counters(h, &c1);
    if (s != PIC_OK) return done(s);
#undef FWD_OK
    const int64_t nex = c1.n_exit - c0.n_exit;
    const __int128 e0 = ((__int128)c0.exit_hi << 64) | (__int128)c0.exit_lo;
    const __int128 e1 = ((__int128)c1.exit_hi << 64) | (__int128)c1.exit_lo;
    out->loss = nex > 0 ? ldexp((double)(e1 - e0), -32) / (double)nex : 0.0;
    out->n_exit = nex;
    float fms = 0;
    (void)hipEventElapsedTime(&fms, ev[0], ev[1]);
    out->forward_ms = fms;
    AdjRecord &r = h->adj;
    r.valid = true;
    r.tape = d_tape;
    r.tape_bytes = tape_bytes;
    r.T = T;
    r.K = K;
    r.n_pre = c0.n_slots;
    r.n_exit = nex;
    r.loss = out->loss;
    r.step_end = h->step;
    r.mut = h->mut;
    r.jb_final = h->jbuf;
    r.forward_ms = fms;
    return done(PIC_OK);
}

// The reverse sweep of the recorded forward: each segment recomputed from its
// checkpoint (on a second stream, one segment ahead), three kernels per
// reversed step, the transposed Poisson solve; gradients scaled by dloss.
pic_status adjoint_backward(pic_handle *h, double dloss, pic_adjoint_out *out)
{
    const AdjRecord &r = h->adj;
    Tape t = carve_tape(h, r.T, r.K, (uint8_t *)r.tape);
    Workspace &w = h->ws;
    const int64_t N = h->c.N, T = r.T, K = r.K, n_pre = r.n_pre, nex = r.n_exit;
    hipEvent_t ev[2] = {};
    for (auto &e : ev) HIP_OK(hipEventCreate(&e));
    auto done = [&](pic_status rc) {
        for (auto &e : ev) (void)hipEventDestroy(e);
        return rc;
    };
#define ADJ_OK(expr)                                                                                  \
    do {                                                                                              \
        const hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess) return done(fail(PIC_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_))); \
    } while (0)
    // The recompute of segment ck-1 runs on a second stream, into the other set
    // of segment slots, while the reverse sweep of segment ck runs on the
    // tube's stream: the two touch disjoint memory (the recompute owns the
    // counters and the current; the sweep reads recorded slots, fields and slot
    // counts and owns the adjoint arrays), and events order each recompute
    // before its sweep and each set's reuse after its sweep.
    ADJ_OK(hipEventRecord(ev[0], h->stream));
    ADJ_OK(launch_zero_f64(h, t.lx, t.cap));
    ADJ_OK(launch_zero_f64(h, t.lu, t.cap));
    ADJ_OK(launch_zero_f64(h, t.lez, N));
    ADJ_OK(launch_zero_f64(h, t.ler[0], N + 1));
    ADJ_OK(launch_zero_f64(h, t.lb, N));
    ADJ_OK(launch_zero_f64(h, t.lbp[0], N));     // B adjoint of the last step: nothing depends on E^T yet
    ADJ_OK(launch_zero_f64(h, (double *)t.lk_lo, N));
    ADJ_OK(launch_zero_f64(h, (double *)t.lk_hi, N));
    ADJ_OK(launch_zero_f64(h, (double *)t.scale, (int64_t)(sizeof(AdjScale) / 8)));
    hipStream_t const main_s = h->stream;
    hipStream_t rec_s = nullptr;
    hipEvent_t sev[5] = {};                       // forward done; recompute done [2]; sweep done [2]
    auto cleanup = [&]() {
        h->stream = main_s;
        for (auto &e : sev)
            if (e) (void)hipEventDestroy(e);
        if (rec_s) {
            (void)hipStreamSynchronize(rec_s);
            (void)hipStreamDestroy(rec_s);
        }
    };
    auto fail_rev = [&](pic_status rc) {
        cleanup();
        return done(rc);
    };
#define REV_OK(expr)                                                                                 \
    do {                                                                                             \
        const hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) return fail_rev(fail(PIC_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_))); \
    } while (0)
    REV_OK(hipStreamCreateWithFlags(&rec_s, hipStreamNonBlocking));
    for (auto &e : sev) REV_OK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    REV_OK(hipEventRecord(sev[0], main_s));
    REV_OK(hipStreamWaitEvent(rec_s, sev[0], 0));
    // recompute steps s0 .. s0+m-1 of segment ck out of place on rec_s: slot k of
    // its set holds the state before step s0+k
    auto recompute = [&](int64_t ck) -> hipError_t {
        const int q = t.nsets == 2 ? (int)(ck & 1) : 0;
        const int64_t s0 = ck * K, m = (T - s0) < K ? (T - s0) : K;
        h->stream = rec_s;
        hipError_t e = hipMemcpyAsync(w.ctr, t.ck_ctr[ck], sizeof(DevCounters), hipMemcpyDeviceToDevice, rec_s);
        if (e == hipSuccess) e = launch_zero_i64(h, w.j[0], N);
        if (e == hipSuccess) e = launch_zero_i64(h, w.j[1], N);
        for (int64_t k = 0; k + 1 < m && e == hipSuccess; ++k) {
            const double *xi = k == 0 ? t.ck_x[ck] : t.sg_x[q][(size_t)k];
            const double *ui = k == 0 ? t.ck_u[ck] : t.sg_u[q][(size_t)k];
            const double *ezo = k == 0 ? t.ck_ez[ck] : t.sg_ez[q][(size_t)k];
            const double *ero = k == 0 ? t.ck_er[ck] : t.sg_er[q][(size_t)k];
            const double *bo = k == 0 ? t.ck_b[ck] : t.sg_b[q][(size_t)k];
            e = launch_push_f64_ptrs(h, xi, ui, t.sg_x[q][(size_t)k + 1], t.sg_u[q][(size_t)k + 1], ezo);
            if (e == hipSuccess)
                e = launch_field_ptrs(h, ezo, ero, bo, t.sg_ez[q][(size_t)k + 1], t.sg_er[q][(size_t)k + 1],
                                      t.sg_b[q][(size_t)k + 1], t.sg_x[q][(size_t)k + 1], t.sg_u[q][(size_t)k + 1]);
            h->jbuf ^= 1;
        }
        h->stream = main_s;
        if (e == hipSuccess) e = hipEventRecord(sev[1 + q], rec_s);
        return e;
    };
    REV_OK(recompute(t.nck - 1));
    int64_t rev = 0;                              // reverse steps done (their parity picks the scale words)
    for (int64_t ck = t.nck - 1; ck >= 0; --ck) {
        const int q = t.nsets == 2 ? (int)(ck & 1) : 0;
        const int64_t s0 = ck * K, m = (T - s0) < K ? (T - s0) : K;
        REV_OK(hipStreamWaitEvent(main_s, sev[1 + q], 0));
        if (ck >= 1) {
            // the other set was last read by the sweep of segment ck+1
            if (ck + 1 <= t.nck - 1) REV_OK(hipStreamWaitEvent(rec_s, sev[3 + (q ^ 1)], 0));
            REV_OK(recompute(ck - 1));
        }
        for (int64_t k = m - 1; k >= 0; --k, ++rev) {
            const int64_t st = s0 + k;
            const int pp = (int)(rev & 1);
            AdjStepPtrs a{k == 0 ? t.ck_x[ck] : t.sg_x[q][(size_t)k], k == 0 ? t.ck_u[ck] : t.sg_u[q][(size_t)k],
                          k == 0 ? t.ck_ez[ck] : t.sg_ez[q][(size_t)k], t.nslots + st, t.nslots + st + 1, n_pre, nex,
                          t.lx, t.lu, t.lez, t.ler[pp], t.ler[pp ^ 1], t.lb, t.lbp[pp], t.lbp[pp ^ 1], t.lk_lo,
                          t.lk_hi, t.scale, (int)(rev % 3)};
            REV_OK(launch_adj_step(h, a));
        }
        REV_OK(hipEventRecord(sev[3 + q], main_s));
    }
#undef REV_OK
    cleanup();
    ADJ_OK(launch_adj_finish(h, t.lez, t.ler[(int)(T & 1)], t.gphi, t.cp, t.dp, t.g_rho, t.params));
    ADJ_OK(hipEventRecord(ev[1], h->stream));
    // restore the end state the forward left
    ADJ_OK(hipMemcpyAsync(w.ctr, t.final_ctr, sizeof(DevCounters), hipMemcpyDeviceToDevice, h->stream));
    h->jbuf = r.jb_final;
    ADJ_OK(launch_zero_i64(h, w.j[h->jbuf], N));
    ADJ_OK(hipMemcpyAsync(w.j[1 - h->jbuf], t.final_jlast, (size_t)N * 8, hipMemcpyDeviceToDevice, h->stream));
    // results
    std::vector<double> params((size_t)h->c.n_knots + 2);
    double grate = 0.0;
    ADJ_OK(hipMemcpyAsync(params.data(), t.params, params.size() * 8, hipMemcpyDeviceToHost, h->stream));
    ADJ_OK(hipMemcpyAsync(&grate, &t.scale->grate, 8, hipMemcpyDeviceToHost, h->stream));
    if (out->g_rho) ADJ_OK(hipMemcpyAsync(out->g_rho, t.g_rho, (size_t)(N + 1) * 8, hipMemcpyDeviceToHost, h->stream));
    ADJ_OK(hipStreamSynchronize(h->stream));
#undef ADJ_OK
    out->loss = r.loss;
    out->n_exit = r.n_exit;
    out->g_rate = dloss * grate;
    out->g_kappa = dloss * params[0];
    out->g_amp = dloss * params[1];
    if (out->g_rho)
        for (int64_t i = 0; i <= N; ++i) out->g_rho[i] *= dloss;
    if (out->g_knots)
        for (int k = 0; k < h->c.n_knots; ++k) out->g_knots[k] = dloss * params[(size_t)k + 2];
    float bms = 0;
    (void)hipEventElapsedTime(&bms, ev[0], ev[1]);
    out->forward_ms = r.forward_ms;
    out->backward_ms = bms;
    return done(PIC_OK);
}

pic_status check_tape(pic_handle *h, int64_t n_steps, int32_t checkpoint_every, void *d_tape, size_t tape_bytes)
{
    if (n_steps < 1 || checkpoint_every < 1) return fail(PIC_EINVAL, "n_steps and checkpoint_every must be >= 1");
    const size_t need = carve_tape(h, n_steps, checkpoint_every, nullptr).bytes;
    if (!d_tape || tape_bytes < need) return fail(PIC_EWORKSPACE, "tape of %zu bytes, %zu needed", tape_bytes, need);
    if (((uintptr_t)d_tape) % ALIGN) return fail(PIC_EWORKSPACE, "tape must be %zu-byte aligned", ALIGN);
    return PIC_OK;
}

}  // namespace

extern "C" {

size_t pic_adjoint_tape_bytes(pic_handle *h, int64_t n_steps, int32_t checkpoint_every)
{
    if (adjoint_supported(h) != PIC_OK) return 0;
    if (n_steps < 1 || checkpoint_every < 1) {
        fail(PIC_EINVAL, "n_steps and checkpoint_every must be >= 1");
        return 0;
    }
    return carve_tape(h, n_steps, checkpoint_every, nullptr).bytes;
}

pic_status pic_adjoint_forward(pic_handle *h, int64_t n_steps, int32_t checkpoint_every, void *d_tape,
                               size_t tape_bytes, pic_adjoint_out *out)
{
    pic_status s = adjoint_supported(h);
    if (s != PIC_OK) return s;
    if (!out) return fail(PIC_EINVAL, "out is NULL");
    if ((s = check_tape(h, n_steps, checkpoint_every, d_tape, tape_bytes)) != PIC_OK) return s;
    if (pic_status sp = resolve_pending(h)) return sp;
    return adjoint_forward(h, n_steps, checkpoint_every, d_tape, tape_bytes, out);
}

pic_status pic_backward(pic_handle *h, double dloss, pic_adjoint_out *out)
{
    pic_status s = adjoint_supported(h);
    if (s != PIC_OK) return s;
    if (!out) return fail(PIC_EINVAL, "out is NULL");
    if (!isfinite(dloss)) return fail(PIC_EINVAL, "dloss must be finite");
    if (!h->adj.valid) return fail(PIC_ESTATE, "no recorded forward (pic_adjoint_forward) on this tube");
    if (h->step != h->adj.step_end || h->mut != h->adj.mut)
        return fail(PIC_ESTATE, "the tube changed after its recorded forward (stepped, injected, loaded or rewritten)");
    return adjoint_backward(h, dloss, out);
}

pic_status pic_run_adjoint(pic_handle *h, int64_t n_steps, int32_t checkpoint_every, void *d_tape,
                           size_t tape_bytes, pic_adjoint_out *out)
{
    pic_status s = pic_adjoint_forward(h, n_steps, checkpoint_every, d_tape, tape_bytes, out);
    if (s != PIC_OK) return s;
    return adjoint_backward(h, 1.0, out);
}

}  // extern "C"
