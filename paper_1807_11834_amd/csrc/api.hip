// api.hip -- C ABI of the coupling library (see include/couple.h).
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "couple.h"
#include "couple_mlp.h"
#include "handle.hpp"
#include "launch.hpp"
#include "mlp_state.hpp"

using namespace cpl;

// Text of the last error reported without a handle (couple_init, the no-alloc
// step): a fixed per-thread buffer, so that reporting allocates nothing.
static thread_local char g_err[512];

static void set_global_err(const char *a, const char *b = "") { snprintf(g_err, sizeof(g_err), "%s%s", a, b); }

static int fail(couple_handle *h, int code, const std::string &msg) {
    if (h) h->err = msg;
    else set_global_err(msg.c_str());
    return code;
}

static void destroy_events(couple_handle *h) {
    for (hipEvent_t e : h->events) (void)hipEventDestroy(e);
    h->events.clear();
    h->names.clear();
    h->mk = Marker{};
}

static void release(couple_handle *h) {
    destroy_events(h);
    void *ptrs[] = {h->sort.keys_a, h->sort.keys_b, h->sort.vals_a, h->sort.vals_b, h->sort.hist,
                    h->sort.totals, h->sp, h->uf4, h->plo, h->dep, h->part, h->fgrid, h->alpha8};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    h->sort = SortScratch{};
    h->sp = h->uf4 = h->plo = h->dep = h->alpha8 = nullptr;
    h->fgrid = nullptr;
    h->part = nullptr;
}

// Configuration check shared by couple_init and couple_step_noalloc; returns
// nullptr when valid, else a static message (allocates nothing).
static const char *validate(const couple_config *c) {
    for (int a = 0; a < 3; ++a) {
        if (!(std::isfinite(c->box[a]) && c->box[a] > 0.0)) return "box lengths must be finite and > 0";
        if (c->nb[a] < 1) return "nb must be >= 1 on every axis";
    }
    if (!(c->ratio == 1 || c->ratio == 2 || c->ratio == 4)) return "ratio must be 1, 2 or 4";
    if (c->nb[0] > 32767) return "nb[0] must be <= 32767 (x-stencil nodes are packed in 16 bits)";
    const int64_t ncell = (int64_t)c->nb[0] * c->nb[1] * c->nb[2];
    if (ncell >= (int64_t(1) << 31) - 1) return "too many bulk cells (must be < 2^31 - 1)";
    const int64_t r3 = (int64_t)c->ratio * c->ratio * c->ratio;
    if (ncell * r3 >= (int64_t(1) << 40)) return "too many fine cells";
    for (int a = 0; a < 3; ++a)
        if ((int64_t)c->nb[a] * c->ratio >= (int64_t(1) << 30)) return "too many fine cells along an axis";
    if (!(std::isfinite(c->rho_f) && c->rho_f > 0.0)) return "rho_f must be finite and > 0";
    if (!(std::isfinite(c->mu_f) && c->mu_f > 0.0)) return "mu_f must be finite and > 0";
    if (!(std::isfinite(c->rho_p) && c->rho_p > 0.0)) return "rho_p must be finite and > 0";
    if (!(std::isfinite(c->eps_min) && c->eps_min >= 0.0 && c->eps_min < 1.0)) return "eps_min must be in [0, 1)";
    if (!std::isfinite(c->phi_fp64)) return "phi_fp64 must be finite";
    if (!(c->deposit == COUPLE_NGP || c->deposit == COUPLE_CIC)) return "deposit must be COUPLE_NGP or COUPLE_CIC";
    if (!(c->precision == COUPLE_FP64 || c->precision == COUPLE_FP32_WIDE || c->precision == COUPLE_FP32_NAIVE ||
          c->precision == COUPLE_FP32_KAHAN))
        return "unknown precision";
    if (!(c->vel_source == COUPLE_VEL_FINE || c->vel_source == COUPLE_VEL_BULK || c->vel_source == COUPLE_VEL_GIVEN ||
          c->vel_source == COUPLE_VEL_MLP))
        return "unknown vel_source";
    if (c->vel_source == COUPLE_VEL_MLP) {
        if (c->precision == COUPLE_FP64) return "vel_source MLP needs an FP32 precision";
        if (!(std::isfinite(c->mlp_tol) && c->mlp_tol >= 0.0)) return "mlp_tol must be finite and >= 0";
        if (c->mlp_period < 1) return "mlp_period must be >= 1";
    }
    if (!(c->semi_implicit == 0 || c->semi_implicit == 1)) return "semi_implicit must be 0 or 1";
    if (!(c->vof == 0 || c->vof == 1)) return "vof must be 0 or 1";
    if (c->vof && !(std::isfinite(c->rho_f2) && c->rho_f2 > 0.0)) return "rho_f2 must be finite and > 0";
    if (c->vof && !(std::isfinite(c->mu_f2) && c->mu_f2 > 0.0)) return "mu_f2 must be finite and > 0";
    if (!(c->advect == 0 || c->advect == 1)) return "advect must be 0 or 1";
    if (c->advect && !(std::isfinite(c->dt) && c->dt >= 0.0)) return "dt must be finite and >= 0";
    if (c->max_particles < 0 || c->max_particles >= (int64_t(1) << 31) - 1)
        return "max_particles must be in [0, 2^31 - 1)";
    return nullptr;
}

// The library scratch of a configuration for up to nmax particles: one buffer
// per entry of Buf, sized here for both couple_init (separate allocations) and
// couple_step_noalloc (carved from the static array).
enum Buf { B_KEYS_A, B_KEYS_B, B_VALS_A, B_VALS_B, B_HIST, B_TOTALS, B_SP, B_UF4, B_PLO, B_DEP, B_PART, B_FGRID,
           B_ALPHA8, B_COUNT };

struct ScratchPlan {
    size_t bytes[B_COUNT];
    int64_t part_stride;
};

static ScratchPlan scratch_plan(const couple_config &c, int64_t nmax) {
    ScratchPlan p{};
    const int64_t ncell = (int64_t)c.nb[0] * c.nb[1] * c.nb[2];
    const size_t fsz = (c.precision == COUPLE_FP64) ? sizeof(double) : sizeof(float);
    const int64_t ntile = sort_tiles(nmax > 0 ? nmax : 1);
    const int64_t pblk = (nmax + kBlock - 1) / kBlock, cblk = (ncell + kBlock - 1) / kBlock;
    // one FP64 partial per workgroup and slot: the stride covers the largest
    // grid of any kernel that writes partials
    const int64_t dblk = deposit_blocks(c.nb, ncell, c.deposit == COUPLE_CIC);
    const int64_t mblk = mlp_check_blocks(bricks_of(c.nb));
    const int64_t prblk = prolong_tiles(c.nb);
    p.part_stride = 1;
    for (int64_t b : {pblk, cblk, ntile, dblk, mblk, prblk})
        if (b > p.part_stride) p.part_stride = b;
    p.bytes[B_KEYS_A] = p.bytes[B_KEYS_B] = p.bytes[B_VALS_A] = p.bytes[B_VALS_B] = sizeof(uint32_t) * nmax;
    p.bytes[B_HIST] = sizeof(uint32_t) * 256 * ntile;
    p.bytes[B_TOTALS] = sizeof(uint32_t) * 256;
    p.bytes[B_SP] = p.bytes[B_UF4] = 4 * fsz * nmax;
    p.bytes[B_PLO] = fsz * ncell;
    const int dep_slots = deposit_group(c.nb) == 1 ? 9 : 4;   // CIC partial slots per cell and component
    p.bytes[B_DEP] = (c.deposit == COUPLE_CIC ? dep_slots * (c.semi_implicit ? 4 : 3) : 1) * fsz * ncell;
    p.bytes[B_PART] = sizeof(double) * (SL_COUNT * p.part_stride + SL_COUNT * 64);
    p.bytes[B_FGRID] = c.vel_source == COUPLE_VEL_MLP ? sizeof(float4) * 2 * ncell : 0;
    p.bytes[B_ALPHA8] = c.vof ? 8 * fsz * ncell : 0;
    return p;
}

// Buffer pointers of a plan in the handle.
static void **buf_slot(couple_handle *h, int b) {
    switch (b) {
    case B_KEYS_A: return (void **)&h->sort.keys_a;
    case B_KEYS_B: return (void **)&h->sort.keys_b;
    case B_VALS_A: return (void **)&h->sort.vals_a;
    case B_VALS_B: return (void **)&h->sort.vals_b;
    case B_HIST: return (void **)&h->sort.hist;
    case B_TOTALS: return (void **)&h->sort.totals;
    case B_SP: return &h->sp;
    case B_UF4: return &h->uf4;
    case B_PLO: return &h->plo;
    case B_DEP: return &h->dep;
    case B_PART: return (void **)&h->part;
    case B_FGRID: return (void **)&h->fgrid;
    default: return &h->alpha8;
    }
}

template <typename X> static bool dev_alloc(X **p, size_t bytes) {
    void *q = nullptr;
    if (bytes == 0) bytes = 256;
    if (hipMalloc(&q, bytes) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return false;
    }
    *p = static_cast<X *>(q);
    return true;
}

extern "C" int couple_init(const couple_config *cfg, couple_handle **out) {
    if (!cfg || !out) return fail(nullptr, COUPLE_EINVAL, "couple_init: NULL argument");
    *out = nullptr;
    if (const char *v = validate(cfg)) {
        set_global_err("couple_init: ", v);
        return COUPLE_EINVAL;
    }
    couple_handle *h = new (std::nothrow) couple_handle();
    if (!h) return fail(nullptr, COUPLE_ENOMEM, "couple_init: host allocation failed");
    h->cfg = *cfg;
    h->ncell = (int64_t)cfg->nb[0] * cfg->nb[1] * cfg->nb[2];
    h->nfine = h->ncell * cfg->ratio * cfg->ratio * cfg->ratio;
    const ScratchPlan plan = scratch_plan(*cfg, cfg->max_particles);
    h->part_stride = plan.part_stride;
    bool ok = true;
    for (int b = 0; b < B_COUNT && ok; ++b)
        if (plan.bytes[b] > 0 || b < B_FGRID) ok = dev_alloc(buf_slot(h, b), plan.bytes[b]);

    if (!ok) {
        release(h);
        delete h;
        return fail(nullptr, COUPLE_ENOMEM, "couple_init: device allocation failed");
    }
    *out = h;
    return COUPLE_OK;
}

extern "C" int couple_free(couple_handle *h) {
    if (!h) return COUPLE_OK;
    release(h);
    delete h;
    return COUPLE_OK;
}

extern "C" const char *couple_last_error(const couple_handle *h) {
    return h ? h->err.c_str() : g_err;
}

// Enqueue the step's kernels with the scratch of `h` (a handle of couple_init, or
// the stack-built view of the static scratch of couple_step_noalloc).  On a launch
// failure returns COUPLE_EHIP with a static description in *what and the HIP
// error in *herr; allocates nothing.
template <typename T>
static int step_impl(couple_handle *h, const couple_inputs *in, couple_outputs *out, hipStream_t st,
                     const char **what, hipError_t *herr, int phases = kPhaseAll, int64_t own_c0 = 0,
                     int64_t own_c1 = -1) {
    const couple_config &c = h->cfg;
    StepArgs<T> a;
    a.g = make_geo<T>(c);
    a.n = in->n;
    a.ratio = c.ratio;
    a.cic = c.deposit == COUPLE_CIC;
    a.sum_mode = c.precision == COUPLE_FP32_KAHAN ? kSumKahan : (c.precision == COUPLE_FP32_WIDE ? kSumWide : kSumPlain);
    a.vel_source = c.vel_source;
    a.advect = c.advect;
    a.semi = c.semi_implicit;
    a.vof = c.vof;
    a.rho_f2 = (T)c.rho_f2;
    a.mu_f2 = (T)c.mu_f2;
    a.fine_alpha = (const T *)in->fine_alpha;
    a.alpha = (T *)out->bulk_alpha;
    a.alpha8 = (T *)h->alpha8;
    a.dt = (T)c.dt;
    a.rho_f = (T)c.rho_f;
    a.mu_f = (T)c.mu_f;
    a.rho_p = (T)c.rho_p;
    a.eps_min = (T)c.eps_min;
    a.phi_fp64 = (float)c.phi_fp64;
    a.pos = (T *)in->pos;
    a.vel = (T *)in->vel;
    a.diam = (const T *)in->diam;
    a.fine[0] = (const T *)in->fine_u;
    a.fine[1] = (const T *)in->fine_v;
    a.fine[2] = (const T *)in->fine_w;
    a.fine[3] = (const T *)in->fine_p;
    a.uf_given = (const T *)in->uf_given;
    a.drag = (T *)out->drag;
    a.beta = (T *)out->beta;
    a.perm = out->perm;
    a.start = out->start;
    a.phi = (T *)out->bulk_phi;
    a.F = (T *)out->bulk_F;
    a.U = (T *)out->bulk_U;
    a.P = (T *)out->bulk_P;
    a.G = (T *)out->bulk_G;
    a.fine_eps = (T *)out->fine_eps;
    a.fine_F = (T *)out->fine_F;
    a.K = (T *)out->bulk_K;
    a.KU = (T *)out->bulk_KU;
    a.fine_K = (T *)out->fine_K;
    a.fine_KU = (T *)out->fine_KU;
    a.diag = out->diag;
    a.sp = (vec4<T> *)h->sp;
    a.uf4 = (vec4<T> *)h->uf4;
    a.Plo = (T *)h->plo;
    a.dep_partial = (T *)h->dep;
    a.part = h->part;
    a.part_stride = h->part_stride;
    a.mk = &h->mk;
    a.uf_out = (T *)out->uf;
    a.net = MlpNet{};
    if (h->mlp) {
        for (int l = 0; l < 4; ++l) a.net.wt[l] = h->mlp->net.wt[l];
        a.net.params = h->mlp->net.params;
        a.net.mean_inv = h->mlp->net.mean_inv;
        for (int k = 0; k < 3; ++k) a.net.scale[k] = (float)h->mlp->scale[k];
    }
    a.fgrid = h->fgrid;
    a.step = in->step;
    a.mlp_period = c.mlp_period > 0 ? c.mlp_period : 1;
    a.mlp_tol = (float)c.mlp_tol;
    a.n_bricks = bricks_of(c.nb);
    a.own_c0 = own_c0;
    a.own_c1 = own_c1 < 0 ? a.g.ncell : own_c1;

    (void)hipGetLastError();  // clear a stale error so that it is not reported as ours
    hipError_t e = hipSuccess;
    if (phases & kPhaseDeposit) {
        const uint32_t *skeys = nullptr;
        e = launch_bin_sort<T>(a.pos, a.diam, a.n, a.g, out->cell, a.uf4, out->perm, out->start, out->count, h->sort,
                               h->part + SL_NOUT * h->part_stride, &skeys, &h->mk, st);
        if (e != hipSuccess) {
            *what = "sort launch failed: ";
            *herr = e;
            return COUPLE_EHIP;
        }
        h->skeys = skeys;
    }
    a.keys = h->skeys;
    e = launch_stages<T>(a, st, phases);
    if (e != hipSuccess) {
        *what = "stage launch failed: ";
        *herr = e;
        return COUPLE_EHIP;
    }
    return COUPLE_OK;
}

int cpl::step_phases(couple_handle *h, const couple_inputs *in, couple_outputs *out, hipStream_t st, int phases,
                     int64_t own_c0, int64_t own_c1, const char **what, hipError_t *herr) {
    return h->cfg.precision == COUPLE_FP64 ? step_impl<double>(h, in, out, st, what, herr, phases, own_c0, own_c1)
                                           : step_impl<float>(h, in, out, st, what, herr, phases, own_c0, own_c1);
}

// Argument checks of a step (no allocation); nullptr when the call is valid.
static const char *check_step(const couple_config &c, const couple_inputs *in, const couple_outputs *out) {
    if (in->n < 0) return "n < 0";
    if (!in->fine_u || !in->fine_v || !in->fine_w || !in->fine_p) return "NULL fine-grid input";
    if (!out->count || !out->start || !out->bulk_phi || !out->bulk_F || !out->bulk_U || !out->bulk_P ||
        !out->bulk_G || !out->fine_eps || !out->fine_F || !out->diag)
        return "NULL grid output";
    if (c.semi_implicit && (!out->bulk_K || !out->bulk_KU || !out->fine_K || !out->fine_KU))
        return "semi_implicit needs bulk_K, bulk_KU, fine_K and fine_KU";
    if (c.vof && (!in->fine_alpha || !out->bulk_alpha)) return "vof needs fine_alpha and bulk_alpha";
    if (in->n > 0) {
        if (!in->pos || !in->vel || !in->diam) return "NULL particle input";
        if (!out->drag || !out->cell || !out->perm) return "NULL particle output";
        if (c.vel_source == COUPLE_VEL_GIVEN && !in->uf_given) return "vel_source GIVEN needs uf_given";
    }
    return nullptr;
}

extern "C" int couple_step(couple_handle *h, const couple_inputs *in, couple_outputs *out, void *stream) {
    if (!h) return fail(nullptr, COUPLE_EINVAL, "couple_step: NULL handle");
    if (!in || !out) return fail(h, COUPLE_EINVAL, "couple_step: NULL inputs or outputs");
    const couple_config &c = h->cfg;
    if (in->n > c.max_particles && in->n >= 0)
        return fail(h, COUPLE_ECAPACITY, "couple_step: n exceeds max_particles");
    if (const char *why = check_step(c, in, out)) return fail(h, COUPLE_EINVAL, std::string("couple_step: ") + why);
    if (c.vel_source == COUPLE_VEL_MLP && !h->mlp)
        return fail(h, COUPLE_ESTATE, "couple_step: vel_source MLP needs a network (couple_set_mlp)");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const char *what = nullptr;
    hipError_t herr = hipSuccess;
    const int rc = c.precision == COUPLE_FP64 ? step_impl<double>(h, in, out, st, &what, &herr)
                                              : step_impl<float>(h, in, out, st, &what, &herr);
    if (rc != COUPLE_OK) return fail(h, rc, std::string("couple_step: ") + what + hipGetErrorString(herr));
    return COUPLE_OK;
}

// ---- the step without allocation ---------------------------------------------
// The scratch of couple_step_noalloc: one array per device (each device that
// loads the library holds its own copy until the process ends).  Its device
// address is taken once per device with hipGetSymbolAddress; in host code the
// array's name is not a device address and is never passed to a kernel or copy.
static __device__ __align__(256) unsigned char scratch[COUPLE_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static void *g_scratch_ptr[kMaxDevices];
static std::mutex g_scratch_mu;

// Device address of this device's scratch array (nullptr on failure).
static void *scratch_on_device(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

extern "C" int couple_step_noalloc(const couple_config *cfg, const couple_inputs *in, couple_outputs *out,
                                   void *stream) {
    if (!cfg || !in || !out) {
        set_global_err("couple_step_noalloc: NULL argument");
        return COUPLE_EINVAL;
    }
    if (const char *v = validate(cfg)) {
        set_global_err("couple_step_noalloc: ", v);
        return COUPLE_EINVAL;
    }
    if (cfg->vel_source == COUPLE_VEL_MLP) {
        set_global_err("couple_step_noalloc: vel_source MLP needs a network handle (use couple_step)");
        return COUPLE_EINVAL;
    }
    if (const char *why = check_step(*cfg, in, out)) {
        set_global_err("couple_step_noalloc: ", why);
        return COUPLE_EINVAL;
    }
    // scratch for exactly these n particles, carved in 256-byte aligned pieces
    const ScratchPlan plan = scratch_plan(*cfg, in->n);
    size_t total = 0;
    for (int b = 0; b < B_COUNT; ++b) total += (plan.bytes[b] + 255) / 256 * 256;
    if (total > (size_t)COUPLE_NOALLOC_SCRATCH_BYTES) {
        snprintf(g_err, sizeof(g_err),
                 "couple_step_noalloc: this step needs %zu bytes of scratch, more than the %lld of the static "
                 "array (fewer particles or bulk cells, or couple_init + couple_step)",
                 total, (long long)COUPLE_NOALLOC_SCRATCH_BYTES);
        return COUPLE_ECAPACITY;
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        set_global_err("couple_step_noalloc: hipGetDevice failed");
        return COUPLE_EHIP;
    }
    unsigned char *base = static_cast<unsigned char *>(scratch_on_device(dev));
    if (!base) {
        set_global_err("couple_step_noalloc: hipGetSymbolAddress of the scratch array failed");
        return COUPLE_EHIP;
    }
    // a stack view of a handle over the static scratch (no events, no network)
    couple_handle h;
    h.cfg = *cfg;
    h.cfg.max_particles = in->n;
    h.ncell = (int64_t)cfg->nb[0] * cfg->nb[1] * cfg->nb[2];
    h.nfine = h.ncell * cfg->ratio * cfg->ratio * cfg->ratio;
    h.part_stride = plan.part_stride;
    size_t off = 0;
    for (int b = 0; b < B_COUNT; ++b) {
        *buf_slot(&h, b) = plan.bytes[b] ? base + off : nullptr;
        off += (plan.bytes[b] + 255) / 256 * 256;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    const char *what = nullptr;
    hipError_t herr = hipSuccess;
    const int rc = cfg->precision == COUPLE_FP64 ? step_impl<double>(&h, in, out, st, &what, &herr)
                                                 : step_impl<float>(&h, in, out, st, &what, &herr);
    // the view owns nothing: release() must not free the static array
    for (int b = 0; b < B_COUNT; ++b) *buf_slot(&h, b) = nullptr;
    if (rc != COUPLE_OK) {
        snprintf(g_err, sizeof(g_err), "couple_step_noalloc: %s%s", what, hipGetErrorString(herr));
        return rc;
    }
    return COUPLE_OK;
}

extern "C" int couple_timing_begin(couple_handle *h, int32_t max_steps) {
    if (!h) return fail(nullptr, COUPLE_EINVAL, "couple_timing_begin: NULL handle");
    if (max_steps < 1 || max_steps > 100000) return fail(h, COUPLE_EINVAL, "couple_timing_begin: max_steps out of range");
    destroy_events(h);
    const int per_step = 32;
    const int cap = max_steps * per_step;
    h->events.resize(cap);
    h->names.assign(cap, nullptr);
    for (int i = 0; i < cap; ++i) {
        if (hipEventCreate(&h->events[i]) != hipSuccess) {
            (void)hipGetLastError();
            h->events.resize(i);
            destroy_events(h);
            return fail(h, COUPLE_EHIP, "couple_timing_begin: hipEventCreate failed");
        }
    }
    h->mk.on = true;
    h->mk.events = h->events.data();
    h->mk.names = h->names.data();
    h->mk.cap = cap;
    h->mk.used = 0;
    return COUPLE_OK;
}

extern "C" int couple_timing_end(couple_handle *h, couple_kernel_stat *stats, int32_t max_stats, int32_t *n_stats) {
    if (!h || !n_stats || (max_stats > 0 && !stats)) return fail(h, COUPLE_EINVAL, "couple_timing_end: NULL argument");
    if (h->events.empty()) return fail(h, COUPLE_ESTATE, "couple_timing_end: timing was not started");
    const int used = h->mk.used;
    h->mk.on = false;
    int nout = 0;
    if (used > 0 && hipEventSynchronize(h->events[used - 1]) != hipSuccess) {
        (void)hipGetLastError();
        destroy_events(h);
        return fail(h, COUPLE_EHIP, "couple_timing_end: hipEventSynchronize failed");
    }
    for (int i = 0; i + 1 < used; ++i) {
        const char *nm = h->names[i];
        if (!nm) continue;  // gap between the end of a step and the next step
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, h->events[i], h->events[i + 1]) != hipSuccess) {
            (void)hipGetLastError();
            continue;
        }
        int k = 0;
        while (k < nout && std::strcmp(stats[k].name, nm) != 0) ++k;
        if (k == nout) {
            if (nout >= max_stats) continue;
            stats[k].name = nm;
            stats[k].launches = 0;
            stats[k].total_ms = 0.0;
            ++nout;
        }
        stats[k].launches += 1;
        stats[k].total_ms += ms;
    }
    *n_stats = nout;
    destroy_events(h);
    return COUPLE_OK;
}

extern "C" int couple_set_mlp(couple_handle *h, const couple_mlp *m) {
    if (!h) return fail(nullptr, COUPLE_EINVAL, "couple_set_mlp: NULL handle");
    h->mlp = m;
    return COUPLE_OK;
}
