// lbm_api.hip — the C-ABI of liblbm.so (declared in include/lbm.h): handle
// life cycle, parameter derivation, memory, HIP-graph replay of the step.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <cstdlib>
#include <new>
#include <string>

#include "d3q19_mrt.hpp"
#include "lbm_internal.hpp"
#include "lbm_observe.hpp"

using namespace lbm;

namespace {

thread_local std::string g_create_error;

lbm_status fail(lbm_handle* h, lbm_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (h) h->err = buf; else g_create_error = buf;
    return st;
}

lbm_status hip_fail(lbm_handle* h, hipError_t e, const char* what) {
    return fail(h, e == hipErrorOutOfMemory ? LBM_ERR_OUT_OF_MEMORY : LBM_ERR_DEVICE,
                "%s: %s", what, hipGetErrorString(e));
}

#define HIPCHK(h, call)                                  \
    do {                                                 \
        hipError_t e_ = (call);                          \
        if (e_ != hipSuccess) return hip_fail(h, e_, #call); \
    } while (0)

size_t elem_bytes_of(int precision) {
    switch (precision) {
        case LBM_FP64: return 8;
        case LBM_FP32: return 4;
        case LBM_FP16_DEV:
        case LBM_BF16_DEV: return 2;
    }
    return 0;
}

// Each direction plane is padded so that consecutive planes do not start at
// addresses that agree in their low ~17 bits: on MI355X, 19 same-cell accesses
// to planes whose stride is a multiple of 128 KiB (e.g. 800^3 floats) crowd
// the same HBM channels, costing ~10% of bandwidth.  1728 elements (27 x 64)
// measured best across FP32/FP16/FP64 at 800^3 and neutral at 100^3.
// LBM_PLANE_PAD (elements, multiple of 32) overrides it for tuning.
uint64_t plane_pad_elems() {
    const char* e = getenv("LBM_PLANE_PAD");
    return e ? (uint64_t)(atoll(e) / 32 * 32) : 1728;
}

uint64_t plane_elems_of(uint64_t ncell) { return (ncell + 63) / 64 * 64 + plane_pad_elems(); }

bool finite_pos(double v) { return isfinite(v) && v > 0.0; }

// Validate a config; on error write the reason into *why.
bool validate(const lbm_config* c, std::string* why) {
    char buf[256];
    auto bad = [&](const char* m) { *why = m; return false; };
    if (!c) return bad("config is NULL");
    if (c->nx < 1 || c->ny < 1 || c->nz < 1) return bad("nx, ny, nz must be >= 1");
    const uint64_t nc = (uint64_t)c->nx * c->ny * c->nz;
    if (nc >= (1ull << 31)) return bad("nx*ny*nz must be < 2^31");
    if (elem_bytes_of(c->precision) == 0) return bad("unknown precision");
    if (plane_elems_of(nc) * elem_bytes_of(c->precision) >= (1ull << 32))
        return bad("one direction plane must be < 4 GiB (FP64: < 536e6 cells)");
    if (c->streaming != LBM_STREAM_AA && c->streaming != LBM_STREAM_AB) return bad("unknown streaming");
    if (c->smag_form != 0 && c->smag_form != 1) return bad("smag_form must be 0 or 1");
    if (!(isfinite(c->tau0) && c->tau0 > 0.5)) return bad("tau0 must be finite and > 1/2");
    if (!(isfinite(c->smag_C) && c->smag_C >= 0.0)) return bad("smag_C must be finite and >= 0");
    if (!finite_pos(c->rho0)) return bad("rho0 must be finite and > 0");
    const double rates[5] = {c->s_e, c->s_eps, c->s_q, c->s_pi, c->s_m};
    for (double r : rates)
        if (!(isfinite(r) && r > 0.0 && r < 2.0)) return bad("relaxation rates must lie in (0, 2)");
    if (!(isfinite(c->storage_scale) && c->storage_scale >= 0.0)) return bad("storage_scale must be >= 0");
    if (c->storage_scale > 0.0) {
        int e;
        if (frexp(c->storage_scale, &e) != 0.5) return bad("storage_scale must be a power of two");
    }
    if (c->n_force_modes < 0 || c->n_force_modes > 64) return bad("n_force_modes must be 0..64");
    if (c->n_force_modes > 0 && !c->force_modes) return bad("force_modes is NULL");
    for (int m = 0; m < c->n_force_modes; ++m) {
        const lbm_force_mode& md = c->force_modes[m];
        if (md.k[0] < -2 || md.k[0] > 2) {
            snprintf(buf, sizeof buf, "force mode %d: |k[0]| must be <= 2", m);
            *why = buf;
            return false;
        }
        if (md.reserved != 0) return bad("force mode reserved field must be 0");
        if (!(isfinite(md.amp[0]) && isfinite(md.amp[1]) && isfinite(md.amp[2]) && isfinite(md.phase)))
            return bad("force mode amplitudes and phase must be finite");
    }
    if (c->steps_per_graph != 0 &&
        (c->steps_per_graph < 2 || c->steps_per_graph > 1024 || (c->steps_per_graph & 1)))
        return bad("steps_per_graph must be 0 or even in [2, 1024]");
    if (c->temporal_block < 0 || c->temporal_block > 2) return bad("temporal_block must be 0, 1 or 2");
    if (c->tau_mode != 0 && c->tau_mode != 1) return bad("tau_mode must be 0 or 1");
    if (c->temporal_block == 2) {
        if (c->streaming != LBM_STREAM_AB) return bad("temporal_block 2 needs A/B streaming");
        if (c->precision == LBM_FP64) return bad("temporal_block 2 needs 32- or 16-bit storage");
        if (c->steps_per_graph % 4) return bad("temporal_block 2 needs steps_per_graph % 4 == 0");
    }
    return true;
}

size_t required_bytes(const lbm_config* c) {
    const uint64_t nc = (uint64_t)c->nx * c->ny * c->nz;
    return (size_t)(19 * plane_elems_of(nc) * elem_bytes_of(c->precision) *
                    (c->streaming == LBM_STREAM_AB ? 2 : 1));
}

double default_scale(int precision) { return precision == LBM_FP16_DEV ? 32768.0 : 1.0; }

lbm_status ensure_staging(lbm_handle* h, size_t doubles) {
    if (h->staging_elems >= doubles) return LBM_OK;
    if (h->staging) (void)hipFree(h->staging);
    h->staging = nullptr;
    h->staging_elems = 0;
    HIPCHK(h, hipMalloc(&h->staging, doubles * sizeof(double)));
    h->staging_elems = doubles;
    return LBM_OK;
}

// Large staging buffers are returned after each observation call.
void trim_staging(lbm_handle* h) {
    if (h->staging && h->staging_elems * sizeof(double) > (256u << 20)) {
        (void)hipFree(h->staging);
        h->staging = nullptr;
        h->staging_elems = 0;
    }
}

lbm_status sync(lbm_handle* h) {
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return LBM_OK;
}

lbm_status capture_graph(lbm_handle* h) {
    const int G = h->cfg.steps_per_graph;
    const bool tb2 = h->cfg.temporal_block == 2;
    if (!h->cap_stream) HIPCHK(h, hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    HIPCHK(h, hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeRelaxed));
    // the graph starts from AA parity 0 / AB array 0 and ends there (G even; G % 4 == 0
    // for pairs of steps, whose launches alternate the arrays)
    const int launches = tb2 ? G / 2 : G;
    for (int k = 0; k < launches; ++k) {
        LatticeArgs a = h->args;
        int pat = PAT_AB;
        if (h->cfg.streaming == LBM_STREAM_AB) {
            set_arrays(a, h->state[k & 1], h->state[(k & 1) ^ 1]);
        } else {
            set_arrays(a, h->state[0], h->state[0]);
            pat = (k & 1) ? PAT_AA_ODD : PAT_AA_EVEN;
        }
        hipError_t e = tb2 ? launch_step_tb2(h->cfg.precision, a, h->cap_stream)
                           : launch_step(h->cfg.precision, pat, a, h->cap_stream);
        if (e != hipSuccess) {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(h->cap_stream, &g);
            if (g) (void)hipGraphDestroy(g);
            return hip_fail(h, e, "launch during capture");
        }
    }
    HIPCHK(h, hipStreamEndCapture(h->cap_stream, &h->graph));
    const hipError_t e = hipGraphInstantiate(&h->gexec, h->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {   // no half-made graph is kept: the next call captures anew
        (void)hipGraphDestroy(h->graph);
        h->graph = nullptr;
        h->gexec = nullptr;
        return hip_fail(h, e, "hipGraphInstantiate");
    }
    return LBM_OK;
}

}  // namespace

namespace lbm {

int current_pattern(const lbm_handle* h) {
    if (h->cfg.streaming == LBM_STREAM_AB) return PAT_AB;
    return (h->steps & 1) ? PAT_AA_ODD : PAT_AA_EVEN;
}

void set_arrays(LatticeArgs& L, void* a, void* b) {
    L.a = a;
    L.b = b;
    const uint64_t pbytes = L.plane * (uint64_t)L.elem_bytes;
    for (int i = 0; i < 19; ++i) {
        L.pa[i] = (char*)a + (uint64_t)i * pbytes;
        L.pb[i] = (char*)b + (uint64_t)i * pbytes;
    }
}

LatticeArgs current_args(const lbm_handle* h) {
    LatticeArgs a = h->args;
    if (h->cfg.streaming == LBM_STREAM_AB) {
        set_arrays(a, h->state[h->cur], h->state[h->cur ^ 1]);
    } else {
        set_arrays(a, h->state[0], h->state[0]);
    }
    return a;
}

void advance(lbm_handle* h) {
    h->steps += 1;
    if (h->cfg.streaming == LBM_STREAM_AB) h->cur ^= 1;
}

hipError_t launch_stats(lbm_handle* h, double** result) {
    const uint64_t nc = h->args.ncell;
    const int nb = (int)std::min<uint64_t>(kDiagBlocks, (nc + 255) / 256);
    *result = h->partials + (size_t)kDiagBlocks * kDiagSlots;
    return launch_diag(h->cfg.precision, current_pattern(h), current_args(h), h->partials, nb,
                       *result, h->stream);
}

void fill_stats(const lbm_handle* h, const double* r, int64_t steps, lbm_stats* out) {
    const uint64_t nc = h->args.ncell;
    memset(out, 0, sizeof *out);
    out->n_cells = (int64_t)nc;
    out->steps = steps;
    out->n_nonfinite = (int64_t)r[12];
    const double n = (double)nc - r[12];
    const double th0 = h->cfg.tau0 - 0.5;
    // central moments of tau_t = theta - theta0 from its raw power sums
    const double m1 = r[0] / n, e2 = r[1] / n, e3 = r[2] / n, e4 = r[3] / n;
    double var = e2 - m1 * m1;
    if (var < 0.0) var = 0.0;
    const double mu3 = e3 - 3.0 * m1 * e2 + 2.0 * m1 * m1 * m1;
    const double mu4 = e4 - 4.0 * m1 * e3 + 6.0 * m1 * m1 * e2 - 3.0 * m1 * m1 * m1 * m1;
    const double skew = var > 0.0 ? mu3 / (var * sqrt(var)) : NAN;
    const double flat = var > 0.0 ? mu4 / (var * var) : NAN;
    out->theta_mean = th0 + m1;
    out->theta_var = var;
    out->theta_skew = skew;
    out->theta_flat = flat;
    out->theta_min = th0 + r[4];
    out->theta_max = th0 + r[5];
    const double s3 = 1.7320508075688772;   // K_t = sqrt(3) theta (ell = delta_x)
    out->kt_mean = s3 * out->theta_mean;
    out->kt_var = 3.0 * var;
    out->kt_skew = skew;
    out->kt_flat = flat;
    out->kt_min = s3 * out->theta_min;
    out->kt_max = s3 * out->theta_max;
    out->mass = (double)nc * h->cfg.rho0 + r[6];
    out->momentum[0] = r[7];
    out->momentum[1] = r[8];
    out->momentum[2] = r[9];
    out->energy = r[10] / n;
    out->energy_rho = r[11] / n;
    out->strain2 = r[13] / n;
    out->nut_strain2 = r[14] / (3.0 * n);   // nu_t = tau_t / 3
    out->injection = r[15] / n;
    for (int a = 0; a < 3; ++a) out->u_mean[a] = r[16 + a] / n;
    for (int a = 0; a < 6; ++a) out->uu[a] = r[19 + a] / n;
}

}  // namespace lbm

extern "C" {

void lbm_config_default(lbm_config* c) {
    if (!c) return;
    memset(c, 0, sizeof *c);
    c->nx = c->ny = c->nz = 32;
    c->precision = LBM_FP32;
    c->streaming = LBM_STREAM_AA;
    c->smag_form = 0;
    c->tau0 = 0.51;
    c->smag_C = 0.1;
    c->rho0 = 1.0;
    c->s_e = 1.19;
    c->s_eps = 1.4;
    c->s_q = 1.2;
    c->s_pi = 1.4;
    c->s_m = 1.98;
    c->storage_scale = 0.0;
    c->steps_per_graph = 64;
}

size_t lbm_required_bytes(const lbm_config* cfg) {
    std::string why;
    if (!validate(cfg, &why)) return 0;
    return required_bytes(cfg);
}

lbm_status lbm_create(const lbm_config* cfg, lbm_handle** out) {
    if (!out) return fail(nullptr, LBM_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    std::string why;
    if (!validate(cfg, &why)) return fail(nullptr, LBM_ERR_INVALID_ARG, "%s", why.c_str());
    const size_t need = required_bytes(cfg);
    if (cfg->device_buffer) {
        if (cfg->device_buffer_bytes < need)
            return fail(nullptr, LBM_ERR_INVALID_ARG, "device_buffer has %llu bytes, %llu needed",
                        (unsigned long long)cfg->device_buffer_bytes, (unsigned long long)need);
        if (((uintptr_t)cfg->device_buffer) & 255u)
            return fail(nullptr, LBM_ERR_INVALID_ARG, "device_buffer must be 256-byte aligned");
    }
    lbm_handle* h = new (std::nothrow) lbm_handle();
    if (!h) return fail(nullptr, LBM_ERR_OUT_OF_MEMORY, "host allocation failed");
    h->cfg = *cfg;
    h->modes.assign(cfg->force_modes, cfg->force_modes + cfg->n_force_modes);
    h->cfg.force_modes = h->modes.empty() ? nullptr : h->modes.data();
    h->stream = (hipStream_t)cfg->hip_stream;
    if (h->cfg.storage_scale == 0.0) h->cfg.storage_scale = default_scale(cfg->precision);
    if (cfg->precision == LBM_FP64 || cfg->precision == LBM_FP32) h->cfg.storage_scale = 1.0;

    auto abort_create = [&](lbm_status st) {
        g_create_error = h->err;
        lbm_destroy(h);
        return st;
    };
    hipError_t e = hipGetDevice(&h->device);
    if (e != hipSuccess) return abort_create(hip_fail(h, e, "hipGetDevice"));

    const uint64_t nc = (uint64_t)cfg->nx * cfg->ny * cfg->nz;
    h->elem_bytes = elem_bytes_of(cfg->precision);
    h->plane_elems = plane_elems_of(nc);
    h->state_bytes = need;
    if (cfg->device_buffer) {
        h->state_base = cfg->device_buffer;
        h->own_state = false;
    } else {
        e = hipMalloc(&h->state_base, need);
        if (e != hipSuccess) return abort_create(hip_fail(h, e, "hipMalloc(state)"));
        h->own_state = true;
    }
    const size_t one = 19 * h->plane_elems * h->elem_bytes;
    h->state[0] = h->state_base;
    h->state[1] = cfg->streaming == LBM_STREAM_AB ? (char*)h->state_base + one : h->state_base;

    const size_t rbytes = cfg->precision == LBM_FP64 ? 8 : 4;
    e = hipMalloc((void**)&h->partials, (kDiagBlocks + 1) * kDiagSlots * sizeof(double));
    if (e != hipSuccess) return abort_create(hip_fail(h, e, "hipMalloc(partials)"));
    if (cfg->n_force_modes > 0) {
        e = hipMalloc((void**)&h->d_modes, cfg->n_force_modes * sizeof(lbm_force_mode));
        if (e == hipSuccess) e = hipMalloc(&h->rowc, (size_t)cfg->ny * cfg->nz * 16 * rbytes);
        if (e == hipSuccess) e = hipMalloc(&h->xtab, (size_t)cfg->nx * 4 * rbytes);
        if (e != hipSuccess) return abort_create(hip_fail(h, e, "hipMalloc(force tables)"));
        e = hipMemcpyAsync(h->d_modes, h->modes.data(), cfg->n_force_modes * sizeof(lbm_force_mode),
                           hipMemcpyHostToDevice, h->stream);
        if (e != hipSuccess) return abort_create(hip_fail(h, e, "hipMemcpy(force modes)"));
    }

    LatticeArgs& a = h->args;
    a.plane = h->plane_elems;
    a.elem_bytes = (uint32_t)h->elem_bytes;
    a.nx = cfg->nx; a.ny = cfg->ny; a.nz = cfg->nz;
    a.nxy = (uint32_t)cfg->nx * cfg->ny;
    a.ncell = (uint32_t)nc;
    a.mx = make_div_magic(cfg->nx);
    a.my = make_div_magic(cfg->ny);
    a.rowc = h->rowc;
    a.xtab = h->xtab;
    // eq. les_viscosity: tau_e = tau0 + 3 C |S| (C^2 for smag_form 1), Delta = 1;
    // eq. yu_strain at delta_t = 1 (rates per tau_mode below)
    const double Cm = cfg->smag_form == 1 ? cfg->smag_C * cfg->smag_C : cfg->smag_C;
    CollideConst<double>& kd = a.kd;
    kd.tau0 = cfg->tau0;
    kd.c3 = 3.0 * Cm;
    // explicit: s_1 = s_e, s_9 = 1/tau0 in eq. yu_strain; self-consistent: no s_1
    // term, strain evaluated at s_9 = 1 and rescaled by 1/tau_e in the closed form
    const bool sc = cfg->tau_mode == 1;
    kd.a_e = sc ? 0.0 : cfg->s_e / (38.0 * cfg->rho0);
    kd.b9 = (sc ? 1.0 : 1.0 / cfg->tau0) / (2.0 * cfg->rho0);
    kd.tau0_sq = cfg->tau0 * cfg->tau0;
    kd.self_consistent = sc ? 1 : 0;
    kd.pad = 0;
    kd.s_e = cfg->s_e; kd.s_eps = cfg->s_eps; kd.s_q = cfg->s_q; kd.s_pi = cfg->s_pi;
    kd.s_m = cfg->s_m;
    kd.rho0 = cfg->rho0;
    CollideConst<float>& kf = a.kf;
    kf.tau0 = (float)kd.tau0; kf.c3 = (float)kd.c3; kf.a_e = (float)kd.a_e; kf.b9 = (float)kd.b9;
    kf.s_e = (float)kd.s_e; kf.s_eps = (float)kd.s_eps; kf.s_q = (float)kd.s_q;
    kf.s_pi = (float)kd.s_pi; kf.s_m = (float)kd.s_m; kf.rho0 = (float)kd.rho0;
    kf.tau0_sq = (float)kd.tau0_sq; kf.self_consistent = kd.self_consistent; kf.pad = 0;
    a.tau0 = cfg->tau0;
    a.rho0 = cfg->rho0;
    a.sigma = h->cfg.storage_scale;
    a.inv_sigma = 1.0 / h->cfg.storage_scale;
    a.sigma_f = (float)a.sigma;
    a.inv_sigma_f = (float)a.inv_sigma;
    // XCD-aware block order of the step kernel: one contiguous range per XCD
    // while the state fits the 256 MB last-level cache, 64-block chunks taken in
    // turn by the 8 XCDs once it does not (measured +2.4 % at 800^3, +3-4 % at
    // 256^3 and 512^3, -1.8 % at 100^3).  LBM_XCD_REMAP = 0 (off), 1 or a chunk
    // size overrides it.
    const char* remap = getenv("LBM_XCD_REMAP");
    a.xcd_remap = remap ? atoi(remap) : (need > ((size_t)256 << 20) ? 64 : 1);
    // non-temporal stores in the step (off by default; LBM_NT=2 turns them on)
    const char* nt = getenv("LBM_NT");
    a.nt_mode = nt ? (atoi(nt) & 2) : 0;

    if (cfg->n_force_modes > 0) {
        e = launch_tables(cfg->precision, a, h->d_modes, cfg->n_force_modes, h->stream);
        if (e != hipSuccess) return abort_create(hip_fail(h, e, "force tables"));
    }
    e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return abort_create(hip_fail(h, e, "hipStreamSynchronize"));
    *out = h;
    return LBM_OK;
}

lbm_status lbm_init_seeded(lbm_handle* h, int32_t kind, double amplitude, uint64_t seed) {
    if (!h) return LBM_ERR_INVALID_ARG;
    if (kind < LBM_INIT_NOISE || kind > LBM_INIT_REST)
        return fail(h, LBM_ERR_INVALID_ARG, "unknown init kind %d", kind);
    if (!isfinite(amplitude)) return fail(h, LBM_ERR_INVALID_ARG, "amplitude must be finite");
    h->steps = 0;
    h->cur = 0;
    const int pat = h->cfg.streaming == LBM_STREAM_AB ? PAT_AB : PAT_AA_EVEN;
    hipError_t e = launch_init(h->cfg.precision, pat, current_args(h), kind, amplitude, seed, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "init kernel");
    h->initialized = true;
    return LBM_OK;
}

lbm_status lbm_step(lbm_handle* h, int64_t n) {
    if (!h) return LBM_ERR_INVALID_ARG;
    if (n < 0) return fail(h, LBM_ERR_INVALID_ARG, "n must be >= 0");
    if (!h->initialized) return fail(h, LBM_ERR_STATE, "lbm_step before lbm_init_seeded/lbm_set_populations");
    const int G = h->cfg.steps_per_graph;
    const bool tb2 = h->cfg.temporal_block == 2;
    while (n > 0) {
        const bool aligned = h->cfg.streaming == LBM_STREAM_AB ? (h->cur == 0) : ((h->steps & 1) == 0);
        if (G > 0 && n >= G && aligned) {
            if (!h->gexec) {
                lbm_status st = capture_graph(h);
                if (st != LBM_OK) return st;
            }
            HIPCHK(h, hipGraphLaunch(h->gexec, h->stream));
            h->steps += G;
            n -= G;
        } else if (tb2 && n >= 2) {
            hipError_t e = launch_step_tb2(h->cfg.precision, current_args(h), h->stream);
            if (e != hipSuccess) return hip_fail(h, e, "two-step kernel");
            h->steps += 2;
            h->cur ^= 1;
            n -= 2;
        } else {
            hipError_t e = launch_step(h->cfg.precision, current_pattern(h), current_args(h), h->stream);
            if (e != hipSuccess) return hip_fail(h, e, "step kernel");
            advance(h);
            n -= 1;
        }
    }
    return LBM_OK;
}

lbm_status lbm_stream_only(lbm_handle* h, int64_t n) {
    if (!h) return LBM_ERR_INVALID_ARG;
    if (n < 0) return fail(h, LBM_ERR_INVALID_ARG, "n must be >= 0");
    if (!h->initialized) return fail(h, LBM_ERR_STATE, "lbm_stream_only before lbm_init_seeded/lbm_set_populations");
    for (int64_t k = 0; k < n; ++k) {
        hipError_t e = launch_stream(h->cfg.precision, current_pattern(h), current_args(h), h->stream);
        if (e != hipSuccess) return hip_fail(h, e, "streaming kernel");
        advance(h);
    }
    return LBM_OK;
}

lbm_status lbm_moments(lbm_handle* h, double* rho, double* u) {
    if (!h) return LBM_ERR_INVALID_ARG;
    if (!h->initialized) return fail(h, LBM_ERR_STATE, "state not initialised");
    const size_t nc = h->args.ncell;
    lbm_status st = ensure_staging(h, 4 * nc);
    if (st != LBM_OK) return st;
    hipError_t e = launch_moments(h->cfg.precision, current_pattern(h), current_args(h), h->staging,
                                  h->staging + nc, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "moments kernel");
    if (rho) HIPCHK(h, hipMemcpyAsync(rho, h->staging, nc * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    if (u) HIPCHK(h, hipMemcpyAsync(u, h->staging + nc, 3 * nc * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    st = sync(h);
    trim_staging(h);
    return st;
}

lbm_status lbm_kt_stats(lbm_handle* h, lbm_stats* out) {
    if (!h || !out) return h ? fail(h, LBM_ERR_INVALID_ARG, "out is NULL") : LBM_ERR_INVALID_ARG;
    if (!h->initialized) return fail(h, LBM_ERR_STATE, "state not initialised");
    double* result = nullptr;
    hipError_t e = launch_stats(h, &result);
    if (e != hipSuccess) return hip_fail(h, e, "diagnostic kernel");
    double r[kDiagSlots];
    HIPCHK(h, hipMemcpyAsync(r, result, kStatSums * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    lbm_status st = sync(h);
    if (st != LBM_OK) return st;
    fill_stats(h, r, h->steps, out);
    if (out->n_nonfinite > 0)
        return fail(h, LBM_ERR_UNSTABLE, "%lld non-finite cells", (long long)out->n_nonfinite);
    return LBM_OK;
}

lbm_status lbm_kt_field(lbm_handle* h, float* kt) {
    if (!h || !kt) return h ? fail(h, LBM_ERR_INVALID_ARG, "kt is NULL") : LBM_ERR_INVALID_ARG;
    if (!h->initialized) return fail(h, LBM_ERR_STATE, "state not initialised");
    const size_t nc = h->args.ncell;
    lbm_status st = ensure_staging(h, (nc + 1) / 2);
    if (st != LBM_OK) return st;
    hipError_t e = launch_ktfield(h->cfg.precision, current_pattern(h), current_args(h),
                                  (float*)h->staging, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "kt kernel");
    HIPCHK(h, hipMemcpyAsync(kt, h->staging, nc * sizeof(float), hipMemcpyDeviceToHost, h->stream));
    st = sync(h);
    trim_staging(h);
    return st;
}

lbm_status lbm_kt_slice(lbm_handle* h, int32_t z, float* kt) {
    if (!h || !kt) return h ? fail(h, LBM_ERR_INVALID_ARG, "kt is NULL") : LBM_ERR_INVALID_ARG;
    if (z < 0 || (uint32_t)z >= h->args.nz)
        return fail(h, LBM_ERR_INVALID_ARG, "z = %d outside 0..%u", z, h->args.nz - 1);
    if (!h->initialized) return fail(h, LBM_ERR_STATE, "state not initialised");
    const size_t n = h->args.nxy;
    lbm_status st = ensure_staging(h, (n + 1) / 2);
    if (st != LBM_OK) return st;
    hipError_t e = launch_ktslice(h->cfg.precision, current_pattern(h), current_args(h),
                                  (uint32_t)z, (float*)h->staging, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "kt slice kernel");
    HIPCHK(h, hipMemcpyAsync(kt, h->staging, n * sizeof(float), hipMemcpyDeviceToHost, h->stream));
    st = sync(h);
    trim_staging(h);
    return st;
}

lbm_status lbm_get_populations(lbm_handle* h, double* f) {
    if (!h || !f) return h ? fail(h, LBM_ERR_INVALID_ARG, "f is NULL") : LBM_ERR_INVALID_ARG;
    if (!h->initialized) return fail(h, LBM_ERR_STATE, "state not initialised");
    const size_t nc = h->args.ncell;
    lbm_status st = ensure_staging(h, nc);
    if (st != LBM_OK) return st;
    const int pat = current_pattern(h);
    const LatticeArgs a = current_args(h);
    for (int i = 0; i < 19; ++i) {
        hipError_t e = launch_gather_plane(h->cfg.precision, pat, a, i, h->staging, h->stream);
        if (e != hipSuccess) return hip_fail(h, e, "gather kernel");
        HIPCHK(h, hipMemcpyAsync(f + (size_t)i * nc, h->staging, nc * sizeof(double),
                                 hipMemcpyDeviceToHost, h->stream));
    }
    st = sync(h);
    trim_staging(h);
    return st;
}

lbm_status lbm_set_populations(lbm_handle* h, const double* f) {
    if (!h || !f) return h ? fail(h, LBM_ERR_INVALID_ARG, "f is NULL") : LBM_ERR_INVALID_ARG;
    const size_t nc = h->args.ncell;
    lbm_status st = ensure_staging(h, nc);
    if (st != LBM_OK) return st;
    const int pat = current_pattern(h);
    const LatticeArgs a = current_args(h);
    for (int i = 0; i < 19; ++i) {
        HIPCHK(h, hipMemcpyAsync(h->staging, f + (size_t)i * nc, nc * sizeof(double),
                                 hipMemcpyHostToDevice, h->stream));
        hipError_t e = launch_scatter_plane(h->cfg.precision, pat, a, i, h->staging, h->stream);
        if (e != hipSuccess) return hip_fail(h, e, "scatter kernel");
    }
    st = sync(h);
    trim_staging(h);
    if (st == LBM_OK) h->initialized = true;
    return st;
}

lbm_status lbm_sample_populations(lbm_handle* h, const int64_t* cells, int64_t n, double* out) {
    if (!h) return LBM_ERR_INVALID_ARG;
    if (n < 0 || (n > 0 && (!cells || !out))) return fail(h, LBM_ERR_INVALID_ARG, "bad sample arguments");
    if (!h->initialized) return fail(h, LBM_ERR_STATE, "state not initialised");
    if (n == 0) return LBM_OK;
    for (int64_t j = 0; j < n; ++j)
        if (cells[j] < 0 || cells[j] >= (int64_t)h->args.ncell)
            return fail(h, LBM_ERR_INVALID_ARG, "cell index %lld out of range", (long long)cells[j]);
    if (h->d_cells_cap < (size_t)n) {
        if (h->d_cells) (void)hipFree(h->d_cells);
        h->d_cells = nullptr;
        h->d_cells_cap = 0;
        HIPCHK(h, hipMalloc((void**)&h->d_cells, n * sizeof(int64_t)));
        h->d_cells_cap = n;
    }
    lbm_status st = ensure_staging(h, (size_t)n * 19);
    if (st != LBM_OK) return st;
    HIPCHK(h, hipMemcpyAsync(h->d_cells, cells, n * sizeof(int64_t), hipMemcpyHostToDevice, h->stream));
    hipError_t e = launch_sample(h->cfg.precision, current_pattern(h), current_args(h), h->d_cells, n,
                                 h->staging, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "sample kernel");
    HIPCHK(h, hipMemcpyAsync(out, h->staging, (size_t)n * 19 * sizeof(double), hipMemcpyDeviceToHost,
                             h->stream));
    st = sync(h);
    trim_staging(h);
    return st;
}

size_t lbm_state_bytes(const lbm_handle* h) {
    return h ? 19 * h->plane_elems * h->elem_bytes : 0;
}

lbm_status lbm_save_state(lbm_handle* h, void* host, size_t bytes, int64_t* steps) {
    if (!h) return LBM_ERR_INVALID_ARG;
    if (!host || bytes != lbm_state_bytes(h)) return fail(h, LBM_ERR_INVALID_ARG, "bad checkpoint buffer");
    if (!h->initialized) return fail(h, LBM_ERR_STATE, "state not initialised");
    HIPCHK(h, hipMemcpyAsync(host, h->state[h->cur], bytes, hipMemcpyDeviceToHost, h->stream));
    lbm_status st = sync(h);
    if (st == LBM_OK && steps) *steps = h->steps;
    return st;
}

lbm_status lbm_load_state(lbm_handle* h, const void* host, size_t bytes, int64_t steps) {
    if (!h) return LBM_ERR_INVALID_ARG;
    if (!host || bytes != lbm_state_bytes(h) || steps < 0)
        return fail(h, LBM_ERR_INVALID_ARG, "bad checkpoint buffer or step count");
    h->cur = 0;
    HIPCHK(h, hipMemcpyAsync(h->state[0], host, bytes, hipMemcpyHostToDevice, h->stream));
    lbm_status st = sync(h);
    if (st == LBM_OK) {
        h->steps = steps;
        h->initialized = true;
    }
    return st;
}

lbm_status lbm_synchronize(lbm_handle* h) {
    if (!h) return LBM_ERR_INVALID_ARG;
    return sync(h);
}

lbm_status lbm_set_stream(lbm_handle* h, void* hip_stream) {
    if (!h) return LBM_ERR_INVALID_ARG;
    h->stream = (hipStream_t)hip_stream;
    h->cfg.hip_stream = hip_stream;
    return LBM_OK;
}

int64_t lbm_steps_done(const lbm_handle* h) { return h ? h->steps : -1; }

int64_t lbm_num_cells(const lbm_handle* h) { return h ? (int64_t)h->args.ncell : -1; }

void lbm_destroy(lbm_handle* h) {
    if (!h) return;
    (void)hipStreamSynchronize(h->stream);
    if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    if (h->own_state && h->state_base) (void)hipFree(h->state_base);
    if (h->rowc) (void)hipFree(h->rowc);
    if (h->xtab) (void)hipFree(h->xtab);
    if (h->d_modes) (void)hipFree(h->d_modes);
    if (h->partials) (void)hipFree(h->partials);
    if (h->staging) (void)hipFree(h->staging);
    if (h->d_cells) (void)hipFree(h->d_cells);
    lbm::release_analysis(h->ana);
    delete h;
}

const char* lbm_status_string(lbm_status s) {
    switch (s) {
        case LBM_OK: return "ok";
        case LBM_ERR_INVALID_ARG: return "invalid argument";
        case LBM_ERR_OUT_OF_MEMORY: return "out of memory";
        case LBM_ERR_DEVICE: return "device error";
        case LBM_ERR_UNSTABLE: return "unstable (non-finite state)";
        case LBM_ERR_STATE: return "call out of order";
    }
    return "unknown status";
}

const char* lbm_last_error(const lbm_handle* h) {
    return h ? h->err.c_str() : g_create_error.c_str();
}

}  // extern "C"
