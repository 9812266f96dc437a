// me_api.cpp -- C ABI of libme.so: contexts, helicity filter, launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "me_internal.h"

static thread_local std::string g_last_error;

int me_fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

static int fail(int code, const std::string& msg) { return me_fail(code, msg); }

#define HIP_CHECK(expr)                                                                          \
    do {                                                                                         \
        hipError_t _e = (expr);                                                                  \
        if (_e != hipSuccess) return fail(ME_EDEVICE, std::string(#expr ": ") + hipGetErrorString(_e)); \
    } while (0)

// Grow the flagged-event index list to hold nevt entries (synchronises the
// device when it has to reallocate).
static int ensure_scratch(me_ctx* c, int64_t nevt) {
    if (!c->d_count) HIP_CHECK(hipMalloc(&c->d_count, sizeof(int)));
    if (nevt > c->idx_cap) {
        if (c->d_idx) {
            HIP_CHECK(hipDeviceSynchronize());
            HIP_CHECK(hipFree(c->d_idx));
            c->d_idx = nullptr;
        }
        HIP_CHECK(hipMalloc(&c->d_idx, nevt * sizeof(int)));
        c->idx_cap = nevt;
    }
    return ME_OK;
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free mixed evaluation (me_eval_mixed_noalloc):
// a flagged-event counter in the first 256 bytes, then the flagged-event
// index list for up to ME_NOALLOC_MAX_NEVT events (4 MiB + 256 B per device,
// held until the process ends).  Host code never uses the array's name as an
// address: the device address is looked up once per device, with that device
// current, and kept in g_scratch_ptr.
// ---------------------------------------------------------------------------
#define ME_SCRATCH_HEAD 64  // ints before the index list (256 bytes)
static __device__ __align__(256) int scratch[ME_SCRATCH_HEAD + ME_NOALLOC_MAX_NEVT];

static std::mutex g_scratch_mu;
static int* g_scratch_ptr[ME_MAX_DEVICES];
static std::string g_scratch_err[ME_MAX_DEVICES];

// Looks up the current device's copy of `scratch` (once per device).
static void resolve_scratch(int device) {
    if (device < 0 || device >= ME_MAX_DEVICES) return;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return;
    int* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        g_scratch_err[device] = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
        return;
    }
    g_scratch_ptr[device] = ptr;
}

// ---------------------------------------------------------------------------
// Probe points for the helicity filter: flat massless n-body momenta from a
// fixed splitmix64 stream, rescaled to the final-state masses (the RAMBO
// construction of Kleiss, Stirling and Ellis).  Generic points: a helicity
// that vanishes on all of them vanishes identically.
// ---------------------------------------------------------------------------
static double probe_uniform(uint64_t& s) {
    s += 0x9E3779B97F4A7C15ull;
    uint64_t z = s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return ((z >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

static void probe_points(const me_process_desc* pd, double roots, const double* masses, int npts,
                         std::vector<double>& out) {
    const int nf = pd->npart - 2;
    out.assign((size_t)npts * pd->npart * 4, 0.0);
    uint64_t seed = 0x1234567ull;
    for (int e = 0; e < npts; ++e) {
        std::vector<double> q(nf * 4);
        double Q[4] = {0, 0, 0, 0};
        for (int i = 0; i < nf; ++i) {
            double c = 2 * probe_uniform(seed) - 1, ph = 2 * M_PI * probe_uniform(seed);
            double q0 = -std::log(probe_uniform(seed) * probe_uniform(seed));
            double st = std::sqrt(1 - c * c);
            double v[4] = {q0, q0 * st * std::cos(ph), q0 * st * std::sin(ph), q0 * c};
            for (int m = 0; m < 4; ++m) {
                q[4 * i + m] = v[m];
                Q[m] += v[m];
            }
        }
        double M = std::sqrt(Q[0] * Q[0] - Q[1] * Q[1] - Q[2] * Q[2] - Q[3] * Q[3]);
        double b[3] = {-Q[1] / M, -Q[2] / M, -Q[3] / M}, x = roots / M, g = Q[0] / M, a = 1 / (1 + g);
        std::vector<double> p(nf * 4);
        for (int i = 0; i < nf; ++i) {
            double bq = b[0] * q[4 * i + 1] + b[1] * q[4 * i + 2] + b[2] * q[4 * i + 3];
            p[4 * i] = x * (g * q[4 * i] + bq);
            for (int k = 0; k < 3; ++k) p[4 * i + 1 + k] = x * (q[4 * i + 1 + k] + b[k] * q[4 * i] + a * bq * b[k]);
        }
        // rescale 3-momenta so that energies with masses add up to roots
        double xi = 0.9;
        for (int it = 0; it < 100; ++it) {
            double f = -roots, df = 0;
            for (int i = 0; i < nf; ++i) {
                double en = std::sqrt(masses[i] * masses[i] + xi * xi * p[4 * i] * p[4 * i]);
                f += en;
                df += xi * p[4 * i] * p[4 * i] / en;
            }
            xi -= f / df;
        }
        double* o = &out[(size_t)e * pd->npart * 4];
        o[0] = roots / 2;
        o[3] = roots / 2;
        o[4] = roots / 2;
        o[7] = -roots / 2;
        for (int i = 0; i < nf; ++i) {
            double* oi = o + 4 * (2 + i);
            for (int k = 1; k < 4; ++k) oi[k] = xi * p[4 * i + k];
            oi[0] = std::sqrt(masses[i] * masses[i] + oi[1] * oi[1] + oi[2] * oi[2] + oi[3] * oi[3]);
        }
    }
}

static int helicity_filter(me_ctx* c) {
    const me_process_desc* pd = c->proc;
    const int npts = 16;
    std::vector<double> fm(pd->npart - 2, 0.0);
    double roots = 13000.0;
    if (pd->kind == ME_KIND_EE) {
        roots = 500.0;
    } else if (pd->kind == ME_KIND_GG) {
        fm[0] = fm[1] = c->prm.mt;
    }  // quark-line + lepton-pair processes: every final state massless
    std::vector<double> pts;
    probe_points(pd, roots, fm.data(), npts, pts);
    double *d_mom = nullptr, *d_out = nullptr, *d_q = nullptr;
    HIP_CHECK(hipMalloc(&d_mom, pts.size() * sizeof(double)));
    HIP_CHECK(hipMalloc(&d_out, npts * sizeof(double)));
    HIP_CHECK(hipMalloc(&d_q, (size_t)npts * pd->nhel * sizeof(double)));
    HIP_CHECK(hipMemcpy(d_mom, pts.data(), pts.size() * sizeof(double), hipMemcpyHostToDevice));
    HIP_CHECK(pd->launch_f64(d_mom, npts, d_out, c->d_all, pd->nhel, c->prm, d_q, 0, nullptr));
    std::vector<double> q((size_t)npts * pd->nhel);
    HIP_CHECK(hipMemcpy(q.data(), d_q, q.size() * sizeof(double), hipMemcpyDeviceToHost));
    HIP_CHECK(hipFree(d_mom));
    HIP_CHECK(hipFree(d_out));
    HIP_CHECK(hipFree(d_q));
    c->good.clear();
    for (int h = 0; h < pd->nhel; ++h) {
        bool nz = false;
        for (int e = 0; e < npts; ++e) nz |= (q[(size_t)e * pd->nhel + h] != 0.0);
        if (nz) c->good.push_back(h);
    }
    c->nhel_good = (int)c->good.size();
    HIP_CHECK(hipMalloc(&c->d_good, std::max(1, c->nhel_good) * sizeof(int)));
    if (c->nhel_good)
        HIP_CHECK(hipMemcpy(c->d_good, c->good.data(), c->nhel_good * sizeof(int), hipMemcpyHostToDevice));
    return ME_OK;
}

// The float64 launcher of the context's colour form.
// Lanes per event when the caller has not fixed them: the smallest 2^k with
// nevt 2^k >= 2^16 lanes in flight (on g g -> t tbar g g the rate is flat
// from there: 2^10 events at 64 lanes run at 94 % of the 2^20-event rate, at
// one lane at 1.6 %), at most 64 and at most the number of helicities kept,
// and at least the process's own floor: g g -> t tbar g g runs 2^20 events
// about 1 % faster at 8 lanes per event (8 helicities per lane) than at one
// (measured: 44.4 against 44.9 ms; gg -> tt, gg -> ttg and the quark-line
// process gain nothing from more lanes at that size).
static int auto_lanes_lg(int64_t nevt, int nhel, const char* process) {
    int lg = 0;
    while (lg < 6 && (nevt << lg) < (int64_t(1) << 16) && (2 << lg) <= nhel) ++lg;
    const int floor_lg = std::strcmp(process, "gg_ttgg") == 0 ? 3 : 0;
    while (lg < floor_lg && (2 << lg) <= nhel) ++lg;
    return lg;
}

static me_launch_fn f64_launcher(const me_ctx* c) {
    return (c->colour_form == ME_COLOUR_MFMA && c->proc->launch_f64_cm) ? c->proc->launch_f64_cm
                                                                       : c->proc->launch_f64;
}

// The float64 form of me_eval: the context's colour form and lane count.
static hipError_t launch_f64_form(const me_ctx* c, const double* momenta, int64_t nevt, double* out,
                                  hipStream_t s) {
    const int lg = c->hel_lg >= 0 ? c->hel_lg : auto_lanes_lg(nevt, c->nhel_good, c->proc->name);
    return f64_launcher(c)(momenta, nevt, out, c->d_good, c->nhel_good, c->prm, nullptr, lg, s);
}

extern "C" {

int me_init(const char* process, const double* couplings, int n_couplings, const double* masses, int n_masses,
            me_ctx** out_ctx) {
    if (!process || !couplings || !masses || !out_ctx) return fail(ME_EINVAL, "null argument");
    if (n_couplings != 3 || n_masses != 4)
        return fail(ME_EINVAL, "expected 3 couplings {alpha_s, 1/alpha, G_F} and 4 masses {MZ, WZ, MT, WT}");
    const me_process_desc* pd = me_find_process(process);
    if (!pd) return fail(ME_EPROCESS, std::string("unknown process ") + process);
    const double alpha_s = couplings[0], alpha = 1.0 / couplings[1], gf = couplings[2];
    const double mz = masses[0], wz = masses[1], mt = masses[2], wt = masses[3];
    if (!(alpha_s > 0) || !(alpha > 0) || !(gf > 0) || !(mz > 0) || !(wz >= 0) || !(mt >= 0) || !(wt >= 0))
        return fail(ME_EINVAL, "couplings and masses must be positive");
    // M_W from (alpha, G_F, M_Z); then sin^2 theta_W = 1 - M_W^2/M_Z^2.
    const double disc = mz * mz * mz * mz / 4 - M_PI * alpha * mz * mz / (std::sqrt(2.0) * gf);
    if (!(disc > 0)) return fail(ME_EINVAL, "(alpha, G_F, M_Z) admit no real M_W");
    const double mw = std::sqrt(mz * mz / 2 + std::sqrt(disc));
    const double sw2 = 1 - mw * mw / (mz * mz);
    me_ctx* c = new (std::nothrow) me_ctx();
    if (!c) return fail(ME_ENOMEM, "host allocation");
    c->proc = pd;
    c->prm.gs = std::sqrt(4 * M_PI * alpha_s);
    c->prm.mt = mt;
    c->prm.wt = wt;
    c->prm.e = std::sqrt(4 * M_PI * alpha);
    c->prm.gz = c->prm.e / std::sqrt(sw2 * (1 - sw2));
    c->prm.gl = -0.5 + sw2;
    c->prm.gr = sw2;
    c->prm.mz = mz;
    c->prm.wz = wz;
    c->prm.sw2 = sw2;
    c->d_good = nullptr;
    c->d_all = nullptr;
    c->mode = ME_FP64;
    c->hel_lg = -1;  // automatic
    c->colour_form = ME_COLOUR_VALU;
    c->tol = 1e-5;
    c->d_count = nullptr;
    c->d_idx = nullptr;
    c->idx_cap = 0;
    c->uw_x = nullptr;
    c->uw_y = nullptr;
    c->uw_s = nullptr;
    c->uw_me2 = nullptr;
    c->uw_idx1 = nullptr;
    c->uw_cap = 0;
    hipError_t e = hipGetDevice(&c->device);
    if (e != hipSuccess) {
        delete c;
        return fail(ME_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    }
    resolve_scratch(c->device);
    std::vector<int> all(pd->nhel);
    for (int h = 0; h < pd->nhel; ++h) all[h] = h;
    if (hipMalloc(&c->d_all, pd->nhel * sizeof(int)) != hipSuccess ||
        hipMemcpy(c->d_all, all.data(), pd->nhel * sizeof(int), hipMemcpyHostToDevice) != hipSuccess) {
        me_free(c);
        return fail(ME_ENOMEM, "device allocation of the helicity table");
    }
    int rc = helicity_filter(c);
    if (rc != ME_OK) {
        std::string keep = g_last_error;
        me_free(c);
        g_last_error = keep;
        return rc;
    }
    *out_ctx = c;
    return ME_OK;
}

int me_eval(me_ctx* c, const double* momenta, int64_t nevt, double* out_me2, void* stream) {
    if (!c || nevt < 0) return fail(ME_EINVAL, "null context or negative nevt");
    if (nevt == 0) return ME_OK;
    if (!momenta || !out_me2) return fail(ME_EINVAL, "null buffer");
    if (nevt > 0x7fffffffLL) return fail(ME_EINVAL, "nevt above 2^31 - 1");
    hipStream_t s = (hipStream_t)stream;
    if (c->mode == ME_MIXED && c->proc->launch_mixed) {
        int rc = ensure_scratch(c, nevt);
        if (rc != ME_OK) return rc;
        HIP_CHECK(c->proc->launch_mixed(momenta, nevt, out_me2, c->d_good, c->nhel_good, c->prm, (float)c->tol,
                                        (float)c->proc->mixed_cest, c->d_count, c->d_idx, nullptr, nullptr, s));
        // float64 rerun of the flagged events, in place, on the same stream
        HIP_CHECK(c->proc->launch_f64_idx(momenta, nevt, out_me2, c->d_good, c->nhel_good, c->prm, c->d_idx,
                                          c->d_count, s));
        return ME_OK;
    }
    HIP_CHECK(launch_f64_form(c, momenta, nevt, out_me2, s));
    return ME_OK;
}

int me_set_colour_form(me_ctx* c, int form) {
    if (!c) return fail(ME_EINVAL, "null context");
    if (form != ME_COLOUR_VALU && form != ME_COLOUR_MFMA)
        return fail(ME_EINVAL, "form must be ME_COLOUR_VALU or ME_COLOUR_MFMA");
    if (form == ME_COLOUR_MFMA && !c->proc->launch_f64_cm)
        return fail(ME_ESTATE, std::string("no matrix-core colour form for ") + c->proc->name);
    c->colour_form = form;
    return ME_OK;
}

int me_set_helicity_lanes(me_ctx* c, int lanes) {
    if (!c) return fail(ME_EINVAL, "null context");
    if (lanes == 0) {
        c->hel_lg = -1;
        return ME_OK;
    }
    int lg = 0;
    while (lg <= 6 && (1 << lg) != lanes) ++lg;
    if (lg > 6) return fail(ME_EINVAL, "lanes per event must be 0 (automatic), 1, 2, 4, 8, 16, 32 or 64");
    c->hel_lg = lg;
    return ME_OK;
}

int me_eval_mixed_noalloc(me_ctx* c, const double* momenta, int64_t nevt, double* out_me2, void* stream) {
    if (!c || nevt < 0) return fail(ME_EINVAL, "null context or negative nevt");
    if (nevt == 0) return ME_OK;
    if (!momenta || !out_me2) return fail(ME_EINVAL, "null buffer");
    if (nevt > ME_NOALLOC_MAX_NEVT)
        return fail(ME_EINVAL, "nevt above ME_NOALLOC_MAX_NEVT (" + std::to_string(ME_NOALLOC_MAX_NEVT) + ")");
    int dev = -1;
    HIP_CHECK(hipGetDevice(&dev));
    if (dev != c->device) return fail(ME_ESTATE, "the current device is not the context's device");
    hipStream_t s = (hipStream_t)stream;
    if (!c->proc->launch_mixed) {  // no mixed form (e+e- -> mu+mu-): float64 as me_eval, no scratch
        HIP_CHECK(launch_f64_form(c, momenta, nevt, out_me2, s));
        return ME_OK;
    }
    int* base = g_scratch_ptr[dev];
    if (!base) return fail(ME_EDEVICE, g_scratch_err[dev].empty() ? "scratch not resolved" : g_scratch_err[dev]);
    int* d_count = base;
    int* d_idx = base + ME_SCRATCH_HEAD;
    // the mixed launch clears the counter with a kernel before it appends
    HIP_CHECK(c->proc->launch_mixed(momenta, nevt, out_me2, c->d_good, c->nhel_good, c->prm, (float)c->tol,
                                    (float)c->proc->mixed_cest, d_count, d_idx, nullptr, nullptr, s));
    HIP_CHECK(c->proc->launch_f64_idx(momenta, nevt, out_me2, c->d_good, c->nhel_good, c->prm, d_idx, d_count, s));
    return ME_OK;
}

int me_set_precision(me_ctx* c, int mode, double rel_tol) {
    if (!c) return fail(ME_EINVAL, "null context");
    if (mode != ME_FP64 && mode != ME_MIXED) return fail(ME_EINVAL, "mode must be ME_FP64 or ME_MIXED");
    if (mode == ME_MIXED && !(rel_tol > 0)) return fail(ME_EINVAL, "tolerance must be positive");
    c->mode = mode;
    if (mode == ME_MIXED) c->tol = rel_tol;
    return ME_OK;
}

int me_eval_mixed_diag(me_ctx* c, const double* momenta, int64_t nevt, double* out_me2, float* out_err,
                       uint8_t* out_flag, void* stream) {
    if (!c || nevt < 0) return fail(ME_EINVAL, "null context or negative nevt");
    if (!c->proc->launch_mixed) return fail(ME_ESTATE, "the process has no mixed-precision form");
    if (nevt == 0) return ME_OK;
    if (!momenta || !out_me2 || !out_err || !out_flag) return fail(ME_EINVAL, "null buffer");
    if (nevt > 0x7fffffffLL) return fail(ME_EINVAL, "nevt above 2^31 - 1");
    HIP_CHECK(c->proc->launch_mixed(momenta, nevt, out_me2, c->d_good, c->nhel_good, c->prm, (float)c->tol,
                                    (float)c->proc->mixed_cest, nullptr, nullptr, out_err, out_flag,
                                    (hipStream_t)stream));
    return ME_OK;
}

int me_fallback_count(me_ctx* c, int64_t* count) {
    if (!c || !count) return fail(ME_EINVAL, "null argument");
    *count = 0;
    if (!c->d_count) return ME_OK;
    int v = 0;
    // the mixed evaluation may have run on a non-blocking stream, which a copy
    // on the null stream does not wait for
    HIP_CHECK(hipDeviceSynchronize());
    HIP_CHECK(hipMemcpy(&v, c->d_count, sizeof(int), hipMemcpyDeviceToHost));
    *count = v;
    return ME_OK;
}

int me_eval_helicities(me_ctx* c, const double* momenta, int64_t nevt, double* out_me2, double* out_qhel,
                       void* stream) {
    if (!c || nevt < 0) return fail(ME_EINVAL, "null context or negative nevt");
    if (nevt == 0) return ME_OK;
    if (!momenta || !out_me2 || !out_qhel) return fail(ME_EINVAL, "null buffer");
    HIP_CHECK(f64_launcher(c)(momenta, nevt, out_me2, c->d_all, c->proc->nhel, c->prm, out_qhel, 0,
                                  (hipStream_t)stream));
    return ME_OK;
}

int me_info(const me_ctx* c, int* npart, int* ndiag, int* ncol, int* nhel, int* nhel_good, double* flops) {
    if (!c) return fail(ME_EINVAL, "null context");
    const me_process_desc* pd = c->proc;
    if (npart) *npart = pd->npart;
    if (ndiag) *ndiag = pd->ndiag;
    if (ncol) *ncol = pd->ncol;
    if (nhel) *nhel = pd->nhel;
    if (nhel_good) *nhel_good = c->nhel_good;
    if (flops) *flops = c->nhel_good * (pd->flops_amp + pd->flops_colour);
    return ME_OK;
}

int me_channels(const me_ctx* c, int* nchan) {
    if (!c || !nchan) return fail(ME_EINVAL, "null argument");
    *nchan = c->proc->launch_mc ? c->proc->nchan : 0;
    return ME_OK;
}

int me_channel_desc(const me_ctx* c, int chan, char* buf, int buflen) {
    if (!c || !buf || buflen < 1) return fail(ME_EINVAL, "null argument");
    if (!c->proc->launch_mc) return fail(ME_ESTATE, std::string("no multi-channel form for ") + c->proc->name);
    if (chan < 0 || chan >= c->proc->nchan) return fail(ME_EINVAL, "channel out of range");
    const char* d = c->proc->chan_desc[chan];
    const size_t len = std::strlen(d);
    if ((int)len >= buflen) return fail(ME_EINVAL, "buffer too short");
    std::memcpy(buf, d, len + 1);
    return ME_OK;
}

int me_eval_multichannel(me_ctx* c, const double* momenta, const int32_t* chan, int64_t nevt, double* out_me2,
                         double* out_alpha, void* stream) {
    if (!c || nevt < 0) return fail(ME_EINVAL, "null context or negative nevt");
    if (!c->proc->launch_mc) return fail(ME_ESTATE, std::string("no multi-channel form for ") + c->proc->name);
    if (nevt == 0) return ME_OK;
    if (!momenta || !chan || !out_me2 || !out_alpha) return fail(ME_EINVAL, "null buffer");
    if (nevt > 0x7fffffffLL) return fail(ME_EINVAL, "nevt above 2^31 - 1");
    HIP_CHECK(c->proc->launch_mc(momenta, nevt, out_me2, c->d_good, c->nhel_good, c->prm, chan, out_alpha,
                                 (hipStream_t)stream));
    return ME_OK;
}

int me_flops(const me_ctx* c, double* amp_per_hel, double* colour_per_hel, double* executed_per_hel) {
    if (!c) return fail(ME_EINVAL, "null context");
    if (amp_per_hel) *amp_per_hel = c->proc->flops_amp;
    if (colour_per_hel) *colour_per_hel = c->proc->flops_colour;
    if (executed_per_hel) *executed_per_hel = c->proc->flops_executed;
    return ME_OK;
}

int me_good_helicities(const me_ctx* c, int* out, int* count) {
    if (!c || !count) return fail(ME_EINVAL, "null argument");
    *count = c->nhel_good;
    if (out)
        for (int i = 0; i < c->nhel_good; ++i) out[i] = c->good[i];
    return ME_OK;
}

int me_free(me_ctx* c) {
    if (!c) return ME_OK;
    hipError_t e = hipSuccess;
    void* bufs[] = {c->d_good, c->d_all, c->d_count, c->d_idx, c->uw_x, c->uw_y, c->uw_s, c->uw_me2, c->uw_idx1};
    for (void* b : bufs)
        if (b) {
            hipError_t r = hipFree(b);
            if (r != hipSuccess) e = r;
        }
    delete c;
    if (e != hipSuccess) return fail(ME_EDEVICE, std::string("hipFree: ") + hipGetErrorString(e));
    return ME_OK;
}

const char* me_strerror(int status) {
    switch (status) {
        case ME_OK: return "ok";
        case ME_EINVAL: return "invalid argument";
        case ME_EPROCESS: return "unknown process";
        case ME_EDEVICE: return "HIP runtime error";
        case ME_ENOMEM: return "out of memory";
        case ME_ESTATE: return "invalid state";
        default: return "unknown status";
    }
}

const char* me_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
