// Host side of the C ABI declared in include/kgs.h: validation, the
// per-half-step constants of the explicit point updates, device memory, and
// the order of kernel launches of a DP-AVF2 step.
//
// Compiled by the host compiler (it uses binary128 for one constant), linked
// with the HIP kernels into libkgs.so.
#include "kgs.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <utility>
#include <string>

#include <hip/hip_runtime_api.h>

#include "kgs_trace.h"
#include "kgs_energy.h"
#include "kgs_internal.h"
#include "kgs_plan.h"
#include "kgs_sim.h"



namespace {

// Longest run of steps in one resident launch (longer runs are split; the
// result does not depend on the split).
constexpr int64_t kResidentRun = 1 << 16;

thread_local std::string g_err;

int fail(kgs_sim *s, int code, const std::string &msg)
{
    if (s)
        s->err = msg;
    else
        g_err = msg;
    return code;
}

int hip_fail(kgs_sim *s, hipError_t e, const char *what)
{
    std::string msg = std::string(what) + ": " + hipGetErrorName(e) + " (" +
                      hipGetErrorString(e) + ")";
    return fail(s, e == hipErrorOutOfMemory ? KGS_ENOMEM : KGS_EDEVICE, msg);
}

bool finite(double x) { return std::isfinite(x); }

size_t elem_bytes(int precision) { return precision == KGS_FP32 ? 4 : 8; }

// Half-step constants.  The expressions (and their evaluation order) state
// the coefficients of the explicit scheme of sec. 4.1 with tau replaced by the
// half step tau' = tau/2 and the 2-D "4" by 2*dim.
kgs::Coef half_step_coef(const kgs_config &c, double h)
{
    const double tau = c.tau / 2.0;
    kgs::Coef k;
    k.b = tau * c.kappa1 / (2.0 * h * h);
    k.a = static_cast<double>(c.dim) * k.b;
    k.e = tau * c.gamma / 2.0;
    k.s = tau * c.kappa2 / (h * h);
    k.beta = static_cast<double>(c.dim) * tau * c.kappa2 / (h * h) + tau * c.mu * c.mu / 2.0;
    k.t2 = tau / 2.0;
    k.g = tau * c.gamma;
    // det of [[1, -t2], [beta, 1]] and its reciprocal to ~1e-32 relative
    const __float128 det = static_cast<__float128>(1.0) +
                           static_cast<__float128>(k.beta) * static_cast<__float128>(k.t2);
    const __float128 inv = static_cast<__float128>(1.0) / det;
    k.rd_hi = static_cast<double>(inv);
    k.rd_lo = static_cast<double>(inv - static_cast<__float128>(k.rd_hi));
    return k;
}

int validate(const kgs_config *c, std::string &msg)
{
    if (!c) {
        msg = "config is NULL";
        return KGS_EINVAL;
    }
    if (c->dim < 1 || c->dim > 3) {
        msg = "dim must be 1, 2 or 3";
        return KGS_EINVAL;
    }
    if (c->n < 2) {
        msg = "n must be >= 2";
        return KGS_EINVAL;
    }
    if (c->n % 2) {
        msg = "n must be even: with periodic wrap an odd n makes two same-colour points "
              "neighbours";
        return KGS_EODDN;
    }
    if (!finite(c->lo) || !finite(c->hi) || !(c->hi > c->lo)) {
        msg = "the box [lo, hi) must be finite with hi > lo";
        return KGS_EINVAL;
    }
    if (!finite(c->tau) || c->tau == 0.0) {
        msg = "tau must be finite and non-zero";
        return KGS_EINVAL;
    }
    if (!finite(c->kappa1) || !finite(c->kappa2) || !finite(c->mu) || !finite(c->gamma)) {
        msg = "kappa1, kappa2, mu and gamma must be finite";
        return KGS_EINVAL;
    }
    if (c->precision != KGS_FP64 && c->precision != KGS_FP32) {
        msg = "precision must be KGS_FP64 or KGS_FP32";
        return KGS_EINVAL;
    }
    if (c->reserved != 0) {
        msg = "reserved must be 0";
        return KGS_EINVAL;
    }
    // n^dim must be representable with room to spare for byte counts
    double pts = 1.0;
    for (int a = 0; a < c->dim; ++a) pts *= c->n;
    if (pts > 4.0e12) {
        msg = "grid too large";
        return KGS_EINVAL;
    }
    const double h = (c->hi - c->lo) / c->n;
    if (!finite(h) || h <= 0.0) {
        msg = "grid spacing is not a positive finite number";
        return KGS_EINVAL;
    }
    const kgs::Coef k = half_step_coef(*c, h);
    const double det = 1.0 + k.beta * k.t2;
    if (!finite(k.b) || !finite(k.a) || !finite(k.s) || !finite(k.beta) || !finite(k.g) ||
        !finite(k.e)) {
        msg = "a coefficient of the point update is not finite";
        return KGS_EINVAL;
    }
    if (det == 0.0 || !finite(k.rd_hi) || !finite(k.rd_lo) || !finite(det)) {
        msg = "the 2x2 (u, v) matrix [[1, -tau/4], [beta, 1]] is singular";
        return KGS_ESINGULAR;
    }
    return KGS_OK;
}

kgs::Geometry make_geometry(const kgs_config &c)
{
    kgs::Geometry g;
    g.dim = c.dim;
    g.n = c.n;
    g.half = c.n / 2;
    g.rows = 1;
    for (int a = 1; a < c.dim; ++a) g.rows *= c.n;
    g.count = g.rows * g.half;
    g.stride = (g.count + 63) / 64 * 64;  // 256-byte aligned planes in float32
    return g;
}

// Library default for a grid, from measurements on MI355X (the branches
// below, in order):
//  * the resident kernel when the grid fits one workgroup (small grids are
//    bound by launch latency otherwise);
//  * 2-D grids below n = 2048: the tiled kernel, 8x8 tiles with 2 steps per
//    launch below n = 512, else 4 steps per launch with 16x16 tiles below
//    n = 1024 and 16x32 (float64) or 32x32 (float32) from there;
//  * 2-D float64 grids from n = 2048: 16x32 tiles, 4 steps per launch;
//  * 2-D float32 grids from n = 2048: the y-streaming kernel, 2 steps per
//    launch, the longest row chunk (8..64) that still gives 8192 waves;
//  * 3-D grids with n >= 96: the z-streaming kernel with two steps per
//    launch and the tile and chunk of z-planes (8..128) that stream3d_plan
//    estimates to end the launch first on this device (the CUs take one
//    workgroup each, so the items should fill whole rounds of them):
//    float64 16x16 tiles or, where they end sooner, 12-wave 32x13 tiles;
//    float32 16x32 tiles from n = 128 (13 waves per workgroup: 17-24%
//    faster than 16x16 at n = 192..512, 3-6% at 128, 30% slower at 96
//    where 16x32 tiles leave most CUs idle);
//  * one colour sweep per launch otherwise (3-D below n = 96, 1-D grids
//    beyond the resident kernel).
kgs_tuning default_tuning(const kgs_config &c, bool with_chunk = true)
{
    kgs_tuning t;
    std::memset(&t, 0, sizeof(t));
    t.kernel = KGS_KERNEL_SWEEP;
    t.block = 256;
    t.tile_x = 16;
    t.tile_y = 16;
    t.chunk = 128;
    t.steps_per_launch = 2;
    const kgs::Geometry g = make_geometry(c);
    if (kgs::resident_fits(g.count, static_cast<int>(elem_bytes(c.precision)))) {
        t.kernel = KGS_KERNEL_RESIDENT;
    } else if (c.dim == 2 && c.n < 2048) {
        // tiles in LDS: 1.5-3x the sweeps below n = 1024 and 1.2x at 1024
        // (measured on MI355X); rows x points of one colour, and 4 steps
        // per launch from n = 512 (5-13% faster than 2 there)
        t.kernel = KGS_KERNEL_TILE;
        if (c.n < 512) {
            t.tile_y = 8;
            t.tile_x = 8;
        } else if (c.n < 1024) {
            t.tile_y = 16;
            t.tile_x = 16;
            t.steps_per_launch = 4;
        } else {
            t.tile_y = c.precision == KGS_FP32 ? 32 : 16;
            t.tile_x = 32;
            t.steps_per_launch = 4;
        }
    } else if (c.dim == 2 && c.precision == KGS_FP64) {
        // long float64 grids: 16 x 32 tiles, 4 steps per launch (measured
        // on MI355X: 1.39e11 against 1.20e11 updates/s streaming along y at
        // 2048^2, 1.43e11 against 1.16e11 at 4096^2)
        t.kernel = KGS_KERNEL_TILE;
        t.tile_y = 16;
        t.tile_x = 32;
        t.steps_per_launch = 4;
    } else if (c.dim == 2) {
        // long float32 grids stream along y (1.61e11 against 1.54e11 updates/s
        // with tiles at 2048^2, 2.10e11 against 1.64e11 at 4096^2): a chunk
        // that still gives about 8192 waves
        t.kernel = KGS_KERNEL_STREAM;
        t.chunk = 64;
        while (t.chunk > 8 && kgs::stream2d_tasks(c.n, t.chunk) < 8192) t.chunk /= 2;
    } else if (c.dim == 3 && c.n >= 96) {
        t.kernel = KGS_KERNEL_STREAM;
        if (with_chunk)
            kgs::stream3d_plan(c.n, static_cast<int>(elem_bytes(c.precision)), kgs::device_cus(),
                               &t.tile_x, &t.tile_y, &t.chunk);
    }
    return t;
}

int64_t bytes_for(const kgs_config &c)
{
    const kgs::Geometry g = make_geometry(c);
    const int64_t state = 8 * g.stride * static_cast<int64_t>(elem_bytes(c.precision));
    const int64_t partials = (2 * kgs::energy_partial_slots() + 2) * 8;
    const int dk = default_tuning(c, false).kernel;
    const bool pingpong = dk == KGS_KERNEL_STREAM || dk == KGS_KERNEL_TILE;
    return state * (pingpong ? 2 : 1) + partials;
}

kgs::StreamShape stream_shape(const kgs_sim *s)
{
    kgs::StreamShape sh;
    sh.tile_x = s->tuning.tile_x;
    sh.tile_y = s->tuning.tile_y;
    sh.chunk = s->tuning.chunk;
    sh.steps = s->tuning.steps_per_launch;
    return sh;
}

int check_device(kgs_sim *s)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(s, e, "hipGetDevice");
    if (dev != s->device) {
        e = hipSetDevice(s->device);
        if (e != hipSuccess) return hip_fail(s, e, "hipSetDevice");
    }
    return KGS_OK;
}

// Frees device memory and returns the runtime's status; a NULL pointer is
// a no-op.  Callers on an error path ignore the status (the first error is
// the one reported); kgs_free reports it.
hipError_t free_device(void *p)
{
    return p ? hipFree(p) : hipSuccess;
}

// Device allocation of a handle: from its pool in stream order, or plain.
hipError_t alloc_device(kgs_sim *s, void **p, size_t bytes)
{
    if (s->pool) return hipMallocFromPoolAsync(p, bytes, s->pool, s->stream);
    return hipMalloc(p, bytes);
}

hipError_t free_handle_memory(kgs_sim *s, void *p)
{
    if (!p) return hipSuccess;
    return s->pool ? hipFreeAsync(p, s->stream) : free_device(p);
}

// Releases everything a handle holds on the device and in pinned host
// memory, and returns the first error of the runtime (every release is
// attempted regardless).
hipError_t release(kgs_sim *s)
{
    if (!s) return hipSuccess;
    kgs::FirstError err;
    err(free_handle_memory(s, s->state));
    err(free_handle_memory(s, s->state2));
    err(free_handle_memory(s, s->partials));
    if (s->host_out) err(hipHostFree(s->host_out));
    s->state = s->state2 = nullptr;
    s->partials = nullptr;
    s->host_out = nullptr;
    return err.e;
}

// Copy four float64 boundary arrays into the colour-split state.
int load_state(kgs_sim *s, const double *P, const double *Q, const double *U, const double *V,
               int32_t mem)
{
    if (!P || !Q || !U || !V) return fail(s, KGS_EINVAL, "state array pointer is NULL");
    if (mem != KGS_HOST && mem != KGS_DEVICE)
        return fail(s, KGS_EINVAL, "mem must be KGS_HOST or KGS_DEVICE");
    const int64_t npts = 2 * s->geo.count;
    const size_t bytes = static_cast<size_t>(npts) * sizeof(double);
    hipError_t e;
    s->open = false;  // the state is replaced
    if (mem == KGS_DEVICE) {
        e = kgs::launch_scatter(s->geo, s->cfg.precision, s->state, P, Q, U, V, s->stream);
        if (e != hipSuccess) return hip_fail(s, e, "scatter kernel");
        e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) return hip_fail(s, e, "hipStreamSynchronize");
        return KGS_OK;
    }
    double *stage = nullptr;
    e = hipMalloc(&stage, 4 * bytes);
    if (e != hipSuccess) return hip_fail(s, e, "hipMalloc (staging)");
    const double *src[4] = {P, Q, U, V};
    for (int f = 0; f < 4 && e == hipSuccess; ++f)
        e = hipMemcpyAsync(stage + f * npts, src[f], bytes, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess)
        e = kgs::launch_scatter(s->geo, s->cfg.precision, s->state, stage, stage + npts,
                                stage + 2 * npts, stage + 3 * npts, s->stream);
    hipError_t e2 = hipStreamSynchronize(s->stream);
    const hipError_t e3 = free_device(stage);
    if (e != hipSuccess) return hip_fail(s, e, "copy-in / scatter");
    if (e2 != hipSuccess) return hip_fail(s, e2, "hipStreamSynchronize");
    if (e3 != hipSuccess) return hip_fail(s, e3, "hipFree (staging)");
    return KGS_OK;
}

// A handle for a validated cfg: constants, device memory for the state and
// the energy partials (from `pool` in stream order when pool != NULL), the
// padding between planes cleared on the stream.  On failure sets g_err.
int new_handle(const kgs_config *cfg, hipStream_t stream, hipMemPool_t pool, kgs_sim **out)
{
    kgs_sim *s = new (std::nothrow) kgs_sim();
    if (!s) return fail(nullptr, KGS_ENOMEM, "host allocation failed");
    s->cfg = *cfg;
    s->geo = make_geometry(*cfg);
    s->h = (cfg->hi - cfg->lo) / cfg->n;
    s->hd = 1.0;
    for (int a = 0; a < cfg->dim; ++a) s->hd *= s->h;
    s->coef = half_step_coef(*cfg, s->h);
    s->ecoef.k1_h2 = cfg->kappa1 / (s->h * s->h);
    s->ecoef.k2_h2 = cfg->kappa2 / (s->h * s->h);
    s->ecoef.mu2 = cfg->mu * cfg->mu;
    s->ecoef.gamma = cfg->gamma;
    s->stream = stream;
    s->pool = pool;
    std::memset(&s->tuning, 0, sizeof(s->tuning));
    s->tuning.kernel = KGS_KERNEL_SWEEP;
    s->tuning.block = 256;

    hipError_t e = hipGetDevice(&s->device);
    if (e != hipSuccess) {
        hip_fail(s, e, "hipGetDevice");
        g_err = s->err;
        delete s;
        return KGS_EDEVICE;
    }
    s->plane_bytes = static_cast<size_t>(s->geo.stride) * elem_bytes(cfg->precision);
    const size_t partial_bytes = (2 * kgs::energy_partial_slots() + 2) * sizeof(double);
    int code = KGS_OK;
    e = alloc_device(s, &s->state, 8 * s->plane_bytes);
    if (e != hipSuccess) code = hip_fail(s, e, "device allocation (state)");
    if (code == KGS_OK) {
        e = alloc_device(s, reinterpret_cast<void **>(&s->partials), partial_bytes);
        if (e != hipSuccess) code = hip_fail(s, e, "device allocation (energy partials)");
    }
    if (code == KGS_OK && !pool) {
        e = hipHostMalloc(reinterpret_cast<void **>(&s->host_out), 2 * sizeof(double),
                          hipHostMallocDefault);
        if (e != hipSuccess) code = hip_fail(s, e, "hipHostMalloc");
    }
    if (code == KGS_OK) {
        // padding between planes is never read by a kernel; clear it anyway
        e = hipMemsetAsync(s->state, 0, 8 * s->plane_bytes, s->stream);
        if (e != hipSuccess) code = hip_fail(s, e, "hipMemsetAsync");
    }
    if (code != KGS_OK) {
        g_err = s->err;
        (void)release(s);  // the first error is the one reported
        delete s;
        return code;
    }
    s->device_bytes = static_cast<int64_t>(8 * s->plane_bytes + partial_bytes);
    *out = s;
    return KGS_OK;
}

// The library's default launch configuration for the handle's grid (the
// sweep kernel stays if the default shape does not fit).
void apply_default_tuning(kgs_sim *s)
{
    const kgs_tuning dt = default_tuning(s->cfg);
    if (dt.kernel != KGS_KERNEL_SWEEP) {
        if (kgs_set_tuning(s, &dt) != KGS_OK) s->err.clear();
    }
}

// Checks a requested launch configuration against the handle's grid and
// fills in what KGS_KERNEL_AUTO leaves open.  `pingpong` tells whether the
// configuration needs the second state buffer.  Allocates nothing.
int resolve_tuning(kgs_sim *s, const kgs_tuning &t, kgs_tuning &nt, bool &pingpong)
{
    nt = t;
    pingpong = false;
    if (nt.reserved[0] || nt.reserved[1]) return fail(s, KGS_EINVAL, "reserved must be 0");
    if (nt.kernel == KGS_KERNEL_AUTO) {
        const kgs_tuning dt = default_tuning(s->cfg);
        nt.kernel = dt.kernel;
        if (nt.tile_x == 0 && nt.tile_y == 0 && nt.chunk == 0 && nt.steps_per_launch == 0) {
            nt.tile_x = dt.tile_x;
            nt.tile_y = dt.tile_y;
            nt.chunk = dt.chunk;
            nt.steps_per_launch = dt.steps_per_launch;
        }
    }
    if (nt.block == 0) nt.block = 256;
    if (nt.block < 64 || nt.block > 1024 || nt.block % 64)
        return fail(s, KGS_EINVAL, "block must be a multiple of 64 in [64, 1024]");
    if (nt.kernel == KGS_KERNEL_STREAM) {
        if (s->cfg.dim == 1) return fail(s, KGS_EINVAL, "the streaming kernels are 2-D and 3-D");
        if (s->cfg.dim == 2) {
            if ((nt.steps_per_launch != 1 && nt.steps_per_launch != 2) || nt.chunk < 1 ||
                kgs::stream2d_tasks(s->geo.n, nt.chunk) < 1)
                return fail(s, KGS_EINVAL, "chunk/steps do not fit the 2-D streaming kernel");
        } else {
            kgs::StreamShape sh = {nt.tile_x, nt.tile_y, nt.chunk, nt.steps_per_launch};
            if (!kgs::stream3d_shape_ok(s->geo, sh, static_cast<int>(elem_bytes(s->cfg.precision))))
                return fail(s, KGS_EINVAL, "tile/chunk/steps do not fit the streaming kernel");
        }
        pingpong = true;
    } else if (nt.kernel == KGS_KERNEL_TILE) {
        if (s->cfg.dim != 2) return fail(s, KGS_EINVAL, "the tiled kernel is 2-D");
        if ((nt.steps_per_launch != 1 && nt.steps_per_launch != 2 && nt.steps_per_launch != 4) ||
            !kgs::tile2d_shape_ok(s->geo, nt.tile_y, nt.tile_x, 2 * nt.steps_per_launch,
                                  static_cast<int>(elem_bytes(s->cfg.precision))))
            return fail(s, KGS_EINVAL, "tile/steps do not fit the 2-D tiled kernel");
        pingpong = true;
    } else if (nt.kernel == KGS_KERNEL_RESIDENT) {
        if (!kgs::resident_fits(s->geo.count, static_cast<int>(elem_bytes(s->cfg.precision))))
            return fail(s, KGS_EINVAL, "the grid does not fit the resident kernel");
    } else if (nt.kernel != KGS_KERNEL_SWEEP) {
        return fail(s, KGS_EINVAL, "kernel family not available for this grid");
    }
    return KGS_OK;
}

}  // namespace

namespace kgs {

int sim_create_pooled(const kgs_config *cfg, const double *P, const double *Q, const double *U,
                      const double *V, hipStream_t stream, hipMemPool_t pool, kgs_sim **out,
                      std::string &err)
{
    *out = nullptr;
    std::string msg;
    int rc = validate(cfg, msg);
    if (rc != KGS_OK) {
        err = msg;
        return rc;
    }
    if (!P || !Q || !U || !V || !pool) {
        err = "NULL input or pool";
        return KGS_EINVAL;
    }
    kgs_sim *s = nullptr;
    rc = new_handle(cfg, stream, pool, &s);
    if (rc != KGS_OK) {
        err = g_err;
        return rc;
    }
    const hipError_t e = launch_scatter(s->geo, cfg->precision, s->state, P, Q, U, V, stream);
    if (e != hipSuccess) {
        rc = hip_fail(s, e, "scatter kernel");
        err = s->err;
        (void)release(s);  // the first error is the one reported
        delete s;
        return rc;
    }
    apply_default_tuning(s);
    *out = s;
    return KGS_OK;
}

int default_kernel(const kgs_config &cfg) { return default_tuning(cfg, false).kernel; }

int sim_close(kgs_sim *s, hipStream_t stream)
{
    if (!s->open) return KGS_OK;
    const int block = s->tuning.block > 0 ? s->tuning.block : 256;
    const hipError_t e =
        launch_sweep(s->geo, s->cfg.precision, s->state, PASS_R_ADJ, s->coef, block, stream);
    if (e != hipSuccess) return hip_fail(s, e, "closing sweep launch");
    s->open = false;
    return KGS_OK;
}

kgs_tuning default_tuning_of(const kgs_config &cfg) { return default_tuning(cfg); }

int64_t state_bytes(const kgs_config &cfg)
{
    return 8 * make_geometry(cfg).stride * static_cast<int64_t>(elem_bytes(cfg.precision));
}

int sim_ensure_state2(kgs_sim *s)
{
    if (s->state2) return KGS_OK;
    int rc = check_device(s);
    if (rc != KGS_OK) return rc;
    hipError_t e = alloc_device(s, &s->state2, 8 * s->plane_bytes);
    if (e != hipSuccess) {
        s->state2 = nullptr;
        return hip_fail(s, e, "device allocation (second state buffer)");
    }
    s->device_bytes += static_cast<int64_t>(8 * s->plane_bytes);
    return KGS_OK;
}

void sim_destroy_pooled(kgs_sim *s)
{
    if (!s) return;
    (void)release(s);  // a server's clean-up: no caller to report to
    delete s;
}

int set_error(int code, const std::string &msg) { return fail(nullptr, code, msg); }

int step_fields_check(const kgs_config *cfg, const double *P, const double *Q, const double *U,
                      const double *V, int64_t nsteps, int64_t scratch_bytes)
{
    std::string msg;
    const int rc = validate(cfg, msg);
    if (rc != KGS_OK) return fail(nullptr, rc, msg);
    if (!P || !Q || !U || !V) return fail(nullptr, KGS_EINVAL, "state array pointer is NULL");
    if (nsteps < 0) return fail(nullptr, KGS_EINVAL, "nsteps must be >= 0");
    const int64_t need = state_bytes(*cfg);
    if (need > scratch_bytes)
        return fail(nullptr, KGS_ENOMEM,
                    "the grid's state needs " + std::to_string(need) +
                        " bytes of device memory; kgs_step_fields has a fixed scratch area of " +
                        std::to_string(scratch_bytes) + " bytes per device");
    return KGS_OK;
}

int step_fields_run(const kgs_config *cfg, double *P, double *Q, double *U, double *V,
                    int64_t nsteps, hipStream_t stream, void *scratch, int64_t scratch_bytes)
{
    // a handle on the stack whose state lives in the scratch area: the
    // kernels and the launch sequence are those of kgs_step
    kgs_sim s;
    s.cfg = *cfg;
    s.geo = make_geometry(*cfg);
    s.h = (cfg->hi - cfg->lo) / cfg->n;
    s.hd = 1.0;
    for (int a = 0; a < cfg->dim; ++a) s.hd *= s.h;
    s.coef = half_step_coef(*cfg, s.h);
    s.stream = stream;
    s.plane_bytes = static_cast<size_t>(s.geo.stride) * elem_bytes(cfg->precision);
    const int64_t sb = state_bytes(*cfg);
    s.state = scratch;
    if (2 * sb <= scratch_bytes) s.state2 = static_cast<char *>(scratch) + sb;
    hipError_t e = hipGetDevice(&s.device);
    if (e != hipSuccess) return set_error(hip_fail(&s, e, "hipGetDevice"), s.err);
    // the library's default launch configuration, unless it needs a second
    // state buffer that the scratch area cannot hold
    kgs_tuning req;
    std::memset(&req, 0, sizeof(req));
    req.kernel = KGS_KERNEL_AUTO;
    bool pingpong = false;
    int rc = resolve_tuning(&s, req, s.tuning, pingpong);
    if (rc != KGS_OK || (pingpong && !s.state2)) {
        std::memset(&s.tuning, 0, sizeof(s.tuning));
        s.tuning.block = 256;
        s.tuning.kernel = kgs::resident_fits(s.geo.count, static_cast<int>(elem_bytes(cfg->precision)))
                              ? KGS_KERNEL_RESIDENT
                              : KGS_KERNEL_SWEEP;
    }
    e = kgs::launch_scatter(s.geo, cfg->precision, s.state, P, Q, U, V, stream);
    if (e != hipSuccess) return set_error(hip_fail(&s, e, "scatter kernel"), s.err);
    rc = kgs_step(&s, nsteps);
    if (rc == KGS_OK) rc = sim_close(&s, stream);
    if (rc != KGS_OK) return set_error(rc, s.err);
    e = kgs::launch_gather(s.geo, cfg->precision, s.state, P, Q, U, V, stream);
    if (e != hipSuccess) return set_error(hip_fail(&s, e, "gather kernel"), s.err);
    return KGS_OK;
}

}  // namespace kgs

extern "C" {

const char *kgs_status_string(int status)
{
    switch (status) {
    case KGS_OK: return "KGS_OK";
    case KGS_EINVAL: return "KGS_EINVAL";
    case KGS_EODDN: return "KGS_EODDN";
    case KGS_ESINGULAR: return "KGS_ESINGULAR";
    case KGS_ENOMEM: return "KGS_ENOMEM";
    case KGS_EDEVICE: return "KGS_EDEVICE";
    case KGS_ENONFINITE: return "KGS_ENONFINITE";
    default: return "KGS_UNKNOWN";
    }
}

const char *kgs_last_error(const kgs_sim *sim)
{
    return sim ? sim->err.c_str() : g_err.c_str();
}

int64_t kgs_required_bytes(const kgs_config *cfg)
{
    std::string msg;
    if (validate(cfg, msg) != KGS_OK) return 0;
    return bytes_for(*cfg);
}

int kgs_init(const kgs_config *cfg, const double *psi_re, const double *psi_im, const double *u,
             const double *v_t, int32_t mem, void *stream, kgs_sim **out)
{
    KGS_TRACE("kgs_init");
    if (!out) return fail(nullptr, KGS_EINVAL, "out is NULL");
    *out = nullptr;
    std::string msg;
    const int rc = validate(cfg, msg);
    if (rc != KGS_OK) return fail(nullptr, rc, msg);
    if (!psi_re || !psi_im || !u || !v_t)
        return fail(nullptr, KGS_EINVAL, "state array pointer is NULL");
    if (mem != KGS_HOST && mem != KGS_DEVICE)
        return fail(nullptr, KGS_EINVAL, "mem must be KGS_HOST or KGS_DEVICE");

    kgs_sim *s = nullptr;
    int code = new_handle(cfg, static_cast<hipStream_t>(stream), nullptr, &s);
    if (code != KGS_OK) return code;
    code = load_state(s, psi_re, psi_im, u, v_t, mem);
    if (code != KGS_OK) {
        g_err = s->err;
        (void)release(s);  // the first error is the one reported
        delete s;
        return code;
    }
    apply_default_tuning(s);
    *out = s;
    return KGS_OK;
}

int kgs_step(kgs_sim *s, int64_t nsteps)
{
    KGS_TRACE("kgs_step");
    if (!s) return fail(nullptr, KGS_EINVAL, "handle is NULL");
    if (nsteps < 0) return fail(s, KGS_EINVAL, "nsteps must be >= 0");
    if (nsteps == 0) return KGS_OK;
    int rc = check_device(s);
    if (rc != KGS_OK) return rc;
    const int prec = s->cfg.precision;
    const int block = s->tuning.block > 0 ? s->tuning.block : 256;
    auto sweep = [&](int kind) {
        hipError_t e = kgs::launch_sweep(s->geo, prec, s->state, kind, s->coef, block, s->stream);
        return e == hipSuccess ? KGS_OK : hip_fail(s, e, "sweep kernel launch");
    };
    if (s->tuning.kernel == KGS_KERNEL_RESIDENT) {
        // one launch per run of at most kResidentRun steps, each closing its
        // last step
        if ((rc = kgs::sim_close(s, s->stream)) != KGS_OK) return rc;
        kgs::ResidentMember m;
        std::memset(&m, 0, sizeof(m));
        m.state = s->state;
        m.stride = s->geo.stride;
        m.k = s->coef;
        m.n = s->geo.n;
        m.count = static_cast<int>(s->geo.count);
        for (int64_t left = nsteps; left > 0;) {
            m.steps = std::min<int64_t>(left, kResidentRun);
            hipError_t e = kgs::launch_resident(s->cfg.dim, prec, m, nullptr, nullptr, 0, 1,
                                                s->geo.count, s->stream);
            if (e != hipSuccess) return hip_fail(s, e, "resident kernel launch");
            left -= m.steps;
        }
        return KGS_OK;
    }
    if (s->tuning.kernel == KGS_KERNEL_STREAM || s->tuning.kernel == KGS_KERNEL_TILE) {
        // launches of 1 or 2 full steps (R, B[, R, B]) from one buffer to the
        // other; a pending adjoint red sweep of the previous call fuses with
        // the first red sweep (R_ADJ_BASE instead of R_BASE), and the one
        // that closes this call's last step is left pending
        const kgs::StreamShape sh = stream_shape(s);
        bool first = !s->open;
        for (int64_t left = nsteps; left > 0 && rc == KGS_OK;) {
            // steps of this launch: steps_per_launch while they last, then 2
            // or 1 (the tiled kernel takes 1, 2 or 4 per launch)
            const int st = left >= sh.steps ? sh.steps : left >= 2 ? 2 : 1;
            hipError_t e;
            if (s->tuning.kernel == KGS_KERNEL_TILE) {
                e = kgs::launch_tile2d(s->geo, prec, 2 * st, s->tuning.tile_y, s->tuning.tile_x,
                                       s->state, s->state2, first, s->coef, s->stream);
            } else if (s->cfg.dim == 2) {
                kgs::Stream2dMember m;
                std::memset(&m, 0, sizeof(m));
                m.in = s->state;
                m.out = s->state2;
                m.stride = s->geo.stride;
                m.k = s->coef;
                m.n = s->geo.n;
                m.chunk = sh.chunk;
                m.tiles_x = kgs::stream2d_tiles_x(s->geo.n);
                m.first = first ? 1 : 0;
                e = kgs::launch_stream2d(prec, 2 * st, m, nullptr, 1,
                                         kgs::stream2d_tasks(s->geo.n, sh.chunk), s->stream);
            } else {
                e = kgs::launch_stream3d(s->geo, prec, sh, 2 * st, s->state, s->state2, first,
                                         s->coef, s->stream);
            }
            if (e != hipSuccess) return hip_fail(s, e, "stream kernel launch");
            std::swap(s->state, s->state2);
            first = false;
            s->open = true;
            left -= st;
        }
        return KGS_OK;
    }
    // one colour sweep per launch, with the same pending closing sweep
    rc = sweep(s->open ? kgs::PASS_R_ADJ_BASE : kgs::PASS_R_BASE);
    for (int64_t i = 1; i < nsteps && rc == KGS_OK; ++i) {
        rc = sweep(kgs::PASS_B_FULL);
        if (rc == KGS_OK) rc = sweep(kgs::PASS_R_ADJ_BASE);
    }
    if (rc == KGS_OK) rc = sweep(kgs::PASS_B_FULL);
    if (rc == KGS_OK) s->open = true;
    return rc;
}

int kgs_energy(kgs_sim *s, double *energy)
{
    KGS_TRACE("kgs_energy");
    if (!s || !energy) return fail(s, KGS_EINVAL, "handle or output is NULL");
    if (!s->host_out) return fail(s, KGS_EINVAL, "handle belongs to a server");
    int rc = check_device(s);
    if (rc != KGS_OK) return rc;
    double *out = s->partials + 2 * kgs::energy_partial_slots();
    hipError_t e = hipErrorNotSupported;
    if (s->open) {
        // the pending closing sweep and the energy in one pass
        e = kgs::launch_energy_closing(s->geo, s->cfg.precision, s->state, s->ecoef, s->coef,
                                       s->partials, out, s->stream);
        if (e == hipSuccess) s->open = false;
        else if (e != hipErrorNotSupported) return hip_fail(s, e, "energy kernel launch");
    }
    if (e == hipErrorNotSupported) {
        if ((rc = kgs::sim_close(s, s->stream)) != KGS_OK) return rc;
        e = kgs::launch_energy(s->geo, s->cfg.precision, s->state, s->ecoef, s->partials, out,
                               s->stream);
        if (e != hipSuccess) return hip_fail(s, e, "energy kernel launch");
    }
    e = hipMemcpyAsync(s->host_out, out, 2 * sizeof(double), hipMemcpyDeviceToHost, s->stream);
    if (e != hipSuccess) return hip_fail(s, e, "hipMemcpyAsync (energy)");
    e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(s, e, "hipStreamSynchronize");
    *energy = s->hd * (s->host_out[0] + s->host_out[1]);
    if (!std::isfinite(*energy)) return fail(s, KGS_ENONFINITE, "energy is not finite");
    return KGS_OK;
}

int kgs_read_state(kgs_sim *s, double *P, double *Q, double *U, double *V, int32_t mem)
{
    KGS_TRACE("kgs_read_state");
    if (!s) return fail(nullptr, KGS_EINVAL, "handle is NULL");
    if (!P || !Q || !U || !V) return fail(s, KGS_EINVAL, "state array pointer is NULL");
    if (mem != KGS_HOST && mem != KGS_DEVICE)
        return fail(s, KGS_EINVAL, "mem must be KGS_HOST or KGS_DEVICE");
    int rc = check_device(s);
    if (rc == KGS_OK) rc = kgs::sim_close(s, s->stream);
    if (rc != KGS_OK) return rc;
    const int64_t npts = 2 * s->geo.count;
    const size_t bytes = static_cast<size_t>(npts) * sizeof(double);
    hipError_t e;
    if (mem == KGS_DEVICE) {
        e = kgs::launch_gather(s->geo, s->cfg.precision, s->state, P, Q, U, V, s->stream);
        if (e != hipSuccess) return hip_fail(s, e, "gather kernel");
        e = hipStreamSynchronize(s->stream);
        return e == hipSuccess ? KGS_OK : hip_fail(s, e, "hipStreamSynchronize");
    }
    double *stage = nullptr;
    e = hipMalloc(&stage, 4 * bytes);
    if (e != hipSuccess) return hip_fail(s, e, "hipMalloc (staging)");
    e = kgs::launch_gather(s->geo, s->cfg.precision, s->state, stage, stage + npts,
                           stage + 2 * npts, stage + 3 * npts, s->stream);
    double *dst[4] = {P, Q, U, V};
    for (int f = 0; f < 4 && e == hipSuccess; ++f)
        e = hipMemcpyAsync(dst[f], stage + f * npts, bytes, hipMemcpyDeviceToHost, s->stream);
    hipError_t e2 = hipStreamSynchronize(s->stream);
    const hipError_t e3 = free_device(stage);
    if (e != hipSuccess) return hip_fail(s, e, "gather / copy-out");
    if (e2 != hipSuccess) return hip_fail(s, e2, "hipStreamSynchronize");
    if (e3 != hipSuccess) return hip_fail(s, e3, "hipFree (staging)");
    return KGS_OK;
}

int kgs_write_state(kgs_sim *s, const double *P, const double *Q, const double *U,
                    const double *V, int32_t mem)
{
    KGS_TRACE("kgs_write_state");
    if (!s) return fail(nullptr, KGS_EINVAL, "handle is NULL");
    int rc = check_device(s);
    if (rc != KGS_OK) return rc;
    return load_state(s, P, Q, U, V, mem);
}

int kgs_sync(kgs_sim *s)
{
    KGS_TRACE("kgs_sync");
    if (!s) return fail(nullptr, KGS_EINVAL, "handle is NULL");
    int rc = check_device(s);
    if (rc == KGS_OK) rc = kgs::sim_close(s, s->stream);  // the step's own last sweep
    if (rc != KGS_OK) return rc;
    hipError_t e = hipStreamSynchronize(s->stream);
    return e == hipSuccess ? KGS_OK : hip_fail(s, e, "hipStreamSynchronize");
}

int kgs_free(kgs_sim *s)
{
    KGS_TRACE("kgs_free");
    if (!s) return KGS_OK;
    int rc = check_device(s);
    if (rc == KGS_OK) {
        hipError_t e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) rc = hip_fail(s, e, "hipStreamSynchronize");
    }
    const hipError_t e = release(s);
    if (rc == KGS_OK && e != hipSuccess) rc = hip_fail(s, e, "releasing device memory");
    if (rc != KGS_OK) g_err = s->err;
    delete s;
    return rc;
}

int kgs_get_tuning(const kgs_sim *s, kgs_tuning *out)
{
    if (!s || !out) return fail(nullptr, KGS_EINVAL, "handle or output is NULL");
    *out = s->tuning;
    return KGS_OK;
}

int kgs_set_tuning(kgs_sim *s, const kgs_tuning *t)
{
    KGS_TRACE("kgs_set_tuning");
    if (!s || !t) return fail(s, KGS_EINVAL, "handle or tuning is NULL");
    kgs_tuning nt;
    bool pingpong = false;
    int rc = resolve_tuning(s, *t, nt, pingpong);
    if (rc != KGS_OK) return rc;
    if (pingpong) {
        rc = kgs::sim_ensure_state2(s);
        if (rc != KGS_OK) return rc;
    }
    s->tuning = nt;
    return KGS_OK;
}

int kgs_get_info(const kgs_sim *s, kgs_info *out)
{
    if (!s || !out) return fail(nullptr, KGS_EINVAL, "handle or output is NULL");
    out->points = 2 * s->geo.count;
    out->device_bytes = s->device_bytes;
    out->kernel = s->tuning.kernel;
    out->precision = s->cfg.precision;
    return KGS_OK;
}

}  // extern "C"
