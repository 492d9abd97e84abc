// C ABI of the lbpf library (declared in include/lbpf.h): parameter validation, derivation of
// the model coefficients, carving of the caller's device workspace and kernel sequencing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "lbpf.h"
#include "lbpf_model.hpp"

namespace lbpf {
int tile_count();
void tile_shape(int i, int* tx, int* rows, int* nt);
hipError_t launch_step(int tile, const Model& m, const float* in, float* out, hipStream_t st);
hipError_t launch_fields(const Model& m, const float* in, float* fields, hipStream_t st);
hipError_t launch_init(const Model& m, const float* phi0, const float* ux0, const float* uy0,
                       const float* p0, float* copy, hipStream_t st);
hipError_t launch_stats(const Model& m, const float* plane, double* red, hipStream_t st);
hipError_t diag_noalloc(const Model& m, const float* copy, const float* fields, hipStream_t st,
                        double* host4);
hipError_t launch_diag(const Model& m, const float* copy, const float* fields, double* red,
                       hipStream_t st);
hipError_t launch_laplace(const Model& m, const float* copy, const float* fields, double* phi64,
                          double xc, double yc, double r_in, double r_out, double* red,
                          hipStream_t st);
hipError_t launch_probe(int mode, const void* src, void* dst, size_t bytes, int blocks, hipStream_t st);
hipError_t batch_kernel_info(int tile, void** fn, int* nt, int* tx, int* ch, int* per_cu);
hipError_t launch_fields_to_nhwc(const Model& m, const float* fields, float* dst, const float* shift,
                                 const float* scale, hipStream_t st);
hipError_t launch_nhwc_to_dense(const Model& m, const float* src, float* phi, float* ux, float* uy,
                                float* p, const float* shift, const float* scale, hipStream_t st);
hipError_t launch_batch(int tile, float* wsb, const BatchInst* insts, const BatchItem* items, int nitems,
                        int grid, int parity, int* ctrs, int slot, hipStream_t st);
}  // namespace lbpf

using namespace lbpf;

struct lbpf_ctx {
    lbpf_params params;
    Model m;
    float* ws;          // base of the caller's workspace
    size_t ws_bytes;
    hipStream_t stream;
    int cur;            // 0: state in copy A, 1: in copy B
    int initialized;
    int tile;
    int64_t step;
    int64_t hdr[8];     // checkpoint header staging (host)
    std::string err;
};

static thread_local std::string g_create_err;
// Default strip shapes (indices into the table of lbpf_tile_shape): for one simulation the
// shape that measured fastest on a 1024^2 grid (64 wide, 32 rows, 512 threads, loads of the
// next step of the march issued before the update); for a batch of small grids 64 wide,
// 16 rows, 256 threads. lbpf_autotune / lbpf_batch_autotune choose per workload.
static const int kDefaultTile = 12;
static const int kDefaultBatchTile = 1;

static lbpf_status fail(lbpf_ctx* c, lbpf_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    else g_create_err = buf;
    return s;
}

static lbpf_status hip_fail(lbpf_ctx* c, hipError_t e, const char* what) {
    return fail(c, LBPF_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

static size_t plane_pad();

static const char* validate(const lbpf_params* p) {
    if (!p) return "params is NULL";
    if (p->nx < 3 || p->ny < 3) return "nx and ny must be >= 3";
    if (p->nx >= (1 << 24) || p->ny >= (1 << 24)) return "nx and ny must be below 2^24";
    // the kernels form a row offset y * pitch with the 24-bit multiplier, so the row stride of
    // a copy must stay below 2^24 floats (interleaved() falls back to separate planes, whose
    // stride is pitch_of(nx))
    if (pitch_of(p->nx) >= (1 << 24)) return "nx rounded up to a multiple of 64 must be below 2^24";
    // kernels address a node inside a plane with a 32-bit byte offset (planes stored separately
    // when the grid is too large to interleave them)
    if ((long long)p->ny * pitch_of(p->nx) + plane_pad() >= (1LL << 30))
        return "grid too large (a plane of ny * pitch nodes must hold fewer than 2^30 floats)";
    if (p->variant != LBPF_QIM && p->variant != LBPF_IM) return "variant must be LBPF_QIM or LBPF_IM";
    if (p->pscheme < 0 || p->pscheme > 2) return "pscheme out of range";
    if (p->fsurf != 0 && p->fsurf != 1) return "fsurf out of range";
    if (p->visc != 0 && p->visc != 1) return "visc out of range";
    if (p->bc != 0 && p->bc != 1) return "bc out of range";
    if (!(p->tau_h > 0.5)) return "tau_h must be > 1/2";
    if (!(p->nu_A > 0.0) || !(p->nu_B > 0.0)) return "nu_A and nu_B must be > 0";
    if (!(p->rho_A > 0.0) || !(p->rho_B > 0.0)) return "rho_A and rho_B must be > 0";
    if (!(p->W > 0.0)) return "W must be > 0";
    if (!(p->sigma >= 0.0)) return "sigma must be >= 0";
    if (!std::isfinite(p->M_phi) || !std::isfinite(p->force_x) || !std::isfinite(p->force_y) ||
        !std::isfinite(p->gravity))
        return "M_phi, forces and gravity must be finite";
    return nullptr;
}

// Distance between consecutive planes: ny rows of `pitch` floats plus a layout pad. The pad
// (LBPF_PLANE_PAD_FLOATS, a multiple of 64, default kDefaultPlanePad) keeps the 21 planes of a
// node from sitting a power of two apart, which would map them to the same DRAM banks. It must
// not change between lbpf_workspace_size() and lbpf_create() of one simulation.
static size_t plane_pad() {
    const char* e = getenv("LBPF_PLANE_PAD_FLOATS");
    long v = e ? strtol(e, nullptr, 10) : kDefaultPlanePad;
    if (v < 0) v = 0;
    return (size_t)(v + 63) / 64 * 64;
}
// Layout of a population copy (see lbpf_model.hpp): planes interleaved by row unless
// LBPF_STATE_LAYOUT=planar, or unless a copy of 21 interleaved planes would need per-lane offsets
// of 2^30 floats or more, or a row stride (21 row planes) of 2^24 floats or more, which the
// kernels' 24-bit row multiply cannot form. The choice must not change between
// lbpf_workspace_size() and lbpf_create() of one simulation.
// Interleaved by row, consecutive planes of a row are row_plane(nx) floats apart: rows of 4 KiB
// or less get 32 floats more, so that the planes of a row do not sit a power of two apart
// (1024^2: 33.9 -> 34.4 GLUPS); longer rows do not (4096^2: 30.4 without, 30.1 with).
static long long row_plane(int nx) { const int xp = pitch_of(nx); return xp + (xp <= 1024 ? 32 : 0); }
static bool interleaved(const lbpf_params* p) {
    const char* e = getenv("LBPF_STATE_LAYOUT");
    if (e && strcmp(e, "planar") == 0) return false;
    const long long stride = kCopyPlanes * row_plane(p->nx);
    return stride < (1LL << 24) && (long long)p->ny * stride < (1LL << 30);
}
static size_t copy_floats(const lbpf_params* p) {
    return interleaved(p) ? kCopyPlanes * (size_t)p->ny * row_plane(p->nx) + plane_pad()
                          : kCopyPlanes * ((size_t)p->ny * pitch_of(p->nx) + plane_pad());
}
static size_t f64_floats(const lbpf_params* p) { return 2 * (size_t)p->ny * pitch_of(p->nx); }

static size_t ws_bytes(const lbpf_params* p) {
    return (2 * copy_floats(p) + f64_floats(p)) * sizeof(float) + kRedDoubles * sizeof(double);
}

// Model coefficients from the physical parameters:
//   beta = 12 sigma / W, kappa = 3 sigma W / 2 (eqs. 6-7 solved for beta and kappa),
//   eta = M_phi / (c_s^2 (tau_h - 1/2)) (eq. 17), gamma = (rho_A - rho_B) / rho_B (Sec. 3.2.1).
static Model make_model(const lbpf_params* p) {
    Model m{};
    m.nx = p->nx;
    m.ny = p->ny;
    m.xpitch = pitch_of(p->nx);
    if (interleaved(p)) {
        m.plane = row_plane(p->nx);
        m.pitch = (int)(kCopyPlanes * m.plane);
    } else {
        m.pitch = m.xpitch;
        m.plane = (long long)p->ny * m.xpitch + (long long)plane_pad();
    }
    m.copy = (long long)copy_floats(p);
    m.variant = p->variant;
    m.pscheme = p->pscheme;
    m.fsurf = p->fsurf;
    m.visc = p->visc;
    m.bc = p->bc;
    m.clamp = p->clamp_props ? 1 : 0;
    const double beta = 12.0 * p->sigma / p->W, kappa = 1.5 * p->sigma * p->W;
    const double eta = p->M_phi / ((p->tau_h - 0.5) / 3.0);
    const double gamma = (p->rho_A - p->rho_B) / p->rho_B;
    m.beta4 = (float)(4.0 * beta);
    m.kappa = (float)kappa;
    m.eta = (float)eta;
    m.gammaM = (float)(gamma * p->M_phi);
    m.rhoA = (float)p->rho_A;
    m.rhoB = (float)p->rho_B;
    m.drho = (float)(p->rho_A - p->rho_B);
    m.inv_nuA = (float)(1.0 / p->nu_A);
    m.inv_nuB = (float)(1.0 / p->nu_B);
    m.muA = (float)(p->rho_A * p->nu_A);
    m.muB = (float)(p->rho_B * p->nu_B);
    m.inv_tau_h = (float)(1.0 / p->tau_h);
    m.src_coef = (float)(1.0 - 0.5 / p->tau_h);
    m.fx = (float)p->force_x;
    m.fy = (float)p->force_y;
    m.grav = (float)p->gravity;
    m.d_beta = beta;
    m.d_kappa = kappa;
    m.d_rhoA = p->rho_A;
    m.d_rhoB = p->rho_B;
    return m;
}

static float* copy_of(lbpf_ctx* c, int k) { return c->ws + (size_t)k * c->m.copy; }
static float* cur_copy(lbpf_ctx* c) { return copy_of(c, c->cur); }
// field scratch: the population copy not holding the state
static float* fields(lbpf_ctx* c) { return copy_of(c, 1 - c->cur); }
static double* phi64(lbpf_ctx* c) { return (double*)copy_of(c, 2); }
static double* red(lbpf_ctx* c) { return (double*)(copy_of(c, 2) + 2 * (size_t)c->m.ny * c->m.xpitch); }

static lbpf_status check_ctx(lbpf_ctx* c, bool need_init) {
    if (!c) return LBPF_E_INVALID;
    c->err.clear();
    if (need_init && !c->initialized) return fail(c, LBPF_E_STATE, "lbpf_init has not been called");
    return LBPF_OK;
}

extern "C" {

lbpf_status lbpf_workspace_size(const lbpf_params* params, size_t* bytes) {
    if (const char* why = validate(params)) return fail(nullptr, LBPF_E_INVALID, "%s", why);
    if (!bytes) return fail(nullptr, LBPF_E_INVALID, "bytes is NULL");
    *bytes = ws_bytes(params);
    return LBPF_OK;
}

lbpf_status lbpf_create(const lbpf_params* params, void* workspace, size_t workspace_bytes,
                        void* hip_stream, lbpf_ctx** out) {
    if (!out) return fail(nullptr, LBPF_E_INVALID, "out is NULL");
    *out = nullptr;
    if (const char* why = validate(params)) return fail(nullptr, LBPF_E_INVALID, "%s", why);
    if (!workspace) return fail(nullptr, LBPF_E_INVALID, "workspace is NULL");
    if (((uintptr_t)workspace) % 256 != 0)
        return fail(nullptr, LBPF_E_INVALID, "workspace must be 256-byte aligned");
    const size_t need = ws_bytes(params);
    if (workspace_bytes < need)
        return fail(nullptr, LBPF_E_NOMEM, "workspace has %zu bytes, needs %zu", workspace_bytes, need);
    lbpf_ctx* c = new (std::nothrow) lbpf_ctx();
    if (!c) return fail(nullptr, LBPF_E_NOMEM, "host allocation failed");
    c->params = *params;
    c->m = make_model(params);
    c->ws = (float*)workspace;
    c->ws_bytes = workspace_bytes;
    c->stream = (hipStream_t)hip_stream;
    c->cur = 0;
    c->initialized = 0;
    c->tile = kDefaultTile;
    c->step = 0;
    *out = c;
    return LBPF_OK;
}

static lbpf_status init_copy(lbpf_ctx* c, int copy, const float* phi, const float* ux,
                             const float* uy, const float* p) {
    if (lbpf_status s = check_ctx(c, false)) return s;
    if (!phi) return fail(c, LBPF_E_INVALID, "phi is NULL");
    c->cur = copy;
    hipError_t e = launch_init(c->m, phi, ux, uy, p, cur_copy(c), c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "init kernel");
    c->initialized = 1;
    c->step = 0;
    return LBPF_OK;
}

lbpf_status lbpf_init(lbpf_ctx* c, const float* phi, const float* ux, const float* uy, const float* p) {
    return init_copy(c, 0, phi, ux, uy, p);
}

lbpf_status lbpf_step(lbpf_ctx* c, int64_t nsteps) {
    if (lbpf_status s = check_ctx(c, true)) return s;
    if (nsteps < 0) return fail(c, LBPF_E_INVALID, "nsteps must be >= 0");
    for (int64_t t = 0; t < nsteps; ++t) {
        const int a = c->cur, b = 1 - a;
        hipError_t e = launch_step(c->tile, c->m, copy_of(c, a), copy_of(c, b), c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "step kernel");
        c->cur = b;
        c->step += 1;
    }
    return LBPF_OK;
}

static lbpf_status run_fields(lbpf_ctx* c) {
    hipError_t e = launch_fields(c->m, cur_copy(c), fields(c), c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "field kernel");
    return LBPF_OK;
}

lbpf_status lbpf_read(lbpf_ctx* c, int32_t field, float* dst) {
    if (lbpf_status s = check_ctx(c, true)) return s;
    if (field < LBPF_FIELD_PHI || field > LBPF_FIELD_MU) return fail(c, LBPF_E_INVALID, "unknown field %d", field);
    if (!dst) return fail(c, LBPF_E_INVALID, "dst is NULL");
    if (lbpf_status s = run_fields(c)) return s;
    const float* src = fields(c) + (size_t)field * c->m.plane;
    hipError_t e = hipMemcpy2DAsync(dst, (size_t)c->m.nx * sizeof(float), src,
                                    (size_t)c->m.pitch * sizeof(float), (size_t)c->m.nx * sizeof(float),
                                    (size_t)c->m.ny, hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "field copy");
    return LBPF_OK;
}

lbpf_status lbpf_diagnostics(lbpf_ctx* c, lbpf_diag* out) {
    if (lbpf_status s = check_ctx(c, true)) return s;
    if (!out) return fail(c, LBPF_E_INVALID, "out is NULL");
    if (lbpf_status s = run_fields(c)) return s;
    hipError_t e = launch_diag(c->m, cur_copy(c), fields(c), red(c), c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "diagnostic kernels");
    double r[4];
    e = hipMemcpyAsync(r, red(c) + (size_t)kRedBlocks * kRedSlots, sizeof r, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "diagnostic readback");
    out->sum_phi = r[0];
    out->sum_rho = r[1];
    out->max_u = r[2];
    out->nonfinite = (int64_t)r[3];
    out->step = c->step;
    if (out->nonfinite != 0 || !std::isfinite(r[0]))
        return fail(c, LBPF_E_UNSTABLE, "%lld non-finite values in the state at step %lld",
                    (long long)out->nonfinite, (long long)c->step);
    return LBPF_OK;
}

lbpf_status lbpf_diagnostics_noalloc(lbpf_ctx* c, lbpf_diag* out) {
    if (lbpf_status s = check_ctx(c, true)) return s;
    if (!out) return fail(c, LBPF_E_INVALID, "out is NULL");
    if (lbpf_status s = run_fields(c)) return s;
    double r[4];
    hipError_t e = diag_noalloc(c->m, cur_copy(c), fields(c), c->stream, r);
    if (e == hipErrorInvalidValue)
        return fail(c, LBPF_E_NOMEM, "the diagnostic partials exceed the fixed scratch");
    if (e != hipSuccess) return hip_fail(c, e, "diagnostic kernels (fixed scratch)");
    out->sum_phi = r[0];
    out->sum_rho = r[1];
    out->max_u = r[2];
    out->nonfinite = (int64_t)r[3];
    out->step = c->step;
    if (out->nonfinite != 0 || !std::isfinite(r[0]))
        return fail(c, LBPF_E_UNSTABLE, "%lld non-finite values in the state at step %lld",
                    (long long)out->nonfinite, (long long)c->step);
    return LBPF_OK;
}

lbpf_status lbpf_field_stats(lbpf_ctx* c, int32_t field, double* out3) {
    if (lbpf_status s = check_ctx(c, true)) return s;
    if (field < LBPF_FIELD_PHI || field > LBPF_FIELD_MU) return fail(c, LBPF_E_INVALID, "unknown field %d", field);
    if (!out3) return fail(c, LBPF_E_INVALID, "out is NULL");
    if (lbpf_status s = run_fields(c)) return s;
    hipError_t e = launch_stats(c->m, fields(c) + (size_t)field * c->m.plane, red(c), c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "field statistics kernels");
    double r[3];
    e = hipMemcpyAsync(r, red(c) + (size_t)kRedBlocks * kRedSlots, sizeof r, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "field statistics readback");
    const double n = (double)c->m.nx * (double)c->m.ny;
    const double mean = r[0] / n;
    const double var = r[1] / n - mean * mean;
    out3[0] = mean;
    out3[1] = var > 0.0 ? std::sqrt(var) : 0.0;
    out3[2] = r[2];
    return LBPF_OK;
}

lbpf_status lbpf_field_stats_many(lbpf_ctx* c, int32_t n, const int32_t* which, double* out) {
    if (lbpf_status s = check_ctx(c, true)) return s;
    constexpr int kMax = LBPF_FIELD_MU + 1;
    if (n < 1 || n > kMax || !which || !out) return fail(c, LBPF_E_INVALID, "n in 1..%d and both arrays required", kMax);
    for (int k = 0; k < n; ++k)
        if (which[k] < LBPF_FIELD_PHI || which[k] > LBPF_FIELD_MU)
            return fail(c, LBPF_E_INVALID, "unknown field %d", which[k]);
    if (lbpf_status s = run_fields(c)) return s;
    // each field's three sums go from the reduction's result slots to slots 16 + 4 k of the same
    // 64-double area (stream order), then all of them come back in one copy
    double* res = red(c) + (size_t)kRedBlocks * kRedSlots;
    hipError_t e = hipSuccess;
    for (int k = 0; k < n && e == hipSuccess; ++k) {
        e = launch_stats(c->m, fields(c) + (size_t)which[k] * c->m.plane, red(c), c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(res + 16 + 4 * k, res, 3 * sizeof(double), hipMemcpyDeviceToDevice, c->stream);
    }
    if (e != hipSuccess) return hip_fail(c, e, "field statistics kernels");
    double r[4 * kMax];
    e = hipMemcpyAsync(r, res + 16, sizeof(double) * 4 * n, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "field statistics readback");
    const double cells = (double)c->m.nx * (double)c->m.ny;
    for (int k = 0; k < n; ++k) {
        const double mean = r[4 * k] / cells;
        const double var = r[4 * k + 1] / cells - mean * mean;
        out[3 * k] = mean;
        out[3 * k + 1] = var > 0.0 ? std::sqrt(var) : 0.0;
        out[3 * k + 2] = r[4 * k + 2];
    }
    return LBPF_OK;
}

lbpf_status lbpf_laplace_dp(lbpf_ctx* c, double xc, double yc, double R, double* dP) {
    if (lbpf_status s = check_ctx(c, true)) return s;
    if (!dP) return fail(c, LBPF_E_INVALID, "dP is NULL");
    if (!(R > 0.0)) return fail(c, LBPF_E_INVALID, "R must be > 0");
    if (lbpf_status s = run_fields(c)) return s;
    hipError_t e = launch_laplace(c->m, cur_copy(c), fields(c), phi64(c),
                                  xc, yc, 0.5 * R, R + 3.0 * c->params.W, red(c), c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "laplace kernels");
    double r[4];
    e = hipMemcpyAsync(r, red(c) + (size_t)kRedBlocks * kRedSlots, sizeof r, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "laplace readback");
    if (r[1] < 1.0 || r[3] < 1.0)
        return fail(c, LBPF_E_INVALID, "empty inner (%g nodes) or outer (%g nodes) region", r[1], r[3]);
    *dP = r[0] / r[1] - r[2] / r[3];
    return LBPF_OK;
}

// checkpoint layout: 64-byte header {magic, version, nx, ny, row stride, step, plane stride,
// copy floats}, then the population copy holding the state, as stored (f_1..8, h, p, (phi u)_x,y;
// see lbpf_model.hpp). A checkpoint loads into a simulation of the same grid and layout.
static const int64_t kMagic = 0x4650424C;  // "LBPF"
static const int64_t kVersion = 2;

lbpf_status lbpf_state_size(const lbpf_ctx* c, size_t* bytes) {
    if (!c || !bytes) return LBPF_E_INVALID;
    *bytes = 64 + (size_t)c->m.copy * sizeof(float);
    return LBPF_OK;
}

lbpf_status lbpf_save_state(lbpf_ctx* c, void* dst) {
    if (lbpf_status s = check_ctx(c, true)) return s;
    if (!dst) return fail(c, LBPF_E_INVALID, "dst is NULL");
    // the header is copied synchronously so that hdr may be reused at once
    c->hdr[0] = kMagic; c->hdr[1] = kVersion; c->hdr[2] = c->m.nx; c->hdr[3] = c->m.ny;
    c->hdr[4] = c->m.pitch; c->hdr[5] = c->step; c->hdr[6] = c->m.plane; c->hdr[7] = c->m.copy;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) e = hipMemcpy(dst, c->hdr, 64, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpyAsync((char*)dst + 64, cur_copy(c), (size_t)c->m.copy * sizeof(float),
                           hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "save state");
    return LBPF_OK;
}

lbpf_status lbpf_load_state(lbpf_ctx* c, const void* src) {
    if (lbpf_status s = check_ctx(c, false)) return s;
    if (!src) return fail(c, LBPF_E_INVALID, "src is NULL");
    int64_t hdr[8];
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) e = hipMemcpy(hdr, src, 64, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(c, e, "load state header");
    if (hdr[0] != kMagic || hdr[1] != kVersion || hdr[2] != c->m.nx || hdr[3] != c->m.ny ||
        hdr[4] != c->m.pitch || hdr[6] != c->m.plane || hdr[7] != c->m.copy)
        return fail(c, LBPF_E_INVALID, "checkpoint does not match this grid and layout");
    c->cur = 0;
    e = hipMemcpyAsync(cur_copy(c), (const char*)src + 64, (size_t)c->m.copy * sizeof(float),
                       hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "load state");
    c->step = hdr[5];
    c->initialized = 1;
    return LBPF_OK;
}

lbpf_status lbpf_set_stream(lbpf_ctx* c, void* hip_stream) {
    if (lbpf_status s = check_ctx(c, false)) return s;
    c->stream = (hipStream_t)hip_stream;
    return LBPF_OK;
}

lbpf_status lbpf_autotune(lbpf_ctx* c, int32_t trial_steps, void* scratch_state, float* ms_out,
                          int32_t* best_out) {
    if (lbpf_status s = check_ctx(c, true)) return s;
    if (trial_steps < 1 || !scratch_state) return fail(c, LBPF_E_INVALID, "trial_steps >= 1 and a state buffer are required");
    if (lbpf_status s = lbpf_save_state(c, scratch_state)) return s;
    const int64_t step0 = c->step;
    const int keep = c->tile;
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) return hip_fail(c, e, "autotune events");
    int best = keep;
    float best_ms = 0.0f;
    lbpf_status st = LBPF_OK;
    for (int t = 0; t < tile_count() && st == LBPF_OK; ++t) {
        c->tile = t;
        st = lbpf_step(c, 1);  // warm-up launch of this shape
        if (st != LBPF_OK) break;
        e = hipEventRecord(e0, c->stream);
        if (e == hipSuccess && (st = lbpf_step(c, trial_steps)) == LBPF_OK) e = hipEventRecord(e1, c->stream);
        if (e == hipSuccess && st == LBPF_OK) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess && st == LBPF_OK) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) { st = hip_fail(c, e, "autotune timing"); break; }
        ms /= (float)trial_steps;
        if (ms_out) ms_out[t] = ms;
        if (t == 0 || ms < best_ms) { best_ms = ms; best = t; }
    }
    (void)hipEventDestroy(e0);  // cleanup: nothing to do on failure
    (void)hipEventDestroy(e1);
    c->tile = keep;
    if (st != LBPF_OK) return st;
    if (lbpf_status s = lbpf_load_state(c, scratch_state)) return s;
    c->step = step0;
    c->tile = best;
    if (best_out) *best_out = best;
    return LBPF_OK;
}

lbpf_status lbpf_fields_to_nhwc(lbpf_ctx* c, float* dst, const float* shift, const float* scale) {
    if (lbpf_status s = check_ctx(c, true)) return s;
    if (!dst || !shift || !scale) return fail(c, LBPF_E_INVALID, "NULL argument");
    for (int k = 0; k < 4; ++k)
        if (!(scale[k] != 0.0f) || !std::isfinite(scale[k]) || !std::isfinite(shift[k]))
            return fail(c, LBPF_E_INVALID, "scale must be finite and nonzero, shift finite");
    if (((uintptr_t)dst) % 16) return fail(c, LBPF_E_INVALID, "dst must be 16-byte aligned");
    if (lbpf_status s = run_fields(c)) return s;
    hipError_t e = launch_fields_to_nhwc(c->m, fields(c), dst, shift, scale, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "fields to NHWC");
    return LBPF_OK;
}

lbpf_status lbpf_init_from_nhwc(lbpf_ctx* c, const float* src, const float* shift, const float* scale,
                                int64_t step) {
    if (lbpf_status s = check_ctx(c, false)) return s;
    if (!src || !shift || !scale) return fail(c, LBPF_E_INVALID, "NULL argument");
    if (((uintptr_t)src) % 16) return fail(c, LBPF_E_INVALID, "src must be 16-byte aligned");
    // dense nx*ny fields in the copy that init does not write (it holds 21 ny*pitch floats)
    float* d[4];
    for (int k = 0; k < 4; ++k) d[k] = fields(c) + (size_t)k * c->m.nx * c->m.ny;
    hipError_t e = launch_nhwc_to_dense(c->m, src, d[0], d[1], d[2], d[3], shift, scale, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "NHWC to fields");
    if (step < 0) return fail(c, LBPF_E_INVALID, "step must be >= 0");
    if (lbpf_status s = init_copy(c, c->cur, d[0], d[1], d[2], d[3])) return s;
    c->step = step;
    return LBPF_OK;
}

int32_t lbpf_tile_count(void) { return tile_count(); }

lbpf_status lbpf_tile_shape(int32_t i, int32_t* tx, int32_t* rows, int32_t* threads) {
    if (i < 0 || i >= tile_count() || !tx || !rows || !threads) return LBPF_E_INVALID;
    int a, b, t;
    tile_shape(i, &a, &b, &t);
    *tx = a; *rows = b; *threads = t;
    return LBPF_OK;
}

lbpf_status lbpf_set_tile(lbpf_ctx* c, int32_t i) {
    if (lbpf_status s = check_ctx(c, false)) return s;
    if (i < 0 || i >= tile_count()) return fail(c, LBPF_E_INVALID, "tile index %d out of range", i);
    c->tile = i;
    return LBPF_OK;
}

lbpf_status lbpf_bw_probe(int32_t mode, const void* src, void* dst, size_t bytes, int32_t blocks,
                          void* hip_stream) {
    if (mode < 0 || mode > 2) return fail(nullptr, LBPF_E_INVALID, "probe mode must be 0, 1 or 2");
    if (bytes % 16 != 0) return fail(nullptr, LBPF_E_INVALID, "probe size must be a multiple of 16 bytes");
    if ((mode != 2 && !src) || !dst) return fail(nullptr, LBPF_E_INVALID, "probe buffer is NULL");
    hipError_t e = launch_probe(mode, src, dst, bytes, blocks, (hipStream_t)hip_stream);
    if (e != hipSuccess) return fail(nullptr, LBPF_E_HIP, "probe kernel: %s", hipGetErrorString(e));
    return LBPF_OK;
}

int64_t lbpf_step_count(const lbpf_ctx* c) { return c ? c->step : -1; }

int32_t lbpf_get_tile(const lbpf_ctx* c) { return c ? c->tile : -1; }

lbpf_status lbpf_destroy(lbpf_ctx* c) {
    delete c;
    return LBPF_OK;
}

const char* lbpf_status_string(lbpf_status s) {
    switch (s) {
        case LBPF_OK: return "ok";
        case LBPF_E_INVALID: return "invalid argument";
        case LBPF_E_HIP: return "HIP runtime error";
        case LBPF_E_NOMEM: return "insufficient memory";
        case LBPF_E_UNSTABLE: return "non-finite state";
        case LBPF_E_STATE: return "call out of order";
    }
    return "unknown status";
}

const char* lbpf_last_error(const lbpf_ctx* c) { return c ? c->err.c_str() : "NULL handle"; }

const char* lbpf_create_error(void) { return g_create_err.c_str(); }

}  // extern "C"

// ---------------------------------------------------------------------------------------------
// Batch of independent simulations
// ---------------------------------------------------------------------------------------------
struct lbpf_batch {
    int n;
    std::vector<lbpf_ctx*> inst;
    std::vector<size_t> inst_off;     // byte offset of each instance workspace
    std::vector<int> frozen;
    char* ws;
    size_t ws_bytes;
    BatchInst* d_insts;               // device arrays at the start of the workspace
    BatchItem* d_items;
    int* d_ctr;                       // kBatchSlots x 8 band counters of the batch kernel
    int slot;                         // counter slot of the next batch-kernel launch
    size_t max_items;
    int nitems;
    int tile;
    int grid;
    int parity;                       // population copy holding the current state
    int64_t step;
    hipStream_t stream;
    hipGraph_t graph[2];
    hipGraphExec_t exec[2];
    int graph_steps;
    std::string err;
};

static const int kBatchGraphSteps = 8;
static_assert(kBatchGraphSteps == kBatchSlots, "a graph replay uses every counter slot once, in order");

static lbpf_status bfail(lbpf_batch* b, lbpf_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (b) b->err = buf;
    else g_create_err = buf;
    return s;
}

static size_t align256(size_t v) { return (v + 255) / 256 * 256; }

static size_t batch_max_items(int n, const lbpf_params* params) {
    size_t best = 0;
    for (int t = 0; t < tile_count(); ++t) {
        int tx, ch, nt;
        tile_shape(t, &tx, &ch, &nt);
        size_t items = 0;
        for (int k = 0; k < n; ++k)
            items += (size_t)((params[k].nx + tx - 1) / tx) * ((params[k].ny + ch - 1) / ch);
        if (items > best) best = items;
    }
    return best;
}

static size_t batch_header_bytes(int n, const lbpf_params* params) {
    return align256(sizeof(BatchInst) * n) + align256(sizeof(BatchItem) * batch_max_items(n, params)) +
           align256(sizeof(int) * 8 * kBatchSlots);
}

static void destroy_graphs(lbpf_batch* b) {
    for (int i = 0; i < 2; ++i) {
        if (b->exec[i]) (void)hipGraphExecDestroy(b->exec[i]);
        if (b->graph[i]) (void)hipGraphDestroy(b->graph[i]);
        b->exec[i] = nullptr;
        b->graph[i] = nullptr;
    }
}

// Work list and persistent grid for the current strip shape, and the two step graphs (starting
// from either population copy), built node by node so that any stream can replay them.
static lbpf_status batch_setup(lbpf_batch* b) {
    void* fn;
    int nt, tx, ch, per;
    hipError_t e = batch_kernel_info(b->tile, &fn, &nt, &tx, &ch, &per);
    if (e != hipSuccess) return bfail(b, LBPF_E_HIP, "batch kernel info: %s", hipGetErrorString(e));
    std::vector<BatchInst> hi(b->n);
    std::vector<BatchItem> items;
    for (int k = 0; k < b->n; ++k) {
        const Model& m = b->inst[k]->m;
        hi[k].m = m;
        // every instance's workspace lies in the batch's (float-aligned offsets)
        hi[k].ws_off = (long long)(reinterpret_cast<char*>(b->inst[k]->ws) - b->ws) / (long long)sizeof(float);
        hi[k].nsx = (m.nx + tx - 1) / tx;
        hi[k].nsy = (m.ny + ch - 1) / ch;
        if (b->frozen[k]) continue;  // held fixed: no work, its state stays in its copy
        for (int c = 0; c < hi[k].nsx * hi[k].nsy; ++c) items.push_back(BatchItem{k, c});
    }
    if (items.size() > b->max_items) return bfail(b, LBPF_E_NOMEM, "work list overflow");
    b->nitems = (int)items.size();
    int dev = 0, cus = 0;
    e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return bfail(b, LBPF_E_HIP, "device query: %s", hipGetErrorString(e));
    b->grid = std::max(1, std::min(b->nitems, cus * per));
    e = hipStreamSynchronize(b->stream);
    if (e == hipSuccess) e = hipMemcpy(b->d_insts, hi.data(), sizeof(BatchInst) * b->n, hipMemcpyHostToDevice);
    if (e == hipSuccess && !items.empty())  // every instance frozen: an empty list
        e = hipMemcpy(b->d_items, items.data(), sizeof(BatchItem) * items.size(), hipMemcpyHostToDevice);
    // counters start at zero, and the next launch uses slot 0 (the first of a graph replay)
    if (e == hipSuccess) e = hipMemsetAsync(b->d_ctr, 0, sizeof(int) * 8 * kBatchSlots, b->stream);
    b->slot = 0;
    if (e != hipSuccess) return bfail(b, LBPF_E_HIP, "work list upload: %s", hipGetErrorString(e));
    destroy_graphs(b);
    for (int start = 0; start < 2; ++start) {
        e = hipGraphCreate(&b->graph[start], 0);
        hipGraphNode_t prev = nullptr;
        int parities[kBatchGraphSteps], slots[kBatchGraphSteps];
        for (int sidx = 0; sidx < kBatchGraphSteps && e == hipSuccess; ++sidx) {
            parities[sidx] = (start + sidx) & 1;
            slots[sidx] = sidx;
            float* wsb = reinterpret_cast<float*>(b->ws);
            const BatchInst* di = b->d_insts;
            const BatchItem* dt = b->d_items;
            int ni = b->nitems;
            int* dc = b->d_ctr;
            void* args[] = {(void*)&wsb, (void*)&di, (void*)&dt, (void*)&ni, (void*)&parities[sidx], (void*)&dc,
                            (void*)&slots[sidx]};
            hipKernelNodeParams kp{};
            kp.func = fn;
            kp.gridDim = dim3(b->grid);
            kp.blockDim = dim3(nt);
            kp.sharedMemBytes = 0;
            kp.kernelParams = args;
            kp.extra = nullptr;
            hipGraphNode_t node;
            e = hipGraphAddKernelNode(&node, b->graph[start], prev ? &prev : nullptr, prev ? 1 : 0, &kp);
            prev = node;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&b->exec[start], b->graph[start], nullptr, nullptr, 0);
        if (e != hipSuccess) {
            destroy_graphs(b);
            return bfail(b, LBPF_E_HIP, "step graph: %s", hipGetErrorString(e));
        }
    }
    b->graph_steps = kBatchGraphSteps;
    return LBPF_OK;
}

extern "C" {

lbpf_status lbpf_batch_workspace_size(int32_t n, const lbpf_params* params, size_t* bytes) {
    if (n < 1 || !params || !bytes) return bfail(nullptr, LBPF_E_INVALID, "n >= 1, params and bytes required");
    size_t total = batch_header_bytes(n, params);
    for (int k = 0; k < n; ++k) {
        if (const char* why = validate(&params[k])) return bfail(nullptr, LBPF_E_INVALID, "instance %d: %s", k, why);
        total += align256(ws_bytes(&params[k]));
    }
    *bytes = total;
    return LBPF_OK;
}

lbpf_status lbpf_batch_create(int32_t n, const lbpf_params* params, void* workspace,
                              size_t workspace_bytes, void* hip_stream, lbpf_batch** out) {
    if (!out) return bfail(nullptr, LBPF_E_INVALID, "out is NULL");
    *out = nullptr;
    size_t need = 0;
    if (lbpf_status s = lbpf_batch_workspace_size(n, params, &need)) return s;
    if (!workspace || ((uintptr_t)workspace) % 256 != 0)
        return bfail(nullptr, LBPF_E_INVALID, "workspace must be non-NULL and 256-byte aligned");
    if (workspace_bytes < need)
        return bfail(nullptr, LBPF_E_NOMEM, "workspace has %zu bytes, needs %zu", workspace_bytes, need);
    lbpf_batch* b = new (std::nothrow) lbpf_batch();
    if (!b) return bfail(nullptr, LBPF_E_NOMEM, "host allocation failed");
    b->n = n;
    b->ws = (char*)workspace;
    b->ws_bytes = workspace_bytes;
    b->stream = (hipStream_t)hip_stream;
    b->d_insts = (BatchInst*)b->ws;
    b->max_items = batch_max_items(n, params);
    b->d_items = (BatchItem*)(b->ws + align256(sizeof(BatchInst) * n));
    b->d_ctr = (int*)(b->ws + align256(sizeof(BatchInst) * n) + align256(sizeof(BatchItem) * b->max_items));
    b->slot = 0;
    b->tile = kDefaultBatchTile;
    b->parity = 0;
    b->step = 0;
    b->graph[0] = b->graph[1] = nullptr;
    b->exec[0] = b->exec[1] = nullptr;
    b->frozen.assign(n, 0);
    size_t off = batch_header_bytes(n, params);
    for (int k = 0; k < n; ++k) {
        lbpf_ctx* c = nullptr;
        const size_t sz = align256(ws_bytes(&params[k]));
        lbpf_status s = lbpf_create(&params[k], b->ws + off, sz, hip_stream, &c);
        if (s != LBPF_OK) {
            for (lbpf_ctx* x : b->inst) lbpf_destroy(x);
            delete b;
            return s;
        }
        b->inst.push_back(c);
        b->inst_off.push_back(off);
        off += sz;
    }
    if (lbpf_status s = batch_setup(b)) {
        g_create_err = b->err;
        for (lbpf_ctx* x : b->inst) lbpf_destroy(x);
        destroy_graphs(b);
        delete b;
        return s;
    }
    *out = b;
    return LBPF_OK;
}

lbpf_ctx* lbpf_batch_instance(lbpf_batch* b, int32_t idx) {
    if (!b || idx < 0 || idx >= b->n) return nullptr;
    return b->inst[idx];
}

int32_t lbpf_batch_count(const lbpf_batch* b) { return b ? b->n : -1; }

lbpf_status lbpf_batch_init(lbpf_batch* b, int32_t idx, const float* phi, const float* ux,
                            const float* uy, const float* p) {
    if (!b) return LBPF_E_INVALID;
    b->err.clear();
    if (idx < 0 || idx >= b->n) return bfail(b, LBPF_E_INVALID, "instance %d out of range", idx);
    lbpf_status s = init_copy(b->inst[idx], b->parity, phi, ux, uy, p);
    if (s != LBPF_OK) return bfail(b, s, "instance %d: %s", idx, b->inst[idx]->err.c_str());
    if (b->frozen[idx]) {  // back in the work list, in step with the batch's parity
        b->frozen[idx] = 0;
        return batch_setup(b);
    }
    return LBPF_OK;
}

static lbpf_status batch_check(lbpf_batch* b) {
    if (!b) return LBPF_E_INVALID;
    b->err.clear();
    for (int k = 0; k < b->n; ++k)
        if (!b->inst[k]->initialized) return bfail(b, LBPF_E_STATE, "instance %d is not initialized", k);
    return LBPF_OK;
}

// frozen instances keep their copy and step count
static void batch_advance(lbpf_batch* b, int64_t nsteps) {
    b->parity = (int)((b->parity + nsteps) & 1);
    b->step += nsteps;
    for (int k = 0; k < b->n; ++k) {
        if (b->frozen[k]) continue;
        b->inst[k]->cur = b->parity;
        b->inst[k]->step += nsteps;
    }
}

lbpf_status lbpf_batch_step(lbpf_batch* b, int64_t nsteps) {
    if (lbpf_status s = batch_check(b)) return s;
    if (nsteps < 0) return bfail(b, LBPF_E_INVALID, "nsteps must be >= 0");
    // launches use the counter slots in cyclic order: single launches up to slot 0, then whole
    // graph replays (slots 0 .. 7), then single launches for the rest
    int64_t done = 0;
    auto single = [&]() -> lbpf_status {
        hipError_t e = launch_batch(b->tile, reinterpret_cast<float*>(b->ws), b->d_insts, b->d_items, b->nitems,
                                    b->grid, b->parity, b->d_ctr, b->slot, b->stream);
        if (e != hipSuccess) return bfail(b, LBPF_E_HIP, "batch kernel: %s", hipGetErrorString(e));
        b->slot = (b->slot + 1) % kBatchSlots;
        batch_advance(b, 1);
        ++done;
        return LBPF_OK;
    };
    while (b->slot != 0 && done < nsteps)
        if (lbpf_status s = single()) return s;
    while (nsteps - done >= b->graph_steps) {
        hipError_t e = hipGraphLaunch(b->exec[b->parity], b->stream);
        if (e != hipSuccess) return bfail(b, LBPF_E_HIP, "graph launch: %s", hipGetErrorString(e));
        batch_advance(b, b->graph_steps);
        done += b->graph_steps;
    }
    while (done < nsteps)
        if (lbpf_status s = single()) return s;
    return LBPF_OK;
}

lbpf_status lbpf_batch_step_each(lbpf_batch* b, int64_t nsteps) {
    if (lbpf_status s = batch_check(b)) return s;
    if (nsteps < 0) return bfail(b, LBPF_E_INVALID, "nsteps must be >= 0");
    for (int64_t t = 0; t < nsteps; ++t) {
        for (int k = 0; k < b->n; ++k) {
            lbpf_ctx* c = b->inst[k];
            if (b->frozen[k]) continue;  // held fixed in its copy
            const int tile = c->tile;
            c->tile = b->tile;
            lbpf_status s = lbpf_step(c, 1);
            c->tile = tile;
            if (s != LBPF_OK) return bfail(b, s, "instance %d: %s", k, c->err.c_str());
        }
        b->parity ^= 1;
        b->step += 1;
    }
    return LBPF_OK;
}

lbpf_status lbpf_batch_status(lbpf_batch* b, int32_t* flags, lbpf_diag* diags) {
    if (lbpf_status s = batch_check(b)) return s;
    bool changed = false;
    for (int k = 0; k < b->n; ++k) {
        lbpf_diag d{};
        lbpf_status s = lbpf_diagnostics(b->inst[k], &d);
        if (s == LBPF_E_UNSTABLE && !b->frozen[k]) {
            b->frozen[k] = 1;
            changed = true;
        } else if (s != LBPF_OK && s != LBPF_E_UNSTABLE) {
            return bfail(b, s, "instance %d: %s", k, b->inst[k]->err.c_str());
        }
        if (diags) diags[k] = d;
        if (flags) flags[k] = b->frozen[k];
    }
    if (changed) return batch_setup(b);  // work list without the newly frozen instances
    return LBPF_OK;
}

lbpf_status lbpf_batch_set_tile(lbpf_batch* b, int32_t tile) {
    if (!b) return LBPF_E_INVALID;
    b->err.clear();
    if (tile < 0 || tile >= tile_count()) return bfail(b, LBPF_E_INVALID, "tile index %d out of range", tile);
    b->tile = tile;
    return batch_setup(b);
}

int32_t lbpf_batch_get_tile(const lbpf_batch* b) { return b ? b->tile : -1; }

lbpf_status lbpf_batch_state_size(const lbpf_batch* b, size_t* bytes) {
    if (!b || !bytes) return LBPF_E_INVALID;
    size_t total = 0;
    for (int k = 0; k < b->n; ++k) {
        size_t s = 0;
        lbpf_state_size(b->inst[k], &s);
        total += align256(s);
    }
    *bytes = total;
    return LBPF_OK;
}

lbpf_status lbpf_batch_autotune(lbpf_batch* b, int32_t trial_steps, void* scratch_state,
                                float* ms_out, int32_t* best_out) {
    if (lbpf_status s = batch_check(b)) return s;
    if (trial_steps < 1 || !scratch_state) return bfail(b, LBPF_E_INVALID, "trial_steps >= 1 and a state buffer are required");
    std::vector<size_t> off(b->n);
    size_t o = 0;
    for (int k = 0; k < b->n; ++k) {
        size_t sz = 0;
        lbpf_state_size(b->inst[k], &sz);
        off[k] = o;
        o += align256(sz);
        if (lbpf_status s = lbpf_save_state(b->inst[k], (char*)scratch_state + off[k])) return bfail(b, s, "save %d", k);
    }
    const int64_t keep_step = b->step;
    std::vector<int64_t> keep_inst_step(b->n);
    for (int k = 0; k < b->n; ++k) keep_inst_step[k] = b->inst[k]->step;
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) return bfail(b, LBPF_E_HIP, "autotune events: %s", hipGetErrorString(e));
    int best = b->tile;
    float best_ms = 0.0f;
    lbpf_status st = LBPF_OK;
    for (int t = 0; t < tile_count() && st == LBPF_OK; ++t) {
        if ((st = lbpf_batch_set_tile(b, t)) != LBPF_OK) break;
        if ((st = lbpf_batch_step(b, 1)) != LBPF_OK) break;
        e = hipEventRecord(e0, b->stream);
        if (e == hipSuccess && (st = lbpf_batch_step(b, trial_steps)) == LBPF_OK) e = hipEventRecord(e1, b->stream);
        float ms = 0.0f;
        if (e == hipSuccess && st == LBPF_OK) e = hipEventSynchronize(e1);
        if (e == hipSuccess && st == LBPF_OK) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) { st = bfail(b, LBPF_E_HIP, "autotune timing: %s", hipGetErrorString(e)); break; }
        ms /= (float)trial_steps;
        if (ms_out) ms_out[t] = ms;
        if (t == 0 || ms < best_ms) { best_ms = ms; best = t; }
    }
    (void)hipEventDestroy(e0);  // cleanup: nothing to do on failure
    (void)hipEventDestroy(e1);
    if (st != LBPF_OK) return st;
    // restore: every instance state back into copy A, then the batch continues from parity 0
    for (int k = 0; k < b->n; ++k)
        if (lbpf_status s = lbpf_load_state(b->inst[k], (char*)scratch_state + off[k])) return bfail(b, s, "load %d", k);
    b->parity = 0;
    b->step = keep_step;
    for (int k = 0; k < b->n; ++k) {
        b->inst[k]->cur = 0;
        b->inst[k]->step = keep_inst_step[k];
    }
    if (lbpf_status s = lbpf_batch_set_tile(b, best)) return s;
    if (best_out) *best_out = best;
    return LBPF_OK;
}

int64_t lbpf_batch_step_count(const lbpf_batch* b) { return b ? b->step : -1; }

lbpf_status lbpf_batch_destroy(lbpf_batch* b) {
    if (!b) return LBPF_OK;
    destroy_graphs(b);
    for (lbpf_ctx* c : b->inst) lbpf_destroy(c);
    delete b;
    return LBPF_OK;
}

const char* lbpf_batch_last_error(const lbpf_batch* b) { return b ? b->err.c_str() : "NULL handle"; }

}  // extern "C"
