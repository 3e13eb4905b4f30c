// cns_api.hip -- the C-ABI (include/cns.h): argument checks, plans, workspace carving,
// error reporting.  All compute is enqueued through the launchers in cns_kernels.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "cns_internal.h"

using namespace cns;

static thread_local char g_err[512] = "";

static int set_err(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

static int check_hip(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_err(CNS_EHIP, "%s: %s", what, hipGetErrorString(e));
    return CNS_OK;
}

struct cns_plan {
    Box box;
    int precision;
    hipStream_t stream;
    Tiles tiles;
    Workspace wl;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    Prof prof;
    ~cns_plan() {
        if (prof.ev[0])
            for (auto &e : prof.ev) hipEventDestroy(e);
    }
};

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static Workspace layout(const Box &b, size_t esz) {
    Workspace w{};
    size_t n3 = b.n3();
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    w.W = take(4 * n3 * esz);
    w.G = take(9 * n3 * esz);
    w.rhs = take(5 * n3 * esz);
    w.stA = take(5 * n3 * esz);
    w.stB = take(5 * n3 * esz);
    w.acc = take(5 * n3 * sizeof(double));
    w.part = take((size_t)kDiagBlocks * CNS_NDIAG * sizeof(double));
    w.dhost = take(CNS_NDIAG * sizeof(double));
    w.total = off;
    return w;
}

static bool aligned(const void *p) { return ((uintptr_t)p & 255u) == 0; }

static int check_plan(const cns_plan *p, bool need_ws) {
    if (!p) return set_err(CNS_EINVAL, "null plan");
    if (need_ws && (!p->ws || p->ws_bytes < p->wl.total))
        return set_err(CNS_EWORKSPACE, "workspace of %zu bytes required (have %zu)", p->wl.total, p->ws_bytes);
    return CNS_OK;
}

static int check_ptr(const void *ptr, const char *name) {
    if (!ptr) return set_err(CNS_EINVAL, "%s is null", name);
    if (!aligned(ptr)) return set_err(CNS_EINVAL, "%s is not 256-byte aligned", name);
    return CNS_OK;
}

template <typename T>
static T *ws_at(const cns_plan *p, size_t off) {
    return (T *)(p->ws + off);
}

template <typename T>
static void rk4_steps(cns_plan *p, T *u, double dt, int nsteps, double *diag) {
    T *A = ws_at<T>(p, p->wl.stA), *Bs = ws_at<T>(p, p->wl.stB), *rhs = ws_at<T>(p, p->wl.rhs);
    T *W = ws_at<T>(p, p->wl.W), *G = ws_at<T>(p, p->wl.G);
    double *acc = ws_at<double>(p, p->wl.acc);
    double *part = ws_at<double>(p, p->wl.part);
    for (int n = 0; n < nsteps; ++n) {
        // stage s reads U_s and writes U_{s+1}; U_1 = u, U_2 -> A, U_3 -> B, U_4 -> A, u^{n+1} -> u
        Prof *pf = p->prof.on ? &p->prof : nullptr;
        launch_rk4_stage<T>(p->box, p->tiles, 1, u, u, A, acc, dt, rhs, W, G, p->stream, pf);
        launch_rk4_stage<T>(p->box, p->tiles, 2, A, u, Bs, acc, dt, rhs, W, G, p->stream, pf);
        launch_rk4_stage<T>(p->box, p->tiles, 3, Bs, u, A, acc, dt, rhs, W, G, p->stream, pf);
        launch_rk4_stage<T>(p->box, p->tiles, 4, A, u, u, acc, dt, rhs, W, G, p->stream, pf);
        if (diag) launch_diag<T>(p->box, u, part, diag + (size_t)n * CNS_NDIAG, p->stream, pf);
        prof_flush(pf);
    }
}

extern "C" {

const char *cns_last_error(void) { return g_err; }

int cns_plan_create(cns_plan **out, const cns_grid *grid, const cns_physics *phys, int32_t precision, void *stream) {
    if (!out || !grid || !phys) return set_err(CNS_EINVAL, "null argument");
    *out = nullptr;
    if (grid->nx < 8 || grid->ny < 8 || grid->nz < 8)
        return set_err(CNS_EINVAL, "grid must have at least 8 points per direction (got %d x %d x %d)", grid->nx,
                       grid->ny, grid->nz);
    if (!(grid->lx > 0 && grid->ly > 0 && grid->lz > 0)) return set_err(CNS_EINVAL, "box lengths must be positive");
    if ((double)grid->nx * grid->ny * grid->nz * 5.0 > 9.0e18) return set_err(CNS_EINVAL, "grid too large");
    if (!(phys->gamma > 1.0)) return set_err(CNS_EINVAL, "gamma must exceed 1");
    if (!(phys->mu_eff >= 0.0) || !std::isfinite(phys->mu_eff)) return set_err(CNS_EINVAL, "mu_eff must be >= 0");
    if (phys->mu_eff > 0.0 && !(phys->prandtl > 0.0)) return set_err(CNS_EINVAL, "prandtl must be > 0");
    if (!(phys->weno_eps > 0.0)) return set_err(CNS_EINVAL, "weno_eps must be > 0");
    if (!(phys->harten_delta >= 0.0)) return set_err(CNS_EINVAL, "harten_delta must be >= 0");
    if (precision != CNS_FP64 && precision != CNS_MIXED) return set_err(CNS_EINVAL, "unknown precision %d", precision);
    cns_plan *p = new (std::nothrow) cns_plan();
    if (!p) return set_err(CNS_EINVAL, "out of host memory");
    p->box.nx = grid->nx;
    p->box.ny = grid->ny;
    p->box.nz = grid->nz;
    p->box.lx = grid->lx;
    p->box.ly = grid->ly;
    p->box.lz = grid->lz;
    p->box.ph = PhysT{phys->gamma, phys->prandtl, phys->mu_eff, phys->weno_eps, phys->harten_delta};
    p->precision = precision;
    p->stream = (hipStream_t)stream;
    p->wl = layout(p->box, precision == CNS_FP64 ? sizeof(double) : sizeof(float));
    *out = p;
    return CNS_OK;
}

int cns_plan_destroy(cns_plan *plan) {
    delete plan;
    return CNS_OK;
}

size_t cns_workspace_bytes(const cns_plan *plan) { return plan ? plan->wl.total : 0; }

int cns_set_workspace(cns_plan *plan, void *ws, size_t bytes) {
    if (!plan) return set_err(CNS_EINVAL, "null plan");
    if (!ws || !aligned(ws)) return set_err(CNS_EINVAL, "workspace must be non-null and 256-byte aligned");
    if (bytes < plan->wl.total)
        return set_err(CNS_EWORKSPACE, "workspace of %zu bytes required (got %zu)", plan->wl.total, bytes);
    plan->ws = (char *)ws;
    plan->ws_bytes = bytes;
    return CNS_OK;
}

int cns_set_tiles(cns_plan *plan, int32_t sx, int32_t sy, int32_t sz, int32_t block) {
    if (!plan) return set_err(CNS_EINVAL, "null plan");
    int32_t s[3] = {sx, sy, sz};
    int n[3] = {plan->box.nx, plan->box.ny, plan->box.nz};
    for (int d = 0; d < 3; ++d) {
        if (s[d] < 0) return set_err(CNS_EINVAL, "segment length must be >= 0");
        if (s[d] > 0) plan->tiles.seg[d] = s[d] > n[d] ? n[d] : s[d];
    }
    if (block != 0) {
        if (block < 64 || block > 256 || (block % 64) != 0)
            return set_err(CNS_EINVAL, "block must be 64, 128, 192 or 256");
        plan->tiles.block = block;
    }
    return CNS_OK;
}

int cns_init_state(const cns_plan *plan, const double *rho, const double *vel, const double *p, void *u) {
    int rc = check_plan(plan, false);
    if (!rc) rc = check_ptr(rho, "rho");
    if (!rc) rc = check_ptr(vel, "vel");
    if (!rc) rc = check_ptr(p, "p");
    if (!rc) rc = check_ptr(u, "u");
    if (rc) return rc;
    if (plan->precision == CNS_FP64)
        launch_init_state<double>(plan->box, rho, vel, p, (double *)u, plan->stream);
    else
        launch_init_state<float>(plan->box, rho, vel, p, (float *)u, plan->stream);
    return check_hip("init_state");
}

int cns_rhs(const cns_plan *plan, const void *u, void *rhs) {
    int rc = check_plan(plan, true);
    if (!rc) rc = check_ptr(u, "u");
    if (!rc) rc = check_ptr(rhs, "rhs");
    if (rc) return rc;
    if (u == rhs) return set_err(CNS_EINVAL, "u and rhs must not alias");
    if (plan->precision == CNS_FP64)
        launch_rhs<double>(plan->box, plan->tiles, (const double *)u, (double *)rhs, ws_at<double>(plan, plan->wl.W),
                           ws_at<double>(plan, plan->wl.G), plan->stream);
    else
        launch_rhs<float>(plan->box, plan->tiles, (const float *)u, (float *)rhs, ws_at<float>(plan, plan->wl.W),
                          ws_at<float>(plan, plan->wl.G), plan->stream);
    return check_hip("rhs");
}

int cns_rhs_dir(const cns_plan *plan, const void *u, int32_t dir, void *out) {
    int rc = check_plan(plan, false);
    if (!rc) rc = check_ptr(u, "u");
    if (!rc) rc = check_ptr(out, "out");
    if (rc) return rc;
    if (dir < 0 || dir > 2) return set_err(CNS_EINVAL, "dir must be 0, 1 or 2");
    if (u == out) return set_err(CNS_EINVAL, "u and out must not alias");
    if (plan->precision == CNS_FP64)
        launch_rhs_dir<double>(plan->box, plan->tiles, (const double *)u, dir, (double *)out, plan->stream);
    else
        launch_rhs_dir<float>(plan->box, plan->tiles, (const float *)u, dir, (float *)out, plan->stream);
    return check_hip("rhs_dir");
}

int cns_viscous(const cns_plan *plan, const void *u, void *out) {
    int rc = check_plan(plan, true);
    if (!rc) rc = check_ptr(u, "u");
    if (!rc) rc = check_ptr(out, "out");
    if (rc) return rc;
    if (u == out) return set_err(CNS_EINVAL, "u and out must not alias");
    if (plan->precision == CNS_FP64)
        launch_viscous<double>(plan->box, (const double *)u, (double *)out, ws_at<double>(plan, plan->wl.W),
                               ws_at<double>(plan, plan->wl.G), plan->stream);
    else
        launch_viscous<float>(plan->box, (const float *)u, (float *)out, ws_at<float>(plan, plan->wl.W),
                              ws_at<float>(plan, plan->wl.G), plan->stream);
    return check_hip("viscous");
}

int cns_rk4(cns_plan *plan, void *u, double dt, int32_t nsteps, double *diag) {
    int rc = check_plan(plan, true);
    if (!rc) rc = check_ptr(u, "u");
    if (rc) return rc;
    if (!(dt > 0.0) || !std::isfinite(dt)) return set_err(CNS_EINVAL, "dt must be positive and finite");
    if (nsteps < 0) return set_err(CNS_EINVAL, "nsteps must be >= 0");
    if (diag && ((uintptr_t)diag & 7u)) return set_err(CNS_EINVAL, "diag must be 8-byte aligned");
    if (plan->precision == CNS_FP64)
        rk4_steps<double>(plan, (double *)u, dt, nsteps, diag);
    else
        rk4_steps<float>(plan, (float *)u, dt, nsteps, diag);
    return check_hip("rk4");
}

int cns_diagnostics(const cns_plan *plan, const void *u, double *out) {
    int rc = check_plan(plan, true);
    if (!rc) rc = check_ptr(u, "u");
    if (rc) return rc;
    if (!out || ((uintptr_t)out & 7u)) return set_err(CNS_EINVAL, "out must be non-null and 8-byte aligned");
    double *part = ws_at<double>(plan, plan->wl.part);
    if (plan->precision == CNS_FP64)
        launch_diag<double>(plan->box, (const double *)u, part, out, plan->stream);
    else
        launch_diag<float>(plan->box, (const float *)u, part, out, plan->stream);
    return check_hip("diagnostics");
}

int cns_diagnostics_host(const cns_plan *plan, const void *u, double *out_host) {
    if (!out_host) return set_err(CNS_EINVAL, "out_host is null");
    int rc = check_plan(plan, true);
    if (rc) return rc;
    double *dev = ws_at<double>(plan, plan->wl.dhost);
    rc = cns_diagnostics(plan, u, dev);
    if (rc) return rc;
    hipError_t e = hipMemcpyAsync(out_host, dev, CNS_NDIAG * sizeof(double), hipMemcpyDeviceToHost, plan->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(plan->stream);
    if (e != hipSuccess) return set_err(CNS_EHIP, "diagnostics_host: %s", hipGetErrorString(e));
    if (out_host[8] > 0) {
        return set_err(std::isfinite(out_host[0]) ? CNS_ENONPHYSICAL : CNS_ENONFINITE,
                       "%.0f bad grid points (non-finite, rho <= 0 or p <= 0)", out_host[8]);
    }
    return CNS_OK;
}

int cns_profile_enable(cns_plan *plan, int32_t enable) {
    if (!plan) return set_err(CNS_EINVAL, "null plan");
    Prof &pf = plan->prof;
    if (enable && !pf.ev[0]) {
        for (auto &e : pf.ev)
            if (hipEventCreate(&e) != hipSuccess) return set_err(CNS_EHIP, "hipEventCreate failed");
    }
    pf.on = enable != 0;
    pf.n = 0;
    for (int k = 0; k < K_NKIND; ++k) {
        pf.ms[k] = 0.0;
        pf.count[k] = 0;
    }
    return CNS_OK;
}

int cns_profile_read(const cns_plan *plan, double *ms_host, int64_t *count_host) {
    if (!plan || !ms_host || !count_host) return set_err(CNS_EINVAL, "null argument");
    for (int k = 0; k < K_NKIND; ++k) {
        ms_host[k] = plan->prof.ms[k];
        count_host[k] = plan->prof.count[k];
    }
    return CNS_OK;
}

}  // extern "C"
