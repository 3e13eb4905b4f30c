// cns_api.hip -- the C-ABI (include/cns.h): argument checks, plans and ensembles,
// workspace carving, device tables, hipGraph capture, the tile autotuner, errors.
// All compute is enqueued through the launchers in cns_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "cns_adjoint.h"
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

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
static bool aligned(const void *p) { return ((uintptr_t)p & 255u) == 0; }

static int check_ptr(const void *ptr, const char *name) {
    if (!ptr) return set_err(CNS_EINVAL, "%s is null", name);
    if (!aligned(ptr)) return set_err(CNS_EINVAL, "%s is not 256-byte aligned", name);
    return CNS_OK;
}

static int validate(const cns_grid *g, const cns_physics *ph) {
    if (!g || !ph) return set_err(CNS_EINVAL, "null grid or physics");
    if (g->nx < 8 || g->ny < 8 || g->nz < 8)
        return set_err(CNS_EINVAL, "grid must have at least 8 points per direction (got %d x %d x %d)", g->nx, g->ny,
                       g->nz);
    // the sweeps address a component of a field (and the FP64 accumulator) with 32-bit byte
    // offsets: 8 n3 < 2^32
    if ((double)g->nx * g->ny * g->nz * 8.0 >= 4294967296.0)
        return set_err(CNS_EINVAL, "grid too large (at most 536870911 points per box)");
    if (!(g->lx > 0 && g->ly > 0 && g->lz > 0)) return set_err(CNS_EINVAL, "box lengths must be positive");
    if (!(ph->gamma > 1.0) || !std::isfinite(ph->gamma)) return set_err(CNS_EINVAL, "gamma must exceed 1");
    if (!(ph->mu_eff >= 0.0) || !std::isfinite(ph->mu_eff)) return set_err(CNS_EINVAL, "mu_eff must be >= 0");
    if (ph->mu_eff > 0.0 && !(ph->prandtl > 0.0)) return set_err(CNS_EINVAL, "prandtl must be > 0");
    // products of up to eight (eps + beta) factors are formed in FP64 (the two weight
    // denominators of an interface share one reciprocal; eps is rounded to FP32 in the
    // mixed form): eps outside [1e-30, 1e30] would leave their range
    if (!(ph->weno_eps >= 1e-30 && ph->weno_eps <= 1e30))
        return set_err(CNS_EINVAL, "weno_eps must lie in [1e-30, 1e30] (got %g)", ph->weno_eps);
    if (!(ph->harten_delta >= 0.0)) return set_err(CNS_EINVAL, "harten_delta must be >= 0");
    if (ph->weno_weights != CNS_WENO_JS && ph->weno_weights != CNS_WENO_Z && ph->weno_weights != CNS_WENO_M)
        return set_err(CNS_EINVAL, "unknown weno_weights %d", ph->weno_weights);
    return CNS_OK;
}

// ----------------------------------------------------------------------------
// Core: a batch of boxes with its workspace, device tables, profiling and graphs
// ----------------------------------------------------------------------------
struct Core {
    int prec = CNS_FP64;
    size_t esz = 8;
    hipStream_t stream = nullptr;
    int block = 256;
    int xrows_pref = 1;
    std::vector<BoxDesc> boxes;
    std::vector<void *> ustate;  // per-box state pointer (ensembles) or null (plans)
    std::vector<char> active;    // boxes given blocks (all, except while autotuning)
    std::vector<int> rows_ov;    // rows per block of the x rows kernel per box (0: default)
    long long grid[F_N] = {};    // launched blocks per kernel family (0: one per virtual block)
    // workspace layout
    std::vector<size_t> box_off;  // per-box scratch base
    size_t table_off = 0, dhost_off = 0, gp_off = 0, need = 0;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    bool dirty = true;
    std::vector<unsigned char> staging;
    long long total[F_N] = {};
    int rowP = 1;
    size_t rowLds = 0;
    bool any_visc = false;
    int weights = CNS_WENO_JS;
    Prof prof;
    bool use_graph = false;
    hipGraphExec_t gexec = nullptr;
    bool g_diag_on = false;
    int g_nsteps = -1, g_scheme = -1;
    long long captures = 0;  // graph captures so far (replays reuse one)
    int scheme = CNS_RK4;  // integrator of cns_ensemble_run

    ~Core() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (prof.ev[0])
            for (auto &e : prof.ev) (void)hipEventDestroy(e);
    }

    int nbox() const { return (int)boxes.size(); }

    static size_t box_scratch_bytes(const BoxDesc &b, size_t esz) {
        size_t n3 = b.n3, off = 0;
        auto take = [&](size_t bytes) { off = align256(off + bytes); };
        take(9 * n3 * esz);  // G
        take(5 * n3 * esz);  // rhs
        take(5 * n3 * esz);  // A
        take(5 * n3 * esz);  // B
        take(5 * n3 * sizeof(double));                         // acc
        take(diag_part_slots(b.nx, b.ny, b.nz) * CNS_NDIAG * sizeof(double));  // part
        return off;
    }

    void layout() {
        size_t off = 0;
        box_off.resize(boxes.size());
        for (size_t i = 0; i < boxes.size(); ++i) {
            box_off[i] = off;
            off += box_scratch_bytes(boxes[i], esz);
        }
        table_off = off;
        off = align256(off + boxes.size() * sizeof(BoxDesc) + (size_t)F_N * (boxes.size() + 1) * sizeof(long long));
        dhost_off = off;
        off = align256(off + CNS_NDIAG * sizeof(double));
        gp_off = off;
        off = align256(off + sizeof(GraphParams));
        need = off;
    }

    void add_box(const cns_grid &g, const cns_physics &ph, double dt, void *u) {
        boxes.push_back(make_box(g, ph, dt));
        weights = ph.weno_weights;
        ustate.push_back(u);
        active.push_back(1);
        rows_ov.push_back(0);
    }

    // shape, spacings, physics and default segment lengths of a box
    static BoxDesc make_box(const cns_grid &g, const cns_physics &ph, double dt) {
        BoxDesc b{};
        b.nx = g.nx;
        b.ny = g.ny;
        b.nz = g.nz;
        // default marching-segment length: 16, doubled (up to 128) while the launch still
        // has at least 2^19 threads (four rounds of two waves per SIMD over 256 CUs); longer
        // segments recompute fewer halo interfaces, shorter ones fill the chip (512^3:
        // 128 points, 0.4 % faster per step than 64 with the same bits)
        const long long nlen[3] = {g.nx, g.ny, g.nz};
        for (int d = 0; d < 3; ++d) {
            const long long lines = (long long)g.nx * g.ny * g.nz / nlen[d];
            int seg = 16;
            while (seg < 128 && lines * ((nlen[d] + 2 * seg - 1) / (2 * seg)) >= (1ll << 19)) seg *= 2;
            b.seg[d] = seg;
        }
        b.n3 = (size_t)g.nx * g.ny * g.nz;
        b.inv_h[0] = g.nx / g.lx;
        b.inv_h[1] = g.ny / g.ly;
        b.inv_h[2] = g.nz / g.lz;
        b.gamma = ph.gamma;
        b.prandtl = ph.prandtl;
        b.mu = ph.mu_eff;
        b.eps = ph.weno_eps;
        b.delta = ph.harten_delta;
        b.dt = dt;
        return b;
    }

    // fill pointers, shapes and prefixes; upload the device table (synchronous)
    int sync_table() {
        if (!dirty) return CNS_OK;
        if (!ws) return set_err(CNS_EWORKSPACE, "no workspace bound");
        const int n = nbox();
        std::vector<long long> off[F_N];
        rowP = 1;
        rowLds = 0;
        any_visc = false;
        for (int i = 0; i < n; ++i) {
            BoxDesc &b = boxes[i];
            const size_t n3 = b.n3;
            char *base = ws + box_off[i];
            size_t o = 0;
            auto take = [&](size_t bytes) {
                char *p = base + o;
                o = align256(o + bytes);
                return (void *)p;
            };
            b.G = take(9 * n3 * esz);
            b.rhs = take(5 * n3 * esz);
            b.A = take(5 * n3 * esz);
            b.B = take(5 * n3 * esz);
            b.acc = (double *)take(5 * n3 * sizeof(double));
            b.part = (double *)take(diag_part_slots(b.nx, b.ny, b.nz) * CNS_NDIAG * sizeof(double));
            b.u = ustate[i];
            int P = 1;
            b.rows = rows_ov[i] > 0 && rows_fit(b.nx, rows_ov[i], esz, nullptr) ? rows_ov[i] : rows_for(b.nx);
            // rows longer than a block go through the chunked rows kernel
            b.xrows = !xrows_pref ? 0 : (b.nx > kRowThreads ? 2 : (rows_fit(b.nx, b.rows, esz, &P) ? 1 : 0));
            if (b.xrows == 1) {
                rowP = std::max(rowP, P);
                rowLds = std::max(rowLds, (size_t)14 * b.rows * b.nx * esz);
            }
            for (int d = 0; d < 3; ++d) {
                const int nl = d == 0 ? b.nx : (d == 1 ? b.ny : b.nz);
                b.seg[d] = std::max(1, std::min(b.seg[d], nl));
            }
            any_visc = any_visc || b.mu > 0.0;
        }
        for (int f = 0; f < F_N; ++f) {
            off[f].assign(n + 1, 0);
            for (int i = 0; i < n; ++i) off[f][i + 1] = off[f][i] + (active[i] ? family_blocks(boxes[i], f, block) : 0);
            total[f] = off[f][n];
        }
        const size_t tb = n * sizeof(BoxDesc) + (size_t)F_N * (n + 1) * sizeof(long long);
        staging.assign(tb, 0);
        memcpy(staging.data(), boxes.data(), n * sizeof(BoxDesc));
        for (int f = 0; f < F_N; ++f)
            memcpy(staging.data() + n * sizeof(BoxDesc) + (size_t)f * (n + 1) * sizeof(long long), off[f].data(),
                   (n + 1) * sizeof(long long));
        hipError_t e = hipMemcpyAsync(ws + table_off, staging.data(), tb, hipMemcpyHostToDevice, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return set_err(CNS_EHIP, "table upload: %s", hipGetErrorString(e));
        dirty = false;
        drop_graph();
        return CNS_OK;
    }

    Batch batch() {
        Batch bt;
        bt.nbox = nbox();
        bt.prec = prec;
        bt.block = block;
        bt.any_visc = any_visc;
        bt.weights = weights;
        bt.d_boxes = (const BoxDesc *)(ws + table_off);
        const long long *offs = (const long long *)(ws + table_off + nbox() * sizeof(BoxDesc));
        for (int f = 0; f < F_N; ++f) {
            bt.d_off[f] = offs + (size_t)f * (nbox() + 1);
            bt.total[f] = total[f];
        }
        bt.rowP = rowP;
        // with one point per thread the rows kernel lays its fields 256 points apart
        bt.rowLds = rowP == 1 && rowLds > 0 ? (size_t)14 * kRowThreads * esz : rowLds;
        bt.esz = esz;
        for (int f = 0; f < F_N; ++f) bt.grid[f] = grid[f];
        bt.stream = stream;
        bt.prof = prof.on ? &prof : nullptr;
        return bt;
    }

    void drop_graph() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        gexec = nullptr;
        g_nsteps = -1;
    }

    // nsteps steps of the integrator `sch`; diag layout [nbox][nsteps][CNS_NDIAG].
    // A graph run captures the launches once per (integrator, nsteps, diagnostics on or
    // off); the state, step size and diagnostics base of each call reach the captured
    // kernels through the GraphParams record, written by a kernel before every replay.
    int run(int sch, const void *u_ov, double dt_ov, int nsteps, double *diag) {
        int rc = sync_table();
        if (rc) return rc;
        Batch bt = batch();
        const bool graph = use_graph && !prof.on && nsteps > 0;
        if (graph && !stream) return set_err(CNS_EUNSUPPORTED, "graph replay needs a non-default stream");
        GraphParams *gp = (GraphParams *)(ws + gp_off);
        if (graph) bt.gp = gp;
        const void *u_l = graph ? nullptr : u_ov;
        const double dt_l = graph ? 0.0 : dt_ov;
        // a step's diagnostics are formed by the next step's first viscous-flux launch,
        // which reads that state anyway (FP64, viscous batches); the last step's by the
        // diagnostics kernels
        const bool fuse = diag && diag_fusable(bt);
        auto enqueue = [&]() {
            for (int n = 0; n < nsteps; ++n) {
                launch_step(bt, sch, u_l, dt_l, diag, nsteps, n, nullptr, fuse && n > 0 ? n - 1 : -1,
                            !fuse || n == nsteps - 1);
                prof_flush(bt.prof);
            }
        };
        if (!graph) {
            enqueue();
            return check_hip("rk4");
        }
        if (!(gexec && g_nsteps == nsteps && g_scheme == sch && g_diag_on == (diag != nullptr))) {
            drop_graph();
            hipGraph_t graph_h = nullptr;
            hipError_t e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return set_err(CNS_EHIP, "begin capture: %s", hipGetErrorString(e));
            enqueue();
            e = hipStreamEndCapture(stream, &graph_h);
            if (e != hipSuccess) return set_err(CNS_EHIP, "end capture: %s", hipGetErrorString(e));
            e = hipGraphInstantiate(&gexec, graph_h, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph_h);
            if (e != hipSuccess) {
                gexec = nullptr;
                return set_err(CNS_EHIP, "graph instantiate: %s", hipGetErrorString(e));
            }
            g_scheme = sch;
            g_diag_on = diag != nullptr;
            g_nsteps = nsteps;
            ++captures;
        }
        launch_set_params(gp, u_ov, diag, dt_ov, stream);
        if ((rc = check_hip("graph parameters"))) return rc;
        hipError_t e = hipGraphLaunch(gexec, stream);
        if (e != hipSuccess) return set_err(CNS_EHIP, "graph launch: %s", hipGetErrorString(e));
        return CNS_OK;
    }

    int profile_enable(int on) {
        if (on && !prof.ev[0])
            for (auto &e : prof.ev)
                if (hipEventCreate(&e) != hipSuccess) return set_err(CNS_EHIP, "hipEventCreate failed");
        prof.on = on != 0;
        prof.n = 0;
        for (int k = 0; k < K_NKIND; ++k) {
            prof.ms[k] = 0.0;
            prof.count[k] = 0;
        }
        return CNS_OK;
    }
};

struct cns_plan {
    Core c;
};
struct cns_ensemble {
    Core c;
};

// ----------------------------------------------------------------------------
// diagnostics with no allocation: device scratch in a static array
// ----------------------------------------------------------------------------
// The scratch of cns_diagnostics_static: the one-box device table and the per-block
// partial sums (at most kDiagBlocksMax records, whatever the grid size).  Each GPU the
// library runs on holds its own copy until the process ends; calls on one GPU share it.
constexpr size_t kStaticScratchBytes = 128 * 1024;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
constexpr int kMaxDevices = 64;
static char *g_scratch_ptr[kMaxDevices];
static std::mutex g_scratch_mu;

// The device address of `scratch` on the current device.  In host code the array's name
// stands for a host-side shadow, so the address is taken with hipGetSymbolAddress, once
// per device with that device current, and only that address reaches the kernels.
static int static_scratch(char **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return set_err(CNS_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return set_err(CNS_EUNSUPPORTED, "device %d (at most %d devices)", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_err(CNS_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = (char *)p;
    }
    *out = g_scratch_ptr[dev];
    return CNS_OK;
}

// ----------------------------------------------------------------------------
// autotuner: segment length of the marching y/z sweeps per box size, then the
// block size of the batch.  The choice never changes results (bitwise).
// ----------------------------------------------------------------------------
static std::string arch_name() {
    int dev = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
    std::string s = p.gcnArchName;
    size_t c = s.find(':');
    return c == std::string::npos ? s : s.substr(0, c);
}

static std::map<std::string, int> read_cache(const char *path) {
    std::map<std::string, int> m;
    if (!path) return m;
    FILE *f = fopen(path, "r");
    if (!f) return m;
    char key[256];
    int val;
    // format: one `"key": value` pair per line inside braces
    char line[512];
    while (fgets(line, sizeof line, f))
        if (sscanf(line, " \"%255[^\"]\" : %d", key, &val) == 2) m[key] = val;
    fclose(f);
    return m;
}

static void write_cache(const char *path, const std::map<std::string, int> &m) {
    if (!path) return;
    FILE *f = fopen(path, "w");
    if (!f) return;
    fprintf(f, "{\n");
    size_t i = 0;
    for (auto &kv : m) fprintf(f, "  \"%s\": %d%s\n", kv.first.c_str(), kv.second, ++i < m.size() ? "," : "");
    fprintf(f, "}\n");
    fclose(f);
}

static int autotune(Core &c, const char *cache_path) {
    int rc = c.sync_table();
    if (rc) return rc;
    const std::string pre = arch_name() + (c.prec == CNS_FP64 ? "|fp64|" : "|mixed|");
    std::map<std::string, int> cache = read_cache(cache_path);
    bool changed = false;
    // size classes
    std::map<std::string, std::vector<int>> cls;
    for (int i = 0; i < c.nbox(); ++i) {
        const BoxDesc &b = c.boxes[i];
        char k[64];
        snprintf(k, sizeof k, "%dx%dx%d|mu%d", b.nx, b.ny, b.nz, b.mu > 0 ? 1 : 0);
        cls[k].push_back(i);
    }
    std::vector<BoxDesc> saved = c.boxes;
    std::vector<int> saved_rows = c.rows_ov;
    // time one size class alone (other boxes get no blocks; every kernel skips them)
    auto only = [&](const std::vector<int> &members) {
        for (int i = 0; i < c.nbox(); ++i)
            c.active[i] = std::find(members.begin(), members.end(), i) != members.end();
    };
    // 1. segment length of the marching y/z sweeps per size class
    const int segs[] = {4, 8, 16, 32, 64};
    for (auto &kv : cls) {
        const std::string key = pre + kv.first + "|seg";
        int best = -1;
        auto it = cache.find(key);
        const BoxDesc &bk = c.boxes[kv.second[0]];
        if (it != cache.end() && it->second >= 1 && it->second <= std::max(bk.ny, bk.nz)) {
            best = it->second;
        } else {
            float best_ms = 1e30f;
            for (int sgl : segs) {
                if (sgl > std::max(bk.ny, bk.nz)) continue;
                c.boxes = saved;
                only(kv.second);
                for (int i : kv.second) c.boxes[i].seg[1] = c.boxes[i].seg[2] = sgl;
                c.dirty = true;
                if ((rc = c.sync_table())) return rc;
                Batch bt = c.batch();
                time_sweeps_yz(bt, 1);  // warm
                float ms = time_sweeps_yz(bt, 3);
                if (ms < best_ms) {
                    best_ms = ms;
                    best = sgl;
                }
            }
            cache[key] = best;
            changed = true;
        }
        for (int i : kv.second) saved[i].seg[1] = saved[i].seg[2] = best;
    }
    c.boxes = saved;
    // 2. rows per block of the x rows kernel per size class: the default (a power of two)
    // and every count with the same points per thread that keeps at least 90 % of the
    // block's threads busy and fits.  The points per thread are a template parameter of
    // the kernel, and another instantiation may contract multiplies and adds into fused
    // operations differently, so only counts with the default's points per thread keep
    // results bitwise independent of the choice.
    for (auto &kv : cls) {
        const int nx = c.boxes[kv.second[0]].nx;
        const std::string key = pre + kv.first + "|rows";
        auto it = cache.find(key);
        int best = 0;
        if (it != cache.end() && it->second >= 0 && (it->second == 0 || rows_fit(nx, it->second, c.esz, nullptr))) {
            best = it->second;
        } else if (c.xrows_pref && nx <= kRowThreads && rows_fit(nx, rows_for(nx), c.esz, nullptr)) {
            std::vector<int> cand = {0};
            int P0 = 0;
            rows_fit(nx, rows_for(nx), c.esz, &P0);
            for (int r = 1; r <= 1024 / nx && (int)cand.size() < 6; ++r) {
                int P = 0;
                if (r == rows_for(nx) || !rows_fit(nx, r, c.esz, &P) || P != P0) continue;
                if ((double)r * nx / (kRowThreads * P) >= 0.9) cand.push_back(r);
            }
            float best_ms = 1e30f;
            for (int r : cand) {
                only(kv.second);
                for (int i : kv.second) c.rows_ov[i] = r;
                c.dirty = true;
                if ((rc = c.sync_table())) return rc;
                Batch bt = c.batch();
                time_rhs_kernels(bt, 1);
                float ms = time_rhs_kernels(bt, 3);
                if (ms < best_ms) {
                    best_ms = ms;
                    best = r;
                }
            }
            cache[key] = best;
            changed = true;
        }
        for (int i : kv.second) saved_rows[i] = best;
    }
    c.rows_ov = saved_rows;
    for (int i = 0; i < c.nbox(); ++i) c.active[i] = 1;
    std::string all = "";
    for (auto &kv : cls) all += "|" + kv.first + "x" + std::to_string(kv.second.size());
    // 3. block size of the marching sweeps, for the whole batch
    const std::string bkey = pre + "block" + all;
    auto bit = cache.find(bkey);
    const bool valid = bit != cache.end() && (bit->second == 64 || bit->second == 128 || bit->second == 192 ||
                                              bit->second == 256);
    if (valid) {
        c.block = bit->second;
    } else {
        float best_ms = 1e30f;
        int best = 256;
        for (int blk : {64, 128, 256}) {
            c.block = blk;
            c.dirty = true;
            if ((rc = c.sync_table())) return rc;
            Batch bt = c.batch();
            time_sweeps_yz(bt, 1);
            float ms = time_sweeps_yz(bt, 3);
            if (ms < best_ms) {
                best_ms = ms;
                best = blk;
            }
        }
        c.block = best;
        cache[bkey] = best;
        changed = true;
    }
    // 4. launched grids: one block per virtual block, or persistent grids of one or two
    // rounds of the blocks the chip holds at once, for the marching sweeps and for the
    // tiled viscous-flux and diagnostics kernels (code 10 * sweeps + tiles)
    c.dirty = true;
    if ((rc = c.sync_table())) return rc;
    {
        Batch bt0 = c.batch();
        const long long Rs = resident_sweep_blocks(bt0), Rt = resident_tile_blocks(bt0);
        const std::string gkey = pre + "grid|b" + std::to_string(c.block) + all;
        auto git = cache.find(gkey);
        int best = 0;
        if (git != cache.end() && git->second >= 0 && git->second <= 22 && git->second % 10 <= 2) {
            best = git->second;
        } else {
            float best_ms = 1e30f;
            for (int gs = 0; gs <= 2; ++gs)
                for (int gt = 0; gt <= 2; ++gt) {
                    Batch bt = c.batch();
                    for (int f = F_SWEEP_X; f <= F_SWEEP_Z; ++f) bt.grid[f] = gs * Rs;
                    bt.grid[F_VISC] = bt.grid[F_DIAG] = gt * Rt;
                    time_rhs_kernels(bt, 1);
                    float ms = time_rhs_kernels(bt, 3);
                    if (ms < best_ms) {
                        best_ms = ms;
                        best = 10 * gs + gt;
                    }
                }
            cache[gkey] = best;
            changed = true;
        }
        for (int f = F_SWEEP_X; f <= F_SWEEP_Z; ++f) c.grid[f] = (best / 10) * Rs;
        c.grid[F_VISC] = c.grid[F_DIAG] = (best % 10) * Rt;
    }
    c.dirty = true;
    if ((rc = c.sync_table())) return rc;
    if (changed) write_cache(cache_path, cache);
    return check_hip("autotune");
}

// ----------------------------------------------------------------------------
// C-ABI
// ----------------------------------------------------------------------------
static int check_plan(const cns_plan *p) {
    if (!p) return set_err(CNS_EINVAL, "null plan");
    if (!p->c.ws) return set_err(CNS_EWORKSPACE, "workspace of %zu bytes required (none bound)", p->c.need);
    return CNS_OK;
}

extern "C" {

const char *cns_last_error(void) { return g_err; }

int cns_stream_copy(const void *src, void *dst, size_t bytes, void *stream) {
    if (!src || !dst || ((uintptr_t)src & 15u) || ((uintptr_t)dst & 15u))
        return set_err(CNS_EINVAL, "src and dst must be non-null and 16-byte aligned");
    if (bytes % 16) return set_err(CNS_EINVAL, "bytes must be a multiple of 16");
    const char *a = (const char *)src, *b = (const char *)dst;
    if (a < b + bytes && b < a + bytes) return set_err(CNS_EINVAL, "src and dst overlap");
    launch_stream_copy(src, dst, bytes, (hipStream_t)stream);
    return check_hip("stream_copy");
}

int cns_plan_create(cns_plan **out, const cns_grid *grid, const cns_physics *phys, int32_t precision, void *stream) {
    if (!out) return set_err(CNS_EINVAL, "null output pointer");
    *out = nullptr;
    int rc = validate(grid, phys);
    if (rc) return rc;
    if (precision != CNS_FP64 && precision != CNS_MIXED) return set_err(CNS_EINVAL, "unknown precision %d", precision);
    cns_plan *p = new (std::nothrow) cns_plan();
    if (!p) return set_err(CNS_EINVAL, "out of host memory");
    p->c.prec = precision;
    p->c.esz = precision == CNS_FP64 ? sizeof(double) : sizeof(float);
    p->c.stream = (hipStream_t)stream;
    p->c.add_box(*grid, *phys, 0.0, nullptr);
    p->c.layout();
    *out = p;
    return CNS_OK;
}

int cns_plan_destroy(cns_plan *plan) {
    delete plan;
    return CNS_OK;
}

size_t cns_workspace_bytes(const cns_plan *plan) { return plan ? plan->c.need : 0; }

int cns_set_workspace(cns_plan *plan, void *ws, size_t bytes) {
    if (!plan) return set_err(CNS_EINVAL, "null plan");
    if (!ws || !aligned(ws)) return set_err(CNS_EINVAL, "workspace must be non-null and 256-byte aligned");
    if (bytes < plan->c.need)
        return set_err(CNS_EWORKSPACE, "workspace of %zu bytes required (got %zu)", plan->c.need, bytes);
    plan->c.ws = (char *)ws;
    plan->c.ws_bytes = bytes;
    plan->c.dirty = true;
    return plan->c.sync_table();
}

int cns_set_tiles(cns_plan *plan, int32_t sx, int32_t sy, int32_t sz, int32_t block) {
    if (!plan) return set_err(CNS_EINVAL, "null plan");
    const int32_t s[3] = {sx, sy, sz};
    for (int d = 0; d < 3; ++d)
        if (s[d] < 0) return set_err(CNS_EINVAL, "segment length must be >= 0");
    if (block != 0 && (block < 64 || block > 256 || (block % 64) != 0))
        return set_err(CNS_EINVAL, "block must be 64, 128, 192 or 256");
    for (int d = 0; d < 3; ++d)
        if (s[d] > 0) plan->c.boxes[0].seg[d] = s[d];
    if (block) plan->c.block = block;
    plan->c.dirty = true;
    return plan->c.ws ? plan->c.sync_table() : CNS_OK;
}

int cns_set_x_kernel(cns_plan *plan, int32_t kind) {
    if (!plan) return set_err(CNS_EINVAL, "null plan");
    if (kind != 0 && kind != 1) return set_err(CNS_EINVAL, "x kernel kind must be 0 (rows in LDS) or 1 (marching)");
    plan->c.xrows_pref = kind == 0 ? 1 : 0;
    plan->c.dirty = true;
    return plan->c.ws ? plan->c.sync_table() : CNS_OK;
}

int cns_set_graph(cns_plan *plan, int32_t enable) {
    if (!plan) return set_err(CNS_EINVAL, "null plan");
    if (enable && !plan->c.stream) return set_err(CNS_EUNSUPPORTED, "graph replay needs a non-default stream");
    plan->c.use_graph = enable != 0;
    plan->c.drop_graph();
    return CNS_OK;
}

int cns_init_state(const cns_plan *plan, const double *rho, const double *vel, const double *p, void *u) {
    if (!plan) return set_err(CNS_EINVAL, "null plan");
    int rc = check_ptr(rho, "rho");
    if (!rc) rc = check_ptr(vel, "vel");
    if (!rc) rc = check_ptr(p, "p");
    if (!rc) rc = check_ptr(u, "u");
    if (rc) return rc;
    const BoxDesc &b = plan->c.boxes[0];
    launch_init_state(plan->c.prec, b.n3, b.gamma, rho, vel, p, u, plan->c.stream);
    return check_hip("init_state");
}

int cns_rhs(const cns_plan *plan, const void *u, void *rhs) {
    int rc = check_plan(plan);
    if (!rc) rc = check_ptr(u, "u");
    if (!rc) rc = check_ptr(rhs, "rhs");
    if (rc) return rc;
    if (u == rhs) return set_err(CNS_EINVAL, "u and rhs must not alias");
    cns_plan *p = const_cast<cns_plan *>(plan);
    if ((rc = p->c.sync_table())) return rc;
    launch_rhs(p->c.batch(), u, rhs);
    return check_hip("rhs");
}

int cns_rhs_dir(const cns_plan *plan, const void *u, int32_t dir, void *out) {
    int rc = check_plan(plan);
    if (!rc) rc = check_ptr(u, "u");
    if (!rc) rc = check_ptr(out, "out");
    if (rc) return rc;
    if (dir < 0 || dir > 2) return set_err(CNS_EINVAL, "dir must be 0, 1 or 2");
    if (u == out) return set_err(CNS_EINVAL, "u and out must not alias");
    cns_plan *p = const_cast<cns_plan *>(plan);
    if ((rc = p->c.sync_table())) return rc;
    launch_rhs_dir(p->c.batch(), u, dir, out);
    return check_hip("rhs_dir");
}

int cns_viscous(const cns_plan *plan, const void *u, void *out) {
    int rc = check_plan(plan);
    if (!rc) rc = check_ptr(u, "u");
    if (!rc) rc = check_ptr(out, "out");
    if (rc) return rc;
    if (u == out) return set_err(CNS_EINVAL, "u and out must not alias");
    cns_plan *p = const_cast<cns_plan *>(plan);
    if ((rc = p->c.sync_table())) return rc;
    if (!(p->c.boxes[0].mu > 0.0)) launch_fill(p->c.prec, 5 * p->c.boxes[0].n3, out, p->c.stream);
    else launch_viscous(p->c.batch(), u, out);
    return check_hip("viscous");
}

int cns_rk4(cns_plan *plan, void *u, double dt, int32_t nsteps, double *diag) {
    int rc = check_plan(plan);
    if (!rc) rc = check_ptr(u, "u");
    if (rc) return rc;
    if (!(dt > 0.0) || !std::isfinite(dt)) return set_err(CNS_EINVAL, "dt must be positive and finite");
    if (nsteps < 0) return set_err(CNS_EINVAL, "nsteps must be >= 0");
    if (diag && ((uintptr_t)diag & 7u)) return set_err(CNS_EINVAL, "diag must be 8-byte aligned");
    return plan->c.run(CNS_RK4, u, dt, nsteps, diag);
}

int cns_tvdrk3(cns_plan *plan, void *u, double dt, int32_t nsteps, double *diag) {
    int rc = check_plan(plan);
    if (!rc) rc = check_ptr(u, "u");
    if (rc) return rc;
    if (!(dt > 0.0) || !std::isfinite(dt)) return set_err(CNS_EINVAL, "dt must be positive and finite");
    if (nsteps < 0) return set_err(CNS_EINVAL, "nsteps must be >= 0");
    if (diag && ((uintptr_t)diag & 7u)) return set_err(CNS_EINVAL, "diag must be 8-byte aligned");
    return plan->c.run(CNS_TVDRK3, u, dt, nsteps, diag);
}

int cns_spectrum_shells(const cns_plan *plan) {
    int rc = check_plan(plan);
    if (rc) return rc;
    return spectrum_shells(plan->c.boxes[0]);
}

int cns_spectrum(const cns_plan *plan, const void *u, double *E, int32_t nshell, double *mom) {
    int rc = check_plan(plan);
    if (!rc) rc = check_ptr(u, "u");
    if (rc) return rc;
    if (!E || !mom || ((uintptr_t)E & 7u) || ((uintptr_t)mom & 7u))
        return set_err(CNS_EINVAL, "E and moments must be non-null and 8-byte aligned");
    cns_plan *p = const_cast<cns_plan *>(plan);
    if ((rc = p->c.sync_table())) return rc;
    const BoxDesc &b = p->c.boxes[0];
    if (nshell != spectrum_shells(b))
        return set_err(CNS_EINVAL, "nshell must be %d for this grid (got %d)", spectrum_shells(b), nshell);
    if (!spectrum_supported(b)) return set_err(CNS_EUNSUPPORTED, "spectrum needs every grid dimension <= 2047 and at most 4096 shells");
    launch_spectrum(b, p->c.prec, p->c.stream, u, E, nshell, mom);
    return check_hip("spectrum");
}

int cns_diagnostics(const cns_plan *plan, const void *u, double *out) {
    int rc = check_plan(plan);
    if (!rc) rc = check_ptr(u, "u");
    if (rc) return rc;
    if (!out || ((uintptr_t)out & 7u)) return set_err(CNS_EINVAL, "out must be non-null and 8-byte aligned");
    cns_plan *p = const_cast<cns_plan *>(plan);
    if ((rc = p->c.sync_table())) return rc;
    launch_diag(p->c.batch(), u, out, 0, 0);
    return check_hip("diagnostics");
}

int cns_diagnostics_host(const cns_plan *plan, const void *u, double *out_host) {
    if (!out_host) return set_err(CNS_EINVAL, "out_host is null");
    int rc = check_plan(plan);
    if (rc) return rc;
    double *dev = (double *)(plan->c.ws + plan->c.dhost_off);
    rc = cns_diagnostics(plan, u, dev);
    if (rc) return rc;
    hipError_t e = hipMemcpyAsync(out_host, dev, CNS_NDIAG * sizeof(double), hipMemcpyDeviceToHost, plan->c.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(plan->c.stream);
    if (e != hipSuccess) return set_err(CNS_EHIP, "diagnostics_host: %s", hipGetErrorString(e));
    if (out_host[8] > 0)
        return set_err(std::isfinite(out_host[0]) ? CNS_ENONPHYSICAL : CNS_ENONFINITE,
                       "%.0f bad grid points (non-finite, rho <= 0 or p <= 0)", out_host[8]);
    return CNS_OK;
}

int cns_diagnostics_static(const cns_grid *grid, const cns_physics *phys, int32_t precision, const void *u,
                           double *out, void *stream) {
    int rc = validate(grid, phys);
    if (rc) return rc;
    if (precision != CNS_FP64 && precision != CNS_MIXED) return set_err(CNS_EINVAL, "unknown precision %d", precision);
    if ((rc = check_ptr(u, "u"))) return rc;
    if (!out || ((uintptr_t)out & 7u)) return set_err(CNS_EINVAL, "out must be non-null and 8-byte aligned");
    if (static_diag_bytes() > kStaticScratchBytes)
        return set_err(CNS_EUNSUPPORTED, "diagnostics need %zu bytes of scratch, the static array holds %zu",
                       static_diag_bytes(), kStaticScratchBytes);
    char *ptr = nullptr;
    if ((rc = static_scratch(&ptr))) return rc;
    launch_diag_static(ptr, Core::make_box(*grid, *phys, 0.0), precision, u, out, (hipStream_t)stream);
    return check_hip("diagnostics_static");
}

int cns_max_wave_speed(const cns_plan *plan, const void *u, double *out) {
    int rc = check_plan(plan);
    if (!rc) rc = check_ptr(u, "u");
    if (rc) return rc;
    if (!out || ((uintptr_t)out & 7u)) return set_err(CNS_EINVAL, "out must be non-null and 8-byte aligned");
    cns_plan *p = const_cast<cns_plan *>(plan);
    if ((rc = p->c.sync_table())) return rc;
    launch_max_wave_speed(p->c.batch(), u, out);
    return check_hip("max_wave_speed");
}

int64_t cns_plan_graph_captures(const cns_plan *plan) {
    if (!plan) return set_err(CNS_EINVAL, "null plan");
    return plan->c.captures;
}

int cns_profile_enable(cns_plan *plan, int32_t enable) {
    if (!plan) return set_err(CNS_EINVAL, "null plan");
    return plan->c.profile_enable(enable);
}

int cns_profile_read(const cns_plan *plan, double *ms_host, int64_t *count_host) {
    if (!plan || !ms_host || !count_host) return set_err(CNS_EINVAL, "null argument");
    for (int k = 0; k < K_NKIND; ++k) {
        ms_host[k] = plan->c.prof.ms[k];
        count_host[k] = plan->c.prof.count[k];
    }
    return CNS_OK;
}

// ---- ensembles ---------------------------------------------------------------
int cns_ensemble_create(cns_ensemble **out, int32_t nbox, const cns_grid *grids, const cns_physics *phys,
                        const double *dt, int32_t precision, void *u_packed, const int64_t *offsets, void *stream) {
    if (!out) return set_err(CNS_EINVAL, "null output pointer");
    *out = nullptr;
    if (nbox < 1 || nbox > 65536) return set_err(CNS_EINVAL, "nbox must be in [1, 65536]");
    if (!grids || !phys || !dt || !offsets) return set_err(CNS_EINVAL, "null argument");
    if (precision != CNS_FP64 && precision != CNS_MIXED) return set_err(CNS_EINVAL, "unknown precision %d", precision);
    if (!u_packed || !aligned(u_packed)) return set_err(CNS_EINVAL, "u_packed must be non-null and 256-byte aligned");
    const size_t esz = precision == CNS_FP64 ? sizeof(double) : sizeof(float);
    cns_ensemble *e = new (std::nothrow) cns_ensemble();
    if (!e) return set_err(CNS_EINVAL, "out of host memory");
    e->c.prec = precision;
    e->c.esz = esz;
    e->c.stream = (hipStream_t)stream;
    for (int i = 0; i < nbox; ++i) {
        int rc = validate(&grids[i], &phys[i]);
        if (!rc && (!(dt[i] > 0.0) || !std::isfinite(dt[i]))) rc = set_err(CNS_EINVAL, "dt[%d] must be positive", i);
        if (!rc && offsets[i] < 0) rc = set_err(CNS_EINVAL, "offsets[%d] is negative", i);
        if (!rc && phys[i].weno_weights != phys[0].weno_weights)
            rc = set_err(CNS_EUNSUPPORTED, "every box of an ensemble must use the same WENO weights");
        void *u = (char *)u_packed + (size_t)offsets[i] * esz;
        if (!rc && !aligned(u)) rc = set_err(CNS_EINVAL, "box %d state is not 256-byte aligned", i);
        if (rc) {
            delete e;
            return rc;
        }
        e->c.add_box(grids[i], phys[i], dt[i], u);
    }
    e->c.layout();
    *out = e;
    return CNS_OK;
}

int cns_ensemble_destroy(cns_ensemble *ens) {
    delete ens;
    return CNS_OK;
}

size_t cns_ensemble_workspace_bytes(const cns_ensemble *ens) { return ens ? ens->c.need : 0; }

int cns_ensemble_set_workspace(cns_ensemble *ens, void *ws, size_t bytes) {
    if (!ens) return set_err(CNS_EINVAL, "null ensemble");
    if (!ws || !aligned(ws)) return set_err(CNS_EINVAL, "workspace must be non-null and 256-byte aligned");
    if (bytes < ens->c.need)
        return set_err(CNS_EWORKSPACE, "workspace of %zu bytes required (got %zu)", ens->c.need, bytes);
    ens->c.ws = (char *)ws;
    ens->c.ws_bytes = bytes;
    ens->c.dirty = true;
    return ens->c.sync_table();
}

int cns_ensemble_set_tiles(cns_ensemble *ens, int32_t box, int32_t sx, int32_t sy, int32_t sz, int32_t block) {
    if (!ens) return set_err(CNS_EINVAL, "null ensemble");
    if (box < -1 || box >= ens->c.nbox()) return set_err(CNS_EINVAL, "box index out of range");
    if (sx < 0 || sy < 0 || sz < 0) return set_err(CNS_EINVAL, "segment length must be >= 0");
    if (block != 0 && (block < 64 || block > 256 || (block % 64) != 0))
        return set_err(CNS_EINVAL, "block must be 64, 128, 192 or 256");
    for (int i = 0; i < ens->c.nbox(); ++i) {
        if (box >= 0 && i != box) continue;
        if (sx) ens->c.boxes[i].seg[0] = sx;
        if (sy) ens->c.boxes[i].seg[1] = sy;
        if (sz) ens->c.boxes[i].seg[2] = sz;
    }
    if (block) ens->c.block = block;
    ens->c.dirty = true;
    return ens->c.ws ? ens->c.sync_table() : CNS_OK;
}

int cns_ensemble_get_tiles(const cns_ensemble *ens, int32_t box, int32_t *seg3, int32_t *block) {
    if (!ens || !seg3 || !block) return set_err(CNS_EINVAL, "null argument");
    if (box < 0 || box >= ens->c.nbox()) return set_err(CNS_EINVAL, "box index out of range");
    for (int d = 0; d < 3; ++d) seg3[d] = ens->c.boxes[box].seg[d];
    *block = ens->c.block;
    return CNS_OK;
}

int cns_ensemble_get_launch(const cns_ensemble *ens, int32_t box, int32_t *rows, int64_t *sweep_grid,
                            int64_t *tile_grid) {
    if (!ens || !rows || !sweep_grid || !tile_grid) return set_err(CNS_EINVAL, "null argument");
    if (box < 0 || box >= ens->c.nbox()) return set_err(CNS_EINVAL, "box index out of range");
    const BoxDesc &b = ens->c.boxes[box];
    *rows = ens->c.ws && b.xrows == 1 ? b.rows : 0;
    *sweep_grid = ens->c.grid[F_SWEEP_Y];
    *tile_grid = ens->c.grid[F_VISC];
    return CNS_OK;
}

int cns_ensemble_set_launch(cns_ensemble *ens, int32_t box, int32_t rows, int64_t sweep_grid, int64_t tile_grid) {
    if (!ens) return set_err(CNS_EINVAL, "null ensemble");
    if (box < -1 || box >= ens->c.nbox()) return set_err(CNS_EINVAL, "box index out of range");
    if (rows < 0 || sweep_grid < 0 || tile_grid < 0) return set_err(CNS_EINVAL, "launch shapes must be >= 0");
    for (int i = 0; i < ens->c.nbox(); ++i) {
        if (box >= 0 && i != box) continue;
        if (rows > 0 && !rows_fit(ens->c.boxes[i].nx, rows, ens->c.esz, nullptr))
            return set_err(CNS_EINVAL, "box %d: %d rows of %d points do not fit a block of the x rows kernel", i, rows,
                           ens->c.boxes[i].nx);
    }
    for (int i = 0; i < ens->c.nbox(); ++i)
        if (box < 0 || i == box) ens->c.rows_ov[i] = rows;
    for (int f = F_SWEEP_X; f <= F_SWEEP_Z; ++f) ens->c.grid[f] = sweep_grid;
    ens->c.grid[F_VISC] = ens->c.grid[F_DIAG] = tile_grid;
    ens->c.dirty = true;
    return ens->c.ws ? ens->c.sync_table() : CNS_OK;
}

int cns_ensemble_autotune(cns_ensemble *ens, const char *cache_path) {
    if (!ens) return set_err(CNS_EINVAL, "null ensemble");
    if (!ens->c.ws) return set_err(CNS_EWORKSPACE, "no workspace bound");
    return autotune(ens->c, cache_path);
}

int cns_ensemble_run(cns_ensemble *ens, int32_t nsteps, double *diag, int32_t use_graph) {
    if (!ens) return set_err(CNS_EINVAL, "null ensemble");
    if (!ens->c.ws) return set_err(CNS_EWORKSPACE, "no workspace bound");
    if (nsteps < 0) return set_err(CNS_EINVAL, "nsteps must be >= 0");
    if (diag && ((uintptr_t)diag & 7u)) return set_err(CNS_EINVAL, "diag must be 8-byte aligned");
    if (use_graph && !ens->c.stream) return set_err(CNS_EUNSUPPORTED, "graph replay needs a non-default stream");
    ens->c.use_graph = use_graph != 0;
    return ens->c.run(ens->c.scheme, nullptr, 0.0, nsteps, diag);
}

int64_t cns_ensemble_graph_captures(const cns_ensemble *ens) {
    if (!ens) return set_err(CNS_EINVAL, "null ensemble");
    return ens->c.captures;
}

int cns_ensemble_set_integrator(cns_ensemble *ens, int32_t scheme) {
    if (!ens) return set_err(CNS_EINVAL, "null ensemble");
    if (scheme != CNS_RK4 && scheme != CNS_TVDRK3) return set_err(CNS_EINVAL, "unknown integrator %d", scheme);
    ens->c.scheme = scheme;
    return CNS_OK;
}

int cns_ensemble_profile_enable(cns_ensemble *ens, int32_t enable) {
    if (!ens) return set_err(CNS_EINVAL, "null ensemble");
    return ens->c.profile_enable(enable);
}

int cns_ensemble_profile_read(const cns_ensemble *ens, double *ms_host, int64_t *count_host) {
    if (!ens || !ms_host || !count_host) return set_err(CNS_EINVAL, "null argument");
    for (int k = 0; k < K_NKIND; ++k) {
        ms_host[k] = ens->c.prof.ms[k];
        count_host[k] = ens->c.prof.count[k];
    }
    return CNS_OK;
}

}  // extern "C"

// ----------------------------------------------------------------------------
// adjoint (FP64, single box): workspace layout and the checkpointed reverse RK4
// ----------------------------------------------------------------------------
struct AdjLayout {
    size_t ck, seg, X, ub, kb, kb2, Ub, S, rec, total;
    int nck, K;
};

static AdjLayout adj_layout(size_t n3, int nsteps, int K) {
    AdjLayout L{};
    const size_t st = align256(5 * n3 * sizeof(double));
    L.K = K > 0 ? K : 1;
    L.nck = nsteps > 0 ? (nsteps + L.K - 1) / L.K : 0;
    size_t off = 0;
    L.ck = off;                      // checkpoints: state at steps 0, K, 2K, ...
    off += (size_t)L.nck * st;
    L.seg = off;                     // per step of one segment: step-start state, stage states U2, U3, U4
    off += (size_t)(nsteps > 0 ? std::min(L.K, nsteps) : 0) * 4 * st;
    L.X = off;                       // running state
    off += st;
    L.ub = off;                      // running adjoint
    off += st;
    L.kb = off;                      // stage-rate adjoint (and forward stage rates)
    off += st;
    L.kb2 = off;                     // the next stage-rate adjoint, while kb is read
    off += st;
    L.Ub = off;                      // adjoint of the current stage state
    off += st;
    L.S = off;                       // sum of the stage adjoints
    off += st;
    L.rec = off;                     // a diagnostics record
    off += align256(CNS_NDIAG * sizeof(double));
    L.total = off;
    return L;
}

static int adj_check(const cns_plan *plan) {
    int rc = check_plan(plan);
    if (rc) return rc;
    if (plan->c.prec != CNS_FP64) return set_err(CNS_EUNSUPPORTED, "the adjoint is available for FP64 plans only");
    return CNS_OK;
}

static int adjoint_args(cns_plan *plan, int scheme, double dt, int32_t nsteps, int32_t ckpt_every, const void *adj_ws,
                        size_t bytes, AdjLayout *L) {
    int rc = adj_check(plan);
    if (!rc) rc = check_ptr(adj_ws, "adj_ws");
    if (rc) return rc;
    if (scheme != CNS_RK4 && scheme != CNS_TVDRK3) return set_err(CNS_EINVAL, "unknown integrator %d", scheme);
    if (!(dt > 0.0) || !std::isfinite(dt)) return set_err(CNS_EINVAL, "dt must be positive and finite");
    if (nsteps < 0 || ckpt_every < 1) return set_err(CNS_EINVAL, "need nsteps >= 0 and ckpt_every >= 1");
    if ((rc = plan->c.sync_table())) return rc;
    *L = adj_layout(plan->c.boxes[0].n3, nsteps, ckpt_every);
    if (bytes < L->total) return set_err(CNS_EWORKSPACE, "adjoint workspace of %zu bytes required", L->total);
    return CNS_OK;
}

// the step-start state and the stage states of step n of a segment starting at n0 (RK4:
// U2, U3, U4; TVD-RK3: U1, U2), kept while the fused step advances X
static void adj_keep_step(const Batch &bt, int scheme, const AdjLayout &L, char *w, size_t n5, double dt, int n,
                          int n0) {
    const size_t st = align256(n5 * sizeof(double));
    auto state = [&](size_t base, int i) { return (double *)(w + base + (size_t)i * st); };
    double *X = state(L.X, 0);
    adj_copy(n5, X, state(L.seg, 4 * (n - n0)), bt.stream);
    void *const st3[3] = {state(L.seg, 4 * (n - n0) + 1), state(L.seg, 4 * (n - n0) + 2),
                          state(L.seg, 4 * (n - n0) + 3)};
    launch_step(bt, scheme, X, dt, nullptr, 0, 0, st3);
}

// Forward pass of the adjoint: nsteps steps from u0 with a checkpoint every K steps; the
// last segment keeps the start and stage states of its steps; J = K(u^N).  Leaves u^N,
// the checkpoints and the last segment in the workspace for adjoint_reverse.
static int adjoint_forward(cns_plan *plan, int scheme, const void *u0, double dt, int32_t nsteps, int32_t ckpt_every,
                           void *adj_ws, size_t bytes, double *J_dev) {
    AdjLayout L;
    int rc = adjoint_args(plan, scheme, dt, nsteps, ckpt_every, adj_ws, bytes, &L);
    if (!rc) rc = check_ptr(u0, "u0");
    if (rc) return rc;
    if (J_dev && ((uintptr_t)J_dev & 7u)) return set_err(CNS_EINVAL, "J must be 8-byte aligned");
    Core &c = plan->c;
    const size_t n5 = 5 * c.boxes[0].n3, st = align256(n5 * sizeof(double));
    char *w = (char *)adj_ws;
    auto state = [&](size_t base, int i) { return (double *)(w + base + (size_t)i * st); };
    double *X = state(L.X, 0), *rec = (double *)(w + L.rec);
    hipStream_t s = c.stream;
    Batch bt = c.batch();
    bt.prof = nullptr;
    const int K = L.K, last0 = (L.nck - 1) * K;
    adj_copy(n5, (const double *)u0, X, s);
    for (int n = 0; n < nsteps; ++n) {
        if (n % K == 0) adj_copy(n5, X, state(L.ck, n / K), s);
        if (n >= last0) adj_keep_step(bt, scheme, L, w, n5, dt, n, last0);
        else launch_step(bt, scheme, X, dt, nullptr, 0, 0);
    }
    launch_diag(bt, X, rec, 0, 0);
    if (J_dev) adj_copy(1, rec, J_dev, s);
    return check_hip("adjoint_forward");
}

// Reverse sweep from what adjoint_forward left in the workspace (same plan, integrator,
// dt, nsteps and checkpoint interval): u0_bar = dJ/du0, one checkpoint segment at a
// time (last first), each recomputed from its checkpoint (the last one is kept).
static int adjoint_reverse(cns_plan *plan, int scheme, double dt, int32_t nsteps, int32_t ckpt_every, void *adj_ws,
                           size_t bytes, void *u0_bar) {
    AdjLayout L;
    int rc = adjoint_args(plan, scheme, dt, nsteps, ckpt_every, adj_ws, bytes, &L);
    if (!rc) rc = check_ptr(u0_bar, "u0_bar");
    if (rc) return rc;
    Core &c = plan->c;
    const BoxDesc &b = c.boxes[0];
    const size_t n3 = b.n3, n5 = 5 * n3, st = align256(n5 * sizeof(double));
    char *w = (char *)adj_ws;
    auto state = [&](size_t base, int i) { return (double *)(w + base + (size_t)i * st); };
    double *X = state(L.X, 0), *ub = state(L.ub, 0), *kb = state(L.kb, 0), *Ub = state(L.Ub, 0), *S = state(L.S, 0);
    double *kb2 = state(L.kb2, 0);
    double *seed = kb, *other = kb2;  // TVD-RK3: the buffer holding the next product's seed
    hipStream_t s = c.stream;
    Batch bt = c.batch();
    bt.prof = nullptr;
    const int K = L.K;
    adj_ke_seed(n3, X, ub, s);  // X holds u^N
    // reverse, one checkpoint segment at a time (last first)
    for (int sg = L.nck - 1; sg >= 0; --sg) {
        const int n0 = sg * K, n1 = std::min(nsteps, n0 + K);
        // recompute the segment (the last one is already kept), keeping every step-start
        // state and the stage states U2, U3, U4 the fused step writes
        if (sg != L.nck - 1) {
            adj_copy(n5, state(L.ck, sg), X, s);
            for (int n = n0; n < n1; ++n) adj_keep_step(bt, scheme, L, w, n5, dt, n, n0);
        }
        for (int n = n1 - 1; n >= n0; --n) {
            const double *Y = state(L.seg, 4 * (n - n0));
            if (scheme == CNS_TVDRK3) {
                // Shu-Osher stages U1 = u + dt R(u), U2 = 3/4 u + 1/4 (U1 + dt R(U1)),
                // u' = 1/3 u + 2/3 (U2 + dt R(U2)), reversed:
                //   Ubar2 = 2/3 ub + R'(U2)^T (2/3 dt ub)
                //   Ubar1 = 1/4 Ubar2 + R'(U1)^T (1/4 dt Ubar2)
                //   ub   <- 1/3 ub + 3/4 Ubar2 + Ubar1 + R'(u)^T (dt Ubar1)
                // (S holds Ubar2 and X, free during the reverse steps, holds Ubar1).  Each
                // combination and the next seed (2/3 dt ub for the next step) are formed
                // at the end of the product that finishes them.
                const double *U1 = state(L.seg, 4 * (n - n0) + 1), *U2 = state(L.seg, 4 * (n - n0) + 2);
                if (n == nsteps - 1) adj_lincomb(n5, 2.0 / 3.0 * dt, ub, 0.0, nullptr, seed, s);
                AdjEpilogue t2, t1, t0;
                t2.la = ub, t2.pa = 2.0 / 3.0, t2.ld = S, t2.lkb = other, t2.ls = 0.25 * dt, t2.store_ub = 0;
                t1.la = S, t1.pa = 0.25, t1.ld = X, t1.lkb = seed, t1.ls = dt, t1.store_ub = 0;
                t0.la = ub, t0.pa = 1.0 / 3.0, t0.lb = S, t0.pb = 0.75, t0.lc = X, t0.pc = 1.0, t0.ld = ub;
                t0.lkb = other, t0.ls = 2.0 / 3.0 * dt, t0.store_ub = 0;
                adj_rhs_vjp_epi(b, c.weights, s, U2, seed, Ub, t2);
                adj_rhs_vjp_epi(b, c.weights, s, U1, other, Ub, t1);
                adj_rhs_vjp_epi(b, c.weights, s, Y, seed, Ub, t0);
                std::swap(seed, other);  // three seeds a step: the buffers trade places
                continue;
            }
            const double *U2 = state(L.seg, 4 * (n - n0) + 1), *U3 = state(L.seg, 4 * (n - n0) + 2),
                         *U4 = state(L.seg, 4 * (n - n0) + 3);
            // reverse stages: kbar_4 = dt/6 ub, kbar_3 = dt/3 ub + dt Ub4, kbar_2 = dt/3 ub + dt/2 Ub3,
            // kbar_1 = dt/6 ub + dt/2 Ub2; ub <- ub + sum_s Ub_s.  Each stage adjoint Ub_s goes
            // straight into the running sum S and the next seed at the end of its product;
            // the seeds alternate between kb and kb2, since the product still reads its
            // own seed (with halos) while it writes the next.
            AdjEpilogue e4, e3, e2, e1;
            e4.S = S, e4.s_first = 1, e4.kb = kb2, e4.ub = ub, e4.a = dt / 3.0, e4.b = dt, e4.store_ub = 0;
            e3.S = S, e3.kb = kb, e3.ub = ub, e3.a = dt / 3.0, e3.b = 0.5 * dt, e3.store_ub = 0;
            e2.S = S, e2.kb = kb2, e2.ub = ub, e2.a = dt / 6.0, e2.b = 0.5 * dt, e2.store_ub = 0;
            e1.S = S, e1.ubf = ub, e1.kb = kb, e1.a = dt / 6.0, e1.store_ub = 0;
            if (n == nsteps - 1) adj_lincomb(n5, dt / 6.0, ub, 0.0, nullptr, kb, s);  // later steps: seeded by e1
            adj_rhs_vjp_epi(b, c.weights, s, U4, kb, Ub, e4);
            adj_rhs_vjp_epi(b, c.weights, s, U3, kb2, Ub, e3);
            adj_rhs_vjp_epi(b, c.weights, s, U2, kb, Ub, e2);
            adj_rhs_vjp_epi(b, c.weights, s, Y, kb2, Ub, e1);
        }
    }
    adj_copy(n5, ub, (double *)u0_bar, s);
    return check_hip("adjoint_reverse");
}

static int adjoint_run(cns_plan *plan, int scheme, const void *u0, double dt, int32_t nsteps, int32_t ckpt_every,
                       void *adj_ws, size_t bytes, double *J_dev, void *u0_bar) {
    int rc = check_ptr(u0_bar, "u0_bar");
    if (rc) return rc;
    if ((rc = adjoint_forward(plan, scheme, u0, dt, nsteps, ckpt_every, adj_ws, bytes, J_dev))) return rc;
    return adjoint_reverse(plan, scheme, dt, nsteps, ckpt_every, adj_ws, bytes, u0_bar);
}

extern "C" {

size_t cns_adjoint_workspace_bytes(const cns_plan *plan, int32_t nsteps, int32_t ckpt_every) {
    if (!plan || nsteps < 0) return 0;
    return adj_layout(plan->c.boxes[0].n3, nsteps, ckpt_every).total;
}

int cns_rhs_vjp(const cns_plan *plan, const void *u, const void *rbar, void *ubar, void *adj_ws, size_t bytes) {
    int rc = adj_check(plan);
    if (!rc) rc = check_ptr(u, "u");
    if (!rc) rc = check_ptr(rbar, "rbar");
    if (!rc) rc = check_ptr(ubar, "ubar");
    if (rc) return rc;
    if (ubar == u || ubar == rbar) return set_err(CNS_EINVAL, "ubar must not alias u or rbar");
    (void)adj_ws;  // the product needs no scratch
    (void)bytes;
    const BoxDesc &b = plan->c.boxes[0];
    adj_rhs_vjp(b, plan->c.weights, plan->c.stream, (const double *)u, (const double *)rbar, (double *)ubar);
    return check_hip("rhs_vjp");
}

int cns_adjoint_rk4(cns_plan *plan, const void *u0, double dt, int32_t nsteps, int32_t ckpt_every, void *adj_ws,
                    size_t bytes, double *J_dev, void *u0_bar) {
    return adjoint_run(plan, CNS_RK4, u0, dt, nsteps, ckpt_every, adj_ws, bytes, J_dev, u0_bar);
}

int cns_adjoint_tvdrk3(cns_plan *plan, const void *u0, double dt, int32_t nsteps, int32_t ckpt_every, void *adj_ws,
                       size_t bytes, double *J_dev, void *u0_bar) {
    return adjoint_run(plan, CNS_TVDRK3, u0, dt, nsteps, ckpt_every, adj_ws, bytes, J_dev, u0_bar);
}

int cns_adjoint_forward(cns_plan *plan, int32_t scheme, const void *u0, double dt, int32_t nsteps,
                        int32_t ckpt_every, void *adj_ws, size_t bytes, double *J_dev) {
    return adjoint_forward(plan, scheme, u0, dt, nsteps, ckpt_every, adj_ws, bytes, J_dev);
}

int cns_adjoint_reverse(cns_plan *plan, int32_t scheme, double dt, int32_t nsteps, int32_t ckpt_every, void *adj_ws,
                        size_t bytes, void *u0_bar) {
    return adjoint_reverse(plan, scheme, dt, nsteps, ckpt_every, adj_ws, bytes, u0_bar);
}

int cns_ic_vjp(const cns_plan *plan, const double *rho, const double *vel, const double *ubar, double *vbar) {
    int rc = adj_check(plan);
    if (!rc) rc = check_ptr(rho, "rho");
    if (!rc) rc = check_ptr(vel, "vel");
    if (!rc) rc = check_ptr(ubar, "ubar");
    if (!rc) rc = check_ptr(vbar, "vbar");
    if (rc) return rc;
    adj_ic_vjp(plan->c.boxes[0].n3, rho, vel, ubar, vbar, plan->c.stream);
    return check_hip("ic_vjp");
}

}  // extern "C"
