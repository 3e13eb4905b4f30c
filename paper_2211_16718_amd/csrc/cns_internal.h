// cns_internal.h -- internals shared by the kernels (cns_kernels.hip) and the C-ABI
// (cns_api.hip).
//
// Every launch works on a *batch* of periodic boxes described by a device table of
// BoxDesc entries.  A kernel's blocks are virtual: for each kernel family a prefix
// array off[0..nbox] gives the first virtual block of every box; a block finds its
// box by binary search and runs the single-box code on its local block index.  A
// single-box plan is a batch of one, so a box advanced inside an ensemble executes
// exactly the machine code of its single-box run.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "cns.h"
#include "cns_device.h"

namespace cns {

constexpr int kPointThreads = 256;    // threads per block of point-wise kernels
constexpr int kDiagThreads = 256;
constexpr int kDiagBlocksMax = 1024;  // partial-sum blocks per box of the diagnostics
constexpr int kRowThreads = 256;      // threads per block of the x rows kernel
constexpr int kRowLdsMax = 64 * 1024;
constexpr int kViscTX = 32, kViscTY = 8;  // (x, y) tile of the viscous-flux kernel (kPointThreads threads)
constexpr int kViscSZ = 16;               // planes per block of the viscous-flux kernel (and its adjoint)
// Planes per tile of the viscous-flux and diagnostics kernels: 32 in boxes at least 256
// deep, where the +-2-plane halo of a tile then costs 1.125x its reads instead of 1.25x
// (512^3: fetch 9.45 -> 8.58 GB per launch), else 16, which keeps small boxes in
// enough tiles to fill the GPU.
__host__ __device__ __forceinline__ int visc_planes(int nz) { return nz >= 256 ? 2 * kViscSZ : kViscSZ; }
// Partial-sum slots of a box's diagnostics: one per block of the diagnostics kernel (at
// most kDiagBlocksMax) or one per viscous-flux tile when the diagnostics ride on that
// kernel.
inline size_t diag_part_slots(int nx, int ny, int nz) {
    const size_t tiles = (size_t)((nx + kViscTX - 1) / kViscTX) * ((ny + kViscTY - 1) / kViscTY) *
                         ((nz + visc_planes(nz) - 1) / visc_planes(nz));
    return tiles > (size_t)kDiagBlocksMax ? tiles : (size_t)kDiagBlocksMax;
}

// buffer roles of a box
enum Buf { BUF_U = 0, BUF_A = 1, BUF_B = 2 };

struct BoxDesc {
    int nx, ny, nz;
    int seg[3];  // marching-sweep segment length per direction
    int xrows;   // x sweep kernel: 1 whole rows in LDS, 2 rows in chunks, 0 marching
    int rows;    // rows per block of the x rows kernel
    size_t n3;
    double inv_h[3];  // 1/dx, 1/dy, 1/dz
    double gamma, prandtl, mu, eps, delta, dt;
    void *u, *A, *B, *rhs, *G;  // state and scratch (element type of the plan)
    double *acc, *part;             // RK4 accumulator [5][n3], diagnostics partials
};

// kernel families with their own virtual-block prefix
enum Family { F_POINT = 0, F_XROWS, F_SWEEP_X, F_SWEEP_Y, F_SWEEP_Z, F_DIAG, F_BOX, F_VISC, F_XCHUNK, F_N };

// Per-call arguments of a replayed hipGraph: the captured launches read the state, the
// step size and the diagnostics base from this device record (written by a small kernel
// before every replay), so one capture serves calls with other pointers and step sizes.
struct GraphParams {
    const void *u;  // replaces the box's state u when non-null
    double *diag;   // diagnostics output base
    double dt;      // replaces the box's dt when positive
    double pad;
};

// per-launch arguments
struct Launch {
    const BoxDesc *boxes;
    const long long *off;  // this family's prefix [nbox + 1]
    int nbox;
    long long total;  // off[nbox]
    int in;           // Buf of the state read by the kernel
    int out;          // Buf written by the fused RK4 stage update
    int stage;        // Runge-Kutta stage 1..4 (fused update) or 0
    int scheme;       // CNS_RK4 or CNS_TVDRK3 for the fused update
    int step;         // diagnostics record index
    // single-box overrides (used when non-null / positive)
    const void *u_ov;  // replaces the box's state u
    void *a_ov, *b_ov;  // replace the box's stage buffers A, B
    void *out_ov;      // replaces rhs as the output of WRITE/ACCUM sweeps and viscous kernels
    double dt_ov;      // replaces the box's dt
    double *diag;      // diagnostics output base (may be null)
    long long diag_box_stride;  // records between consecutive boxes in `diag`
    int diag_fused;             // the diagnostics partials come from the viscous-flux tiles
    const GraphParams *gp;      // graph replay: u_ov, dt_ov and diag come from here
};

// optional per-kernel timing with HIP events on the plan's stream
enum KernelKind { K_PRIM = 0, K_VISC_FLUX, K_SWEEP_X, K_SWEEP_Y, K_SWEEP_Z, K_DIAG, K_NKIND };
constexpr int kMaxProfLaunch = 48;

struct Prof {
    bool on = false;
    hipEvent_t ev[2 * kMaxProfLaunch] = {};
    int kind[kMaxProfLaunch] = {};
    int n = 0;
    double ms[K_NKIND] = {};
    long long count[K_NKIND] = {};
    hipStream_t s = nullptr;
};

struct ProfScope {
    Prof *p;
    int slot = -1;
    ProfScope(Prof *pf, int kind, hipStream_t s) : p(pf) {
        if (p && p->on && p->n < kMaxProfLaunch) {
            slot = p->n++;
            p->kind[slot] = kind;
            (void)hipEventRecord(p->ev[2 * slot], s);
            p->s = s;
        }
    }
    ~ProfScope() {
        if (slot >= 0) (void)hipEventRecord(p->ev[2 * slot + 1], p->s);
    }
};
void prof_flush(Prof *p);

// host view of a batch: what the launchers need
struct Batch {
    int nbox = 0;
    int prec = CNS_FP64;
    int block = 256;  // threads per block of the marching sweeps
    bool any_visc = false;
    int weights = CNS_WENO_JS;  // WENO weights (every box of a batch uses the same)
    const BoxDesc *d_boxes = nullptr;  // device table
    const long long *d_off[F_N] = {};  // device prefixes
    long long total[F_N] = {};
    int rowP = 1;       // points per thread of the rows kernel (max over boxes)
    size_t rowLds = 0;  // LDS bytes of the rows kernel (max over boxes)
    size_t esz = 8;     // bytes per state element
    hipStream_t stream = nullptr;
    Prof *prof = nullptr;
    const GraphParams *gp = nullptr;  // set while a run is captured for graph replay
    long long grid[F_N] = {};         // launched blocks per family (0: one per virtual block)
};

// host-side helpers (cns_kernels.hip)
int rows_for(int nx);
// rows per block of the x rows kernel fit (at most 4 points per thread, 64 KiB of LDS);
// *P receives the points per thread
bool rows_fit(int nx, int rows, size_t esz, int *P);
long long family_blocks(const BoxDesc &b, int fam, int block);

// launchers (cns_kernels.hip); all enqueue on bt.stream
void launch_init_state(int prec, size_t n3, double gamma, const double *rho, const double *vel, const double *p,
                       void *u, hipStream_t s);
void launch_fill(int prec, size_t n, void *out, hipStream_t s);
// full RHS of every box into `out_ov` (single box) or each box's rhs buffer
void launch_rhs(const Batch &bt, const void *u_ov, void *out_ov);
void launch_rhs_dir(const Batch &bt, const void *u_ov, int dir, void *out_ov);
void launch_viscous(const Batch &bt, const void *u_ov, void *out_ov);
// one RK4 step of every box (4 stages with fused updates), then diagnostics if diag
// stage_states (single box, may be null): three buffers that receive the stage states
// U2, U3, U4 of the step (they replace the stage buffers A, B).
// diag_prev >= 0 (FP64, viscous batches): the first stage's viscous-flux launch also
// forms the diagnostics of the state it reads into record diag_prev; diag_own: the
// step's own record `step` is formed after the step (by the diagnostics kernels).
void launch_rk4_step(const Batch &bt, const void *u_ov, double dt_ov, double *diag, long long diag_box_stride,
                     int step, void *const *stage_states = nullptr, int diag_prev = -1, bool diag_own = true);
// one step of the integrator `scheme` (CNS_RK4 or CNS_TVDRK3), then diagnostics as above
void launch_step(const Batch &bt, int scheme, const void *u_ov, double dt_ov, double *diag,
                 long long diag_box_stride, int step, void *const *stage_states = nullptr, int diag_prev = -1,
                 bool diag_own = true);
// whether a batch's diagnostics can ride on the next step's first viscous-flux launch
inline bool diag_fusable(const Batch &bt) { return bt.prec == CNS_FP64 && bt.any_visc; }
void launch_diag(const Batch &bt, const void *u_ov, double *diag, long long diag_box_stride, int step);
// max over points and directions of |v_d| + c of every box into out[box] (NaN for a box
// with a non-finite state, rho <= 0 or p <= 0)
void launch_max_wave_speed(const Batch &bt, const void *u_ov, double *out);
// Diagnostics of one box with its device table and partial sums in caller-given device
// scratch (scratch_dev, 256-byte aligned, static_diag_bytes() bytes): the table is
// written by a kernel from a kernel argument, so nothing is copied from the host.
struct OneBoxTable {
    BoxDesc b;
    long long off[F_N][2];
};
inline size_t align_up256(size_t x) { return (x + 255) & ~(size_t)255; }
size_t static_diag_bytes();
void launch_diag_static(char *scratch_dev, const BoxDesc &b, int prec, const void *u, double *out, hipStream_t s);
// a plain streaming copy (bytes a multiple of 16, 16-byte aligned pointers)
void launch_stream_copy(const void *src, void *dst, size_t bytes, hipStream_t s);
// the per-call record of a graph replay (enqueued before the replay)
void launch_set_params(GraphParams *gp, const void *u, double *diag, double dt, hipStream_t s);
// time the y and z marching sweeps over the batch (autotuning); milliseconds per launch pair
float time_sweeps_yz(const Batch &bt, int reps);
// time one RHS evaluation's kernels into scratch only (viscous fluxes, x sweep, y and z
// sweeps accumulating into rhs): milliseconds per evaluation (autotuning)
float time_rhs_kernels(const Batch &bt, int reps);
// blocks of the marching sweeps / tiled kernels the chip holds at once (persistent grids)
long long resident_sweep_blocks(const Batch &bt);
long long resident_tile_blocks(const Batch &bt);

// kinetic-energy spectrum (cns_spectrum.hip), one box: E[nshell] and mom = {sum E, M2, lambda};
// scratch: the box's A, B and rhs buffers
int spectrum_shells(const BoxDesc &b);
bool spectrum_supported(const BoxDesc &b);
void launch_spectrum(const BoxDesc &b, int prec, hipStream_t s, const void *u, double *E, int nshell, double *mom);

}  // namespace cns
