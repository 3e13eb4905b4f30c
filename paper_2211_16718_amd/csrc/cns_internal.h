// cns_internal.h -- host-side internals shared by the kernel launchers and the C-ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "cns.h"
#include "cns_device.h"

namespace cns {

// workspace layout of a plan (byte offsets into the caller's buffer)
struct Workspace {
    size_t W, G, rhs, stA, stB, acc, part, dhost, total;
};

constexpr int kDiagBlocks = 1024;  // partial-sum blocks of the diagnostics reduction
constexpr int kDiagThreads = 256;

struct Box {
    int nx, ny, nz;
    double lx, ly, lz;
    PhysT ph;
    size_t n3() const { return (size_t)nx * ny * nz; }
};

// optional per-kernel timing with HIP events on the plan's stream
enum KernelKind { K_PRIM = 0, K_VISC_FLUX, K_SWEEP_X, K_SWEEP_Y, K_SWEEP_Z, K_DIAG, K_NKIND };
constexpr int kMaxProfLaunch = 32;

struct Prof {
    bool on = false;
    hipEvent_t ev[2 * kMaxProfLaunch] = {};
    int kind[kMaxProfLaunch] = {};
    int n = 0;
    double ms[K_NKIND] = {};
    long long count[K_NKIND] = {};
    hipStream_t s = nullptr;
};

// brackets one launch with a pair of events when profiling is on
struct ProfScope {
    Prof *p;
    int slot = -1;
    ProfScope(Prof *pf, int kind, hipStream_t s) : p(pf) {
        if (p && p->on && p->n < kMaxProfLaunch) {
            slot = p->n++;
            p->kind[slot] = kind;
            hipEventRecord(p->ev[2 * slot], s);
            p->s = s;
        }
    }
    ~ProfScope() {
        if (slot >= 0) hipEventRecord(p->ev[2 * slot + 1], p->s);
    }
};
// wait for the recorded events and add their durations to the totals
void prof_flush(Prof *p);

struct Tiles {
    int seg[3] = {16, 16, 16};
    int block = 256;
};

// kernel launchers (cns_kernels.hip); T = double or float
template <typename T>
void launch_init_state(const Box &b, const double *rho, const double *vel, const double *p, T *u, hipStream_t s);
// full RHS, or RK stage (stage 1..4) when stage > 0: see cns_kernels.hip
template <typename T>
void launch_rhs(const Box &b, const Tiles &t, const T *u, T *rhs, T *W, T *G, hipStream_t s);
template <typename T>
void launch_rhs_dir(const Box &b, const Tiles &t, const T *u, int dir, T *out, hipStream_t s);
template <typename T>
void launch_viscous(const Box &b, const T *u, T *out, T *W, T *G, hipStream_t s);
template <typename T>
void launch_rk4_stage(const Box &b, const Tiles &t, int stage, const T *ustage, T *un, T *unext, double *acc,
                      double dt, T *rhs, T *W, T *G, hipStream_t s, Prof *pf = nullptr);
template <typename T>
void launch_diag(const Box &b, const T *u, double *part, double *out, hipStream_t s, Prof *pf = nullptr);

}  // namespace cns
