// cns_kernels.hip -- gfx950 kernels of the WENO5-Roe / central-viscous RHS and RK4.
//
// Data layout in HBM: SoA state u[v][k][j][i] (x fastest) per box.  One RHS
// evaluation of a batch of boxes is
//   1. k_visc_flux  : u -> viscous fluxes G = (tau_xx, tau_yy, tau_zz, tau_xy,
//                     tau_xz, tau_yz, E_x, E_y, E_z), E_d = v.tau_d - q_d       [9][N3]
//                     (primitives formed in the kernel; skipped when mu_eff = 0)
//   2. x sweep      : u, G -> rhs (write).  Whole periodic rows staged in LDS, one
//                     thread per interface (k_sweep_x_rows); the marching kernel
//                     when a row does not fit.
//   3. k_sweep<y>   : u, G -> rhs (accumulate)
//   4. k_sweep<z>   : u, G -> rhs (accumulate), or the fused Runge-Kutta stage update.
// A marching thread owns a segment of one grid line and walks along it with a
// six-point state window: every point flux is computed once, every interface
// flux once per segment, the flux difference is formed in registers.  The viscous
// term along d enters through the interface flux (-G_{j-1} + 7 G_j + 7 G_{j+1} -
// G_{j+2}) / 12, whose difference is the 5-point central derivative of G.
// Periodic boundaries wrap the line index; there are no ghost cells.
//
// Every kernel takes a Launch over a batch of boxes (see cns_internal.h) and loops
// over virtual blocks, so one launch advances every box of an ensemble.
#include <hip/hip_runtime.h>

#include <type_traits>

#include <algorithm>

#include "cns_internal.h"

namespace cns {

__device__ __forceinline__ int wrapi(int j, int n) { return j < 0 ? j + n : (j >= n ? j - n : j); }
// the same for any j >= -n (tile halos can reach several periods past a short line);
// the division only runs for lines shorter than the halo
__device__ __forceinline__ int wrapm(int j, int n) {
    int r = j < 0 ? j + n : j;
    r = r >= n ? r - n : r;
    return r >= n ? r % n : r;
}

// box owning virtual block vb: the last i with off[i] <= vb
__device__ __forceinline__ int find_box(const long long *off, int nbox, long long vb) {
    int lo = 0, hi = nbox;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (off[mid] <= vb) lo = mid;
        else hi = mid;
    }
    return lo;
}

// The virtual blocks a launched block runs.  Workgroups are dispatched to the 8 XCDs of
// the chip round-robin (block b on XCD b % 8), and each XCD has its own L2.  The
// virtual blocks are cut into one contiguous range per XCD, and the launched blocks of
// XCD x walk range x with a stride of their number, so blocks that touch neighbouring
// data (stencil halos) share an L2.  With one launched block per virtual block each
// runs exactly one; with fewer (a persistent launch, its grid sized to the blocks the
// chip holds at once) each loops over several.  Every virtual block runs exactly once
// for any grid size.
struct VbRange {
    long long vb, end, stride;
};
__device__ __forceinline__ VbRange vb_range(long long total) {
    const long long G = gridDim.x, b = blockIdx.x;
    const long long X = G < 8 ? G : 8;  // ranges: one per XCD that has blocks
    const long long x = b % X, l = b / X;
    const long long nbx = G / X + (x < G % X ? 1 : 0);
    const long long q = total / X, r = total % X;
    const long long lo = x * q + (x < r ? x : r), hi = lo + q + (x < r ? 1 : 0);
    return VbRange{lo + l, hi, nbx};
}

// Classical RK4 keeps u^n, the stage state and an FP64 accumulator of
// u^n + dt sum_s b_s k_s.  With FP64 stage states (U2 = u + dt k1/2, U4 = u + dt k3)
// the terms of k1 and k3 are recovered from them when the accumulator is next
// touched, so it is written in stage 2 and read in stage 4 only; FP32 stage states
// could not give those terms back to FP64 accuracy, so the mixed form updates it in
// every stage.
template <typename T>
constexpr bool kFp64Stages = std::is_same<T, double>::value;

// the launch with the per-call record of a graph replay applied (read once per kernel)
__device__ __forceinline__ Launch with_params(Launch L) {
    if (L.gp) {
        L.u_ov = L.gp->u;
        L.dt_ov = L.gp->dt;
        L.diag = L.gp->diag;
    }
    return L;
}

// Pointers into HBM taken from the device tables are generic (flat) pointers to the
// compiler, and accesses through them become FLAT instructions, which count against
// the LDS counter as well as the vector-memory counter: every wait for an LDS read then
// also waits for all HBM loads in flight, which undoes the loads issued ahead of the
// arithmetic.  The kernels cast them to the global address space (HBM), whose
// accesses count against the vector-memory counter only.
template <typename T>
using gptr = __attribute__((address_space(1))) T *;
template <typename T>
__device__ __forceinline__ gptr<T> glob(T *p) {
    return (gptr<T>)p;
}

// A value all lanes hold alike (read from the box table) moved into scalar registers.
// The compiler cannot prove that table reads are the same on every lane; marked
// uniform, the pointers stay in scalar registers across the loops instead of being
// copied back from vector registers before each access.
__device__ __forceinline__ uint64_t uni64(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}
template <typename T>
__device__ __forceinline__ gptr<T> uni(gptr<T> p) {
    return (gptr<T>)uni64((uint64_t)p);
}

// Component c of a component-major array (component c at element c * n3) at a lane's
// byte offset: the array base and the component offset are uniform and stay in scalar
// registers, and every load and store of a point shares the lane's one 32-bit offset
// register (global memory instructions with a scalar base address).  Needs
// n3 * 8 < 2^32, which plan and ensemble creation check.
template <typename T>
__device__ __forceinline__ gptr<T> elem(gptr<T> a, size_t n3, int c, uint32_t boff) {
    using Byte = typename std::conditional<std::is_const<T>::value, const char, char>::type;
    return (gptr<T>)((gptr<Byte>)(a + (size_t)c * n3) + boff);
}

__device__ __forceinline__ const void *state_ptr(const BoxDesc &b, const Launch &L, int which) {
    if (which == BUF_U) return L.u_ov ? L.u_ov : b.u;
    if (which == BUF_A) return L.a_ov ? L.a_ov : b.A;
    return L.b_ov ? L.b_ov : b.B;
}

// ----------------------------------------------------------------------------
// state from primitives (Sec. 2.1 equation of state); single box
// ----------------------------------------------------------------------------
template <typename T>
__global__ void k_init_state(size_t n3, double gm1, const double *rho, const double *vel, const double *p, T *u) {
    size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (i >= n3) return;
    double r = rho[i], a = vel[i], b = vel[n3 + i], c = vel[2 * n3 + i];
    u[i] = T(r);
    u[n3 + i] = T(r * a);
    u[2 * n3 + i] = T(r * b);
    u[3 * n3 + i] = T(r * c);
    u[4 * n3 + i] = T(p[i] / gm1 + 0.5 * r * (a * a + b * b + c * c));
}

template <typename T>
__global__ void k_fill(size_t n, T *out) {
    size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (i < n) out[i] = T(0);
}

// ----------------------------------------------------------------------------
// viscous terms: primitives, then viscous fluxes at points
// ----------------------------------------------------------------------------
// primitives (u, v, w, T = gamma p / rho) of the state at linear index i
template <typename T>
__device__ __forceinline__ void prim_at(gptr<const T> u, size_t n3, size_t i, T gamma, T W[4]) {
#pragma clang fp contract(off)
    const T r = u[i], mx = u[n3 + i], my = u[2 * n3 + i], mz = u[3 * n3 + i], e = u[4 * n3 + i];
    const T inv = rcp(r);
    W[0] = mx * inv;
    W[1] = my * inv;
    W[2] = mz * inv;
    const T p = (gamma - T(1)) * (e - T(0.5) * (mx * W[0] + my * W[1] + mz * W[2]));
    W[3] = gamma * p * inv;
}

// The halo ring of a kViscTX x kViscTY tile in its (kViscTX + 4) x (kViscTY + 4) staging
// plane: rows 0, 1, kViscTY + 2, kViscTY + 3 in full, then columns 0, 1, kViscTX + 2,
// kViscTX + 3 of the rows between.  Thread t < kViscRing owns ring position t.
constexpr int kViscRingRows = 4 * (kViscTX + 4);
constexpr int kViscRing = kViscRingRows + 4 * kViscTY;
static_assert(kViscRing <= kPointThreads && kViscRing <= kDiagThreads, "one halo point per thread");
__device__ __forceinline__ void ring_pos(int t, int &hx, int &hy) {
    if (t < kViscRingRows) {
        const int r = t / (kViscTX + 4);
        hx = t % (kViscTX + 4);
        hy = r < 2 ? r : kViscTY + r;
    } else {
        const int q = t - kViscRingRows, c = q & 3;
        hy = 2 + (q >> 2);
        hx = c < 2 ? c : kViscTX + c;
    }
}

// The 5-point central difference (times h) rounded as written (no fused multiply-add):
// the viscous-flux kernel forms every value of G with contraction off, so that the
// variant that also accumulates the diagnostics (extra uses of the gradients) gives the
// same bits.
template <typename T>
__device__ __forceinline__ T dcen_nc(T m2, T m1, T p1, T p2) {
#pragma clang fp contract(off)
    return (T(8) * (p1 - m1) - (p2 - m2)) * (T(1) / T(12));
}

// Primitives of the state at linear index i, as prim_at, and (FP64 only) the point
// quantities of the diagnostics when `count`: kinetic energy, mass, momentum, energy,
// the largest wave speed and the bad-point count in acc, `good` set when the point is
// valid (finite, rho > 0, p > 0).  The primitives are the same bits as prim_at's.
__device__ __forceinline__ void prim_stats(gptr<const double> u, size_t n3, size_t i, double gamma, double W[4],
                                           bool count, double acc[CNS_NDIAG], bool &good) {
#pragma clang fp contract(off)
    const double r = u[i], mx = u[n3 + i], my = u[2 * n3 + i], mz = u[3 * n3 + i], e = u[4 * n3 + i];
    const double inv = rcp(r);
    W[0] = mx * inv;
    W[1] = my * inv;
    W[2] = mz * inv;
    const double ke = 0.5 * (mx * W[0] + my * W[1] + mz * W[2]);
    const double p = (gamma - 1.0) * (e - ke);
    W[3] = gamma * p * inv;
    good = false;
    if (count) {
        const bool finite = isfinite(r) && isfinite(mx) && isfinite(my) && isfinite(mz) && isfinite(e);
        if (!finite || !(r > 0.0) || !(p > 0.0)) {
            acc[8] += 1.0;
        } else {
            acc[0] += ke;
            acc[2] += r;
            acc[3] += mx;
            acc[4] += my;
            acc[5] += mz;
            acc[6] += e;
            const double c = sqrt(gamma * p * inv);
            acc[7] = fmax(acc[7], fmax(fabs(W[0]), fmax(fabs(W[1]), fabs(W[2]))) + c);
            good = true;
        }
    }
}
__device__ __forceinline__ void block_reduce_diag(const double acc[CNS_NDIAG], double (*red)[CNS_NDIAG],
                                                  gptr<double> dst, const double scale[CNS_NDIAG]);

// Viscous fluxes at points: the 12 first derivatives of (u, v, w, T) by the 5-point
// central stencil, then tau, q and G.  A block owns a 32 x 8 (x, y) tile and marches
// along z over visc_planes(nz) planes.  Each thread keeps its own column's primitives at planes
// k-2 .. k+2 in registers (z derivatives); a thread that owns a point of the tile's halo
// ring keeps that point's primitives at planes k .. k+2 in its own LDS slots.  Plane k
// is staged in LDS from the two windows (x and y derivatives).  Each state value of a
// plane is loaded once per tile, and the column and the ring point of plane k+2 are
// loaded together, while the neighbouring tiles (same XCD, launched together) load the
// same lines for their own columns, so the halo comes from L2.
//
// With DIAG (FP64 plans, the first stage of a step) the kernel also forms the partial
// diagnostics of the state it reads, one partial per tile: the point quantities of a
// plane as its column is loaded, the enstrophy from the velocity gradients it computes
// anyway (the same central derivatives as the diagnostics kernel).  The state's
// diagnostics then cost no read of their own.
template <typename T, bool DIAG>
__global__ __launch_bounds__(kPointThreads) void k_visc_flux(Launch L0) {
#pragma clang fp contract(off)
    static_assert(!DIAG || std::is_same<T, double>::value, "fused diagnostics in FP64 plans only");
    const Launch L = with_params(L0);
    __shared__ T pl[4][kViscTY + 4][kViscTX + 4];
    __shared__ T rw[3][4][kViscRing];  // ring primitives, slot (plane - z0) mod 3
    __shared__ double red[DIAG ? kPointThreads / 64 : 1][CNS_NDIAG];
    const double one[CNS_NDIAG] = {1, 1, 1, 1, 1, 1, 1, 1, 1};
    int rhx, rhy;
    ring_pos(threadIdx.x, rhx, rhy);
    const bool ring = threadIdx.x < kViscRing;
    const int rt = ring ? threadIdx.x : 0;
    const VbRange R = vb_range(L.total);
    for (long long vb = R.vb; vb < R.end; vb += R.stride) {
        const int bi = find_box(L.off, L.nbox, vb);
        const BoxDesc &b = L.boxes[bi];
        const int nx = b.nx, ny = b.ny, nz = b.nz;
        const size_t n3 = b.n3, sz = (size_t)nx * ny;
        const long long lb = vb - L.off[bi];
        const int ntx = (nx + kViscTX - 1) / kViscTX, nty = (ny + kViscTY - 1) / kViscTY;
        const int x0 = (int)(lb % ntx) * kViscTX, y0 = (int)((lb / ntx) % nty) * kViscTY;
        const int vsz = visc_planes(nz);
        const int z0 = (int)(lb / ((long long)ntx * nty)) * vsz, z1 = min(z0 + vsz, nz);
        const int tx = threadIdx.x % kViscTX, ty = threadIdx.x / kViscTX;
        const bool act = x0 + tx < nx && y0 + ty < ny;
        // a column past a ragged edge wraps periodically: its primitives are halo values
        // of the active columns beside it
        const size_t col = (size_t)wrapm(y0 + ty, ny) * nx + wrapm(x0 + tx, nx);
        const size_t rcol = (size_t)wrapm(y0 - 2 + rhy, ny) * nx + wrapm(x0 - 2 + rhx, nx);
        const gptr<const T> u = glob((const T *)state_ptr(b, L, L.in));
        const gptr<T> G = glob((T *)b.G);
        const T gamma = T(b.gamma);
        const T ihx = T(b.inv_h[0]), ihy = T(b.inv_h[1]), ihz = T(b.inv_h[2]);
        const T mu = T(b.mu), kcond = T(b.mu / ((b.gamma - 1.0) * b.prandtl));
        T Wz[5][4];  // this column's primitives at planes k-2 .. k+2
        double acc[CNS_NDIAG] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        unsigned good = 0;  // bit m: the column's point at plane k-2+m is valid (DIAG)
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const size_t ic = col + wrapi(z0 - 2 + m, nz) * sz;
            if constexpr (DIAG) {
                const int zp = z0 - 2 + m;
                bool gd;
                prim_stats(u, n3, ic, gamma, Wz[m], act && zp >= z0 && zp < z1, acc, gd);
                if (gd) good |= 1u << m;
            } else {
                prim_at(u, n3, ic, gamma, Wz[m]);
            }
        }
        if (ring) {
            for (int m = 0; m < 2; ++m) {
                T w4[4];
                prim_at(u, n3, rcol + wrapi(z0 + m, nz) * sz, gamma, w4);
#pragma unroll
                for (int c = 0; c < 4; ++c) rw[m][c][rt] = w4[c];
            }
        }
        int slot = 0;  // (k - z0) mod 3
        for (int k = z0; k < z1; ++k) {
            const int slot2 = slot == 0 ? 2 : slot - 1;  // (k + 2 - z0) mod 3
            if constexpr (DIAG) {
                bool gd;
                prim_stats(u, n3, col + wrapi(k + 2, nz) * sz, gamma, Wz[4], act && k + 2 < z1, acc, gd);
                if (gd) good |= 1u << 4;
            } else {
                prim_at(u, n3, col + wrapi(k + 2, nz) * sz, gamma, Wz[4]);
            }
            if (ring) {
                T w4[4];
                prim_at(u, n3, rcol + wrapi(k + 2, nz) * sz, gamma, w4);
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    rw[slot2][c][rt] = w4[c];
                    pl[c][rhy][rhx] = rw[slot][c][rt];
                }
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) pl[c][ty + 2][tx + 2] = Wz[2][c];
            __syncthreads();
            if (act) {
                T g[4][3];  // g[a][c] = d W_a / d x_c
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    g[a][0] = dcen_nc(pl[a][ty + 2][tx], pl[a][ty + 2][tx + 1], pl[a][ty + 2][tx + 3], pl[a][ty + 2][tx + 4]) * ihx;
                    g[a][1] = dcen_nc(pl[a][ty][tx + 2], pl[a][ty + 1][tx + 2], pl[a][ty + 3][tx + 2], pl[a][ty + 4][tx + 2]) * ihy;
                    g[a][2] = dcen_nc(Wz[0][a], Wz[1][a], Wz[3][a], Wz[4][a]) * ihz;
                }
                if constexpr (DIAG) {
                    if (good & 4u) {
                        // vorticity of the velocity, as the diagnostics kernel forms it
                        const double ox = g[2][1] - g[1][2], oy = g[0][2] - g[2][0], oz = g[1][0] - g[0][1];
                        if (isfinite(ox) && isfinite(oy) && isfinite(oz)) acc[1] += 0.5 * (ox * ox + oy * oy + oz * oz);
                    }
                }
                T div = g[0][0] + g[1][1] + g[2][2];
                T tdiv = T(2) / T(3) * div;
                T txx = mu * (T(2) * g[0][0] - tdiv);
                T tyy = mu * (T(2) * g[1][1] - tdiv);
                T tzz = mu * (T(2) * g[2][2] - tdiv);
                T txy = mu * (g[0][1] + g[1][0]);
                T txz = mu * (g[0][2] + g[2][0]);
                T tyz = mu * (g[1][2] + g[2][1]);
                const T vx = Wz[2][0], vy = Wz[2][1], vz = Wz[2][2];
                const size_t idx = (size_t)k * sz + col;
                // non-temporal stores: G is streamed to memory and read back by the sweeps
                // (at 128^3: 1.3 % faster step, at 512^3: 1.9 %)
                __builtin_nontemporal_store(txx, &G[idx]);
                __builtin_nontemporal_store(tyy, &G[n3 + idx]);
                __builtin_nontemporal_store(tzz, &G[2 * n3 + idx]);
                __builtin_nontemporal_store(txy, &G[3 * n3 + idx]);
                __builtin_nontemporal_store(txz, &G[4 * n3 + idx]);
                __builtin_nontemporal_store(tyz, &G[5 * n3 + idx]);
                __builtin_nontemporal_store(vx * txx + vy * txy + vz * txz + kcond * g[3][0], &G[6 * n3 + idx]);
                __builtin_nontemporal_store(vx * txy + vy * tyy + vz * tyz + kcond * g[3][1], &G[7 * n3 + idx]);
                __builtin_nontemporal_store(vx * txz + vy * tyz + vz * tzz + kcond * g[3][2], &G[8 * n3 + idx]);
            }
            __syncthreads();  // the next plane overwrites the LDS tile
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int c = 0; c < 4; ++c) Wz[m][c] = Wz[m + 1][c];
            slot = slot == 2 ? 0 : slot + 1;
            good >>= 1;
        }
        if constexpr (DIAG) block_reduce_diag(acc, red, glob(b.part) + (size_t)lb * CNS_NDIAG, one);
    }
}

// which G field holds component (momentum x, y, z, energy) of the viscous flux along DIR
template <int DIR>
__device__ __forceinline__ constexpr int gcomp(int c) {
    return DIR == 0 ? (c == 0 ? 0 : c == 1 ? 3 : c == 2 ? 4 : 6)
                    : (DIR == 1 ? (c == 0 ? 3 : c == 1 ? 1 : c == 2 ? 5 : 7) : (c == 0 ? 4 : c == 1 ? 5 : c == 2 ? 2 : 8));
}

// A stage's sweeps run x, y, z.  The G field of component c along DIR is read for the
// last time in that stage by this sweep when no later sweep reads it (tau_xy: x then y;
// tau_xz: x then z; tau_yz: y then z); such loads, and the z sweep's loads of rhs and
// of the FP64 accumulator, are marked non-temporal so they do not displace lines that
// are read again.
template <int DIR, int C>
__device__ __forceinline__ constexpr bool g_last_read() {
    return DIR == 2 || (DIR == 1 && C != 2) || (DIR == 0 && (C == 0 || C == 3));
}
template <int DIR, int C, typename T>
__device__ __forceinline__ T load_g(gptr<const T> G, size_t n3, size_t o) {
    if constexpr (g_last_read<DIR, C>()) return __builtin_nontemporal_load(&G[gcomp<DIR>(C) * n3 + o]);
    else return G[gcomp<DIR>(C) * n3 + o];
}
// the same with the point's byte offset
template <int DIR, int C, typename T>
__device__ __forceinline__ T load_gb(gptr<const T> G, size_t n3, uint32_t bo) {
    if constexpr (g_last_read<DIR, C>()) return __builtin_nontemporal_load(elem(G, n3, gcomp<DIR>(C), bo));
    else return *elem(G, n3, gcomp<DIR>(C), bo);
}

// viscous term alone: out = sum_d D_d G_d (the viscous-only entry point)
template <typename T>
__global__ __launch_bounds__(kPointThreads) void k_visc_div(Launch L0) {
    const Launch L = with_params(L0);
    const VbRange R = vb_range(L.total);
    for (long long vb = R.vb; vb < R.end; vb += R.stride) {
        const int bi = find_box(L.off, L.nbox, vb);
        const BoxDesc &b = L.boxes[bi];
        const int nx = b.nx, ny = b.ny, nz = b.nz;
        const size_t n3 = b.n3;
        const size_t idx = (size_t)(vb - L.off[bi]) * kPointThreads + threadIdx.x;
        if (idx >= n3) continue;
        const gptr<const T> G = glob((const T *)b.G);
        const gptr<T> out = glob((T *)(L.out_ov ? L.out_ov : b.rhs));
        const T ihx = T(b.inv_h[0]), ihy = T(b.inv_h[1]), ihz = T(b.inv_h[2]);
        const int i = (int)(idx % nx);
        const int j = (int)((idx / nx) % ny);
        const int k = (int)(idx / ((size_t)nx * ny));
        const size_t sy = nx, sz = (size_t)nx * ny;
        const size_t row = idx - i, col = idx - j * sy, pil = idx - k * sz;
        const size_t x[4] = {row + wrapi(i - 2, nx), row + wrapi(i - 1, nx), row + wrapi(i + 1, nx),
                             row + wrapi(i + 2, nx)};
        const size_t y[4] = {col + wrapi(j - 2, ny) * sy, col + wrapi(j - 1, ny) * sy, col + wrapi(j + 1, ny) * sy,
                             col + wrapi(j + 2, ny) * sy};
        const size_t z[4] = {pil + wrapi(k - 2, nz) * sz, pil + wrapi(k - 1, nz) * sz, pil + wrapi(k + 1, nz) * sz,
                             pil + wrapi(k + 2, nz) * sz};
        out[idx] = T(0);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const gptr<const T> gx = G + gcomp<0>(c) * n3;
            const gptr<const T> gy = G + gcomp<1>(c) * n3;
            const gptr<const T> gz = G + gcomp<2>(c) * n3;
            T s = dcen(gx[x[0]], gx[x[1]], gx[x[2]], gx[x[3]]) * ihx;
            s += dcen(gy[y[0]], gy[y[1]], gy[y[2]], gy[y[3]]) * ihy;
            s += dcen(gz[z[0]], gz[z[1]], gz[z[2]], gz[z[3]]) * ihz;
            out[(1 + c) * n3 + idx] = s;
        }
    }
}

// ----------------------------------------------------------------------------
// interface flux at j+1/2 from the states w and point fluxes f at j-2 .. j+3 and
// (VISC) the viscous fluxes g at j-1 .. j+2:
//   H = (f^L + f^R)/2 - |A| (u^R - u^L)/2 - (-g_{j-1} + 7 g_j + 7 g_{j+1} - g_{j+2})/12
// ----------------------------------------------------------------------------
template <typename T, typename B, int DIR, bool VISC, int WW>
__device__ __forceinline__ void interface_flux(const T w[6][5], const T f[6][5], const T g[4][4], T gamma, T eps4,
                                               T delta, T H[5]) {
    // six-fold reconstructions (eps4 = 4 eps); D is linear in du, so H = (6 F - 6 D) / 12
    T FL[5], FR[5], UL[5], UR[5], du[5], D[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        weno5_lr6<T, B, WW>(f[0][v], f[1][v], f[2][v], f[3][v], f[4][v], f[5][v], eps4, FL[v], FR[v]);
        weno5_lr6<T, B, WW>(w[0][v], w[1][v], w[2][v], w[3][v], w[4][v], w[5][v], eps4, UL[v], UR[v]);
        du[v] = UR[v] - UL[v];
    }
    roe_dissipation<T, DIR>(w[2], w[3], du, gamma, delta, D);
#pragma unroll
    for (int v = 0; v < 5; ++v) H[v] = (FL[v] + FR[v] - D[v]) * (T(1) / T(12));
    if constexpr (VISC) {
#pragma unroll
        for (int c = 0; c < 4; ++c)
            H[1 + c] -= (T(7) * (g[1][c] + g[2][c]) - (g[0][c] + g[3][c])) * (T(1) / T(12));
    }
}

// The same interface flux with the point fluxes read from the per-thread LDS ring of the
// marching sweep (slot sl[m] holds point j-2+m), one component at a time: the fence
// between components keeps the scheduler from hoisting all thirty LDS reads, which
// would hold them in registers across the whole reconstruction.  Same arithmetic, in
// the same order, as interface_flux.
template <typename T, typename B, int DIR, bool VISC, int WW>
__device__ __forceinline__ void interface_flux_ring(const T w[6][5], const T *ring, const int sl[6], int bdim,
                                                    const T g[4][4], T gamma, T eps4, T delta, T H[5]) {
    T Fs[5], du[5], D[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        T fm[6];
#pragma unroll
        for (int m = 0; m < 6; ++m) fm[m] = ring[(sl[m] * 5 + v) * bdim];
        T FL, FR, UL, UR;
        weno5_lr6<T, B, WW>(fm[0], fm[1], fm[2], fm[3], fm[4], fm[5], eps4, FL, FR);
        weno5_lr6<T, B, WW>(w[0][v], w[1][v], w[2][v], w[3][v], w[4][v], w[5][v], eps4, UL, UR);
        Fs[v] = FL + FR;
        du[v] = UR - UL;
        __builtin_amdgcn_sched_barrier(0);
    }
    roe_dissipation<T, DIR>(w[2], w[3], du, gamma, delta, D);
#pragma unroll
    for (int v = 0; v < 5; ++v) H[v] = (Fs[v] - D[v]) * (T(1) / T(12));
    if constexpr (VISC) {
#pragma unroll
        for (int c = 0; c < 4; ++c)
            H[1 + c] -= (T(7) * (g[1][c] + g[2][c]) - (g[0][c] + g[3][c])) * (T(1) / T(12));
    }
}

// The same interface flux with every operand read from the rows kernel's LDS staging
// (component-major arrays of `per` points; q[m] is the position of point i-2+m), one
// component at a time behind a scheduling fence, so that the reconstruction holds
// only the operands of the component in flight.
template <typename T, typename B, int DIR, bool VISC, int WW>
__device__ __forceinline__ void interface_flux_lds(const T *su, const T *sf, const T *sg, int per, const int q[6],
                                                   T gamma, T eps4, T delta, T H[5]) {
    T Fs[5], du[5], D[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        const T *fv = sf + v * per, *uv = su + v * per;
        T FL, FR, UL, UR;
        weno5_lr6<T, B, WW>(fv[q[0]], fv[q[1]], fv[q[2]], fv[q[3]], fv[q[4]], fv[q[5]], eps4, FL, FR);
        weno5_lr6<T, B, WW>(uv[q[0]], uv[q[1]], uv[q[2]], uv[q[3]], uv[q[4]], uv[q[5]], eps4, UL, UR);
        Fs[v] = FL + FR;
        du[v] = UR - UL;
        __builtin_amdgcn_sched_barrier(0);
    }
    T a[5], b[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        a[v] = su[v * per + q[2]];
        b[v] = su[v * per + q[3]];
    }
    roe_dissipation<T, DIR>(a, b, du, gamma, delta, D);
#pragma unroll
    for (int v = 0; v < 5; ++v) H[v] = (Fs[v] - D[v]) * (T(1) / T(12));
    if constexpr (VISC) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const T *gc = sg + c * per;
            H[1 + c] -= (T(7) * (gc[q[2]] + gc[q[3]]) - (gc[q[1]] + gc[q[4]])) * (T(1) / T(12));
        }
    }
}

// ----------------------------------------------------------------------------
// marching WENO5-Roe sweep along one direction
// ----------------------------------------------------------------------------
enum { MODE_WRITE = 0, MODE_ACCUM = 1, MODE_RK = 2 };

// geometry of a sweep along DIR: lanes run over the plane normal to DIR (p fastest)
struct SweepGeom {
    int nline, np, npq;
    size_t lstride, pstride, qstride;
};
template <int DIR>
__host__ __device__ __forceinline__ SweepGeom sweep_geom(int nx, int ny, int nz) {
    const size_t sy = (size_t)nx, sz = (size_t)nx * ny;
    if (DIR == 0) return SweepGeom{nx, ny, ny * nz, 1, sy, sz};
    if (DIR == 1) return SweepGeom{ny, nx, nx * nz, sy, 1, sz};
    return SweepGeom{nz, nx, nx * ny, sz, 1, sy};
}

// Lanes run over consecutive lines of the plane (coalesced).  For y, a block of W
// waves covers 64 lines times W consecutive segments, so neighbouring segments share
// their six-point halos in the CU's cache; for x and z a block covers 64 W lines of one
// segment (stacking z segments spreads a block over planes far apart in memory).
//
// The six point fluxes live in a per-thread ring in LDS (6 slots x 5 components,
// component-major across the wave so lanes hit distinct banks), read one component
// at a time; the registers this frees carry the loads of the next point and of the
// point's rhs, issued before the interface-flux arithmetic so their latency overlaps
// it (y sweep 12 % and fused-update sweep 6 % faster than a register window).  The
// fused update's u^n and accumulator are loaded ahead in the same way.
template <typename T, typename B, int DIR, int MODE, bool VISC, int WW>
__global__ __launch_bounds__(256, 2) void k_sweep(Launch L0) {
    const Launch L = with_params(L0);
    extern __shared__ unsigned char lds_raw[];
    // each wave's ring: slot s, component v of lane l at (s * 5 + v) * 64 + l, so the
    // component and slot strides are constants (immediate LDS offsets)
    constexpr int bdim = 64;
    T *ring = reinterpret_cast<T *>(lds_raw) + (threadIdx.x >> 6) * (30 * 64) + (threadIdx.x & 63);
    const VbRange R = vb_range(L.total);
    for (long long vb = R.vb; vb < R.end; vb += R.stride) {
        const int bi = find_box(L.off, L.nbox, vb);
        const BoxDesc &bx = L.boxes[bi];
        const SweepGeom sg = sweep_geom<DIR>(bx.nx, bx.ny, bx.nz);
        const int n = sg.nline;
        const int seg = bx.seg[DIR];
        const int nseg = (n + seg - 1) / seg;
        const long long lb = vb - L.off[bi];
        int pq, sgi;
        if constexpr (DIR == 1) {
            const int wpb = blockDim.x >> 6;
            const long long ncg = (sg.npq + 63) >> 6;
            pq = (int)((lb % ncg) << 6) + (int)(threadIdx.x & 63);
            sgi = (int)(lb / ncg) * wpb + (int)(threadIdx.x >> 6);
            if (pq >= sg.npq || sgi >= nseg) continue;
        } else {
            const size_t t = (size_t)lb * blockDim.x + threadIdx.x;
            if (t >= (size_t)sg.npq * nseg) continue;
            pq = (int)(t % sg.npq);
            sgi = (int)(t / sg.npq);
        }
        const int p = pq % sg.np, q = pq / sg.np;
        const size_t base = p * sg.pstride + q * sg.qstride;
        const int j0 = sgi * seg;
        const int j1 = min(j0 + seg, n);
        const size_t n3 = uni64(bx.n3);
        const gptr<const T> u = uni(glob((const T *)state_ptr(bx, L, L.in)));
        const gptr<const T> G = uni(glob((const T *)bx.G));
        const T gamma = T(bx.gamma), eps4 = T(4.0 * bx.eps), delta = T(bx.delta);
        const T gm1 = gamma - T(1);
        const T inv_dx = T(bx.inv_h[DIR]);
        const double dt = L.dt_ov > 0.0 ? L.dt_ov : bx.dt;
        // Every pointer the loop uses is read from the box table here, once: the loop
        // stores to global memory, which the compiler cannot tell apart from the table, so
        // a table read inside the loop would be repeated after every store, each time
        // behind a wait for all loads in flight (the ones issued ahead included).
        const gptr<const T> rhs_in = uni(glob((const T *)(MODE == MODE_RK ? bx.rhs : (L.out_ov ? L.out_ov : bx.rhs))));
        const gptr<const T> un = uni(glob((const T *)state_ptr(bx, L, BUF_U)));
        const gptr<double> acc = uni(glob(bx.acc));
        const gptr<T> unext = uni(glob((T *)state_ptr(bx, L, L.out)));
        const gptr<T> rhs_out = uni(glob((T *)(L.out_ov ? L.out_ov : bx.rhs)));

        T w[6][5], g[4][4], Hp[5], nw[5];
        // One step body computes everything, so every point flux and every interface
        // flux takes the same arithmetic in the same order wherever a segment starts:
        // results are bitwise independent of the segment length.  Step j takes point
        // j+3 (loaded one step ahead) and the viscous fluxes of point j+2; from j = j0-1
        // on it forms the interface flux at j+1/2 and from j = j0 on the flux difference
        // at point j.
        {
            const uint32_t bo = (uint32_t)((base + wrapi(j0 - 3, n) * sg.lstride) * sizeof(T));
#pragma unroll
            for (int v = 0; v < 5; ++v) nw[v] = *elem(u, n3, v, bo);
        }
        int snew = 3;  // ring slot of point j+3; point j-2+m sits in slot (snew + 1 + m) mod 6
        auto step = [&](const int j) {
#pragma unroll
            for (int m = 0; m < 5; ++m)
#pragma unroll
                for (int v = 0; v < 5; ++v) w[m][v] = w[m + 1][v];
#pragma unroll
            for (int v = 0; v < 5; ++v) w[5][v] = nw[v];
            // The window enters each step through an empty asm, so the two steps of a
            // pass share no arithmetic (the optimiser would otherwise form a point's Roe
            // terms once for both interfaces, outside the block where the other step
            // fuses them into multiply-adds): every interface flux is computed by the
            // same instructions in either step, bitwise as with one step per pass.
#pragma unroll
            for (int m = 0; m < 6; ++m)
#pragma unroll
                for (int v = 0; v < 5; ++v) asm volatile("" : "+v"(w[m][v]));
            {
                const uint32_t bo = (uint32_t)((base + wrapi(j + 4, n) * sg.lstride) * sizeof(T));
#pragma unroll
                for (int v = 0; v < 5; ++v) nw[v] = *elem(u, n3, v, bo);
            }
            if constexpr (VISC) {
#pragma unroll
                for (int m = 0; m < 3; ++m)
#pragma unroll
                    for (int c = 0; c < 4; ++c) g[m][c] = g[m + 1][c];
                const uint32_t bog = (uint32_t)((base + wrapi(j + 2, n) * sg.lstride) * sizeof(T));
                g[3][0] = load_gb<DIR, 0>(G, n3, bog);
                g[3][1] = load_gb<DIR, 1>(G, n3, bog);
                g[3][2] = load_gb<DIR, 2>(G, n3, bog);
                g[3][3] = load_gb<DIR, 3>(G, n3, bog);
#pragma unroll
                for (int m = 0; m < 3; ++m)
#pragma unroll
                    for (int c = 0; c < 4; ++c) asm volatile("" : "+v"(g[m][c]));
            }
            const int sold = snew;
            {
                T fn[5];
                euler_flux<T, DIR>(w[5], gm1, fn);
#pragma unroll
                for (int v = 0; v < 5; ++v) ring[(snew * 5 + v) * bdim] = fn[v];
                snew = snew == 5 ? 0 : snew + 1;
            }
            if (j < j0 - 1) return;

            // output operands of point j, loaded before the interface-flux arithmetic
            const size_t o = base + (size_t)(j >= j0 ? j : j0) * sg.lstride;
            const uint32_t bo = (uint32_t)(o * sizeof(T)), boa = (uint32_t)(o * sizeof(double));
            T pr[5], pu[5];
            double pa[5];
            if (MODE != MODE_WRITE && j >= j0) {
#pragma unroll
                for (int v = 0; v < 5; ++v) {
                    if constexpr (MODE == MODE_RK) pr[v] = __builtin_nontemporal_load(elem(rhs_in, n3, v, bo));
                    else pr[v] = *elem(rhs_in, n3, v, bo);
                }
                if (MODE == MODE_RK && L.stage >= 2) {
                    // u^n: every later stage but the mixed form's RK4 stage 4, which
                    // needs only the accumulator
                    if (L.scheme == CNS_TVDRK3 || kFp64Stages<T> || L.stage != 4) {
#pragma unroll
                        for (int v = 0; v < 5; ++v) pu[v] = *elem(un, n3, v, bo);
                    }
                    // the FP64 form reads the accumulator in the last stage only
                    if (L.scheme != CNS_TVDRK3 && (!kFp64Stages<T> || L.stage == 4)) {
#pragma unroll
                        for (int v = 0; v < 5; ++v) pa[v] = __builtin_nontemporal_load(elem(acc, n3, v, boa));
                    }
                }
            }

            T H[5];
            {
                int sl[6];
#pragma unroll
                for (int m = 0; m < 6; ++m) {
                    const int sm = sold + 1 + m;  // slot of point j-2+m (point j+3 is in sold)
                    sl[m] = sm >= 6 ? sm - 6 : sm;
                }
                interface_flux_ring<T, B, DIR, VISC, WW>(w, ring, sl, bdim, g, gamma, eps4, delta, H);
            }
            if (j >= j0) {
                if constexpr (MODE == MODE_RK) {
#pragma unroll
                    for (int v = 0; v < 5; ++v) {
                        const T r = -(H[v] - Hp[v]) * inv_dx;
                        const gptr<T> ue = elem(unext, n3, v, bo);
                        const gptr<double> ae = elem(acc, n3, v, boa);
                        const double k = double(pr[v] + r);
                        // w[2] holds the stage state at j: u^n itself in the first stage
                        const double us = double(w[2][v]);
                        if (L.scheme == CNS_TVDRK3) {
                            // Shu-Osher: U1 = u + dt k; U2 = 3/4 u + 1/4 (U1 + dt k);
                            // u^{n+1} = 1/3 u + 2/3 (U2 + dt k)
                            if (L.stage == 1) {
                                *ue = T(us + dt * k);
                            } else {
                                const double uo = double(pu[v]);
                                if (L.stage == 2) *ue = T(0.75 * uo + 0.25 * (us + dt * k));
                                else *ue = T((1.0 / 3.0) * uo + (2.0 / 3.0) * (us + dt * k));
                            }
                        } else if constexpr (kFp64Stages<T>) {
                            // FP64 stage states give back dt k1 / 6 = (U2 - u) / 3 and
                            // dt k3 / 3 = (U4 - u) / 3, so the accumulator is written in
                            // stage 2 and read in stage 4 only
                            if (L.stage == 1) {
                                *ue = us + (0.5 * dt) * k;
                            } else if (L.stage == 2) {
                                const double uo = pu[v];
                                __builtin_nontemporal_store((uo + (1.0 / 3.0) * (us - uo)) + (dt / 3.0) * k, ae);
                                *ue = uo + (0.5 * dt) * k;
                            } else if (L.stage == 3) {
                                *ue = pu[v] + dt * k;
                            } else {
                                *ue = (pa[v] + (1.0 / 3.0) * (us - pu[v])) + (dt / 6.0) * k;
                            }
                        } else if (L.stage == 1) {
                            *ae = us + (dt / 6.0) * k;
                            *ue = T(us + (0.5 * dt) * k);
                        } else if (L.stage == 2) {
                            const double uo = double(pu[v]);
                            *ae = pa[v] + (dt / 3.0) * k;
                            *ue = T(uo + (0.5 * dt) * k);
                        } else if (L.stage == 3) {
                            const double uo = double(pu[v]);
                            *ae = pa[v] + (dt / 3.0) * k;
                            *ue = T(uo + dt * k);
                        } else {
                            *ue = T(pa[v] + (dt / 6.0) * k);
                        }
                    }
                } else {
#pragma unroll
                    for (int v = 0; v < 5; ++v) {
                        const T r = -(H[v] - Hp[v]) * inv_dx;
                        if constexpr (MODE == MODE_WRITE) *elem(rhs_out, n3, v, bo) = r;
                        else *elem(rhs_out, n3, v, bo) = pr[v] + r;
                    }
                }
            }
#pragma unroll
            for (int v = 0; v < 5; ++v) Hp[v] = H[v];
        };
        // Two steps per pass: the window shifts of the first step become register
        // renamings instead of copies (y sweep 64 -> 26, z sweep 66 -> 30 64-bit moves
        // per point).
        int j = j0 - 6;
#pragma nounroll
        for (; j + 1 < j1; j += 2) {
            step(j);
            step(j + 1);
        }
        if (j < j1) step(j);
    }
}

// ----------------------------------------------------------------------------
// x sweep with whole periodic rows staged in LDS: one thread per point and per
// interface, lanes along x (coalesced loads and stores), `rows` rows per block of
// 256 threads, each thread handling up to P points.  Every interface of a row is
// computed once; the periodic wrap happens in LDS.
// ----------------------------------------------------------------------------
template <typename T, typename B, bool VISC, int P, int WW>
__global__ __launch_bounds__(kRowThreads, 2) void k_sweep_x_rows(Launch L0) {
    const Launch L = with_params(L0);
    extern __shared__ unsigned char lds_raw[];
    T *lds = reinterpret_cast<T *>(lds_raw);
    // A block walks over several row groups (grid stride).  With one point per thread
    // the global loads of the next group are issued into registers before the
    // interface arithmetic of the current one, so their latency overlaps it; with more
    // points per thread the extra registers would halve the occupancy, so the loads
    // stay at the top of each group.
    constexpr bool kPrefetch = P == 1;
    T pw[P][5], pg[P][4];
    auto fetch = [&](long long vb) {
        const int bi = find_box(L.off, L.nbox, vb);
        const BoxDesc &bx = L.boxes[bi];
        const int nx = bx.nx;
        const long long nrows = (long long)bx.ny * bx.nz;
        const long long row0 = (vb - L.off[bi]) * bx.rows;
        const int nact = (int)min((long long)bx.rows, nrows - row0) * nx;
        const size_t obase = (size_t)row0 * nx, n3 = bx.n3;
        const gptr<const T> u = glob((const T *)state_ptr(bx, L, L.in));
        const gptr<const T> G = glob((const T *)bx.G);
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const int t = threadIdx.x + k * kRowThreads;
            if (t < nact) {
                const size_t o = obase + t;
#pragma unroll
                for (int v = 0; v < 5; ++v) pw[k][v] = u[v * n3 + o];
                if constexpr (VISC) {
                    pg[k][0] = load_g<0, 0>(G, n3, o);
                    pg[k][1] = load_g<0, 1>(G, n3, o);
                    pg[k][2] = load_g<0, 2>(G, n3, o);
                    pg[k][3] = load_g<0, 3>(G, n3, o);
                }
            }
        }
    };
    const VbRange R = vb_range(L.total);
    if (kPrefetch && R.vb < R.end) fetch(R.vb);
    for (long long vb = R.vb; vb < R.end; vb += R.stride) {
        const int bi = find_box(L.off, L.nbox, vb);
        const BoxDesc &bx = L.boxes[bi];
        const int nx = bx.nx;
        // LDS stride of a field: the block's points, or with one point per thread (every
        // block of rows fits 256 points) the constant 256, which turns the component
        // offsets of the stencil reads into immediates
        const int per = P == 1 ? kRowThreads : bx.rows * nx;
        T *su = lds;           // [5][per] states, later the interface fluxes
        T *sf = su + 5 * per;  // [5][per] point fluxes
        T *sg = sf + 5 * per;  // [4][per] viscous fluxes (VISC)
        const size_t n3 = bx.n3;
        const T gamma = T(bx.gamma), eps4 = T(4.0 * bx.eps), delta = T(bx.delta);
        const T gm1 = gamma - T(1);
        const T inv_dx = T(bx.inv_h[0]);
        const long long nrows = (long long)bx.ny * bx.nz;
        const long long row0 = (vb - L.off[bi]) * bx.rows;
        const int nact = (int)min((long long)bx.rows, nrows - row0) * nx;  // active points
        const size_t obase = (size_t)row0 * nx;
        const gptr<T> out = glob((T *)(L.out_ov ? L.out_ov : bx.rhs));

#pragma unroll
        for (int k = 0; k < P; ++k) {
            const int t = threadIdx.x + k * kRowThreads;
            if (t < nact) {
                T wk[5], gk[4], f[5];
                if constexpr (kPrefetch) {
#pragma unroll
                    for (int v = 0; v < 5; ++v) wk[v] = pw[k][v];
#pragma unroll
                    for (int c = 0; c < 4; ++c) gk[c] = pg[k][c];
                } else {
                    const gptr<const T> u = glob((const T *)state_ptr(bx, L, L.in));
                    const gptr<const T> G = glob((const T *)bx.G);
                    const size_t o = obase + t;
#pragma unroll
                    for (int v = 0; v < 5; ++v) wk[v] = u[v * n3 + o];
                    if constexpr (VISC) {
                        gk[0] = load_g<0, 0>(G, n3, o);
                        gk[1] = load_g<0, 1>(G, n3, o);
                        gk[2] = load_g<0, 2>(G, n3, o);
                        gk[3] = load_g<0, 3>(G, n3, o);
                    }
                }
                euler_flux<T, 0>(wk, gm1, f);
#pragma unroll
                for (int v = 0; v < 5; ++v) {
                    su[v * per + t] = wk[v];
                    sf[v * per + t] = f[v];
                }
                if constexpr (VISC) {
#pragma unroll
                    for (int c = 0; c < 4; ++c) sg[c * per + t] = gk[c];
                }
            }
        }
        __syncthreads();
        if (kPrefetch && vb + R.stride < R.end) fetch(vb + R.stride);
        T H[P][5];
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const int t = threadIdx.x + k * kRowThreads;
            if (t < nact) {
                const int r = t / nx, i = t - r * nx, rb = r * nx;
                int q[6];
#pragma unroll
                for (int m = 0; m < 6; ++m) q[m] = rb + wrapi(i - 2 + m, nx);
                interface_flux_lds<T, B, 0, VISC, WW>(su, sf, sg, per, q, gamma, eps4, delta, H[k]);  // at i+1/2
            }
        }
        __syncthreads();  // every thread has read the staged states
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const int t = threadIdx.x + k * kRowThreads;
            if (t < nact)
#pragma unroll
                for (int v = 0; v < 5; ++v) su[v * per + t] = H[k][v];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const int t = threadIdx.x + k * kRowThreads;
            if (t < nact) {
                const int r = t / nx, i = t - r * nx;
                const int qm = r * nx + wrapi(i - 1, nx);
                const size_t o = obase + t;
#pragma unroll
                for (int v = 0; v < 5; ++v) out[v * n3 + o] = -(H[k][v] - su[v * per + qm]) * inv_dx;
            }
        }
        __syncthreads();  // LDS is reused by the next virtual block
    }
}

// ----------------------------------------------------------------------------
// x sweep for rows longer than a block: one block walks one periodic row in chunks of
// kRowThreads interfaces.  Chunk c stages the points c*256-2 .. c*256+258 (the six-point
// stencils of its interfaces, wrapped) in LDS and one thread forms one interface flux.
// The flux difference of point i takes the interface fluxes at i-1/2 and i+1/2; the first
// point of a chunk takes i-1/2 from the previous chunk (carried in LDS), and the row's
// first point waits for the last chunk.  Compared with staging the whole row, the LDS of
// a block no longer grows with the row (29 KB in FP64), so the CU holds twice the blocks
// at 512 points per row; each chunk re-reads five stencil points of its neighbour.
// ----------------------------------------------------------------------------
constexpr int kChunkPts = kRowThreads + 5;  // points staged per chunk
__host__ __device__ __forceinline__ size_t chunk_lds_bytes(size_t esz) { return (14 * kChunkPts + 5) * esz; }

// FP64 Jiang-Shu and WENO-Z: at least five waves per SIMD (96 VGPRs, two of them
// spilled around the chunk loop) hide the chunk barriers better than four: 512^3 x
// sweep -3 %.  The mapped weights would spill more; FP32 states need fewer registers
// (more waves by themselves, which the bound would cap).
template <typename T, typename B, bool VISC, int WW>
__global__ __launch_bounds__(kRowThreads)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 && WW != CNS_WENO_M ? 5 : 2))) void k_sweep_x_chunks(Launch L0) {
    const Launch L = with_params(L0);
    extern __shared__ unsigned char lds_raw[];
    T *su = reinterpret_cast<T *>(lds_raw);  // [5][kChunkPts] states, later the interface fluxes
    T *sf = su + 5 * kChunkPts;              // [5][kChunkPts] point fluxes
    T *sg = sf + 5 * kChunkPts;              // [4][kChunkPts] viscous fluxes (VISC)
    T *carry = sg + 4 * kChunkPts;           // [5] interface flux carried to the next chunk
    const int t = threadIdx.x;
    const VbRange R = vb_range(L.total);
    for (long long vb = R.vb; vb < R.end; vb += R.stride) {
        const int bi = find_box(L.off, L.nbox, vb);
        const BoxDesc &bx = L.boxes[bi];
        const int nx = bx.nx;
        const size_t n3 = uni64(bx.n3), obase = (size_t)(vb - L.off[bi]) * nx;
        const gptr<const T> u = uni(glob((const T *)state_ptr(bx, L, L.in)));
        const gptr<const T> G = uni(glob((const T *)bx.G));
        const gptr<T> out = uni(glob((T *)(L.out_ov ? L.out_ov : bx.rhs)));
        const T gamma = T(bx.gamma), eps4 = T(4.0 * bx.eps), delta = T(bx.delta);
        const T gm1 = gamma - T(1);
        const T inv_dx = T(bx.inv_h[0]);
        const int nch = (nx + kRowThreads - 1) / kRowThreads;
        T Hfirst[5];  // interface 1/2 of the row (thread 0)
        for (int c = 0; c < nch; ++c) {
            const int i0 = c * kRowThreads;
            for (int sp = t; sp < kChunkPts; sp += kRowThreads) {
                const size_t o = obase + wrapm(i0 - 2 + sp, nx);
                T wk[5], f[5];
#pragma unroll
                for (int v = 0; v < 5; ++v) wk[v] = u[v * n3 + o];
                euler_flux<T, 0>(wk, gm1, f);
#pragma unroll
                for (int v = 0; v < 5; ++v) {
                    su[v * kChunkPts + sp] = wk[v];
                    sf[v * kChunkPts + sp] = f[v];
                }
                if constexpr (VISC) {
                    sg[0 * kChunkPts + sp] = load_g<0, 0>(G, n3, o);
                    sg[1 * kChunkPts + sp] = load_g<0, 1>(G, n3, o);
                    sg[2 * kChunkPts + sp] = load_g<0, 2>(G, n3, o);
                    sg[3 * kChunkPts + sp] = load_g<0, 3>(G, n3, o);
                }
            }
            __syncthreads();
            const int i = i0 + t;
            const bool act = i < nx;
            T H[5];
            if (act) {
                int q[6];
#pragma unroll
                for (int m = 0; m < 6; ++m) q[m] = t + m;  // point i-2+m
                interface_flux_lds<T, B, 0, VISC, WW>(su, sf, sg, kChunkPts, q, gamma, eps4, delta, H);  // at i+1/2
            }
            __syncthreads();  // every thread has read the staged chunk
            if (act)
#pragma unroll
                for (int v = 0; v < 5; ++v) su[v * kChunkPts + t] = H[v];
            if (c == 0 && t == 0)
#pragma unroll
                for (int v = 0; v < 5; ++v) Hfirst[v] = H[v];
            __syncthreads();
            // point i from the interfaces at i-1/2 and i+1/2; the row's first point waits
            if (act && (c > 0 || t > 0)) {
                const size_t o = obase + i;
#pragma unroll
                for (int v = 0; v < 5; ++v) {
                    const T hm = t > 0 ? su[v * kChunkPts + t - 1] : carry[v];
                    out[v * n3 + o] = -(H[v] - hm) * inv_dx;
                }
            }
            __syncthreads();  // carry read; the next chunk overwrites the staging
            if (i == min(i0 + kRowThreads, nx) - 1)
#pragma unroll
                for (int v = 0; v < 5; ++v) carry[v] = H[v];
        }
        __syncthreads();  // carry now holds the interface at nx-1/2
        if (t == 0) {
#pragma unroll
            for (int v = 0; v < 5; ++v) out[v * n3 + obase] = -(Hfirst[v] - carry[v]) * inv_dx;
        }
        __syncthreads();  // LDS is reused by the next row
    }
}

// ----------------------------------------------------------------------------
// diagnostics: deterministic two-pass reduction per box
// ----------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
// the diagnostics walk the box in the tiles of the viscous-flux kernel (32 x 8 columns,
// visc_planes(nz) planes); one partial-sum block per tile, at most kDiagBlocksMax (then a
// block takes every kDiagBlocksMax-th tile)
__host__ __device__ __forceinline__ long long diag_tiles(int nx, int ny, int nz) {
    return (long long)((nx + kViscTX - 1) / kViscTX) * ((ny + kViscTY - 1) / kViscTY) *
           ((nz + visc_planes(nz) - 1) / visc_planes(nz));
}
__host__ __device__ __forceinline__ int diag_blocks(int nx, int ny, int nz) {
    const long long t = diag_tiles(nx, ny, nz);
    return (int)(t < kDiagBlocksMax ? t : kDiagBlocksMax);
}

// block reduction of CNS_NDIAG values (slot 7 a max, the others sums) in a fixed order
__device__ __forceinline__ void block_reduce_diag(const double acc[CNS_NDIAG], double (*red)[CNS_NDIAG], gptr<double> dst,
                                                  const double scale[CNS_NDIAG]) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int d = 0; d < CNS_NDIAG; ++d) {
        double v = (d == 7) ? wave_max(acc[d]) : wave_sum(acc[d]);
        if (lane == 0) red[wid][d] = v;
    }
    __syncthreads();
    if (threadIdx.x < CNS_NDIAG) {
        const int d = threadIdx.x;
        double v = red[0][d];
        for (int w2 = 1; w2 < kDiagThreads / 64; ++w2) v = (d == 7) ? fmax(v, red[w2][d]) : v + red[w2][d];
        if (dst) dst[d] = v * scale[d];
    }
    __syncthreads();
}

static_assert(kDiagThreads == kViscTX * kViscTY && kPointThreads == kViscTX * kViscTY,
              "the tiled kernels map one thread to each column of a kViscTX x kViscTY tile");

// velocity m/rho of the state at linear index i (FP64, for the diagnostics)
template <typename T>
__device__ __forceinline__ void vel_at(gptr<const T> u, size_t n3, size_t i, double v[3]) {
    const double ir = rcp(double(u[i]));
    v[0] = double(u[n3 + i]) * ir;
    v[1] = double(u[2 * n3 + i]) * ir;
    v[2] = double(u[3 * n3 + i]) * ir;
}

__device__ __forceinline__ void vel_of(const double s[5], double v[3]) {
    const double ir = rcp(s[0]);
    v[0] = s[1] * ir;
    v[1] = s[2] * ir;
    v[2] = s[3] * ir;
}

// Point quantities of one state (kinetic energy, mass, momentum, energy, the largest
// wave speed |v_d| + c, the bad-point count) added to acc; returns whether the point is
// valid (finite, rho > 0, p > 0) and its velocity in v.
__device__ __forceinline__ bool point_stats(const double s[5], double gamma, double acc[CNS_NDIAG], double v[3]) {
    const double r = s[0], mx = s[1], my = s[2], mz = s[3], e = s[4];
    const double inv = rcp(r);
    v[0] = mx * inv;
    v[1] = my * inv;
    v[2] = mz * inv;
    const double ke = 0.5 * (mx * v[0] + my * v[1] + mz * v[2]);
    const double p = (gamma - 1.0) * (e - ke);
    const bool finite = isfinite(r) && isfinite(mx) && isfinite(my) && isfinite(mz) && isfinite(e);
    if (!finite || !(r > 0.0) || !(p > 0.0)) {
        acc[8] += 1.0;
        return false;
    }
    acc[0] += ke;
    acc[2] += r;
    acc[3] += mx;
    acc[4] += my;
    acc[5] += mz;
    acc[6] += e;
    const double c = sqrt(gamma * p * inv);
    acc[7] = fmax(acc[7], fmax(fabs(v[0]), fmax(fabs(v[1]), fabs(v[2]))) + c);
    return true;
}

// Per-block partial diagnostics on the tiles of the viscous-flux kernel.  Each state
// value is loaded once per tile: a thread loads its column at plane k+2 (the point
// quantities of that plane are summed then, in plane order) and, if it owns a point of
// the halo ring, that point at plane k+2 as well; the vorticity of plane k takes the
// 4th-order central derivative of the velocity, whose x and y neighbours come from an
// LDS copy of plane k staged from the column and ring windows, and whose z neighbours
// from the column's window of five planes in registers.
template <typename T>
__global__ __launch_bounds__(kDiagThreads) void k_diag_partial(Launch L0) {
    const Launch L = with_params(L0);
    __shared__ double red[kDiagThreads / 64][CNS_NDIAG];
    __shared__ double pv[3][kViscTY + 4][kViscTX + 4];
    __shared__ double rv[3][3][kViscRing];  // ring velocities, slot (plane - z0) mod 3
    const double one[CNS_NDIAG] = {1, 1, 1, 1, 1, 1, 1, 1, 1};
    int rhx, rhy;
    ring_pos(threadIdx.x, rhx, rhy);
    const bool ring = threadIdx.x < kViscRing;
    const int rt = ring ? threadIdx.x : 0;
    const VbRange R = vb_range(L.total);
    for (long long vb = R.vb; vb < R.end; vb += R.stride) {
        const int bi = find_box(L.off, L.nbox, vb);
        const BoxDesc &bx = L.boxes[bi];
        const int nx = bx.nx, ny = bx.ny, nz = bx.nz;
        const size_t n3 = bx.n3, sz = (size_t)nx * ny;
        const int nblk = diag_blocks(nx, ny, nz);
        const long long ntile = diag_tiles(nx, ny, nz);
        const int lb = (int)(vb - L.off[bi]);
        const gptr<const T> u = glob((const T *)state_ptr(bx, L, BUF_U));
        const double gamma = bx.gamma, ihx = bx.inv_h[0], ihy = bx.inv_h[1], ihz = bx.inv_h[2];
        const int ntx = (nx + kViscTX - 1) / kViscTX, nty = (ny + kViscTY - 1) / kViscTY;
        const int tx = threadIdx.x % kViscTX, ty = threadIdx.x / kViscTX;
        double acc[CNS_NDIAG] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (long long tile = lb; tile < ntile; tile += nblk) {
            const int x0 = (int)(tile % ntx) * kViscTX, y0 = (int)((tile / ntx) % nty) * kViscTY;
            const int z0 = (int)(tile / ((long long)ntx * nty)) * visc_planes(nz), z1 = min(z0 + visc_planes(nz), nz);
            const bool act = x0 + tx < nx && y0 + ty < ny;
            // a column past a ragged edge wraps periodically (halo of the columns beside it)
            const size_t col = (size_t)wrapm(y0 + ty, ny) * nx + wrapm(x0 + tx, nx);
            const size_t rcol = (size_t)wrapm(y0 - 2 + rhy, ny) * nx + wrapm(x0 - 2 + rhx, nx);
            double vz[5][3];    // this column's velocity at planes k-2 .. k+2
            unsigned good = 0;  // bit m: the column's point at plane k-2+m is valid
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int zp = z0 - 2 + m;
                const size_t i = col + wrapi(zp, nz) * sz;
                double s[5] = {double(u[i]), double(u[n3 + i]), double(u[2 * n3 + i]), double(u[3 * n3 + i]),
                               double(u[4 * n3 + i])};
                if (act && zp >= z0 && zp < z1) {
                    if (point_stats(s, gamma, acc, vz[m])) good |= 1u << m;
                } else {
                    vel_of(s, vz[m]);
                }
            }
            if (ring) {
                for (int m = 0; m < 2; ++m) {
                    double v3[3];
                    vel_at(u, n3, rcol + wrapi(z0 + m, nz) * sz, v3);
#pragma unroll
                    for (int c = 0; c < 3; ++c) rv[m][c][rt] = v3[c];
                }
            }
            int slot = 0;  // (k - z0) mod 3
            for (int k = z0; k < z1; ++k) {
                const int slot2 = slot == 0 ? 2 : slot - 1;  // (k + 2 - z0) mod 3
                {
                    const size_t i = col + wrapi(k + 2, nz) * sz;
                    double s[5] = {double(u[i]), double(u[n3 + i]), double(u[2 * n3 + i]), double(u[3 * n3 + i]),
                                   double(u[4 * n3 + i])};
                    if (act && k + 2 < z1) {
                        if (point_stats(s, gamma, acc, vz[4])) good |= 1u << 4;
                    } else {
                        vel_of(s, vz[4]);
                    }
                }
                if (ring) {
                    double v3[3];
                    vel_at(u, n3, rcol + wrapi(k + 2, nz) * sz, v3);
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        rv[slot2][c][rt] = v3[c];
                        pv[c][rhy][rhx] = rv[slot][c][rt];
                    }
                }
#pragma unroll
                for (int c = 0; c < 3; ++c) pv[c][ty + 2][tx + 2] = vz[2][c];
                __syncthreads();
                if (act && (good & 4u)) {
                    // vorticity with the 4th-order central derivative
                    const int X = tx + 2, Y = ty + 2;
                    const double dvzdy = dcen(pv[2][Y - 2][X], pv[2][Y - 1][X], pv[2][Y + 1][X], pv[2][Y + 2][X]) * ihy;
                    const double dvydz = dcen(vz[0][1], vz[1][1], vz[3][1], vz[4][1]) * ihz;
                    const double dvxdz = dcen(vz[0][0], vz[1][0], vz[3][0], vz[4][0]) * ihz;
                    const double dvzdx = dcen(pv[2][Y][X - 2], pv[2][Y][X - 1], pv[2][Y][X + 1], pv[2][Y][X + 2]) * ihx;
                    const double dvydx = dcen(pv[1][Y][X - 2], pv[1][Y][X - 1], pv[1][Y][X + 1], pv[1][Y][X + 2]) * ihx;
                    const double dvxdy = dcen(pv[0][Y - 2][X], pv[0][Y - 1][X], pv[0][Y + 1][X], pv[0][Y + 2][X]) * ihy;
                    const double ox = dvzdy - dvydz, oy = dvxdz - dvzdx, oz = dvydx - dvxdy;
                    if (isfinite(ox) && isfinite(oy) && isfinite(oz)) acc[1] += 0.5 * (ox * ox + oy * oy + oz * oz);
                }
                __syncthreads();  // the next plane overwrites the LDS tile
#pragma unroll
                for (int m = 0; m < 4; ++m)
#pragma unroll
                    for (int c = 0; c < 3; ++c) vz[m][c] = vz[m + 1][c];
                good >>= 1;
                slot = slot == 2 ? 0 : slot + 1;
            }
        }
        block_reduce_diag(acc, red, glob(bx.part) + (size_t)lb * CNS_NDIAG, one);
    }
}

__global__ __launch_bounds__(kDiagThreads) void k_diag_final(Launch L0) {
    const Launch L = with_params(L0);
    __shared__ double red[kDiagThreads / 64][CNS_NDIAG];
    for (long long vb = blockIdx.x; vb < L.total; vb += gridDim.x) {
        const int bi = (int)vb;  // one virtual block per box
        const BoxDesc &bx = L.boxes[bi];
        const int nblk = L.diag_fused ? (int)diag_tiles(bx.nx, bx.ny, bx.nz) : diag_blocks(bx.nx, bx.ny, bx.nz);
        double acc[CNS_NDIAG] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int b = threadIdx.x; b < nblk; b += kDiagThreads)
#pragma unroll
            for (int d = 0; d < CNS_NDIAG; ++d) {
                const double v = glob(bx.part)[(size_t)b * CNS_NDIAG + d];
                acc[d] = (d == 7) ? fmax(acc[d], v) : acc[d] + v;
            }
        const double inv = 1.0 / (double)bx.n3;
        const double scale[CNS_NDIAG] = {inv, inv, inv, inv, inv, inv, inv, 1.0, 1.0};
        const gptr<double> dst = L.diag ? glob(L.diag) + ((size_t)bi * L.diag_box_stride + L.step) * CNS_NDIAG : nullptr;
        block_reduce_diag(acc, red, dst, scale);
    }
}

// ----------------------------------------------------------------------------
// the CFL wave speed alone: max over points and directions of |v_d| + c (the same
// point arithmetic as slot 7 of the diagnostics), two passes per box
// ----------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kDiagThreads) void k_speed_partial(Launch L0) {
    const Launch L = with_params(L0);
    __shared__ double red[kDiagThreads / 64][2];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const VbRange R = vb_range(L.total);
    for (long long vb = R.vb; vb < R.end; vb += R.stride) {
        const int bi = find_box(L.off, L.nbox, vb);
        const BoxDesc &bx = L.boxes[bi];
        const int nblk = diag_blocks(bx.nx, bx.ny, bx.nz);
        const int lb = (int)(vb - L.off[bi]);
        const gptr<const T> u = glob((const T *)state_ptr(bx, L, BUF_U));
        const size_t n3 = bx.n3;
        const double gamma = bx.gamma;
        double smax = 0.0, bad = 0.0;
        for (size_t i = (size_t)lb * kDiagThreads + threadIdx.x; i < n3; i += (size_t)nblk * kDiagThreads) {
            const double r = double(u[i]), mx = double(u[n3 + i]), my = double(u[2 * n3 + i]),
                         mz = double(u[3 * n3 + i]), e = double(u[4 * n3 + i]);
            const double inv = rcp(r);
            const double vx = mx * inv, vy = my * inv, vzc = mz * inv;
            const double ke = 0.5 * (mx * vx + my * vy + mz * vzc);
            const double p = (gamma - 1.0) * (e - ke);
            const bool finite = isfinite(r) && isfinite(mx) && isfinite(my) && isfinite(mz) && isfinite(e);
            if (!finite || !(r > 0.0) || !(p > 0.0)) {
                bad += 1.0;
            } else {
                const double c = sqrt(gamma * p * inv);
                smax = fmax(smax, fmax(fabs(vx), fmax(fabs(vy), fabs(vzc))) + c);
            }
        }
        smax = wave_max(smax);
        bad = wave_sum(bad);
        if (lane == 0) {
            red[wid][0] = smax;
            red[wid][1] = bad;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double m = red[0][0], b = red[0][1];
            for (int w2 = 1; w2 < kDiagThreads / 64; ++w2) {
                m = fmax(m, red[w2][0]);
                b += red[w2][1];
            }
            glob(bx.part)[(size_t)lb * CNS_NDIAG + 7] = m;
            glob(bx.part)[(size_t)lb * CNS_NDIAG + 8] = b;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(64) void k_speed_final(Launch L0, double *out) {
    const Launch L = with_params(L0);
    for (long long vb = blockIdx.x; vb < L.total; vb += gridDim.x) {
        const int bi = (int)vb;  // one virtual block per box
        const BoxDesc &bx = L.boxes[bi];
        const int nblk = diag_blocks(bx.nx, bx.ny, bx.nz);
        double m = 0.0, b = 0.0;
        for (int k = threadIdx.x; k < nblk; k += 64) {
            m = fmax(m, glob(bx.part)[(size_t)k * CNS_NDIAG + 7]);
            b += glob(bx.part)[(size_t)k * CNS_NDIAG + 8];
        }
        m = wave_max(m);
        b = wave_sum(b);
        if (threadIdx.x == 0) out[bi] = b > 0.0 ? __builtin_nan("") : m;
    }
}

// streaming copy of n16 16-byte words (bandwidth reference): each thread moves four
// words per round, the loads of a round issued before its stores
typedef double v2d __attribute__((ext_vector_type(2)));
__global__ __launch_bounds__(256) void k_stream_copy(const v2d *__restrict__ src, v2d *__restrict__ dst,
                                                     size_t n16) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n16; i += 4 * stride) {
        v2d a = __builtin_nontemporal_load(&src[i]);
        v2d b = __builtin_nontemporal_load(&src[i + stride]);
        v2d c = __builtin_nontemporal_load(&src[i + 2 * stride]);
        v2d d = __builtin_nontemporal_load(&src[i + 3 * stride]);
        __builtin_nontemporal_store(a, &dst[i]);
        __builtin_nontemporal_store(b, &dst[i + stride]);
        __builtin_nontemporal_store(c, &dst[i + 2 * stride]);
        __builtin_nontemporal_store(d, &dst[i + 3 * stride]);
    }
    for (; i < n16; i += stride) __builtin_nontemporal_store(__builtin_nontemporal_load(&src[i]), &dst[i]);
}

__global__ void k_set_params(GraphParams *gp, const void *u, double *diag, double dt) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        gp->u = u;
        gp->diag = diag;
        gp->dt = dt;
        gp->pad = 0.0;
    }
}

// ----------------------------------------------------------------------------
// host side: shapes, block counts, launchers
// ----------------------------------------------------------------------------
int rows_for(int nx) {
    int g = 1;
    while (nx * g * 2 <= kRowThreads) g *= 2;
    return g;
}

bool rows_fit(int nx, int rows, size_t esz, int *P) {
    const long long per = (long long)rows * nx;
    const long long p = (per + kRowThreads - 1) / kRowThreads;
    if (P) *P = (int)p;
    return rows >= 1 && p <= 4 && (size_t)14 * per * esz <= (size_t)kRowLdsMax;
}

static long long cdiv(long long a, long long b) { return (a + b - 1) / b; }

long long family_blocks(const BoxDesc &b, int fam, int block) {
    switch (fam) {
        case F_POINT: return cdiv((long long)b.n3, kPointThreads);
        case F_XROWS: return b.xrows == 1 ? cdiv((long long)b.ny * b.nz, b.rows) : 0;
        case F_XCHUNK: return b.xrows == 2 ? (long long)b.ny * b.nz : 0;
        case F_SWEEP_X:
        case F_SWEEP_Y:
        case F_SWEEP_Z: {
            const int d = fam - F_SWEEP_X;
            if (d == 0 && b.xrows) return 0;
            const SweepGeom g = d == 0 ? sweep_geom<0>(b.nx, b.ny, b.nz)
                                       : (d == 1 ? sweep_geom<1>(b.nx, b.ny, b.nz) : sweep_geom<2>(b.nx, b.ny, b.nz));
            if (d == 1)  // blocks of 64 lines x (block/64) segments
                return cdiv(g.npq, 64) * cdiv(cdiv(g.nline, b.seg[d]), block / 64);
            return cdiv((long long)g.npq * cdiv(g.nline, b.seg[d]), block);
        }
        case F_DIAG: return diag_blocks(b.nx, b.ny, b.nz);
        case F_VISC:
            return cdiv(b.nx, kViscTX) * cdiv(b.ny, kViscTY) * cdiv(b.nz, visc_planes(b.nz));
        case F_BOX: return 1;
    }
    return 0;
}

static Launch make_launch(const Batch &bt, int fam) {
    Launch L{};
    L.gp = bt.gp;
    L.boxes = bt.d_boxes;
    L.off = bt.d_off[fam];
    L.nbox = bt.nbox;
    L.total = bt.total[fam];
    return L;
}

static Launch with_family(const Batch &bt, Launch L, int fam) {
    L.off = bt.d_off[fam];
    L.total = bt.total[fam];
    return L;
}

static inline unsigned grid_for(long long total) {
    const long long cap = 1ll << 30;
    return (unsigned)(total < cap ? total : cap);
}

// launched blocks of family fam: bt.grid[fam] when set (a persistent launch), else one
// per virtual block
static inline unsigned grid_of(const Batch &bt, int fam, long long total) {
    const long long g = bt.grid[fam];
    return grid_for(g > 0 && g < total ? g : total);
}

void launch_init_state(int prec, size_t n3, double gamma, const double *rho, const double *vel, const double *p,
                       void *u, hipStream_t s) {
    const unsigned g = (unsigned)((n3 + 255) / 256);
    if (prec == CNS_FP64)
        hipLaunchKernelGGL(k_init_state<double>, dim3(g), dim3(256), 0, s, n3, gamma - 1.0, rho, vel, p, (double *)u);
    else
        hipLaunchKernelGGL(k_init_state<float>, dim3(g), dim3(256), 0, s, n3, gamma - 1.0, rho, vel, p, (float *)u);
}

void launch_fill(int prec, size_t n, void *out, hipStream_t s) {
    const unsigned g = (unsigned)((n + 255) / 256);
    if (prec == CNS_FP64) hipLaunchKernelGGL(k_fill<double>, dim3(g), dim3(256), 0, s, n, (double *)out);
    else hipLaunchKernelGGL(k_fill<float>, dim3(g), dim3(256), 0, s, n, (float *)out);
}

template <typename T, bool DIAG = false>
static void visc_fields(const Batch &bt, Launch L) {
    L = with_family(bt, L, F_VISC);
    if (!L.total) return;
    ProfScope ps(bt.prof, K_VISC_FLUX, bt.stream);
    hipLaunchKernelGGL((k_visc_flux<T, DIAG>), dim3(grid_of(bt, F_VISC, L.total)), dim3(kPointThreads), 0, bt.stream,
                       L);
}

template <typename T, int DIR, int MODE, bool VISC>
static void sweep_t(const Batch &bt, const Launch &L) {
    const dim3 g(grid_of(bt, F_SWEEP_X + DIR, L.total)), b(bt.block);
    const size_t ring = 30 * (size_t)bt.block * sizeof(T);  // point-flux ring, 6 slots x 5 per thread
    if (bt.weights == CNS_WENO_Z)
        hipLaunchKernelGGL((k_sweep<T, double, DIR, MODE, VISC, CNS_WENO_Z>), g, b, ring, bt.stream, L);
    else if (bt.weights == CNS_WENO_M)
        hipLaunchKernelGGL((k_sweep<T, double, DIR, MODE, VISC, CNS_WENO_M>), g, b, ring, bt.stream, L);
    else
        hipLaunchKernelGGL((k_sweep<T, double, DIR, MODE, VISC, CNS_WENO_JS>), g, b, ring, bt.stream, L);
}

template <typename T, int MODE>
static void sweep(const Batch &bt, Launch L, int dir, bool visc) {
    L = with_family(bt, L, F_SWEEP_X + dir);
    if (!L.total) return;
    if (visc) {
        if (dir == 0) sweep_t<T, 0, MODE, true>(bt, L);
        else if (dir == 1) sweep_t<T, 1, MODE, true>(bt, L);
        else sweep_t<T, 2, MODE, true>(bt, L);
    } else {
        if (dir == 0) sweep_t<T, 0, MODE, false>(bt, L);
        else if (dir == 1) sweep_t<T, 1, MODE, false>(bt, L);
        else sweep_t<T, 2, MODE, false>(bt, L);
    }
}

template <typename T, bool VISC, int WW>
static void xrows_tw(const Batch &bt, const Launch &L) {
    // about four row groups per block when the loads of the next one are prefetched
    const long long nb = bt.grid[F_XROWS] > 0 ? std::min<long long>(bt.grid[F_XROWS], L.total)
                         : (bt.rowP == 1 ? std::max<long long>(std::min<long long>(L.total, 2048), L.total / 4)
                                         : L.total);
    const dim3 g(grid_for(nb)), b(kRowThreads);
    switch (bt.rowP) {
        case 1: hipLaunchKernelGGL((k_sweep_x_rows<T, double, VISC, 1, WW>), g, b, bt.rowLds, bt.stream, L); break;
        case 2: hipLaunchKernelGGL((k_sweep_x_rows<T, double, VISC, 2, WW>), g, b, bt.rowLds, bt.stream, L); break;
        case 3: hipLaunchKernelGGL((k_sweep_x_rows<T, double, VISC, 3, WW>), g, b, bt.rowLds, bt.stream, L); break;
        default: hipLaunchKernelGGL((k_sweep_x_rows<T, double, VISC, 4, WW>), g, b, bt.rowLds, bt.stream, L); break;
    }
}

template <typename T, bool VISC>
static void xrows_t(const Batch &bt, const Launch &L) {
    if (bt.weights == CNS_WENO_Z) xrows_tw<T, VISC, CNS_WENO_Z>(bt, L);
    else if (bt.weights == CNS_WENO_M) xrows_tw<T, VISC, CNS_WENO_M>(bt, L);
    else xrows_tw<T, VISC, CNS_WENO_JS>(bt, L);
}

template <typename T, bool VISC>
static void xchunks_t(const Batch &bt, const Launch &L) {
    const dim3 g(grid_of(bt, F_XCHUNK, L.total)), b(kRowThreads);
    const size_t lds = chunk_lds_bytes(sizeof(T));
    if (bt.weights == CNS_WENO_Z)
        hipLaunchKernelGGL((k_sweep_x_chunks<T, double, VISC, CNS_WENO_Z>), g, b, lds, bt.stream, L);
    else if (bt.weights == CNS_WENO_M)
        hipLaunchKernelGGL((k_sweep_x_chunks<T, double, VISC, CNS_WENO_M>), g, b, lds, bt.stream, L);
    else
        hipLaunchKernelGGL((k_sweep_x_chunks<T, double, VISC, CNS_WENO_JS>), g, b, lds, bt.stream, L);
}

// x sweep (always the first, writing sweep): the rows kernel for boxes whose rows fill at
// most one block, the chunked rows kernel for longer rows, the marching kernel when chosen
template <typename T>
static void sweep_x(const Batch &bt, const Launch &L, bool visc) {
    ProfScope ps(bt.prof, K_SWEEP_X, bt.stream);
    const Launch R = with_family(bt, L, F_XROWS);
    if (R.total) {
        if (visc) xrows_t<T, true>(bt, R);
        else xrows_t<T, false>(bt, R);
    }
    const Launch C = with_family(bt, L, F_XCHUNK);
    if (C.total) {
        if (visc) xchunks_t<T, true>(bt, C);
        else xchunks_t<T, false>(bt, C);
    }
    sweep<T, MODE_WRITE>(bt, L, 0, visc);
}

template <typename T>
static void rhs_t(const Batch &bt, const void *u_ov, void *out_ov) {
    Launch L = make_launch(bt, F_POINT);
    L.in = BUF_U;
    L.u_ov = u_ov;
    L.out_ov = out_ov;
    if (bt.any_visc) visc_fields<T>(bt, L);
    sweep_x<T>(bt, L, bt.any_visc);
    {
        ProfScope ps(bt.prof, K_SWEEP_Y, bt.stream);
        sweep<T, MODE_ACCUM>(bt, L, 1, bt.any_visc);
    }
    ProfScope ps(bt.prof, K_SWEEP_Z, bt.stream);
    sweep<T, MODE_ACCUM>(bt, L, 2, bt.any_visc);
}

void launch_rhs(const Batch &bt, const void *u_ov, void *out_ov) {
    if (bt.prec == CNS_FP64) rhs_t<double>(bt, u_ov, out_ov);
    else rhs_t<float>(bt, u_ov, out_ov);
}

template <typename T>
static void rhs_dir_t(const Batch &bt, const void *u_ov, int dir, void *out_ov) {
    Launch L = make_launch(bt, F_POINT);
    L.in = BUF_U;
    L.u_ov = u_ov;
    L.out_ov = out_ov;
    if (dir == 0) sweep_x<T>(bt, L, false);
    else sweep<T, MODE_WRITE>(bt, L, dir, false);
}

void launch_rhs_dir(const Batch &bt, const void *u_ov, int dir, void *out_ov) {
    if (bt.prec == CNS_FP64) rhs_dir_t<double>(bt, u_ov, dir, out_ov);
    else rhs_dir_t<float>(bt, u_ov, dir, out_ov);
}

template <typename T>
static void viscous_t(const Batch &bt, const void *u_ov, void *out_ov) {
    Launch L = make_launch(bt, F_POINT);
    L.in = BUF_U;
    L.u_ov = u_ov;
    L.out_ov = out_ov;
    visc_fields<T>(bt, L);
    hipLaunchKernelGGL(k_visc_div<T>, dim3(grid_for(L.total)), dim3(kPointThreads), 0, bt.stream, L);
}

void launch_viscous(const Batch &bt, const void *u_ov, void *out_ov) {
    if (bt.prec == CNS_FP64) viscous_t<double>(bt, u_ov, out_ov);
    else viscous_t<float>(bt, u_ov, out_ov);
}

template <typename T>
static void diag_t(const Batch &bt, const void *u_ov, double *diag, long long stride, int step) {
    ProfScope ps(bt.prof, K_DIAG, bt.stream);
    Launch L = make_launch(bt, F_DIAG);
    L.u_ov = u_ov;
    L.diag = diag;
    L.diag_box_stride = stride;
    L.step = step;
    hipLaunchKernelGGL(k_diag_partial<T>, dim3(grid_of(bt, F_DIAG, L.total)), dim3(kDiagThreads), 0, bt.stream, L);
    const Launch F = with_family(bt, L, F_BOX);
    hipLaunchKernelGGL(k_diag_final, dim3(grid_for(F.total)), dim3(kDiagThreads), 0, bt.stream, F);
}

void launch_max_wave_speed(const Batch &bt, const void *u_ov, double *out) {
    Launch L = make_launch(bt, F_DIAG);
    L.u_ov = u_ov;
    if (bt.prec == CNS_FP64)
        hipLaunchKernelGGL(k_speed_partial<double>, dim3(grid_for(L.total)), dim3(kDiagThreads), 0, bt.stream, L);
    else
        hipLaunchKernelGGL(k_speed_partial<float>, dim3(grid_for(L.total)), dim3(kDiagThreads), 0, bt.stream, L);
    const Launch F = with_family(bt, L, F_BOX);
    hipLaunchKernelGGL(k_speed_final, dim3(grid_for(F.total)), dim3(64), 0, bt.stream, F, out);
}

void launch_stream_copy(const void *src, void *dst, size_t bytes, hipStream_t s) {
    const size_t n16 = bytes / 16;
    // 8 blocks of 256 threads per CU on the 256 CUs
    const unsigned g = (unsigned)std::min<size_t>((n16 + 255) / 256, 2048);
    if (n16) hipLaunchKernelGGL(k_stream_copy, dim3(g), dim3(256), 0, s, (const v2d *)src, (v2d *)dst, n16);
}

void launch_set_params(GraphParams *gp, const void *u, double *diag, double dt, hipStream_t s) {
    hipLaunchKernelGGL(k_set_params, dim3(1), dim3(64), 0, s, gp, u, diag, dt);
}

void launch_diag(const Batch &bt, const void *u_ov, double *diag, long long stride, int step) {
    if (bt.prec == CNS_FP64) diag_t<double>(bt, u_ov, diag, stride, step);
    else diag_t<float>(bt, u_ov, diag, stride, step);
}

// the device table of one box, written from a kernel argument (no host-to-device copy)
__global__ void k_write_table(OneBoxTable t, OneBoxTable *dst) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = t;
}

size_t static_diag_bytes() { return align_up256(sizeof(OneBoxTable)) + (size_t)kDiagBlocksMax * CNS_NDIAG * sizeof(double); }

void launch_diag_static(char *scratch_dev, const BoxDesc &b, int prec, const void *u, double *out, hipStream_t s) {
    OneBoxTable t{};
    t.b = b;
    t.b.part = (double *)(scratch_dev + align_up256(sizeof(OneBoxTable)));
    for (int f = 0; f < F_N; ++f) {
        t.off[f][0] = 0;
        t.off[f][1] = family_blocks(t.b, f, 256);
    }
    OneBoxTable *dt = (OneBoxTable *)scratch_dev;
    hipLaunchKernelGGL(k_write_table, dim3(1), dim3(64), 0, s, t, dt);
    Batch bt;
    bt.nbox = 1;
    bt.prec = prec;
    bt.d_boxes = &dt->b;
    for (int f = 0; f < F_N; ++f) {
        bt.d_off[f] = dt->off[f];
        bt.total[f] = t.off[f][1];
    }
    bt.stream = s;
    launch_diag(bt, u, out, 0, 0);
}



// The first stage's viscous-flux launch of a step, forming the diagnostics of the state
// it reads (record diag_prev) when diag_prev >= 0 (FP64, viscous batches), then their
// per-box reduction.
template <typename T>
static void first_visc(const Batch &bt, Launch L, double *diag, long long stride, int diag_prev) {
    if constexpr (std::is_same<T, double>::value) {
        if (diag_prev >= 0) {
            L.diag = diag;
            L.diag_box_stride = stride;
            L.step = diag_prev;
            L.diag_fused = 1;
            visc_fields<T, true>(bt, L);
            const Launch F = with_family(bt, L, F_BOX);
            hipLaunchKernelGGL(k_diag_final, dim3(grid_for(F.total)), dim3(kDiagThreads), 0, bt.stream, F);
            return;
        }
    }
    visc_fields<T>(bt, L);
}

template <typename T>
static void rk4_step_t(const Batch &bt, const void *u_ov, double dt_ov, double *diag, long long stride, int step,
                       void *const *stage_states, int diag_prev, bool diag_own) {
    // stage s reads U_s and writes U_{s+1}: U_1 = u, U_2 -> A, U_3 -> B, U_4 -> A, u^{n+1} -> u;
    // with stage_states, A is U2's buffer for stages 1-2 and U4's for stages 3-4, B is U3's
    const int in_of[4] = {BUF_U, BUF_A, BUF_B, BUF_A};
    const int out_of[4] = {BUF_A, BUF_B, BUF_A, BUF_U};
    for (int s = 0; s < 4; ++s) {
        Launch L = make_launch(bt, F_POINT);
        L.in = in_of[s];
        L.out = out_of[s];
        L.stage = s + 1;
        L.u_ov = u_ov;
        if (stage_states) {
            L.a_ov = stage_states[s < 2 ? 0 : 2];
            L.b_ov = stage_states[1];
        }
        L.dt_ov = dt_ov;
        if (bt.any_visc) {
            if (s == 0) first_visc<T>(bt, L, diag, stride, diag_prev);
            else visc_fields<T>(bt, L);
        }
        sweep_x<T>(bt, L, bt.any_visc);
        {
            ProfScope ps(bt.prof, K_SWEEP_Y, bt.stream);
            sweep<T, MODE_ACCUM>(bt, L, 1, bt.any_visc);
        }
        ProfScope ps(bt.prof, K_SWEEP_Z, bt.stream);
        sweep<T, MODE_RK>(bt, L, 2, bt.any_visc);
    }
    if (diag && diag_own) diag_t<T>(bt, u_ov, diag, stride, step);
}

void launch_rk4_step(const Batch &bt, const void *u_ov, double dt_ov, double *diag, long long stride, int step,
                     void *const *stage_states, int diag_prev, bool diag_own) {
    if (bt.prec == CNS_FP64) rk4_step_t<double>(bt, u_ov, dt_ov, diag, stride, step, stage_states, diag_prev, diag_own);
    else rk4_step_t<float>(bt, u_ov, dt_ov, diag, stride, step, stage_states, diag_prev, diag_own);
}

template <typename T>
static void tvdrk3_step_t(const Batch &bt, const void *u_ov, double dt_ov, double *diag, long long stride,
                          int step, void *const *stage_states, int diag_prev, bool diag_own) {
    // stage s reads U_s and writes U_{s+1}: U_1 = u, U_2 -> A, U_3 -> B, u^{n+1} -> u;
    // with stage_states, A is stage_states[0] and B stage_states[1]
    const int in_of[3] = {BUF_U, BUF_A, BUF_B};
    const int out_of[3] = {BUF_A, BUF_B, BUF_U};
    for (int s = 0; s < 3; ++s) {
        Launch L = make_launch(bt, F_POINT);
        L.in = in_of[s];
        L.out = out_of[s];
        L.stage = s + 1;
        L.scheme = CNS_TVDRK3;
        L.u_ov = u_ov;
        L.dt_ov = dt_ov;
        if (stage_states) {
            L.a_ov = stage_states[0];
            L.b_ov = stage_states[1];
        }
        if (bt.any_visc) {
            if (s == 0) first_visc<T>(bt, L, diag, stride, diag_prev);
            else visc_fields<T>(bt, L);
        }
        sweep_x<T>(bt, L, bt.any_visc);
        {
            ProfScope ps(bt.prof, K_SWEEP_Y, bt.stream);
            sweep<T, MODE_ACCUM>(bt, L, 1, bt.any_visc);
        }
        ProfScope ps(bt.prof, K_SWEEP_Z, bt.stream);
        sweep<T, MODE_RK>(bt, L, 2, bt.any_visc);
    }
    if (diag && diag_own) diag_t<T>(bt, u_ov, diag, stride, step);
}

void launch_step(const Batch &bt, int scheme, const void *u_ov, double dt_ov, double *diag, long long stride,
                 int step, void *const *stage_states, int diag_prev, bool diag_own) {
    if (scheme == CNS_RK4)
        return launch_rk4_step(bt, u_ov, dt_ov, diag, stride, step, stage_states, diag_prev, diag_own);
    if (bt.prec == CNS_FP64)
        tvdrk3_step_t<double>(bt, u_ov, dt_ov, diag, stride, step, stage_states, diag_prev, diag_own);
    else tvdrk3_step_t<float>(bt, u_ov, dt_ov, diag, stride, step, stage_states, diag_prev, diag_own);
}

float time_sweeps_yz(const Batch &bt, int reps) {
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    Launch L = make_launch(bt, F_POINT);
    L.in = BUF_U;
    (void)hipEventRecord(a, bt.stream);
    for (int r = 0; r < reps; ++r) {
        if (bt.prec == CNS_FP64) {
            sweep<double, MODE_WRITE>(bt, L, 1, bt.any_visc);
            sweep<double, MODE_WRITE>(bt, L, 2, bt.any_visc);
        } else {
            sweep<float, MODE_WRITE>(bt, L, 1, bt.any_visc);
            sweep<float, MODE_WRITE>(bt, L, 2, bt.any_visc);
        }
    }
    (void)hipEventRecord(b, bt.stream);
    (void)hipEventSynchronize(b);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return ms / (float)(reps > 0 ? reps : 1);
}

float time_rhs_kernels(const Batch &bt, int reps) {
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    (void)hipEventRecord(a, bt.stream);
    for (int r = 0; r < reps; ++r) launch_rhs(bt, nullptr, nullptr);
    (void)hipEventRecord(b, bt.stream);
    (void)hipEventSynchronize(b);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return ms / (float)(reps > 0 ? reps : 1);
}

static long long cu_count() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                                 hipSuccess)
        return 256;
    return cus;
}

long long resident_sweep_blocks(const Batch &bt) {
    int n = 0;
    const size_t ring = 30 * (size_t)bt.block * (bt.prec == CNS_FP64 ? sizeof(double) : sizeof(float));
    hipError_t e = bt.prec == CNS_FP64
                       ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                             &n, k_sweep<double, double, 2, MODE_RK, true, CNS_WENO_JS>, bt.block, ring)
                       : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                             &n, k_sweep<float, double, 2, MODE_RK, true, CNS_WENO_JS>, bt.block, ring);
    return (e == hipSuccess && n > 0 ? n : 1) * cu_count();
}

long long resident_tile_blocks(const Batch &bt) {
    int n = 0;
    hipError_t e = bt.prec == CNS_FP64
                       ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_visc_flux<double, false>, kPointThreads, 0)
                       : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_visc_flux<float, false>, kPointThreads, 0);
    return (e == hipSuccess && n > 0 ? n : 1) * cu_count();
}

void prof_flush(Prof *p) {
    if (!p || !p->on || p->n == 0) return;
    (void)hipEventSynchronize(p->ev[2 * p->n - 1]);
    for (int i = 0; i < p->n; ++i) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p->ev[2 * i], p->ev[2 * i + 1]) == hipSuccess) {
            p->ms[p->kind[i]] += ms;
            p->count[p->kind[i]] += 1;
        }
    }
    p->n = 0;
}

}  // namespace cns
