// cns_kernels.hip -- gfx950 kernels of the WENO5-Roe / central-viscous RHS and RK4.
//
// Data layout in HBM: SoA state u[v][k][j][i] (x fastest).  One RHS evaluation is
//   1. k_prim       : u -> W = (u, v, w, T)                          [4][N3]
//   2. k_visc_flux  : W -> viscous fluxes G = (tau_xx, tau_yy, tau_zz, tau_xy,
//                     tau_xz, tau_yz, E_x, E_y, E_z), E_d = v.tau_d - q_d   [9][N3]
//   3. k_sweep<x>   : u, G -> rhs  (write)
//   4. k_sweep<y>   : u, G -> rhs  (accumulate)
//   5. k_sweep<z>   : u, G -> rhs  (accumulate), or the fused RK4 stage update
// Each sweep thread owns a segment of one grid line along the sweep direction and
// marches along it with a six-point register window: every point's flux is
// computed once, every interface flux once per segment, and the flux difference
// is formed in registers.  The viscous term along d enters the same difference as
// the interface flux (-G_{j-1} + 7 G_j + 7 G_{j+1} - G_{j+2}) / 12, whose
// difference is the 5-point central derivative of G.  Periodic boundaries wrap
// the line index; there are no ghost cells.
#include <hip/hip_runtime.h>

#include "cns_internal.h"

namespace cns {

__device__ __forceinline__ int wrapi(int j, int n) { return j < 0 ? j + n : (j >= n ? j - n : j); }

// ----------------------------------------------------------------------------
// state from primitives (Sec. 2.1 equation of state)
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
__global__ void k_fill(size_t n, T v, T *out) {
    size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (i < n) out[i] = v;
}

// ----------------------------------------------------------------------------
// viscous terms: primitives, then viscous fluxes at points
// ----------------------------------------------------------------------------
template <typename T>
__global__ void k_prim(size_t n3, T gamma, const T *__restrict__ u, T *__restrict__ W) {
    size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (i >= n3) return;
    T r = u[i], mx = u[n3 + i], my = u[2 * n3 + i], mz = u[3 * n3 + i], e = u[4 * n3 + i];
    T inv = T(1) / r;
    T vx = mx * inv, vy = my * inv, vz = mz * inv;
    T p = (gamma - T(1)) * (e - T(0.5) * (mx * vx + my * vy + mz * vz));
    W[i] = vx;
    W[n3 + i] = vy;
    W[2 * n3 + i] = vz;
    W[3 * n3 + i] = gamma * p * inv;  // T = gamma p / rho
}

template <typename T>
__global__ void k_visc_flux(int nx, int ny, int nz, T ihx, T ihy, T ihz, T mu, T kcond, const T *__restrict__ W,
                            T *__restrict__ G) {
    size_t n3 = (size_t)nx * ny * nz;
    size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (idx >= n3) return;
    int i = (int)(idx % nx);
    int j = (int)((idx / nx) % ny);
    int k = (int)(idx / ((size_t)nx * ny));
    const size_t sy = nx, sz = (size_t)nx * ny;
    size_t row = idx - i;
    size_t xm2 = row + wrapi(i - 2, nx), xm1 = row + wrapi(i - 1, nx), xp1 = row + wrapi(i + 1, nx),
           xp2 = row + wrapi(i + 2, nx);
    size_t col = idx - j * sy;
    size_t ym2 = col + wrapi(j - 2, ny) * sy, ym1 = col + wrapi(j - 1, ny) * sy, yp1 = col + wrapi(j + 1, ny) * sy,
           yp2 = col + wrapi(j + 2, ny) * sy;
    size_t pil = idx - k * sz;
    size_t zm2 = pil + wrapi(k - 2, nz) * sz, zm1 = pil + wrapi(k - 1, nz) * sz, zp1 = pil + wrapi(k + 1, nz) * sz,
           zp2 = pil + wrapi(k + 2, nz) * sz;
    T g[4][3];  // g[a][b] = d W_a / d x_b
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const T *f = W + a * n3;
        g[a][0] = dcen(f[xm2], f[xm1], f[xp1], f[xp2]) * ihx;
        g[a][1] = dcen(f[ym2], f[ym1], f[yp1], f[yp2]) * ihy;
        g[a][2] = dcen(f[zm2], f[zm1], f[zp1], f[zp2]) * ihz;
    }
    T div = g[0][0] + g[1][1] + g[2][2];
    T tdiv = T(2) / T(3) * div;
    T txx = mu * (T(2) * g[0][0] - tdiv);
    T tyy = mu * (T(2) * g[1][1] - tdiv);
    T tzz = mu * (T(2) * g[2][2] - tdiv);
    T txy = mu * (g[0][1] + g[1][0]);
    T txz = mu * (g[0][2] + g[2][0]);
    T tyz = mu * (g[1][2] + g[2][1]);
    T vx = W[idx], vy = W[n3 + idx], vz = W[2 * n3 + idx];
    G[idx] = txx;
    G[n3 + idx] = tyy;
    G[2 * n3 + idx] = tzz;
    G[3 * n3 + idx] = txy;
    G[4 * n3 + idx] = txz;
    G[5 * n3 + idx] = tyz;
    // E_d = v . tau_d - q_d,  q_d = -kcond dT/dx_d
    G[6 * n3 + idx] = vx * txx + vy * txy + vz * txz + kcond * g[3][0];
    G[7 * n3 + idx] = vx * txy + vy * tyy + vz * tyz + kcond * g[3][1];
    G[8 * n3 + idx] = vx * txz + vy * tyz + vz * tzz + kcond * g[3][2];
}

// which G field holds component (momentum x, y, z, energy) of the viscous flux along DIR
template <int DIR>
__device__ __forceinline__ constexpr int gcomp(int c) {
    return DIR == 0 ? (c == 0 ? 0 : c == 1 ? 3 : c == 2 ? 4 : 6)
                    : (DIR == 1 ? (c == 0 ? 3 : c == 1 ? 1 : c == 2 ? 5 : 7) : (c == 0 ? 4 : c == 1 ? 5 : c == 2 ? 2 : 8));
}

// viscous term alone: out = sum_d D_d G_d (used by the viscous-only entry point)
template <typename T>
__global__ void k_visc_div(int nx, int ny, int nz, T ihx, T ihy, T ihz, const T *__restrict__ G, T *__restrict__ out) {
    size_t n3 = (size_t)nx * ny * nz;
    size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (idx >= n3) return;
    int i = (int)(idx % nx);
    int j = (int)((idx / nx) % ny);
    int k = (int)(idx / ((size_t)nx * ny));
    const size_t sy = nx, sz = (size_t)nx * ny;
    size_t row = idx - i, col = idx - j * sy, pil = idx - k * sz;
    size_t x[4] = {row + wrapi(i - 2, nx), row + wrapi(i - 1, nx), row + wrapi(i + 1, nx), row + wrapi(i + 2, nx)};
    size_t y[4] = {col + wrapi(j - 2, ny) * sy, col + wrapi(j - 1, ny) * sy, col + wrapi(j + 1, ny) * sy,
                   col + wrapi(j + 2, ny) * sy};
    size_t z[4] = {pil + wrapi(k - 2, nz) * sz, pil + wrapi(k - 1, nz) * sz, pil + wrapi(k + 1, nz) * sz,
                   pil + wrapi(k + 2, nz) * sz};
    out[idx] = T(0);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const T *gx = G + gcomp<0>(c) * n3;
        const T *gy = G + gcomp<1>(c) * n3;
        const T *gz = G + gcomp<2>(c) * n3;
        T s = dcen(gx[x[0]], gx[x[1]], gx[x[2]], gx[x[3]]) * ihx;
        s += dcen(gy[y[0]], gy[y[1]], gy[y[2]], gy[y[3]]) * ihy;
        s += dcen(gz[z[0]], gz[z[1]], gz[z[2]], gz[z[3]]) * ihz;
        out[(1 + c) * n3 + idx] = s;
    }
}

// ----------------------------------------------------------------------------
// the WENO5-Roe sweep along one direction
// ----------------------------------------------------------------------------
enum { MODE_WRITE = 0, MODE_ACCUM = 1, MODE_RK = 2 };

template <typename T>
struct SweepArgs {
    const T *u;  // state being differentiated
    const T *G;  // viscous fluxes [9][N3] (VISC only)
    T *rhs;      // output / accumulation buffer
    // fused RK4 stage update (MODE_RK)
    const T *un;
    double *acc;
    T *unext;
    double dt;
    int stage;
    // geometry: lanes run over the plane (p fastest), threads march along the line
    size_t n3;
    int nline;
    size_t lstride;
    int np;
    size_t pstride, qstride;
    int npq, seg, nseg;
    T inv_dx;
    T gamma, eps, delta;
};

template <typename T, typename B, int DIR, int MODE, bool VISC>
__global__ __launch_bounds__(256) void k_sweep(SweepArgs<T> a) {
    const size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (t >= (size_t)a.npq * a.nseg) return;
    const int pq = (int)(t % a.npq);
    const int sg = (int)(t / a.npq);
    const int p = pq % a.np, q = pq / a.np;
    const size_t base = p * a.pstride + q * a.qstride;
    const int n = a.nline;
    const int j0 = sg * a.seg;
    const int j1 = min(j0 + a.seg, n);
    const size_t n3 = a.n3;
    const T gm1 = a.gamma - T(1);

    T w[6][5], f[6][5], g[4][4], Hp[5];
    // One loop computes everything, so every point flux and every interface flux
    // runs the same machine code wherever a segment starts: results are bitwise
    // independent of the segment length.  Iteration j loads point j+3 (and the
    // viscous fluxes of point j+2); from j = j0-1 on it forms the interface flux at
    // j+1/2 and from j = j0 on the flux difference at point j.
#pragma nounroll
    for (int j = j0 - 6; j < j1; ++j) {
#pragma unroll
        for (int m = 0; m < 5; ++m)
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                w[m][v] = w[m + 1][v];
                f[m][v] = f[m + 1][v];
            }
        {
            const size_t o = base + wrapi(j + 3, n) * a.lstride;
#pragma unroll
            for (int v = 0; v < 5; ++v) w[5][v] = a.u[v * n3 + o];
            euler_flux<T, DIR>(w[5], gm1, f[5]);
        }
        if constexpr (VISC) {
#pragma unroll
            for (int m = 0; m < 3; ++m)
#pragma unroll
                for (int c = 0; c < 4; ++c) g[m][c] = g[m + 1][c];
            const size_t o = base + wrapi(j + 2, n) * a.lstride;
#pragma unroll
            for (int c = 0; c < 4; ++c) g[3][c] = a.G[gcomp<DIR>(c) * n3 + o];
        }
        if (j < j0 - 1) continue;

        // interface flux at j+1/2 from the window j-2 .. j+3
        T H[5];
        {
            T FL[5], FR[5], UL[5], UR[5], du[5], D[5];
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                weno5_lr<T, B>(f[0][v], f[1][v], f[2][v], f[3][v], f[4][v], f[5][v], a.eps, FL[v], FR[v]);
                weno5_lr<T, B>(w[0][v], w[1][v], w[2][v], w[3][v], w[4][v], w[5][v], a.eps, UL[v], UR[v]);
                du[v] = UR[v] - UL[v];
            }
            roe_dissipation<T, DIR>(w[2], w[3], du, a.gamma, a.delta, D);
#pragma unroll
            for (int v = 0; v < 5; ++v) H[v] = T(0.5) * (FL[v] + FR[v]) - T(0.5) * D[v];
            if constexpr (VISC) {
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    H[1 + c] -= (T(7) * (g[1][c] + g[2][c]) - (g[0][c] + g[3][c])) * (T(1) / T(12));
            }
        }
        if (j >= j0) {
            const size_t o = base + (size_t)j * a.lstride;
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                const T r = -(H[v] - Hp[v]) * a.inv_dx;
                const size_t e = v * n3 + o;
                if constexpr (MODE == MODE_WRITE) {
                    a.rhs[e] = r;
                } else if constexpr (MODE == MODE_ACCUM) {
                    a.rhs[e] += r;
                } else {
                    const double k = double(a.rhs[e] + r);
                    const double un = double(a.un[e]);
                    if (a.stage == 1) {
                        a.acc[e] = un + (a.dt / 6.0) * k;
                        a.unext[e] = T(un + (0.5 * a.dt) * k);
                    } else if (a.stage == 2) {
                        a.acc[e] += (a.dt / 3.0) * k;
                        a.unext[e] = T(un + (0.5 * a.dt) * k);
                    } else if (a.stage == 3) {
                        a.acc[e] += (a.dt / 3.0) * k;
                        a.unext[e] = T(un + a.dt * k);
                    } else {
                        a.unext[e] = T(a.acc[e] + (a.dt / 6.0) * k);
                    }
                }
            }
        }
#pragma unroll
        for (int v = 0; v < 5; ++v) Hp[v] = H[v];
    }
}

// ----------------------------------------------------------------------------
// diagnostics: deterministic two-pass reduction
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

template <typename T>
__global__ __launch_bounds__(kDiagThreads) void k_diag_partial(int nx, int ny, int nz, double gamma, double ihx,
                                                               double ihy, double ihz, const T *__restrict__ u,
                                                               double *__restrict__ part) {
    const size_t n3 = (size_t)nx * ny * nz;
    double acc[CNS_NDIAG] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    const size_t sy = nx, sz = (size_t)nx * ny;
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < n3; idx += (size_t)gridDim.x * blockDim.x) {
        double r = double(u[idx]), mx = double(u[n3 + idx]), my = double(u[2 * n3 + idx]), mz = double(u[3 * n3 + idx]),
               e = double(u[4 * n3 + idx]);
        double inv = 1.0 / r;
        double vx = mx * inv, vy = my * inv, vz = mz * inv;
        double ke = 0.5 * (mx * vx + my * vy + mz * vz);
        double p = (gamma - 1.0) * (e - ke);
        bool finite = isfinite(r) && isfinite(mx) && isfinite(my) && isfinite(mz) && isfinite(e);
        if (!finite || !(r > 0.0) || !(p > 0.0)) {
            acc[8] += 1.0;
            continue;
        }
        acc[0] += ke;
        acc[2] += r;
        acc[3] += mx;
        acc[4] += my;
        acc[5] += mz;
        acc[6] += e;
        double c = sqrt(gamma * p * inv);
        acc[7] = fmax(acc[7], fmax(fabs(vx), fmax(fabs(vy), fabs(vz))) + c);
        // vorticity with the 4th-order central derivative
        int i = (int)(idx % nx), j = (int)((idx / nx) % ny), k = (int)(idx / sz);
        size_t row = idx - i, col = idx - j * sy, pil = idx - k * sz;
        const int off[4] = {-2, -1, 1, 2};
        double vyx[4], vzx[4], vxy[4], vzy[4], vxz[4], vyz[4];
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            size_t px = row + wrapi(i + off[o], nx), py = col + wrapi(j + off[o], ny) * sy,
                   pz = pil + wrapi(k + off[o], nz) * sz;
            double rx = 1.0 / double(u[px]), ry = 1.0 / double(u[py]), rz = 1.0 / double(u[pz]);
            vyx[o] = double(u[2 * n3 + px]) * rx;
            vzx[o] = double(u[3 * n3 + px]) * rx;
            vxy[o] = double(u[n3 + py]) * ry;
            vzy[o] = double(u[3 * n3 + py]) * ry;
            vxz[o] = double(u[n3 + pz]) * rz;
            vyz[o] = double(u[2 * n3 + pz]) * rz;
        }
        double ox = dcen(vzy[0], vzy[1], vzy[2], vzy[3]) * ihy - dcen(vyz[0], vyz[1], vyz[2], vyz[3]) * ihz;
        double oy = dcen(vxz[0], vxz[1], vxz[2], vxz[3]) * ihz - dcen(vzx[0], vzx[1], vzx[2], vzx[3]) * ihx;
        double oz = dcen(vyx[0], vyx[1], vyx[2], vyx[3]) * ihx - dcen(vxy[0], vxy[1], vxy[2], vxy[3]) * ihy;
        if (isfinite(ox) && isfinite(oy) && isfinite(oz)) acc[1] += 0.5 * (ox * ox + oy * oy + oz * oz);
    }
    __shared__ double red[kDiagThreads / 64][CNS_NDIAG];
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
        part[(size_t)blockIdx.x * CNS_NDIAG + d] = v;
    }
}

__global__ __launch_bounds__(kDiagThreads) void k_diag_final(int nblk, double inv_n3, const double *__restrict__ part,
                                                            double *__restrict__ out) {
    double acc[CNS_NDIAG] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblk; b += blockDim.x)
#pragma unroll
        for (int d = 0; d < CNS_NDIAG; ++d)
            acc[d] = (d == 7) ? fmax(acc[d], part[(size_t)b * CNS_NDIAG + d]) : acc[d] + part[(size_t)b * CNS_NDIAG + d];
    __shared__ double red[kDiagThreads / 64][CNS_NDIAG];
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
        out[d] = (d == 7 || d == 8) ? v : v * inv_n3;
    }
}

// ----------------------------------------------------------------------------
// launchers
// ----------------------------------------------------------------------------
static inline unsigned blocks_for(size_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }

template <typename T>
void launch_init_state(const Box &b, const double *rho, const double *vel, const double *p, T *u, hipStream_t s) {
    size_t n3 = b.n3();
    hipLaunchKernelGGL(k_init_state<T>, dim3(blocks_for(n3, 256)), dim3(256), 0, s, n3, b.ph.gamma - 1.0, rho, vel, p,
                       u);
}

template <typename T>
static void launch_visc_fields(const Box &b, const T *u, T *W, T *G, hipStream_t s, Prof *pf = nullptr) {
    size_t n3 = b.n3();
    {
        ProfScope ps(pf, K_PRIM, s);
        hipLaunchKernelGGL(k_prim<T>, dim3(blocks_for(n3, 256)), dim3(256), 0, s, n3, T(b.ph.gamma), u, W);
    }
    T mu = T(b.ph.mu_eff);
    T kc = T(b.ph.mu_eff / ((b.ph.gamma - 1.0) * b.ph.prandtl));
    ProfScope ps(pf, K_VISC_FLUX, s);
    hipLaunchKernelGGL(k_visc_flux<T>, dim3(blocks_for(n3, 256)), dim3(256), 0, s, b.nx, b.ny, b.nz,
                       T(b.nx / b.lx), T(b.ny / b.ly), T(b.nz / b.lz), mu, kc, (const T *)W, G);
}

template <typename T>
static SweepArgs<T> sweep_args(const Box &b, const Tiles &t, int dir, const T *u, const T *G, T *rhs) {
    SweepArgs<T> a{};
    a.u = u;
    a.G = G;
    a.rhs = rhs;
    a.n3 = b.n3();
    const size_t sx = 1, sy = (size_t)b.nx, sz = (size_t)b.nx * b.ny;
    if (dir == 0) {
        a.nline = b.nx, a.lstride = sx, a.np = b.ny, a.pstride = sy, a.qstride = sz, a.npq = b.ny * b.nz;
        a.inv_dx = T(b.nx / b.lx);
    } else if (dir == 1) {
        a.nline = b.ny, a.lstride = sy, a.np = b.nx, a.pstride = sx, a.qstride = sz, a.npq = b.nx * b.nz;
        a.inv_dx = T(b.ny / b.ly);
    } else {
        a.nline = b.nz, a.lstride = sz, a.np = b.nx, a.pstride = sx, a.qstride = sy, a.npq = b.nx * b.ny;
        a.inv_dx = T(b.nz / b.lz);
    }
    a.seg = t.seg[dir] > 0 ? t.seg[dir] : a.nline;
    a.nseg = (a.nline + a.seg - 1) / a.seg;
    a.gamma = T(b.ph.gamma);
    a.eps = T(b.ph.eps);
    a.delta = T(b.ph.delta);
    return a;
}

template <typename T, int DIR, int MODE, bool VISC>
static void launch_sweep_t(const SweepArgs<T> &a, int block, hipStream_t s) {
    size_t total = (size_t)a.npq * a.nseg;
    hipLaunchKernelGGL((k_sweep<T, double, DIR, MODE, VISC>), dim3(blocks_for(total, block)), dim3(block), 0, s, a);
}

template <typename T, int MODE>
static void launch_sweep(const SweepArgs<T> &a, int dir, bool visc, int block, hipStream_t s, Prof *pf = nullptr) {
    ProfScope ps(pf, K_SWEEP_X + dir, s);
    if (visc) {
        if (dir == 0) launch_sweep_t<T, 0, MODE, true>(a, block, s);
        else if (dir == 1) launch_sweep_t<T, 1, MODE, true>(a, block, s);
        else launch_sweep_t<T, 2, MODE, true>(a, block, s);
    } else {
        if (dir == 0) launch_sweep_t<T, 0, MODE, false>(a, block, s);
        else if (dir == 1) launch_sweep_t<T, 1, MODE, false>(a, block, s);
        else launch_sweep_t<T, 2, MODE, false>(a, block, s);
    }
}

template <typename T>
void launch_rhs(const Box &b, const Tiles &t, const T *u, T *rhs, T *W, T *G, hipStream_t s) {
    const bool visc = b.ph.mu_eff > 0.0;
    if (visc) launch_visc_fields<T>(b, u, W, G, s);
    launch_sweep<T, MODE_WRITE>(sweep_args<T>(b, t, 0, u, G, rhs), 0, visc, t.block, s);
    launch_sweep<T, MODE_ACCUM>(sweep_args<T>(b, t, 1, u, G, rhs), 1, visc, t.block, s);
    launch_sweep<T, MODE_ACCUM>(sweep_args<T>(b, t, 2, u, G, rhs), 2, visc, t.block, s);
}

template <typename T>
void launch_rhs_dir(const Box &b, const Tiles &t, const T *u, int dir, T *out, hipStream_t s) {
    launch_sweep<T, MODE_WRITE>(sweep_args<T>(b, t, dir, u, (const T *)nullptr, out), dir, false, t.block, s);
}

template <typename T>
void launch_viscous(const Box &b, const T *u, T *out, T *W, T *G, hipStream_t s) {
    size_t n3 = b.n3();
    if (!(b.ph.mu_eff > 0.0)) {
        hipLaunchKernelGGL(k_fill<T>, dim3(blocks_for(5 * n3, 256)), dim3(256), 0, s, 5 * n3, T(0), out);
        return;
    }
    launch_visc_fields<T>(b, u, W, G, s);
    hipLaunchKernelGGL(k_visc_div<T>, dim3(blocks_for(n3, 256)), dim3(256), 0, s, b.nx, b.ny, b.nz, T(b.nx / b.lx),
                       T(b.ny / b.ly), T(b.nz / b.lz), (const T *)G, out);
}

template <typename T>
void launch_rk4_stage(const Box &b, const Tiles &t, int stage, const T *ustage, T *un, T *unext, double *acc,
                      double dt, T *rhs, T *W, T *G, hipStream_t s, Prof *pf) {
    const bool visc = b.ph.mu_eff > 0.0;
    if (visc) launch_visc_fields<T>(b, ustage, W, G, s, pf);
    launch_sweep<T, MODE_WRITE>(sweep_args<T>(b, t, 0, ustage, G, rhs), 0, visc, t.block, s, pf);
    launch_sweep<T, MODE_ACCUM>(sweep_args<T>(b, t, 1, ustage, G, rhs), 1, visc, t.block, s, pf);
    SweepArgs<T> a = sweep_args<T>(b, t, 2, ustage, G, rhs);
    a.un = un;
    a.acc = acc;
    a.unext = unext;
    a.dt = dt;
    a.stage = stage;
    launch_sweep<T, MODE_RK>(a, 2, visc, t.block, s, pf);
}

template <typename T>
void launch_diag(const Box &b, const T *u, double *part, double *out, hipStream_t s, Prof *pf) {
    ProfScope ps(pf, K_DIAG, s);
    size_t n3 = b.n3();
    int nblk = (int)std::min<size_t>(kDiagBlocks, blocks_for(n3, kDiagThreads));
    hipLaunchKernelGGL(k_diag_partial<T>, dim3(nblk), dim3(kDiagThreads), 0, s, b.nx, b.ny, b.nz, b.ph.gamma,
                       b.nx / b.lx, b.ny / b.ly, b.nz / b.lz, u, part);
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(kDiagThreads), 0, s, nblk, 1.0 / (double)n3, (const double *)part,
                       out);
}

void prof_flush(Prof *p) {
    if (!p || !p->on || p->n == 0) return;
    hipEventSynchronize(p->ev[2 * p->n - 1]);
    for (int i = 0; i < p->n; ++i) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p->ev[2 * i], p->ev[2 * i + 1]) == hipSuccess) {
            p->ms[p->kind[i]] += ms;
            p->count[p->kind[i]] += 1;
        }
    }
    p->n = 0;
}

// explicit instantiations
#define CNS_INSTANTIATE(T)                                                                                            \
    template void launch_init_state<T>(const Box &, const double *, const double *, const double *, T *, hipStream_t); \
    template void launch_rhs<T>(const Box &, const Tiles &, const T *, T *, T *, T *, hipStream_t);                   \
    template void launch_rhs_dir<T>(const Box &, const Tiles &, const T *, int, T *, hipStream_t);                    \
    template void launch_viscous<T>(const Box &, const T *, T *, T *, T *, hipStream_t);                              \
    template void launch_rk4_stage<T>(const Box &, const Tiles &, int, const T *, T *, T *, double *, double, T *, T *, \
                                      T *, hipStream_t, Prof *);                                                      \
    template void launch_diag<T>(const Box &, const T *, double *, double *, hipStream_t, Prof *);
CNS_INSTANTIATE(double)
CNS_INSTANTIATE(float)

}  // namespace cns
