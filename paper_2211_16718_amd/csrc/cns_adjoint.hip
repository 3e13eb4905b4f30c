// cns_adjoint.hip -- reverse-mode kernels of the RHS (vector-Jacobian products) and the
// small kernels of the checkpointed reverse RK4, FP64, single box.
//
// (dR/du)^T rbar of the semi-discrete operator R(u) = -sum_d (H_{j+1/2} - H_{j-1/2})/dx_d
// + sum_d D_d G^v_d is assembled as
//   convective part, per direction d:  Hbar_{j+1/2} = (rbar_{j+1} - rbar_j)/dx_d;
//     k_adj_conv<d>: one thread per interface forms the local product of the
//     interface flux (30 contributions to the six cells it reads) and adds them,
//     in a fixed order, into LDS accumulators of the cells, which are then written;
//   viscous part: the adjoint of a central difference is minus the same central
//     difference, so Gbar_d = -D_d rbar; k_adj_visc1 maps it through the viscous
//     fluxes to the adjoints of the velocity/temperature gradients and of the
//     point velocities; k_adj_visc2 applies -D once more and the primitive map.
// Every sum is formed in a fixed order (deterministic, no atomics).
#include <hip/hip_runtime.h>

#include "cns_adjoint.h"
#include "cns_device_adj.h"
#include "cns_internal.h"

namespace cns {

__device__ __forceinline__ int wrapj(int j, int n) { return j < 0 ? j + n : (j >= n ? j - n : j); }
// any number of periods (the halo of a 64-wide tile over a shorter line)
__device__ __forceinline__ int wrapn(int j, int n) {
    const int r = j % n;
    return r < 0 ? r + n : r;
}

struct AdjGeom {
    int nx, ny, nz;
    size_t n3;
    double ih[3];
    double gamma, prandtl, mu, eps, delta;
};

static AdjGeom adj_geom(const BoxDesc &b) {
    AdjGeom g;
    g.nx = b.nx;
    g.ny = b.ny;
    g.nz = b.nz;
    g.n3 = b.n3;
    for (int d = 0; d < 3; ++d) g.ih[d] = b.inv_h[d];
    g.gamma = b.gamma;
    g.prandtl = b.prandtl;
    g.mu = b.mu;
    g.eps = b.eps;
    g.delta = b.delta;
    return g;
}

// linear index of (i,j,k) displaced by off along d
__device__ __forceinline__ size_t shift_idx(const AdjGeom &g, int i, int j, int k, int d, int off) {
    if (d == 0) i = wrapj(i + off, g.nx);
    else if (d == 1) j = wrapj(j + off, g.ny);
    else k = wrapj(k + off, g.nz);
    return ((size_t)k * g.ny + j) * g.nx + i;
}

// ---------------------------------------------------------------------------
// Convective adjoint along DIR, fused with the gather: ubar(=|+=) sum over the six
// interfaces that read each cell of their contributions.
//
// A block of 256 threads owns TB whole periodic lines along DIR and marches along
// them in chunks of TA interfaces; each wave owns LW of the lines and all TA
// interfaces of a chunk on them (x: one row, 64 interfaces; y, z: 8 lines consecutive
// in x, 8 interfaces each).  Each thread forms the product of one interface (j+1/2,
// cells j-2 .. j+3) and adds its terms, as they are formed, to two LDS rings of cell
// accumulators: the adjoints of the cells' point fluxes (ringF) and those of their
// states through the dissipation (ringU).  Every cell of a wave's lines is touched by
// that wave alone, and a wave's LDS operations take effect in program order, so no
// barrier orders the additions; they are LDS atomic adds, and the six terms of one
// instruction (cells j-2+m of the interfaces j of the wave) go to six different
// cells, so the order of the additions into every cell is fixed (deterministic).  A
// complete cell leaves as J(u)^T ringF + ringU, J the Jacobian of the point flux: the
// transpose is applied once per cell instead of once per interface and cell.
//
// Cells are indexed along the line without wrapping, e = -2 .. n+2; e and e+n are
// the same grid cell.  After the chunk with interfaces I .. I+TA-1 the cells up to
// I+TA-3 are complete: cells 3 .. n-3 are written out, and the finished parts of
// cells -2 .. 2 are set aside ("head") until the last chunk adds the rest of those
// five grid cells (e = n-2 .. n+2); the transpose is linear, so the two parts are
// transposed separately.  The rings hold RS >= TA + 5 cells, the cells one chunk
// touches.  Before each chunk the block stages the states of the cells I-2 .. I+TA+2
// of its lines and their point fluxes along DIR in LDS (coalesced along x in every
// direction; each flux formed once instead of by each of the six interfaces that
// read it), so the stages of the interface product, which re-read the states rather
// than hold them, and the transposes at write-out read LDS instead of the caches.
// ---------------------------------------------------------------------------
template <int DIR> struct AdjConvShape;
template <> struct AdjConvShape<0> { static constexpr int TA = 64, LW = 1, RS = 128; };
template <> struct AdjConvShape<1> { static constexpr int TA = 8, LW = 8, RS = 16; };
template <> struct AdjConvShape<2> { static constexpr int TA = 8, LW = 8, RS = 16; };

template <int DIR, int WW>
__global__ __launch_bounds__(256, 2) void k_adj_conv(AdjGeom g, const double *__restrict__ u,
                                                     const double *__restrict__ rbar, double *__restrict__ ubar,
                                                     int accumulate) {
    using S = AdjConvShape<DIR>;
    constexpr int TA = S::TA, LW = S::LW, RS = S::RS, TB = 4 * LW;
    constexpr int NC = TA + 5;  // staged cells per line
    static_assert(TA * LW == 64 && RS >= TA + 5 && (RS & (RS - 1)) == 0, "chunk shape");
    // staged component v of line l, cell k (v = 0-4 the state, 5-9 its point flux along
    // DIR): x: (l * 10 + v) * NC + k; y, z: k * KS + v * TB + l, the cell stride padded
    // so that the eight cells a wave reads in one instruction fall in both halves of
    // the LDS banks.  Both rings, the head and the staged cells of a block fit twice
    // in the 160 KiB of LDS of a compute unit.
    constexpr int KS = 10 * TB + 8;
    constexpr int cs = DIR == 0 ? NC : TB;  // component stride of stg
    __shared__ double ringF[4 * 5 * RS * LW];
    __shared__ double ringU[4 * 5 * RS * LW];
    __shared__ double head[TB * 25];
    __shared__ double stg[DIR == 0 ? TB * 10 * NC : NC * KS];
    const int lane = (int)threadIdx.x & 63, w = (int)threadIdx.x >> 6;
    const int ta = DIR == 0 ? lane : lane >> 3;  // interface within the chunk
    const int tl = DIR == 0 ? 0 : lane & 7;      // line within the wave
    const int tb = w * LW + tl;                   // line within the block
    // ring slot of cell e for component v: the wave's own region, consecutive lanes
    // on consecutive doubles
    auto slot = [&](int e, int v) -> int { return ((w * 5 + v) * RS + ((e + 2) & (RS - 1))) * LW + tl; };
    // offset in stg of this lane's line at staged cell k
    auto cell = [&](int k) -> int { return DIR == 0 ? tb * 10 * NC + k : k * KS + tb; };
    const size_t n3 = g.n3;
    const int n = DIR == 0 ? g.nx : (DIR == 1 ? g.ny : g.nz);
    const size_t stride = DIR == 0 ? 1 : (DIR == 1 ? (size_t)g.nx : (size_t)g.nx * g.ny);
    const int ntx = (g.nx + TB - 1) / TB;
    const double gm1 = g.gamma - 1.0;
    // the line of lane column t: whether it exists, and the offset of its cell 0
    auto line = [&](int t, size_t &lb) -> bool {
        if (DIR == 0) {
            const size_t row = (size_t)blockIdx.x * TB + t;
            lb = row * g.nx;
            return row < (size_t)g.ny * g.nz;
        }
        const int x = (int)(blockIdx.x % ntx) * TB + t, o = (int)(blockIdx.x / ntx);
        lb = (DIR == 1 ? (size_t)o * g.nx * g.ny : (size_t)o * g.nx) + (size_t)x;
        return x < g.nx;
    };
    // the finished adjoint of cell e, staged at k: J^T ringF + ringU
    auto finish = [&](int e, int k, double out[5]) {
        double wc[5], fb[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            wc[v] = stg[v * cs + cell(k)];
            fb[v] = ringF[slot(e, v)];
            out[v] = ringU[slot(e, v)];
        }
        euler_flux_vjp<DIR>(wc, gm1, fb, out);
    };
    size_t base;
    const bool lane_ok = line(tb, base);
    const double ih = g.ih[DIR];
    for (int t = threadIdx.x; t < 4 * 5 * RS * LW; t += 256) {
        ringF[t] = 0.0;
        ringU[t] = 0.0;
    }
    int I = 0;
    for (;; I += TA) {
        // the previous chunk's write-out has read stg
        __syncthreads();
        // stage cells I-2 .. I+TA+2 (any number of periods: short lines wrap more than
        // once) and their point fluxes
        for (int t = threadIdx.x; t < TB * NC; t += 256) {
            const int k = DIR == 0 ? t % NC : t / TB, l = DIR == 0 ? t / NC : t % TB;
            const int at = DIR == 0 ? l * 10 * NC + k : k * KS + l;
            size_t lb;
            if (line(l, lb)) {
                int c = (I - 2 + k) % n;
                if (c < 0) c += n;
                double wc[5];
#pragma unroll
                for (int v = 0; v < 5; ++v) wc[v] = u[v * n3 + lb + (size_t)c * stride];
#pragma unroll
                for (int v = 0; v < 5; ++v) {
                    stg[at + v * cs] = wc[v];
                    stg[at + (5 + v) * cs] = euler_flux_comp<DIR>(wc, gm1, v);
                }
            }
        }
        __syncthreads();
        const int j = I + ta;
        if (lane_ok && j < n) {
            // cell j-2+m is staged cell ta+m
            int c[6];
#pragma unroll
            for (int m = 0; m < 6; ++m) c[m] = cell(ta + m);
            const size_t p = base + (size_t)j * stride, pn = base + (size_t)wrapj(j + 1, n) * stride;
            double Hb[5];
#pragma unroll
            for (int v = 0; v < 5; ++v) Hb[v] = (rbar[v * n3 + pn] - rbar[v * n3 + p]) * ih;
            interface_flux_vjp<DIR, WW>(
                stg, cs, c, Hb, g.gamma, g.eps, g.delta,
                [&](int m, int v, double x) { atomicAdd(&ringF[slot(j + m - 2, v)], x); },
                [&](int m, int v, double x) { atomicAdd(&ringU[slot(j + m - 2, v)], x); });
        }
        // every addition of this wave precedes the reads of the write-out
        adj_stage_fence();
        const bool last = I + TA >= n;
        const int e = I - 2 + ta;  // completed by this chunk (all of them unless last)
        if (lane_ok && e <= 2) {
            double out[5];
            finish(e, ta, out);
#pragma unroll
            for (int v = 0; v < 5; ++v) head[tb * 25 + (e + 2) * 5 + v] = out[v];
        } else if (lane_ok && !last && e <= n - 3) {
            double out[5];
            finish(e, ta, out);
            const size_t q = base + (size_t)e * stride;
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                if (accumulate) ubar[v * n3 + q] += out[v];
                else ubar[v * n3 + q] = out[v];
            }
        }
        if (last) break;
        adj_stage_fence();
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            ringF[slot(e, v)] = 0.0;
            ringU[slot(e, v)] = 0.0;
        }
        adj_stage_fence();
    }
    // the rest of the line: cells max(I-2, 3) .. n+2 (staged at e - (I-2)), folding
    // e >= n-2 with the head; the wave reads only what it wrote itself
    adj_stage_fence();
    for (int e = I - 2 + ta; e <= n + 2; e += TA) {
        if (!lane_ok || e < 3) continue;
        const int r = e >= n ? e - n : e;
        const size_t q = base + (size_t)r * stride;
        double out[5];
        finish(e, e - (I - 2), out);
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            double s = out[v];
            if (e >= n - 2) s += head[tb * 25 + (e - n + 2) * 5 + v];
            if (accumulate) ubar[v * n3 + q] += s;
            else ubar[v * n3 + q] = s;
        }
    }
}

// ---------------------------------------------------------------------------
// Viscous adjoint on the tiles of the forward viscous-flux kernel: a block owns a
// 32 x 8 (x, y) tile and marches along z over kViscSZ planes; the x and y stencil
// operands of the current plane sit in LDS (with a +-2 halo), each thread keeps its
// own column's z operands at planes k-2 .. k+2 in registers.
//
// Part 1: Gbar_d = -D_d rbar (momentum and energy rows), through tau, q and E to the
// adjoints of the 12 gradients g[a][b] = d W_a / dx_b (W = u, v, w, T) and of the
// point velocities.  tau is symmetric, so the 12 gradient adjoints hold 9 distinct
// values; Gb stores gxx, gyy, gzz, gxy, gxz, gyz, kappa E_x, kappa E_y, kappa E_z,
// then the three point-velocity adjoints: kAdjGbFields fields.
// ---------------------------------------------------------------------------

// W = (u, v, w, T = gamma p / rho) of the state at linear index i: the forward's
// primitive map, the linearisation point of the viscous terms
__device__ __forceinline__ void adj_prim_at(const double *__restrict__ u, size_t n3, size_t i, double gamma,
                                            double W[4]) {
    const double r = u[i], mx = u[n3 + i], my = u[2 * n3 + i], mz = u[3 * n3 + i], e = u[4 * n3 + i];
    const double inv = rcp(r);
    W[0] = mx * inv;
    W[1] = my * inv;
    W[2] = mz * inv;
    const double p = (gamma - 1.0) * (e - 0.5 * (mx * W[0] + my * W[1] + mz * W[2]));
    W[3] = gamma * p * inv;
}

struct AdjTile {
    int x0, y0, z0, z1, tx, ty;
    bool act;
    size_t col;
};
__device__ __forceinline__ AdjTile adj_tile(const AdjGeom &g) {
    AdjTile t;
    const int ntx = (g.nx + kViscTX - 1) / kViscTX, nty = (g.ny + kViscTY - 1) / kViscTY;
    const long long lb = blockIdx.x;
    t.x0 = (int)(lb % ntx) * kViscTX;
    t.y0 = (int)((lb / ntx) % nty) * kViscTY;
    t.z0 = (int)(lb / ((long long)ntx * nty)) * kViscSZ;
    t.z1 = min(t.z0 + kViscSZ, g.nz);
    t.tx = threadIdx.x % kViscTX;
    t.ty = threadIdx.x / kViscTX;
    t.act = t.x0 + t.tx < g.nx && t.y0 + t.ty < g.ny;
    t.col = (size_t)min(t.y0 + t.ty, g.ny - 1) * g.nx + min(t.x0 + t.tx, g.nx - 1);
    return t;
}

__global__ __launch_bounds__(kPointThreads) void k_adj_visc1(AdjGeom g, const double *__restrict__ u,
                                                             const double *__restrict__ rbar, double *__restrict__ Gb) {
    constexpr int TX = kViscTX, TY = kViscTY;
    __shared__ double pw[4][TY + 4][TX + 4];  // W of the plane
    __shared__ double pr[4][TY + 4][TX + 4];  // rbar rows 1..4 of the plane
    const AdjTile t = adj_tile(g);
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const size_t n3 = g.n3, sz = (size_t)nx * ny;
    const double *rb = rbar + n3;  // rows 1..4: momentum x, y, z, energy
    double Wz[5][4], Rz[5][4];     // this column at planes k-2 .. k+2
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const size_t q = t.col + (size_t)wrapj(t.z0 - 2 + m, nz) * sz;
        adj_prim_at(u, n3, q, g.gamma, Wz[m]);
#pragma unroll
        for (int c = 0; c < 4; ++c) Rz[m][c] = rb[c * n3 + q];
    }
    const double mu = g.mu, kc = g.mu / ((g.gamma - 1.0) * g.prandtl);
    for (int k = t.z0; k < t.z1; ++k) {
        {
            const size_t q = t.col + (size_t)wrapj(k + 2, nz) * sz;
            adj_prim_at(u, n3, q, g.gamma, Wz[4]);
#pragma unroll
            for (int c = 0; c < 4; ++c) Rz[4][c] = rb[c * n3 + q];
        }
        for (int h = threadIdx.x; h < (TX + 4) * (TY + 4); h += blockDim.x) {
            const int hx = h % (TX + 4), hy = h / (TX + 4);
            const size_t q = (size_t)k * sz + (size_t)wrapn(t.y0 - 2 + hy, ny) * nx + wrapn(t.x0 - 2 + hx, nx);
            double w4[4];
            adj_prim_at(u, n3, q, g.gamma, w4);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                pw[c][hy][hx] = w4[c];
                pr[c][hy][hx] = rb[c * n3 + q];
            }
        }
        __syncthreads();
        if (t.act) {
            const int X = t.tx + 2, Y = t.ty + 2;
            // forward at the point: gradients and stresses
            double gr[4][3];
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                gr[a][0] = dcen(pw[a][Y][X - 2], pw[a][Y][X - 1], pw[a][Y][X + 1], pw[a][Y][X + 2]) * g.ih[0];
                gr[a][1] = dcen(pw[a][Y - 2][X], pw[a][Y - 1][X], pw[a][Y + 1][X], pw[a][Y + 2][X]) * g.ih[1];
                gr[a][2] = dcen(Wz[0][a], Wz[1][a], Wz[3][a], Wz[4][a]) * g.ih[2];
            }
            const double div = gr[0][0] + gr[1][1] + gr[2][2];
            const double tdiv = 2.0 / 3.0 * div;
            const double txx = mu * (2.0 * gr[0][0] - tdiv), tyy = mu * (2.0 * gr[1][1] - tdiv),
                         tzz = mu * (2.0 * gr[2][2] - tdiv);
            const double txy = mu * (gr[0][1] + gr[1][0]), txz = mu * (gr[0][2] + gr[2][0]),
                         tyz = mu * (gr[1][2] + gr[2][1]);
            const double vx = Wz[2][0], vy = Wz[2][1], vz = Wz[2][2];
            // Gbar_d[c] = -(D_d rbar_{1+c}), c: x-, y-, z-momentum, energy
            double Gbar[3][4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                Gbar[0][c] = -dcen(pr[c][Y][X - 2], pr[c][Y][X - 1], pr[c][Y][X + 1], pr[c][Y][X + 2]) * g.ih[0];
                Gbar[1][c] = -dcen(pr[c][Y - 2][X], pr[c][Y - 1][X], pr[c][Y + 1][X], pr[c][Y + 2][X]) * g.ih[1];
                Gbar[2][c] = -dcen(Rz[0][c], Rz[1][c], Rz[3][c], Rz[4][c]) * g.ih[2];
            }
            // G_x = [txx, txy, txz, Ex], G_y = [txy, tyy, tyz, Ey], G_z = [txz, tyz, tzz, Ez],
            // E_x = vx txx + vy txy + vz txz + kc dT/dx, etc.
            const double Ex = Gbar[0][3], Ey = Gbar[1][3], Ez = Gbar[2][3];
            const double bxx = Gbar[0][0] + Ex * vx;
            const double byy = Gbar[1][1] + Ey * vy;
            const double bzz = Gbar[2][2] + Ez * vz;
            const double bxy = Gbar[0][1] + Gbar[1][0] + Ex * vy + Ey * vx;
            const double bxz = Gbar[0][2] + Gbar[2][0] + Ex * vz + Ez * vx;
            const double byz = Gbar[1][2] + Gbar[2][1] + Ey * vz + Ez * vy;
            // tau_aa = mu (2 g_aa - 2/3 div), tau_ab = mu (g_ab + g_ba)
            const double divb = -2.0 / 3.0 * mu * (bxx + byy + bzz);
            const size_t idx = (size_t)k * sz + t.col;
            // non-temporal stores: the fields are streamed to memory for the second
            // kernel, so they do not displace the state's halo lines in L2
            __builtin_nontemporal_store(2.0 * mu * bxx + divb, &Gb[idx]);
            __builtin_nontemporal_store(2.0 * mu * byy + divb, &Gb[n3 + idx]);
            __builtin_nontemporal_store(2.0 * mu * bzz + divb, &Gb[2 * n3 + idx]);
            __builtin_nontemporal_store(mu * bxy, &Gb[3 * n3 + idx]);
            __builtin_nontemporal_store(mu * bxz, &Gb[4 * n3 + idx]);
            __builtin_nontemporal_store(mu * byz, &Gb[5 * n3 + idx]);
            __builtin_nontemporal_store(kc * Ex, &Gb[6 * n3 + idx]);
            __builtin_nontemporal_store(kc * Ey, &Gb[7 * n3 + idx]);
            __builtin_nontemporal_store(kc * Ez, &Gb[8 * n3 + idx]);
            __builtin_nontemporal_store(Ex * txx + Ey * txy + Ez * txz, &Gb[9 * n3 + idx]);
            __builtin_nontemporal_store(Ex * txy + Ey * tyy + Ez * tyz, &Gb[10 * n3 + idx]);
            __builtin_nontemporal_store(Ex * txz + Ey * tyz + Ez * tzz, &Gb[11 * n3 + idx]);
        }
        __syncthreads();  // the next plane overwrites the LDS tile
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                Wz[m][c] = Wz[m + 1][c];
                Rz[m][c] = Rz[m + 1][c];
            }
    }
}

// Part 2: Wbar_a = (point adjoint) - sum_b D_b gbar[a][b], then through
// W(u) = (m/rho, gamma p / rho) to ubar (accumulated).  The x derivatives act on
// (gxx, gxy, gxz, kappa E_x), the y derivatives on (gxy, gyy, gyz, kappa E_y), the z
// derivatives on (gxz, gyz, gzz, kappa E_z).
__global__ __launch_bounds__(kPointThreads) void k_adj_visc2(AdjGeom g, const double *__restrict__ u,
                                                             const double *__restrict__ Gb, double *__restrict__ ubar,
                                                             AdjEpilogue ep) {
    constexpr int TX = kViscTX, TY = kViscTY;
    constexpr int fx[4] = {0, 3, 4, 6}, fy[4] = {3, 1, 5, 7}, fz[4] = {4, 5, 2, 8};
    __shared__ double qx[4][TY][TX + 4];  // x-differenced fields of the plane, x halo
    __shared__ double qy[4][TY + 4][TX];  // y-differenced fields of the plane, y halo
    const AdjTile t = adj_tile(g);
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const size_t n3 = g.n3, sz = (size_t)nx * ny;
    double Gz[5][4];  // z-differenced fields of this column at planes k-2 .. k+2
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const size_t q = t.col + (size_t)wrapj(t.z0 - 2 + m, nz) * sz;
#pragma unroll
        for (int a = 0; a < 4; ++a) Gz[m][a] = Gb[fz[a] * n3 + q];
    }
    const double gm1 = g.gamma - 1.0;
    for (int k = t.z0; k < t.z1; ++k) {
        {
            const size_t q = t.col + (size_t)wrapj(k + 2, nz) * sz;
#pragma unroll
            for (int a = 0; a < 4; ++a) Gz[4][a] = Gb[fz[a] * n3 + q];
        }
        const size_t plane = (size_t)k * sz;
        // the point's own operands, loaded ahead of the plane staging and its barrier
        const size_t p = plane + t.col;
        double pa[3], us[5], ub[5];
#pragma unroll
        for (int a = 0; a < 3; ++a) pa[a] = Gb[(9 + a) * n3 + p];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            us[v] = u[v * n3 + p];
            ub[v] = ubar[v * n3 + p];
        }
        for (int h = threadIdx.x; h < (TX + 4) * TY; h += blockDim.x) {
            const int hx = h % (TX + 4), hy = h / (TX + 4);
            const size_t q = plane + (size_t)min(t.y0 + hy, ny - 1) * nx + wrapn(t.x0 - 2 + hx, nx);
#pragma unroll
            for (int a = 0; a < 4; ++a) qx[a][hy][hx] = Gb[fx[a] * n3 + q];
        }
        for (int h = threadIdx.x; h < TX * (TY + 4); h += blockDim.x) {
            const int hx = h % TX, hy = h / TX;
            const size_t q = plane + (size_t)wrapn(t.y0 - 2 + hy, ny) * nx + min(t.x0 + hx, nx - 1);
#pragma unroll
            for (int a = 0; a < 4; ++a) qy[a][hy][hx] = Gb[fy[a] * n3 + q];
        }
        __syncthreads();
        if (t.act) {
            const int X = t.tx + 2, Y = t.ty + 2;
            double Wb[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                double s = a < 3 ? pa[a] : 0.0;
                s -= dcen(qx[a][t.ty][X - 2], qx[a][t.ty][X - 1], qx[a][t.ty][X + 1], qx[a][t.ty][X + 2]) * g.ih[0];
                s -= dcen(qy[a][Y - 2][t.tx], qy[a][Y - 1][t.tx], qy[a][Y + 1][t.tx], qy[a][Y + 2][t.tx]) * g.ih[1];
                s -= dcen(Gz[0][a], Gz[1][a], Gz[3][a], Gz[4][a]) * g.ih[2];
                Wb[a] = s;
            }
            // W = (m_k / rho, gamma p / rho), p = (gamma-1)(e - m.v/2)
            const double r = us[0], m[3] = {us[1], us[2], us[3]}, e = us[4];
            const double inv = rcp(r);
            const double v[3] = {m[0] * inv, m[1] * inv, m[2] * inv};
            const double qq = m[0] * v[0] + m[1] * v[1] + m[2] * v[2];
            const double pr = gm1 * (e - 0.5 * qq);
            // T = gamma pr inv
            const double prb = g.gamma * inv * Wb[3];
            double invb = g.gamma * pr * Wb[3];
            const double eb = gm1 * prb;
            const double qqb = -0.5 * gm1 * prb;
            double mb[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double vb = Wb[c] + qqb * m[c];
                mb[c] = qqb * v[c] + vb * inv;
                invb += vb * m[c];
            }
            const double fin[5] = {ub[0] + -invb * inv * inv, ub[1] + mb[0], ub[2] + mb[1], ub[3] + mb[2],
                                   ub[4] + eb};
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                const size_t o = v * n3 + p;
                if (ep.store_ub) ubar[o] = fin[v];
                if (ep.ubf) {
                    const double t = ep.S[o] + fin[v];
                    ep.ubf[o] = ep.ubf[o] + t;
                } else if (ep.S) {
                    ep.S[o] = ep.s_first ? fin[v] : ep.S[o] + fin[v];
                }
                if (ep.kb) ep.kb[o] = __fma_rn(ep.a, ep.ub[o], ep.b * fin[v]);
            }
        }
        __syncthreads();  // the next plane overwrites the LDS tiles
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int a = 0; a < 4; ++a) Gz[m][a] = Gz[m + 1][a];
    }
}

// out = a x + b y (y may be null)
__global__ void k_lincomb(size_t n, double a, const double *__restrict__ x, double b, const double *__restrict__ y,
                          double *__restrict__ out) {
    const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = y ? a * x[i] + b * y[i] : a * x[i];
}

// out += x
__global__ void k_accum(size_t n, const double *__restrict__ x, double *__restrict__ out) {
    const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (i < n) out[i] += x[i];
}

__global__ void k_copy(size_t n, const double *__restrict__ x, double *__restrict__ out) {
    const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (i < n) out[i] = x[i];
}

// ubar = dK/du with K = <|m|^2 / (2 rho)>
__global__ void k_ke_seed(size_t n3, const double *__restrict__ u, double *__restrict__ ubar) {
    const size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (p >= n3) return;
    const double s = 1.0 / (double)n3;
    const double r = u[p], mx = u[n3 + p], my = u[2 * n3 + p], mz = u[3 * n3 + p];
    const double inv = 1.0 / r;
    ubar[p] = -0.5 * (mx * mx + my * my + mz * mz) * inv * inv * s;
    ubar[n3 + p] = mx * inv * s;
    ubar[2 * n3 + p] = my * inv * s;
    ubar[3 * n3 + p] = mz * inv * s;
    ubar[4 * n3 + p] = 0.0;
}

// vbar_i = rho (mbar_i + ebar v_i): the initial-state map u(rho, v, p) transposed at fixed rho, p
__global__ void k_ic_vjp(size_t n3, const double *__restrict__ rho, const double *__restrict__ vel,
                         const double *__restrict__ ubar, double *__restrict__ vbar) {
    const size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (p >= n3) return;
    const double r = rho[p], eb = ubar[4 * n3 + p];
#pragma unroll
    for (int c = 0; c < 3; ++c) vbar[c * n3 + p] = r * (ubar[(1 + c) * n3 + p] + eb * vel[c * n3 + p]);
}

// ----------------------------------------------------------------------------
// launchers
// ----------------------------------------------------------------------------
static inline dim3 grid1(size_t n) { return dim3((unsigned)((n + 255) / 256)); }

template <int WW>
static void adj_conv(const BoxDesc &b, hipStream_t s, const AdjGeom &g, const double *u, const double *rbar,
                     double *ubar) {
    // blocks: x, TB = 4 rows each; y, z: one 32-wide x tile of the lines at one z (y) each
    const unsigned bx = (unsigned)(((size_t)b.ny * b.nz + 3) / 4);
    const unsigned ntx = (unsigned)((b.nx + 31) / 32);
    hipLaunchKernelGGL((k_adj_conv<0, WW>), dim3(bx), dim3(256), 0, s, g, u, rbar, ubar, 0);
    hipLaunchKernelGGL((k_adj_conv<1, WW>), dim3(ntx * (unsigned)b.nz), dim3(256), 0, s, g, u, rbar, ubar, 1);
    hipLaunchKernelGGL((k_adj_conv<2, WW>), dim3(ntx * (unsigned)b.ny), dim3(256), 0, s, g, u, rbar, ubar, 1);
}

// the stage-combination epilogue by separate launches (boxes without viscous terms)
__global__ void k_epilogue(size_t n, const double *__restrict__ fin, AdjEpilogue e) {
    const size_t o = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (o >= n) return;
    const double f = fin[o];
    if (e.ubf) {
        const double t = e.S[o] + f;
        e.ubf[o] = e.ubf[o] + t;
    } else if (e.S) {
        e.S[o] = e.s_first ? f : e.S[o] + f;
    }
    if (e.kb) e.kb[o] = __fma_rn(e.a, e.ub[o], e.b * f);
}

static void rhs_vjp(const BoxDesc &b, int weights, hipStream_t s, const double *u, const double *rbar, double *ubar,
                    double *Gb, const AdjEpilogue *epi) {
    const AdjGeom g = adj_geom(b);
    const bool visc = b.mu > 0.0;
    const unsigned tiles = (unsigned)(((b.nx + kViscTX - 1) / kViscTX) * (long long)((b.ny + kViscTY - 1) / kViscTY) *
                                      ((b.nz + kViscSZ - 1) / kViscSZ));
    if (visc) hipLaunchKernelGGL(k_adj_visc1, dim3(tiles), dim3(kPointThreads), 0, s, g, u, rbar, Gb);
    if (weights == CNS_WENO_Z) adj_conv<CNS_WENO_Z>(b, s, g, u, rbar, ubar);
    else if (weights == CNS_WENO_M) adj_conv<CNS_WENO_M>(b, s, g, u, rbar, ubar);
    else adj_conv<CNS_WENO_JS>(b, s, g, u, rbar, ubar);
    AdjEpilogue e;
    if (epi) e = *epi;
    if (visc) {
        hipLaunchKernelGGL(k_adj_visc2, dim3(tiles), dim3(kPointThreads), 0, s, g, u, (const double *)Gb, ubar, e);
    } else if (epi) {
        // ubar holds the finished product; the epilogue reads it from there
        const size_t n5 = 5 * b.n3;
        hipLaunchKernelGGL(k_epilogue, dim3((unsigned)((n5 + 255) / 256)), dim3(256), 0, s, n5, (const double *)ubar, e);
    }
}

void adj_rhs_vjp(const BoxDesc &b, int weights, hipStream_t s, const double *u, const double *rbar, double *ubar,
                 double *Gb) {
    rhs_vjp(b, weights, s, u, rbar, ubar, Gb, nullptr);
}

void adj_rhs_vjp_epi(const BoxDesc &b, int weights, hipStream_t s, const double *u, const double *rbar, double *ubar,
                     double *Gb, const AdjEpilogue &epi) {
    rhs_vjp(b, weights, s, u, rbar, ubar, Gb, &epi);
}

void adj_lincomb(size_t n, double a, const double *x, double b, const double *y, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_lincomb, grid1(n), dim3(256), 0, s, n, a, x, b, y, out);
}
void adj_accum(size_t n, const double *x, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_accum, grid1(n), dim3(256), 0, s, n, x, out);
}
void adj_copy(size_t n, const double *x, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_copy, grid1(n), dim3(256), 0, s, n, x, out);
}
void adj_ke_seed(size_t n3, const double *u, double *ubar, hipStream_t s) {
    hipLaunchKernelGGL(k_ke_seed, grid1(n3), dim3(256), 0, s, n3, u, ubar);
}
void adj_ic_vjp(size_t n3, const double *rho, const double *vel, const double *ubar, double *vbar, hipStream_t s) {
    hipLaunchKernelGGL(k_ic_vjp, grid1(n3), dim3(256), 0, s, n3, rho, vel, ubar, vbar);
}

}  // namespace cns
