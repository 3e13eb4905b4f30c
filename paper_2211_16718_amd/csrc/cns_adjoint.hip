// cns_adjoint.hip -- reverse-mode kernels of the RHS (vector-Jacobian products) and the
// small kernels of the checkpointed reverse RK4, FP64, single box.
//
// (dR/du)^T rbar of the semi-discrete operator R(u) = -sum_d (H_{j+1/2} - H_{j-1/2})/dx_d
// + sum_d D_d G^v_d is assembled as
//   convective part, per direction d:  Hbar_{j+1/2} = (rbar_{j+1} - rbar_j)/dx_d;
//     k_adj_conv<d>: one thread per interface forms the local product of the
//     interface flux (the point-flux and state adjoints of the six cells it reads)
//     and adds them, in a fixed order, into LDS accumulators of the cells, which are
//     then finished and written;
//   viscous part: the adjoint of a central difference is minus the same central
//     difference, so Gbar_d = -D_d rbar; k_adj_visc maps it through the viscous
//     fluxes to the adjoints of the velocity/temperature gradients and of the
//     point velocities, applies -D once more and the primitive map, in one pass.
// Every sum is formed in a fixed order (deterministic: the LDS atomic adds into a cell
// come from one wave, whose LDS operations take effect in program order).
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
// interfaces of a chunk on them (x: one row, 64 interfaces; y, z: 4 lines consecutive
// in x, 16 interfaces each).  Each thread forms the product of one interface (j+1/2,
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
template <> struct AdjConvShape<0> { static constexpr int TA = 64, LW = 1, RS = 128, PAD = 0; };
template <> struct AdjConvShape<1> { static constexpr int TA = 16, LW = 4, RS = 32, PAD = 4; };
template <> struct AdjConvShape<2> { static constexpr int TA = 16, LW = 4, RS = 32, PAD = 4; };

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
    // so that the sixteen cells a wave reads in one instruction spread over all LDS
    // banks.  Both rings, the head and the staged cells of a block fit twice in the
    // 160 KiB of LDS of a compute unit.
    constexpr int KS = 10 * TB + S::PAD;
    constexpr int cs = DIR == 0 ? NC : TB;  // component stride of stg
    __shared__ double ringF[4 * 5 * RS * LW];
    __shared__ double ringU[4 * 5 * RS * LW];
    __shared__ double head[TB * 25];
    __shared__ double stg[DIR == 0 ? TB * 10 * NC : NC * KS];
    const int lane = (int)threadIdx.x & 63, w = (int)threadIdx.x >> 6;
    const int ta = lane / LW;  // interface within the chunk
    const int tl = lane % LW;  // line within the wave
    const int tb = w * LW + tl;  // line within the block
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
// Viscous adjoint in one pass.  With Gbar_d = -D_d rbar (rows 1-4: momentum x, y, z and
// energy) the viscous fluxes give at every point
//   the stencil fields f_d, the adjoints that the transposed gradients D_d carry back:
//     f_x = (gxx, gxy, gxz, kappa E_x), f_y = (gxy, gyy, gyz, kappa E_y),
//     f_z = (gxz, gyz, gzz, kappa E_z), linear in Gbar with the point velocity as
//     coefficient (tau is symmetric: nine distinct values);
//   the point fields pa, the adjoints of the point velocities in the energy fluxes;
// and Wbar = pa - sum_d D_d f_d for W = (u, v, w, T), which the primitive map takes to
// ubar.  A block owns a 32 x 8 (x, y) tile and marches along z.  Per plane it forms f_x
// on the tile and its +-2 x halo and f_y on the tile and its +-2 y halo, from rbar
// staged in LDS with the +-4 halo these need and from the z derivatives of rbar at
// those points (register rings of five planes for the tile's columns, an LDS ring for
// the halo points), and f_z on the tile, whose z difference is applied two planes
// later from a register ring: the fields never go through memory.
// ---------------------------------------------------------------------------
constexpr int kAvTX = kViscTX, kAvTY = kViscTY;
constexpr int kAvRX = kAvTX + 8, kAvRY = kAvTY + 8;    // rbar box, origin (x0-4, y0-4)
constexpr int kAvHalo = 4 * kAvTY + 4 * kAvTX;         // x-halo then y-halo points of the tile
constexpr int kAvExt = 16 + 4 * kAvTY + 4 * kAvTX;     // further rbar points: corners, x and y extensions
static_assert(kAvHalo <= kPointThreads && kAvExt <= kPointThreads && kAvTX * kAvTY == kPointThreads, "tile");

// planes per block: the two planes of lookahead on either side are formed again by the
// next block along z, so long columns take more planes
__host__ __device__ __forceinline__ int adj_visc_planes(int nz) { return nz >= 256 ? 32 : 16; }

// position in the rbar box of halo point h (x-halo: columns x0-2, x0-1, x0+TX, x0+TX+1
// of the tile's rows; y-halo: rows y0-2, y0-1, y0+TY, y0+TY+1 of the tile's columns)
__device__ __forceinline__ void av_halo_pos(int h, int &bx, int &by) {
    if (h < 4 * kAvTY) {
        const int c = h & 3;
        bx = c < 2 ? 2 + c : kAvTX + 2 + c;
        by = 4 + (h >> 2);
    } else {
        const int q = h - 4 * kAvTY, r = q / kAvTX;
        bx = 4 + q % kAvTX;
        by = r < 2 ? 2 + r : kAvTY + 2 + r;
    }
}
// position in the rbar box of further point e: the 2 x 2 corners between the halos,
// then columns x0-4, x0-3, x0+TX+2, x0+TX+3 of the tile's rows, then rows y0-4, y0-3,
// y0+TY+2, y0+TY+3 of its columns
__device__ __forceinline__ void av_ext_pos(int e, int &bx, int &by) {
    if (e < 16) {
        const int cc = e >> 2;
        bx = (cc & 1 ? kAvTX + 4 : 2) + (e & 1);
        by = (cc & 2 ? kAvTY + 4 : 2) + ((e >> 1) & 1);
    } else if (e < 16 + 4 * kAvTY) {
        const int q = e - 16, c = q & 3;
        bx = c < 2 ? c : kAvTX + 4 + c;
        by = 4 + (q >> 2);
    } else {
        const int q = e - 16 - 4 * kAvTY, r = q / kAvTX;
        bx = 4 + q % kAvTX;
        by = r < 2 ? r : kAvTY + 4 + r;
    }
}

// the fields of a point from its rbar gradient (Gbar[d][c] = -D_d rbar_c) and velocity
struct AvFields {
    double gxx, gyy, gzz, gxy, gxz, gyz, ex, ey, ez;
};
__device__ __forceinline__ AvFields av_fields(const double Gbar[3][4], const double v[3], double mu, double kc) {
    const double Ex = Gbar[0][3], Ey = Gbar[1][3], Ez = Gbar[2][3];
    const double bxx = Gbar[0][0] + Ex * v[0];
    const double byy = Gbar[1][1] + Ey * v[1];
    const double bzz = Gbar[2][2] + Ez * v[2];
    const double bxy = Gbar[0][1] + Gbar[1][0] + Ex * v[1] + Ey * v[0];
    const double bxz = Gbar[0][2] + Gbar[2][0] + Ex * v[2] + Ez * v[0];
    const double byz = Gbar[1][2] + Gbar[2][1] + Ey * v[2] + Ez * v[1];
    // tau_aa = mu (2 g_aa - 2/3 div), tau_ab = mu (g_ab + g_ba)
    const double divb = -2.0 / 3.0 * mu * (bxx + byy + bzz);
    AvFields f;
    f.gxx = 2.0 * mu * bxx + divb;
    f.gyy = 2.0 * mu * byy + divb;
    f.gzz = 2.0 * mu * bzz + divb;
    f.gxy = mu * bxy;
    f.gxz = mu * bxz;
    f.gyz = mu * byz;
    f.ex = kc * Ex;
    f.ey = kc * Ey;
    f.ez = kc * Ez;
    return f;
}

__global__ __launch_bounds__(kPointThreads, 2) void k_adj_visc(AdjGeom g, const double *__restrict__ u,
                                                               const double *__restrict__ rbar,
                                                               double *__restrict__ ubar, AdjEpilogue ep) {
    constexpr int TX = kAvTX, TY = kAvTY, RX = kAvRX, RY = kAvRY;
    __shared__ double sR[4][RY][RX];             // rbar rows 1-4 of the plane
    __shared__ double sV[3][TY + 4][TX + 4];     // velocity of the plane, tile and +-2 halo
    __shared__ double sFx[4][TY][TX + 4];        // f_x, tile rows, x halo
    __shared__ double sFy[4][TY + 4][TX];        // f_y, tile columns, y halo
    __shared__ double hR[5][4][kAvHalo];         // rbar of the halo points, slot (plane - z0 + 4) mod 5
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const size_t n3 = g.n3, sz = (size_t)nx * ny;
    const int ntx = (nx + TX - 1) / TX, nty = (ny + TY - 1) / TY, zp = adj_visc_planes(nz);
    const long long lb = blockIdx.x;
    const int x0 = (int)(lb % ntx) * TX, y0 = (int)((lb / ntx) % nty) * TY;
    const int z0 = (int)(lb / ((long long)ntx * nty)) * zp, z1 = min(z0 + zp, nz);
    const int t = threadIdx.x, tx = t % TX, ty = t / TX;
    const bool act = x0 + tx < nx && y0 + ty < ny;
    // a column past a ragged edge wraps periodically: its values are halo values of the
    // active columns beside it
    const size_t col = (size_t)wrapn(y0 + ty, ny) * nx + wrapn(x0 + tx, nx);
    const bool own_h = t < kAvHalo, own_e = t < kAvExt;
    int hbx = 0, hby = 0, ebx = 0, eby = 0;
    if (own_h) av_halo_pos(t, hbx, hby);
    if (own_e) av_ext_pos(t, ebx, eby);
    const size_t hcol = (size_t)wrapn(y0 - 4 + hby, ny) * nx + wrapn(x0 - 4 + hbx, nx);
    const size_t ecol = (size_t)wrapn(y0 - 4 + eby, ny) * nx + wrapn(x0 - 4 + ebx, nx);
    const double *rb = rbar + n3;  // rows 1..4
    const double mu = g.mu, kc = g.mu / ((g.gamma - 1.0) * g.prandtl), gm1 = g.gamma - 1.0;
    const double ihx = g.ih[0], ihy = g.ih[1], ihz = g.ih[2];
    auto slot = [&](int p) { return (p - z0 + 4) % 5; };
    auto vel_at = [&](size_t i, double v[3]) {
        const double inv = rcp(u[i]);
        v[0] = u[n3 + i] * inv;
        v[1] = u[2 * n3 + i] * inv;
        v[2] = u[3 * n3 + i] * inv;
    };
    double Rz[5][4];  // rbar of this column at planes k-2 .. k+2
    double Vz[5][3];  // velocity of this column at planes k-2 .. k+2
    // Wbar of this column at planes k-2 .. k+2 as it accumulates: pa - D_x f_x - D_y f_y
    // when its plane is formed, and the terms of -D_z f_z as the f_z of the planes two
    // on either side are formed (the plane k-2 is complete after plane k)
    double Tq[5][4];
    const int k0 = z0 - 2;
    auto is_full = [&](int k) { return k >= z0 && k < z1; };
#pragma unroll
    for (int m = 0; m < 5; ++m) {
        const size_t q = col + (size_t)wrapn(k0 - 2 + m, nz) * sz;
#pragma unroll
        for (int c = 0; c < 4; ++c) Rz[m][c] = rb[c * n3 + q];
        vel_at(q, Vz[m]);
        if (own_h) {
            const size_t qh = hcol + (size_t)wrapn(k0 - 2 + m, nz) * sz;
#pragma unroll
            for (int c = 0; c < 4; ++c) hR[slot(k0 - 2 + m)][c][t] = rb[c * n3 + qh];
        }
    }
#pragma unroll
    for (int m = 0; m < 5; ++m)
#pragma unroll
        for (int c = 0; c < 4; ++c) Tq[m][c] = 0.0;
    const double cz = ihz * (1.0 / 12.0);
    // loads for the plane after the current one (halo velocities, further rbar points)
    double hu[4] = {1.0, 0.0, 0.0, 0.0}, er[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = k0; k < z1 + 2; ++k) {
        // planes z0 .. z1-1 are formed in full; the two planes on either side only for f_z.
        // Every load is issued one iteration (the rings three planes) ahead of its use.
        const bool full = is_full(k);
        double Rn[4], Un[4], Hn[4];  // plane k+3 of the column and of the halo point
        {
            const size_t q = col + (size_t)wrapn(k + 3, nz) * sz;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                Rn[c] = rb[c * n3 + q];
                Un[c] = u[c * n3 + q];
            }
            if (own_h) {
                const size_t qh = hcol + (size_t)wrapn(k + 3, nz) * sz;
#pragma unroll
                for (int c = 0; c < 4; ++c) Hn[c] = rb[c * n3 + qh];
            }
        }
        const int ko = k - 2;  // finished in this iteration: its f_z are known two planes on either side
        const bool out = ko >= z0 && act;
        const size_t po = (size_t)wrapn(ko, nz) * sz + col;
        double us[5], ubv[5];
        if (out) {
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                us[v] = u[v * n3 + po];
                ubv[v] = ubar[v * n3 + po];
            }
        }
        if (own_h) {
            const int s0 = slot(k);
#pragma unroll
            for (int c = 0; c < 4; ++c) sR[c][hby][hbx] = hR[s0][c][t];
            if (full) {
                const double inv = rcp(hu[0]);
#pragma unroll
                for (int c = 0; c < 3; ++c) sV[c][hby - 2][hbx - 2] = hu[1 + c] * inv;
            }
        }
        if (own_e && full) {
#pragma unroll
            for (int c = 0; c < 4; ++c) sR[c][eby][ebx] = er[c];
        }
        if (is_full(k + 1)) {
            if (own_h) {
                const size_t qh = hcol + (size_t)wrapn(k + 1, nz) * sz;
#pragma unroll
                for (int c = 0; c < 4; ++c) hu[c] = u[c * n3 + qh];
            }
            if (own_e) {
                const size_t qe = ecol + (size_t)wrapn(k + 1, nz) * sz;
#pragma unroll
                for (int c = 0; c < 4; ++c) er[c] = rb[c * n3 + qe];
            }
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) sR[c][ty + 4][tx + 4] = Rz[2][c];
#pragma unroll
        for (int c = 0; c < 3; ++c) sV[c][ty + 2][tx + 2] = Vz[2][c];
        __syncthreads();
        double pa[3] = {0.0, 0.0, 0.0};
        {
            // the tile's point: rbar gradient, fields
            const int X = tx + 4, Y = ty + 4;
            double Gbar[3][4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                Gbar[0][c] = -dcen(sR[c][Y][X - 2], sR[c][Y][X - 1], sR[c][Y][X + 1], sR[c][Y][X + 2]) * ihx;
                Gbar[1][c] = -dcen(sR[c][Y - 2][X], sR[c][Y - 1][X], sR[c][Y + 1][X], sR[c][Y + 2][X]) * ihy;
                Gbar[2][c] = -dcen(Rz[0][c], Rz[1][c], Rz[3][c], Rz[4][c]) * ihz;
            }
            const AvFields f = av_fields(Gbar, Vz[2], mu, kc);
            // -D_z f_z: dcen(m2, m1, p1, p2) = (8 (p1 - m1) - (p2 - m2)) / 12, so f_z of this
            // plane enters the planes k+2, k+1, k-1, k-2 with -1, 8, -8, 1 times cz
            const double fz[4] = {f.gxz, f.gyz, f.gzz, f.ez};
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const double w = cz * fz[a];
                Tq[4][a] = -w;
                Tq[3][a] += 8.0 * w;
                Tq[1][a] -= 8.0 * w;
                Tq[0][a] += w;
            }
            if (full) {
                sFx[0][ty][tx + 2] = f.gxx;
                sFx[1][ty][tx + 2] = f.gxy;
                sFx[2][ty][tx + 2] = f.gxz;
                sFx[3][ty][tx + 2] = f.ex;
                sFy[0][ty + 2][tx] = f.gxy;
                sFy[1][ty + 2][tx] = f.gyy;
                sFy[2][ty + 2][tx] = f.gyz;
                sFy[3][ty + 2][tx] = f.ey;
                // point fields: the velocity gradients of the plane, tau
                double gv[3][3];  // gv[a][b] = d v_a / d x_b
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    gv[a][0] = dcen(sV[a][ty + 2][tx], sV[a][ty + 2][tx + 1], sV[a][ty + 2][tx + 3],
                                    sV[a][ty + 2][tx + 4]) * ihx;
                    gv[a][1] = dcen(sV[a][ty][tx + 2], sV[a][ty + 1][tx + 2], sV[a][ty + 3][tx + 2],
                                    sV[a][ty + 4][tx + 2]) * ihy;
                    gv[a][2] = dcen(Vz[0][a], Vz[1][a], Vz[3][a], Vz[4][a]) * ihz;
                }
                const double div = gv[0][0] + gv[1][1] + gv[2][2];
                const double tdiv = 2.0 / 3.0 * div;
                const double txx = mu * (2.0 * gv[0][0] - tdiv), tyy = mu * (2.0 * gv[1][1] - tdiv),
                             tzz = mu * (2.0 * gv[2][2] - tdiv);
                const double txy = mu * (gv[0][1] + gv[1][0]), txz = mu * (gv[0][2] + gv[2][0]),
                             tyz = mu * (gv[1][2] + gv[2][1]);
                const double Ex = Gbar[0][3], Ey = Gbar[1][3], Ez = Gbar[2][3];
                pa[0] = Ex * txx + Ey * txy + Ez * txz;
                pa[1] = Ex * txy + Ey * tyy + Ez * tyz;
                pa[2] = Ex * txz + Ey * tyz + Ez * tzz;
            }
        }
        if (own_h && full) {
            // a halo point: rbar gradient (z from the halo ring), its f_x or f_y
            double Gbar[3][4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                Gbar[0][c] = -dcen(sR[c][hby][hbx - 2], sR[c][hby][hbx - 1], sR[c][hby][hbx + 1],
                                   sR[c][hby][hbx + 2]) * ihx;
                Gbar[1][c] = -dcen(sR[c][hby - 2][hbx], sR[c][hby - 1][hbx], sR[c][hby + 1][hbx],
                                   sR[c][hby + 2][hbx]) * ihy;
                Gbar[2][c] = -dcen(hR[slot(k - 2)][c][t], hR[slot(k - 1)][c][t], hR[slot(k + 1)][c][t],
                                   hR[slot(k + 2)][c][t]) * ihz;
            }
            const double v[3] = {sV[0][hby - 2][hbx - 2], sV[1][hby - 2][hbx - 2], sV[2][hby - 2][hbx - 2]};
            const AvFields f = av_fields(Gbar, v, mu, kc);
            if (t < 4 * TY) {
                const int r = hby - 4, cx = hbx - 2;
                sFx[0][r][cx] = f.gxx;
                sFx[1][r][cx] = f.gxy;
                sFx[2][r][cx] = f.gxz;
                sFx[3][r][cx] = f.ex;
            } else {
                const int r = hby - 2, cx = hbx - 4;
                sFy[0][r][cx] = f.gxy;
                sFy[1][r][cx] = f.gyy;
                sFy[2][r][cx] = f.gyz;
                sFy[3][r][cx] = f.ey;
            }
        }
        __syncthreads();
        if (full) {
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                double s = a < 3 ? pa[a] : 0.0;
                s -= dcen(sFx[a][ty][tx], sFx[a][ty][tx + 1], sFx[a][ty][tx + 3], sFx[a][ty][tx + 4]) * ihx;
                s -= dcen(sFy[a][ty][tx], sFy[a][ty + 1][tx], sFy[a][ty + 3][tx], sFy[a][ty + 4][tx]) * ihy;
                Tq[2][a] += s;
            }
        }
        if (out) {
            const double *Wb = Tq[0];
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
            const double fin[5] = {ubv[0] + -invb * inv * inv, ubv[1] + mb[0], ubv[2] + mb[1], ubv[3] + mb[2],
                                   ubv[4] + eb};
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                const size_t o = v * n3 + po;
                if (ep.store_ub) ubar[o] = fin[v];
                adj_epilogue_at(ep, o, fin[v]);
            }
        }
        // advance the rings; plane k+3 enters them
#pragma unroll
        for (int m = 0; m < 4; ++m) {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                Rz[m][c] = Rz[m + 1][c];
                Tq[m][c] = Tq[m + 1][c];
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) Vz[m][c] = Vz[m + 1][c];
        }
        {
            const double inv = rcp(Un[0]);
#pragma unroll
            for (int c = 0; c < 4; ++c) Rz[4][c] = Rn[c];
#pragma unroll
            for (int c = 0; c < 3; ++c) Vz[4][c] = Un[1 + c] * inv;
        }
        if (own_h) {
            const int s3 = slot(k + 3);
#pragma unroll
            for (int c = 0; c < 4; ++c) hR[s3][c][t] = Hn[c];
        }
    }
}

// out = a x + b y (y may be null)
__global__ void k_lincomb(size_t n, double a, const double *__restrict__ x, double b, const double *__restrict__ y,
                          double *__restrict__ out) {
    const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = y ? a * x[i] + b * y[i] : a * x[i];
}

// out = x
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
    // blocks: x, 4 rows each; y, z: one x tile of the lines at one z (y) each
    const unsigned bx = (unsigned)(((size_t)b.ny * b.nz + 3) / 4);
    constexpr int TB = 4 * AdjConvShape<1>::LW;
    static_assert(AdjConvShape<2>::LW == AdjConvShape<1>::LW, "y and z blocks alike");
    const unsigned ntx = (unsigned)((b.nx + TB - 1) / TB);
    hipLaunchKernelGGL((k_adj_conv<0, WW>), dim3(bx), dim3(256), 0, s, g, u, rbar, ubar, 0);
    hipLaunchKernelGGL((k_adj_conv<1, WW>), dim3(ntx * (unsigned)b.nz), dim3(256), 0, s, g, u, rbar, ubar, 1);
    hipLaunchKernelGGL((k_adj_conv<2, WW>), dim3(ntx * (unsigned)b.ny), dim3(256), 0, s, g, u, rbar, ubar, 1);
}

// the stage-combination epilogue by separate launches (boxes without viscous terms)
__global__ void k_epilogue(size_t n, const double *__restrict__ fin, AdjEpilogue e) {
    const size_t o = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (o >= n) return;
    adj_epilogue_at(e, o, fin[o]);
}

static void rhs_vjp(const BoxDesc &b, int weights, hipStream_t s, const double *u, const double *rbar, double *ubar,
                    const AdjEpilogue *epi) {
    const AdjGeom g = adj_geom(b);
    if (weights == CNS_WENO_Z) adj_conv<CNS_WENO_Z>(b, s, g, u, rbar, ubar);
    else if (weights == CNS_WENO_M) adj_conv<CNS_WENO_M>(b, s, g, u, rbar, ubar);
    else adj_conv<CNS_WENO_JS>(b, s, g, u, rbar, ubar);
    AdjEpilogue e;
    if (epi) e = *epi;
    if (b.mu > 0.0) {
        const unsigned tiles = (unsigned)(((b.nx + kAvTX - 1) / kAvTX) * (long long)((b.ny + kAvTY - 1) / kAvTY) *
                                          ((b.nz + adj_visc_planes(b.nz) - 1) / adj_visc_planes(b.nz)));
        hipLaunchKernelGGL(k_adj_visc, dim3(tiles), dim3(kPointThreads), 0, s, g, u, rbar, ubar, e);
    } else if (epi) {
        // ubar holds the finished product; the epilogue reads it from there
        const size_t n5 = 5 * b.n3;
        hipLaunchKernelGGL(k_epilogue, dim3((unsigned)((n5 + 255) / 256)), dim3(256), 0, s, n5, (const double *)ubar, e);
    }
}

void adj_rhs_vjp(const BoxDesc &b, int weights, hipStream_t s, const double *u, const double *rbar, double *ubar) {
    rhs_vjp(b, weights, s, u, rbar, ubar, nullptr);
}

void adj_rhs_vjp_epi(const BoxDesc &b, int weights, hipStream_t s, const double *u, const double *rbar, double *ubar,
                     const AdjEpilogue &epi) {
    rhs_vjp(b, weights, s, u, rbar, ubar, &epi);
}

void adj_lincomb(size_t n, double a, const double *x, double b, const double *y, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_lincomb, grid1(n), dim3(256), 0, s, n, a, x, b, y, out);
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
