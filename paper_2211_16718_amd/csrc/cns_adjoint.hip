// cns_adjoint.hip -- reverse-mode kernels of the RHS (vector-Jacobian products) and the
// small kernels of the checkpointed reverse RK4, FP64, single box.
//
// (dR/du)^T rbar of the semi-discrete operator R(u) = -sum_d (H_{j+1/2} - H_{j-1/2})/dx_d
// + sum_d D_d G^v_d is assembled as
//   convective part, per direction d:  Hbar_{j+1/2} = (rbar_{j+1} - rbar_j)/dx_d;
//     k_adj_iface<d>: one thread per interface forms the local product of the
//     interface flux (30 contributions to the six cells it reads) into C;
//     k_adj_gather<d>: one thread per point sums the six contributions it receives;
//   viscous part: the adjoint of a central difference is minus the same central
//     difference, so Gbar_d = -D_d rbar; k_adj_visc1 maps it through the viscous
//     fluxes to the adjoints of the velocity/temperature gradients and of the
//     point velocities; k_adj_visc2 applies -D once more and the primitive map.
// Every sum is formed in a fixed order (deterministic, no atomics).
#include <hip/hip_runtime.h>

#include "cns_device_adj.h"
#include "cns_internal.h"

namespace cns {

__device__ __forceinline__ int wrapj(int j, int n) { return j < 0 ? j + n : (j >= n ? j - n : j); }

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

template <int DIR>
__global__ __launch_bounds__(256) void k_adj_iface(AdjGeom g, const double *__restrict__ u,
                                                   const double *__restrict__ rbar, double *__restrict__ C) {
    const size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (p >= g.n3) return;
    const int i = (int)(p % g.nx), j = (int)((p / g.nx) % g.ny), k = (int)(p / ((size_t)g.nx * g.ny));
    const size_t n3 = g.n3;
    double w[6][5];
#pragma unroll
    for (int m = 0; m < 6; ++m) {
        const size_t q = shift_idx(g, i, j, k, DIR, m - 2);
#pragma unroll
        for (int v = 0; v < 5; ++v) w[m][v] = u[v * n3 + q];
    }
    const size_t pn = shift_idx(g, i, j, k, DIR, 1);
    double Hb[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) Hb[v] = (rbar[v * n3 + pn] - rbar[v * n3 + p]) * g.ih[DIR];
    double wb[6][5];
#pragma unroll
    for (int m = 0; m < 6; ++m)
#pragma unroll
        for (int v = 0; v < 5; ++v) wb[m][v] = 0.0;
    interface_flux_vjp<DIR>(w, Hb, g.gamma, g.eps, g.delta, wb);
#pragma unroll
    for (int m = 0; m < 6; ++m)
#pragma unroll
        for (int v = 0; v < 5; ++v) C[(size_t)(m * 5 + v) * n3 + p] = wb[m][v];
}

// ubar(p) (=|+=) sum_m C[m](p - (m - 2) e_d): point p is cell m of the interface at p-(m-2)
template <int DIR>
__global__ __launch_bounds__(256) void k_adj_gather(AdjGeom g, const double *__restrict__ C, double *__restrict__ ubar,
                                                    int accumulate) {
    const size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (p >= g.n3) return;
    const int i = (int)(p % g.nx), j = (int)((p / g.nx) % g.ny), k = (int)(p / ((size_t)g.nx * g.ny));
    const size_t n3 = g.n3;
    size_t src[6];
#pragma unroll
    for (int m = 0; m < 6; ++m) src[m] = shift_idx(g, i, j, k, DIR, 2 - m);
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        double s = 0.0;
#pragma unroll
        for (int m = 0; m < 6; ++m) s += C[(size_t)(m * 5 + v) * n3 + src[m]];
        if (accumulate) ubar[v * n3 + p] += s;
        else ubar[v * n3 + p] = s;
    }
}

// viscous adjoint, part 1: Gbar_d = -D_d rbar; through tau, q, E to the adjoints of the
// 12 gradients g[a][b] = d W_a/dx_b (W = u, v, w, T) and of the point velocities.
// Output Gb: [12] gradient adjoints (a-major), then [3] point-velocity adjoints.
__global__ __launch_bounds__(256) void k_adj_visc1(AdjGeom g, const double *__restrict__ W,
                                                   const double *__restrict__ rbar, double *__restrict__ Gb) {
    const size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (p >= g.n3) return;
    const int i = (int)(p % g.nx), j = (int)((p / g.nx) % g.ny), k = (int)(p / ((size_t)g.nx * g.ny));
    const size_t n3 = g.n3;
    size_t nb[3][4];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        nb[d][0] = shift_idx(g, i, j, k, d, -2);
        nb[d][1] = shift_idx(g, i, j, k, d, -1);
        nb[d][2] = shift_idx(g, i, j, k, d, 1);
        nb[d][3] = shift_idx(g, i, j, k, d, 2);
    }
    // forward at p: gradients, stresses
    double gr[4][3];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double *f = W + a * n3;
            gr[a][d] = dcen(f[nb[d][0]], f[nb[d][1]], f[nb[d][2]], f[nb[d][3]]) * g.ih[d];
        }
    const double mu = g.mu, kc = g.mu / ((g.gamma - 1.0) * g.prandtl);
    const double div = gr[0][0] + gr[1][1] + gr[2][2];
    const double tdiv = 2.0 / 3.0 * div;
    const double txx = mu * (2.0 * gr[0][0] - tdiv), tyy = mu * (2.0 * gr[1][1] - tdiv),
                 tzz = mu * (2.0 * gr[2][2] - tdiv);
    const double txy = mu * (gr[0][1] + gr[1][0]), txz = mu * (gr[0][2] + gr[2][0]),
                 tyz = mu * (gr[1][2] + gr[2][1]);
    const double vx = W[p], vy = W[n3 + p], vz = W[2 * n3 + p];
    // Gbar_d[c] = -(D_d rbar_{1+c})(p), c: x-, y-, z-momentum, energy
    double Gbar[3][4];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const double *r = rbar + (1 + c) * n3;
            Gbar[d][c] = -dcen(r[nb[d][0]], r[nb[d][1]], r[nb[d][2]], r[nb[d][3]]) * g.ih[d];
        }
    // G_x = [txx, txy, txz, Ex], G_y = [txy, tyy, tyz, Ey], G_z = [txz, tyz, tzz, Ez]
    // E_x = vx txx + vy txy + vz txz + kc dT/dx, etc.
    const double Ex = Gbar[0][3], Ey = Gbar[1][3], Ez = Gbar[2][3];
    const double bxx = Gbar[0][0] + Ex * vx;
    const double byy = Gbar[1][1] + Ey * vy;
    const double bzz = Gbar[2][2] + Ez * vz;
    const double bxy = Gbar[0][1] + Gbar[1][0] + Ex * vy + Ey * vx;
    const double bxz = Gbar[0][2] + Gbar[2][0] + Ex * vz + Ez * vx;
    const double byz = Gbar[1][2] + Gbar[2][1] + Ey * vz + Ez * vy;
    const double vbx = Ex * txx + Ey * txy + Ez * txz;
    const double vby = Ex * txy + Ey * tyy + Ez * tyz;
    const double vbz = Ex * txz + Ey * tyz + Ez * tzz;
    // tau_aa = mu (2 g_aa - 2/3 div), tau_ab = mu (g_ab + g_ba)
    const double divb = -2.0 / 3.0 * mu * (bxx + byy + bzz);
    double gb[4][3];
    gb[0][0] = 2.0 * mu * bxx + divb;
    gb[1][1] = 2.0 * mu * byy + divb;
    gb[2][2] = 2.0 * mu * bzz + divb;
    gb[0][1] = mu * bxy;
    gb[1][0] = mu * bxy;
    gb[0][2] = mu * bxz;
    gb[2][0] = mu * bxz;
    gb[1][2] = mu * byz;
    gb[2][1] = mu * byz;
    gb[3][0] = kc * Ex;
    gb[3][1] = kc * Ey;
    gb[3][2] = kc * Ez;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int d = 0; d < 3; ++d) Gb[(size_t)(a * 3 + d) * n3 + p] = gb[a][d];
    Gb[12 * n3 + p] = vbx;
    Gb[13 * n3 + p] = vby;
    Gb[14 * n3 + p] = vbz;
}

// viscous adjoint, part 2: Wbar = point adjoints - sum_b D_b gbar[.][b]; then through
// W(u) = (m/rho, gamma p / rho) to ubar (accumulated)
__global__ __launch_bounds__(256) void k_adj_visc2(AdjGeom g, const double *__restrict__ u,
                                                   const double *__restrict__ Gb, double *__restrict__ ubar) {
    const size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (p >= g.n3) return;
    const int i = (int)(p % g.nx), j = (int)((p / g.nx) % g.ny), k = (int)(p / ((size_t)g.nx * g.ny));
    const size_t n3 = g.n3;
    size_t nb[3][4];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        nb[d][0] = shift_idx(g, i, j, k, d, -2);
        nb[d][1] = shift_idx(g, i, j, k, d, -1);
        nb[d][2] = shift_idx(g, i, j, k, d, 1);
        nb[d][3] = shift_idx(g, i, j, k, d, 2);
    }
    double Wb[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        double s = a < 3 ? Gb[(12 + a) * n3 + p] : 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double *f = Gb + (size_t)(a * 3 + d) * n3;
            s -= dcen(f[nb[d][0]], f[nb[d][1]], f[nb[d][2]], f[nb[d][3]]) * g.ih[d];
        }
        Wb[a] = s;
    }
    // W = (m_k / rho, gamma p / rho), p = (gamma-1)(e - m.v/2)
    const double gm1 = g.gamma - 1.0;
    const double r = u[p], m[3] = {u[n3 + p], u[2 * n3 + p], u[3 * n3 + p]}, e = u[4 * n3 + p];
    const double inv = 1.0 / r;
    const double v[3] = {m[0] * inv, m[1] * inv, m[2] * inv};
    const double qq = m[0] * v[0] + m[1] * v[1] + m[2] * v[2];
    const double pr = gm1 * (e - 0.5 * qq);
    // T = gamma pr inv
    const double prb = g.gamma * inv * Wb[3];
    double invb = g.gamma * pr * Wb[3];
    const double eb = gm1 * prb;
    const double qqb = -0.5 * gm1 * prb;
    double mb[3], vb[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        vb[c] = Wb[c] + qqb * m[c];
        mb[c] = qqb * v[c] + vb[c] * inv;
        invb += vb[c] * m[c];
    }
    ubar[p] += -invb * inv * inv;
    ubar[n3 + p] += mb[0];
    ubar[2 * n3 + p] += mb[1];
    ubar[3 * n3 + p] += mb[2];
    ubar[4 * n3 + p] += eb;
}

// W = (u, v, w, T) at the linearisation point (same arithmetic as the forward k_prim)
__global__ void k_adj_prim(AdjGeom g, const double *__restrict__ u, double *__restrict__ W) {
    const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (i >= g.n3) return;
    const size_t n3 = g.n3;
    const double r = u[i], mx = u[n3 + i], my = u[2 * n3 + i], mz = u[3 * n3 + i], e = u[4 * n3 + i];
    const double inv = 1.0 / r;
    const double vx = mx * inv, vy = my * inv, vz = mz * inv;
    const double p = (g.gamma - 1.0) * (e - 0.5 * (mx * vx + my * vy + mz * vz));
    W[i] = vx;
    W[n3 + i] = vy;
    W[2 * n3 + i] = vz;
    W[3 * n3 + i] = g.gamma * p * inv;
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

// out = u + c k (an RK4 stage state, same arithmetic as the fused stage update)
__global__ void k_stage(size_t n, double c, const double *__restrict__ u, const double *__restrict__ k,
                        double *__restrict__ out) {
    const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (i < n) out[i] = u[i] + c * k[i];
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

void adj_rhs_vjp(const BoxDesc &b, hipStream_t s, const double *u, const double *rbar, double *ubar, double *W,
                 double *C, double *Gb) {
    const AdjGeom g = adj_geom(b);
    const size_t n3 = b.n3;
    const bool visc = b.mu > 0.0;
    if (visc) hipLaunchKernelGGL(k_adj_prim, grid1(n3), dim3(256), 0, s, g, u, W);
    if (visc) hipLaunchKernelGGL(k_adj_visc1, grid1(n3), dim3(256), 0, s, g, (const double *)W, rbar, Gb);
    hipLaunchKernelGGL(k_adj_iface<0>, grid1(n3), dim3(256), 0, s, g, u, rbar, C);
    hipLaunchKernelGGL(k_adj_gather<0>, grid1(n3), dim3(256), 0, s, g, (const double *)C, ubar, 0);
    hipLaunchKernelGGL(k_adj_iface<1>, grid1(n3), dim3(256), 0, s, g, u, rbar, C);
    hipLaunchKernelGGL(k_adj_gather<1>, grid1(n3), dim3(256), 0, s, g, (const double *)C, ubar, 1);
    hipLaunchKernelGGL(k_adj_iface<2>, grid1(n3), dim3(256), 0, s, g, u, rbar, C);
    hipLaunchKernelGGL(k_adj_gather<2>, grid1(n3), dim3(256), 0, s, g, (const double *)C, ubar, 1);
    if (visc) hipLaunchKernelGGL(k_adj_visc2, grid1(n3), dim3(256), 0, s, g, u, (const double *)Gb, ubar);
}

void adj_lincomb(size_t n, double a, const double *x, double b, const double *y, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_lincomb, grid1(n), dim3(256), 0, s, n, a, x, b, y, out);
}
void adj_accum(size_t n, const double *x, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_accum, grid1(n), dim3(256), 0, s, n, x, out);
}
void adj_stage(size_t n, double c, const double *u, const double *k, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_stage, grid1(n), dim3(256), 0, s, n, c, u, k, out);
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
