/*
 * cns_oracle.c -- plain FP64 CPU oracle (TEST INFRASTRUCTURE ONLY; see cns_oracle.h).
 *
 * Written straight from the paper's equations, in their order and notation,
 * with plain loops and explicit 5x5 eigenvector matrices.  Nothing here is
 * blocked, fused or reordered for speed; OpenMP only splits the independent
 * per-point loops across threads, so results do not depend on the thread count.
 * Built with -O2 -ffp-contract=off (no fused multiply-add).
 *
 * Readings of the paper taken here (each is listed in the design notes):
 *  - viscous stress uses the symmetric (+) form  mu_eff[(d_j u_i + d_i u_j) - 2/3 delta_ij div v]
 *    (the printed minus sign would give a negative bulk viscosity);
 *  - WENO weight exponent p = 2 (Jiang-Shu), epsilon added before the power;
 *  - f^{L,R} and u^{L,R} are component-wise WENO5 reconstructions of the
 *    cell-centred flux f(u_j) and state u_j (no flux splitting, no
 *    characteristic projection); R is the mirror image of L about j+1/2;
 *  - the Roe average is taken between the cell states u_j and u_{j+1};
 *  - Harten's fix: |lam|_H = |lam| if |lam| >= delta else (lam^2 + delta^2)/(2 delta),
 *    on all five eigenvalues;
 *  - viscous derivatives: the 5-point 4th-order central first derivative applied
 *    twice (inner on u, v, w, T; outer on the viscous flux G^v_d);
 *  - periodic wrap of indices instead of ghost points.
 */
#include "cns_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Scalar type of everything that depends on the state.  As it stands this file is
 * the FP64 oracle.  cns_oracle_cs.c compiles it a second time with a complex type
 * (complex-step derivatives): it defines ORC_REAL, the three helpers below and new
 * names for the exported functions before including this file.  ORC_RE takes the
 * real part wherever the method compares or tests a value. */
#ifndef ORC_REAL
#define ORC_REAL double
#define ORC_SQRT sqrt
#define ORC_ABS fabs
#define ORC_RE(x) (x)
#endif
typedef ORC_REAL real;

/* ------------------------------------------------------------------------- */
/* grid helpers                                                              */
/* ------------------------------------------------------------------------- */
static int wrapi(int i, int n) {
    int r = i % n;
    return r < 0 ? r + n : r;
}

static size_t npts(const orc_grid *g) { return (size_t)g->nx * g->ny * g->nz; }

static size_t lin(const orc_grid *g, int i, int j, int k) {
    return ((size_t)k * g->ny + j) * g->nx + i;
}

/* linear index of the point displaced by `off` along `dir` from (i,j,k), periodic */
static size_t shifted(const orc_grid *g, int i, int j, int k, int dir, int off) {
    int c[3] = {i, j, k};
    int n[3] = {g->nx, g->ny, g->nz};
    c[dir] = wrapi(c[dir] + off, n[dir]);
    return lin(g, c[0], c[1], c[2]);
}

static double spacing(const orc_grid *g, int dir) {
    if (dir == 0) return g->lx / g->nx;
    if (dir == 1) return g->ly / g->ny;
    return g->lz / g->nz;
}

static int check_grid(const orc_grid *g, const orc_phys *ph) {
    if (!g || g->nx < 8 || g->ny < 8 || g->nz < 8) return ORC_EINVAL;
    if (!(g->lx > 0 && g->ly > 0 && g->lz > 0)) return ORC_EINVAL;
    if (ph && !(ph->gamma > 1.0 && ph->mu_eff >= 0.0 && ph->weno_eps > 0.0 && ph->harten_delta >= 0.0))
        return ORC_EINVAL;
    if (ph && ph->weno_weights != ORC_WENO_JS && ph->weno_weights != ORC_WENO_Z && ph->weno_weights != ORC_WENO_M)
        return ORC_EINVAL;
    if (ph && ph->mu_eff > 0.0 && !(ph->prandtl > 0.0)) return ORC_EINVAL;
    return ORC_OK;
}

/* gather the conserved state at linear index p */
static void load_state(const real *u, size_t n3, size_t p, real s[5]) {
    for (int v = 0; v < 5; ++v) s[v] = u[(size_t)v * n3 + p];
}

/* Sec. 2.1: primitive variables from the conserved state; e = p/(gamma-1) + rho|v|^2/2 */
static int primitives(const real s[5], double gamma, real vel[3], real *p, real *T) {
    real rho = s[0];
    vel[0] = s[1] / rho;
    vel[1] = s[2] / rho;
    vel[2] = s[3] / rho;
    real q2 = vel[0] * vel[0] + vel[1] * vel[1] + vel[2] * vel[2];
    *p = (gamma - 1.0) * (s[4] - 0.5 * rho * q2);
    *T = gamma * (*p) / rho; /* T = gamma p / rho (Sec. 2.1, heat flux) */
    if (!isfinite(ORC_RE(rho)) || !isfinite(ORC_RE(*p)) || !isfinite(ORC_RE(q2))) return ORC_ENONFINITE;
    if (!(ORC_RE(rho) > 0.0) || !(ORC_RE(*p) > 0.0)) return ORC_ENONPHYSICAL;
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Sec. 2.2: WENO5 (three third-order candidates, optimal weights 1/10, 6/10, */
/* 3/10, Jiang-Shu smoothness indicators, alpha_k = c_k/(eps+beta_k)^2)       */
/* ------------------------------------------------------------------------- */
real oracle_weno5(real a, real b, real c, real d, real e, double eps, real *parts) {
    /* a..e = f_{j-2}, f_{j-1}, f_j, f_{j+1}, f_{j+2} */
    real fhat1 = (1.0 / 3.0) * a - (7.0 / 6.0) * b + (11.0 / 6.0) * c;
    real fhat2 = -(1.0 / 6.0) * b + (5.0 / 6.0) * c + (1.0 / 3.0) * d;
    real fhat3 = (1.0 / 3.0) * c + (5.0 / 6.0) * d - (1.0 / 6.0) * e;

    real beta1 = (13.0 / 12.0) * (a - 2.0 * b + c) * (a - 2.0 * b + c) +
                 0.25 * (a - 4.0 * b + 3.0 * c) * (a - 4.0 * b + 3.0 * c);
    real beta2 = (13.0 / 12.0) * (b - 2.0 * c + d) * (b - 2.0 * c + d) + 0.25 * (b - d) * (b - d);
    real beta3 = (13.0 / 12.0) * (c - 2.0 * d + e) * (c - 2.0 * d + e) +
                 0.25 * (3.0 * c - 4.0 * d + e) * (3.0 * c - 4.0 * d + e);

    real alpha1 = 0.1 / ((eps + beta1) * (eps + beta1));
    real alpha2 = 0.6 / ((eps + beta2) * (eps + beta2));
    real alpha3 = 0.3 / ((eps + beta3) * (eps + beta3));
    real asum = alpha1 + alpha2 + alpha3;
    real w1 = alpha1 / asum, w2 = alpha2 / asum, w3 = alpha3 / asum;

    if (parts) {
        parts[0] = beta1;
        parts[1] = beta2;
        parts[2] = beta3;
        parts[3] = w1;
        parts[4] = w2;
        parts[5] = w3;
        parts[6] = fhat1;
        parts[7] = fhat2;
        parts[8] = fhat3;
    }
    return w1 * fhat1 + w2 * fhat2 + w3 * fhat3;
}

/* ------------------------------------------------------------------------- */
/* WENO-Z weights (Borges, Carmona, Costa & Don, J. Comput. Phys. 227, 2008), */
/* one of the low-dissipation successors the paper names: the same candidates */
/* and smoothness indicators, alpha_k = c_k (1 + (tau5/(eps+beta_k))^2) with  */
/* the global indicator tau5 = |beta_1 - beta_3|.                             */
/* ------------------------------------------------------------------------- */
real oracle_weno5z(real a, real b, real c, real d, real e, double eps, real *parts) {
    real fhat1 = (1.0 / 3.0) * a - (7.0 / 6.0) * b + (11.0 / 6.0) * c;
    real fhat2 = -(1.0 / 6.0) * b + (5.0 / 6.0) * c + (1.0 / 3.0) * d;
    real fhat3 = (1.0 / 3.0) * c + (5.0 / 6.0) * d - (1.0 / 6.0) * e;

    real beta1 = (13.0 / 12.0) * (a - 2.0 * b + c) * (a - 2.0 * b + c) +
                 0.25 * (a - 4.0 * b + 3.0 * c) * (a - 4.0 * b + 3.0 * c);
    real beta2 = (13.0 / 12.0) * (b - 2.0 * c + d) * (b - 2.0 * c + d) + 0.25 * (b - d) * (b - d);
    real beta3 = (13.0 / 12.0) * (c - 2.0 * d + e) * (c - 2.0 * d + e) +
                 0.25 * (3.0 * c - 4.0 * d + e) * (3.0 * c - 4.0 * d + e);
    real tau5 = ORC_ABS(beta1 - beta3);

    real r1 = tau5 / (eps + beta1), r2 = tau5 / (eps + beta2), r3 = tau5 / (eps + beta3);
    real alpha1 = 0.1 * (1.0 + r1 * r1);
    real alpha2 = 0.6 * (1.0 + r2 * r2);
    real alpha3 = 0.3 * (1.0 + r3 * r3);
    real asum = alpha1 + alpha2 + alpha3;
    real w1 = alpha1 / asum, w2 = alpha2 / asum, w3 = alpha3 / asum;

    if (parts) {
        parts[0] = beta1;
        parts[1] = beta2;
        parts[2] = beta3;
        parts[3] = w1;
        parts[4] = w2;
        parts[5] = w3;
        parts[6] = fhat1;
        parts[7] = fhat2;
        parts[8] = fhat3;
    }
    return w1 * fhat1 + w2 * fhat2 + w3 * fhat3;
}

/* ------------------------------------------------------------------------- */
/* Mapped WENO weights (Henrick, Aslam & Powers, J. Comput. Phys. 207, 2005),  */
/* the other improvement of the nonlinear weights the paper cites: the Jiang-  */
/* Shu weights w_k pass through g_k(w) = w (d_k + d_k^2 - 3 d_k w + w^2) /    */
/* (d_k^2 + w (1 - 2 d_k)), d_k the optimal weight, and are renormalised.      */
/* ------------------------------------------------------------------------- */
real oracle_weno_map(real w, double d) {
    return w * (d + d * d - 3.0 * d * w + w * w) / (d * d + w * (1.0 - 2.0 * d));
}

real oracle_weno5m(real a, real b, real c, real d, real e, double eps, real *parts) {
    real js[9];
    oracle_weno5(a, b, c, d, e, eps, js); /* candidates, indicators, Jiang-Shu weights */
    const double dk[3] = {0.1, 0.6, 0.3};
    real g[3], gsum = 0.0;
    for (int k = 0; k < 3; ++k) {
        g[k] = oracle_weno_map(js[3 + k], dk[k]);
        gsum += g[k];
    }
    real w[3];
    for (int k = 0; k < 3; ++k) w[k] = g[k] / gsum;
    if (parts) {
        for (int k = 0; k < 3; ++k) {
            parts[k] = js[k];
            parts[3 + k] = w[k];
            parts[6 + k] = js[6 + k];
        }
    }
    return w[0] * js[6] + w[1] * js[7] + w[2] * js[8];
}

/* ------------------------------------------------------------------------- */
/* Sec. 2.1: convective fluxes f, g, h                                        */
/* ------------------------------------------------------------------------- */
void oracle_flux(const real *u, int dir, double gamma, real *f) {
    real rho = u[0];
    real vel[3] = {u[1] / rho, u[2] / rho, u[3] / rho};
    real p = (gamma - 1.0) * (u[4] - 0.5 * rho * (vel[0] * vel[0] + vel[1] * vel[1] + vel[2] * vel[2]));
    real vn = vel[dir];
    f[0] = rho * vn;
    f[1] = rho * vel[0] * vn;
    f[2] = rho * vel[1] * vn;
    f[3] = rho * vel[2] * vn;
    f[1 + dir] += p;
    f[4] = (u[4] + p) * vn;
}

/* ------------------------------------------------------------------------- */
/* Sec. 2.2: Roe-averaged eigensystem |A| = X |Lambda| X^{-1}                 */
/* ------------------------------------------------------------------------- */
int oracle_roe_eigensystem(const real *uL, const real *uR, int dir, double gamma, real *X, real *Xinv,
                           real *lam) {
    real vL[3], vR[3], pL, pR, TL, TR;
    int rc = primitives(uL, gamma, vL, &pL, &TL);
    if (rc) return rc;
    rc = primitives(uR, gamma, vR, &pR, &TR);
    if (rc) return rc;
    real HL = (uL[4] + pL) / uL[0]; /* total enthalpy (e + p)/rho */
    real HR = (uR[4] + pR) / uR[0];

    /* Roe average: sqrt(rho)-weighted velocity and enthalpy */
    real Rr = ORC_SQRT(uR[0] / uL[0]);
    real v[3];
    for (int c = 0; c < 3; ++c) v[c] = (vL[c] + Rr * vR[c]) / (1.0 + Rr);
    real H = (HL + Rr * HR) / (1.0 + Rr);
    real q2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    real c2 = (gamma - 1.0) * (H - 0.5 * q2);
    if (!isfinite(ORC_RE(c2))) return ORC_ENONFINITE;
    if (!(ORC_RE(c2) > 0.0)) return ORC_ENONPHYSICAL;
    real c = ORC_SQRT(c2);

    int n = dir, t1 = (dir + 1) % 3, t2 = (dir + 2) % 3;
    real vn = v[n];

    memset(X, 0, 25 * sizeof(real));
    memset(Xinv, 0, 25 * sizeof(real));
#define XS(r, col) X[(r)*5 + (col)]
#define LS(r, col) Xinv[(r)*5 + (col)]
    /* column 0: acoustic wave vn - c */
    XS(0, 0) = 1.0;
    for (int k = 0; k < 3; ++k) XS(1 + k, 0) = v[k];
    XS(1 + n, 0) -= c;
    XS(4, 0) = H - vn * c;
    /* column 1: entropy wave vn */
    XS(0, 1) = 1.0;
    for (int k = 0; k < 3; ++k) XS(1 + k, 1) = v[k];
    XS(4, 1) = 0.5 * q2;
    /* columns 2, 3: shear waves vn along the two tangential directions */
    XS(1 + t1, 2) = 1.0;
    XS(4, 2) = v[t1];
    XS(1 + t2, 3) = 1.0;
    XS(4, 3) = v[t2];
    /* column 4: acoustic wave vn + c */
    XS(0, 4) = 1.0;
    for (int k = 0; k < 3; ++k) XS(1 + k, 4) = v[k];
    XS(1 + n, 4) += c;
    XS(4, 4) = H + vn * c;

    /* rows of X^{-1}: left eigenvectors */
    real b1 = (gamma - 1.0) / c2;
    real b2 = 0.5 * q2 * b1;
    LS(0, 0) = 0.5 * (b2 + vn / c);
    for (int k = 0; k < 3; ++k) LS(0, 1 + k) = -0.5 * b1 * v[k];
    LS(0, 1 + n) -= 0.5 / c;
    LS(0, 4) = 0.5 * b1;

    LS(1, 0) = 1.0 - b2;
    for (int k = 0; k < 3; ++k) LS(1, 1 + k) = b1 * v[k];
    LS(1, 4) = -b1;

    LS(2, 0) = -v[t1];
    LS(2, 1 + t1) = 1.0;
    LS(3, 0) = -v[t2];
    LS(3, 1 + t2) = 1.0;

    LS(4, 0) = 0.5 * (b2 - vn / c);
    for (int k = 0; k < 3; ++k) LS(4, 1 + k) = -0.5 * b1 * v[k];
    LS(4, 1 + n) += 0.5 / c;
    LS(4, 4) = 0.5 * b1;
#undef XS
#undef LS

    lam[0] = vn - c;
    lam[1] = vn;
    lam[2] = vn;
    lam[3] = vn;
    lam[4] = vn + c;
    return ORC_OK;
}

real oracle_harten(real lam, double delta) {
    real a = ORC_ABS(lam);
    if (ORC_RE(a) >= delta) return a;
    return (lam * lam + delta * delta) / (2.0 * delta);
}

/* ------------------------------------------------------------------------- */
/* Sec. 2.2 eq. (Roe): F = (f^L + f^R)/2 - |A| (u^R - u^L)/2 at j+1/2         */
/* ------------------------------------------------------------------------- */
int oracle_interface_flux(const real *s, int dir, const orc_phys *ph, real *F) {
    const double gamma = ph->gamma, eps = ph->weno_eps;
    real (*W)(real, real, real, real, real, double, real *) =
        ph->weno_weights == ORC_WENO_Z ? oracle_weno5z : (ph->weno_weights == ORC_WENO_M ? oracle_weno5m : oracle_weno5);
    real f[6][5];
    for (int m = 0; m < 6; ++m) oracle_flux(s + 5 * m, dir, gamma, f[m]);

    /* component-wise WENO5: left-biased from j-2..j+2, right-biased = mirror (j+3..j-1) */
    real fL[5], fR[5], uL[5], uR[5];
    for (int v = 0; v < 5; ++v) {
        fL[v] = W(f[0][v], f[1][v], f[2][v], f[3][v], f[4][v], eps, NULL);
        fR[v] = W(f[5][v], f[4][v], f[3][v], f[2][v], f[1][v], eps, NULL);
        uL[v] = W(s[0 * 5 + v], s[1 * 5 + v], s[2 * 5 + v], s[3 * 5 + v], s[4 * 5 + v], eps, NULL);
        uR[v] = W(s[5 * 5 + v], s[4 * 5 + v], s[3 * 5 + v], s[2 * 5 + v], s[1 * 5 + v], eps, NULL);
    }

    /* eigensystem at the Roe average of the cell states u_j (m=2) and u_{j+1} (m=3) */
    real X[25], Xinv[25], lam[5];
    int rc = oracle_roe_eigensystem(s + 10, s + 15, dir, gamma, X, Xinv, lam);
    if (rc) return rc;

    real du[5], w[5], diss[5];
    for (int v = 0; v < 5; ++v) du[v] = uR[v] - uL[v];
    for (int r = 0; r < 5; ++r) {
        real acc = 0.0;
        for (int col = 0; col < 5; ++col) acc += Xinv[r * 5 + col] * du[col];
        w[r] = oracle_harten(lam[r], ph->harten_delta) * acc;
    }
    for (int r = 0; r < 5; ++r) {
        real acc = 0.0;
        for (int col = 0; col < 5; ++col) acc += X[r * 5 + col] * w[col];
        diss[r] = acc;
    }
    for (int v = 0; v < 5; ++v) F[v] = 0.5 * (fL[v] + fR[v]) - 0.5 * diss[v];
    for (int v = 0; v < 5; ++v)
        if (!isfinite(ORC_RE(F[v]))) return ORC_ENONFINITE;
    return ORC_OK;
}

/* interface flux at (i,j,k) + 1/2 along dir */
static int interface_at(const orc_grid *g, const orc_phys *ph, const real *u, int i, int j, int k, int dir,
                        real F[5]) {
    size_t n3 = npts(g);
    real s[30];
    for (int m = 0; m < 6; ++m) load_state(u, n3, shifted(g, i, j, k, dir, m - 2), s + 5 * m);
    return oracle_interface_flux(s, dir, ph, F);
}

/* ------------------------------------------------------------------------- */
/* Sec. 2.2 conservative finite difference along one direction               */
/* ------------------------------------------------------------------------- */
int oracle_rhs_hyp_dir(const orc_grid *g, const orc_phys *ph, const real *u, int dir, real *out) {
    int rc = check_grid(g, ph);
    if (rc) return rc;
    if (dir < 0 || dir > 2 || !u || !out) return ORC_EINVAL;
    size_t n3 = npts(g);
    real *Fh = (real *)malloc(5 * n3 * sizeof(real)); /* F_{p+1/2} stored at point p */
    if (!Fh) return ORC_EINVAL;
    int err = 0;
#pragma omp parallel for collapse(2) reduction(min : err)
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                real F[5];
                int r = interface_at(g, ph, u, i, j, k, dir, F);
                if (r < err) err = r;
                size_t p = lin(g, i, j, k);
                for (int v = 0; v < 5; ++v) Fh[(size_t)v * n3 + p] = F[v];
            }
    if (err) {
        free(Fh);
        return err;
    }
    double dx = spacing(g, dir);
#pragma omp parallel for collapse(2)
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                size_t p = lin(g, i, j, k);
                size_t pm = shifted(g, i, j, k, dir, -1);
                for (int v = 0; v < 5; ++v)
                    out[(size_t)v * n3 + p] = -(Fh[(size_t)v * n3 + p] - Fh[(size_t)v * n3 + pm]) / dx;
            }
    free(Fh);
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Sec. 2.1 viscous fluxes with 4th-order central first derivatives         */
/* ------------------------------------------------------------------------- */
/* 5-point 4th-order central first derivative of a point function phi along dir */
static real central_d(real pm2, real pm1, real pp1, real pp2, double h) {
    return (8.0 * (pp1 - pm1) - (pp2 - pm2)) / (12.0 * h);
}

/* velocity and temperature at linear index p */
static int vel_temp_at(const real *u, size_t n3, size_t p, double gamma, real w[4]) {
    real s[5], vel[3], pr, T;
    load_state(u, n3, p, s);
    int rc = primitives(s, gamma, vel, &pr, &T);
    w[0] = vel[0];
    w[1] = vel[1];
    w[2] = vel[2];
    w[3] = T;
    return rc;
}

/* viscous fluxes G^v_d (d = x, y, z; five components each) at point (i,j,k) */
static int gvisc_at(const orc_grid *g, const orc_phys *ph, const real *u, int i, int j, int k, real G[3][5]) {
    size_t n3 = npts(g);
    real w0[4];
    int rc = vel_temp_at(u, n3, lin(g, i, j, k), ph->gamma, w0);
    if (rc) return rc;
    /* grad[a][b] = d(w_a)/dx_b, a over (u, v, w, T) */
    real grad[4][3];
    for (int b = 0; b < 3; ++b) {
        real wm2[4], wm1[4], wp1[4], wp2[4];
        rc = vel_temp_at(u, n3, shifted(g, i, j, k, b, -2), ph->gamma, wm2);
        if (!rc) rc = vel_temp_at(u, n3, shifted(g, i, j, k, b, -1), ph->gamma, wm1);
        if (!rc) rc = vel_temp_at(u, n3, shifted(g, i, j, k, b, 1), ph->gamma, wp1);
        if (!rc) rc = vel_temp_at(u, n3, shifted(g, i, j, k, b, 2), ph->gamma, wp2);
        if (rc) return rc;
        double h = spacing(g, b);
        for (int a = 0; a < 4; ++a) grad[a][b] = central_d(wm2[a], wm1[a], wp1[a], wp2[a], h);
    }
    const double mu = ph->mu_eff;
    real divv = grad[0][0] + grad[1][1] + grad[2][2];
    real tau[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            tau[a][b] = mu * ((grad[a][b] + grad[b][a]) - (a == b ? (2.0 / 3.0) * divv : 0.0));
    double kcond = mu / ((ph->gamma - 1.0) * ph->prandtl);
    for (int d = 0; d < 3; ++d) {
        real q = -kcond * grad[3][d];
        G[d][0] = 0.0;
        G[d][1] = tau[0][d];
        G[d][2] = tau[1][d];
        G[d][3] = tau[2][d];
        G[d][4] = (w0[0] * tau[0][d] + w0[1] * tau[1][d] + w0[2] * tau[2][d]) - q;
    }
    return ORC_OK;
}

int oracle_viscous(const orc_grid *g, const orc_phys *ph, const real *u, real *out) {
    int rc = check_grid(g, ph);
    if (rc) return rc;
    if (!u || !out) return ORC_EINVAL;
    size_t n3 = npts(g);
    if (ph->mu_eff == 0.0) {
        memset(out, 0, 5 * n3 * sizeof(real));
        return ORC_OK;
    }
    /* G[d][v][p] */
    real *G = (real *)malloc(15 * n3 * sizeof(real));
    if (!G) return ORC_EINVAL;
    int err = 0;
#pragma omp parallel for collapse(2) reduction(min : err)
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                real Gp[3][5];
                int r = gvisc_at(g, ph, u, i, j, k, Gp);
                if (r < err) err = r;
                size_t p = lin(g, i, j, k);
                for (int d = 0; d < 3; ++d)
                    for (int v = 0; v < 5; ++v) G[((size_t)d * 5 + v) * n3 + p] = Gp[d][v];
            }
    if (err) {
        free(G);
        return err;
    }
#pragma omp parallel for collapse(2)
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                size_t p = lin(g, i, j, k);
                for (int v = 0; v < 5; ++v) {
                    real acc = 0.0;
                    for (int d = 0; d < 3; ++d) {
                        const real *Gd = G + ((size_t)d * 5 + v) * n3;
                        acc += central_d(Gd[shifted(g, i, j, k, d, -2)], Gd[shifted(g, i, j, k, d, -1)],
                                         Gd[shifted(g, i, j, k, d, 1)], Gd[shifted(g, i, j, k, d, 2)],
                                         spacing(g, d));
                    }
                    out[(size_t)v * n3 + p] = acc;
                }
            }
    free(G);
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* full right-hand side: du/dt = -(D_x f + D_y g + D_z h) + sum_d D_d G^v_d  */
/* ------------------------------------------------------------------------- */
int oracle_rhs(const orc_grid *g, const orc_phys *ph, const real *u, real *out) {
    int rc = check_grid(g, ph);
    if (rc) return rc;
    if (!u || !out) return ORC_EINVAL;
    size_t n3 = npts(g);
    real *tmp = (real *)malloc(5 * n3 * sizeof(real));
    if (!tmp) return ORC_EINVAL;
    rc = oracle_rhs_hyp_dir(g, ph, u, 0, out);
    for (int d = 1; d < 3 && !rc; ++d) {
        rc = oracle_rhs_hyp_dir(g, ph, u, d, tmp);
        if (!rc)
            for (size_t q = 0; q < 5 * n3; ++q) out[q] += tmp[q];
    }
    if (!rc && ph->mu_eff > 0.0) {
        rc = oracle_viscous(g, ph, u, tmp);
        if (!rc)
            for (size_t q = 0; q < 5 * n3; ++q) out[q] += tmp[q];
    }
    free(tmp);
    return rc;
}

#ifndef ORC_COMPLEX_STEP
int oracle_rhs_point(const orc_grid *g, const orc_phys *ph, const double *u, int i, int j, int k, double *out5) {
    int rc = check_grid(g, ph);
    if (rc) return rc;
    if (!u || !out5 || i < 0 || j < 0 || k < 0 || i >= g->nx || j >= g->ny || k >= g->nz) return ORC_EINVAL;
    double acc[5];
    for (int d = 0; d < 3; ++d) {
        int c[3] = {i, j, k};
        int n[3] = {g->nx, g->ny, g->nz};
        double Fp[5], Fm[5];
        rc = interface_at(g, ph, u, i, j, k, d, Fp);
        c[d] = wrapi(c[d] - 1, n[d]);
        if (!rc) rc = interface_at(g, ph, u, c[0], c[1], c[2], d, Fm);
        if (rc) return rc;
        double dx = spacing(g, d);
        for (int v = 0; v < 5; ++v) {
            double t = -(Fp[v] - Fm[v]) / dx;
            acc[v] = (d == 0) ? t : acc[v] + t;
        }
    }
    if (ph->mu_eff > 0.0) {
        double vis[5];
        for (int v = 0; v < 5; ++v) vis[v] = 0.0;
        /* G^v_d at the four neighbours along each direction d */
        for (int v = 0; v < 5; ++v) vis[v] = 0.0;
        double Gs[3][4][5];
        for (int d = 0; d < 3; ++d) {
            const int offs[4] = {-2, -1, 1, 2};
            for (int o = 0; o < 4; ++o) {
                int c[3] = {i, j, k};
                int n[3] = {g->nx, g->ny, g->nz};
                c[d] = wrapi(c[d] + offs[o], n[d]);
                double Gp[3][5];
                rc = gvisc_at(g, ph, u, c[0], c[1], c[2], Gp);
                if (rc) return rc;
                for (int v = 0; v < 5; ++v) Gs[d][o][v] = Gp[d][v];
            }
        }
        for (int v = 0; v < 5; ++v) {
            double a = 0.0;
            for (int d = 0; d < 3; ++d)
                a += central_d(Gs[d][0][v], Gs[d][1][v], Gs[d][2][v], Gs[d][3][v], spacing(g, d));
            vis[v] = a;
        }
        for (int v = 0; v < 5; ++v) acc[v] += vis[v];
    }
    for (int v = 0; v < 5; ++v) out5[v] = acc[v];
    return ORC_OK;
}
#endif

/* ------------------------------------------------------------------------- */
/* diagnostics: kinetic energy, enstrophy, means, max wave speed, bad points */
/* ------------------------------------------------------------------------- */
int oracle_diag(const orc_grid *g, const orc_phys *ph, const real *u, real *out) {
    int rc = check_grid(g, ph);
    if (rc) return rc;
    if (!u || !out) return ORC_EINVAL;
    size_t n3 = npts(g);
    real K = 0, Om = 0, mr = 0, mm[3] = {0, 0, 0}, me = 0, smax = 0;
    double bad = 0;
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                size_t p = lin(g, i, j, k);
                real s[5], vel[3], pr, T;
                load_state(u, n3, p, s);
                int r = primitives(s, ph->gamma, vel, &pr, &T);
                int finite = 1;
                for (int v = 0; v < 5; ++v) finite = finite && isfinite(ORC_RE(s[v]));
                if (r || !finite) {
                    bad += 1.0;
                    continue;
                }
                K += 0.5 * (s[1] * s[1] + s[2] * s[2] + s[3] * s[3]) / s[0];
                mr += s[0];
                mm[0] += s[1];
                mm[1] += s[2];
                mm[2] += s[3];
                me += s[4];
                real c = ORC_SQRT(ph->gamma * pr / s[0]);
                for (int d = 0; d < 3; ++d) {
                    real sp = ORC_ABS(vel[d]) + c;
                    if (ORC_RE(sp) > ORC_RE(smax)) smax = sp;
                }
                /* vorticity from the 4th-order central derivative */
                real dv[3][3]; /* dv[a][b] = d v_a / d x_b */
                int ok = 1;
                for (int b = 0; b < 3 && ok; ++b) {
                    real w[4][4];
                    const int offs[4] = {-2, -1, 1, 2};
                    for (int o = 0; o < 4; ++o)
                        if (vel_temp_at(u, n3, shifted(g, i, j, k, b, offs[o]), ph->gamma, w[o])) ok = 0;
                    double h = spacing(g, b);
                    for (int a = 0; a < 3; ++a) dv[a][b] = central_d(w[0][a], w[1][a], w[2][a], w[3][a], h);
                }
                if (!ok) continue; /* a neighbour is bad: counted at that neighbour */
                real ox = dv[2][1] - dv[1][2];
                real oy = dv[0][2] - dv[2][0];
                real oz = dv[1][0] - dv[0][1];
                Om += 0.5 * (ox * ox + oy * oy + oz * oz);
            }
    double inv = 1.0 / (double)n3;
    out[0] = K * inv;
    out[1] = Om * inv;
    out[2] = mr * inv;
    out[3] = mm[0] * inv;
    out[4] = mm[1] * inv;
    out[5] = mm[2] * inv;
    out[6] = me * inv;
    out[7] = smax;
    out[8] = bad;
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* classical RK4                                                             */
/* ------------------------------------------------------------------------- */
int oracle_rk4(const orc_grid *g, const orc_phys *ph, real *u, double dt, int nsteps, real *diag) {
    int rc = check_grid(g, ph);
    if (rc) return rc;
    if (!u || !(dt > 0.0) || nsteps < 0) return ORC_EINVAL;
    size_t n5 = 5 * npts(g);
    real *k1 = (real *)malloc(n5 * sizeof(real));
    real *k2 = (real *)malloc(n5 * sizeof(real));
    real *k3 = (real *)malloc(n5 * sizeof(real));
    real *k4 = (real *)malloc(n5 * sizeof(real));
    real *U = (real *)malloc(n5 * sizeof(real));
    if (!k1 || !k2 || !k3 || !k4 || !U) {
        free(k1), free(k2), free(k3), free(k4), free(U);
        return ORC_EINVAL;
    }
    for (int n = 0; n < nsteps && !rc; ++n) {
        rc = oracle_rhs(g, ph, u, k1);
        if (rc) break;
        for (size_t q = 0; q < n5; ++q) U[q] = u[q] + 0.5 * dt * k1[q];
        rc = oracle_rhs(g, ph, U, k2);
        if (rc) break;
        for (size_t q = 0; q < n5; ++q) U[q] = u[q] + 0.5 * dt * k2[q];
        rc = oracle_rhs(g, ph, U, k3);
        if (rc) break;
        for (size_t q = 0; q < n5; ++q) U[q] = u[q] + dt * k3[q];
        rc = oracle_rhs(g, ph, U, k4);
        if (rc) break;
        for (size_t q = 0; q < n5; ++q) u[q] = u[q] + (dt / 6.0) * (k1[q] + 2.0 * k2[q] + 2.0 * k3[q] + k4[q]);
        if (diag) {
            rc = oracle_diag(g, ph, u, diag + (size_t)n * ORC_NDIAG);
            if (!rc && ORC_RE(diag[(size_t)n * ORC_NDIAG + 8]) > 0) rc = ORC_ENONFINITE;
        }
    }
    free(k1), free(k2), free(k3), free(k4), free(U);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* third-order TVD Runge-Kutta (Shu-Osher), the paper's production scheme    */
/* ------------------------------------------------------------------------- */
int oracle_tvdrk3(const orc_grid *g, const orc_phys *ph, real *u, double dt, int nsteps, real *diag) {
    int rc = check_grid(g, ph);
    if (rc) return rc;
    if (!u || !(dt > 0.0) || nsteps < 0) return ORC_EINVAL;
    size_t n5 = 5 * npts(g);
    real *k = (real *)malloc(n5 * sizeof(real));
    real *U1 = (real *)malloc(n5 * sizeof(real));
    real *U2 = (real *)malloc(n5 * sizeof(real));
    if (!k || !U1 || !U2) {
        free(k), free(U1), free(U2);
        return ORC_EINVAL;
    }
    for (int n = 0; n < nsteps && !rc; ++n) {
        /* U1 = u + dt R(u) */
        rc = oracle_rhs(g, ph, u, k);
        if (rc) break;
        for (size_t q = 0; q < n5; ++q) U1[q] = u[q] + dt * k[q];
        /* U2 = 3/4 u + 1/4 (U1 + dt R(U1)) */
        rc = oracle_rhs(g, ph, U1, k);
        if (rc) break;
        for (size_t q = 0; q < n5; ++q) U2[q] = 0.75 * u[q] + 0.25 * (U1[q] + dt * k[q]);
        /* u^{n+1} = 1/3 u + 2/3 (U2 + dt R(U2)) */
        rc = oracle_rhs(g, ph, U2, k);
        if (rc) break;
        for (size_t q = 0; q < n5; ++q) u[q] = (1.0 / 3.0) * u[q] + (2.0 / 3.0) * (U2[q] + dt * k[q]);
        if (diag) {
            rc = oracle_diag(g, ph, u, diag + (size_t)n * ORC_NDIAG);
            if (!rc && ORC_RE(diag[(size_t)n * ORC_NDIAG + 8]) > 0) rc = ORC_ENONFINITE;
        }
    }
    free(k), free(U1), free(U2);
    return rc;
}

#ifndef ORC_COMPLEX_STEP
int oracle_init_state(const orc_grid *g, double gamma, const double *rho, const double *vel, const double *p,
                      double *u) {
    int rc = check_grid(g, NULL);
    if (rc) return rc;
    if (!rho || !vel || !p || !u || !(gamma > 1.0)) return ORC_EINVAL;
    size_t n3 = npts(g);
    for (size_t q = 0; q < n3; ++q) {
        double r = rho[q], a = vel[q], b = vel[n3 + q], c = vel[2 * n3 + q];
        if (!(r > 0.0) || !(p[q] > 0.0)) return ORC_ENONPHYSICAL;
        u[q] = r;
        u[n3 + q] = r * a;
        u[2 * n3 + q] = r * b;
        u[3 * n3 + q] = r * c;
        u[4 * n3 + q] = p[q] / (gamma - 1.0) + 0.5 * r * (a * a + b * b + c * c);
    }
    return ORC_OK;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
#endif
