/*
 * cns_oracle.h -- plain FP64 CPU oracle for the WENO5 / Roe / 4th-order-central
 * discretisation of the 3-D compressible Navier-Stokes equations on a triply
 * periodic grid, advanced by classical RK4.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline of the benchmark may load this library.  It shares no source with
 * the HIP library: the two are written separately from the paper's equations.
 *
 * Paper: "GPU-accelerated DNS of compressible turbulent flows" (arXiv 2211.16718),
 *   Sec. 2.1 (governing equations: conserved state, Euler fluxes, equation of
 *   state, viscous stress and heat flux) and Sec. 2.2 (conservative finite
 *   differences, Roe flux with Harten's entropy fix, component-wise WENO5 with
 *   Jiang-Shu weights, 4th-order central viscous derivatives, RK4).
 *
 * Layout: a state u is SoA, u[v][k][j][i] with v = 0..4 the conserved variable
 * (rho, rho*u, rho*v, rho*w, e) and i (x) fastest.  Every array is host memory
 * owned by the caller.  Every function returns 0 on success or a negative
 * ORC_E* code and leaves outputs unspecified on error.
 */
#ifndef CNS_ORACLE_H
#define CNS_ORACLE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENONFINITE (-3)
#define ORC_ENONPHYSICAL (-4)

#define ORC_NDIAG 9 /* K, Omega, <rho>, <rho u>, <rho v>, <rho w>, <e>, max(|v_d|+c), bad-point count */

typedef struct {
    int nx, ny, nz;
    double lx, ly, lz;
} orc_grid;

typedef struct {
    double gamma;        /* ratio of specific heats (paper: 1.4) */
    double prandtl;      /* Prandtl number (paper: 0.72) */
    double mu_eff;       /* mu * M_inf / Re_inf; 0 disables the viscous terms */
    double weno_eps;     /* epsilon of the WENO weights (paper: 1e-6) */
    double harten_delta; /* Harten entropy-fix threshold; 0 gives the plain |lambda| */
    int weno_weights;    /* ORC_WENO_JS (the paper's Jiang-Shu weights), ORC_WENO_Z or ORC_WENO_M */
} orc_phys;

#define ORC_WENO_JS 0
#define ORC_WENO_Z 1
#define ORC_WENO_M 2

/* ---- building blocks (exported so tests can pin each one) ---- */

/* WENO5 left-biased interface value at j+1/2 from the five values
 * (a,b,c,d,e) = (f_{j-2}, f_{j-1}, f_j, f_{j+1}, f_{j+2}).  parts (may be NULL)
 * receives beta1..3, omega1..3, fhat1..3. */
double oracle_weno5(double a, double b, double c, double d, double e, double eps, double *parts);

/* Same with the WENO-Z weights of Borges et al. (2008), exponent 2:
 * alpha_k = c_k (1 + (|beta1 - beta3| / (eps + beta_k))^2). */
double oracle_weno5z(double a, double b, double c, double d, double e, double eps, double *parts);

/* Same with the mapped weights of Henrick et al. (2005): the Jiang-Shu weights w_k
 * mapped by g_k (oracle_weno_map with d_k = 1/10, 6/10, 3/10) and renormalised. */
double oracle_weno5m(double a, double b, double c, double d, double e, double eps, double *parts);
/* The mapping g(w) = w (d + d^2 - 3 d w + w^2) / (d^2 + w (1 - 2 d)). */
double oracle_weno_map(double w, double d);

/* Euler flux along dir (0=x,1=y,2=z) of the conserved state u[5]. */
void oracle_flux(const double *u, int dir, double gamma, double *f);

/* Roe-averaged eigensystem between cell states uL, uR along dir: X (5x5, columns
 * = right eigenvectors, row-major X[r*5+c]), Xinv, eigenvalues lam[5]. */
int oracle_roe_eigensystem(const double *uL, const double *uR, int dir, double gamma,
                           double *X, double *Xinv, double *lam);

/* Harten's entropy-fixed |lambda|. */
double oracle_harten(double lam, double delta);

/* Interface flux at j+1/2 from the six cell states s[m*5+v], m = 0..5 for
 * points j-2..j+3. */
int oracle_interface_flux(const double *s, int dir, const orc_phys *ph, double *F);

/* ---- grid operators ---- */
/* out = -(F_{j+1/2} - F_{j-1/2}) / dx_dir : the hyperbolic term along one direction. */
int oracle_rhs_hyp_dir(const orc_grid *g, const orc_phys *ph, const double *u, int dir, double *out);
/* out = sum_d D_d G^v_d : the viscous and heat-flux terms. */
int oracle_viscous(const orc_grid *g, const orc_phys *ph, const double *u, double *out);
/* out = full right-hand side du/dt. */
int oracle_rhs(const orc_grid *g, const orc_phys *ph, const double *u, double *out);
/* RHS at the single point (i,j,k); bitwise equal to oracle_rhs there. */
int oracle_rhs_point(const orc_grid *g, const orc_phys *ph, const double *u, int i, int j, int k,
                     double *out5);
/* nsteps classical RK4 steps in place; diag (may be NULL) receives
 * [nsteps][ORC_NDIAG] diagnostics of the state after each step. */
int oracle_rk4(const orc_grid *g, const orc_phys *ph, double *u, double dt, int nsteps, double *diag);
/* nsteps third-order TVD Runge-Kutta (Shu-Osher) steps in place; diag as oracle_rk4. */
int oracle_tvdrk3(const orc_grid *g, const orc_phys *ph, double *u, double dt, int nsteps, double *diag);
/* diagnostics of u: see ORC_NDIAG. */
int oracle_diag(const orc_grid *g, const orc_phys *ph, const double *u, double *out);
/* conserved state from primitives rho[N3], vel[3][N3], p[N3]. */
int oracle_init_state(const orc_grid *g, double gamma, const double *rho, const double *vel,
                      const double *p, double *u);
/* threads used by the OpenMP loops (1 if built without OpenMP). */
int oracle_num_threads(void);

/* ---- complex-step derivatives (cns_oracle_cs.c) ---- */
/* jvp = R'(u) d, the derivative of the right-hand side at u along d, as
 * Im R(u + i h d) / h (h > 0, e.g. 1e-20); value (may be NULL) receives Re R(u + i h d). */
int oracle_cs_rhs_jvp(const orc_grid *g, const orc_phys *ph, const double *u, const double *d, double h,
                      double *jvp, double *value);
/* Derivatives along d of nsteps time steps from u0 (scheme 0 = classical RK4, 1 =
 * TVD-RK3): du (may be NULL) = d u_N / d u0 . d; dK (may be NULL) = the derivative of
 * the final mean kinetic energy K(u_N); K (may be NULL) = K(u_N) itself. */
int oracle_cs_step_jvp(const orc_grid *g, const orc_phys *ph, int scheme, const double *u0, const double *d,
                       double dt, int nsteps, double h, double *du, double *dK, double *K);
/* The gradient dK/du0 of the final mean kinetic energy after nsteps steps (scheme 0 =
 * RK4, 1 = TVD-RK3) from u0, every component by its own complex-step derivative (5 N^3
 * complex runs: small grids only); K (may be NULL) = K(u_N). */
int oracle_adjoint_rk4(const orc_grid *g, const orc_phys *ph, int scheme, const double *u0, double dt, int nsteps,
                       double h, double *grad, double *K);

#ifdef __cplusplus
}
#endif
#endif
