/*
 * cns_oracle_cs.c -- complex-step derivatives of the oracle (TEST INFRASTRUCTURE ONLY).
 *
 * The oracle's arithmetic (cns_oracle.c) is compiled a second time here with the
 * scalar type double complex.  For a real analytic map F and a real direction d,
 *     F(u + i h d) = F(u) + i h F'(u) d + O(h^2),
 * so Im F(u + i h d) / h is the directional derivative F'(u) d with an error of
 * order h^2 and no subtractive cancellation (Squire and Trapp, SIAM Review 40, 1998;
 * Martins, Sturdza and Alonso, ACM TOMS 29, 2003).  With h = 1e-20 the result is the
 * derivative to rounding.  Every operation of the method is analytic away from its
 * branch points: sqrt is the principal complex root, and the branches of the method
 * (|x| in the Harten fix and in WENO-Z, the Harten threshold, the validity tests)
 * are decided on the real part, with |x| = x for Re x >= 0 and -x otherwise, which
 * is the derivative of |x| wherever it exists.
 *
 * These derivatives pin the adjoints: <w, R'(u) d> must equal <R'(u)^T w, d>, and the
 * derivative of the final kinetic energy along d must equal <dK/du0, d>.  On small grids
 * oracle_adjoint_rk4 forms the whole gradient dK/du0 by its definition, one complex-step
 * derivative per component of u0.
 */
#include "cns_oracle.h"

#include <complex.h>
#include <stdlib.h>

static double complex cs_abs(double complex x) { return creal(x) < 0.0 ? -x : x; }

#define ORC_COMPLEX_STEP 1
#define ORC_REAL double complex
#define ORC_SQRT csqrt
#define ORC_ABS cs_abs
#define ORC_RE(x) creal(x)
/* the complex instantiation gets names of its own */
#define oracle_weno5 orc_cs_weno5
#define oracle_weno5z orc_cs_weno5z
#define oracle_weno_map orc_cs_weno_map
#define oracle_weno5m orc_cs_weno5m
#define oracle_flux orc_cs_flux
#define oracle_roe_eigensystem orc_cs_roe_eigensystem
#define oracle_harten orc_cs_harten
#define oracle_interface_flux orc_cs_interface_flux
#define oracle_rhs_hyp_dir orc_cs_rhs_hyp_dir
#define oracle_viscous orc_cs_viscous
#define oracle_rhs orc_cs_rhs
#define oracle_diag orc_cs_diag
#define oracle_rk4 orc_cs_rk4
#define oracle_tvdrk3 orc_cs_tvdrk3
#include "cns_oracle.c"

/* u + i h d in a new complex array */
static double complex *perturbed(const double *u, const double *d, double h, size_t n) {
    double complex *z = (double complex *)malloc(n * sizeof(double complex));
    if (!z) return NULL;
    for (size_t q = 0; q < n; ++q) z[q] = u[q] + I * (h * d[q]);
    return z;
}

int oracle_cs_rhs_jvp(const orc_grid *g, const orc_phys *ph, const double *u, const double *d, double h,
                      double *jvp, double *value) {
    if (!g || !u || !d || !jvp || !(h > 0.0)) return ORC_EINVAL;
    size_t n5 = 5 * npts(g);
    double complex *z = perturbed(u, d, h, n5);
    double complex *r = (double complex *)malloc(n5 * sizeof(double complex));
    int rc = (z && r) ? orc_cs_rhs(g, ph, z, r) : ORC_EINVAL;
    if (!rc)
        for (size_t q = 0; q < n5; ++q) {
            jvp[q] = cimag(r[q]) / h;
            if (value) value[q] = creal(r[q]);
        }
    free(z);
    free(r);
    return rc;
}

int oracle_cs_step_jvp(const orc_grid *g, const orc_phys *ph, int scheme, const double *u0, const double *d,
                       double dt, int nsteps, double h, double *du, double *dK, double *K) {
    if (!g || !u0 || !d || !(h > 0.0) || nsteps < 0 || (scheme != 0 && scheme != 1)) return ORC_EINVAL;
    size_t n5 = 5 * npts(g);
    double complex *z = perturbed(u0, d, h, n5);
    double complex diag[ORC_NDIAG];
    if (!z) return ORC_EINVAL;
    int rc = scheme == 0 ? orc_cs_rk4(g, ph, z, dt, nsteps, NULL) : orc_cs_tvdrk3(g, ph, z, dt, nsteps, NULL);
    if (!rc) rc = orc_cs_diag(g, ph, z, diag);
    if (!rc) {
        if (du)
            for (size_t q = 0; q < n5; ++q) du[q] = cimag(z[q]) / h;
        if (dK) *dK = cimag(diag[0]) / h;
        if (K) *K = creal(diag[0]);
    }
    free(z);
    return rc;
}

/* The gradient of the final mean kinetic energy with respect to every component of u0,
 * each entry the complex-step derivative along that unit vector: 5 N^3 complex runs of
 * nsteps steps (small grids only).  The runs are independent; OpenMP shares them out, and
 * the loops inside a run stay serial (nested regions are inactive). */
int oracle_adjoint_rk4(const orc_grid *g, const orc_phys *ph, int scheme, const double *u0, double dt, int nsteps,
                       double h, double *grad, double *K) {
    if (!g || !u0 || !grad || !(h > 0.0) || nsteps < 0 || (scheme != 0 && scheme != 1)) return ORC_EINVAL;
    const long n5 = (long)(5 * npts(g));
    int rc = 0;
#pragma omp parallel for schedule(dynamic, 8) reduction(| : rc)
    for (long q = 0; q < n5; ++q) {
        double complex *z = (double complex *)malloc((size_t)n5 * sizeof(double complex));
        double complex diag[ORC_NDIAG];
        int r = z ? 0 : ORC_EINVAL;
        if (!r) {
            for (long i = 0; i < n5; ++i) z[i] = u0[i];
            z[q] += I * h;
            r = scheme == 0 ? orc_cs_rk4(g, ph, z, dt, nsteps, NULL) : orc_cs_tvdrk3(g, ph, z, dt, nsteps, NULL);
        }
        if (!r) r = orc_cs_diag(g, ph, z, diag);
        if (!r) {
            grad[q] = cimag(diag[0]) / h;
            if (K && q == 0) *K = creal(diag[0]);
        }
        free(z);
        rc |= r;
    }
    return rc;
}
