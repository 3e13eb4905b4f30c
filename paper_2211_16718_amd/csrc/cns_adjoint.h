// cns_adjoint.h -- launchers of the reverse-mode kernels (cns_adjoint.hip), FP64, one box,
// and the stage-combination epilogue of the reverse sweeps.
#pragma once

#include "cns_internal.h"

namespace cns {

// What the reverse sweep does with a finished stage adjoint Ub at each point, done by
// the last kernel of the product when the box is viscous (else by a separate launch).
// The reverse RK4 stages:
//   S = Ub (s_first) or S += Ub, when S is set;
//   kb = a ub + b Ub, when kb is set and ubf is not (the next product's seed: a buffer
//   other than the seed rbar of this product, which its last kernel still reads around
//   each point);
//   ubf = ubf + (S + Ub), when ubf is set (the step's last stage; S is read, not written),
//   and then kb = a ubf, when kb is set as well (the seed of the next step's first product).
// The reverse TVD-RK3 stages, when ld is set (instead of the above):
//   ld = pa la + pb lb + pc lc + Ub (the terms whose array is set), then lkb = ls ld
//   when lkb is set (the next seed, again a buffer other than this product's rbar).
// Ub itself is stored only when store_ub is set.
struct AdjEpilogue {
    double *S = nullptr;
    int s_first = 0;
    double *kb = nullptr;
    const double *ub = nullptr;
    double a = 0.0, b = 0.0;
    double *ubf = nullptr;
    const double *la = nullptr, *lb = nullptr, *lc = nullptr;
    double pa = 0.0, pb = 0.0, pc = 0.0, ls = 0.0;
    double *ld = nullptr, *lkb = nullptr;
    int store_ub = 1;
};

// the combination at element o of a finished stage adjoint f
__device__ __forceinline__ void adj_epilogue_at(const AdjEpilogue &ep, size_t o, double f) {
    if (ep.ld) {
        double t = f;
        if (ep.la) t += ep.pa * ep.la[o];
        if (ep.lb) t += ep.pb * ep.lb[o];
        if (ep.lc) t += ep.pc * ep.lc[o];
        ep.ld[o] = t;
        if (ep.lkb) ep.lkb[o] = ep.ls * t;
    } else if (ep.ubf) {
        const double tt = ep.S[o] + f, nu = ep.ubf[o] + tt;
        ep.ubf[o] = nu;
        if (ep.kb) ep.kb[o] = ep.a * nu;
    } else {
        if (ep.S) ep.S[o] = ep.s_first ? f : ep.S[o] + f;
        if (ep.kb) ep.kb[o] = __fma_rn(ep.a, ep.ub[o], ep.b * f);
    }
}

// adjoint of the full RHS at u: ubar = (dR/du)^T rbar
void adj_rhs_vjp(const BoxDesc &b, int weights, hipStream_t s, const double *u, const double *rbar, double *ubar);
void adj_lincomb(size_t n, double a, const double *x, double b, const double *y, double *out, hipStream_t s);
void adj_copy(size_t n, const double *x, double *out, hipStream_t s);
void adj_ke_seed(size_t n3, const double *u, double *ubar, hipStream_t s);
void adj_ic_vjp(size_t n3, const double *rho, const double *vel, const double *ubar, double *vbar, hipStream_t s);

// adj_rhs_vjp followed by the epilogue
void adj_rhs_vjp_epi(const BoxDesc &b, int weights, hipStream_t s, const double *u, const double *rbar, double *ubar,
                     const AdjEpilogue &epi);

}  // namespace cns
