// cns_adjoint.h -- the stage-combination epilogue of the reverse RK4 sweep (cns_adjoint.hip).
#pragma once

#include "cns_internal.h"

namespace cns {

// What the reverse RK4 sweep does with a finished stage adjoint Ub at each point, done
// by the last kernel of the product when the box is viscous (else by a separate launch):
//   S = Ub (s_first) or S += Ub, when S is set;
//   kb = a ub + b Ub, when kb is set and ubf is not (the next product's seed: a buffer
//   other than the seed rbar of this product, which its last kernel still reads around
//   each point);
//   ubf = ubf + (S + Ub), when ubf is set (the step's last stage; S is read, not written),
//   and then kb = a ubf, when kb is set as well (the seed of the next step's first product);
//   Ub itself is stored only when store_ub is set.
struct AdjEpilogue {
    double *S = nullptr;
    int s_first = 0;
    double *kb = nullptr;
    const double *ub = nullptr;
    double a = 0.0, b = 0.0;
    double *ubf = nullptr;
    int store_ub = 1;
};

// adj_rhs_vjp followed by the epilogue
void adj_rhs_vjp_epi(const BoxDesc &b, int weights, hipStream_t s, const double *u, const double *rbar, double *ubar,
                     const AdjEpilogue &epi);

}  // namespace cns
