// cns_device.h -- device arithmetic of the WENO5-Roe / central-viscous discretisation
// for gfx950.  Templated on the arithmetic type T (double, or float in the mixed form)
// and on B, the type of the WENO smoothness-indicator sums (always double).
//
// Formulation choices (same operator as Sec. 2.2 of the paper, different
// arithmetic order):
//  * WENO5: the left-biased value at j+1/2 reads q_{j-2..j+2}, the right-biased one
//    is its mirror image and reads q_{j-1..j+3}.  The two share two of their three
//    candidate interpolants and two of their four second differences, so one
//    interface evaluates 4 candidates and 4 second differences instead of 6 and 6.
//  * Nonlinear weights: alpha_k = c_k / d_k with d_k = (eps + beta_k)^2 are scaled by
//    d_1 d_2 d_3, so omega needs one division per reconstruction instead of four.
//  * The sweeps carry 6 x the reconstructed values and 4 x the indicators (with 4 eps),
//    which removes the constant factors from the inner arithmetic; the interface flux
//    divides once by 12 at the end.
//  * Roe dissipation |A| (u^R - u^L) is evaluated with wave strengths (projections
//    on the left eigenvectors, written out) instead of explicit 5x5 matrices;
//    |A| = X |Lambda| X^-1 is basis independent so the operator is the same.
#pragma once
#include <hip/hip_runtime.h>

#include "cns.h"

namespace cns {

struct PhysT {
    double gamma, prandtl, mu_eff, eps, delta;
};

// Reciprocal: the hardware estimate r (relative error below 2^-24 on gfx950, measured)
// refined once to third order, 1/b = r / (1 - e) ~ r (1 + e + e^2) with e = 1 - b r
// (truncation e^3 < 2^-72), three instructions against four for two Newton-Raphson
// steps; in FP32 one Newton-Raphson step r <- r + r e.  Within an ulp or two of the
// IEEE division, at about half its instructions.
__device__ __forceinline__ double rcp(double b) {
    const double r = __builtin_amdgcn_rcp(b);
    const double e = fma(-b, r, 1.0);
    return fma(r, fma(e, e, e), r);
}
__device__ __forceinline__ float rcp(float b) {
    float r = __builtin_amdgcn_rcpf(b);
    float e = fmaf(-b, r, 1.0f);
    return fmaf(r, e, r);
}

// Reciprocal square root: the hardware estimate y (relative error below 2^-24) refined
// once to third order, x^-1/2 = y (1 - e)^-1/2 ~ y (1 + e/2 + 3 e^2 / 8) with
// e = 1 - x y^2 (truncation 5 e^3 / 16); in FP32 one Newton-Raphson step
// y <- y + y e / 2.
__device__ __forceinline__ double rsq(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y, y, 1.0);
    return fma(y * e, fma(e, 0.375, 0.5), y);
}
__device__ __forceinline__ float rsq(float x) {
    float y = __builtin_amdgcn_rsqf(x);
    float r = fmaf(-x * y, y, 1.0f);
    return fmaf(0.5f * y, r, y);
}

template <typename T>
__device__ __forceinline__ T harten_abs(T lam, T delta) {
    // |lam| if |lam| >= delta, else (lam^2 + delta^2) / (2 delta)  (Harten's entropy fix)
    T a = fabs(lam);
    return (a >= delta) ? a : (lam * lam + delta * delta) / (T(2) * delta);
}
// the same with h = 1 / (2 delta) given (no division inside the flux loop)
template <typename T>
__device__ __forceinline__ T harten_abs(T lam, T delta, T h) {
    T a = fabs(lam);
    return (a >= delta) ? a : (lam * lam + delta * delta) * h;
}

// ---------------------------------------------------------------------------
// WENO5, left- and right-biased values at j+1/2 from q_{j-2} .. q_{j+3}
// ---------------------------------------------------------------------------
// Nonlinear weights of one reconstruction from its three indicators b1..b3 (in B) and
// candidates c1..c3 (any common scale of b and eps, and of the c, passes through).
// WW selects the weights: CNS_WENO_JS, Jiang-Shu alpha_k = c_k / s_k^2 with
// s_k = eps + b_k; CNS_WENO_Z, the WENO-Z weights of Borges et al. (2008),
// alpha_k = c_k (1 + (tau5/s_k)^2) with tau5 = |b1 - b3|; CNS_WENO_M, the mapped
// weights of Henrick et al. (2005), the Jiang-Shu weights w_k passed through
// g_k(w) = w (c_k + c_k^2 - 3 c_k w + w^2) / (c_k^2 + w (1 - 2 c_k)) and renormalised.
// The alpha are scaled by s_1^2 s_2^2 s_3^2, the mapped values by the product of the
// three denominators, so one reciprocal serves the three weights of each
// normalisation.  The Z and mapped weights are formed in B (FP64) and normalised
// before any narrowing.
template <typename T, typename B, int WW>
__device__ __forceinline__ T weno5_combine(B b1, B b2, B b3, T eps, T c1, T c2, T c3) {
    if constexpr (WW == CNS_WENO_JS && sizeof(T) == sizeof(B)) {
        // 10 alpha_k s1^2 s2^2 s3^2 = (d2 d3, 6 d1 d3, 3 d1 d2) with d_k = s_k^2
        T s1 = eps + T(b1), s2 = eps + T(b2), s3 = eps + T(b3);
        T d1 = s1 * s1, d2 = s2 * s2, d3 = s3 * s3;
        T a1 = d2 * d3, a2 = d1 * d3, a3 = d1 * d2;
        T num = a1 * c1 + a2 * (T(6) * c2) + a3 * (T(3) * c3);
        return num * rcp(a1 + T(6) * a2 + T(3) * a3);
    } else if constexpr (WW == CNS_WENO_JS) {
        // FP32 (the mixed form): products of four (eps + beta) factors would leave the
        // FP32 range at jumps of about 3e4 in the reconstructed value.  The s_k are first
        // scaled by the power of two of the smallest (exact), which puts t_k in [0.5, inf),
        // and capped at 2^31: a stencil whose t is capped has a weight below 2^-62 of the
        // smoothest one's, where the cap changes its contribution by less than the FP32
        // rounding of the smooth candidates (unless a jump exceeds the neighbouring values
        // by 1e11).  Then every product lies in [2^-4, 2^127), and the weights are
        // normalised before they multiply the candidates.
        T s1 = eps + T(b1), s2 = eps + T(b2), s3 = eps + T(b3);
        const int e = -__builtin_amdgcn_frexp_expf(fminf(s1, fminf(s2, s3)));
        const T cap = T(2147483648.0);
        T t1 = fminf(__builtin_amdgcn_ldexpf(s1, e), cap), t2 = fminf(__builtin_amdgcn_ldexpf(s2, e), cap),
          t3 = fminf(__builtin_amdgcn_ldexpf(s3, e), cap);
        T d1 = t1 * t1, d2 = t2 * t2, d3 = t3 * t3;
        T a1 = d2 * d3, a2 = T(6) * (d1 * d3), a3 = T(3) * (d1 * d2);
        T ir = rcp(a1 + a2 + a3);
        return (a1 * ir) * c1 + (a2 * ir) * c2 + (a3 * ir) * c3;
    } else if constexpr (WW == CNS_WENO_Z) {
        const B e = B(eps);
        B t = fabs(b1 - b3);
        B t2 = t * t;
        B s1 = e + b1, s2 = e + b2, s3 = e + b3;
        B d1 = s1 * s1, d2 = s2 * s2, d3 = s3 * s3;
        B a1 = B(0.1) * (d1 + t2) * (d2 * d3), a2 = B(0.6) * (d2 + t2) * (d1 * d3), a3 = B(0.3) * (d3 + t2) * (d1 * d2);
        if constexpr (sizeof(T) == sizeof(B)) {
            return (a1 * c1 + a2 * c2 + a3 * c3) * rcp(a1 + a2 + a3);
        } else {
            B ia = rcp(a1 + a2 + a3);
            return T(a1 * ia) * c1 + T(a2 * ia) * c2 + T(a3 * ia) * c3;
        }
    } else {
        static_assert(WW == CNS_WENO_M, "unknown WENO weights");
        const B e = B(eps);
        B s1 = e + b1, s2 = e + b2, s3 = e + b3;
        B d1 = s1 * s1, d2 = s2 * s2, d3 = s3 * s3;
        B a1 = B(0.1) * (d2 * d3), a2 = B(0.6) * (d1 * d3), a3 = B(0.3) * (d1 * d2);
        B ia = rcp(a1 + a2 + a3);
        B w1 = a1 * ia, w2 = a2 * ia, w3 = a3 * ia;  // Jiang-Shu weights
        // g_k = N_k / D_k with c = 1/10, 6/10, 3/10
        B N1 = w1 * (B(0.1) + B(0.1) * B(0.1) - B(0.3) * w1 + w1 * w1), D1 = B(0.1) * B(0.1) + w1 * B(0.8);
        B N2 = w2 * (B(0.6) + B(0.6) * B(0.6) - B(1.8) * w2 + w2 * w2), D2 = B(0.6) * B(0.6) + w2 * B(-0.2);
        B N3 = w3 * (B(0.3) + B(0.3) * B(0.3) - B(0.9) * w3 + w3 * w3), D3 = B(0.3) * B(0.3) + w3 * B(0.4);
        B g1 = N1 * (D2 * D3), g2 = N2 * (D1 * D3), g3 = N3 * (D1 * D2);
        B ig = rcp(g1 + g2 + g3);
        if constexpr (sizeof(T) == sizeof(B)) {
            return (g1 * c1 + g2 * c2 + g3 * c3) * ig;
        } else {
            return T(g1 * ig) * c1 + T(g2 * ig) * c2 + T(g3 * ig) * c3;
        }
    }
}

// The Jiang-Shu weighted sum of one reconstruction as numerator and denominator
// (the weights' common scale s_1^2 s_2^2 s_3^2 divided out by the caller): 10 alpha_k
// s1^2 s2^2 s3^2 = (d2 d3, 6 d1 d3, 3 d1 d2) with d_k = s_k^2, s_k = eps + beta_k (in
// any common scale).
template <typename T>
__device__ __forceinline__ void weno5_js_terms(T s1, T s2, T s3, T c1, T c2, T c3, T &num, T &den) {
    T d1 = s1 * s1, d2 = s2 * s2, d3 = s3 * s3;
    T a1 = d2 * d3, a2 = d1 * d3, a3 = d1 * d2;
    num = a1 * c1 + a2 * (T(6) * c2) + a3 * (T(3) * c3);
    den = a1 + T(6) * a2 + T(3) * a3;
}

// Six times the left- and right-biased values, from four times the Jiang-Shu
// indicators: with eps4 = 4 eps every alpha_k scales by the same 1/16, so the weights
// are those of the plain form; dropping the 1/6 of the candidates and the 13/12, 1/4 of
// the indicators saves a multiplication per candidate and per indicator.
template <typename T, typename B, int WW = CNS_WENO_JS>
__device__ __forceinline__ void weno5_lr6(T m2, T m1, T c0, T p1, T p2, T p3, T eps4, T &L6, T &R6) {
    // 4 x Jiang-Shu smoothness indicators, (13/3) D^2 + E^2, accumulated in B, from the
    // first differences g_i = q_{i+1} - q_i of the stencil (q = m2, m1, c0, p1, p2, p3):
    // the second differences D and the one-sided E are short combinations of them
    const B k = B(13) / B(3);
    const B bm2 = B(m2), bm1 = B(m1), bc0 = B(c0), bp1 = B(p1), bp2 = B(p2), bp3 = B(p3);
    const B g0 = bm1 - bm2, g1 = bc0 - bm1, g2 = bp1 - bc0, g3 = bp2 - bp1, g4 = bp3 - bp2;
    B da = g1 - g0;  // second differences centred at j-1, j, j+1, j+2
    B db = g2 - g1;
    B dc = g3 - g2;
    B dd = g4 - g3;
    // the one-sided terms only enter squared, so each is formed with whichever sign
    // keeps it one fused multiply-add
    B ea = B(3) * g1 - g0;  // m2 - 4 m1 + 3 c0
    B eb = g1 + g2;         // -(m1 - p1)
    B ec = B(3) * g2 - g3;  // -(3 c0 - 4 p1 + p2)
    B fa = B(3) * g3 - g4;  // -(p3 - 4 p2 + 3 p1)
    B fb = g2 + g3;         // p2 - c0
    B fc = B(3) * g2 - g1;  // 3 p1 - 4 c0 + m1
    // third-order candidates (times 6); the mirror reconstruction reuses L2 and L3.  In
    // FP64 from the same first differences (L1 = 6 c0 + 5 g1 - 2 g0, L2 = 6 c0 + g1 +
    // 2 g2, L3 = 6 c0 + 4 g2 - g3, R1 = 6 p1 - 5 g3 + 2 g4), in FP32 from the points.
    T L1, L2, L3, R1;
    if constexpr (sizeof(T) == sizeof(B)) {
        // 6 c0 enters last, by an addition: as the accumulator of a chain of fused
        // multiply-adds it would be copied for each of the three
        const T c6 = T(6) * c0;
        L1 = (T(5) * g1 - T(2) * g0) + c6;
        L2 = (g1 + T(2) * g2) + c6;
        L3 = (T(4) * g2 - g3) + c6;
        R1 = T(6) * p1 - T(5) * g3 + T(2) * g4;
    } else {
        L1 = T(2) * m2 - T(7) * m1 + T(11) * c0;
        L2 = -m1 + T(5) * c0 + T(2) * p1;
        L3 = T(2) * c0 + T(5) * p1 - p2;
        R1 = T(2) * p3 - T(7) * p2 + T(11) * p1;
    }
    if constexpr (WW == CNS_WENO_JS && sizeof(T) == sizeof(B)) {
        // FP64 Jiang-Shu.  eps4 enters each sum before the E^2 term, S = ((13/3) D^2 +
        // eps4) + E^2 = 4 (eps + beta): one fused multiply-add per indicator instead of a
        // product and an addition.  The two weight denominators share one reciprocal,
        // 1/D_L = D_R / (D_L D_R) (one refined reciprocal and three products instead of
        // two reciprocals; the product of the two is a product of eight (eps + beta)
        // factors, inside the FP64 range for the eps and beta the plan admits)
        const T kda = k * da, kdb = k * db, kdc = k * dc, kdd = k * dd;
        const T sb = kdb * db + eps4, sc = kdc * dc + eps4;  // shared by the two biases
        const T SL1 = (kda * da + eps4) + ea * ea, SL2 = sb + eb * eb, SL3 = sc + ec * ec;
        const T SR1 = (kdd * dd + eps4) + fa * fa, SR2 = sc + fb * fb, SR3 = sb + fc * fc;
        T nL, dL, nR, dR;
        weno5_js_terms<T>(SL1, SL2, SL3, L1, L2, L3, nL, dL);
        weno5_js_terms<T>(SR1, SR2, SR3, R1, L3, L2, nR, dR);
        const T r = rcp(dL * dR);
        L6 = nL * (dR * r);
        R6 = nR * (dL * r);
    } else {
        const B qb = k * db * db, qc = k * dc * dc;  // shared by the two biases
        B bL1 = k * da * da + ea * ea;
        B bL2 = qb + eb * eb;
        B bL3 = qc + ec * ec;
        B bR1 = k * dd * dd + fa * fa;
        B bR2 = qc + fb * fb;
        B bR3 = qb + fc * fc;
        L6 = weno5_combine<T, B, WW>(bL1, bL2, bL3, eps4, L1, L2, L3);
        R6 = weno5_combine<T, B, WW>(bR1, bR2, bR3, eps4, R1, L3, L2);
    }
}

// the left- and right-biased values themselves
template <typename T, typename B, int WW = CNS_WENO_JS>
__device__ __forceinline__ void weno5_lr(T m2, T m1, T c0, T p1, T p2, T p3, T eps, T &L, T &R) {
    T L6, R6;
    weno5_lr6<T, B, WW>(m2, m1, c0, p1, p2, p3, T(4) * eps, L6, R6);
    L = L6 * (T(1) / T(6));
    R = R6 * (T(1) / T(6));
}

// ---------------------------------------------------------------------------
// Sec. 2.1: convective flux along DIR of the conserved state w[5]
// ---------------------------------------------------------------------------
template <typename T, int DIR>
__device__ __forceinline__ void euler_flux(const T w[5], T gm1, T f[5]) {
    T inv = rcp(w[0]);
    T vx = w[1] * inv, vy = w[2] * inv, vz = w[3] * inv;
    T p = gm1 * (w[4] - T(0.5) * (w[1] * vx + w[2] * vy + w[3] * vz));
    T vn = DIR == 0 ? vx : (DIR == 1 ? vy : vz);
    f[0] = w[1 + DIR];
    f[1] = w[1] * vn;
    f[2] = w[2] * vn;
    f[3] = w[3] * vn;
    f[1 + DIR] += p;
    f[4] = (w[4] + p) * vn;
}

// ---------------------------------------------------------------------------
// Sec. 2.2: Roe dissipation D = |A| (uR - uL) at the Roe average of the cell
// states a (= u_j) and b (= u_{j+1}), with Harten's fix on every eigenvalue.
// ---------------------------------------------------------------------------
template <typename T, int DIR>
__device__ __forceinline__ void roe_dissipation(const T a[5], const T b[5], const T du[5], T gamma, T delta,
                                                T D[5]) {
    constexpr int N = DIR, T1 = (DIR + 1) % 3, T2 = (DIR + 2) % 3;
    const T gm1 = gamma - T(1);
    // 1/sqrt(rho) gives both sqrt(rho) = rho / sqrt(rho) and 1/rho
    T ra = rsq(a[0]), rb = rsq(b[0]);
    T ia = ra * ra, ib = rb * rb;
    T va[3] = {a[1] * ia, a[2] * ia, a[3] * ia};
    T vb[3] = {b[1] * ib, b[2] * ib, b[3] * ib};
    T pa = gm1 * (a[4] - T(0.5) * (a[1] * va[0] + a[2] * va[1] + a[3] * va[2]));
    T pb = gm1 * (b[4] - T(0.5) * (b[1] * vb[0] + b[2] * vb[1] + b[3] * vb[2]));
    T Ha = (a[4] + pa) * ia, Hb = (b[4] + pb) * ib;
    T sa = a[0] * ra, sb = b[0] * rb;
    T iw = rcp(sa + sb);
    T wa = sa * iw, wb = sb * iw;
    T v[3] = {wa * va[0] + wb * vb[0], wa * va[1] + wb * vb[1], wa * va[2] + wb * vb[2]};
    T H = wa * Ha + wb * Hb;
    T q2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    T c2 = gm1 * (H - T(0.5) * q2);
    T ic = rsq(c2);
    T c = c2 * ic;
    T vn = v[N];

    // wave strengths alpha = X^-1 du
    T at1 = du[1 + T1] - v[T1] * du[0];
    T at2 = du[1 + T2] - v[T2] * du[0];
    T dEb = du[4] - at1 * v[T1] - at2 * v[T2];
    T a2 = gm1 * (ic * ic) * (du[0] * (H - vn * vn) + vn * du[1 + N] - dEb);
    T a1 = (du[0] * (vn + c) - du[1 + N] - c * a2) * (T(0.5) * ic);
    T a5 = du[0] - (a1 + a2);

    const T hd = T(0.5) / delta;  // loop invariant
    T l1 = harten_abs(vn - c, delta, hd), l2 = harten_abs(vn, delta, hd), l5 = harten_abs(vn + c, delta, hd);
    T s1 = l1 * a1, s2 = l2 * a2, s5 = l5 * a5, st1 = l2 * at1, st2 = l2 * at2;

    // D = sum_k |lam_k| alpha_k K_k with the right eigenvectors K_k
    T ssum = s1 + s2 + s5;
    D[0] = ssum;
    D[1] = ssum * v[0];
    D[2] = ssum * v[1];
    D[3] = ssum * v[2];
    D[1 + N] += c * (s5 - s1);
    D[1 + T1] += st1;
    D[1 + T2] += st2;
    D[4] = s1 * (H - vn * c) + s2 * (T(0.5) * q2) + s5 * (H + vn * c) + st1 * v[T1] + st2 * v[T2];
}

// 5-point 4th-order central first derivative (times h)
template <typename T>
__device__ __forceinline__ T dcen(T m2, T m1, T p1, T p2) {
    return (T(8) * (p1 - m1) - (p2 - m2)) * (T(1) / T(12));
}

}  // namespace cns
