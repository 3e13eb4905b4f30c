// cns_device_adj.h -- hand-written reverse-mode (vector-Jacobian) products of the
// device arithmetic in cns_device.h, FP64.  Each *_vjp function recomputes the
// forward values it needs and ADDS the input adjoints to its outputs (weno5_lr_vjp
// sets them).
#pragma once
#include "cns_device.h"

namespace cns {

// d|lam|_H / d lam of Harten's fix (0 at lam = 0 when delta = 0); idelta = 1/delta.
// Written with selects, no branches.
__device__ __forceinline__ double harten_dabs(double lam, double delta, double idelta) {
    const double sgn = lam > 0.0 ? 1.0 : (lam < 0.0 ? -1.0 : 0.0);
    return fabs(lam) >= delta ? sgn : lam * idelta;
}

// ---------------------------------------------------------------------------
// One biased reconstruction V = sum_k w_k q_k from the plain candidates q_k and the
// smoothness sums s_k = eps + beta_k: the value, the final weights w_k and dV/dbeta_k.
// With w_k = alpha_k / A and A = sum alpha:  dV/dbeta_j = sum_k (q_k - V) dalpha_k/dbeta_j / A.
//   JS: alpha_k = c_k / s_k^2, so dV/dbeta_j = -2 (q_j - V) w_j / s_j; the weights in
//       product form, t_k = prod_{i != k} s_i, P = s1 s2 s3, a_k = c_k t_k^2,
//       w_k = a_k P iPA and w_k / s_k = a_k t_k iPA with iPA = 1 / (P sum a).
//   Z:  alpha_k = c_k + tau z_k with z_k = c_k tau / s_k^2, tau = |beta1 - beta3|:
//       dV/dbeta_j = (1/A) [-2 (q_j - V) tau z_j / s_j + dtau/dbeta_j 2 sum_k (q_k - V) z_k].
//   M:  the JS weights u_k mapped, g_k = c_k + (u_k - c_k)^3 / D_k, D_k = c_k^2 + u_k (1 - 2 c_k),
//       w_k = g_k / G; with gamma_k = (q_k - V) g'_k / G,
//       dV/dbeta_j = -2 (u_j / s_j) (gamma_j - sum_k gamma_k u_k).
// ---------------------------------------------------------------------------
template <int WW>
__device__ __forceinline__ void weno_side_vjp(double s1, double s2, double s3, double q1, double q2, double q3,
                                              double &V, double w[3], double dV[3]) {
    if constexpr (WW == CNS_WENO_Z) {
        const double tau = fabs(s1 - s3);
        const double i1 = rcp(s1), i2 = rcp(s2), i3 = rcp(s3);
        const double z1 = 0.1 * tau * (i1 * i1), z2 = 0.6 * tau * (i2 * i2), z3 = 0.3 * tau * (i3 * i3);
        const double a1 = 0.1 + tau * z1, a2 = 0.6 + tau * z2, a3 = 0.3 + tau * z3;
        const double iA = rcp(a1 + a2 + a3);
        w[0] = a1 * iA, w[1] = a2 * iA, w[2] = a3 * iA;
        V = w[0] * q1 + w[1] * q2 + w[2] * q3;
        const double sg = s1 > s3 ? 1.0 : (s1 < s3 ? -1.0 : 0.0);
        const double P = 2.0 * ((q1 - V) * z1 + (q2 - V) * z2 + (q3 - V) * z3);
        dV[0] = iA * (-2.0 * (q1 - V) * tau * z1 * i1 + sg * P);
        dV[1] = iA * (-2.0 * (q2 - V) * tau * z2 * i2);
        dV[2] = iA * (-2.0 * (q3 - V) * tau * z3 * i3 - sg * P);
    } else {
        const double t1 = s2 * s3, t2 = s1 * s3, t3 = s1 * s2;
        const double a1 = 0.1 * (t1 * t1), a2 = 0.6 * (t2 * t2), a3 = 0.3 * (t3 * t3);
        const double iPA = rcp((t3 * s3) * (a1 + a2 + a3));
        const double iA = (t3 * s3) * iPA;
        const double u1 = a1 * iA, u2 = a2 * iA, u3 = a3 * iA;                     // Jiang-Shu weights
        const double r1 = a1 * t1 * iPA, r2 = a2 * t2 * iPA, r3 = a3 * t3 * iPA;  // u_k / s_k
        if constexpr (WW == CNS_WENO_JS) {
            w[0] = u1, w[1] = u2, w[2] = u3;
            V = u1 * q1 + u2 * q2 + u3 * q3;
            dV[0] = -2.0 * (q1 - V) * r1;
            dV[1] = -2.0 * (q2 - V) * r2;
            dV[2] = -2.0 * (q3 - V) * r3;
        } else {
            static_assert(WW == CNS_WENO_M, "unknown WENO weights");
            const double c[3] = {0.1, 0.6, 0.3}, u[3] = {u1, u2, u3}, r[3] = {r1, r2, r3}, q[3] = {q1, q2, q3};
            double g[3], gp[3], G = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double e = u[k] - c[k], D = c[k] * c[k] + u[k] * (1.0 - 2.0 * c[k]), iD = rcp(D);
                g[k] = c[k] + e * e * e * iD;
                gp[k] = e * e * (3.0 * D - e * (1.0 - 2.0 * c[k])) * (iD * iD);
                G += g[k];
            }
            const double iG = rcp(G);
            V = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                w[k] = g[k] * iG;
                V += w[k] * q[k];
            }
            double gam[3], S = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                gam[k] = (q[k] - V) * gp[k] * iG;
                S += gam[k] * u[k];
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) dV[k] = -2.0 * r[k] * (gam[k] - S);
        }
    }
}

// One Jiang-Shu side in the scaled form of the forward (weno5_lr6): candidates Q_k six
// times the plain ones, S_k = 4 (eps + beta_k), weights w_k = g_k A_k / sum with
// g = (1, 6, 3), A_k = t_k^2 and t_k the product of the other two S.  Given the
// adjoint Vb6 of V6 = sum w_k Q_k: V6, the candidate adjoints Qb_k = Vb6 w_k and TWICE
// the adjoints of S_k, from dV6/dS_k = -2 w_k (Q_k - V6) / S_k with 1/S_k = t_k / P,
// P = S1 S2 S3 (one reciprocal, of P sum).
__device__ __forceinline__ void js_side_vjp(double S1, double S2, double S3, double Q1, double Q2, double Q3,
                                            double Vb6, double &V6, double Qb[3], double Sb2[3]) {
    const double t1 = S2 * S3, t2 = S1 * S3, t3 = S1 * S2;
    const double B1 = t1 * t1, B2 = 6.0 * (t2 * t2), B3 = 3.0 * (t3 * t3);  // g_k A_k
    const double P = t1 * S1;
    const double sum = B1 + B2 + B3;
    const double num = B1 * Q1 + B2 * Q2 + B3 * Q3;
    const double iD = rcp(P * sum);
    const double iS = P * iD;
    V6 = num * iS;
    const double h = Vb6 * iS;
    Qb[0] = h * B1;
    Qb[1] = h * B2;
    Qb[2] = h * B3;
    const double g = -4.0 * Vb6 * iD;
    Sb2[0] = g * ((Q1 - V6) * (B1 * t1));
    Sb2[1] = g * ((Q2 - V6) * (B2 * t2));
    Sb2[2] = g * ((Q3 - V6) * (B3 * t3));
}

// ---------------------------------------------------------------------------
// WENO5 pair (weno5_lr with the weights WW): given the adjoints Lb, Rb of the left-
// and right-biased values at j+1/2, SET qb[0..5] to dL/dq^T Lb + dR/dq^T Rb
// (q = j-2 .. j+3); the values L and R themselves are returned in Lv, Rv.
// ---------------------------------------------------------------------------
template <int WW = CNS_WENO_JS>
__device__ __forceinline__ void weno5_lr_vjp(const double q[6], double eps, double Lb, double Rb, double qb[6],
                                             double &Lv, double &Rv) {
    const double m2 = q[0], m1 = q[1], c0 = q[2], p1 = q[3], p2 = q[4], p3 = q[5];
    if constexpr (WW == CNS_WENO_JS) {
        // six times the candidates (the right-biased side reuses L2, L3 mirrored), the
        // second differences and the one-sided terms, all from the first differences
        // g_i = q_{i+1} - q_i as in the forward (the terms keep their signs here: the
        // scatter below uses them unsquared)
        const double g0 = m1 - m2, g1 = c0 - m1, g2 = p1 - c0, g3 = p2 - p1, g4 = p3 - p2;
        const double c6 = 6.0 * c0;
        const double L1 = (5.0 * g1 - 2.0 * g0) + c6;     // 2 m2 - 7 m1 + 11 c0
        const double L2 = (g1 + 2.0 * g2) + c6;           // -m1 + 5 c0 + 2 p1
        const double L3 = (4.0 * g2 - g3) + c6;           // 2 c0 + 5 p1 - p2
        const double R1 = 6.0 * p1 - 5.0 * g3 + 2.0 * g4;  // 2 p3 - 7 p2 + 11 p1
        const double da = g1 - g0, db = g2 - g1, dc = g3 - g2, dd = g4 - g3;
        const double ea = 3.0 * g1 - g0;     // m2 - 4 m1 + 3 c0
        const double eb = -(g1 + g2);        // m1 - p1
        const double ec = -(3.0 * g2 - g3);  // 3 c0 - 4 p1 + p2
        const double fa = -(3.0 * g3 - g4);  // p3 - 4 p2 + 3 p1
        const double fb = g2 + g3;           // p2 - c0
        const double fc = 3.0 * g2 - g1;     // 3 p1 - 4 c0 + m1
        // S = 4 eps + (13/3) d^2 + e^2
        const double k = 13.0 / 3.0, e4 = 4.0 * eps;
        const double kda = k * da, kdb = k * db, kdc = k * dc, kdd = k * dd;
        const double sb = kdb * db + e4, sc = kdc * dc + e4;
        const double SL1 = (kda * da + e4) + ea * ea, SL2 = sb + eb * eb, SL3 = sc + ec * ec;
        const double SR1 = (kdd * dd + e4) + fa * fa, SR2 = sc + fb * fb, SR3 = sb + fc * fc;
        double VL, VR, QL[3], QR[3], BL[3], BR[3];
        js_side_vjp(SL1, SL2, SL3, L1, L2, L3, Lb * (1.0 / 6.0), VL, QL, BL);
        js_side_vjp(SR1, SR2, SR3, R1, L3, L2, Rb * (1.0 / 6.0), VR, QR, BR);
        Lv = VL * (1.0 / 6.0);
        Rv = VR * (1.0 / 6.0);
        // adjoints of the candidates, and of d and e through S (dS/dd = 2 k d, dS/de = 2 e;
        // BL, BR carry the factor 2)
        const double cL1 = QL[0], cL2 = QL[1] + QR[2], cL3 = QL[2] + QR[1], cR1 = QR[0];
        const double dab = kda * BL[0], dbb = kdb * (BL[1] + BR[2]), dcb = kdc * (BL[2] + BR[1]), ddb = kdd * BR[0];
        const double eab = ea * BL[0], ebb = eb * BL[1], ecb = ec * BL[2];
        const double fab = fa * BR[0], fbb = fb * BR[1], fcb = fc * BR[2];
        qb[0] = dab + eab + 2.0 * cL1;
        qb[1] = -2.0 * dab + dbb - 4.0 * eab + ebb + fcb - 7.0 * cL1 - cL2;
        qb[2] = dab - 2.0 * dbb + dcb + 3.0 * eab + 3.0 * ecb - fbb - 4.0 * fcb + 11.0 * cL1 + 5.0 * cL2 + 2.0 * cL3;
        qb[3] = dbb - 2.0 * dcb + ddb - ebb - 4.0 * ecb + 3.0 * fab + 3.0 * fcb + 2.0 * cL2 + 5.0 * cL3 + 11.0 * cR1;
        qb[4] = dcb - 2.0 * ddb + ecb - 4.0 * fab + fbb - cL3 - 7.0 * cR1;
        qb[5] = ddb + fab + 2.0 * cR1;
        return;
    }
    const double r6 = 1.0 / 6.0, k13 = 13.0 / 12.0;
    const double L1 = (2.0 * m2 - 7.0 * m1 + 11.0 * c0) * r6;
    const double L2 = (-m1 + 5.0 * c0 + 2.0 * p1) * r6;
    const double L3 = (2.0 * c0 + 5.0 * p1 - p2) * r6;
    const double R1 = (2.0 * p3 - 7.0 * p2 + 11.0 * p1) * r6;
    const double da = m2 - 2.0 * m1 + c0, db = m1 - 2.0 * c0 + p1, dc = c0 - 2.0 * p1 + p2, dd = p1 - 2.0 * p2 + p3;
    const double ea = m2 - 4.0 * m1 + 3.0 * c0, eb = m1 - p1, ec = 3.0 * c0 - 4.0 * p1 + p2;
    const double fa = p3 - 4.0 * p2 + 3.0 * p1, fb = p2 - c0, fc = 3.0 * p1 - 4.0 * c0 + m1;
    const double s1 = eps + (k13 * da * da + 0.25 * ea * ea);
    const double s2 = eps + (k13 * db * db + 0.25 * eb * eb);
    const double s3 = eps + (k13 * dc * dc + 0.25 * ec * ec);
    const double u1 = eps + (k13 * dd * dd + 0.25 * fa * fa);
    const double u2 = eps + (k13 * dc * dc + 0.25 * fb * fb);
    const double u3 = eps + (k13 * db * db + 0.25 * fc * fc);
    double L, R, w[3], v[3], dL[3], dR[3];
    weno_side_vjp<WW>(s1, s2, s3, L1, L2, L3, L, w, dL);  // left-biased
    weno_side_vjp<WW>(u1, u2, u3, R1, L3, L2, R, v, dR);  // right-biased (mirrored stencils)

    // candidates
    const double cL1 = Lb * w[0], cL2 = Lb * w[1] + Rb * v[2], cL3 = Lb * w[2] + Rb * v[1], cR1 = Rb * v[0];
    // indicators
    const double bL1 = Lb * dL[0], bL2 = Lb * dL[1], bL3 = Lb * dL[2];
    const double bR1 = Rb * dR[0], bR2 = Rb * dR[1], bR3 = Rb * dR[2];
    const double dab = 2.0 * k13 * da * bL1, eab = 0.5 * ea * bL1;
    const double dbb = 2.0 * k13 * db * (bL2 + bR3), ebb = 0.5 * eb * bL2, fcb = 0.5 * fc * bR3;
    const double dcb = 2.0 * k13 * dc * (bL3 + bR2), ecb = 0.5 * ec * bL3, fbb = 0.5 * fb * bR2;
    const double ddb = 2.0 * k13 * dd * bR1, fab = 0.5 * fa * bR1;
    qb[0] = 2.0 * r6 * cL1 + dab + eab;
    qb[1] = -7.0 * r6 * cL1 - r6 * cL2 - 2.0 * dab + dbb - 4.0 * eab + ebb + fcb;
    qb[2] = 11.0 * r6 * cL1 + 5.0 * r6 * cL2 + 2.0 * r6 * cL3 + dab - 2.0 * dbb + dcb + 3.0 * eab + 3.0 * ecb -
             fbb - 4.0 * fcb;
    qb[3] = 2.0 * r6 * cL2 + 5.0 * r6 * cL3 + 11.0 * r6 * cR1 + dbb - 2.0 * dcb + ddb - ebb - 4.0 * ecb + 3.0 * fab +
             3.0 * fcb;
    qb[4] = -r6 * cL3 - 7.0 * r6 * cR1 + dcb - 2.0 * ddb + ecb - 4.0 * fab + fbb;
    qb[5] = 2.0 * r6 * cR1 + ddb + fab;
    Lv = L;
    Rv = R;
}

// component v of the convective flux along DIR
template <int DIR>
__device__ __forceinline__ double euler_flux_comp(const double w[5], double gm1, int v) {
    const double inv = rcp(w[0]);
    const double vn = w[1 + DIR] * inv;
    if (v == 0) return w[1 + DIR];
    const double p = gm1 * (w[4] - 0.5 * (w[1] * (w[1] * inv) + w[2] * (w[2] * inv) + w[3] * (w[3] * inv)));
    if (v == 4) return (w[4] + p) * vn;
    return w[v] * vn + (v == 1 + DIR ? p : 0.0);
}

// wb += (df/dw)^T fb for the convective flux along DIR (the Euler flux Jacobian).
// With v = m / rho, K = |v|^2 / 2, p = (gamma-1)(e - rho K), H = (e + p) / rho,
// phi = fb[1..3], psi = fb[4] and s = (gamma-1)(phi_n + psi v_n):
//   rho:  s K - v_n (phi.v + psi H)
//   m_j:  v_n phi_j - s v_j, plus fb[0] + phi.v + psi H for j = n
//   e:    s + psi v_n
template <int DIR>
__device__ __forceinline__ void euler_flux_vjp(const double w[5], double gm1, const double fb[5], double wb[5]) {
    const double inv = rcp(w[0]);
    const double v[3] = {w[1] * inv, w[2] * inv, w[3] * inv};
    const double K = 0.5 * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    const double p = gm1 * (w[4] - w[0] * K);
    const double H = (w[4] + p) * inv;
    const double vn = v[DIR];
    const double s = gm1 * (fb[1 + DIR] + fb[4] * vn);
    const double dotH = fb[1] * v[0] + fb[2] * v[1] + fb[3] * v[2] + fb[4] * H;
    wb[0] += s * K - vn * dotH;
#pragma unroll
    for (int j = 0; j < 3; ++j) wb[1 + j] += vn * fb[1 + j] - s * v[j] + (j == DIR ? fb[0] + dotH : 0.0);
    wb[4] += s + fb[4] * vn;
}

// ---------------------------------------------------------------------------
// Roe dissipation (roe_dissipation, wave-strength form) D = M(a, b) du: linear in the
// jump du, with M from the Roe average of the cell states a, b alone (Harten's fix
// acts on the eigenvalues).  Given Db, the two parts of its transpose product:
//   STATES = false: dub += M^T Db (needs no du);
//   STATES = true:  ab, bb += the adjoints of a and b through M (needs du).
// ---------------------------------------------------------------------------
// The Roe average of the cell states a, b and the fixed eigenvalues: formed once per
// interface for both parts of the transpose product.
struct RoeAvg {
    double ra, rb, ia, ib, va[3], vb[3], pa, pb, Ha, Hb, sa, sb, iw, wa, wb, v[3], H, q2, c, ic, ic2, l1, l2, l5;
};
template <int DIR>
__device__ __forceinline__ RoeAvg roe_avg(const double a[5], const double b[5], double gamma, double delta) {
    const double gm1 = gamma - 1.0;
    RoeAvg R;
    R.ra = rsq(a[0]), R.rb = rsq(b[0]);
    R.ia = R.ra * R.ra, R.ib = R.rb * R.rb;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        R.va[k] = a[1 + k] * R.ia;
        R.vb[k] = b[1 + k] * R.ib;
    }
    const double qa = a[1] * R.va[0] + a[2] * R.va[1] + a[3] * R.va[2];
    const double qb = b[1] * R.vb[0] + b[2] * R.vb[1] + b[3] * R.vb[2];
    R.pa = gm1 * (a[4] - 0.5 * qa), R.pb = gm1 * (b[4] - 0.5 * qb);
    R.Ha = (a[4] + R.pa) * R.ia, R.Hb = (b[4] + R.pb) * R.ib;
    R.sa = a[0] * R.ra, R.sb = b[0] * R.rb;
    R.iw = rcp(R.sa + R.sb);
    R.wa = R.sa * R.iw, R.wb = R.sb * R.iw;
#pragma unroll
    for (int k = 0; k < 3; ++k) R.v[k] = R.wa * R.va[k] + R.wb * R.vb[k];
    R.H = R.wa * R.Ha + R.wb * R.Hb;
    R.q2 = R.v[0] * R.v[0] + R.v[1] * R.v[1] + R.v[2] * R.v[2];
    const double c2 = gm1 * (R.H - 0.5 * R.q2);
    R.ic = rsq(c2);
    R.c = c2 * R.ic, R.ic2 = R.ic * R.ic;
    const double vn = R.v[DIR], hd = 0.5 / delta;
    R.l1 = harten_abs(vn - R.c, delta, hd), R.l2 = harten_abs(vn, delta, hd), R.l5 = harten_abs(vn + R.c, delta, hd);
    return R;
}

template <int DIR, bool STATES>
__device__ __forceinline__ void roe_dissipation_vjp(const RoeAvg &R, const double a[5], const double b[5],
                                                    const double du[5], double gamma, double delta,
                                                    const double Db[5], double ab[5], double bb[5], double dub[5]) {
    constexpr int N = DIR, T1 = (DIR + 1) % 3, T2 = (DIR + 2) % 3;
    const double gm1 = gamma - 1.0;
    const double ra = R.ra, rb = R.rb, ia = R.ia, ib = R.ib, pa = R.pa, pb = R.pb, Ha = R.Ha, Hb = R.Hb;
    const double sa = R.sa, sb = R.sb, iw = R.iw, wa = R.wa, wb = R.wb, H = R.H, q2 = R.q2;
    const double c = R.c, ic = R.ic, ic2 = R.ic2, l1 = R.l1, l2 = R.l2, l5 = R.l5;
    const double *va = R.va, *vb = R.vb, *v = R.v;
    const double vn = v[N];
    const double idelta = 1.0 / delta;
    // ---- forward recompute: the wave strengths of du (only the state adjoints need them)
    double at1 = 0, at2 = 0, a1 = 0, a2 = 0, a5 = 0, s1 = 0, s2 = 0, s5 = 0, st1 = 0, st2 = 0, ssum = 0;
    if constexpr (STATES) {
        at1 = du[1 + T1] - v[T1] * du[0];
        at2 = du[1 + T2] - v[T2] * du[0];
        const double dEb = du[4] - at1 * v[T1] - at2 * v[T2];
        const double X = du[0] * (H - vn * vn) + vn * du[1 + N] - dEb;
        a2 = gm1 * ic2 * X;
        const double num = du[0] * (vn + c) - du[1 + N] - c * a2;
        a1 = num * (0.5 * ic);
        a5 = du[0] - (a1 + a2);
        s1 = l1 * a1, s2 = l2 * a2, s5 = l5 * a5, st1 = l2 * at1, st2 = l2 * at2;
        ssum = s1 + s2 + s5;
    }

    // ---- reverse
    double s1b = 0, s2b = 0, s5b = 0, st1b = 0, st2b = 0, ssumb = 0, Hbar = 0, vnb = 0, cb = 0, q2b = 0;
    double vbar[3] = {0, 0, 0};
    // D4 = s1 (H - vn c) + s2 q2/2 + s5 (H + vn c) + st1 v_t1 + st2 v_t2
    s1b += Db[4] * (H - vn * c);
    s5b += Db[4] * (H + vn * c);
    s2b += Db[4] * 0.5 * q2;
    st1b += Db[4] * v[T1];
    st2b += Db[4] * v[T2];
    if constexpr (STATES) {
        Hbar += Db[4] * (s1 + s5);
        vnb += Db[4] * (s5 - s1) * c;
        cb += Db[4] * (s5 - s1) * vn;
        q2b += Db[4] * 0.5 * s2;
        vbar[T1] += Db[4] * st1;
        vbar[T2] += Db[4] * st2;
    }
    // D[1+T1] += st1, D[1+T2] += st2, D[1+N] += c (s5 - s1)
    st1b += Db[1 + T1];
    st2b += Db[1 + T2];
    s5b += Db[1 + N] * c;
    s1b -= Db[1 + N] * c;
    if constexpr (STATES) cb += Db[1 + N] * (s5 - s1);
    // D0 = ssum, D[1+k] = ssum v_k (before the additions above)
    ssumb += Db[0];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        ssumb += Db[1 + k] * v[k];
        if constexpr (STATES) vbar[k] += Db[1 + k] * ssum;
    }
    s1b += ssumb;
    s2b += ssumb;
    s5b += ssumb;
    // s = |lam| alpha
    double a1b = s1b * l1, a2b = s2b * l2, a5b = s5b * l5, at1b = st1b * l2, at2b = st2b * l2;
    if constexpr (STATES) {
        const double l1b = s1b * a1, l2b = s2b * a2 + st1b * at1 + st2b * at2, l5b = s5b * a5;
        const double x1 = l1b * harten_dabs(vn - c, delta, idelta);
        const double x5 = l5b * harten_dabs(vn + c, delta, idelta);
        vnb += x1 + l2b * harten_dabs(vn, delta, idelta) + x5;
        cb += x5 - x1;
    }
    // a5 = du0 - (a1 + a2)
    if constexpr (!STATES) dub[0] += a5b;
    a1b -= a5b;
    a2b -= a5b;
    // a1 = num / (2c)
    const double numb = a1b * (0.5 * ic);
    if constexpr (STATES) {
        cb -= a1b * a1 * ic;
        vnb += numb * du[0];
        cb += numb * du[0];
        cb -= numb * a2;
    } else {
        dub[0] += numb * (vn + c);
        dub[1 + N] -= numb;
    }
    a2b -= numb * c;
    // a2 = gm1/c2 X
    const double Xb = a2b * gm1 * ic2;
    // X = du0 (H - vn^2) + vn du_n - dEb;  dEb = du4 - at1 v_t1 - at2 v_t2;  at = du_t - v_t du0
    const double dEbb = -Xb;
    at1b -= dEbb * v[T1];
    at2b -= dEbb * v[T2];
    if constexpr (!STATES) {
        dub[0] += Xb * (H - vn * vn);
        dub[1 + N] += Xb * vn;
        dub[4] += dEbb;
        dub[1 + T1] += at1b;
        dub[0] -= at1b * v[T1];
        dub[1 + T2] += at2b;
        dub[0] -= at2b * v[T2];
        return;
    }
    double c2b = -a2b * a2 * ic2;
    Hbar += Xb * du[0];
    vnb += Xb * (du[1 + N] - 2.0 * vn * du[0]);
    vbar[T1] -= dEbb * at1;
    vbar[T2] -= dEbb * at2;
    vbar[T1] -= at1b * du[0];
    vbar[T2] -= at2b * du[0];
    vbar[N] += vnb;
    // c = sqrt(c2); c2 = gm1 (H - q2/2); q2 = |v|^2
    c2b += cb * (0.5 * ic);
    Hbar += c2b * gm1;
    q2b -= 0.5 * gm1 * c2b;
#pragma unroll
    for (int k = 0; k < 3; ++k) vbar[k] += 2.0 * v[k] * q2b;
    // H = wa Ha + wb Hb;  v = wa va + wb vb
    double wab = Hbar * Ha, wbb = Hbar * Hb;
    const double Hab = Hbar * wa, Hbb = Hbar * wb;
    double vab[3], vbb[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        wab += vbar[k] * va[k];
        wbb += vbar[k] * vb[k];
        vab[k] = vbar[k] * wa;
        vbb[k] = vbar[k] * wb;
    }
    // wa = sa iw, wb = sb iw, iw = 1/(sa + sb)
    const double iwb = wab * sa + wbb * sb;
    const double sab = wab * iw - iwb * iw * iw;
    const double sbb = wbb * iw - iwb * iw * iw;
    // Ha = (a4 + pa) ia; pa = gm1 (a4 - qa/2); qa = sum a_k va_k; va = a_k ia; ia = 1/a0
    {
        const double pab = Hab * ia;
        double iab = Hab * (a[4] + pa);
        ab[4] += Hab * ia + pab * gm1;
        const double qab = -0.5 * gm1 * pab;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double vk = vab[k] + qab * a[1 + k];
            ab[1 + k] += qab * va[k] + vk * ia;
            iab += vk * a[1 + k];
        }
        ab[0] += -iab * ia * ia + sab * (0.5 * ra);  // d sqrt(rho)/d rho = 1/(2 sqrt(rho))
    }
    {
        const double pbb = Hbb * ib;
        double ibb = Hbb * (b[4] + pb);
        bb[4] += Hbb * ib + pbb * gm1;
        const double qbb = -0.5 * gm1 * pbb;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double vk = vbb[k] + qbb * b[1 + k];
            bb[1 + k] += qbb * vb[k] + vk * ib;
            ibb += vk * b[1 + k];
        }
        bb[0] += -ibb * ib * ib + sbb * (0.5 * rb);
    }
}

// ---------------------------------------------------------------------------
// Convective interface flux H = (FL + FR)/2 - D/2 (interface_flux without the viscous
// part), transposed for the six cell states j-2 .. j+3, which sit at offsets c[0..5]
// of the array st, components 0-4, with their point fluxes along DIR as components
// 5-9 (component stride cs; the caller stages them in LDS).  The
// contributions leave through two callbacks as soon as they are formed, so that no
// 6 x 5 array of them is ever held:
//   addF(m, v, x): x is a term of the adjoint of the POINT FLUX of cell j-2+m, component
//     v (each reconstruction carries Hb/2); the flux Jacobian transpose that takes it to
//     the cell state is linear in it, so the caller sums these terms over the six
//     interfaces that read a cell and applies the transpose once per cell;
//   addU(m, v, x): a term of the adjoint of the STATE of cell j-2+m, through the Roe
//     dissipation and the reconstructed states.
// For each (m, v) the terms are produced in a fixed order.  The states are read again
// from st at each stage instead of being held, and the compiler barrier between stages
// keeps it from merging the loads back into one live set.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void adj_stage_fence() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
}

template <int DIR, int WW, class AddF, class AddU>
__device__ __forceinline__ void interface_flux_vjp(const double *st, int cs, const int c[6], const double Hb[5],
                                                   double gamma, double eps, double delta, AddF addF, AddU addU) {
    {
        // component by component, the adjoints of the reconstructions of the point fluxes
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            const double *f = st + (5 + v) * cs;
            double q[6], qb[6];
#pragma unroll
            for (int m = 0; m < 6; ++m) q[m] = f[c[m]];
            double Lv, Rv;
            weno5_lr_vjp<WW>(q, eps, 0.5 * Hb[v], 0.5 * Hb[v], qb, Lv, Rv);
#pragma unroll
            for (int m = 0; m < 6; ++m) addF(m, v, qb[m]);
            adj_stage_fence();
        }
    }
    // dissipation D = M(a, b) du at cells a = j, b = j+1: first dub = M^T Db, which needs
    // no du; the reverse of the reconstructed states then yields du itself (UR - UL);
    // last the adjoints of a and b through M
    double a[5], b[5], Db[5], du[5], dub[5] = {0, 0, 0, 0, 0};
    double ab[5] = {0, 0, 0, 0, 0}, bb[5] = {0, 0, 0, 0, 0};
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        a[v] = st[v * cs + c[2]];
        b[v] = st[v * cs + c[3]];
        Db[v] = -0.5 * Hb[v];
        du[v] = 0.0;
    }
    const RoeAvg R = roe_avg<DIR>(a, b, gamma, delta);
    roe_dissipation_vjp<DIR, false>(R, a, b, du, gamma, delta, Db, ab, bb, dub);
    adj_stage_fence();
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        const double *f = st + v * cs;
        double q[6], qb[6], UL, UR;
#pragma unroll
        for (int m = 0; m < 6; ++m) q[m] = f[c[m]];
        weno5_lr_vjp<WW>(q, eps, -dub[v], dub[v], qb, UL, UR);
        du[v] = UR - UL;
#pragma unroll
        for (int m = 0; m < 6; ++m) addU(m, v, qb[m]);
        adj_stage_fence();
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        a[v] = st[v * cs + c[2]];
        b[v] = st[v * cs + c[3]];
    }
    roe_dissipation_vjp<DIR, true>(R, a, b, du, gamma, delta, Db, ab, bb, dub);
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        addU(2, v, ab[v]);
        addU(3, v, bb[v]);
    }
}

}  // namespace cns
