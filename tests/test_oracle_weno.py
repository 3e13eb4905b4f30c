"""Pins of the oracle's WENO5 reconstruction (paper Sec. 2.2, eqs. for the three
third-order candidates, the fifth-order combination, the weights and the
smoothness indicators).  Each pin checks the oracle against something fixed
independently of its code: exact integrals, printed coefficients, the
Jiang-Shu integral definition of the indicators, and convergence order."""
import math
from fractions import Fraction as Fr

import numpy as np
import pytest


def cell_avgs_poly(coeffs, centres, h=1.0):
    """Exact cell averages over [x - h/2, x + h/2] of the polynomial sum c_n x^n (Fractions)."""
    out = []
    for x in centres:
        a = Fr(x) - Fr(h) / 2
        b = Fr(x) + Fr(h) / 2
        s = Fr(0)
        for n, c in enumerate(coeffs):
            s += Fr(c) * (b ** (n + 1) - a ** (n + 1)) / (n + 1)
        out.append(s / Fr(h))
    return out


def poly_val(coeffs, x):
    return sum(Fr(c) * Fr(x) ** n for n, c in enumerate(coeffs))


def test_candidates_exact_for_quadratic_cell_averages(orc):
    # interface j+1/2 with j = 0 at x = 0 and unit spacing: evaluate at x = 1/2
    rng = np.random.default_rng(1)
    for _ in range(20):
        coeffs = [Fr(int(c), 7) for c in rng.integers(-20, 20, size=3)]
        avg = cell_avgs_poly(coeffs, [-2, -1, 0, 1, 2])
        exact = float(poly_val(coeffs, Fr(1, 2)))
        _, parts = orc.weno5(*[float(v) for v in avg], eps=1e-6, parts=True)
        for k in range(3):
            assert parts[6 + k] == pytest.approx(exact, rel=1e-14, abs=1e-13)


def test_linear_weights_give_printed_fifth_order_interpolant(orc):
    # Data with equal smoothness indicators (affine data) makes alpha_k
    # proportional to c_k, so omega = c and the result must be the printed
    # fifth-order interpolant (2, -13, 47, 27, -3)/60.
    rng = np.random.default_rng(2)
    for _ in range(20):
        a0, a1 = rng.uniform(-3, 3, size=2)
        f = [a0 + a1 * m for m in (-2, -1, 0, 1, 2)]
        r, parts = orc.weno5(*f, eps=1e-6, parts=True)
        np.testing.assert_allclose(parts[3:6], [0.1, 0.6, 0.3], rtol=1e-13)
        printed = (2 * f[0] - 13 * f[1] + 47 * f[2] + 27 * f[3] - 3 * f[4]) / 60.0
        assert r == pytest.approx(printed, rel=1e-13, abs=1e-13)


def test_linear_scheme_is_exact_for_quartic_cell_averages(orc):
    # With the optimal weights the scheme is the fifth-order interpolant, exact
    # for cell averages of polynomials up to degree 4.  Check through the
    # returned candidates: sum c_k fhat_k must equal the exact point value.
    rng = np.random.default_rng(3)
    for _ in range(20):
        coeffs = [Fr(int(c), 5) for c in rng.integers(-9, 9, size=5)]
        avg = [float(v) for v in cell_avgs_poly(coeffs, [-2, -1, 0, 1, 2])]
        _, parts = orc.weno5(*avg, eps=1e-6, parts=True)
        lin = 0.1 * parts[6] + 0.6 * parts[7] + 0.3 * parts[8]
        assert lin == pytest.approx(float(poly_val(coeffs, Fr(1, 2))), rel=1e-12, abs=1e-12)


def js_indicator(avgs3, offset):
    """Jiang-Shu smoothness indicator from its integral definition:
    beta = sum_{l=1,2} h^{2l-1} int_{cell j} (d^l p / dx^l)^2 dx, with p the
    quadratic whose cell averages over the three cells (offset, offset+1,
    offset+2) relative to j=0 equal avgs3; h = 1, cell j = [-1/2, 1/2]."""
    # solve for p(x) = q0 + q1 x + q2 x^2 from exact cell-average conditions
    rows = []
    for m in range(3):
        c = offset + m
        a, b = Fr(c) - Fr(1, 2), Fr(c) + Fr(1, 2)
        rows.append([b - a, (b ** 2 - a ** 2) / 2, (b ** 3 - a ** 3) / 3])
    A = np.array(rows, dtype=object)
    # 3x3 solve with Fractions (Cramer)
    def det3(M):
        return (M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1])
                - M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0])
                + M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]))
    D = det3(A)
    q = []
    for col in range(3):
        M = [list(r) for r in A]
        for r in range(3):
            M[r][col] = avgs3[r]
        q.append(det3(M) / D)
    q0, q1, q2 = q
    # p' = q1 + 2 q2 x ; p'' = 2 q2 ; integrate over [-1/2, 1/2]
    int_p1sq = q1 * q1 + Fr(4) * q2 * q2 * Fr(1, 12)  # int (q1 + 2 q2 x)^2 dx
    int_p2sq = Fr(4) * q2 * q2
    return int_p1sq + int_p2sq


def test_smoothness_indicators_match_integral_definition(orc):
    rng = np.random.default_rng(4)
    for _ in range(30):
        f = [Fr(int(v), 3) for v in rng.integers(-30, 30, size=5)]
        _, parts = orc.weno5(*[float(v) for v in f], eps=1e-6, parts=True)
        b1 = js_indicator(f[0:3], -2)
        b2 = js_indicator(f[1:4], -1)
        b3 = js_indicator(f[2:5], 0)
        np.testing.assert_allclose(parts[0:3], [float(b1), float(b2), float(b3)], rtol=1e-13, atol=1e-12)


def test_weights_are_convex_and_reject_a_discontinuous_stencil(orc):
    # A unit jump between f_{j+1} and f_{j+2}: only stencil 3 crosses it.
    r, parts = orc.weno5(0.0, 0.0, 0.0, 0.0, 1.0, eps=1e-6, parts=True)
    w = parts[3:6]
    assert w.sum() == pytest.approx(1.0, rel=1e-15)
    assert np.all(w >= 0)
    # exponent 2 with eps = 1e-6 puts the crossing stencil's weight near
    # c3 * (eps/beta3)^2 / (c1 + c2) ~ 1e-13; exponent 1 would leave ~1e-6.
    assert w[2] < 1e-10
    assert abs(r) < 1e-10  # the two smooth stencils both give 0


def weno_flux_difference(f, eps=1e-6):
    """(W_{j+1/2} - W_{j-1/2}) on a periodic array through the oracle's W."""
    n = len(f)
    W = np.array([orc_w(f[(j - 2) % n], f[(j - 1) % n], f[j], f[(j + 1) % n], f[(j + 2) % n], eps)
                  for j in range(n)])
    return W - np.roll(W, 1)


orc_w = None


def test_fifth_order_convergence_on_smooth_data(orc):
    global orc_w
    orc_w = orc.weno5
    errs = []
    ns = [32, 64, 128, 256]
    for n in ns:
        h = 2 * math.pi / n
        x = np.arange(n) * h
        f = np.sin(x + 0.3)
        d = weno_flux_difference(f) / h
        errs.append(np.abs(d - np.cos(x + 0.3)).max())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    # Jiang-Shu weights keep fifth order on sin (no critical-point degeneracy)
    assert min(orders) > 4.8 and max(orders) < 5.5, (errs, orders)


# ---- WENO-Z weights (Borges et al. 2008, exponent 2) -------------------------
def test_wenoz_reduces_to_the_linear_scheme_when_beta1_equals_beta3(orc):
    # tau5 = |beta1 - beta3| = 0 gives alpha_k = c_k exactly, whatever beta2 is:
    # data symmetric about f_j (a = e, b = d) has beta1 = beta3.  The JS weights
    # on the same data are far from c (beta2 = 0 << beta1 in the first case).
    rng = np.random.default_rng(11)
    cases = [(1.0, 0.0, 0.0, 0.0, 1.0)] + [tuple(rng.uniform(-2, 2, size=3)) for _ in range(10)]
    for cs in cases:
        f = cs if len(cs) == 5 else (cs[0], cs[1], cs[2], cs[1], cs[0])
        r, parts = orc.weno5(*f, eps=1e-6, parts=True, weights=orc.WENO_Z)
        assert parts[0] == pytest.approx(parts[2], rel=1e-14)
        np.testing.assert_allclose(parts[3:6], [0.1, 0.6, 0.3], rtol=1e-14)
        printed = (2 * f[0] - 13 * f[1] + 47 * f[2] + 27 * f[3] - 3 * f[4]) / 60.0
        assert r == pytest.approx(printed, rel=1e-13, abs=1e-13)
    _, pj = orc.weno5(1.0, 0.0, 0.0, 0.0, 1.0, eps=1e-6, parts=True)
    assert pj[4] > 0.99  # JS puts nearly all weight on the smooth central stencil


def test_wenoz_shares_candidates_and_indicators_and_is_convex(orc):
    rng = np.random.default_rng(12)
    for _ in range(50):
        f = rng.normal(size=5)
        _, pz = orc.weno5(*f, eps=1e-6, parts=True, weights=orc.WENO_Z)
        _, pj = orc.weno5(*f, eps=1e-6, parts=True)
        np.testing.assert_array_equal(pz[[0, 1, 2, 6, 7, 8]], pj[[0, 1, 2, 6, 7, 8]])
        assert pz[3:6].sum() == pytest.approx(1.0, rel=1e-15) and np.all(pz[3:6] > 0)


def test_wenoz_rejects_a_discontinuous_stencil(orc):
    r, parts = orc.weno5(0.0, 0.0, 0.0, 0.0, 1.0, eps=1e-6, parts=True, weights=orc.WENO_Z)
    assert parts[5] < 1e-10 and abs(r) < 1e-10


def test_wenoz_keeps_fifth_order_at_critical_points(orc):
    # f(x) = sin(x - sin(x)/pi) has points with f' = 0 and f''' != 0 (Henrick et
    # al. 2005).  With eps negligible the JS weights drop to about third order
    # there; the Z weights with exponent 2 keep fifth (exponent 1 gives about 4).
    def orders(weights):
        errs = []
        for n in (64, 128, 256, 512):
            h = 2 * math.pi / n
            x = np.arange(n) * h + 0.1
            f = np.sin(x - np.sin(x) / math.pi)
            W = np.array([orc.weno5(f[(j - 2) % n], f[(j - 1) % n], f[j], f[(j + 1) % n], f[(j + 2) % n],
                                    1e-40, weights=weights) for j in range(n)])
            d = (W - np.roll(W, 1)) / h
            ex = np.cos(x - np.sin(x) / math.pi) * (1 - np.cos(x) / math.pi)
            errs.append(np.abs(d - ex).max())
        return [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]

    oz, oj = orders(orc.WENO_Z), orders(orc.WENO_JS)
    assert min(oz[1:]) > 4.6, oz
    assert max(oj[1:]) < 3.4, oj


# ---- mapped weights (Henrick, Aslam & Powers 2005) --------------------------
def _map_factored(w, d):
    # g(w) - d = (w - d)^3 / (d^2 + w (1 - 2 d)): the mapping's numerator minus d times
    # its denominator is (w - d)^3, so d is a triple fixed point (g(d) = d, g' = g'' = 0)
    return d + (w - d) ** 3 / (d * d + w * (1.0 - 2.0 * d))


def test_wenom_mapping_closed_form_and_fixed_points(orc):
    rng = np.random.default_rng(21)
    for d in (0.1, 0.6, 0.3):
        for w in rng.uniform(0.0, 1.0, size=40):
            assert orc.weno_map(w, d) == pytest.approx(_map_factored(w, d), rel=1e-13, abs=1e-15)
        assert orc.weno_map(0.0, d) == 0.0
        assert orc.weno_map(d, d) == pytest.approx(d, rel=1e-15)
        assert orc.weno_map(1.0, d) == pytest.approx(1.0, rel=1e-15)
        # flat to second order at d: the deviation shrinks like its cube
        for dw in (1e-2, 1e-3):
            assert abs(orc.weno_map(d + dw, d) - d) <= 2.0 * dw ** 3 / (d * d + d * (1 - 2 * d))


def test_wenom_weights_are_the_mapped_js_weights(orc):
    rng = np.random.default_rng(22)
    for _ in range(50):
        f = rng.normal(size=5)
        _, pm = orc.weno5(*f, eps=1e-6, parts=True, weights=orc.WENO_M)
        _, pj = orc.weno5(*f, eps=1e-6, parts=True)
        np.testing.assert_array_equal(pm[[0, 1, 2, 6, 7, 8]], pj[[0, 1, 2, 6, 7, 8]])
        g = np.array([_map_factored(pj[3 + k], dk) for k, dk in enumerate((0.1, 0.6, 0.3))])
        np.testing.assert_allclose(pm[3:6], g / g.sum(), rtol=1e-12)
        assert pm[3:6].sum() == pytest.approx(1.0, rel=1e-15) and np.all(pm[3:6] > 0)


def test_wenom_recovers_the_linear_weights_on_smooth_data(orc):
    # smooth data: the JS weights deviate from c by O(h^2); mapped, by O(h^6)
    x0, dev_j, dev_m = 0.3, [], []
    for h in (0.1, 0.05):
        f = [math.sin(x0 + (k - 2) * h) for k in range(5)]
        _, pj = orc.weno5(*f, eps=1e-40, parts=True)
        _, pm = orc.weno5(*f, eps=1e-40, parts=True, weights=orc.WENO_M)
        dev_j.append(np.abs(pj[3:6] - [0.1, 0.6, 0.3]).max())
        dev_m.append(np.abs(pm[3:6] - [0.1, 0.6, 0.3]).max())
    assert dev_m[0] < 1e-2 * dev_j[0]
    assert math.log2(dev_m[0] / dev_m[1]) > 5.0 and math.log2(dev_j[0] / dev_j[1]) < 2.5


def test_wenom_rejects_a_discontinuous_stencil(orc):
    r, parts = orc.weno5(0.0, 0.0, 0.0, 0.0, 1.0, eps=1e-6, parts=True, weights=orc.WENO_M)
    assert parts[5] < 1e-10 and abs(r) < 1e-10


def test_wenom_keeps_fifth_order_at_critical_points(orc):
    # the test function of Henrick et al. (2005), f' = 0 with f''' != 0: the mapped
    # weights keep fifth order where the JS weights drop to about third
    def orders(weights):
        errs = []
        for n in (64, 128, 256, 512):
            h = 2 * math.pi / n
            x = np.arange(n) * h + 0.1
            f = np.sin(x - np.sin(x) / math.pi)
            W = np.array([orc.weno5(f[(j - 2) % n], f[(j - 1) % n], f[j], f[(j + 1) % n], f[(j + 2) % n],
                                    1e-40, weights=weights) for j in range(n)])
            d = (W - np.roll(W, 1)) / h
            ex = np.cos(x - np.sin(x) / math.pi) * (1 - np.cos(x) / math.pi)
            errs.append(np.abs(d - ex).max())
        return [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]

    om = orders(orc.WENO_M)
    assert min(om[1:]) > 4.6, om
