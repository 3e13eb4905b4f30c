"""Plain PyTorch (CPU, float64) restatement of the oracle's discrete operator.

TEST INFRASTRUCTURE ONLY: used by the tests to obtain reference gradients of the
WENO5-Roe / central-viscous RHS and of RK4 trajectories by reverse-mode automatic
differentiation.  It follows the same equations as cns_oracle.c (paper Sec. 2.1
governing equations, Sec. 2.2 conservative differences, Roe flux with Harten's
fix and explicit eigenvector matrices, component-wise WENO5 with Jiang-Shu
weights, 4th-order central viscous derivatives, classical RK4), vectorised over
grid points with periodic rolls.  Its forward values are pinned to the C oracle
and its gradients to central differences of the C oracle (tests/test_torch_ref.py).

Arrays: a state is a tensor [5, nz, ny, nx]; direction d = 0, 1, 2 (x, y, z) is
tensor dimension -1, -2, -3.
"""
from __future__ import annotations

import math

import torch
import torch.utils.checkpoint as tcp

DIM = {0: -1, 1: -2, 2: -3}


def at(q, k, d):
    """q at offset +k along direction d (periodic)."""
    return torch.roll(q, shifts=-k, dims=DIM[d])


def primitives(u, gamma):
    rho = u[0]
    vel = u[1:4] / rho
    p = (gamma - 1.0) * (u[4] - 0.5 * rho * (vel * vel).sum(0))
    return rho, vel, p


def flux(u, d, gamma):
    """Sec. 2.1 convective flux along d."""
    rho, vel, p = primitives(u, gamma)
    vn = vel[d]
    f = [rho * vn, rho * vel[0] * vn, rho * vel[1] * vn, rho * vel[2] * vn, (u[4] + p) * vn]
    f[1 + d] = f[1 + d] + p
    return torch.stack(f)


def weno5(a, b, c, dd, e, eps, weights="js"):
    """Sec. 2.2 WENO5 value at j+1/2 from f_{j-2..j+2} (candidates, optimal
    weights 1/10, 6/10, 3/10, Jiang-Shu indicators, alpha = c/(eps+beta)^2);
    weights "z": WENO-Z, alpha = c (1 + (|beta1 - beta3| / (eps+beta))^2) (Borges
    et al. 2008); "m": the Jiang-Shu weights mapped by
    g(w) = w (c + c^2 - 3 c w + w^2) / (c^2 + w (1 - 2 c)) and renormalised
    (Henrick et al. 2005)."""
    f1 = a / 3.0 - 7.0 * b / 6.0 + 11.0 * c / 6.0
    f2 = -b / 6.0 + 5.0 * c / 6.0 + dd / 3.0
    f3 = c / 3.0 + 5.0 * dd / 6.0 - e / 6.0
    b1 = 13.0 / 12.0 * (a - 2 * b + c) ** 2 + 0.25 * (a - 4 * b + 3 * c) ** 2
    b2 = 13.0 / 12.0 * (b - 2 * c + dd) ** 2 + 0.25 * (b - dd) ** 2
    b3 = 13.0 / 12.0 * (c - 2 * dd + e) ** 2 + 0.25 * (3 * c - 4 * dd + e) ** 2
    opt = (0.1, 0.6, 0.3)
    if weights == "z":
        tau = torch.abs(b1 - b3)
        al = [ck * (1.0 + (tau / (eps + bk)) ** 2) for ck, bk in zip(opt, (b1, b2, b3))]
    else:
        al = [ck / (eps + bk) ** 2 for ck, bk in zip(opt, (b1, b2, b3))]
    s = al[0] + al[1] + al[2]
    w = [ak / s for ak in al]
    if weights == "m":
        g = [wk * (ck + ck * ck - 3.0 * ck * wk + wk * wk) / (ck * ck + wk * (1.0 - 2.0 * ck)) for ck, wk in zip(opt, w)]
        gs = g[0] + g[1] + g[2]
        w = [gk / gs for gk in g]
    return w[0] * f1 + w[1] * f2 + w[2] * f3


def roe_eigensystem(uL, uR, d, gamma):
    """Right eigenvectors X[r][c], left eigenvectors Xi[r][c] and eigenvalues of the
    flux Jacobian along d at the Roe average of uL and uR (lists of tensors)."""
    rL, vL, pL = primitives(uL, gamma)
    rR, vR, pR = primitives(uR, gamma)
    HL = (uL[4] + pL) / rL
    HR = (uR[4] + pR) / rR
    R = torch.sqrt(rR / rL)
    v = [(vL[k] + R * vR[k]) / (1.0 + R) for k in range(3)]
    H = (HL + R * HR) / (1.0 + R)
    q2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2]
    c2 = (gamma - 1.0) * (H - 0.5 * q2)
    c = torch.sqrt(c2)
    n, t1, t2 = d, (d + 1) % 3, (d + 2) % 3
    vn = v[n]
    z = torch.zeros_like(vn)
    one = torch.ones_like(vn)
    X = [[z for _ in range(5)] for _ in range(5)]
    Xi = [[z for _ in range(5)] for _ in range(5)]
    # columns: acoustic (vn - c), entropy, shear t1, shear t2, acoustic (vn + c)
    for col, sgn in ((0, -1.0), (4, 1.0)):
        X[0][col] = one
        for k in range(3):
            X[1 + k][col] = v[k] + (sgn * c if k == n else 0.0)
        X[4][col] = H + sgn * vn * c
    X[0][1] = one
    for k in range(3):
        X[1 + k][1] = v[k]
    X[4][1] = 0.5 * q2
    X[1 + t1][2] = one
    X[4][2] = v[t1]
    X[1 + t2][3] = one
    X[4][3] = v[t2]
    b1 = (gamma - 1.0) / c2
    b2 = 0.5 * q2 * b1
    for row, sgn in ((0, 1.0), (4, -1.0)):
        Xi[row][0] = 0.5 * (b2 + sgn * vn / c)
        for k in range(3):
            Xi[row][1 + k] = -0.5 * b1 * v[k] - (sgn * 0.5 / c if k == n else 0.0)
        Xi[row][4] = 0.5 * b1
    Xi[1][0] = 1.0 - b2
    for k in range(3):
        Xi[1][1 + k] = b1 * v[k]
    Xi[1][4] = -b1
    Xi[2][0] = -v[t1]
    Xi[2][1 + t1] = one
    Xi[3][0] = -v[t2]
    Xi[3][1 + t2] = one
    lam = [vn - c, vn, vn, vn, vn + c]
    return X, Xi, lam


def harten(lam, delta):
    a = torch.abs(lam)
    if delta <= 0.0:
        return a
    return torch.where(a >= delta, a, (lam * lam + delta * delta) / (2.0 * delta))


def interface_flux(u, d, ph):
    """F_{j+1/2} for every j along d (eq. (Roe) of Sec. 2.2)."""
    g, eps = ph["gamma"], ph["eps"]
    s = [at(u, m - 2, d) for m in range(6)]  # states at j-2 .. j+3
    f = [flux(sm, d, g) for sm in s]
    wt = ph.get("weights", "js")
    fL = weno5(f[0], f[1], f[2], f[3], f[4], eps, wt)
    fR = weno5(f[5], f[4], f[3], f[2], f[1], eps, wt)
    uL = weno5(s[0], s[1], s[2], s[3], s[4], eps, wt)
    uR = weno5(s[5], s[4], s[3], s[2], s[1], eps, wt)
    X, Xi, lam = roe_eigensystem(s[2], s[3], d, g)
    du = uR - uL
    w = [harten(lam[r], ph["delta"]) * sum(Xi[r][c] * du[c] for c in range(5)) for r in range(5)]
    diss = torch.stack([sum(X[r][c] * w[c] for c in range(5)) for r in range(5)])
    return 0.5 * (fL + fR) - 0.5 * diss


def rhs_hyp_dir(u, d, ph):
    F = interface_flux(u, d, ph)
    dx = ph["length"][d] / u.shape[DIM[d]]
    return -(F - at(F, -1, d)) / dx


def central_d(q, d, h):
    return (8.0 * (at(q, 1, d) - at(q, -1, d)) - (at(q, 2, d) - at(q, -2, d))) / (12.0 * h)


def viscous(u, ph):
    g, mu, pr = ph["gamma"], ph["mu"], ph["prandtl"]
    rho, vel, p = primitives(u, g)
    T = g * p / rho
    h = [ph["length"][d] / u.shape[DIM[d]] for d in range(3)]
    w = [vel[0], vel[1], vel[2], T]
    grad = [[central_d(w[a], b, h[b]) for b in range(3)] for a in range(4)]
    div = grad[0][0] + grad[1][1] + grad[2][2]
    tau = [[mu * ((grad[a][b] + grad[b][a]) - ((2.0 / 3.0) * div if a == b else 0.0)) for b in range(3)]
           for a in range(3)]
    kc = mu / ((g - 1.0) * pr)
    out = [torch.zeros_like(rho) for _ in range(5)]
    for d in range(3):
        q = -kc * grad[3][d]
        G = [tau[0][d], tau[1][d], tau[2][d], (vel[0] * tau[0][d] + vel[1] * tau[1][d] + vel[2] * tau[2][d]) - q]
        for c in range(4):
            out[1 + c] = out[1 + c] + central_d(G[c], d, h[d])
    return torch.stack(out)


def rhs(u, ph):
    r = rhs_hyp_dir(u, 0, ph) + rhs_hyp_dir(u, 1, ph) + rhs_hyp_dir(u, 2, ph)
    if ph["mu"] > 0:
        r = r + viscous(u, ph)
    return r


def rk4_step(u, dt, ph):
    k1 = rhs(u, ph)
    k2 = rhs(u + 0.5 * dt * k1, ph)
    k3 = rhs(u + 0.5 * dt * k2, ph)
    k4 = rhs(u + dt * k3, ph)
    return u + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


def tvdrk3_step(u, dt, ph):
    """Three-stage TVD Runge-Kutta step in Shu-Osher form (Sec. 5 integrator)."""
    u1 = u + dt * rhs(u, ph)
    u2 = 0.75 * u + 0.25 * (u1 + dt * rhs(u1, ph))
    return (1.0 / 3.0) * u + (2.0 / 3.0) * (u2 + dt * rhs(u2, ph))


def kinetic_energy(u):
    return 0.5 * ((u[1] ** 2 + u[2] ** 2 + u[3] ** 2) / u[0]).mean()


def ic_state(rho, vel, p, gamma):
    """Sec. 2.1 equation of state: conserved state from primitives."""
    return torch.stack([rho, rho * vel[0], rho * vel[1], rho * vel[2],
                        p / (gamma - 1.0) + 0.5 * rho * (vel * vel).sum(0)])


def make_phys(gamma=1.4, prandtl=0.72, mu=0.01, eps=1e-6, delta=1e-6, length=(2 * math.pi,) * 3, weights="js"):
    return dict(gamma=gamma, prandtl=prandtl, mu=mu, eps=eps, delta=delta, length=length, weights=weights)


def final_ke_and_grad(rho, vel, p, dt, nsteps, ph, step=None):
    """J = K(u^N) after nsteps steps (RK4 unless ``step`` is given) from the primitives,
    and dJ/dvel (with rho and p held fixed), by reverse-mode AD with per-step
    recomputation."""
    step = rk4_step if step is None else step
    vel = torch.as_tensor(vel, dtype=torch.float64).clone().requires_grad_(True)
    rho = torch.as_tensor(rho, dtype=torch.float64)
    p = torch.as_tensor(p, dtype=torch.float64)
    u = ic_state(rho, vel, p, ph["gamma"])
    for _ in range(nsteps):
        u = tcp.checkpoint(step, u, dt, ph, use_reentrant=False)
    J = kinetic_energy(u)
    (gv,) = torch.autograd.grad(J, vel)
    return float(J.detach()), gv.detach()


def rhs_vjp(u, rbar, ph):
    """(dR/du)^T rbar at u."""
    u = torch.as_tensor(u, dtype=torch.float64).clone().requires_grad_(True)
    r = rhs(u, ph)
    (g,) = torch.autograd.grad(r, u, grad_outputs=torch.as_tensor(rbar, dtype=torch.float64))
    return g.detach()


def rk4_vjp(u, ubar, dt, nsteps, ph, step=None):
    """(d u^N / d u^0)^T ubar for nsteps RK4 steps (or ``step``) from u."""
    step = rk4_step if step is None else step
    u0 = torch.as_tensor(u, dtype=torch.float64).clone().requires_grad_(True)
    x = u0
    for _ in range(nsteps):
        x = tcp.checkpoint(step, x, dt, ph, use_reentrant=False)
    (g,) = torch.autograd.grad(x, u0, grad_outputs=torch.as_tensor(ubar, dtype=torch.float64))
    return g.detach()
