"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test ties one part of the oracle to something other than itself:
brute-force quadrature, closed forms from gas dynamics (Euler/Navier-Stokes
fluxes, kinetic flux-vector splitting), limits stated in the paper, symmetries,
exact Riemann solutions and analytic decay rates.
"""
import json
import math
import os

import mpmath
import numpy as np
import pytest

import oracle
from inputs import cases as C
from quadrature import Maxwell, lin, maxwell_from_cons, psi_list, time_weights_quad

HERE = os.path.dirname(os.path.abspath(__file__))
G = 1.4


def cons(rho, U, p, gamma=G):
    U = np.asarray(U, dtype=float)
    return np.array([rho] + list(rho * U) + [p / (gamma - 1.0) + 0.5 * rho * float(U @ U)])


def rand_prim(rng, dim, umax=1.0):
    return float(rng.uniform(0.5, 2.0)), rng.uniform(-umax, umax, size=dim), float(rng.uniform(0.5, 2.0))


def rand_face(rng, dim, slope=0.3, jump=True):
    rl, Ul, pl = rand_prim(rng, dim)
    if jump:
        rr, Ur, pr = rand_prim(rng, dim)
    else:
        rr, Ur, pr = rl, Ul.copy(), pl
    Wl, Wr = cons(rl, Ul, pl), cons(rr, Ur, pr)
    sl = slope * rng.uniform(-1, 1, size=dim + 2) * np.abs(Wl)
    sr = slope * rng.uniform(-1, 1, size=dim + 2) * np.abs(Wr)
    dxl, dxr = float(rng.uniform(0.02, 0.05)), float(rng.uniform(0.02, 0.05))
    return dict(Wl=Wl, Wr=Wr, sl=sl, sr=sr, Wi=Wl - sl * dxl, Wi1=Wr + sr * dxr, dxl=dxl, dxr=dxr)


def euler_flux(W, dim, gamma=G):
    """Textbook Euler flux through an x-normal face (works on complex input)."""
    rho = W[0]
    U = [W[1 + d] / rho for d in range(dim)]
    E = W[dim + 1]
    p = (gamma - 1.0) * (E - 0.5 * rho * sum(u * u for u in U))
    F = [rho * U[0]] + [rho * U[0] * U[d] + (p if d == 0 else 0.0) for d in range(dim)] + [U[0] * (E + p)]
    return np.array(F)


def jac_vec(W, v, dim):
    """J(W) v by complex-step differentiation (exact to rounding)."""
    h = 1e-30
    return np.imag(euler_flux(np.asarray(W, dtype=complex) + 1j * h * np.asarray(v), dim)) / h


def rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


# ---------------------------------------------------------------------------
# P1: Maxwellian moments (full line and half lines) against 40-digit quadrature
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("U,lam", [(0.0, 1.0), (0.7, 0.35), (-1.3, 2.5), (2.4, 3.0), (-0.2, 0.05)])
def test_p1_moments_vs_mpmath(U, lam):
    mpmath.mp.dps = 40
    M = oracle.moments_u(U, lam)
    dens = lambda u: mpmath.sqrt(lam / mpmath.pi) * mpmath.exp(-lam * (u - U) ** 2)
    for n in range(9):
        pos = mpmath.quad(lambda u: u ** n * dens(u), [0, U + 5, mpmath.inf]) if U + 5 > 0 else \
            mpmath.quad(lambda u: u ** n * dens(u), [0, mpmath.inf])
        neg = mpmath.quad(lambda u: u ** n * dens(u), [-mpmath.inf, min(U - 5, -1), 0])
        scale = float(pos + (-1) ** n * neg)          # <|u|^n>, never cancels
        assert abs(M[1, n] - float(pos)) <= 2e-15 * scale * (n + 1)
        assert abs(M[2, n] - float(neg)) <= 2e-15 * scale * (n + 1)
        assert abs(M[0, n] - float(pos + neg)) <= 2e-15 * scale * (n + 1)


# ---------------------------------------------------------------------------
# Time weights of the Kogan solution (and the paper's alpha(eps), P13)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("ratio", [0.0, 1e-6, 1e-3, 0.1, 0.49, 0.51, 1.7, 12.0, 1e4])
def test_kogan_weights_vs_time_quadrature(ratio):
    dt = 2.3e-3
    tau = ratio * dt
    k = oracle.kogan(tau, dt)
    q = time_weights_quad(tau, dt)
    scales = [dt, max(tau, dt) ** 2, dt * dt, dt, max(tau, dt) ** 2, max(tau, dt) ** 2]
    for i in range(6):
        assert abs(k[i] - q[i]) <= 1e-13 * scales[i], (i, k[i], q[i])
    if tau > 0:
        # ratios used by the time-integrated compatibility condition
        assert k[6] == pytest.approx(q[1] / (tau * q[0]), rel=1e-11, abs=1e-14)
        assert k[7] == pytest.approx(q[4] / (tau * q[0]), rel=1e-11, abs=1e-14)
        assert k[8] == pytest.approx(q[5] / (tau * q[0]), rel=1e-11, abs=1e-14)
        # gam3/dt is the paper's alpha(eps) = eps (1 - e^{-1/eps}), eps = tau/dt
        eps = tau / dt
        assert k[3] / dt == pytest.approx(eps * (1.0 - math.exp(-1.0 / eps)), rel=1e-14)
    else:
        assert (k[6], k[7], k[8]) == (-1.0, 0.0, 0.0)
    # gam0 + gam3 = dt: the interface state terms of the compatibility condition cancel
    assert abs(k[0] + k[3] - dt) <= 1e-15 * dt


# ---------------------------------------------------------------------------
# P2: moment systems <psi psi^T>_g x = r against a quadrature-assembled matrix and
#     the closed form of Xu's scheme
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dim", [2, 3])
def test_p2_moment_solve(dim):
    rng = np.random.default_rng(10 + dim)
    for _ in range(4):
        rho, U, p = rand_prim(rng, dim)
        lam = rho / (2 * p)
        K = 2.0 / (G - 1.0) - dim
        r = rng.normal(size=dim + 2)
        x = oracle.moment_solve(dim, G, rho, U, lam, r)
        mw = Maxwell(1.0, U, lam, K, dim, nh=16, nlag=8)
        Mq = np.array([[mw.integrate(lambda u, v, w, X, m=m, n=n: psi_list(dim, u, v, w, X)[m] *
                                     psi_list(dim, u, v, w, X)[n]) for n in range(dim + 2)]
                       for m in range(dim + 2)])
        assert rel(Mq @ x, r) < 1e-13
        # closed form (b = total degrees of freedom)
        b = 2.0 / (G - 1.0)
        U2 = float(U @ U)
        aE = 4 * lam * lam / b * (2 * r[-1] - 2 * float(U @ r[1:1 + dim]) + r[0] * (U2 - b / (2 * lam)))
        ad = 2 * lam * (r[1:1 + dim] - U * r[0]) - U * aE
        a0 = r[0] - float(U @ ad) - 0.5 * aE * (U2 + b / (2 * lam))
        assert rel(x, np.concatenate([[a0], ad, [aE]])) < 1e-12


# ---------------------------------------------------------------------------
# Defining conditions of every coefficient, checked by quadrature
# ---------------------------------------------------------------------------
def _maxwells(fc, info, dim, nh=16):
    out = {}
    for nm, W in (("l", fc["Wl"]), ("r", fc["Wr"]), ("0", info["W0"])):
        rho, U, lam, K, _ = maxwell_from_cons(W, dim, G)
        out[nm] = Maxwell(rho, U, lam, K, dim, nh=nh, nlag=8)
    return out


@pytest.mark.parametrize("dim", [2, 3])
def test_coefficient_definitions_by_quadrature(dim):
    rng = np.random.default_rng(20 + dim)
    fc = rand_face(rng, dim)
    dt = 1e-2
    res = oracle.face_flux(dim, fc["Wl"], fc["Wr"], fc["sl"], fc["sr"], fc["Wi"], fc["Wi1"], fc["dxl"],
                           fc["dxr"], 2e-3, 5.0, 3.0, dt, mu=2e-3, c_a=0.3)
    inf = res["info"]
    mw = _maxwells(fc, inf, dim)
    P = lambda u, v, w, X: psi_list(dim, u, v, w, X)
    # interface state: left Maxwellian over u>0, right over u<0
    W0q = mw["l"].integrate(P, "pos") + mw["r"].integrate(P, "neg")
    assert rel(inf["W0"], W0q) < 1e-13
    for s, slope in (("l", fc["sl"]), ("r", fc["sr"])):
        a, A = inf["a_" + s], inf["A_" + s]
        # rho <psi (a.psi)>_g = dW/dx
        got = mw[s].integrate(lambda u, v, w, X: [p * lin(a, dim, u, v, w, X) for p in P(u, v, w, X)])
        assert rel(got, slope) < 1e-12
        # compatibility at t = 0:  <psi (a.psi u + A.psi)>_g = 0
        comp = mw[s].integrate(lambda u, v, w, X: [p * (u * lin(a, dim, u, v, w, X) + lin(A, dim, u, v, w, X))
                                                   for p in P(u, v, w, X)])
        scale = np.max(np.abs(mw[s].integrate(lambda u, v, w, X: [p * u * lin(a, dim, u, v, w, X)
                                                                  for p in P(u, v, w, X)])))
        assert np.max(np.abs(comp)) < 1e-12 * scale
    # equilibrium slopes through W0
    for s, target in (("abar_l", (inf["W0"] - fc["Wi"]) / fc["dxl"]), ("abar_r", (fc["Wi1"] - inf["W0"]) / fc["dxr"])):
        got = mw["0"].integrate(lambda u, v, w, X: [p * lin(inf[s], dim, u, v, w, X) for p in P(u, v, w, X)])
        assert rel(got, target) < 1e-12


def _bruteforce_flux(fc, res, dim, dt, nh=16):
    """F, G and heat flux of the exact Kogan solution by quadrature in t and velocity space."""
    inf = res["info"]
    mw = _maxwells(fc, inf, dim, nh)
    tau = inf["tau"]
    gam = time_weights_quad(tau, dt)
    U0 = np.zeros(3)
    U0[:dim] = maxwell_from_cons(inf["W0"], dim, G)[1]
    L = lambda a: (lambda u, v, w, X: lin(a, dim, u, v, w, X))
    one = lambda u, v, w, X: 1.0 + 0 * u
    # (time weight index, maxwellian, u range, polynomial factor)
    terms = [
        (0, "0", "all", one),
        (1, "0", "pos", lambda u, v, w, X: u * L(inf["abar_l"])(u, v, w, X)),
        (1, "0", "neg", lambda u, v, w, X: u * L(inf["abar_r"])(u, v, w, X)),
        (2, "0", "all", L(inf["Abar"])),
        (3, "l", "pos", one),
        (4, "l", "pos", lambda u, v, w, X: u * L(inf["a_l"])(u, v, w, X)),
        (5, "l", "pos", L(inf["A_l"])),
        (3, "r", "neg", one),
        (4, "r", "neg", lambda u, v, w, X: u * L(inf["a_r"])(u, v, w, X)),
        (5, "r", "neg", L(inf["A_r"])),
    ]
    rho_w = {"0": mw["0"], "l": mw["l"], "r": mw["r"]}
    F = np.zeros(dim + 2)
    Gv = np.zeros(dim + 2)
    q = 0.0

    def heat(u, v, w, X):
        c2 = (u - U0[0]) ** 2 + (v - U0[1]) ** 2 + ((w - U0[2]) ** 2 if dim == 3 else 0.0) + X
        return (u - U0[0]) * 0.5 * c2

    for gi, m, rg, poly in terms:
        F += gam[gi] * rho_w[m].integrate(lambda u, v, w, X: [u * p * poly(u, v, w, X)
                                                                for p in psi_list(dim, u, v, w, X)], rg)
        Gv += gam[gi] * rho_w[m].integrate(lambda u, v, w, X: [p * poly(u, v, w, X)
                                                                 for p in psi_list(dim, u, v, w, X)], rg)
        q += gam[gi] * rho_w[m].integrate(lambda u, v, w, X: heat(u, v, w, X) * poly(u, v, w, X), rg)
    return F, Gv, q


@pytest.mark.parametrize("dim,ratio", [(2, 0.05), (2, 1.0), (2, 30.0), (3, 0.7)])
def test_p16_flux_bruteforce(dim, ratio):
    """P16: the whole per-face formula against quadrature of the exact Kogan solution."""
    rng = np.random.default_rng(30 + dim + int(ratio * 10))
    fc = rand_face(rng, dim)
    dt = 1e-2
    # pick mu so that tau/dt is about `ratio`
    p0 = 1.0
    mu = ratio * dt * p0
    pr = 0.72
    res = oracle.face_flux(dim, fc["Wl"], fc["Wr"], fc["sl"], fc["sr"], fc["Wi"], fc["Wi1"], fc["dxl"],
                           fc["dxr"], 1e-3, 4.0, 2.0, dt, prandtl=pr, mu=mu, c_a=0.2)
    F, Gq, q = _bruteforce_flux(fc, res, dim, dt)
    F[-1] += (1.0 / pr - 1.0) * q
    assert rel(res["F"], F) < 1e-12
    assert rel(res["G"], Gq) < 1e-12
    assert abs(res["q"] - q) < 1e-12 * np.max(np.abs(F))
    # time-integrated compatibility: int int psi g = int int psi f
    inf = res["info"]
    mw0 = _maxwells(fc, inf, dim)["0"]
    Ab = mw0.integrate(lambda u, v, w, X: [p * lin(inf["Abar"], dim, u, v, w, X)
                                           for p in psi_list(dim, u, v, w, X)])
    Gg = dt * inf["W0"] + 0.5 * dt * dt * Ab
    assert rel(Gq, Gg) < 1e-12


# ---------------------------------------------------------------------------
# P5: continuous linear data -> Navier-Stokes flux + second-order time term
# ---------------------------------------------------------------------------
def ns_flux_1d(W, dW, dim, mu_eff, gamma=G):
    """Euler + viscous flux through an x-face with gradients only along x.
    sigma_xx = mu (2 - 2/b) U_x, sigma_xt = mu V_x, q = -mu c_p T_x, c_p = (b+2)/2, T = p/rho."""
    b = 2.0 / (gamma - 1.0)
    rho = W[0]
    U = W[1:1 + dim] / rho
    p = (gamma - 1.0) * (W[-1] - 0.5 * rho * float(U @ U))
    drho = dW[0]
    dU = (dW[1:1 + dim] - U * drho) / rho
    dp = (gamma - 1.0) * (dW[-1] - 0.5 * drho * float(U @ U) - rho * float(U @ dU))
    dT = (dp - p / rho * drho) / rho
    sig = mu_eff * dU.copy()
    sig[0] = mu_eff * (2.0 - 2.0 / b) * dU[0]
    heat = -mu_eff * (b + 2.0) / 2.0 * dT
    F = euler_flux(W, dim, gamma)
    F[1:1 + dim] -= sig
    F[-1] += -float(U @ sig) + heat
    return F


@pytest.mark.parametrize("dim", [2, 3])
def test_p5_continuous_data_navier_stokes(dim):
    rng = np.random.default_rng(40 + dim)
    for trial in range(4):
        rho, U, p = rand_prim(rng, dim)
        W = cons(rho, U, p)
        dW = 0.4 * rng.uniform(-1, 1, size=dim + 2) * np.abs(W)
        dxl, dxr = 0.03, 0.02
        dt = [1e-3, 5e-3, 2e-2, 4e-2][trial]
        mu, kf, wf, Sf = 3e-3, 2e-3, 3.0, 5.0
        res = oracle.face_flux(dim, W, W, dW, dW, W - dW * dxl, W + dW * dxr, dxl, dxr, kf, wf, Sf, dt,
                               prandtl=1.0, mu=mu, c_a=0.7)
        tau = res["info"]["tau"]
        # tau = mu/p + k/(omega T sqrt(1 + eta^2)); tau_a vanishes without a pressure jump
        eta = Sf / (0.09 * wf)
        assert tau == pytest.approx(mu / p + kf / (wf * (p / rho) * math.sqrt(1 + eta * eta)), rel=1e-13)
        expect = dt * ns_flux_1d(W, dW, dim, tau * p) - 0.5 * dt * dt * jac_vec(W, jac_vec(W, dW, dim), dim)
        assert rel(res["F"], expect) < 2e-13, trial
        assert rel(res["info"]["W0"], W) < 1e-15
        assert rel(res["info"]["Abar"], res["info"]["A_l"]) < 1e-11


@pytest.mark.parametrize("dim", [2, 3])
def test_p5_prandtl_correction_heat_flux(dim):
    """With Pr != 1 only the energy flux changes, by (1/Pr - 1) q; as dt -> 0, q/dt is the
    Navier-Stokes heat flux -mu c_p dT/dx with mu = tau p."""
    rng = np.random.default_rng(50 + dim)
    rho, U, p = rand_prim(rng, dim)
    W = cons(rho, U, p)
    dW = 0.3 * rng.uniform(-1, 1, size=dim + 2) * np.abs(W)
    pr = 0.72
    vals = []
    for dt in (1e-4, 2e-4):
        a = oracle.face_flux(dim, W, W, dW, dW, W - dW * 0.02, W + dW * 0.02, 0.02, 0.02, 0.0, 1.0, 0.0, dt,
                             prandtl=1.0, mu=2e-3)
        b = oracle.face_flux(dim, W, W, dW, dW, W - dW * 0.02, W + dW * 0.02, 0.02, 0.02, 0.0, 1.0, 0.0, dt,
                             prandtl=pr, mu=2e-3)
        assert np.all(a["F"][:-1] == b["F"][:-1])
        vals.append((b["F"][-1] - a["F"][-1]) / ((1 / pr - 1) * dt))
    q0 = 2 * vals[0] - vals[1]            # linear extrapolation to dt = 0
    tau = 2e-3 / p
    bdof = 2.0 / (G - 1.0)
    drho = dW[0]
    Uv = W[1:1 + dim] / rho
    dU = (dW[1:1 + dim] - Uv * drho) / rho
    dp = (G - 1.0) * (dW[-1] - 0.5 * drho * float(Uv @ Uv) - rho * float(Uv @ dU))
    dT = (dp - p / rho * drho) / rho
    assert q0 == pytest.approx(-tau * p * (bdof + 2) / 2 * dT, rel=1e-8)


# ---------------------------------------------------------------------------
# P6: tau = 0 -> the flux is dt F_Euler(W0) + dt^2/2 rho0 <u psi Abar.psi> (hydrodynamic limit)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dim", [2, 3])
def test_p6_euler_limit(dim):
    rng = np.random.default_rng(60 + dim)
    fc = rand_face(rng, dim)
    ys = []
    dts = (1e-3, 3e-3)
    for dt in dts:
        r = oracle.face_flux(dim, fc["Wl"], fc["Wr"], fc["sl"], fc["sr"], fc["Wi"], fc["Wi1"], fc["dxl"],
                             fc["dxr"], 0.0, 1.0, 0.0, dt, prandtl=1.0, mu=0.0, c_a=0.0)
        assert r["info"]["tau"] == 0.0
        ys.append(r["F"] / dt)
        W0 = r["info"]["W0"]
    intercept = (dts[1] * ys[0] - dts[0] * ys[1]) / (dts[1] - dts[0])
    assert rel(intercept, euler_flux(W0, dim)) < 1e-12
    # slope: Abar from the tau -> 0 limit of the compatibility condition, by quadrature
    inf = r["info"]
    rho0, U0, lam0, K, _ = maxwell_from_cons(W0, dim, G)
    m0 = Maxwell(rho0, U0, lam0, K, dim, nh=16, nlag=8)
    P = lambda u, v, w, X: psi_list(dim, u, v, w, X)
    lhs = m0.integrate(lambda u, v, w, X: [p * lin(inf["Abar"], dim, u, v, w, X) for p in P(u, v, w, X)])
    rhs = -(m0.integrate(lambda u, v, w, X: [u * p * lin(inf["abar_l"], dim, u, v, w, X) for p in P(u, v, w, X)], "pos")
            + m0.integrate(lambda u, v, w, X: [u * p * lin(inf["abar_r"], dim, u, v, w, X) for p in P(u, v, w, X)], "neg"))
    assert rel(lhs, rhs) < 1e-12
    slope = m0.integrate(lambda u, v, w, X: [u * p * lin(inf["Abar"], dim, u, v, w, X) for p in P(u, v, w, X)])
    assert rel((ys[1] - ys[0]) / (dts[1] - dts[0]), 0.5 * slope) < 1e-9


# ---------------------------------------------------------------------------
# P7: tau/dt -> infinity, piecewise-constant data -> kinetic flux-vector splitting
# ---------------------------------------------------------------------------
def kfvs(W, dim, sign, gamma=G):
    """Textbook equilibrium-flux-method (Pullin / Deshpande) half fluxes, x-normal face."""
    rho = W[0]
    U = W[1:1 + dim] / rho
    p = (gamma - 1.0) * (W[-1] - 0.5 * rho * float(U @ U))
    lam = rho / (2 * p)
    b = 2.0 / (gamma - 1.0)
    u = U[0]
    A = 0.5 * math.erfc(-sign * math.sqrt(lam) * u)
    B = sign * math.exp(-lam * u * u) / (2.0 * math.sqrt(math.pi * lam))
    m0, m1 = A, u * A + B
    m2 = (u * u + 1 / (2 * lam)) * A + u * B
    m3 = (u ** 3 + 3 * u / (2 * lam)) * A + (u * u + 1 / lam) * B
    tan = float(U[1:] @ U[1:]) + (b - 1) / (2 * lam)   # <v^2 + w^2 + xi^2>
    F = [rho * m1, rho * m2] + [rho * U[d] * m1 for d in range(1, dim)] + [0.5 * rho * (m3 + m1 * tan)]
    return np.array(F)


@pytest.mark.parametrize("dim", [2, 3])
def test_p7_collisionless_limit_kfvs(dim):
    rng = np.random.default_rng(70 + dim)
    fc = rand_face(rng, dim, slope=0.0)
    z = np.zeros(dim + 2)
    dt = 1e-3
    r = oracle.face_flux(dim, fc["Wl"], fc["Wr"], z, z, fc["Wl"], fc["Wr"], 0.02, 0.02, 0.0, 1.0, 0.0, dt,
                         prandtl=1.0, mu=1e5, c_a=0.0)
    assert r["info"]["tau"] / dt > 1e7
    assert rel(r["F"] / dt, kfvs(fc["Wl"], dim, +1) + kfvs(fc["Wr"], dim, -1)) < 1e-6


# ---------------------------------------------------------------------------
# P8: consistency and symmetries of one interface
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dim", [2, 3])
def test_p8_symmetries(dim):
    rng = np.random.default_rng(80 + dim)
    kw = dict(prandtl=0.72, mu=2e-3, c_a=0.5)
    args = (1e-3, 4.0, 2.0, 5e-3)
    # equal states -> interface state equals them
    fc = rand_face(rng, dim, jump=False)
    r = oracle.face_flux(dim, fc["Wl"], fc["Wr"], fc["sl"], fc["sr"], fc["Wi"], fc["Wi1"], fc["dxl"],
                         fc["dxr"], *args, **kw)
    assert rel(r["info"]["W0"], fc["Wl"]) < 2e-16 * 8
    fc = rand_face(rng, dim)
    base = oracle.face_flux(dim, fc["Wl"], fc["Wr"], fc["sl"], fc["sr"], fc["Wi"], fc["Wi1"], fc["dxl"],
                            fc["dxr"], *args, **kw)["F"]
    # mirror x -> -x: swap sides, flip normal momentum and slopes
    R = np.ones(dim + 2)
    R[1] = -1.0
    mir = oracle.face_flux(dim, R * fc["Wr"], R * fc["Wl"], -R * fc["sr"], -R * fc["sl"], R * fc["Wi1"],
                           R * fc["Wi"], fc["dxr"], fc["dxl"], *args, **kw)["F"]
    assert rel(mir, -R * base) < 1e-13
    # tangential Galilean shift V -> V + c
    c = 0.37

    def shift(W):
        W = W.copy()
        E = W[-1] + c * W[2] + 0.5 * c * c * W[0]
        W[2] = W[2] + c * W[0]
        W[-1] = E
        return W

    sh = oracle.face_flux(dim, shift(fc["Wl"]), shift(fc["Wr"]), shift(fc["sl"]), shift(fc["sr"]),
                          shift(fc["Wi"]), shift(fc["Wi1"]), fc["dxl"], fc["dxr"], *args, **kw)["F"]
    expect = base.copy()
    expect[2] = base[2] + c * base[0]
    expect[-1] = base[-1] + c * base[2] + 0.5 * c * c * base[0]
    assert rel(sh, expect) < 1e-13


# ---------------------------------------------------------------------------
# P11: turbulent relaxation time -> Wilcox eddy viscosity
# ---------------------------------------------------------------------------
def test_p11_turbulent_tau():
    rho0, p0, kf, wf = 1.3, 0.8, 2e-2, 7.0
    t = oracle.tau_value(0.0, 0.0, 0.09, rho0, p0, p0, p0, kf, wf, 0.0, 1e-3)
    assert t * p0 == pytest.approx(rho0 * kf / wf, rel=1e-15)       # mu_t = rho k / omega
    # strong strain: tau_t -> (k/omega)/(T eta), eta = S/(C_mu omega)
    S = 1e9
    t = oracle.tau_value(0.0, 0.0, 0.09, rho0, p0, p0, p0, kf, wf, S, 1e-3)
    assert t == pytest.approx((kf / wf) / ((p0 / rho0) * S / (0.09 * wf)), rel=1e-12)
    # artificial part: C_a |dp| / (p_l + p_r) dt, laminar part mu/p0
    t = oracle.tau_value(1e-3, 0.5, 0.09, rho0, p0, 1.0, 3.0, 0.0, wf, 0.0, 2e-3)
    assert t == pytest.approx(1e-3 / p0 + 0.5 * 2.0 / 4.0 * 2e-3, rel=1e-15)


# ---------------------------------------------------------------------------
# Grid level
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dim,bc", [
    (2, None),
    (2, [["dirichlet", "outflow"], ["periodic", "periodic"]]),
    (2, [["outflow", "outflow"], ["profile", "dirichlet"]]),
    (3, None),
    (3, [["periodic", "periodic"], ["outflow", "dirichlet"], ["profile", "outflow"]]),
])
def test_p4_free_stream(dim, bc):
    n = (14, 11, 1) if dim == 2 else (7, 6, 5)
    case = C.uniform_flow(dim=dim, n=n, bc=bc)
    r = oracle.run(case, 3)
    F = euler_flux(case.W[:, 0, 0, 0] if dim == 2 else case.W[:, 0, 0, 0], dim)
    assert np.max(np.abs(r["W"] - case.W)) <= 1e-14 * np.max(np.abs(case.W))
    assert np.max(r["res"]) <= 1e-13 * np.max(np.abs(F))


def test_p4_free_stream_at_rest_with_walls():
    case = C.uniform_flow(dim=2, n=(10, 9, 1), vel=(0.0, 0.0, 0.0),
                          bc=[["wall", "wall"], ["wall", "outflow"]])
    r = oracle.run(case, 3)
    assert np.max(np.abs(r["W"] - case.W)) <= 1e-14


def test_p10_conservation_periodic():
    case = C.mixing_layer(32, seed=3)
    vol = np.outer(np.diff(case.xf[1]), np.diff(case.xf[0]))
    before = np.array([np.sum(case.W[m, 0] * vol) for m in range(4)])
    r = oracle.run(case, 20)
    after = np.array([np.sum(r["W"][m, 0] * vol) for m in range(4)])
    scale = np.array([np.sum(np.abs(case.W[m, 0]) * vol) for m in range(4)])
    assert np.all(np.abs(after - before) <= 1e-13 * scale)


def test_p9_rotation_transpose():
    """A y-face flux equals the x-face flux of the transposed state: running the transposed
    problem gives the transposed result."""
    case = C.mixing_layer(24, seed=5)
    case.xf = [case.xf[0], np.concatenate([[0.0], np.cumsum(np.linspace(1, 2, 24))]) / np.sum(np.linspace(1, 2, 24))]
    tr = case.copy()
    tr.n = (case.n[1], case.n[0], 1)
    tr.xf = [case.xf[1], case.xf[0]]
    tr.W = np.ascontiguousarray(np.stack([case.W[0], case.W[2], case.W[1], case.W[3]]).transpose(0, 1, 3, 2))
    tr.k = np.ascontiguousarray(case.k.transpose(0, 2, 1))
    tr.omega = np.ascontiguousarray(case.omega.transpose(0, 2, 1))
    a = oracle.run(case, 5)["W"]
    b = oracle.run(tr, 5)["W"]
    bt = np.stack([b[0], b[2], b[1], b[3]]).transpose(0, 1, 3, 2)
    assert rel(bt, a) < 1e-13


def test_p9_periodic_seam_invariance():
    """A periodic axis has no special point: relabelling the cells of a stretched periodic
    grid cyclically (moving the seam) gives the cyclically relabelled result."""
    rng = np.random.default_rng(17)
    n, k = 24, 7
    w = rng.uniform(0.5, 2.0, size=n)
    w /= w.sum()

    def make(widths, roll):
        c = C.mixing_layer(n, seed=4)
        xf = np.concatenate([[0.0], np.cumsum(widths)])
        c.xf = [xf, xf.copy()]
        c.W = np.roll(np.roll(c.W, -roll, axis=3), -roll, axis=2).copy()
        c.k = np.roll(np.roll(c.k, -roll, axis=2), -roll, axis=1).copy()
        c.omega = np.roll(np.roll(c.omega, -roll, axis=2), -roll, axis=1).copy()
        return c

    a = oracle.run(make(w, 0), 4)["W"]
    b = oracle.run(make(np.roll(w, -k), k), 4)["W"]
    b = np.roll(np.roll(b, k, axis=3), k, axis=2)
    assert rel(b, a) < 1e-12


def test_p9_y_invariant_rows_identical():
    case = C.sod_tube(40, ny=4, t_end=0.0, steps=10)
    r = oracle.run(case, 10)
    for j in range(1, 4):
        assert np.array_equal(r["W"][:, 0, j], r["W"][:, 0, 0])


def test_ghost_fill_rules():
    case = C.uniform_flow(dim=2, n=(5, 4, 1), vel=(0.3, -0.2, 0.0),
                          bc=[["wall", "outflow"], ["dirichlet", "profile"]])
    rng = np.random.default_rng(1)
    W = case.W * (1 + 0.1 * rng.uniform(-1, 1, size=case.W.shape))
    case.bc_data[1][0] = cons(0.9, [0.1, 0.2], 1.1)
    case.bc_data[1][1] = np.stack([cons(1 + 0.1 * i, [0.1 * i, 0.0], 1.0) for i in range(5)], axis=1)
    We = oracle.ghost_fill(case, W)[:, 0]        # (4, ny+4, nx+4)
    I = lambda j, i: (j + 2, i + 2)
    # x-low wall: mirror, momentum negated
    for j in range(4):
        for g, s in ((-1, 0), (-2, 1)):
            exp = W[:, 0, j, s] * np.array([1, -1, -1, 1])
            assert np.array_equal(We[(slice(None),) + I(j, g)], exp)
        # x-high outflow: copy of the last cell
        for g in (5, 6):
            assert np.array_equal(We[(slice(None),) + I(j, g)], W[:, 0, j, 4])
    # y-low dirichlet, everywhere along x including the x-ghost columns
    for i in range(-2, 7):
        for g in (-1, -2):
            assert np.array_equal(We[(slice(None),) + I(g, i)], case.bc_data[1][0])
    # y-high profile indexed by the (clamped) column
    for i in range(-2, 7):
        for g in (4, 5):
            assert np.array_equal(We[(slice(None),) + I(g, i)], case.bc_data[1][1][:, min(max(i, 0), 4)])


def test_cfl_dt_uniform():
    case = C.uniform_flow(dim=2, n=(8, 6, 1), stretched=False, rho=1.3, vel=(0.7, -0.4, 0), p=0.9)
    case.k[:] = 0.02
    case.omega[:] = 4.0
    dx, dy = 1 / 8, 1 / 6
    c = math.sqrt(G * 0.9 / 1.3)
    nu = (case.mu + 1.3 * 0.02 / 4.0) / 1.3 * max(4 / 3, G / case.prandtl)
    rate = (0.7 + c) / dx + (0.4 + c) / dy + 2 * nu * (1 / dx ** 2 + 1 / dy ** 2)
    assert oracle.cfl_dt(case) == pytest.approx(case.cfl / rate, rel=1e-14)


def test_strain_rate_linear_field():
    """Central differences are exact for a linear velocity field on interior cells."""
    n = 12
    case = C.uniform_flow(dim=2, n=(n, n, 1), stretched=False, bc=[["outflow", "outflow"]] * 2)
    x = (np.arange(n) + 0.5) / n
    Y, X = np.meshgrid(x, x, indexing="ij")
    U, V = 0.3 * X + 0.2 * Y, -0.1 * X + 0.4 * Y
    case.W = C.cons_from_prim(np.ones_like(U), [U, V], np.ones_like(U), G)[:, None]
    S = oracle.strain(case)[0]
    sxx, syy, sxy = 0.3, 0.4, 0.5 * (0.2 - 0.1)
    ex = math.sqrt(2 * (sxx ** 2 + syy ** 2 + 2 * sxy ** 2))
    assert np.allclose(S[1:-1, 1:-1], ex, rtol=1e-13)


def test_inputs_oblique_shock_against_chart():
    g = json.load(open(os.path.join(HERE, "golden", "oblique_shock.json")))
    beta, p21, r21 = C.oblique_shock(g["M1"], g["theta_deg"])
    assert math.degrees(beta) == pytest.approx(g["beta_deg"], rel=g["tol_rel"])
    assert p21 == pytest.approx(g["p2_p1"], rel=g["tol_rel"])
    assert r21 == pytest.approx(g["rho2_rho1"], rel=g["tol_rel"])


# ---------------------------------------------------------------------------
# P12: Sod's shock tube against the exact Riemann solution
# ---------------------------------------------------------------------------
def test_p12_sod_exact():
    import exact_riemann as ER
    star = json.load(open(os.path.join(HERE, "golden", "sod_star.json")))
    ps, us, rl, rr = ER.star_state((1, 0, 1), (0.125, 0, 0.1))
    assert ps == pytest.approx(star["p_star"], abs=1e-5)
    assert us == pytest.approx(star["u_star"], abs=1e-5)
    assert rl == pytest.approx(star["rho_star_left"], abs=1e-5)
    assert rr == pytest.approx(star["rho_star_right"], abs=1e-5)
    errs = []
    for N in (100, 200, 400):
        case = C.sod_tube(N, ny=2, t_end=0.2)
        r = oracle.run(case, 100000, nthreads=8)
        assert r["t"] == 0.2
        x = 0.5 * (case.xf[0][1:] + case.xf[0][:-1])
        ex = ER.sample((1, 0, 1), (0.125, 0, 0.1), x, 0.2)
        rho = r["W"][0, 0, 0]
        errs.append(float(np.mean(np.abs(rho - ex[0]))))
        if N == 400:
            u = r["W"][1, 0, 0] / rho
            p = (G - 1) * (r["W"][3, 0, 0] - 0.5 * rho * u * u)
            # p and u are constant between the rarefaction tail and the shock
            tail, shock = 0.5 + 0.2 * (us - math.sqrt(G * ps / rl)), 0.5 + 0.2 * 1.752156
            plateau = (x > tail + 0.04) & (x < shock - 0.04)
            assert np.all(np.abs(p[plateau] - ps) < 0.01 * ps)
            assert np.all(np.abs(u[plateau] - us) < 0.01 * us)
    assert errs[0] > errs[1] > errs[2]


# ---------------------------------------------------------------------------
# P14: viscous shear-wave decay with laminar plus turbulent viscosity
# ---------------------------------------------------------------------------
def _shear_decay(N, k_val, omega_val, mu):
    case = C.shear_wave(N, mu=mu, k_val=k_val, omega_val=omega_val)
    case.prandtl = 1.0
    y = 0.5 * (case.xf[1][1:] + case.xf[1][:-1])
    s = np.sin(2 * math.pi * y)
    a0 = float(np.sum(case.W[1, 0, :, 0] * s) / np.sum(s * s))
    r = oracle.run(case, 400, nthreads=8)
    a1 = float(np.sum(r["W"][1, 0, :, 0] * s) / np.sum(s * s))
    return -math.log(a1 / a0) / r["t"]


def test_p14_shear_wave_decay():
    """Decay rate nu_eff (2 pi)^2 with nu_eff = (mu + rho k/omega)/rho.  Minmod clips the
    slopes at the extrema of the sine (locally first order), so the error shrinks faster
    than first order but not at a clean second order; it must fall monotonically and be
    below 1 % on 64 cells."""
    mu, k_val, om = 4e-3, 2e-3, 1.0
    # eta = S/(C_mu omega) stays below 1e-2 for this amplitude, so tau_t p = rho k / omega
    nu = mu + k_val / om
    exact = nu * (2 * math.pi) ** 2
    errs = [abs(_shear_decay(N, k_val, om, mu) / exact - 1) for N in (16, 32, 64)]
    assert errs[0] > errs[1] > errs[2], errs
    assert errs[2] < 0.01, errs


# ---------------------------------------------------------------------------
# P15: entropy wave (exact Euler solution) converges at order > 1.5 in L1
# ---------------------------------------------------------------------------
def test_p15_entropy_wave_order():
    errs = []
    for N in (32, 64, 128):
        case = C.entropy_wave(N, t_end=0.5)
        r = oracle.run(case, 10 ** 6, nthreads=8)
        assert r["t"] == 0.5
        xf = case.xf[0]
        dx = np.diff(xf)
        amp, U = 0.2, 1.0
        xa, xb = xf[:-1] - U * 0.5, xf[1:] - U * 0.5
        exact = 1.0 - amp * (np.cos(2 * math.pi * xb) - np.cos(2 * math.pi * xa)) / (2 * math.pi * dx)
        errs.append(float(np.mean(np.abs(r["W"][0, 0, 0] - exact))))
    o1 = math.log2(errs[0] / errs[1])
    o2 = math.log2(errs[1] / errs[2])
    assert o2 > 1.5 and o1 > 1.3, errs
