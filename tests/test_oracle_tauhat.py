"""Pins of the oracle's tau_hat rarefaction mode (eps = tau/tau_hat, Eqs. tautautilde,
tautilde, rarefactionkepsilon, epsilonkomega) against what the paper and the mathematics fix.

* The time weights are the time integrals, over [0, dt], of the coefficients of
  Eq. resultingf regrouped as in Eq. resultingf2 (slope term written out exactly), with the
  exponential decay time tau_e = dt tau/tau_hat in place of tau and the physical tau in
  f_c and f_u.  They are checked against Gauss-Legendre quadrature of those coefficients,
  against the Kogan weights at tau_e = tau (the dt mode), and in the hydrodynamic limit
  tau_e -> 0, where the average distribution is f_c (1 + Abar dt/2) (Eq. hydroturbolimit).
* tau_hat = rho/|D rho| with D rho the material derivative: a convected density wave has
  D rho = 0, a velocity gradient b gives D rho = -rho b, so eps_hat = tau |b|.
* For continuous linear data the flux is the Navier-Stokes flux whatever eps is (f_u = f_c
  and Abar = A), as in the dt mode (pin P5).
* Runs: free stream preserved, conservation on a periodic mesh.
"""
import numpy as np
import pytest

import oracle
from inputs import cases as C
from test_oracle_pins import cons, jac_vec, ns_flux_1d, rand_prim, rel

G = 1.4


def _quad_weights(tau, tau_e, dt, n=400):
    """Gauss-Legendre quadrature over [0, dt] of the coefficients of g0, u abar g0, Abar g0,
    g_lr, u a g_lr and A g_lr in
    f = f_c (1 + Abar t) + e (f_u - f_c) + t e u (abar g0 - a g_lr),  e = exp(-t/tau_e),
    f_c = g0 (1 - tau (abar u + Abar)),  f_u = g_lr (1 - tau (a u + A))."""
    x, w = np.polynomial.legendre.leggauss(n)
    t = 0.5 * dt * (x + 1.0)
    w = 0.5 * dt * w
    e = np.exp(-t / tau_e)
    coef = [1.0 - e,                       # g0
            -tau * (1.0 - e) + t * e,      # u abar g0
            t - tau * (1.0 - e),           # Abar g0
            e,                             # g_lr
            -tau * e - t * e,              # u a g_lr
            -tau * e]                      # A g_lr
    return np.array([float(np.sum(w * c)) for c in coef])


@pytest.mark.parametrize("x", [0.01, 0.3, 0.49, 0.51, 2.0, 30.0])
@pytest.mark.parametrize("ratio", [0.1, 1.0, 7.0])
def test_time_weights_by_quadrature(x, ratio):
    dt = 2e-3
    tau_e = dt / x
    tau = ratio * tau_e
    got = oracle.kogan_e(tau, tau_e, dt)
    q = _quad_weights(tau, tau_e, dt)
    scale = np.array([dt, tau * dt, dt * dt, dt, tau * dt + dt * dt, tau * dt])
    assert np.all(np.abs(got[:6] - q) <= 1e-13 * scale), (got[:6], q)
    # the integrated compatibility coefficients c_j = gam_j / (tau gam0)
    c = np.array([q[1], q[4], q[5]]) / (tau * q[0])
    assert np.allclose(got[6:9], c, rtol=1e-10, atol=0)


@pytest.mark.parametrize("x", [0.02, 0.4, 0.6, 5.0])
def test_weights_reduce_to_the_dt_mode_when_tau_e_is_tau(x):
    dt = 1e-3
    tau = dt / x
    a, b = oracle.kogan_e(tau, tau, dt), oracle.kogan(tau, dt)
    scale = np.array([dt, tau * dt, dt * dt, dt, tau * dt, tau * dt])
    assert np.all(np.abs(a[:6] - b[:6]) <= 1e-14 * scale / min(x, 1.0))
    assert np.allclose(a[6:], b[6:], rtol=1e-11 / min(x, 1.0), atol=1e-14)


def test_hydrodynamic_limit():
    """tau_e -> 0: the average distribution is f_c (1 + Abar dt/2): gam0 = dt, gam1 = -tau dt,
    gam2 = dt^2/2 - tau dt, no upwind part; c1 = -1 (Abar = -<u abar>), c4 = c5 = 0."""
    dt, tau = 1e-3, 4e-4
    lim = oracle.kogan_e(tau, 0.0, dt)
    want = np.array([dt, -tau * dt, 0.5 * dt * dt - tau * dt, 0.0, 0.0, 0.0, -1.0, 0.0, 0.0])
    assert np.allclose(lim, want, rtol=1e-15, atol=0)
    near = oracle.kogan_e(tau, 1e-9 * dt, dt)          # the approach is continuous, O(tau_e/dt)
    scale = np.array([dt, tau * dt, dt * dt, dt, tau * dt, tau * dt, 1.0, 1.0, 1.0])
    assert np.all(np.abs(near - want) <= 1e-8 * scale)


def _linear_face(dim, Wfun, dWfun, dxl, dxr, eps_mode, **kw):
    W0 = Wfun(0.0)
    dW = dWfun(0.0)
    return oracle.face_flux(dim, W0, W0, dW, dW, Wfun(-dxl), Wfun(dxr), dxl, dxr, kw.pop("kf", 2e-3),
                            kw.pop("wf", 3.0), kw.pop("Sf", 4.0), kw.pop("dt", 1e-3), eps_mode=eps_mode, **kw)


def _prim_fields(rho_f, U_f, p, dim):
    """Conservative state and its x-derivative for primitive fields rho(x), U(x) (vector),
    uniform p."""
    def Wfun(x):
        return cons(rho_f(x)[0], U_f(x)[0], p)

    def dWfun(x):
        rho, drho = rho_f(x)
        U, dU = U_f(x)
        m = rho * U
        dm = drho * U + rho * dU
        dE = 0.5 * drho * float(U @ U) + rho * float(U @ dU)
        return np.concatenate([[drho], dm, [dE]])
    return Wfun, dWfun


@pytest.mark.parametrize("dim", [2, 3])
def test_eps_hat_of_a_velocity_gradient(dim):
    """Uniform rho, p; U_n = U_f + b x: D rho = -rho b, so eps_hat = tau |b|, on any mesh."""
    b = -3.7
    Ut = np.array([0.1, -0.2, 0.05])[:dim - 1]
    rho_f = lambda x: (1.2, 0.0)                                           # noqa: E731
    U_f = lambda x: (np.concatenate([[0.3 + b * x], Ut]), np.concatenate([[b], 0 * Ut]))   # noqa: E731
    Wf, dWf = _prim_fields(rho_f, U_f, 0.9, dim)
    r = _linear_face(dim, Wf, dWf, 0.03, 0.02, "tauhat", gamma=G)
    assert r["info"]["eps_hat"] == pytest.approx(r["info"]["tau"] * abs(b), rel=1e-12)


@pytest.mark.parametrize("dim", [2, 3])
def test_eps_hat_of_a_convected_density_wave_is_zero(dim):
    """rho = rho_f (1 + a x) with uniform U and p is an exact Euler solution with
    D rho / Dt = 0: tau_hat is infinite."""
    a = 2.5
    U = np.array([0.6, 0.2, -0.1])[:dim]
    rho_f = lambda x: (1.1 * (1 + a * x), 1.1 * a)                        # noqa: E731
    U_f = lambda x: (U, 0 * U)                                             # noqa: E731
    Wf, dWf = _prim_fields(rho_f, U_f, 0.8, dim)
    r = _linear_face(dim, Wf, dWf, 0.025, 0.025, "tauhat", gamma=G)
    assert r["info"]["eps_hat"] <= 1e-13 * r["info"]["tau"] * abs(a) * float(np.linalg.norm(U))


def test_eps_hat_of_density_and_velocity_gradients():
    """rho = rho_f (1 + a x), U_n = U_f + b x (rho U quadratic; centred cells, so the mean
    one-sided gradient is exact): D rho = U rho_x - (rho U)_x = -rho b."""
    a, b = 1.7, 2.9
    rho_f = lambda x: (1.3 * (1 + a * x), 1.3 * a)                         # noqa: E731
    U_f = lambda x: (np.array([0.4 + b * x, 0.15]), np.array([b, 0.0]))    # noqa: E731
    Wf, dWf = _prim_fields(rho_f, U_f, 1.1, 2)
    r = _linear_face(2, Wf, dWf, 0.02, 0.02, "tauhat", gamma=G)
    assert r["info"]["eps_hat"] == pytest.approx(r["info"]["tau"] * abs(b), rel=1e-12)


@pytest.mark.parametrize("dim", [2, 3])
def test_continuous_data_navier_stokes_flux_in_tauhat_mode(dim):
    """P5 in the tau_hat mode: continuous linear data give the Navier-Stokes flux minus
    dt^2/2 J^2 dW/dx whatever eps_hat is (here eps_hat != tau/dt)."""
    rng = np.random.default_rng(140 + dim)
    for trial in range(4):
        rho, U, p = rand_prim(rng, dim)
        W = cons(rho, U, p)
        dW = 0.4 * rng.uniform(-1, 1, size=dim + 2) * np.abs(W)
        dxl, dxr = 0.03, 0.02
        dt = [1e-3, 5e-3, 2e-2, 4e-2][trial]
        res = oracle.face_flux(dim, W, W, dW, dW, W - dW * dxl, W + dW * dxr, dxl, dxr, 2e-3, 3.0, 5.0, dt,
                               prandtl=1.0, mu=3e-3, c_a=0.7, eps_mode="tauhat")
        tau = res["info"]["tau"]
        eps = res["info"]["eps_hat"]
        assert eps > 0 and abs(eps - tau / dt) > 1e-3 * tau / dt      # the weights differ from the dt mode
        expect = dt * ns_flux_1d(W, dW, dim, tau * p) - 0.5 * dt * dt * jac_vec(W, jac_vec(W, dW, dim), dim)
        assert rel(res["F"], expect) < 2e-13, trial
        assert rel(res["info"]["Abar"], res["info"]["A_l"]) < 1e-11


def test_free_stream_preserved_in_tauhat_mode():
    bc = [["dirichlet", "outflow"], ["outflow", "profile"]]
    c = C.uniform_flow(dim=2, n=(20, 17, 1), bc=bc, seed=8)
    c.eps_mode = "tauhat"
    r = oracle.run(c, 5)
    assert np.max(np.abs(r["W"] - c.W)) <= 1e-14 * np.max(np.abs(c.W))
    assert np.max(oracle.eps_field(c)) == 0.0


def test_conservation_in_tauhat_mode():
    c = C.mixing_layer(24, seed=7)
    c.eps_mode = "tauhat"
    vol = np.outer(np.diff(c.xf[1]), np.diff(c.xf[0]))
    r = oracle.run(c, 10)
    for m in range(4):
        before, after = np.sum(c.W[m, 0] * vol), np.sum(r["W"][m, 0] * vol)
        assert abs(after - before) <= 1e-13 * np.sum(np.abs(c.W[m, 0]) * vol)
    # and the mode changed the solution
    c_dt = c.copy()
    c_dt.eps_mode = "dt"
    d = oracle.run(c_dt, 10)
    assert np.max(np.abs(d["W"] - r["W"])) > 1e-10
