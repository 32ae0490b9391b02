"""Pins of the oracle's k-omega transport mode (og_run_kw) against what the model and the
mathematics fix: the closed-form decay of homogeneous turbulence, consistency of the
convected k with the mass flux, conservation of rho k and rho omega, upwinding, the
production and cross-diffusion sources on fields where central differences are exact,
the diffusion rate of a sine mode, and mirror symmetry.

Model constants (Wilcox 2006 k-omega): beta* = 0.09, beta = 0.0708, alpha = 13/25,
sigma* = 3/5, sigma = 1/2, sigma_do = 1/8."""
import numpy as np
import pytest

import oracle
from inputs import cases as C

BETA_STAR, BETA, ALPHA, SIGMA_STAR, SIGMA, SIGMA_DO = 0.09, 0.0708, 13 / 25, 0.6, 0.5, 0.125


def _rest(n=8, dim=2, rho=1.0, p=1.0, vel=(0.0, 0.0, 0.0), stretched=True, mu=1e-3, seed=5):
    c = C.uniform_flow(dim=dim, n=(n, n, n if dim == 3 else 1), rho=rho, vel=vel, p=p,
                       stretched=stretched, mu=mu, seed=seed)
    return c


def _step_by_step(c, nsteps):
    """Run one step at a time, collecting dt and the fields after each step."""
    W, k, w, t = c.W.copy(), c.k.copy(), c.omega.copy(), 0.0
    out = []
    for _ in range(nsteps):
        r = oracle.run_kw(c, 1, W=W, k=k, omega=w, t0=t)
        W, k, w, t = r["W"], r["k"], r["omega"], r["t"]
        out.append((r["dt"], k.copy(), w.copy()))
    return out


@pytest.mark.parametrize("dim", [2, 3])
def test_homogeneous_decay_follows_the_point_implicit_recurrence(dim):
    """Uniform turbulence at rest: no flux difference, no production; each step is
    k' = k/(1 + dt beta* omega), omega' = omega/(1 + dt beta omega), on any stretched grid."""
    c = _rest(dim=dim)
    c.k[...] = 0.3
    c.omega[...] = 7.0
    k, w = 0.3, 7.0
    for dt, kf, wf in _step_by_step(c, 6):
        k, w = k / (1 + dt * BETA_STAR * w), w / (1 + dt * BETA * w)
        assert np.max(np.abs(kf - k)) <= 1e-14 * k
        assert np.max(np.abs(wf - w)) <= 1e-14 * w


def test_homogeneous_decay_converges_to_the_closed_form():
    """dk/dt = -beta* k omega, domega/dt = -beta omega^2 have omega = w0/(1 + beta w0 t),
    k = k0 (1 + beta w0 t)^(-beta*/beta).  The point-implicit omega step is exact for this
    equation (1/omega grows by beta dt per step), so omega matches to rounding; k, which
    uses the old omega, is first order in dt."""
    errs = []
    for cfl in (0.4, 0.2, 0.1):
        c = _rest(n=6, stretched=False)
        c.k[...] = 0.2
        c.omega[...] = 40.0
        c.cfl = cfl
        c.t_end = 0.05                           # the last step is clipped to land on t_end
        r = oracle.run_kw(c, 100000)
        t, k, w = r["t"], r["k"].mean(), r["omega"].mean()
        assert t == 0.05
        wex = 40.0 / (1 + BETA * 40.0 * t)
        kex = 0.2 * (1 + BETA * 40.0 * t) ** (-BETA_STAR / BETA)
        errs.append((abs(k - kex) / kex, abs(w - wex) / wex))
    for a, b in zip(errs, errs[1:]):
        assert 1.6 < a[0] / b[0] < 2.4, errs
    assert errs[-1][0] < 2e-3, errs
    assert all(e[1] < 1e-14 for e in errs), errs


def test_uniform_k_stays_uniform_in_a_density_wave():
    """Uniform k, omega convected by a flow whose density varies: the rho k flux is the mass
    flux times k and the diffusive flux vanishes, so rho' k' (1 + dt beta* omega) =
    rho' k + dt Qk exactly.  The first step starts from uniform U (no strain): k stays
    uniform.  Later steps (the flow has picked up small velocity differences) restart from
    uniform k, omega on the evolved flow and check the identity with the sources of that
    state."""
    c = C.entropy_wave(32, ny=2, U=1.0, amp=0.2)
    k0, w0 = 0.05, 3.0
    W, t = c.W.copy(), 0.0
    for step in range(4):
        kk, ww = np.full_like(c.k, k0), np.full_like(c.omega, w0)
        Qk, Qw = oracle.kw_sources(c, W=W, k=kk, omega=ww)
        r = oracle.run_kw(c, 1, W=W, k=kk, omega=ww, t0=t)
        dt, rho1 = r["dt"], r["W"][0]
        ek = (k0 + dt * Qk / rho1) / (1 + dt * BETA_STAR * w0)
        ew = (w0 + dt * Qw / rho1) / (1 + dt * BETA * w0)
        assert np.max(np.abs(r["k"] - ek)) <= 1e-14 * k0
        assert np.max(np.abs(r["omega"] - ew)) <= 1e-14 * w0
        if step == 0:
            assert np.ptp(r["k"]) <= 1e-14 * k0 and np.ptp(r["omega"]) <= 1e-14 * w0
        else:
            assert np.ptp(r["k"]) > 1e-12 * k0        # production is active from step 2 on
        W, t = r["W"], r["t"]


def _volumes(c):
    dx = [np.diff(c.xf[d]) for d in range(c.dim)]
    if c.dim == 2:
        return (dx[1][:, None] * dx[0][None, :])[None]
    return dx[2][:, None, None] * dx[1][None, :, None] * dx[0][None, None, :]


@pytest.mark.parametrize("case", ["mixing", "stretched3d"])
def test_rho_k_and_rho_omega_conserved_up_to_their_sources(case):
    """Periodic meshes: sum V [rho k' (1 + dt beta* omega) - dt Qk] = sum V rho k exactly
    (every face flux cancels), and likewise for rho omega."""
    if case == "mixing":
        c = C.mixing_layer(24, seed=7)
    else:
        c = C.uniform_flow(dim=3, n=(6, 5, 4), vel=(0.3, -0.2, 0.1), seed=9)
        rng = np.random.default_rng(3)
        c.W = c.W * (1 + 0.05 * rng.uniform(-1, 1, size=c.W.shape))
    Qk, Qw = oracle.kw_sources(c)
    r = oracle.run_kw(c, 1)
    dt, V = r["dt"], _volumes(c)
    rho0, rho1 = c.W[0], r["W"][0]
    lhs_k = np.sum(V * (rho1 * r["k"] * (1 + dt * BETA_STAR * c.omega) - dt * Qk))
    lhs_w = np.sum(V * (rho1 * r["omega"] * (1 + dt * BETA * c.omega) - dt * Qw))
    rk0, rw0 = np.sum(V * rho0 * c.k), np.sum(V * rho0 * c.omega)
    assert abs(lhs_k - rk0) <= 1e-13 * np.sum(V * rho0 * np.abs(c.k))
    assert abs(lhs_w - rw0) <= 1e-13 * np.sum(V * rho0 * c.omega)


def test_convection_is_upwind():
    """Uniform flow in +x over a k step: with no diffusion, a cell upstream of the step
    only decays; the first cell downstream of it receives k."""
    c = _rest(n=16, vel=(0.5, 0.0, 0.0), stretched=False, mu=0.0)
    c.omega[...] = 1e6                       # rho k / omega ~ 1e-7: diffusion negligible ...
    c.k[...] = 1e-3
    c.k[:, :, 8:] = 2e-3                      # ... so only convection moves the step
    dt, kf, wf = _step_by_step(c, 1)[0]
    decay = 1.0 / (1 + dt * BETA_STAR * 1e6)
    up = kf[0, :, 6] / (1e-3 * decay)        # two cells upstream of the jump at i = 8
    down = kf[0, :, 8] / (2e-3 * decay)      # first cell of the high state: receives k = 1e-3
    assert np.all(np.abs(up - 1.0) < 1e-6), up
    assert np.all(down < 1.0 - 1e-3), down
    # and the cell just before the jump (i = 7) is fed from upstream only: unchanged but for decay
    assert np.all(np.abs(kf[0, :, 7] / (1e-3 * decay) - 1.0) < 1e-6)


def test_production_of_a_linear_shear():
    """U = a y (div U = 0, S = |a|): at interior cells Qk = mu_t a^2 with
    mu_t = rho k/(omega sqrt(1 + eta^2)), eta = a/(C_mu omega); uniform k, omega so no
    cross-diffusion; Qw = alpha rho a^2/sqrt(1 + eta^2)."""
    n = 12
    c = C.uniform_flow(dim=2, n=(n, n, 1), vel=(0.0, 0.0, 0.0), stretched=True, seed=4,
                       bc=[["periodic", "periodic"], ["outflow", "outflow"]])
    a, rho, p, g = 0.7, 1.3, 0.9, c.gamma
    yc = 0.5 * (c.xf[1][1:] + c.xf[1][:-1])
    u = a * yc[None, :, None] * np.ones((1, n, n))
    c.W[1] = rho * u
    c.W[2] = 0.0
    c.W[3] = p / (g - 1) + 0.5 * rho * u ** 2
    c.k[...] = 0.02
    c.omega[...] = 5.0
    Qk, Qw = oracle.kw_sources(c)
    eta = a / (c.c_mu * 5.0)
    mut = rho * 0.02 / (5.0 * np.sqrt(1 + eta ** 2))
    inner = (slice(None), slice(1, n - 1), slice(None))
    assert np.allclose(Qk[inner], mut * a * a, rtol=1e-12, atol=0)
    assert np.allclose(Qw[inner], ALPHA * rho * a * a / np.sqrt(1 + eta ** 2), rtol=1e-12, atol=0)


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_cross_diffusion_only_where_gradients_align(sign):
    """At rest, k and omega linear in x: grad k . grad omega = k' w' at interior cells.
    sigma_do (rho/omega) k' w' is added to Qw when positive, nothing when negative."""
    n = 10
    c = C.uniform_flow(dim=2, n=(n, 4, 1), vel=(0.0, 0.0, 0.0), stretched=True, seed=6,
                       bc=[["outflow", "outflow"], ["periodic", "periodic"]])
    xc = 0.5 * (c.xf[0][1:] + c.xf[0][:-1])
    kp, wp = 0.01, sign * 2.0
    c.k[...] = 0.05 + kp * xc[None, None, :]
    c.omega[...] = 4.0 + wp * xc[None, None, :]
    Qk, Qw = oracle.kw_sources(c)
    rho = c.W[0]
    inner = (slice(None), slice(None), slice(1, n - 1))
    assert np.all(Qk[inner] == 0.0)
    expect = SIGMA_DO * rho / c.omega * kp * wp if sign > 0 else 0.0 * rho
    assert np.allclose(Qw[inner], expect[inner], rtol=1e-12, atol=1e-300)


@pytest.mark.parametrize("field", ["k", "omega"])
def test_diffusion_rate_of_a_sine_mode(field):
    """At rest with uniform rho, p: a small sine perturbation of k (or omega) decays at the
    linearised rate beta* omega0 + D (2 pi)^2/rho (or 2 beta omega0 + D (2 pi)^2/rho), with
    D = mu + sigma* rho k0/omega0 (or sigma); measured over 20 steps, converging with N."""
    errs = []
    for n in (16, 32, 64):
        c = _rest(n=n, dim=2, stretched=False, mu=2e-3)
        xc = (np.arange(n) + 0.5) / n
        k0, w0, eps = 0.4, 0.6, 1e-4
        c.k[...] = k0
        c.omega[...] = w0
        f = getattr(c, "k" if field == "k" else "omega")
        f[...] = (k0 if field == "k" else w0) * (1 + eps * np.sin(2 * np.pi * xc))[None, None, :]
        c.cfl = 0.1
        W, kk, ww, t = c.W.copy(), c.k.copy(), c.omega.copy(), 0.0
        for _ in range(20):
            r = oracle.run_kw(c, 1, W=W, k=kk, omega=ww, t0=t)
            W, kk, ww, t = r["W"], r["k"], r["omega"], r["t"]
        g = kk if field == "k" else ww
        mean = g.mean()
        amp = 2 * np.mean(g[0, 0] * np.sin(2 * np.pi * xc)) / mean
        rate_meas = -np.log(amp / eps) / t
        D = 2e-3 + (SIGMA_STAR if field == "k" else SIGMA) * 1.0 * k0 / w0
        sink = BETA_STAR * w0 if field == "k" else BETA * w0   # relative to the decaying mean
        rate = D * (2 * np.pi) ** 2 + (0.0 if field == "k" else sink)
        errs.append(abs(rate_meas - rate) / rate)
    assert errs[-1] < 0.02 and errs[0] > errs[1] > errs[2], errs


def test_mirror_symmetry():
    """Reflecting the data in x (velocity negated) reflects the transported fields; k and
    omega vary strongly along x, so a one-sided face diffusivity would break the symmetry."""
    c = C.mixing_layer(16, seed=2)
    rng = np.random.default_rng(11)
    c.k = 0.01 * (1 + 0.5 * rng.uniform(-1, 1, size=c.k.shape))
    c.omega = 2.0 * (1 + 0.5 * rng.uniform(-1, 1, size=c.omega.shape))
    u = 0.1 * np.sin(2 * np.pi * (np.arange(16) + 0.5) / 16)[None, None, :]
    p = 1.0 / c.gamma
    c.W[1] = c.W[0] * u
    c.W[2] = 0.0
    c.W[3] = p / (c.gamma - 1) + 0.5 * c.W[0] * u ** 2
    m = c.copy()
    m.W = c.W[:, :, :, ::-1].copy()
    m.W[1] = -m.W[1]
    m.k = c.k[:, :, ::-1].copy()
    m.omega = c.omega[:, :, ::-1].copy()
    a, b = oracle.run_kw(c, 3), oracle.run_kw(m, 3)
    assert np.allclose(b["k"][:, :, ::-1], a["k"], rtol=1e-12, atol=0)
    assert np.allclose(b["omega"][:, :, ::-1], a["omega"], rtol=1e-12, atol=0)
