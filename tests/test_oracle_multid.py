"""Pins of the oracle's multi-dimensional expansion (multi_d: the initial and equilibrium
distributions also expanded along the tangential axes, the alternative the implementation
section describes; tangential slopes b from the tangential gradients, b_bar from their
mean, A and Abar from the compatibility conditions with the b terms).

* Continuous linear data with gradients along every axis give the Navier-Stokes flux with
  the full velocity-gradient tensor (shear stress mu (U_y + V_x), bulk term on div U) minus
  dt^2/2 J_x (J_x W_x + J_y W_y + J_z W_z): the time derivative from all directions.
  Without the expansion the tangential parts are missing (checked, so the pin has teeth).
* Zero tangential gradients reproduce the one-dimensional flux exactly.
* Runs: transposing the data transposes the solution; free stream and conservation hold.
"""
import numpy as np
import pytest

import oracle
from inputs import cases as C
from test_oracle_pins import G, cons, euler_flux, rand_prim, rel


def _perm(v, dim, a):
    """Swap the momentum components of the x axis and axis a (a state or a gradient)."""
    v = np.array(v, dtype=complex if np.iscomplexobj(v) else float)
    v[[1, 1 + a]] = v[[1 + a, 1]]
    return v


def _jac_axis(W, v, dim, a):
    """J_a(W) v, the Jacobian of the flux along axis a, by complex step on the x flux of the
    axis-swapped state."""
    h = 1e-30
    Wp = _perm(np.asarray(W, dtype=complex), dim, a) + 1j * h * _perm(np.asarray(v, dtype=complex), dim, a)
    return _perm(np.imag(euler_flux(Wp, dim)) / h, dim, a)


def ns_flux_md(W, grads, dim, mu_eff, gamma=G):
    """Euler + Navier-Stokes flux through an x-face, gradients grads[b] = dW/dx_b:
    sigma_xa = mu (dU_a/dx + dU_x/dx_a) - (2/b) mu delta_xa div U (b = 2/(gamma - 1)),
    q = -mu c_p dT/dx."""
    bdof = 2.0 / (gamma - 1.0)
    rho = W[0]
    U = W[1:1 + dim] / rho
    p = (gamma - 1.0) * (W[-1] - 0.5 * rho * float(U @ U))
    gU = np.zeros((dim, dim))                 # gU[a, b] = dU_a/dx_b
    for b in range(dim):
        dW = grads[b]
        gU[:, b] = (dW[1:1 + dim] - U * dW[0]) / rho
    div = np.trace(gU)
    sig = np.array([mu_eff * (gU[a, 0] + gU[0, a]) for a in range(dim)])
    sig[0] -= 2.0 / bdof * mu_eff * div
    dW = grads[0]
    drho = dW[0]
    dU = gU[:, 0]
    dp = (gamma - 1.0) * (dW[-1] - 0.5 * drho * float(U @ U) - rho * float(U @ dU))
    dT = (dp - p / rho * drho) / rho
    F = euler_flux(W, dim, gamma)
    F[1:1 + dim] -= sig
    F[-1] += -float(U @ sig) - mu_eff * (bdof + 2.0) / 2.0 * dT
    return F


@pytest.mark.parametrize("dim", [2, 3])
def test_continuous_data_full_navier_stokes_flux(dim):
    rng = np.random.default_rng(300 + dim)
    for trial in range(4):
        rho, U, p = rand_prim(rng, dim)
        W = cons(rho, U, p)
        grads = [0.4 * rng.uniform(-1, 1, size=dim + 2) * np.abs(W) for _ in range(dim)]
        dxl, dxr = 0.03, 0.02
        dt = [1e-3, 5e-3, 2e-2, 4e-2][trial]
        args = (dim, W, W, grads[0], grads[0], W - grads[0] * dxl, W + grads[0] * dxr, dxl, dxr,
                2e-3, 3.0, 5.0, dt)
        kw = dict(prandtl=1.0, mu=3e-3, c_a=0.7)
        res = oracle.face_flux(*args, tsl=np.array(grads[1:]), tsr=np.array(grads[1:]), **kw)
        tau = res["info"]["tau"]
        dWdt = -sum(_jac_axis(W, grads[b], dim, b) for b in range(dim))
        expect = dt * ns_flux_md(W, grads, dim, tau * p) + 0.5 * dt * dt * _jac_axis(W, dWdt, dim, 0)
        assert rel(res["F"], expect) < 2e-13, trial
        assert rel(res["info"]["Abar"], res["info"]["A_l"]) < 1e-11
        one_d = oracle.face_flux(*args, **kw)
        assert rel(one_d["F"], expect) > 1e-6          # the one-dimensional expansion misses these terms


@pytest.mark.parametrize("dim", [2, 3])
def test_zero_tangential_gradients_reproduce_the_1d_flux(dim):
    rng = np.random.default_rng(320 + dim)
    from test_oracle_pins import rand_face
    for _ in range(3):
        fc = rand_face(rng, dim)
        args = (dim, fc["Wl"], fc["Wr"], fc["sl"], fc["sr"], fc["Wi"], fc["Wi1"], fc["dxl"], fc["dxr"],
                1e-3, 2.0, 3.0, 2e-3)
        z = np.zeros((dim - 1, dim + 2))
        a = oracle.face_flux(*args, tsl=z, tsr=z)
        b = oracle.face_flux(*args)
        assert np.array_equal(a["F"], b["F"])


def _transpose(c):
    t = c.copy()
    t.n = (c.n[1], c.n[0], 1)
    t.xf = [c.xf[1].copy(), c.xf[0].copy()]
    t.bc = [list(c.bc[1]), list(c.bc[0])]
    W = np.transpose(c.W, (0, 1, 3, 2)).copy()
    W[[1, 2]] = W[[2, 1]]
    t.W = W
    t.k = np.transpose(c.k, (0, 2, 1)).copy()
    t.omega = np.transpose(c.omega, (0, 2, 1)).copy()
    return t


def test_transposed_data_give_the_transposed_solution():
    c = C.mixing_layer(16, seed=5)
    rng = np.random.default_rng(7)
    c.W = c.W * (1 + 0.05 * rng.uniform(-1, 1, size=c.W.shape))
    c.xf = [np.cumsum(np.r_[0, rng.uniform(0.5, 1.5, 16)]), np.cumsum(np.r_[0, rng.uniform(0.5, 1.5, 16)])]
    c.multi_d = True
    t = _transpose(c)
    a, b = oracle.run(c, 4), oracle.run(t, 4)
    bt = np.transpose(b["W"], (0, 1, 3, 2)).copy()
    bt[[1, 2]] = bt[[2, 1]]
    assert np.allclose(a["W"], bt, rtol=1e-12, atol=1e-14)
    c.multi_d = False
    d = oracle.run(c, 4)
    assert np.max(np.abs(d["W"] - a["W"])) > 1e-8       # the expansion changes the solution


def test_free_stream_and_conservation_with_the_expansion():
    bc = [["dirichlet", "outflow"], ["wall", "profile"], ["outflow", "wall"]]
    c = C.uniform_flow(dim=3, n=(6, 5, 4), bc=bc, vel=(0.4, 0.1, -0.2), seed=3)
    c.multi_d = True
    c.W = c.W.copy()
    r = oracle.run(c, 3)
    u = C.uniform_flow(dim=2, n=(12, 9, 1), bc=[["dirichlet", "outflow"], ["outflow", "profile"]], seed=8)
    u.multi_d = True
    ru = oracle.run(u, 5)
    assert np.max(np.abs(ru["W"] - u.W)) <= 1e-14 * np.max(np.abs(u.W))
    m = C.mixing_layer(24, seed=7)
    m.multi_d = True
    vol = np.outer(np.diff(m.xf[1]), np.diff(m.xf[0]))
    rm = oracle.run(m, 10)
    for k in range(4):
        before, after = np.sum(m.W[k, 0] * vol), np.sum(rm["W"][k, 0] * vol)
        assert abs(after - before) <= 1e-13 * np.sum(np.abs(m.W[k, 0]) * vol)
    assert np.all(np.isfinite(r["W"]))


def test_mirror_in_the_tangential_direction():
    """Reflecting the data in y (rho V negated, stretched cells reversed) reflects the
    solution: the tangential slopes of the x-faces treat both y-neighbours alike."""
    c = C.mixing_layer(16, seed=9)
    rng = np.random.default_rng(2)
    c.W = c.W * (1 + 0.05 * rng.uniform(-1, 1, size=c.W.shape))
    widths = rng.uniform(0.5, 1.5, 16)
    c.xf = [c.xf[0], np.cumsum(np.r_[0, widths])]
    c.multi_d = True
    m = c.copy()
    m.xf = [c.xf[0], np.cumsum(np.r_[0, widths[::-1]])]
    m.W = c.W[:, :, ::-1, :].copy()
    m.W[2] = -m.W[2]
    m.k = c.k[:, ::-1, :].copy()
    m.omega = c.omega[:, ::-1, :].copy()
    a, b = oracle.run(c, 4), oracle.run(m, 4)
    bm = b["W"][:, :, ::-1, :].copy()
    bm[2] = -bm[2]
    assert np.allclose(a["W"], bm, rtol=1e-12, atol=1e-14)
