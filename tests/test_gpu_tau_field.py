"""The relaxation-time field (gks_fields TAU) on the GPU against the oracle's og_tau_field
on the same state: tau = mu/p0 + tau_a + the k-omega part (Eqs. relaxation time, taua,
tautchenadjusted) of every face at the state's CFL step, largest per cell, within 1e-12 of
the field's maximum.  The diagnostic always evaluates in FP64, so the FP32-flux solves are
held to the same bound.  Cases: the shock tube with the artificial part (C_a = 1) and a
turbulent k field, the boundary-layer interaction, the mixing layer with k-omega transport
(the field then uses the transported k and omega), and the isotropic box."""
import numpy as np
import pytest

import oracle
from gpu_util import banner
from inputs import cases as C

pytestmark = pytest.mark.gpu


def _tau(case, nsteps):
    from paper_1302_2132_amd import Solver
    s = Solver(case)
    try:
        s.step(nsteps)
        W = s.fields("cons")
        kw = s.fields("turb")
        t = s.fields("tau")
        W2 = s.fields("cons")
    finally:
        s.close()
    assert np.array_equal(W, W2)                  # reading the diagnostic leaves the state alone
    return W, kw, t


def _check(case, nsteps):
    banner(f"tau field: {case.name} {case.precision} after {nsteps} steps")
    W, kw, t = _tau(case, nsteps)
    to = oracle.tau_field(case, W, kw[0], kw[1])
    err = np.max(np.abs(t - to))
    print(f"  tau max {to.max():.3e} min {to.min():.3e}  gpu-oracle {err:.3e}", flush=True)
    assert to.min() > 0
    assert err <= 1e-12 * to.max()
    return t, to


def test_tau_field_shock_tube_with_the_artificial_part():
    c = C.shock_tube(64, 8, x0=0.4, mu=1e-4, c_a=1.0, k_val=1e-4, omega_val=10.0)
    t, to = _check(c, 20)
    # the artificial part is present: without it tau falls by a large share near the waves
    c0 = c.copy()
    c0.c_a = 0.0
    W, kw, _ = _tau(c, 20)
    t0 = oracle.tau_field(c0, W, kw[0], kw[1])
    assert np.max((to - t0) / t0) > 0.3


@pytest.mark.parametrize("precision", ["fp64", "fp32_flux"])
def test_tau_field_sbli(precision):
    _check(C.sbli(96, 48, precision=precision), 30)


def test_tau_field_mixing_layer_with_transport():
    c = C.mixing_layer(48, seed=4)
    c.kw_transport = True
    _check(c, 25)


@pytest.mark.parametrize("precision", ["fp64", "fp32_flux"])
def test_tau_field_isotropic_3d(precision):
    _check(C.isotropic_box(16, precision=precision), 8)
