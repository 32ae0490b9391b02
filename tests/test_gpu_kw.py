"""k-omega transport on the GPU (libgks with turb_transport) against the oracle's transport
mode (og_run_kw) on the same seeded inputs.

The flow state, k and omega are compared per field, normwise (max |gpu - oracle| /
max |oracle|): FP64 flux <= 1e-12, FP32 flux <= 1e-5 (momentum against the momentum
magnitude, as in the frozen-field parity tests).  Time, step count and residuals are
compared as there too.
"""
import numpy as np
import pytest

import oracle
from gpu_util import assert_matches_oracle, banner, field_errors
from inputs import cases as C

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


def _rel(a, b):
    return float(np.max(np.abs(a - b))) / max(float(np.max(np.abs(b))), 1e-300)


def _run_gpu_kw(case, nsteps):
    from paper_1302_2132_amd import Solver
    s = Solver(case)
    try:
        s.step(nsteps)
        r = s.residual()
        W = s.fields("cons")
        kw = s.fields("turb")
    finally:
        s.close()
    return W, kw[0], kw[1], r


def _compare_kw(case, nsteps, tol):
    case = case.copy()
    case.kw_transport = True
    banner(f"k-omega transport: {case.name} {case.precision} steps={nsteps}")
    Wg, kg, wg, rg = _run_gpu_kw(case, nsteps)
    ro = oracle.run_kw(case, nsteps)
    err = assert_matches_oracle(Wg, case, ro, tol)
    ek, ew = _rel(kg, ro["k"]), _rel(wg, ro["omega"])
    print(f"  flow errors {err}  k {ek:.3e}  omega {ew:.3e}", flush=True)
    assert rg["steps"] == ro["steps"]
    assert ek <= tol and ew <= tol, (ek, ew)
    assert abs(rg["t"] - ro["t"]) <= (1e-13 if tol <= TOL64 else 1e-5) * max(ro["t"], 1e-300)
    rr = np.max(np.abs(rg["res"] - ro["res"])) / max(np.max(np.abs(ro["res"])), 1e-300)
    assert rr <= (1e-9 if tol <= TOL64 else 1e-2), (rg["res"], ro["res"])
    # the transport must have done something: k differs from the frozen input
    assert _rel(kg, case.k) > 1e-6
    return Wg, kg, wg


def test_kw_mixing_layer_fp64():
    _compare_kw(C.mixing_layer(64, seed=3), 60, TOL64)


def test_kw_sbli_fp64_all_boundaries():
    # wall, fixed inflow, outflow and post-shock profile; wall-stretched grid
    _compare_kw(C.sbli(96, 48), 40, TOL64)


def test_kw_isotropic_3d_fp64():
    _compare_kw(C.isotropic_box(16, precision="fp64"), 15, TOL64)


def test_kw_3d_mixed_boundaries_fp64():
    bc = [["dirichlet", "outflow"], ["wall", "profile"], ["outflow", "wall"]]
    c = C.uniform_flow(dim=3, n=(9, 7, 6), bc=bc, vel=(0.4, 0.1, -0.2))
    rng = np.random.default_rng(3)
    c.W = c.W * (1.0 + 0.05 * rng.uniform(-1, 1, size=c.W.shape))
    c.k = 0.01 * (1.0 + 0.5 * rng.uniform(-1, 1, size=c.k.shape))
    c.omega = 3.0 * (1.0 + 0.5 * rng.uniform(-1, 1, size=c.omega.shape))
    _compare_kw(c, 6, TOL64)


@pytest.mark.parametrize("n", [(2, 2, 1), (67, 3, 1), (5, 130, 1), (9, 7, 5)])
def test_kw_ragged_and_minimal_sizes(n):
    dim = 3 if n[2] > 1 else 2
    c = C.uniform_flow(dim=dim, n=n, bc=[["periodic", "periodic"]] * dim)
    rng = np.random.default_rng(sum(n))
    c.W = c.W * (1.0 + 0.05 * rng.uniform(-1, 1, size=c.W.shape))
    c.k = 0.02 * (1.0 + 0.5 * rng.uniform(-1, 1, size=c.k.shape))
    c.omega = 2.0 * (1.0 + 0.5 * rng.uniform(-1, 1, size=c.omega.shape))
    _compare_kw(c, 4, TOL64)


def test_kw_mixing_layer_fp32_flux():
    _compare_kw(C.mixing_layer(64, seed=3, precision="fp32_flux"), 60, TOL32)


def test_kw_isotropic_3d_fp32_flux():
    _compare_kw(C.isotropic_box(16, precision="fp32_flux"), 15, TOL32)


def test_kw_conserves_rho_k_up_to_sources():
    """Periodic mixing layer, one step: sum V (rho k)' (1 + dt beta* omega) - dt Qk equals
    sum V rho k (every face flux of rho k cancels), with Qk from the oracle."""
    from paper_1302_2132_amd import Solver
    c = C.mixing_layer(48, seed=7)
    c.kw_transport = True
    s = Solver(c)
    try:
        s.step(1)
        W = s.fields("cons")
        kk = s.fields("turb")
        r = s.residual()
    finally:
        s.close()
    Qk, _ = oracle.kw_sources(c)
    V = np.outer(np.diff(c.xf[1]), np.diff(c.xf[0]))[None]
    lhs = np.sum(V * (W[0] * kk[0] * (1 + r["dt"] * 0.09 * c.omega) - r["dt"] * Qk))
    rhs = np.sum(V * c.W[0] * c.k)
    assert abs(lhs - rhs) <= 1e-12 * np.sum(V * c.W[0] * c.k)


def test_turb_field_of_a_frozen_solve_is_the_input():
    from paper_1302_2132_amd import Solver
    c = C.mixing_layer(32, seed=2)
    s = Solver(c)
    try:
        s.step(3)
        kw = s.fields("turb")
    finally:
        s.close()
    assert np.array_equal(kw[0], c.k) and np.array_equal(kw[1], c.omega)


def test_kw_sbli_full_size_one_step():
    """SBLI at 1024 x 512 with transport: after 10 steps on the GPU, the next step from the
    GPU's state (flow, k, omega) compared over the whole mesh with one oracle step."""
    from paper_1302_2132_amd import Solver
    c = C.sbli()
    c.kw_transport = True
    banner(f"k-omega transport: {c.name} full size, one step after 10")
    s = Solver(c)
    try:
        s.step(10)
        Wa, ka = s.fields("cons"), s.fields("turb")
        ra = s.residual()
        s.step(1)
        Wb, kb = s.fields("cons"), s.fields("turb")
        rb = s.residual()
    finally:
        s.close()
    ro = oracle.run_kw(c, 1, W=Wa, k=ka[0], omega=ka[1], t0=ra["t"])
    assert abs(rb["dt"] - ro["dt"]) <= 1e-13 * ro["dt"]
    err = field_errors(Wb, ro["W"])
    ek, ew = _rel(kb[0], ro["k"]), _rel(kb[1], ro["omega"])
    print(f"  flow errors {err}  k {ek:.3e}  omega {ew:.3e}", flush=True)
    assert np.all(err <= TOL64) and ek <= TOL64 and ew <= TOL64


@pytest.mark.parametrize("precision", ["fp64", "fp32_flux"])
def test_marching_transport_strain_equals_the_per_cell_pass(precision):
    """A 3D transported solve stepped alone takes the z-marching transport strain pass
    (k_strain3kw); stepped in a batch it takes the per-cell pass (k_strain<true>).  The two
    form the same strain rate, k, omega, rho k/omega and sources (shared gradient and output
    arithmetic), so the states agree bitwise, with every boundary type on the three axes, a
    ragged column tile and runs of z-planes shorter than the mesh."""
    from paper_1302_2132_amd import Batch, Solver
    bc = [["dirichlet", "outflow"], ["wall", "profile"], ["outflow", "wall"]]
    c = C.uniform_flow(dim=3, n=(70, 9, 13), bc=bc, vel=(0.4, 0.1, -0.2))
    rng = np.random.default_rng(11)
    c.W = c.W * (1.0 + 0.05 * rng.uniform(-1, 1, size=c.W.shape))
    c.kw_transport = True
    c.precision = precision
    banner(f"marching vs per-cell transport strain, {precision}")
    a = Solver(c)
    a.step(7)
    Wa, Ta, Ka = a.fields("cons"), a.fields("turb_cons"), a.fields("turb")
    a.close()
    s = Solver(c)
    b = Batch([s])
    b.step(7)
    assert b.status()["steps"][0] == 7
    Wb, Tb, Kb = s.fields("cons"), s.fields("turb_cons"), s.fields("turb")
    b.close()
    s.close()
    assert np.array_equal(Wa, Wb)
    assert np.array_equal(Ta, Tb)
    assert np.array_equal(Ka, Kb)
