"""Third-order MUSCL face values (recon = GKS_RECON_MUSCL3) on the GPU against the oracle on
the same seeded inputs: FP64 flux <= 1e-12 and FP32 flux <= 1e-5 per field, normwise, as in
the second-order parity tests; also combined with k-omega transport and the tau_hat mode."""
import numpy as np
import pytest

import oracle
from gpu_util import assert_matches_oracle, banner, field_errors, run_gpu
from inputs import cases as C

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


def _compare(case, nsteps, tol, changes=True):
    case = case.copy()
    case.recon = "muscl3"
    banner(f"muscl3: {case.name} {case.precision} steps={nsteps}")
    Wg, rg = run_gpu(case, nsteps)
    ro = oracle.run(case, nsteps)
    err = assert_matches_oracle(Wg, case, ro, tol)
    assert rg["steps"] == ro["steps"]
    assert abs(rg["t"] - ro["t"]) <= (1e-13 if tol <= TOL64 else 1e-5) * max(ro["t"], 1e-300)
    if changes:       # the reconstruction changed the result
        case.recon = "muscl2"
        r2 = oracle.run(case, nsteps)
        assert np.max(field_errors(r2["W"], ro["W"])) > 10 * tol


def test_muscl3_mixing_layer_fp64():
    _compare(C.mixing_layer(64, seed=3), 60, TOL64)


def test_muscl3_sbli_fp64_all_boundaries():
    _compare(C.sbli(96, 48), 40, TOL64)


def test_muscl3_isotropic_3d_fp64():
    _compare(C.isotropic_box(16, precision="fp64"), 12, TOL64)


def test_muscl3_3d_mixed_boundaries_fp64():
    bc = [["dirichlet", "outflow"], ["wall", "profile"], ["outflow", "wall"]]
    c = C.uniform_flow(dim=3, n=(9, 7, 6), bc=bc, vel=(0.4, 0.1, -0.2))
    rng = np.random.default_rng(3)
    c.W = c.W * (1.0 + 0.05 * rng.uniform(-1, 1, size=c.W.shape))
    _compare(c, 6, TOL64)


@pytest.mark.parametrize("n", [(2, 2, 1), (67, 3, 1), (9, 7, 5)])
def test_muscl3_ragged_sizes(n):
    dim = 3 if n[2] > 1 else 2
    c = C.uniform_flow(dim=dim, n=n, bc=[["periodic", "periodic"]] * dim)
    rng = np.random.default_rng(sum(n))
    c.W = c.W * (1.0 + 0.05 * rng.uniform(-1, 1, size=c.W.shape))
    # with two cells on a periodic axis the one-sided slopes always differ in sign, so
    # both reconstructions give zero slopes there
    _compare(c, 4, TOL64, changes=min(n[:dim]) > 2)


def test_muscl3_fp32_flux_2d_and_3d():
    _compare(C.mixing_layer(64, seed=3, precision="fp32_flux"), 60, TOL32)
    _compare(C.isotropic_box(16, precision="fp32_flux"), 12, TOL32)


@pytest.mark.parametrize("dim", [2, 3])
def test_muscl3_with_transport_and_tauhat(dim):
    from paper_1302_2132_amd import Solver
    c = C.mixing_layer(48, seed=4) if dim == 2 else C.isotropic_box(12, precision="fp64")
    c.recon, c.eps_mode, c.kw_transport = "muscl3", "tauhat", True
    n = 30 if dim == 2 else 8
    banner(f"muscl3 + tau_hat + k-omega transport: {c.name} steps={n}")
    s = Solver(c)
    try:
        s.step(n)
        W, kw, e = s.fields("cons"), s.fields("turb"), s.fields("eps")
    finally:
        s.close()
    ro = oracle.run_kw(c, n)
    err = field_errors(W, ro["W"])
    ek = np.max(np.abs(kw[0] - ro["k"])) / np.max(np.abs(ro["k"]))
    ew = np.max(np.abs(kw[1] - ro["omega"])) / np.max(np.abs(ro["omega"]))
    print(f"  flow errors {err}  k {ek:.3e}  omega {ew:.3e}", flush=True)
    assert np.all(err <= TOL64) and ek <= TOL64 and ew <= TOL64
    eo = oracle.eps_field(c, W, kw[0], kw[1])
    assert np.max(np.abs(e - eo)) <= 1e-12 * max(eo.max(), 1e-300)


def test_muscl3_sbli_full_size_one_step():
    from paper_1302_2132_amd import Solver
    c = C.sbli()
    c.recon = "muscl3"
    banner(f"muscl3: {c.name} full size, one step after 10")
    s = Solver(c)
    try:
        s.step(10)
        Wa = s.fields("cons")
        ra = s.residual()
        s.step(1)
        Wb = s.fields("cons")
        rb = s.residual()
    finally:
        s.close()
    ro = oracle.run(c, 1, W=Wa, t0=ra["t"])
    assert abs(rb["dt"] - ro["dt"]) <= 1e-13 * ro["dt"]
    err = field_errors(Wb, ro["W"])
    print(f"  field errors {err}", flush=True)
    assert np.all(err <= TOL64)
