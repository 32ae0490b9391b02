"""Multi-dimensional expansion (multi_d) on the GPU against the oracle on the same seeded
inputs: FP64 flux <= 1e-12 and FP32 flux <= 1e-5 per field, normwise.  The cases cover
every boundary type, so the corner ghosts of the tangential gradients (two ghost axes)
are exercised in 2D and 3D."""
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
    case.multi_d = True
    banner(f"multi-d: {case.name} {case.precision} steps={nsteps}")
    Wg, rg = run_gpu(case, nsteps)
    ro = oracle.run(case, nsteps)
    err = assert_matches_oracle(Wg, case, ro, tol)
    assert rg["steps"] == ro["steps"]
    assert abs(rg["t"] - ro["t"]) <= (1e-13 if tol <= TOL64 else 1e-5) * max(ro["t"], 1e-300)
    if changes:
        case.multi_d = False
        r1 = oracle.run(case, nsteps)
        assert np.max(field_errors(r1["W"], ro["W"])) > 10 * tol


def test_multid_mixing_layer_fp64():
    _compare(C.mixing_layer(64, seed=3), 40, TOL64)


def test_multid_sbli_fp64_all_boundaries():
    _compare(C.sbli(96, 48), 30, TOL64)


def test_multid_2d_corners_of_every_boundary_pair():
    bc = [["dirichlet", "outflow"], ["wall", "profile"]]
    c = C.uniform_flow(dim=2, n=(19, 17, 1), bc=bc, vel=(0.3, -0.2, 0.0), seed=4)
    rng = np.random.default_rng(8)
    c.W = c.W * (1.0 + 0.05 * rng.uniform(-1, 1, size=c.W.shape))
    _compare(c, 6, TOL64)


def test_multid_isotropic_3d_fp64():
    _compare(C.isotropic_box(16, precision="fp64"), 8, TOL64)


def test_multid_3d_mixed_boundaries_fp64():
    bc = [["dirichlet", "outflow"], ["wall", "profile"], ["outflow", "wall"]]
    c = C.uniform_flow(dim=3, n=(9, 7, 6), bc=bc, vel=(0.4, 0.1, -0.2))
    rng = np.random.default_rng(3)
    c.W = c.W * (1.0 + 0.05 * rng.uniform(-1, 1, size=c.W.shape))
    _compare(c, 5, TOL64)


@pytest.mark.parametrize("n", [(2, 2, 1), (67, 3, 1), (9, 7, 5)])
def test_multid_ragged_sizes(n):
    dim = 3 if n[2] > 1 else 2
    c = C.uniform_flow(dim=dim, n=n, bc=[["periodic", "periodic"]] * dim)
    rng = np.random.default_rng(sum(n))
    c.W = c.W * (1.0 + 0.05 * rng.uniform(-1, 1, size=c.W.shape))
    _compare(c, 4, TOL64, changes=min(n[:dim]) > 2)


def test_multid_fp32_flux_2d_and_3d():
    _compare(C.mixing_layer(64, seed=3, precision="fp32_flux"), 40, TOL32)
    _compare(C.isotropic_box(16, precision="fp32_flux"), 8, TOL32)


def test_multid_sbli_full_size_one_step():
    from paper_1302_2132_amd import Solver
    c = C.sbli()
    c.multi_d = True
    banner(f"multi-d: {c.name} full size, one step after 10")
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


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("mode", ["dt", "tauhat"])
def test_multid_with_transport(dim, mode):
    """The expansion with k and omega transported, in either eps_mode, against the oracle's
    transport run; the eps_hat field of the same state."""
    from paper_1302_2132_amd import Solver
    c = C.mixing_layer(48, seed=4) if dim == 2 else C.isotropic_box(12, precision="fp64")
    c.multi_d, c.eps_mode, c.kw_transport = True, mode, True
    n = 30 if dim == 2 else 6
    banner(f"multi-d + k-omega transport, eps_mode {mode}: {c.name} steps={n}")
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


def test_multid_with_tauhat_frozen():
    c = C.mixing_layer(48, seed=6)
    c.eps_mode = "tauhat"
    _compare(c, 30, TOL64)


def test_multid_with_higher_order_face_values_refused():
    from paper_1302_2132_amd import GKS_ERR_ARG, GksError, Solver
    for recon in ("muscl3", "weno5"):
        c = C.mixing_layer(32, seed=2)
        c.multi_d, c.recon = True, recon
        with pytest.raises(GksError) as e:
            Solver(c)
        assert e.value.status == GKS_ERR_ARG
