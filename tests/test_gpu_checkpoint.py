"""Checkpoint/resume: stepping n, saving the solve (gks_fields CONS, TURB_CONS with
transport, and what gks_residual reports), re-initialising a new handle from the saved
state with gks_resume and stepping m gives, bitwise, the state, residuals, time and step
count of n + m steps straight through.  Covered: the frozen 2D SBLI case in FP64 and FP32
flux, the transported mixing layer, the fused 3D box, WENO5 with the tau_hat mode, a
t_end-clipped shock tube, max_steps and res_tol stops that straddle the checkpoint, and a
resumed solve inside a batch.  Misuse is refused with the documented status."""
import numpy as np
import pytest

from gpu_util import banner
from inputs import cases as C

pytestmark = pytest.mark.gpu


def _straight(case, steps):
    from paper_1302_2132_amd import Solver
    s = Solver(case)
    try:
        s.step(steps)
        return s.checkpoint()
    finally:
        s.close()


def _resumed(case, n, m):
    from paper_1302_2132_amd import Solver
    a = Solver(case)
    try:
        a.step(n)
        ck = a.checkpoint()
    finally:
        a.close()
    b = Solver(case, resume=ck)
    try:
        b.step(m)
        return b.checkpoint()
    finally:
        b.close()


def _same(x, y):
    assert x["steps"] == y["steps"], (x["steps"], y["steps"])
    assert x["t"] == y["t"] and x["dt"] == y["dt"], (x["t"], y["t"], x["dt"], y["dt"])
    assert np.array_equal(x["res"], y["res"]) and np.array_equal(x["res_first"], y["res_first"])
    assert np.array_equal(x["W"], y["W"])
    if "turb_cons" in x:
        assert np.array_equal(x["turb_cons"], y["turb_cons"])


def _check(case, n, m):
    banner(f"checkpoint/resume: {case.name} {case.precision} {n} + {m} steps")
    _same(_straight(case, n + m), _resumed(case, n, m))


@pytest.mark.parametrize("precision", ["fp64", "fp32_flux"])
def test_resume_sbli(precision):
    _check(C.sbli(96, 48, precision=precision), 17, 13)


def test_resume_mixing_layer_with_transport():
    c = C.mixing_layer(48, seed=4)
    c.kw_transport = True
    _check(c, 12, 9)


def test_resume_fused_3d_box():
    _check(C.isotropic_box(16, precision="fp32_flux"), 5, 4)


def test_resume_weno5_tauhat():
    c = C.mixing_layer(40, seed=6)
    c.recon = "weno5"
    c.eps_mode = "tauhat"
    _check(c, 10, 10)


def test_resume_clips_at_t_end():
    c = C.shock_tube(64, 4, mu=1e-4)
    c.t_end = 0.73 * _straight(c, 40)["t"]
    full = _straight(c, 100)
    assert full["t"] == c.t_end and full["steps"] < 40
    half = full["steps"] // 2
    _same(full, _resumed(c, half, 100))


def test_resume_counts_towards_max_steps():
    c = C.sbli(64, 32)
    c.max_steps = 20
    full = _straight(c, 50)
    assert full["steps"] == 20
    _same(full, _resumed(c, 12, 50))


def test_resume_keeps_the_residual_stop():
    c = C.uniform_flow(dim=2, n=(24, 20, 1), vel=(0.3, 0.1), mu=5e-2, stretched=False)
    rng = np.random.default_rng(21)
    c.W = c.W * (1 + 1e-3 * rng.uniform(-1, 1, c.W.shape))
    c.k[:] = 0.0
    c.res_tol = 0.1
    full = _straight(c, 400)
    assert 4 < full["steps"] < 400
    _same(full, _resumed(c, full["steps"] // 2, 400))
    # saved after the stop, the resumed solve takes no further step
    _same(full, _resumed(c, full["steps"] + 5, 50))


def test_resumed_solve_in_a_batch():
    from paper_1302_2132_amd import Batch, Solver
    cases = [C.mixing_layer(32, seed=1), C.sbli(48, 24, precision="fp32_flux"), C.isotropic_box(12)]
    want = [_straight(c, 16) for c in cases]
    first = []
    for c in cases:
        s = Solver(c)
        s.step(7)
        first.append(s.checkpoint())
        s.close()
    solvers = [Solver(c, resume=ck) for c, ck in zip(cases, first)]
    b = Batch(solvers)
    try:
        b.step(9)
        b.status()
        got = [s.checkpoint() for s in solvers]
    finally:
        b.close()
        for s in solvers:
            s.close()
    for x, y in zip(want, got):
        _same(x, y)


def test_resume_misuse_is_refused():
    from paper_1302_2132_amd import GKS_ERR_ARG, GKS_ERR_STATE, GksError, Solver, gks_resume
    c = C.mixing_layer(16)
    s = Solver(c)
    try:
        s.step(2)
        ck = s.checkpoint()
        with pytest.raises(GksError) as e:            # the handle has stepped
            gks_resume(s.h, ck["res"], ck["res_first"], ck["dt"], ck["t"], ck["steps"])
        assert e.value.status == GKS_ERR_STATE
    finally:
        s.close()
    fresh = Solver(c)
    try:
        for args in [(ck["res"], ck["res_first"], ck["dt"], -1.0, 2), (ck["res"], ck["res_first"], ck["dt"], 0.1, -1),
                     (np.full(4, np.nan), None, 0.0, 0.1, 2), (None, None, np.inf, 0.1, 2)]:
            with pytest.raises(GksError) as e:
                gks_resume(fresh.h, *args)
            assert e.value.status == GKS_ERR_ARG, args
        with pytest.raises(GksError) as e:            # rho k without transport
            gks_resume(fresh.h, None, None, 0.0, 0.0, 0, np.ones((2,) + c.k.shape))
        assert e.value.status == GKS_ERR_ARG
        # the refusals left the handle usable
        fresh.step(2)
        assert fresh.residual()["steps"] == 2
    finally:
        fresh.close()
