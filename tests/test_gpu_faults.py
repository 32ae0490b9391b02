"""Failure detection: a non-finite value planted in a solve's device state (through
gks_state_device_ptr, between calls) is caught by the kernels' positivity and finiteness
checks and reported by the next synchronising call as GKS_ERR_NONPHYSICAL; the handle then
refuses steps (GKS_ERR_STATE) but still gives its fields and is destroyed normally.  In a
batch only the poisoned member stops (status 2); the others run on and equal their solves
stepped alone, bitwise, and the serving loop retires just that request.  Every kernel
still exits normally: the planted value only flows through arithmetic."""
import numpy as np
import pytest

from gpu_util import banner
from inputs import cases as C

pytestmark = pytest.mark.gpu


def _plant(solver, field, cell, value=np.nan):
    """Write `value` into component `field` of cell `cell` (flat index) of the current state."""
    import torch
    from paper_1302_2132_amd import gks_state_device_ptr
    ptr = gks_state_device_ptr(solver.h)            # synchronises the solve's stream
    off = ptr - solver.ws.data_ptr()
    n = solver.case.k.size
    assert off % 8 == 0 and 0 <= off and off + 8 * (field + 1) * n <= solver.nbytes
    solver.ws.view(torch.float64)[off // 8 + field * n + cell] = value
    torch.cuda.synchronize()


def _alone(case, steps):
    from paper_1302_2132_amd import Solver
    s = Solver(case)
    try:
        s.step(steps)
        return s.fields("cons")
    finally:
        s.close()


@pytest.mark.parametrize("which", ["density", "energy", "rho_k"])
def test_planted_nan_is_reported(which):
    from paper_1302_2132_amd import GKS_ERR_NONPHYSICAL, GKS_ERR_STATE, GKS_OK, GksError, Solver
    c = C.sbli(64, 32) if which != "rho_k" else C.mixing_layer(32, seed=2)
    if which == "rho_k":
        c.kw_transport = True
    field = {"density": 0, "energy": c.dim + 1, "rho_k": c.dim + 2}[which]
    banner(f"NaN planted in {which} of {c.name}")
    s = Solver(c)
    try:
        s.step(4)
        assert s.residual()["steps"] == 4
        _plant(s, field, c.k.size // 2 + 3)
        s.step(3)
        with pytest.raises(GksError) as e:
            s.residual()
        assert e.value.status == GKS_ERR_NONPHYSICAL
        with pytest.raises(GksError) as e:
            s.step(1)
        assert e.value.status == GKS_ERR_STATE
        W = s.fields("cons")                        # still readable
        assert W.shape == c.W.shape
        planted = s.fields("turb_cons") if which == "rho_k" else W
        assert not np.all(np.isfinite(planted))
    finally:
        assert s.close() in (GKS_OK, GKS_ERR_NONPHYSICAL)


def test_planted_nan_in_k_of_a_frozen_solve():
    """The frozen k field is an input: a NaN written into it on the device reaches the
    relaxation time and the CFL rate, and is reported the same way."""
    import torch
    from paper_1302_2132_amd import GKS_ERR_NONPHYSICAL, GksError, Solver
    c = C.mixing_layer(32, seed=5)
    s = Solver(c)
    try:
        s.step(2)
        # find the k array in the workspace by its values (arrays start on 256-byte bounds)
        ws = s.ws.view(torch.float64)
        host = ws.cpu().numpy()
        k = c.k.reshape(-1)
        n = k.size
        hits = [i for i in range(0, host.size - n + 1, 32) if np.array_equal(host[i:i + n], k)]
        assert len(hits) == 1, hits
        ws[hits[0] + n // 3] = float("nan")
        torch.cuda.synchronize()
        s.step(2)
        with pytest.raises(GksError) as e:
            s.residual()
        assert e.value.status == GKS_ERR_NONPHYSICAL
    finally:
        s.close()


def test_batch_retires_only_the_poisoned_member():
    from paper_1302_2132_amd import Batch, Solver
    cases = [C.mixing_layer(32, seed=1), C.sbli(48, 24, precision="fp32_flux"), C.isotropic_box(12),
             C.mixing_layer(24, seed=3)]
    banner("batch of 4, NaN planted in member 1")
    solvers = [Solver(c) for c in cases]
    b = Batch(solvers)
    try:
        b.step(5)
        b.status()
        _plant(solvers[1], 0, 100)
        b.step(10)
        st = b.status()
        assert list(st["state"]) == [0, 2, 0, 0], st["state"]
        assert st["steps"][0] == st["steps"][2] == st["steps"][3] == 15
        assert st["steps"][1] <= 6
        for i in (0, 2, 3):
            assert np.array_equal(solvers[i].fields("cons"), _alone(cases[i], 15)), i
    finally:
        b.close()
        for s in solvers:
            s.close()


def test_server_retires_a_failing_request():
    """A request whose solve blows up (CFL 50) ends with state 2; the other requests of
    the trace finish with their full step counts and the results of their solves alone."""
    from paper_1302_2132_amd.serve import run_batched

    def make(req):
        c = C.mixing_layer(req["side"], seed=req["seed"])
        if req["bad"]:
            c.cfl = 50.0
        c.max_steps = req["max_steps"]
        return c

    reqs = [{"id": i, "arrival": 0.01 * i, "side": 24 + 4 * i, "seed": i, "max_steps": 20 + i, "tol": 1e-12,
             "bad": i == 2} for i in range(5)]
    summ, recs = run_batched(reqs, make, hbm_budget=1 << 34, capacity=4, quantum=6, keep_fields=True)
    assert recs[2]["state"] == 2
    for r in reqs:
        if r["bad"]:
            continue
        rec = recs[r["id"]]
        assert rec["state"] == 1 and rec["steps"] == r["max_steps"], rec
        assert np.array_equal(rec["fields"], _alone(make(r), r["max_steps"])), r["id"]
