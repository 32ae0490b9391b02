"""Served form: requests admitted by HBM footprint into a running batch give, each, the
same result as the same solve run alone (bitwise), the FIFO loop agrees too, and every
served result matches the oracle (FP64 1e-12, FP32 flux 1e-5, per field).  A request
whose residual falls by its tolerance before its step cap is stopped by the device at
that step, alone, in the mix and in the FIFO loop alike, as the oracle's residuals say."""
import numpy as np
import pytest

import oracle
from gpu_util import assert_matches_oracle, banner, oracle_reference
from inputs import cases as C

pytestmark = pytest.mark.gpu


def _damped_noise(seed):
    """A uniform flow with a small random perturbation on a coarse periodic grid with a
    large viscosity: its residual falls steadily (by 10x in ~50 steps)."""
    c = C.uniform_flow(dim=2, n=(24, 20, 1), vel=(0.3, 0.1), mu=5e-2, stretched=False)
    rng = np.random.default_rng(seed)
    c.W = c.W * (1 + 1e-3 * rng.uniform(-1, 1, c.W.shape))
    c.k[:] = 0.0
    c.name = f"damped_noise_{seed}"
    return c


def _make(req):
    fam, side, seed = req["family"], req["side"], req["seed"]
    if fam == 0:
        c = C.mixing_layer(side, seed=seed, precision="fp64")
    elif fam == 1:
        c = C.sbli(side, side // 2, seed=seed, precision="fp32_flux")
    elif fam == 2:
        c = C.isotropic_box(side, seed=seed, precision="fp32_flux")
    else:
        c = _damped_noise(seed)
    c.max_steps = req["max_steps"]
    return c


def _trace(converging=False):
    rng = np.random.default_rng(9)
    reqs, t = [], 0.0
    for i in range(7):
        t += float(rng.exponential(0.05))
        fam = i % 3
        side = int(rng.integers(10, 16)) if fam == 2 else int(rng.integers(24, 48))
        reqs.append({"id": i, "arrival": t, "family": fam, "side": side, "seed": int(rng.integers(1 << 30)),
                     "max_steps": int(rng.integers(15, 40)), "tol": 1e-12})
    if converging:
        for j, tol in enumerate((0.1, 0.05)):
            reqs.append({"id": 7 + j, "arrival": reqs[2 + 2 * j]["arrival"] + 1e-3, "family": 3, "side": 0,
                         "seed": 21 + j, "max_steps": 400, "tol": tol})
    return reqs


def _alone(case, tol, nsteps):
    from paper_1302_2132_amd import Solver
    case = case.copy()
    case.res_tol = tol
    s = Solver(case)
    try:
        s.step(nsteps)
        return s.fields("cons"), s.residual()
    finally:
        s.close()


def _oracle_until_converged(case, tol, max_steps):
    """The oracle stepped one step at a time with the stopping rule: the first step n >= 2
    with max_m res_m / res_first_m <= tol over the fields with res_first_m > 0."""
    W, t, first = case.W, 0.0, None
    for n in range(1, max_steps + 1):
        r = oracle.run(case, 1, W=W, t0=t)
        W, t = r["W"], r["t"]
        if first is None:
            first = r["res"].copy()
        mask = first > 0
        if n >= 2 and np.any(mask) and np.max(r["res"][mask] / first[mask]) <= tol:
            return W, n
    return W, max_steps


def test_served_equals_standalone_and_the_oracle():
    from paper_1302_2132_amd import config_from_case, gks_workspace_bytes
    from paper_1302_2132_amd.serve import run_batched, run_fifo
    reqs = _trace()
    biggest = max(gks_workspace_bytes(config_from_case(_make(r))) for r in reqs)
    banner("serving 7 requests, budget 2 solves")
    summ, recs = run_batched(reqs, _make, hbm_budget=2 * biggest, capacity=4, quantum=6, keep_fields=True)
    assert summ["requests"] == len(reqs)
    fsumm, frecs = run_fifo(reqs, _make, quantum=6, keep_fields=True)
    for r in reqs:
        rec = recs[r["id"]]
        assert rec["steps"] == r["max_steps"]
        case = _make(r)
        W, _ = _alone(case, r["tol"], r["max_steps"])
        assert np.array_equal(rec["fields"], W), r
        assert np.array_equal(frecs[r["id"]]["fields"], W), r
        tol = 1e-12 if case.precision == "fp64" else 1e-5
        assert_matches_oracle(rec["fields"], case, oracle.run(case, r["max_steps"]), tol, label=f"req {r['id']}: ")


def test_served_request_stops_when_converged():
    from paper_1302_2132_amd import config_from_case, gks_workspace_bytes
    from paper_1302_2132_amd.serve import run_batched, run_fifo
    reqs = _trace(converging=True)
    biggest = max(gks_workspace_bytes(config_from_case(_make(r))) for r in reqs)
    banner("serving 9 requests, two of them converging before their cap")
    summ, recs = run_batched(reqs, _make, hbm_budget=3 * biggest, capacity=4, quantum=6, keep_fields=True)
    fsumm, frecs = run_fifo(reqs, _make, quantum=6, keep_fields=True)
    for r in reqs[7:]:
        case = _make(r)
        Wo, n_oracle = _oracle_until_converged(case, r["tol"], r["max_steps"])
        assert 2 < n_oracle < r["max_steps"]
        W, res = _alone(case, r["tol"], r["max_steps"])      # the device stops it by itself
        assert res["steps"] == n_oracle, (res["steps"], n_oracle)
        for rec in (recs[r["id"]], frecs[r["id"]]):
            assert rec["steps"] == n_oracle
            assert np.array_equal(rec["fields"], W), r
        assert_matches_oracle(W, case, {"W": Wo}, 1e-12, label=f"req {r['id']}: ")
    # the throughput counts the steps the solves took, not the quanta that ran past them
    total = sum(recs[r["id"]]["steps"] * recs[r["id"]]["cells"] for r in reqs)
    assert abs(summ["cell_updates_per_s"] * summ["makespan_s"] - total) <= 1e-6 * total


def _make_with_options(req):
    """The same requests carrying options: WENO5 with transport (mixing layers), the
    multi-dimensional expansion with transport (SBLI), and the multi-dimensional expansion
    in the tau_hat mode (isotropic boxes)."""
    c = _make(req)
    opts = [dict(recon="weno5", kw_transport=True), dict(multi_d=True, kw_transport=True),
            dict(multi_d=True, eps_mode="tauhat")][req["family"]]
    for k, v in opts.items():
        setattr(c, k, v)
    return c


def test_served_with_options_equals_standalone_and_the_oracle():
    from paper_1302_2132_amd import config_from_case, gks_workspace_bytes
    from paper_1302_2132_amd.serve import run_batched
    reqs = _trace()
    biggest = max(gks_workspace_bytes(config_from_case(_make_with_options(r))) for r in reqs)
    banner("serving 7 requests with options, budget 2 solves")
    summ, recs = run_batched(reqs, _make_with_options, hbm_budget=2 * biggest, capacity=4, quantum=6,
                             keep_fields=True)
    assert summ["requests"] == len(reqs)
    for r in reqs:
        rec = recs[r["id"]]
        assert rec["steps"] == r["max_steps"]
        case = _make_with_options(r)
        W, _ = _alone(case, r["tol"], r["max_steps"])
        assert np.array_equal(rec["fields"], W), r
        tol = 1e-12 if case.precision == "fp64" else 1e-5
        assert_matches_oracle(rec["fields"], case, oracle_reference(case, r["max_steps"]), tol,
                              label=f"req {r['id']}: ")
