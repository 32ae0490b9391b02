"""Served form: requests admitted by HBM footprint into a running batch give, each, the
same result as the same solve run alone (bitwise), and the FIFO loop agrees too."""
import numpy as np
import pytest

from gpu_util import banner
from inputs import cases as C

pytestmark = pytest.mark.gpu


def _make(req):
    fam, side, seed = req["family"], req["side"], req["seed"]
    if fam == 0:
        c = C.mixing_layer(side, seed=seed, precision="fp64")
    elif fam == 1:
        c = C.sbli(side, side // 2, seed=seed, precision="fp32_flux")
    else:
        c = C.isotropic_box(side, seed=seed, precision="fp32_flux")
    c.max_steps = req["max_steps"]
    return c


def _trace():
    rng = np.random.default_rng(9)
    reqs, t = [], 0.0
    for i in range(7):
        t += float(rng.exponential(0.05))
        fam = i % 3
        side = int(rng.integers(10, 16)) if fam == 2 else int(rng.integers(24, 48))
        reqs.append({"id": i, "arrival": t, "family": fam, "side": side, "seed": int(rng.integers(1 << 30)),
                     "max_steps": int(rng.integers(15, 40)), "tol": 1e-12})
    return reqs


def test_served_equals_standalone():
    from paper_1302_2132_amd import Solver, gks_workspace_bytes, config_from_case
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
        s = Solver(_make(r))
        s.step(r["max_steps"])
        W = s.fields("cons")
        s.close()
        assert np.array_equal(rec["fields"], W), r
        assert np.array_equal(frecs[r["id"]]["fields"], W), r


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


def test_served_with_options_equals_standalone():
    from paper_1302_2132_amd import Solver, gks_workspace_bytes, config_from_case
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
        s = Solver(_make_with_options(r))
        s.step(r["max_steps"])
        W = s.fields("cons")
        s.close()
        assert np.array_equal(rec["fields"], W), r
