"""A seeded sweep of random configurations against the oracle: dimension, ragged sizes,
the boundary type of every side (periodic pairs, walls, fixed states and profiles,
outflow), reconstruction (MUSCL2, MUSCL3, WENO5), eps mode, k-omega transport, the
multi-dimensional expansion (with MUSCL2 only) and the precision form, drawn per seed
(numpy default_rng).  Each solve takes 12 steps from a perturbed uniform state on a
randomly stretched grid and is compared per field with the oracle (FP64 1e-12, FP32 flux
1e-5, as the other parity tests)."""
import numpy as np
import pytest

import oracle
from gpu_util import assert_matches_oracle, banner
from inputs import cases as C

pytestmark = pytest.mark.gpu

SIDES = ["wall", "dirichlet", "profile", "outflow"]


def random_case(seed):
    rng = np.random.default_rng(1000 + seed)
    dim = int(rng.choice([2, 3]))
    recon = str(rng.choice(["muscl2", "muscl3", "weno5"]))
    lo = 3 if recon == "weno5" else 2
    n = [int(rng.integers(lo + 3, 40 if dim == 2 else 14)) for _ in range(dim)] + ([1] if dim == 2 else [])
    bc = []
    for d in range(dim):
        if rng.uniform() < 0.3:
            bc.append(["periodic", "periodic"])
        else:
            bc.append([str(rng.choice(SIDES)), str(rng.choice(SIDES))])
    vel = tuple(0.3 * rng.uniform(-1, 1, 3))
    c = C.uniform_flow(dim=dim, n=tuple(n), bc=bc, vel=vel, seed=int(seed), mu=float(10 ** rng.uniform(-4, -2)))
    c.W = c.W * (1.0 + 0.04 * rng.uniform(-1, 1, size=c.W.shape))
    c.recon = recon
    c.eps_mode = str(rng.choice(["dt", "tauhat"]))
    c.kw_transport = bool(rng.uniform() < 0.4)
    c.multi_d = bool(recon == "muscl2" and rng.uniform() < 0.3)
    c.precision = str(rng.choice(["fp64", "fp32_flux"]))
    c.c_a = float(rng.choice([0.0, 0.3]))
    return c


@pytest.mark.parametrize("seed", range(16))
def test_random_configuration_matches_the_oracle(seed):
    from paper_1302_2132_amd import Solver
    c = random_case(seed)
    label = (f"seed {seed}: {c.dim}D {c.n[:c.dim]} bc {c.bc} {c.recon} {c.eps_mode} kw={c.kw_transport} "
             f"md={c.multi_d} {c.precision} c_a={c.c_a}")
    banner(label)
    s = Solver(c)
    try:
        s.step(12)
        W = s.fields("cons")
        turb = s.fields("turb") if c.kw_transport else None        # k, omega of the state
        r = s.residual()
    finally:
        s.close()
    ref = oracle.run_kw(c, 12) if c.kw_transport else oracle.run(c, 12)
    tol = 1e-12 if c.precision == "fp64" else 1e-5
    assert r["steps"] == 12
    assert abs(r["t"] - ref["t"]) <= tol * ref["t"]
    assert_matches_oracle(W, c, ref, tol, label)
    if c.kw_transport:
        for m, key in enumerate(("k", "omega")):
            e = float(np.max(np.abs(turb[m] - ref[key]))) / float(np.max(np.abs(ref[key])))
            assert e <= tol, (label, key, e)
