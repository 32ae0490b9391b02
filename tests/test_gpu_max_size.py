"""The largest mesh the library accepts: 2^29 cells (32768 x 16384 in 2D), the limit of the
kernels' 32-bit cell and face indexing.  A perturbed uniform flow on a stretched grid with
inflow/outflow in x and a wall and a fixed profile in y takes one step, checked against the
oracle's per-cell step (the oracle's checker for full-size meshes) at sampled cells, the first
and last 64 cells and the last tile's among them.  About 50 GB of HBM and 70 GB of host
memory; each phase prints its time."""
import time

import numpy as np
import pytest

import oracle
from gpu_util import banner
from inputs import cases as C

pytestmark = pytest.mark.gpu

NX, NY = 32768, 16384
TOL64 = 1e-12


def _case():
    """Built in place (row blocks) rather than through the generic generators, whose
    broadcast copies and temporaries would take minutes at this size."""
    g = 1.4
    rng = np.random.default_rng(29)
    xf = []
    for n in (NX, NY):
        w = rng.uniform(0.5, 2.0, size=n)
        xf.append(np.concatenate([[0.0], np.cumsum(w)]) / w.sum())
    W0 = C.cons_from_prim(1.3, [0.4, -0.1], 0.9, g)
    W = np.empty((4, 1, NY, NX))
    k = np.empty((1, NY, NX))
    om = np.empty((1, NY, NX))
    sx = np.sin(np.arange(NX) * 0.37)
    for j0 in range(0, NY, 1024):
        j1 = min(NY, j0 + 1024)
        sy = np.cos(np.arange(j0, j1) * 0.23)
        pert = np.outer(sy, sx)
        for m in range(4):
            W[m, 0, j0:j1] = W0[m] * (1.0 + (0.02 + 0.005 * m) * pert)
        k[0, j0:j1] = 1e-3 * (1.5 + pert)
        om[0, j0:j1] = 5.0 * (1.5 - 0.5 * pert)
    bcd = [[W0.copy(), None], [None, np.repeat(W0[:, None], NX, axis=1).copy()]]
    return C.Case(name="uniform_2d_2^29", dim=2, n=(NX, NY, 1), xf=xf, bc=[["dirichlet", "outflow"], ["wall", "profile"]],
                  bc_data=bcd, W=W, k=k, omega=om, gamma=g, prandtl=0.72, mu=1e-3, c_a=0.0, cfl=0.5, steps=1)


def test_largest_accepted_mesh_one_step_sampled():
    from paper_1302_2132_amd import Solver
    t0 = time.perf_counter()
    case = _case()
    assert case.ncells == 1 << 29
    banner(f"2^29-cell mesh built in {time.perf_counter() - t0:.1f} s")
    s = Solver(case)
    try:
        banner(f"initialised at {time.perf_counter() - t0:.1f} s")
        s.step(1)
        r = s.residual()
        Wb = s.fields("cons")
    finally:
        s.close()
    banner(f"stepped and read back at {time.perf_counter() - t0:.1f} s")
    assert r["steps"] == 1
    dt = oracle.cfl_dt(case, case.W)
    assert abs(r["dt"] - dt) <= 1e-13 * dt, (r["dt"], dt)
    rng = np.random.default_rng(3)
    N = case.ncells
    last_tile = [(NY - 1 - j) * NX + NX - 1 - i for j in range(3) for i in range(20)]
    cells = np.unique(np.concatenate([rng.integers(0, N, size=3000), np.arange(64), np.arange(N - 64, N),
                                      np.array(last_tile), NX * np.arange(0, NY, 997)]))
    new = oracle.step_cells(case, case.W, r["dt"], cells)
    got = Wb.reshape(4, -1)[:, cells].T
    old = case.W.reshape(4, -1)[:, cells].T
    scale = np.max(np.abs(case.W.reshape(4, -1)), axis=1)
    err = np.max(np.abs(got - new), axis=0) / scale
    change = np.max(np.abs(new - old), axis=0)
    banner(f"checked at {time.perf_counter() - t0:.1f} s: per-field errors {err}, step's largest change {change}")
    assert np.all(change > 0.0)
    assert np.all(err <= TOL64), err
