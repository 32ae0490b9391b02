"""Fused tiles whose state window lies inside the mesh address their cells directly; the
others (and, in 3D, planes whose staged plane lies beyond the top) take the ghost rules.
The meshes here hold both kinds: a 16 x 15 tile is direct when its x-y window (two-cell
halo) lies inside the mesh, so x-y extents of at least 34 x 32 cells give interior tiles
beside edge tiles.  Each run is checked against the oracle per field, normwise, after
several steps: FP64 flux <= 1e-12, FP32 flux <= 1e-5.
"""
import numpy as np
import pytest

import oracle
from gpu_util import assert_matches_oracle, banner, run_gpu
from inputs import cases as C

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5

MIXED_BC = [["dirichlet", "outflow"], ["wall", "profile"], ["outflow", "wall"]]


def _mixed_box(precision="fp64", seed=5):
    c = C.uniform_flow(dim=3, n=(40, 34, 7), bc=MIXED_BC, vel=(0.4, 0.1, -0.2))
    rng = np.random.default_rng(seed)
    c.W = c.W * (1.0 + 0.05 * rng.uniform(-1, 1, size=c.W.shape))
    c.precision = precision
    return c


def _compare(case, nsteps, tol):
    banner(f"{case.name} {case.precision} n={case.n} recon={case.recon} eps={case.eps_mode} "
           f"kw={case.kw_transport} steps={nsteps}")
    if case.kw_transport:
        from paper_1302_2132_amd import Solver
        s = Solver(case)
        try:
            s.step(nsteps)
            rg = s.residual()
            Wg = s.fields("cons")
            kw = s.fields("turb")
        finally:
            s.close()
        ro = oracle.run_kw(case, nsteps)
        for got, ref in ((kw[0], ro["k"]), (kw[1], ro["omega"])):
            e = float(np.max(np.abs(got - ref))) / max(float(np.max(np.abs(ref))), 1e-300)
            assert e <= tol, e
    else:
        Wg, rg = run_gpu(case, nsteps)
        ro = oracle.run(case, nsteps, nthreads=0)
    assert_matches_oracle(Wg, case, ro, tol)
    assert rg["steps"] == ro["steps"]
    assert abs(rg["t"] - ro["t"]) <= (1e-13 if tol <= TOL64 else 1e-5) * max(ro["t"], 1e-300)


def test_isotropic_40_fp64():
    # periodic on every axis: interior tiles, and edge tiles whose halos wrap
    _compare(C.isotropic_box(40, precision="fp64"), 8, TOL64)


@pytest.mark.parametrize("option", ["plain", "kw", "muscl3", "tauhat"])
def test_mixed_boundaries_fp64(option):
    # every boundary type on the x-y edges, outflow below and a wall above: the top two
    # planes of each column stage ghost planes
    c = _mixed_box()
    if option == "kw":
        c.kw_transport = True
    elif option == "muscl3":
        c.recon = "muscl3"
    elif option == "tauhat":
        c.eps_mode = "tauhat"
    _compare(c, 6, TOL64)


def test_mixed_boundaries_fp32_flux():
    _compare(_mixed_box("fp32_flux"), 6, TOL32)


def test_mixed_boundaries_2d_fp64():
    # 2D tiles: interior ones beside edge tiles on all four boundary types
    c = C.uniform_flow(dim=2, n=(50, 47, 1), bc=MIXED_BC[:2], vel=(0.4, 0.1))
    rng = np.random.default_rng(6)
    c.W = c.W * (1.0 + 0.05 * rng.uniform(-1, 1, size=c.W.shape))
    _compare(c, 8, TOL64)
