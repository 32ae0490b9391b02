"""Pins of the oracle's sampled-cell step and of the k-omega ghost-density reading.

`oracle.step_cells` (og_step_cells) recomputes the update of selected cells on its own
(the two faces per axis of each cell, then the flux differences), separately from the
whole-mesh step of `oracle.run` (every face once, then og_update).  It is the checker of
the full-size GPU tests, so it is tied here to one step of `oracle.run` at every cell, on
small stretched meshes with every boundary type, each reconstruction and the
multi-dimensional expansion: the two may differ only by the rounding order of the flux
differences (the update of the finite-volume section, W - sum_d (F_hi - F_lo)/dx_d).

The k-omega transport takes a ghost cell's k and omega from its interior image (the
zero-gradient reading: the API supplies k and omega for interior cells only).  At every
non-periodic boundary face the ghost's image is the face's interior cell itself, so the
k and omega differences across that face vanish and the diffusive flux is zero whatever
density the face's eddy-viscosity mean takes for the ghost; at a periodic face the ghost
is an interior cell.  The second test builds the oracle with the other reading (the
ghost-filled density, e.g. a Dirichlet state's) and shows the two runs agree bitwise on
a case whose boundary densities differ from the interior.
"""
import subprocess

import numpy as np
import pytest

import oracle
from inputs import cases as C


def _perturbed(case, seed, amp=0.05):
    rng = np.random.default_rng(seed)
    case.W = case.W * (1.0 + amp * rng.uniform(-1, 1, size=case.W.shape))
    for d in range(case.dim):
        for s in range(2):
            bd = case.bc_data[d][s]
            if bd is not None:
                case.bc_data[d][s] = bd * (1.0 + amp * rng.uniform(-1, 1, size=bd.shape))
    return case


def _mixed(dim, **opts):
    if dim == 2:
        bc = [["dirichlet", "outflow"], ["wall", "profile"]]
        c = C.uniform_flow(dim=2, n=(9, 7, 1), bc=bc, vel=(0.4, 0.1))
    else:
        bc = [["dirichlet", "outflow"], ["wall", "profile"], ["periodic", "periodic"]]
        c = C.uniform_flow(dim=3, n=(6, 5, 4), bc=bc, vel=(0.4, 0.1, -0.2))
    c = _perturbed(c, 7 + dim)
    for k, v in opts.items():
        setattr(c, k, v)
    return c


CASES = {
    "2d_mixed_bc": lambda: _mixed(2),
    "2d_mixed_bc_c_a": lambda: _mixed(2, c_a=1.0),
    "2d_mixed_bc_muscl3": lambda: _mixed(2, recon="muscl3"),
    "2d_mixed_bc_weno5": lambda: _mixed(2, recon="weno5"),
    "2d_mixed_bc_multi_d": lambda: _mixed(2, multi_d=True),
    "2d_mixed_bc_tauhat": lambda: _mixed(2, eps_mode="tauhat"),
    "2d_mixing_layer": lambda: C.mixing_layer(16, seed=3),
    "2d_sbli": lambda: C.sbli(24, 12),
    "3d_mixed_bc": lambda: _mixed(3),
    "3d_mixed_bc_weno5": lambda: _mixed(3, recon="weno5"),
    "3d_mixed_bc_multi_d": lambda: _mixed(3, multi_d=True),
    "3d_isotropic": lambda: C.isotropic_box(8, precision="fp64"),
}


def step_cells_matches_run(name):
    case = CASES[name]()
    W0 = case.W.copy()
    r = oracle.run(case, 1, nthreads=2)
    assert r["steps"] == 1
    cells = np.arange(case.ncells)
    got = oracle.step_cells(case, W0, r["dt"], cells, nthreads=2).T.reshape(case.W.shape)
    ref = r["W"]
    for m in range(case.nvar):
        scale = np.max(np.abs(ref[m]))
        err = np.max(np.abs(got[m] - ref[m])) / scale
        # one subtraction of the flux differences rounded in another order: a few ulps of |W|
        assert err <= 8 * np.finfo(np.float64).eps, (name, m, err)
        # and the change over the step agrees far beyond the FP64 parity bound
        dW = ref[m] - W0[m]
        if np.max(np.abs(dW)) > 0:
            assert np.max(np.abs(got[m] - ref[m])) <= 1e-12 * np.max(np.abs(dW)) + 8 * np.finfo(float).eps * scale


@pytest.mark.parametrize("name", sorted(CASES))
def test_step_cells_equals_one_step_of_run(name):
    step_cells_matches_run(name)


def test_step_cells_on_a_sample_equals_the_full_list():
    case = _mixed(2)
    dt = oracle.cfl_dt(case)
    all_ = oracle.step_cells(case, case.W, dt, np.arange(case.ncells))
    pick = np.array([0, 5, 17, case.ncells - 1])
    some = oracle.step_cells(case, case.W, dt, pick)
    assert np.array_equal(some, all_[pick])


# --------------------------------------------------------------------------------------
# k-omega ghost density: the two readings coincide
# --------------------------------------------------------------------------------------
GHOST_DENSITY_READING = [
    ("static void og_kw_face(const og_grid* gr, const double* W, const double* kk, const double* om, int d,",
     "static void og_kw_face(const og_grid* gr, const double* W, const double* We, const double* kk, const double* om, int d,"),
    ("const double rl = og_kw_at(gr, W, cl), rr = og_kw_at(gr, W, cr);",
     "const double rl = We[gidx(gr, cl[0], cl[1], cl[2])], rr = We[gidx(gr, cr[0], cr[1], cr[2])];"),
    ("og_kw_face(gr, W, kk, om, d, fi, fj, fk, Fl[0], dt, &Fk[d][f], &Fw[d][f]);",
     "og_kw_face(gr, W, We, kk, om, d, fi, fj, fk, Fl[0], dt, &Fk[d][f], &Fw[d][f]);"),
]


def _transport_case(dim):
    case = _mixed(dim, kw_transport=True)
    rng = np.random.default_rng(11)
    # strongly varying k and omega, and boundary states whose density differs from the
    # interior by up to 30 %
    case.k = rng.uniform(1e-3, 5e-2, size=case.k.shape)
    case.omega = rng.uniform(0.5, 20.0, size=case.k.shape)
    for d in range(case.dim):
        for s in range(2):
            bd = case.bc_data[d][s]
            if bd is not None:
                case.bc_data[d][s] = bd * (1.0 + 0.3 * rng.uniform(0.2, 1.0))
    return case


@pytest.mark.parametrize("dim", [2, 3])
def test_kw_ghost_density_reading_does_not_change_results(dim, tmp_path):
    with open(oracle.SRC) as f:
        src = f.read()
    for old, new in GHOST_DENSITY_READING:
        assert src.count(old) == 1, old
        src = src.replace(old, new)
    path = tmp_path / "ghost_density.c"
    path.write_text(src)
    so = tmp_path / "libghost_density.so"
    subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                           "-o", str(so), str(path), "-lm"])
    case = _transport_case(dim)
    ref = oracle.run_kw(case, 6, nthreads=2)
    oracle.use_library(str(so))
    try:
        alt = oracle.run_kw(case, 6, nthreads=2)
    finally:
        oracle.use_library(None)
    assert ref["steps"] == alt["steps"] == 6
    for key in ("W", "k", "omega"):
        assert np.array_equal(ref[key], alt[key]), key
    # the case does exercise boundary diffusion coefficients that differ between the readings
    ghost = oracle.ghost_fill(case)
    assert abs(ghost[0, 0 if dim == 2 else 2, 2 if dim == 2 else 2, 1] - case.W[0, 0, 0, 0]) > 1e-3
