"""Batched form: every solve gives the same result alone and inside a persistent batch
(mixed sizes, dimensions, precisions and options; with and without a captured graph), and
the members of an uneven batch and of a batch with every option match the oracle."""
import math

import numpy as np
import pytest

import oracle
from gpu_util import assert_matches_oracle, banner, oracle_reference
from inputs import cases as C

pytestmark = pytest.mark.gpu


def _cases():
    out = [
        C.mixing_layer(40, seed=11),
        C.sbli(48, 24, precision="fp32_flux"),
        C.isotropic_box(10, precision="fp64"),
        C.uniform_flow(dim=3, n=(9, 7, 5), bc=[["dirichlet", "outflow"], ["wall", "wall"], ["periodic", "periodic"]]),
        C.sod_tube(60, ny=2, t_end=0.02),
        C.mixing_layer(33, seed=12, precision="fp32_flux"),
    ]
    out[3].precision = "fp32_flux"
    rng = np.random.default_rng(4)
    out[3].W = out[3].W * (1 + 0.03 * rng.uniform(-1, 1, size=out[3].W.shape))
    return out


def _alone(case, n):
    from paper_1302_2132_amd import Solver
    s = Solver(case)
    s.step(n)
    r = s.residual()
    W = s.fields("cons")
    s.close()
    return W, r


@pytest.mark.parametrize("graph", [False, True])
def test_batch_equals_alone_bitwise(graph):
    from paper_1302_2132_amd import Batch, Solver
    n = 25
    cases = _cases()
    ref = [_alone(c, n) for c in cases]
    banner(f"batch of {len(cases)} graph={graph}")
    solvers = [Solver(c) for c in cases]
    b = Batch(solvers, capacity=8)
    if graph:
        b.capture()
    b.step(n)
    st = b.status()
    for i, (c, s) in enumerate(zip(cases, solvers)):
        W = s.fields("cons")
        r = s.residual()
        assert st["steps"][i] == ref[i][1]["steps"]
        assert np.array_equal(W, ref[i][0]), (i, c.name)
        assert np.array_equal(r["res"], ref[i][1]["res"]), (i, c.name)
        assert r["t"] == ref[i][1]["t"]
    assert st["state"][4] == 1          # the shock tube reached its end time
    b.close()
    for s in solvers:
        s.close()


def test_batch_membership_change_keeps_graph():
    """Admit and retire members between replays of one captured graph."""
    from paper_1302_2132_amd import Batch, Solver
    a, bcase, ccase = C.mixing_layer(24, seed=1), C.mixing_layer(30, seed=2), C.sbli(40, 20)
    ref_b = _alone(bcase, 10)
    ref_c = _alone(ccase, 6)
    sa, sb, sc = Solver(a), Solver(bcase), Solver(ccase)
    b = Batch([sa, sb], capacity=4)
    b.capture()
    b.step(4)
    b.set_members([sb, sc])          # retire a, admit c (same classes: graph kept)
    b.step(6)
    assert np.array_equal(sb.fields("cons"), ref_b[0])
    assert np.array_equal(sc.fields("cons"), ref_c[0])
    b.close()
    for s in (sa, sb, sc):
        s.close()


def test_two_dimensional_batch_then_a_three_dimensional_member():
    """Admitting a 3D member into a captured batch of 2D members brings a new launch class
    (the graph is dropped and the 3D face and update launches join), and every member,
    old and new, still matches its solve alone, bitwise."""
    from paper_1302_2132_amd import Batch, Solver
    a, bcase, ccase = C.mixing_layer(36, seed=3), C.sbli(40, 20, precision="fp32_flux"), C.isotropic_box(8, precision="fp64")
    ref_a, ref_b, ref_c = _alone(a, 9), _alone(bcase, 9), _alone(ccase, 5)
    sa, sb, sc = Solver(a), Solver(bcase), Solver(ccase)
    b = Batch([sa, sb], capacity=4)
    b.capture()
    b.step(4)
    b.set_members([sa, sb, sc])
    b.step(5)
    for s, r in ((sa, ref_a), (sb, ref_b), (sc, ref_c)):
        assert np.array_equal(s.fields("cons"), r[0])
        assert np.array_equal(s.residual()["res"], r[1]["res"])
    b.close()
    for s in (sa, sb, sc):
        s.close()


def _option_cases():
    """Solves with every option and combination class: frozen and transported k-omega, both
    eps modes, the three reconstructions, the multi-dimensional expansion; 2D and 3D, FP64
    and FP32 flux."""
    out = []

    def add(case, **kw):
        for k, v in kw.items():
            setattr(case, k, v)
        out.append(case)

    add(C.mixing_layer(40, seed=11))
    add(C.mixing_layer(36, seed=12), kw_transport=True)
    add(C.mixing_layer(33, seed=13), eps_mode="tauhat")
    add(C.sbli(96, 48, precision="fp32_flux"), recon="muscl3")
    add(C.mixing_layer(34, seed=14), recon="weno5", kw_transport=True)
    add(C.sbli(40, 20), multi_d=True)
    add(C.isotropic_box(10, precision="fp32_flux"), kw_transport=True)
    add(C.isotropic_box(9, precision="fp64"), recon="weno5")
    add(C.isotropic_box(8, precision="fp64"), multi_d=True, eps_mode="tauhat")
    add(C.isotropic_box(10, precision="fp64"))
    return out


def _alone_full(case, n):
    from paper_1302_2132_amd import Solver
    s = Solver(case)
    s.step(n)
    out = (s.fields("cons"), s.residual(), s.fields("turb"))
    s.close()
    return out


@pytest.mark.parametrize("graph", [False, True])
def test_batch_with_every_option_equals_alone_bitwise(graph):
    """Members of every option share one batch: a face launch per (class, variant) pair
    present, the transported form's strain and update passes beside the frozen form's; each
    member's state, residual, time and k, omega equal its solve alone, bitwise."""
    from paper_1302_2132_amd import Batch, Solver
    n = 12
    cases = _option_cases()
    ref = [_alone_full(c, n) for c in cases]
    banner(f"batch of {len(cases)} solves with options, graph={graph}")
    solvers = [Solver(c) for c in cases]
    b = Batch(solvers, capacity=12)
    if graph:
        b.capture()
    b.step(n)
    for i, (c, s) in enumerate(zip(cases, solvers)):
        W, r, kw = s.fields("cons"), s.residual(), s.fields("turb")
        assert np.array_equal(W, ref[i][0]), (i, c.name)
        assert np.array_equal(r["res"], ref[i][1]["res"]), (i, c.name)
        assert r["t"] == ref[i][1]["t"] and r["steps"] == ref[i][1]["steps"], (i, c.name)
        assert np.array_equal(kw, ref[i][2]), (i, c.name)
    b.close()
    for s in solvers:
        s.close()


def test_batch_admitting_a_new_variant_drops_the_graph():
    from paper_1302_2132_amd import Batch, Solver
    a, w5 = C.mixing_layer(24, seed=1), C.mixing_layer(30, seed=2)
    w5.recon, w5.kw_transport = "weno5", True
    ref_a, ref_w = _alone_full(a, 9), _alone_full(w5, 5)
    sa, sw = Solver(a), Solver(w5)
    b = Batch([sa], capacity=4)
    b.capture()
    b.step(4)
    b.set_members([sa, sw])          # a new (class, variant) pair and the transported form
    b.step(5)
    assert np.array_equal(sa.fields("cons"), ref_a[0])
    assert np.array_equal(sw.fields("cons"), ref_w[0])
    assert np.array_equal(sw.fields("turb"), ref_w[2])
    b.close()
    for s in (sa, sw):
        s.close()


def test_launch_shapes_do_not_change_results():
    """Every persistent grid gives the same fields, bitwise, also for members with options
    (their kernels walk the same persistent grids); the tiles are fixed, and a face-kernel
    tile the library does not have is refused."""
    from paper_1302_2132_amd import Batch, Solver
    cases = _cases()[:4] + [_option_cases()[i] for i in (1, 4, 8)]
    ref = [_alone(c, 15) for c in cases]
    solvers = [Solver(c) for c in cases]
    b = Batch(solvers, capacity=8)
    from paper_1302_2132_amd import GKS_ERR_ARG, GksError
    with pytest.raises(GksError) as e:
        b.set_launch(3, 0, 128)
    assert e.value.status == GKS_ERR_ARG
    # (3D tile, 2D tile shape, grid): 2D shapes 16 x 15, 32 x 7, 8 x 28
    shapes = [(64, 0, 0), (0, 1, 512), (256, 2, 0), (64, 1, 4096), (0, 0, 0)]
    for i, (tile, shape2, grid) in enumerate(shapes):
        for kind in (1, 2):
            b.set_launch(kind, grid, shape2)
        for kind in (3, 4):
            b.set_launch(kind, grid, tile)
        b.set_launch(0, grid, 0)
        b.set_launch(5, grid, 0)
        b.step(3)
    for s, r in zip(solvers, ref):
        assert np.array_equal(s.fields("cons"), r[0])
    b.close()
    for s in solvers:
        s.close()


def test_autotuner_steps_are_real_steps():
    from paper_1302_2132_amd import Batch, Solver
    from paper_1302_2132_amd.autotune import autotune
    cases = [C.mixing_layer(48, seed=5, precision="fp32_flux"), C.sbli(40, 20, precision="fp32_flux")]
    solvers = [Solver(c) for c in cases]
    b = Batch(solvers, capacity=2)
    shape, steps, _ = autotune(b, steps_per_trial=1, use_cache=False)
    assert steps > 0
    b.capture()
    b.step(5)
    st = b.status()
    assert np.all(st["steps"] == steps + 5)
    for c, s in zip(cases, solvers):
        W, r = _alone(c, steps + 5)
        assert np.array_equal(s.fields("cons"), W)
    b.close()
    for s in solvers:
        s.close()


# --------------------------------------------------------------------------------------
# batch members against the oracle
# --------------------------------------------------------------------------------------
def _config3_small(precision):
    """The uneven batch's recipe at sizes the oracle runs in seconds: mixing layers and
    Galilean-shifted Sod tubes (Ma up to 2) of sides 40..100 (none a tile multiple in both
    directions), plus two shifted tubes at Ma 1.6 and 2.0 on 71 x 13 and 97 x 23 meshes."""
    import math
    cases = C.batch_cases(14, seed=3, nmin=40, nmax=100, steps=200, precision=precision)
    for Ma, nx, ny in ((1.6, 71, 13), (2.0, 97, 23)):
        c = C.shock_tube(nx, ny, x0=0.25, shift=Ma * math.sqrt(1.4), mu=1e-4, c_a=1.0, k_val=1e-6,
                         omega_val=10.0, steps=200, precision=precision, bc_x=("dirichlet", "outflow"),
                         name=f"shifted_sod_Ma{Ma}")
        cases.append(c)
    return cases


@pytest.fixture(scope="module")
def config3_oracle():
    cases = _config3_small("fp64")
    banner(f"oracle: {len(cases)} batch members, 200 steps each")
    return [oracle.run(c, 200) for c in cases]


@pytest.mark.parametrize("precision,tol", [("fp32_flux", 1e-5), ("fp64", 1e-12)])
def test_uneven_batch_members_match_the_oracle(config3_oracle, precision, tol):
    from paper_1302_2132_amd import Batch, Solver
    from paper_1302_2132_amd.autotune import autotune
    cases = _config3_small(precision)
    assert any(c.meta.get("shift", 0.0) >= 1.5 * math.sqrt(1.4) for c in cases)
    banner(f"uneven batch of {len(cases)} ({precision}), autotuned, captured, 200 steps")
    solvers = [Solver(c) for c in cases]
    b = Batch(solvers, capacity=len(cases))
    try:
        _, tune_steps, _ = autotune(b, steps_per_trial=1, use_cache=False)
        b.capture()
        b.step(200 - tune_steps)
        st = b.status()
        assert np.all(st["steps"] == 200)
        for c, s, ro in zip(cases, solvers, config3_oracle):
            assert_matches_oracle(s.fields("cons"), c, ro, tol, label=f"{c.name}: ")
    finally:
        b.close()
        for s in solvers:
            s.close()


@pytest.mark.parametrize("graph", [False, True])
def test_batch_with_every_option_matches_the_oracle(graph):
    """Each member of the every-option batch against the oracle (FP64 1e-12, FP32 flux
    1e-5; transported k and omega too)."""
    from paper_1302_2132_amd import Batch, Solver
    n = 12
    cases = _option_cases()
    solvers = [Solver(c) for c in cases]
    b = Batch(solvers, capacity=12)
    try:
        if graph:
            b.capture()
        b.step(n)
        for c, s in zip(cases, solvers):
            ro = oracle_reference(c, n)
            tol = 1e-12 if c.precision == "fp64" else 1e-5
            assert_matches_oracle(s.fields("cons"), c, ro, tol, label=f"{c.name}: ")
            if c.kw_transport:
                kw = s.fields("turb")
                for got, ref in ((kw[0], ro["k"]), (kw[1], ro["omega"])):
                    assert np.max(np.abs(got - ref)) <= tol * np.max(np.abs(ref)), c.name
    finally:
        b.close()
        for s in solvers:
            s.close()


def test_multi_step_graph_replays_equal_alone():
    """A graph of 8 captured steps, replayed twice with status reads (synchronising eager
    work) between the replays, then 5 more steps launched directly: every member equals its
    solve alone after each stage, bitwise."""
    from paper_1302_2132_amd import Batch, Solver
    cases = _cases()[:4] + [_option_cases()[1]]
    refs = {n: [_alone(c, n) for c in cases] for n in (8, 16, 21)}
    solvers = [Solver(c) for c in cases]
    b = Batch(solvers, capacity=8)
    try:
        b.capture(steps=8)
        done = 0
        for n in (8, 8, 5):
            b.step(n)
            done += n
            st = b.status()
            for i, (c, s) in enumerate(zip(cases, solvers)):
                W, r = refs[done][i]
                assert st["steps"][i] == r["steps"], (done, c.name)
                assert np.array_equal(s.fields("cons"), W), (done, c.name)
    finally:
        b.close()
        for s in solvers:
            s.close()
